// Host assembly of the coupled Stokes-Darcy system.
//
// Model (Sec. 2 of the paper): creeping Stokes flow, momentum flux
// (pI - tau) n with tau = mu (grad v + grad v^T), in the free flow; Darcy's law
// with mass continuity in the porous medium; on the interface the normal-stress
// balance, Beavers-Joseph-Saffman slip and normal mass-flux continuity.
// Staggered finite volumes (free flow) and two-point fluxes (porous medium),
// unknowns in the pressure-velocity block order.  Every row states
// "sum of outward fluxes = source x |CV|".  Closures the paper leaves to its
// references:
//   * BJS at Gamma: slip velocity eliminated over the half cell, south shear
//     flux gamma mu [(2 dx/dy) u + (v_i - v_{i-1})], gamma = beta/(beta+2/dy),
//     beta = alpha/sqrt(K_f), K_f harmonic mean of the two porous cells below;
//   * traction outflow: n.(pI - tau)n at the last cell centre = data;
//   * Gamma rows: dx [p - 2 mu (v_1 - v_0)/dy - q_top + (mu/K)(dy_pm/2) v_0] = 0;
//   * porous top cells: interface flux dx * v_{i,0};
//   * full Beavers-Joseph (phys.bj_full): the slip velocity is measured
//     against the porous tangential velocity -(K_f/mu)(q_i - q_{i-1})/dx, so
//     Gamma's u rows couple to the two top cells with +-cg (K_f/mu)/dx;
//   * dt > 0: the transient momentum equation with the paper's backward Euler
//     step adds |CV|/dt (rho = 1) to the diagonal of every interior u and v
//     face row; the outflow u rows, the Gamma rows and the Darcy rows are
//     conditions without a time derivative.  b holds the data part only.
// Each coefficient is evaluated as one fixed IEEE-double expression (the file
// is compiled without floating-point contraction), so the values are
// reproducible bit-for-bit.
#include <algorithm>
#include <cmath>
#include <utility>

#include "sd_internal.h"

namespace sd {

namespace {

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

void check_array(const double* a, int64_t n, const char* what) {
  if (!a) return;
  for (int64_t k = 0; k < n; ++k)
    if (!std::isfinite(a[k]))
      throw Error(SD_E_INVALID, std::string("non-finite value in ") + what);
}

}  // namespace

void RowBuilder::finish() {
  std::sort(row.begin(), row.end(),
            [](const std::pair<int32_t, double>& a, const std::pair<int32_t, double>& b) {
              return a.first < b.first;
            });
  for (size_t k = 1; k < row.size(); ++k)
    if (row[k].first == row[k - 1].first)
      throw Error(SD_E_INVALID, "internal: duplicate matrix entry");
  for (auto& e : row) {
    A.col.push_back(e.first);
    A.val.push_back(e.second);
  }
  A.rowptr.push_back((int64_t)A.col.size());
  row.clear();
}

void assemble_host(const sd_grid* g, const sd_physics* ph, const sd_bcs* bcs,
                   const double* K, const sd_forcing* f, HostProblem& P) {
  TraceRange trace("sd: assembly");
  if (!g || !ph || !bcs || !K) throw Error(SD_E_INVALID, "null argument");
  if (g->nz < 0) throw Error(SD_E_INVALID, "nz must be >= 0 (0 = 2-D)");
  if (g->nz > 0) {
    assemble_host_3d(g, ph, bcs, K, f, P);
    return;
  }
  const int nx = g->nx, ny = g->ny, nyp = g->ny_pm;
  const int npm = g->nx_pm > 0 ? g->nx_pm : nx, i0 = g->pm_i0;
  if (nx < 2 || ny < 2 || nyp < 1)
    throw Error(SD_E_INVALID, "need nx >= 2, ny >= 2, ny_pm >= 1");
  if (g->nx_pm < 0 || i0 < 0 || i0 + npm > nx)
    throw Error(SD_E_INVALID, "the porous block must lie under the free flow");
  if (!finite_pos(g->Lx) || !finite_pos(g->H_ff) || !finite_pos(g->H_pm))
    throw Error(SD_E_INVALID, "extents must be finite and positive");
  if (!finite_pos(ph->mu) || !finite_pos(ph->alpha_bj))
    throw Error(SD_E_INVALID, "mu and alpha_bj must be finite and positive");
  if (!(std::isfinite(ph->dt) && ph->dt >= 0.0))
    throw Error(SD_E_INVALID, "dt must be finite and >= 0 (0 = stationary)");
  if (bcs->ff_top != SD_BC_VELOCITY)
    throw Error(SD_E_INVALID, "the free-flow top boundary must be SD_BC_VELOCITY");
  for (int t : {bcs->ff_left, bcs->ff_right})
    if (t != SD_BC_VELOCITY && t != SD_BC_TRACTION)
      throw Error(SD_E_INVALID,
                  "free-flow left/right boundaries: SD_BC_VELOCITY or SD_BC_TRACTION");
  for (int t : {bcs->pm_left, bcs->pm_right, bcs->pm_bottom})
    if (t != SD_BC_PRESSURE && t != SD_BC_NOFLOW)
      throw Error(SD_E_INVALID, "porous boundaries: SD_BC_PRESSURE or SD_BC_NOFLOW");
  const int64_t nK = (int64_t)npm * nyp;
  for (int64_t k = 0; k < nK; ++k)
    if (!finite_pos(K[k])) throw Error(SD_E_INVALID, "K must be finite and positive");
  check_array(bcs->ff_left_n, ny, "ff_left_n");
  check_array(bcs->ff_left_t, ny + 1, "ff_left_t");
  check_array(bcs->ff_right_n, ny, "ff_right_n");
  check_array(bcs->ff_right_t, ny + 1, "ff_right_t");
  check_array(bcs->ff_top_t, nx + 1, "ff_top_t");
  check_array(bcs->ff_top_n, nx, "ff_top_n");
  check_array(bcs->pm_left_p, nyp, "pm_left_p");
  check_array(bcs->pm_right_p, nyp, "pm_right_p");
  check_array(bcs->pm_bottom_p, npm, "pm_bottom_p");
  if (f) {
    check_array(f->f_u, (int64_t)ny * (nx + 1), "f_u");
    check_array(f->f_v, (int64_t)(ny + 1) * nx, "f_v");
    check_array(f->q_pm, nK, "q_pm");
  }

  const bool right_tr = bcs->ff_right == SD_BC_TRACTION;
  const bool left_tr = bcs->ff_left == SD_BC_TRACTION;
  Layout L;
  L.nx = nx;
  L.ny = ny;
  L.nyp = nyp;
  L.nx_pm = npm;
  L.i0 = i0;
  L.i_first = left_tr ? 0 : 1;
  L.nux = (right_tr ? nx : nx - 1) - L.i_first + 1;
  L.off_v = (int64_t)L.nux * ny;
  L.off_p = L.off_v + npm + (int64_t)nx * (ny - 1);
  L.off_w = L.off_p;
  L.off_q = L.off_p + (int64_t)nx * ny;
  L.N = L.off_q + (int64_t)npm * nyp;
  if (L.N >= (int64_t)1 << 31) throw Error(SD_E_INVALID, "problem too large for 32-bit indices");
  auto over = [&](int i) { return i >= i0 && i < i0 + npm; };

  P.grid = *g;
  P.phys = *ph;
  P.bc[0] = bcs->ff_left; P.bc[1] = bcs->ff_right; P.bc[2] = bcs->ff_top;
  P.bc[3] = bcs->pm_left; P.bc[4] = bcs->pm_right; P.bc[5] = bcs->pm_bottom;
  P.L = L;
  P.pm_singular = bcs->pm_left == SD_BC_NOFLOW && bcs->pm_right == SD_BC_NOFLOW &&
                  bcs->pm_bottom == SD_BC_NOFLOW;
  P.K.assign(K, K + nK);

  auto data = [](const double* a, int64_t k) { return a ? a[k] : 0.0; };
  const double* uL = bcs->ff_left_n;
  const double* vL = bcs->ff_left_t;
  const double* uR = bcs->ff_right_n;
  const double* vR = bcs->ff_right_t;
  const double* uT = bcs->ff_top_t;
  const double* vT = bcs->ff_top_n;
  const double* pL = bcs->pm_left_p;
  const double* pR = bcs->pm_right_p;
  const double* pB = bcs->pm_bottom_p;
  const double* fu = f ? f->f_u : nullptr;
  const double* fv = f ? f->f_v : nullptr;
  const double* fq = f ? f->q_pm : nullptr;

  const double mu = ph->mu, alpha = ph->alpha_bj;
  const double dx = g->Lx / (double)nx;
  const double dy = g->H_ff / (double)ny;
  const double dyp = g->H_pm / (double)nyp;
  const double vol = dx * dy;
  const double volp = dx * dyp;
  const bool transient = ph->dt > 0.0;
  const double mvol = transient ? vol / ph->dt : 0.0;
  P.mass = mvol;
  const double cx = (2.0 * mu) * (dy / dx);
  const double cy = mu * (dx / dy);
  const double cyt = mu * (dx / (0.5 * dy));
  const double cyy = (2.0 * mu) * (dx / dy);
  const double cxv = mu * (dy / dx);
  const double cxw = mu * (dy / (0.5 * dx));
  auto Kat = [&](int ipm, int k) { return K[(int64_t)k * npm + ipm]; };

  HostCSR& A = P.A;
  A.n_rows = A.n_cols = L.N;
  A.rowptr.assign(1, 0);
  A.col.reserve((size_t)(L.N * 8));
  A.val.reserve((size_t)(L.N * 8));
  P.b.assign((size_t)L.N, 0.0);
  RowBuilder rb(A);

  // ---- u rows ----
  for (int j = 0; j < ny; ++j) {
    for (int i = L.i_first; i <= L.i_first + L.nux - 1; ++i) {
      const int64_t r = L.u(i, j);
      if (i == 0) {  // traction (pressure) face on the left
        rb.add(r, cx);
        rb.add(L.u(1, j), -cx);
        rb.add(L.p(0, j), dy);
        rb.finish();
        P.b[r] = data(uL, j) * dy;
        continue;
      }
      if (i == nx) {  // outflow face (traction)
        rb.add(r, cx);
        rb.add(L.u(nx - 1, j), -cx);
        rb.add(L.p(nx - 1, j), -dy);
        rb.finish();
        P.b[r] = (-data(uR, j)) * dy;
        continue;
      }
      const bool top = j == ny - 1, bot = j == 0;
      // faces of the first row with both cells over the porous block obey BJS;
      // the others meet the bottom wall (no slip over half a cell)
      const bool gam = bot && over(i - 1) && over(i);
      const int ia = std::min(std::max(i - 1 - i0, 0), npm - 1);
      const int ib = std::min(std::max(i - i0, 0), npm - 1);
      const double Ka = Kat(ia, nyp - 1), Kb = Kat(ib, nyp - 1);
      const double Kf = (2.0 * Ka * Kb) / (Ka + Kb);
      const double beta = alpha / std::sqrt(Kf);
      const double gg = beta / (beta + 2.0 / dy);
      const double cg = (gg * mu) * ((2.0 * dx) / dy);
      const double gm = gg * mu;
      const double aN = top ? cyt : cy;
      const double aS = gam ? cg : (bot ? cyt : cy);
      double d = ((cx + cx) + aN) + aS;
      if (transient) d = d + mvol;
      rb.add(r, d);
      if (i - 1 >= 1 || left_tr) rb.add(L.u(i - 1, j), -cx);
      if (i + 1 <= nx - 1 || right_tr) rb.add(L.u(i + 1, j), -cx);
      if (!top) rb.add(L.u(i, j + 1), -cy);
      if (!bot) rb.add(L.u(i, j - 1), -cy);
      if (!top) {
        rb.add(L.v(i, j + 1), -mu);
        rb.add(L.v(i - 1, j + 1), mu);
      }
      if (!bot || over(i)) rb.add(L.v(i, j), gam ? gm : mu);
      if (!bot || over(i - 1)) rb.add(L.v(i - 1, j), gam ? -gm : -mu);
      rb.add(L.p(i, j), dy);
      rb.add(L.p(i - 1, j), -dy);
      if (ph->bj_full && gam) {   // porous tangential velocity in the slip condition
        const double cbj = cg * ((Kf / mu) / dx);
        rb.add(L.q(ib, nyp - 1), cbj);
        rb.add(L.q(ia, nyp - 1), -cbj);
      }
      rb.finish();
      double rhs = data(fu, (int64_t)j * (nx + 1) + i) * vol;
      if (!left_tr && i - 1 == 0) rhs = rhs + cx * data(uL, j);
      if (!right_tr && i + 1 == nx) rhs = rhs + cx * data(uR, j);
      if (top) rhs = rhs + cyt * data(uT, i);
      if (top) rhs = rhs + mu * (data(vT, i) - data(vT, i - 1));
      P.b[r] = rhs;
    }
  }
  // ---- v rows: Gamma (first row over the block) then interior ----
  for (int j = 0; j < ny; ++j) {
    for (int i = 0; i < nx; ++i) {
      if (j == 0) {
        if (!over(i)) continue;   // wall face: zero velocity, not an unknown
        const int64_t r = L.v(i, 0);
        const double Kt = Kat(i - i0, nyp - 1);
        const double dg = ((mu / Kt) * (0.5 * dyp)) * dx;
        rb.add(r, cyy + dg);
        rb.add(L.v(i, 1), -cyy);
        rb.add(L.p(i, 0), dx);
        rb.add(L.q(i - i0, nyp - 1), -dx);
        rb.finish();
        P.b[r] = 0.0;
        continue;
      }
      const int64_t r = L.v(i, j);
      const bool west = i == 0, east = i == nx - 1;
      const double aE = east ? (right_tr ? 0.0 : cxw) : cxv;
      const double aW = west ? (left_tr ? 0.0 : cxw) : cxv;
      double d = ((cyy + cyy) + aE) + aW;
      if (transient) d = d + mvol;
      rb.add(r, d);
      if (j + 1 <= ny - 1) rb.add(L.v(i, j + 1), -cyy);
      if (j - 1 >= 1 || over(i)) rb.add(L.v(i, j - 1), -cyy);
      if (!east) rb.add(L.v(i + 1, j), -cxv);
      if (!west) rb.add(L.v(i - 1, j), -cxv);
      if (i + 1 <= nx - 1) {
        rb.add(L.u(i + 1, j), -mu);
        rb.add(L.u(i + 1, j - 1), mu);
      }
      if (!west) {
        rb.add(L.u(i, j), mu);
        rb.add(L.u(i, j - 1), -mu);
      }
      rb.add(L.p(i, j), dx);
      rb.add(L.p(i, j - 1), -dx);
      rb.finish();
      double rhs = data(fv, (int64_t)j * nx + i) * vol;
      if (j + 1 == ny) rhs = rhs + cyy * data(vT, i);
      if (left_tr) {
        if (west) rhs = rhs - data(vL, j) * dy;
      } else {
        if (west) rhs = rhs + cxw * data(vL, j);
        if (west) rhs = rhs - mu * (data(uL, j) - data(uL, j - 1));
      }
      if (right_tr) {
        if (east) rhs = rhs - data(vR, j) * dy;
      } else {
        if (east) rhs = rhs + cxw * data(vR, j);
        if (east) rhs = rhs + mu * (data(uR, j) - data(uR, j - 1));
      }
      P.b[r] = rhs;
    }
  }
  // ---- free-flow continuity ----
  for (int j = 0; j < ny; ++j) {
    for (int i = 0; i < nx; ++i) {
      const int64_t r = L.p(i, j);
      if (i + 1 <= nx - 1 || right_tr) rb.add(L.u(i + 1, j), dy);
      if (i >= 1 || left_tr) rb.add(L.u(i, j), -dy);
      if (j + 1 <= ny - 1) rb.add(L.v(i, j + 1), dx);
      if (j >= 1 || over(i)) rb.add(L.v(i, j), -dx);
      rb.finish();
      double rhs = 0.0;
      if (!left_tr && i == 0) rhs = rhs + dy * data(uL, j);
      if (!right_tr && i + 1 == nx) rhs = rhs - dy * data(uR, j);
      if (j + 1 == ny) rhs = rhs - dx * data(vT, i);
      P.b[r] = rhs;
    }
  }
  // ---- porous medium, two-point fluxes (porous columns 0..npm-1) ----
  const bool pr_d = bcs->pm_right == SD_BC_PRESSURE;
  const bool pl_d = bcs->pm_left == SD_BC_PRESSURE;
  const bool pb_d = bcs->pm_bottom == SD_BC_PRESSURE;
  for (int k = 0; k < nyp; ++k) {
    for (int i = 0; i < npm; ++i) {
      const int64_t r = L.q(i, k);
      const double Kc = Kat(i, k);
      auto t_int = [&](double area, double dd, double Kn) {
        return ((area / mu) * ((2.0 * Kc * Kn) / (Kc + Kn))) / dd;
      };
      auto t_dir = [&](double area, double dd) { return ((area / mu) * Kc) / (0.5 * dd); };
      const double TE = (i + 1 <= npm - 1) ? t_int(dyp, dx, Kat(i + 1, k))
                                           : (pr_d ? t_dir(dyp, dx) : 0.0);
      const double TW = (i >= 1) ? t_int(dyp, dx, Kat(i - 1, k))
                                 : (pl_d ? t_dir(dyp, dx) : 0.0);
      const double TN = (k + 1 <= nyp - 1) ? t_int(dx, dyp, Kat(i, k + 1)) : 0.0;
      const double TS = (k >= 1) ? t_int(dx, dyp, Kat(i, k - 1))
                                 : (pb_d ? t_dir(dx, dyp) : 0.0);
      rb.add(r, ((TE + TW) + TN) + TS);
      if (i + 1 <= npm - 1) rb.add(L.q(i + 1, k), -TE);
      if (i >= 1) rb.add(L.q(i - 1, k), -TW);
      if (k + 1 <= nyp - 1) rb.add(L.q(i, k + 1), -TN);
      if (k >= 1) rb.add(L.q(i, k - 1), -TS);
      if (k == nyp - 1) rb.add(L.v(i + i0, 0), dx);
      rb.finish();
      double rhs = data(fq, (int64_t)k * npm + i) * volp;
      if (pr_d && i == npm - 1) rhs = rhs + TE * data(pR, k);
      if (pl_d && i == 0) rhs = rhs + TW * data(pL, k);
      if (pb_d && k == 0) rhs = rhs + TS * data(pB, i);
      P.b[r] = rhs;
    }
  }
  if ((int64_t)A.rowptr.size() != L.N + 1) throw Error(SD_E_INVALID, "internal: row count");
}

HostCSR extract_block(const HostCSR& A, int64_t r0, int64_t r1, int64_t c0, int64_t c1) {
  HostCSR B;
  B.n_rows = r1 - r0;
  B.n_cols = c1 - c0;
  B.rowptr.assign(1, 0);
  for (int64_t r = r0; r < r1; ++r) {
    for (int64_t k = A.rowptr[r]; k < A.rowptr[r + 1]; ++k) {
      const int64_t c = A.col[k];
      if (c >= c0 && c < c1) {
        B.col.push_back((int32_t)(c - c0));
        B.val.push_back(A.val[k]);
      }
    }
    B.rowptr.push_back((int64_t)B.col.size());
  }
  return B;
}

static double diag_of(const HostCSR& A, int64_t r) {
  for (int64_t k = A.rowptr[r]; k < A.rowptr[r + 1]; ++k)
    if (A.col[k] == r) return A.val[k];
  throw Error(SD_E_INVALID, "internal: missing diagonal entry");
}

HostCSR darcy_interface_block(const HostCSR& D, const HostCSR& C1, const HostCSR& B1,
                              const HostCSR& V) {
  HostCSR Dt = D;
  for (int64_t t = 0; t < D.n_rows; ++t) {
    for (int64_t kk = C1.rowptr[t]; kk < C1.rowptr[t + 1]; ++kk) {
      const int64_t gidx = C1.col[kk];
      const double c1 = C1.val[kk];
      const double vgg = diag_of(V, gidx);
      for (int64_t ll = B1.rowptr[gidx]; ll < B1.rowptr[gidx + 1]; ++ll) {
        const int64_t tp = B1.col[ll];
        const double b1 = B1.val[ll];
        int64_t pos = -1;
        for (int64_t m = Dt.rowptr[t]; m < Dt.rowptr[t + 1]; ++m)
          if (Dt.col[m] == tp) pos = m;
        if (pos < 0) throw Error(SD_E_INVALID, "internal: Darcy correction outside pattern");
        Dt.val[pos] = Dt.val[pos] - (c1 * b1) / vgg;
      }
    }
  }
  return Dt;
}

}  // namespace sd
