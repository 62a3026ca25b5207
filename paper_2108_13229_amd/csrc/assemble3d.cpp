// Host assembly of the coupled Stokes-Darcy system on a 3-D box grid.
//
// The model of Sec. 2 of the paper (creeping Stokes flow in symmetric-gradient
// form, two-point-flux Darcy, normal-stress balance, Beavers-Joseph-Saffman
// slip and mass-flux continuity on Gamma, optional backward-Euler mass) with
// the closures of the 2-D assembly, extended by a spanwise direction z:
//   * x streamwise (nx cells), y normal to Gamma, z spanwise (nz cells);
//     face areas Ax = dy dz, Ay = dx dz, Az = dx dy; every row is "sum of
//     outward fluxes = source x |CV|";
//   * w faces k = 1..nz-1 are unknowns; the free-flow z walls are velocity
//     walls, eliminated and lifted into b;
//   * BJS holds for u and for w: the south shear flux at Gamma is
//     g mu [(2 Ay/dy) u + dz (v_i - v_{i-1})] for u and
//     g mu [(2 Ay/dy) w + dx (v_k - v_{k-1})] for w, g = beta/(beta + 2/dy),
//     beta = alpha/sqrt(K_f), K_f the harmonic mean of the two porous top
//     cells beside the face;
//   * Gamma rows: Ay [p - 2 mu (v_1 - v_0)/dy - q_top + (mu/K)(dy_pm/2) v_0] = 0;
//   * porous cells: six two-point fluxes, interface flux Ay v_{i,0,k};
//   * full Beavers-Joseph (phys.bj_full): as in 2-D, along x for u and along
//     z for w.
// Unknowns u, v, w, p, q, each ordered (j, k, i) with i fastest.  Every
// coefficient is one fixed IEEE-double expression (no contraction), so the
// values are reproducible bit for bit.
#include <cmath>

#include "sd_internal.h"

namespace sd {

namespace {

bool finite_pos3(double x) { return std::isfinite(x) && x > 0.0; }

void check3(const double* a, int64_t n, const char* what) {
  if (!a) return;
  for (int64_t k = 0; k < n; ++k)
    if (!std::isfinite(a[k])) throw Error(SD_E_INVALID, std::string("non-finite value in ") + what);
}

}  // namespace

void assemble_host_3d(const sd_grid* g, const sd_physics* ph, const sd_bcs* bcs,
                      const double* K, const sd_forcing* f, HostProblem& P) {
  const int nx = g->nx, ny = g->ny, nyp = g->ny_pm, nz = g->nz;
  if (nx < 2 || ny < 2 || nyp < 1 || nz < 1)
    throw Error(SD_E_INVALID, "need nx >= 2, ny >= 2, ny_pm >= 1, nz >= 1");
  if ((g->nx_pm != 0 && g->nx_pm != nx) || g->pm_i0 != 0)
    throw Error(SD_E_INVALID, "3-D: the porous block spans the free flow (nx_pm = 0, pm_i0 = 0)");
  if (!finite_pos3(g->Lx) || !finite_pos3(g->H_ff) || !finite_pos3(g->H_pm) ||
      !finite_pos3(g->Lz))
    throw Error(SD_E_INVALID, "extents must be finite and positive");
  if (!finite_pos3(ph->mu) || !finite_pos3(ph->alpha_bj))
    throw Error(SD_E_INVALID, "mu and alpha_bj must be finite and positive");
  if (!(std::isfinite(ph->dt) && ph->dt >= 0.0))
    throw Error(SD_E_INVALID, "dt must be finite and >= 0 (0 = stationary)");
  if (bcs->ff_left != SD_BC_VELOCITY || bcs->ff_top != SD_BC_VELOCITY)
    throw Error(SD_E_INVALID, "free-flow left and top boundaries must be SD_BC_VELOCITY");
  if (bcs->ff_right != SD_BC_VELOCITY && bcs->ff_right != SD_BC_TRACTION)
    throw Error(SD_E_INVALID, "free-flow right boundary: SD_BC_VELOCITY or SD_BC_TRACTION");
  for (int t : {bcs->pm_left, bcs->pm_right, bcs->pm_bottom, bcs->pm_back, bcs->pm_front})
    if (t != SD_BC_PRESSURE && t != SD_BC_NOFLOW)
      throw Error(SD_E_INVALID, "porous boundaries: SD_BC_PRESSURE or SD_BC_NOFLOW");
  const int64_t nK = (int64_t)nx * nyp * nz;
  for (int64_t k = 0; k < nK; ++k)
    if (!finite_pos3(K[k])) throw Error(SD_E_INVALID, "K must be finite and positive");
  const int64_t X1 = nx + 1, Y1 = ny + 1, Z1 = nz + 1;
  check3(bcs->ff_left_n, ny * (int64_t)nz, "ff_left_n");
  check3(bcs->ff_left_t, Y1 * nz, "ff_left_t");
  check3(bcs->ff_left_tz, ny * Z1, "ff_left_tz");
  check3(bcs->ff_right_n, ny * (int64_t)nz, "ff_right_n");
  check3(bcs->ff_right_t, Y1 * nz, "ff_right_t");
  check3(bcs->ff_right_tz, ny * Z1, "ff_right_tz");
  check3(bcs->ff_top_t, nz * X1, "ff_top_t");
  check3(bcs->ff_top_n, nz * (int64_t)nx, "ff_top_n");
  check3(bcs->ff_top_tz, Z1 * nx, "ff_top_tz");
  check3(bcs->ff_back_u, ny * X1, "ff_back_u");
  check3(bcs->ff_back_v, Y1 * nx, "ff_back_v");
  check3(bcs->ff_back_n, ny * (int64_t)nx, "ff_back_n");
  check3(bcs->ff_front_u, ny * X1, "ff_front_u");
  check3(bcs->ff_front_v, Y1 * nx, "ff_front_v");
  check3(bcs->ff_front_n, ny * (int64_t)nx, "ff_front_n");
  check3(bcs->pm_left_p, nyp * (int64_t)nz, "pm_left_p");
  check3(bcs->pm_right_p, nyp * (int64_t)nz, "pm_right_p");
  check3(bcs->pm_bottom_p, nz * (int64_t)nx, "pm_bottom_p");
  check3(bcs->pm_back_p, nyp * (int64_t)nx, "pm_back_p");
  check3(bcs->pm_front_p, nyp * (int64_t)nx, "pm_front_p");
  if (f) {
    check3(f->f_u, ny * (int64_t)nz * X1, "f_u");
    check3(f->f_v, Y1 * nz * nx, "f_v");
    check3(f->f_w, ny * Z1 * nx, "f_w");
    check3(f->q_pm, nK, "q_pm");
  }

  const bool right_tr = bcs->ff_right == SD_BC_TRACTION;
  Layout L;
  L.nx = nx;
  L.ny = ny;
  L.nyp = nyp;
  L.nz = nz;
  L.nux = right_tr ? nx : nx - 1;
  L.off_v = (int64_t)L.nux * ny * nz;
  L.off_w = L.off_v + (int64_t)nx * ny * nz;
  L.off_p = L.off_w + (int64_t)nx * ny * (nz - 1);
  L.off_q = L.off_p + (int64_t)nx * ny * nz;
  L.N = L.off_q + (int64_t)nx * nyp * nz;
  if (L.N >= (int64_t)1 << 31) throw Error(SD_E_INVALID, "problem too large for 32-bit indices");

  P.grid = *g;
  P.phys = *ph;
  P.bc[0] = bcs->ff_left; P.bc[1] = bcs->ff_right; P.bc[2] = bcs->ff_top;
  P.bc[3] = bcs->pm_left; P.bc[4] = bcs->pm_right; P.bc[5] = bcs->pm_bottom;
  P.L = L;
  P.pm_singular = bcs->pm_left == SD_BC_NOFLOW && bcs->pm_right == SD_BC_NOFLOW &&
                  bcs->pm_bottom == SD_BC_NOFLOW && bcs->pm_back == SD_BC_NOFLOW &&
                  bcs->pm_front == SD_BC_NOFLOW;
  P.K.assign(K, K + nK);

  auto d = [](const double* a, int64_t k) { return a ? a[k] : 0.0; };
  const double *uL = bcs->ff_left_n, *vL = bcs->ff_left_t, *wL = bcs->ff_left_tz;
  const double *uR = bcs->ff_right_n, *vR = bcs->ff_right_t, *wR = bcs->ff_right_tz;
  const double *uT = bcs->ff_top_t, *vT = bcs->ff_top_n, *wT = bcs->ff_top_tz;
  const double *uB = bcs->ff_back_u, *vB = bcs->ff_back_v, *wB = bcs->ff_back_n;
  const double *uF = bcs->ff_front_u, *vF = bcs->ff_front_v, *wF = bcs->ff_front_n;
  const double *pL = bcs->pm_left_p, *pR = bcs->pm_right_p, *pBo = bcs->pm_bottom_p;
  const double *pBk = bcs->pm_back_p, *pFr = bcs->pm_front_p;
  const double* fu = f ? f->f_u : nullptr;
  const double* fv = f ? f->f_v : nullptr;
  const double* fw = f ? f->f_w : nullptr;
  const double* fq = f ? f->q_pm : nullptr;

  const double mu = ph->mu, alpha = ph->alpha_bj;
  const double dx = g->Lx / (double)nx, dy = g->H_ff / (double)ny;
  const double dyp = g->H_pm / (double)nyp, dz = g->Lz / (double)nz;
  const double Ax = dy * dz, Ay = dx * dz, Az = dx * dy;
  const double vol = (dx * dy) * dz;
  const double volp = (dx * dyp) * dz;
  const bool transient = ph->dt > 0.0;
  const double mvol = transient ? vol / ph->dt : 0.0;
  P.mass = mvol;
  const double cx = (2.0 * mu) * (Ax / dx);
  const double cy = mu * (Ay / dy);
  const double cyt = mu * (Ay / (0.5 * dy));
  const double cz = mu * (Az / dz);
  const double czt = mu * (Az / (0.5 * dz));
  const double cyy = (2.0 * mu) * (Ay / dy);
  const double cxv = mu * (Ax / dx);
  const double cxw = mu * (Ax / (0.5 * dx));
  const double czz = (2.0 * mu) * (Az / dz);
  const double mdx = mu * dx, mdy = mu * dy, mdz = mu * dz;
  auto Kat = [&](int i, int jj, int k) { return K[((int64_t)jj * nz + k) * nx + i]; };
  auto harm = [](double a, double c) { return (2.0 * a * c) / (a + c); };

  HostCSR& A = P.A;
  A.n_rows = A.n_cols = L.N;
  A.rowptr.assign(1, 0);
  A.col.reserve((size_t)(L.N * 12));
  A.val.reserve((size_t)(L.N * 12));
  P.b.assign((size_t)L.N, 0.0);
  RowBuilder rb(A);

  // ---- u rows ----
  for (int j = 0; j < ny; ++j) {
    for (int k = 0; k < nz; ++k) {
      for (int i = 1; i <= L.nux; ++i) {
        const int64_t r = L.u3(i, j, k);
        const int64_t jk = (int64_t)j * nz + k;
        if (i == nx) {  // outflow face (traction)
          rb.add(r, cx);
          rb.add(L.u3(nx - 1, j, k), -cx);
          rb.add(L.p3(nx - 1, j, k), -Ax);
          rb.finish();
          P.b[r] = (-d(uR, jk)) * Ax;
          continue;
        }
        const bool top = j == ny - 1, gam = j == 0, front = k == nz - 1, back = k == 0;
        const double beta = alpha / std::sqrt(harm(Kat(i - 1, nyp - 1, k), Kat(i, nyp - 1, k)));
        const double gg = beta / (beta + 2.0 / dy);
        const double cg = (gg * mu) * ((2.0 * Ay) / dy);
        const double gm = (gg * mu) * dz;
        double dd = ((((cx + cx) + (top ? cyt : cy)) + (gam ? cg : cy)) + (front ? czt : cz)) +
                    (back ? czt : cz);
        if (transient) dd = dd + mvol;
        rb.add(r, dd);
        if (i - 1 >= 1) rb.add(L.u3(i - 1, j, k), -cx);
        if (i + 1 <= nx - 1 || right_tr) rb.add(L.u3(i + 1, j, k), -cx);
        if (!top) rb.add(L.u3(i, j + 1, k), -cy);
        if (!gam) rb.add(L.u3(i, j - 1, k), -cy);
        if (!front) rb.add(L.u3(i, j, k + 1), -cz);
        if (!back) rb.add(L.u3(i, j, k - 1), -cz);
        if (!top) {
          rb.add(L.v3(i, j + 1, k), -mdz);
          rb.add(L.v3(i - 1, j + 1, k), mdz);
        }
        rb.add(L.v3(i, j, k), gam ? gm : mdz);
        rb.add(L.v3(i - 1, j, k), gam ? -gm : -mdz);
        if (!front) {
          rb.add(L.w3(i, j, k + 1), -mdy);
          rb.add(L.w3(i - 1, j, k + 1), mdy);
        }
        if (!back) {
          rb.add(L.w3(i, j, k), mdy);
          rb.add(L.w3(i - 1, j, k), -mdy);
        }
        rb.add(L.p3(i, j, k), Ax);
        rb.add(L.p3(i - 1, j, k), -Ax);
        if (ph->bj_full && gam) {   // porous tangential velocity in the slip condition
          const double Kf = harm(Kat(i - 1, nyp - 1, k), Kat(i, nyp - 1, k));
          const double cbj = cg * ((Kf / mu) / dx);
          rb.add(L.q3(i, nyp - 1, k), cbj);
          rb.add(L.q3(i - 1, nyp - 1, k), -cbj);
        }
        rb.finish();
        double rhs = d(fu, jk * (nx + 1) + i) * vol;
        if (i - 1 == 0) rhs = rhs + cx * d(uL, jk);
        if (!right_tr && i + 1 == nx) rhs = rhs + cx * d(uR, jk);
        if (top) rhs = rhs + cyt * d(uT, (int64_t)k * (nx + 1) + i);
        if (top) rhs = rhs + mdz * (d(vT, (int64_t)k * nx + i) - d(vT, (int64_t)k * nx + i - 1));
        if (back) rhs = rhs + czt * d(uB, (int64_t)j * (nx + 1) + i);
        if (back) rhs = rhs - mdy * (d(wB, (int64_t)j * nx + i) - d(wB, (int64_t)j * nx + i - 1));
        if (front) rhs = rhs + czt * d(uF, (int64_t)j * (nx + 1) + i);
        if (front) rhs = rhs + mdy * (d(wF, (int64_t)j * nx + i) - d(wF, (int64_t)j * nx + i - 1));
        P.b[r] = rhs;
      }
    }
  }
  // ---- v rows: Gamma (j = 0) then interior ----
  for (int j = 0; j < ny; ++j) {
    for (int k = 0; k < nz; ++k) {
      for (int i = 0; i < nx; ++i) {
        const int64_t r = L.v3(i, j, k);
        if (j == 0) {
          const double dg = ((mu / Kat(i, nyp - 1, k)) * (0.5 * dyp)) * Ay;
          rb.add(r, cyy + dg);
          rb.add(L.v3(i, 1, k), -cyy);
          rb.add(L.p3(i, 0, k), Ay);
          rb.add(L.q3(i, nyp - 1, k), -Ay);
          rb.finish();
          P.b[r] = 0.0;
          continue;
        }
        const bool west = i == 0, east = i == nx - 1, front = k == nz - 1, back = k == 0;
        const double aE = east ? (right_tr ? 0.0 : cxw) : cxv;
        const double aW = west ? cxw : cxv;
        double dd = ((((cyy + cyy) + aE) + aW) + (front ? czt : cz)) + (back ? czt : cz);
        if (transient) dd = dd + mvol;
        rb.add(r, dd);
        if (j + 1 <= ny - 1) rb.add(L.v3(i, j + 1, k), -cyy);
        rb.add(L.v3(i, j - 1, k), -cyy);
        if (!east) rb.add(L.v3(i + 1, j, k), -cxv);
        if (!west) rb.add(L.v3(i - 1, j, k), -cxv);
        if (!front) rb.add(L.v3(i, j, k + 1), -cz);
        if (!back) rb.add(L.v3(i, j, k - 1), -cz);
        if (i + 1 <= nx - 1) {
          rb.add(L.u3(i + 1, j, k), -mdz);
          rb.add(L.u3(i + 1, j - 1, k), mdz);
        }
        if (!west) {
          rb.add(L.u3(i, j, k), mdz);
          rb.add(L.u3(i, j - 1, k), -mdz);
        }
        if (!front) {
          rb.add(L.w3(i, j, k + 1), -mdx);
          rb.add(L.w3(i, j - 1, k + 1), mdx);
        }
        if (!back) {
          rb.add(L.w3(i, j, k), mdx);
          rb.add(L.w3(i, j - 1, k), -mdx);
        }
        rb.add(L.p3(i, j, k), Ay);
        rb.add(L.p3(i, j - 1, k), -Ay);
        rb.finish();
        const int64_t jk = (int64_t)j * nz + k, jm = (int64_t)(j - 1) * nz + k;
        double rhs = d(fv, jk * nx + i) * vol;
        if (j + 1 == ny) rhs = rhs + cyy * d(vT, (int64_t)k * nx + i);
        if (west) rhs = rhs + cxw * d(vL, jk);
        if (west) rhs = rhs - mdz * (d(uL, jk) - d(uL, jm));
        if (right_tr) {
          if (east) rhs = rhs - d(vR, jk) * Ax;
        } else {
          if (east) rhs = rhs + cxw * d(vR, jk);
          if (east) rhs = rhs + mdz * (d(uR, jk) - d(uR, jm));
        }
        if (back) rhs = rhs + czt * d(vB, (int64_t)j * nx + i);
        if (back) rhs = rhs - mdx * (d(wB, (int64_t)j * nx + i) - d(wB, (int64_t)(j - 1) * nx + i));
        if (front) rhs = rhs + czt * d(vF, (int64_t)j * nx + i);
        if (front) rhs = rhs + mdx * (d(wF, (int64_t)j * nx + i) - d(wF, (int64_t)(j - 1) * nx + i));
        P.b[r] = rhs;
      }
    }
  }
  // ---- w rows (interior z faces) ----
  for (int j = 0; j < ny; ++j) {
    for (int k = 1; k <= nz - 1; ++k) {
      for (int i = 0; i < nx; ++i) {
        const int64_t r = L.w3(i, j, k);
        const bool west = i == 0, east = i == nx - 1, top = j == ny - 1, gam = j == 0;
        const double beta = alpha / std::sqrt(harm(Kat(i, nyp - 1, k - 1), Kat(i, nyp - 1, k)));
        const double gg = beta / (beta + 2.0 / dy);
        const double cgw = (gg * mu) * ((2.0 * Ay) / dy);
        const double gmw = (gg * mu) * dx;
        const double aE = east ? (right_tr ? 0.0 : cxw) : cxv;
        const double aW = west ? cxw : cxv;
        double dd = ((((czz + czz) + aE) + aW) + (top ? cyt : cy)) + (gam ? cgw : cy);
        if (transient) dd = dd + mvol;
        rb.add(r, dd);
        if (k + 1 <= nz - 1) rb.add(L.w3(i, j, k + 1), -czz);
        if (k - 1 >= 1) rb.add(L.w3(i, j, k - 1), -czz);
        if (!east) rb.add(L.w3(i + 1, j, k), -cxv);
        if (!west) rb.add(L.w3(i - 1, j, k), -cxv);
        if (!top) rb.add(L.w3(i, j + 1, k), -cy);
        if (!gam) rb.add(L.w3(i, j - 1, k), -cy);
        if (i + 1 <= nx - 1) {
          rb.add(L.u3(i + 1, j, k), -mdy);
          rb.add(L.u3(i + 1, j, k - 1), mdy);
        }
        if (!west) {
          rb.add(L.u3(i, j, k), mdy);
          rb.add(L.u3(i, j, k - 1), -mdy);
        }
        if (!top) {
          rb.add(L.v3(i, j + 1, k), -mdx);
          rb.add(L.v3(i, j + 1, k - 1), mdx);
        }
        rb.add(L.v3(i, j, k), gam ? gmw : mdx);
        rb.add(L.v3(i, j, k - 1), gam ? -gmw : -mdx);
        rb.add(L.p3(i, j, k), Az);
        rb.add(L.p3(i, j, k - 1), -Az);
        if (ph->bj_full && gam) {
          const double Kf = harm(Kat(i, nyp - 1, k - 1), Kat(i, nyp - 1, k));
          const double cbj = cgw * ((Kf / mu) / dz);
          rb.add(L.q3(i, nyp - 1, k), cbj);
          rb.add(L.q3(i, nyp - 1, k - 1), -cbj);
        }
        rb.finish();
        const int64_t jz1 = (int64_t)j * (nz + 1) + k;
        double rhs = d(fw, jz1 * nx + i) * vol;
        if (k - 1 == 0) rhs = rhs + czz * d(wB, (int64_t)j * nx + i);
        if (k + 1 == nz) rhs = rhs + czz * d(wF, (int64_t)j * nx + i);
        if (top) rhs = rhs + cyt * d(wT, (int64_t)k * nx + i);
        if (top) rhs = rhs + mdx * (d(vT, (int64_t)k * nx + i) - d(vT, (int64_t)(k - 1) * nx + i));
        if (west) rhs = rhs + cxw * d(wL, jz1);
        if (west) rhs = rhs - mdy * (d(uL, (int64_t)j * nz + k) - d(uL, (int64_t)j * nz + k - 1));
        if (right_tr) {
          if (east) rhs = rhs - d(wR, jz1) * Ax;
        } else {
          if (east) rhs = rhs + cxw * d(wR, jz1);
          if (east)
            rhs = rhs + mdy * (d(uR, (int64_t)j * nz + k) - d(uR, (int64_t)j * nz + k - 1));
        }
        P.b[r] = rhs;
      }
    }
  }
  // ---- free-flow continuity ----
  for (int j = 0; j < ny; ++j) {
    for (int k = 0; k < nz; ++k) {
      for (int i = 0; i < nx; ++i) {
        const int64_t r = L.p3(i, j, k);
        if (i + 1 <= nx - 1 || right_tr) rb.add(L.u3(i + 1, j, k), Ax);
        if (i >= 1) rb.add(L.u3(i, j, k), -Ax);
        if (j + 1 <= ny - 1) rb.add(L.v3(i, j + 1, k), Ay);
        rb.add(L.v3(i, j, k), -Ay);
        if (k + 1 <= nz - 1) rb.add(L.w3(i, j, k + 1), Az);
        if (k >= 1) rb.add(L.w3(i, j, k), -Az);
        rb.finish();
        const int64_t jk = (int64_t)j * nz + k;
        double rhs = 0.0;
        if (i == 0) rhs = rhs + Ax * d(uL, jk);
        if (!right_tr && i + 1 == nx) rhs = rhs - Ax * d(uR, jk);
        if (j + 1 == ny) rhs = rhs - Ay * d(vT, (int64_t)k * nx + i);
        if (k == 0) rhs = rhs + Az * d(wB, (int64_t)j * nx + i);
        if (k + 1 == nz) rhs = rhs - Az * d(wF, (int64_t)j * nx + i);
        P.b[r] = rhs;
      }
    }
  }
  // ---- porous medium, six two-point fluxes ----
  const bool pr_d = bcs->pm_right == SD_BC_PRESSURE, pl_d = bcs->pm_left == SD_BC_PRESSURE;
  const bool pb_d = bcs->pm_bottom == SD_BC_PRESSURE;
  const bool pf_d = bcs->pm_front == SD_BC_PRESSURE, pk_d = bcs->pm_back == SD_BC_PRESSURE;
  const double Apx = dyp * dz, Apy = dx * dz, Apz = dx * dyp;
  for (int jj = 0; jj < nyp; ++jj) {
    for (int k = 0; k < nz; ++k) {
      for (int i = 0; i < nx; ++i) {
        const int64_t r = L.q3(i, jj, k);
        const double Kc = Kat(i, jj, k);
        auto t_int = [&](double area, double dd, double Kn) {
          return ((area / mu) * ((2.0 * Kc * Kn) / (Kc + Kn))) / dd;
        };
        auto t_dir = [&](double area, double dd) { return ((area / mu) * Kc) / (0.5 * dd); };
        const double TE = (i + 1 <= nx - 1) ? t_int(Apx, dx, Kat(i + 1, jj, k))
                                            : (pr_d ? t_dir(Apx, dx) : 0.0);
        const double TW = (i >= 1) ? t_int(Apx, dx, Kat(i - 1, jj, k))
                                   : (pl_d ? t_dir(Apx, dx) : 0.0);
        const double TN = (jj + 1 <= nyp - 1) ? t_int(Apy, dyp, Kat(i, jj + 1, k)) : 0.0;
        const double TS = (jj >= 1) ? t_int(Apy, dyp, Kat(i, jj - 1, k))
                                    : (pb_d ? t_dir(Apy, dyp) : 0.0);
        const double TF = (k + 1 <= nz - 1) ? t_int(Apz, dz, Kat(i, jj, k + 1))
                                            : (pf_d ? t_dir(Apz, dz) : 0.0);
        const double TB = (k >= 1) ? t_int(Apz, dz, Kat(i, jj, k - 1))
                                   : (pk_d ? t_dir(Apz, dz) : 0.0);
        rb.add(r, ((((TE + TW) + TN) + TS) + TF) + TB);
        if (i + 1 <= nx - 1) rb.add(L.q3(i + 1, jj, k), -TE);
        if (i >= 1) rb.add(L.q3(i - 1, jj, k), -TW);
        if (jj + 1 <= nyp - 1) rb.add(L.q3(i, jj + 1, k), -TN);
        if (jj >= 1) rb.add(L.q3(i, jj - 1, k), -TS);
        if (k + 1 <= nz - 1) rb.add(L.q3(i, jj, k + 1), -TF);
        if (k >= 1) rb.add(L.q3(i, jj, k - 1), -TB);
        if (jj == nyp - 1) rb.add(L.v3(i, 0, k), Ay);
        rb.finish();
        const int64_t jk = (int64_t)jj * nz + k;
        double rhs = d(fq, jk * nx + i) * volp;
        if (pr_d && i == nx - 1) rhs = rhs + TE * d(pR, jk);
        if (pl_d && i == 0) rhs = rhs + TW * d(pL, jk);
        if (pb_d && jj == 0) rhs = rhs + TS * d(pBo, (int64_t)k * nx + i);
        if (pf_d && k == nz - 1) rhs = rhs + TF * d(pFr, (int64_t)jj * nx + i);
        if (pk_d && k == 0) rhs = rhs + TB * d(pBk, (int64_t)jj * nx + i);
        P.b[r] = rhs;
      }
    }
  }
  if ((int64_t)A.rowptr.size() != L.N + 1) throw Error(SD_E_INVALID, "internal: row count");
}

}  // namespace sd
