// Partitioned Dirichlet-Neumann coupling on the GPU (Sec. 3 of the paper).
//
// The monolithic system is split into its free-flow part (velocity faces off
// Gamma, free-flow pressures) and its porous part.  One coupling iteration
// maps the interface normal velocity v (Dirichlet data of the free flow) to
//   sigma = p_{.,0} - 2 mu (v_{.,1} - v)/dy      (free-flow normal stress), then
//   vt    = (K_top/mu) (q_top - sigma)/(dy_pm/2)  (Darcy flux over the half cell)
// after a free-flow solve with v given and a porous solve whose top cells see
// sigma through the half-cell transmissibility TB = Ay K_top/(mu dy_pm/2).
// The fixed point S_pm(S_ff(v)) = v is accelerated by Aitken relaxation or by
// IQN-ILS (inverse Jacobian from a least-squares fit of the input/output
// history, Degroote, Bathe, Vierendeels 2009) and stops on the paper's two
// relative measures (interface pressure change, interface residual).  Both
// subdomain systems are solved by the same device solver as the monolithic
// one (block preconditioner with the empty block left out); the interface
// vectors (nx or nx nz values) live on the host.
#include <hip/hip_runtime.h>

#include <cmath>
#include <memory>
#include <vector>

#include "handles.h"
#include "sd.h"
#include "solver.h"

namespace sd {

namespace {

// Incremental QR of the IQN-ILS residual-difference matrix: columns are
// appended one per coupling iteration (earlier ones never change), each
// orthogonalised against the kept ones by classical Gram-Schmidt applied
// twice; a column left with less than 1e-12 of its norm depends on the
// earlier ones and is dropped together with its output difference.
struct IncrementalQR {
  int64_t m = 0;
  std::vector<std::vector<double>> q;    // orthonormal columns
  std::vector<std::vector<double>> rcol; // column t of R (length t + 1)
  std::vector<std::vector<double>> dv;   // output differences of kept columns
  void clear() { q.clear(); rcol.clear(); dv.clear(); }
  void append(const std::vector<double>& c0, const std::vector<double>& dvt) {
    std::vector<double> c = c0;
    const size_t k = q.size();
    std::vector<double> h(k + 1, 0.0);
    double n0 = 0.0;
    for (double x : c) n0 += x * x;
    n0 = std::sqrt(n0);
    if (!(n0 > 0.0)) return;
    for (int pass = 0; pass < 2; ++pass)
      for (size_t t = 0; t < k; ++t) {
        double d = 0.0;
        for (int64_t i = 0; i < m; ++i) d += q[t][(size_t)i] * c[(size_t)i];
        for (int64_t i = 0; i < m; ++i) c[(size_t)i] -= d * q[t][(size_t)i];
        h[t] += d;
      }
    double rho = 0.0;
    for (double x : c) rho += x * x;
    rho = std::sqrt(rho);
    if (rho <= 1e-12 * n0) return;
    for (double& x : c) x /= rho;
    h[k] = rho;
    q.push_back(std::move(c));
    rcol.push_back(std::move(h));
    dv.push_back(dvt);
  }
  // coefficients c of min ||dR c + r||: R c = -Q^T r
  std::vector<double> solve(const std::vector<double>& r) const {
    const size_t k = q.size();
    std::vector<double> y(k, 0.0), c(k, 0.0);
    for (size_t t = 0; t < k; ++t) {
      double d = 0.0;
      for (int64_t i = 0; i < m; ++i) d += q[t][(size_t)i] * r[(size_t)i];
      y[t] = -d;
    }
    for (size_t t = k; t-- > 0;) {
      double acc = y[t];
      for (size_t u = t + 1; u < k; ++u) acc -= rcol[u][t] * c[u];
      c[t] = acc / rcol[t][t];
    }
    return c;
  }
};

double norm2(const std::vector<double>& a) {
  double s = 0.0;
  for (double x : a) s += x * x;
  return std::sqrt(s);
}

}  // namespace

struct DNSolver {
  HostProblem ff, pm;
  std::unique_ptr<Solver> sff, spm;
  const HostProblem* mono = nullptr;
  int64_t nG = 0, g0 = 0, off_q = 0, N = 0, Nff = 0, Npm = 0;
  int64_t ff_p0 = 0, ff_v1 = 0, pm_top = 0;
  std::vector<double> TB, Kt;
  double dy = 0.0, dyp = 0.0, mu = 0.0;
  HostCSR AffG;             // -(free-flow rows x interface columns)
  std::unique_ptr<DeviceMem> mem;
  Sell<double> AffG_dev;
  double *b_ff = nullptr, *b_pm = nullptr, *rhs_ff = nullptr, *rhs_pm = nullptr;
  double *x_ff = nullptr, *x_pm = nullptr, *vG = nullptr, *tmp = nullptr;
  std::vector<double> b_pm_top;

  void build(const HostProblem& P, const sd_solver_opts* o, const sd_allocator* alloc,
             hipStream_t s);
  int solve(const sd_dn_opts& d, const double* d_b, double* d_x, sd_dn_stats* st,
            hipStream_t s);
};

void DNSolver::build(const HostProblem& P, const sd_solver_opts* o, const sd_allocator* alloc,
                     hipStream_t s) {
  mono = &P;
  const Layout& L = P.L;
  nG = L.n_gamma();
  g0 = L.off_v;
  off_q = L.off_q;
  N = L.N;
  Nff = off_q - nG;
  Npm = N - off_q;
  const double dz = L.nz > 0 ? P.grid.Lz / (double)P.grid.nz : 1.0;
  const double dx = P.grid.Lx / (double)P.grid.nx;
  const double Ay = dx * dz;
  dy = P.grid.H_ff / (double)P.grid.ny;
  dyp = P.grid.H_pm / (double)P.grid.ny_pm;
  mu = P.phys.mu;
  // ---- free-flow subsystem: rows/columns [0, off_q) without Gamma faces
  auto ffcol = [&](int64_t c) { return c < g0 ? c : c - nG; };
  ff = HostProblem();
  ff.grid = P.grid;
  ff.phys = P.phys;
  ff.mass = P.mass;
  ff.L = L;
  ff.L.off_w = L.off_w - nG;
  ff.L.off_p = L.off_p - nG;
  ff.L.off_q = L.off_q - nG;
  ff.L.N = Nff;
  ff.L.gamma_rows = false;
  ff.A.n_rows = ff.A.n_cols = Nff;
  ff.A.rowptr.assign(1, 0);
  AffG.n_rows = Nff;
  AffG.n_cols = nG;
  AffG.rowptr.assign(1, 0);
  for (int64_t r = 0; r < off_q; ++r) {
    if (r >= g0 && r < g0 + nG) continue;
    for (int64_t k = P.A.rowptr[r]; k < P.A.rowptr[r + 1]; ++k) {
      const int64_t c = P.A.col[k];
      if (c >= off_q) throw Error(SD_E_INVALID, "internal: free-flow row couples to the porous block");
      if (c >= g0 && c < g0 + nG) {
        AffG.col.push_back((int32_t)(c - g0));
        AffG.val.push_back(-P.A.val[k]);
      } else {
        ff.A.col.push_back((int32_t)ffcol(c));
        ff.A.val.push_back(P.A.val[k]);
      }
    }
    ff.A.rowptr.push_back((int64_t)ff.A.col.size());
    AffG.rowptr.push_back((int64_t)AffG.col.size());
    ff.b.push_back(P.b[(size_t)r]);
  }
  // ---- porous subsystem with the half-cell transmissibility on top cells
  pm = HostProblem();
  pm.grid = P.grid;
  pm.phys = P.phys;
  pm.L = L;
  pm.L.off_v = pm.L.off_w = pm.L.off_p = pm.L.off_q = 0;
  pm.L.N = Npm;
  pm.A.n_rows = pm.A.n_cols = Npm;
  pm.A.rowptr.assign(1, 0);
  pm_top = (int64_t)(L.nyp - 1) * nG;       // top porous layer, in interface order
  for (int64_t r = off_q; r < N; ++r) {
    for (int64_t k = P.A.rowptr[r]; k < P.A.rowptr[r + 1]; ++k) {
      const int64_t c = P.A.col[k];
      if (c < off_q) continue;   // interface flux column: replaced by the coupling
      pm.A.col.push_back((int32_t)(c - off_q));
      pm.A.val.push_back(P.A.val[k]);
    }
    pm.A.rowptr.push_back((int64_t)pm.A.col.size());
    pm.b.push_back(P.b[(size_t)r]);
  }
  // permeability of the porous top cell under each interface face (the top
  // layer of K, in the interface order) and its half-cell transmissibility
  TB.assign((size_t)nG, 0.0);
  Kt.assign(P.K.begin() + (size_t)((int64_t)(L.nyp - 1) * nG), P.K.begin() + (size_t)(L.nyp * nG));
  for (int64_t g = 0; g < nG; ++g) TB[(size_t)g] = (Ay * Kt[(size_t)g]) / ((mu * 0.5) * dyp);
  for (int64_t g = 0; g < nG; ++g) {
    const int64_t rr = pm_top + g;
    for (int64_t k = pm.A.rowptr[rr]; k < pm.A.rowptr[rr + 1]; ++k)
      if (pm.A.col[k] == rr) pm.A.val[k] = pm.A.val[k] + TB[(size_t)g];
  }
  ff_p0 = ff.L.off_p + L.i0;   // p(., 0) over the block in the free-flow subsystem
  ff_v1 = ff.L.off_v + L.i0;   // v(., 1) over the block
  // ---- sub-solvers and device buffers
  // the free-flow subsystem keeps the requested middle block (the
  // Cahouet-Chabard one needs its backward-Euler mass); the porous
  // subsystem has no pressure-velocity block, so it takes the default
  sd_solver_opts so = *o;
  if (so.schur == SD_SCHUR_CC && !(ff.mass > 0.0)) so.schur = SD_SCHUR_MASS;
  sd_solver_opts so_pm = so;
  if (so_pm.schur == SD_SCHUR_CC) so_pm.schur = SD_SCHUR_MASS;
  sff.reset(new Solver());
  sff->setup_host(&ff, &so);
  sff->upload(alloc, s);
  spm.reset(new Solver());
  spm->setup_host(&pm, &so_pm);
  spm->upload(alloc, s);
  mem.reset(new DeviceMem(alloc, s));
  AffG_dev = upload_sell<double>(AffG, *mem, s);
  b_ff = sff->b_dev;
  b_pm = spm->b_dev;
  rhs_ff = mem->array<double>((size_t)Nff);
  rhs_pm = mem->array<double>((size_t)Npm);
  x_ff = mem->array<double>((size_t)Nff);
  x_pm = mem->array<double>((size_t)Npm);
  vG = mem->array<double>((size_t)nG);
  tmp = mem->array<double>((size_t)Nff);
  b_pm_top.assign(pm.b.begin() + pm_top, pm.b.begin() + pm_top + nG);
  SD_HIP(hipStreamSynchronize(s));
}

int DNSolver::solve(const sd_dn_opts& d, const double* d_b, double* d_x, sd_dn_stats* out,
                    hipStream_t s) {
  TraceRange trace("sd: partitioned coupling");
  const double t0 = wall_time();
  sd_dn_stats st{};
  // right-hand sides of the subsystems: the assembled ones or slices of d_b
  if (d_b) {
    std::vector<double> bg((size_t)nG);
    SD_HIP(hipMemcpyAsync(bg.data(), d_b + g0, (size_t)nG * 8, hipMemcpyDeviceToHost, s));
    SD_HIP(hipStreamSynchronize(s));
    for (double x : bg)
      if (x != 0.0) throw Error(SD_E_INVALID, "interface rows of b must be zero");
    SD_HIP(hipMemcpyAsync(b_ff, d_b, (size_t)g0 * 8, hipMemcpyDeviceToDevice, s));
    SD_HIP(hipMemcpyAsync(b_ff + g0, d_b + g0 + nG, (size_t)(off_q - g0 - nG) * 8,
                          hipMemcpyDeviceToDevice, s));
    SD_HIP(hipMemcpyAsync(b_pm, d_b + off_q, (size_t)Npm * 8, hipMemcpyDeviceToDevice, s));
    SD_HIP(hipMemcpyAsync(b_pm_top.data(), d_b + off_q + pm_top, (size_t)nG * 8,
                          hipMemcpyDeviceToHost, s));
  } else {
    SD_HIP(hipMemcpyAsync(b_ff, ff.b.data(), (size_t)Nff * 8, hipMemcpyHostToDevice, s));
    SD_HIP(hipMemcpyAsync(b_pm, pm.b.data(), (size_t)Npm * 8, hipMemcpyHostToDevice, s));
    b_pm_top.assign(pm.b.begin() + pm_top, pm.b.begin() + pm_top + nG);
  }
  SD_HIP(hipMemsetAsync(x_ff, 0, (size_t)Nff * 8, s));
  SD_HIP(hipMemsetAsync(x_pm, 0, (size_t)Npm * 8, s));
  SD_HIP(hipStreamSynchronize(s));
  std::vector<double> v((size_t)nG, 0.0), sigma((size_t)nG), vt((size_t)nG), r((size_t)nG);
  std::vector<double> sigma_old, r_old, top((size_t)nG), p0((size_t)nG), v1((size_t)nG);
  std::vector<double> r_prev, vt_prev;
  IncrementalQR qr;
  qr.m = nG;
  double omega = d.omega0;
  int status = SD_E_NOCONV;
  for (int k = 1; k <= d.maxit; ++k) {
    st.iters = k;
    // free flow with Dirichlet interface velocity v
    SD_HIP(hipMemcpyAsync(vG, v.data(), (size_t)nG * 8, hipMemcpyHostToDevice, s));
    launch_spmv<double, double, double>(AffG_dev, vG, tmp, nullptr, s);
    SD_HIP(hipMemcpyAsync(rhs_ff, b_ff, (size_t)Nff * 8, hipMemcpyDeviceToDevice, s));
    launch_add<double>(tmp, rhs_ff, (int)Nff, nullptr, s);
    SD_HIP(hipGetLastError());
    sd_stats a{};
    const int rc1 = sff->solve(rhs_ff, x_ff, 1, &a, s);
    st.ff_iters += a.iters;
    if (rc1 != SD_OK) {
      status = rc1;
      break;
    }
    SD_HIP(hipMemcpyAsync(p0.data(), x_ff + ff_p0, (size_t)nG * 8, hipMemcpyDeviceToHost, s));
    SD_HIP(hipMemcpyAsync(v1.data(), x_ff + ff_v1, (size_t)nG * 8, hipMemcpyDeviceToHost, s));
    SD_HIP(hipStreamSynchronize(s));
    for (int64_t g = 0; g < nG; ++g) sigma[g] = p0[g] - 2.0 * mu * (v1[g] - v[g]) / dy;
    // porous medium with the interface stress sigma
    for (int64_t g = 0; g < nG; ++g) top[g] = b_pm_top[g] + TB[g] * sigma[g];
    SD_HIP(hipMemcpyAsync(rhs_pm, b_pm, (size_t)Npm * 8, hipMemcpyDeviceToDevice, s));
    SD_HIP(hipMemcpyAsync(rhs_pm + pm_top, top.data(), (size_t)nG * 8, hipMemcpyHostToDevice, s));
    sd_stats b{};
    const int rc2 = spm->solve(rhs_pm, x_pm, 1, &b, s);
    st.pm_iters += b.iters;
    if (rc2 != SD_OK) {
      status = rc2;
      break;
    }
    SD_HIP(hipMemcpyAsync(top.data(), x_pm + pm_top, (size_t)nG * 8, hipMemcpyDeviceToHost, s));
    SD_HIP(hipStreamSynchronize(s));
    for (int64_t g = 0; g < nG; ++g) vt[g] = (Kt[g] / mu) * (top[g] - sigma[g]) / (0.5 * dyp);
    for (int64_t g = 0; g < nG; ++g) r[g] = vt[g] - v[g];
    // the paper's stopping rule on the interface pressure and velocity
    bool ok_p = false;
    if (!sigma_old.empty()) {
      std::vector<double> ds((size_t)nG);
      for (int64_t g = 0; g < nG; ++g) ds[g] = sigma[g] - sigma_old[g];
      ok_p = norm2(ds) < d.eps * norm2(sigma);
    }
    const bool ok_v = norm2(r) < d.eps * norm2(vt);
    st.dv_rel = norm2(r) / norm2(vt);
    if (!sigma_old.empty()) {
      double dd = 0.0;
      for (int64_t g = 0; g < nG; ++g) dd += (sigma[g] - sigma_old[g]) * (sigma[g] - sigma_old[g]);
      st.dp_rel = std::sqrt(dd) / norm2(sigma);
    }
    if (ok_p && ok_v) {
      st.converged = 1;
      status = SD_OK;
      break;
    }
    if (d.accel == SD_DN_AITKEN) {
      if (!r_old.empty()) {
        double num = 0.0, den = 0.0;
        for (int64_t g = 0; g < nG; ++g) {
          const double dr = r[g] - r_old[g];
          num += r_old[g] * dr;
          den += dr * dr;
        }
        omega = den > 0.0 ? -omega * num / den : d.omega0;
      }
      for (int64_t g = 0; g < nG; ++g) v[g] = v[g] + omega * r[g];
    } else {
      // IQN-ILS: secant pairs (r_k - r_{k-1}, vt_k - vt_{k-1}); the next input
      // is vt_k + dVt c with c = argmin ||dR c + r_k||; the first iteration
      // relaxes with omega0
      if (!r_prev.empty()) {
        std::vector<double> dr((size_t)nG), dvt((size_t)nG);
        for (int64_t g = 0; g < nG; ++g) {
          dr[g] = r[g] - r_prev[g];
          dvt[g] = vt[g] - vt_prev[g];
        }
        qr.append(dr, dvt);
      }
      if (qr.q.empty()) {
        for (int64_t g = 0; g < nG; ++g) v[g] = v[g] + d.omega0 * r[g];
      } else {
        const std::vector<double> cf = qr.solve(r);
        for (int64_t g = 0; g < nG; ++g) {
          double acc = vt[g];
          for (size_t c = 0; c < cf.size(); ++c) acc += qr.dv[c][(size_t)g] * cf[c];
          v[g] = acc;
        }
      }
      r_prev = r;
      vt_prev = vt;
    }
    r_old = r;
    sigma_old = sigma;
  }
  // monolithic solution from the subsystem states and the interface velocity
  SD_HIP(hipMemcpyAsync(d_x, x_ff, (size_t)g0 * 8, hipMemcpyDeviceToDevice, s));
  SD_HIP(hipMemcpyAsync(d_x + g0, v.data(), (size_t)nG * 8, hipMemcpyHostToDevice, s));
  SD_HIP(hipMemcpyAsync(d_x + g0 + nG, x_ff + g0, (size_t)(Nff - g0) * 8,
                        hipMemcpyDeviceToDevice, s));
  SD_HIP(hipMemcpyAsync(d_x + off_q, x_pm, (size_t)Npm * 8, hipMemcpyDeviceToDevice, s));
  SD_HIP(hipStreamSynchronize(s));
  st.t_solve = wall_time() - t0;
  if (out) *out = st;
  return status;
}

}  // namespace sd

struct sd_dn {
  sd::DNSolver dn;
  sd_problem* pb = nullptr;
};

extern "C" {

void sd_dn_opts_default(sd_dn_opts* o) {
  if (!o) return;
  o->accel = SD_DN_IQN_ILS;
  o->eps = 1e-8;
  o->maxit = 200;
  o->omega0 = 0.5;
}

int sd_dn_setup(sd_problem* pb, const sd_solver_opts* sub, sd_dn** out) {
  return sd::guarded_call([&] {
    if (!pb || !out) throw sd::Error(SD_E_INVALID, "NULL argument");
    *out = nullptr;
    if (!pb->device) throw sd::Error(SD_E_INVALID, "problem was assembled without a device");
    if (pb->hp.phys.bj_full)
      throw sd::Error(SD_E_INVALID, "the partitioned coupling supports the BJS condition only");
    SD_HIP(hipSetDevice(pb->device_id));
    sd_solver_opts d;
    sd_solver_opts_default(&d);
    std::unique_ptr<sd_dn> h(new sd_dn());
    h->pb = pb;
    h->dn.build(pb->hp, sub ? sub : &d, pb->has_alloc ? &pb->alloc : nullptr, pb->stream);
    *out = h.release();
    return (int)SD_OK;
  });
}

int sd_dn_solve(sd_dn* h, const sd_dn_opts* o, const double* d_b, double* d_x, sd_dn_stats* st,
                void* hip_stream) {
  return sd::guarded_call([&] {
    if (!h || !d_x) throw sd::Error(SD_E_INVALID, "NULL argument");
    sd_dn_opts d;
    sd_dn_opts_default(&d);
    if (o) d = *o;
    if (d.accel != SD_DN_AITKEN && d.accel != SD_DN_IQN_ILS)
      throw sd::Error(SD_E_INVALID, "accel must be SD_DN_AITKEN or SD_DN_IQN_ILS");
    if (!(d.eps > 0.0) || d.maxit < 1 || !(d.omega0 > 0.0))
      throw sd::Error(SD_E_INVALID, "eps > 0, maxit >= 1 and omega0 > 0 required");
    SD_HIP(hipSetDevice(h->pb->device_id));
    const int rc = h->dn.solve(d, d_b, d_x, st, (hipStream_t)hip_stream);
    if (rc == SD_E_NOCONV) sd::set_last_error("coupling iteration did not converge");
    return rc;
  });
}

void sd_dn_destroy(sd_dn* h) {
  if (!h) return;
  if (h->pb && h->pb->device) (void)hipSetDevice(h->pb->device_id);
  delete h;
}

}  // extern "C"
