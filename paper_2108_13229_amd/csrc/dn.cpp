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

// Least squares min ||M c + r|| by Householder QR of the m x k matrix M
// (column-major); a column whose remaining norm falls below 1e-12 ||M||_F
// (dependent on the earlier ones) is dropped and gets coefficient 0.
std::vector<double> lsq(std::vector<double> M, int64_t m, int k, std::vector<double> r) {
  double fro = 0.0;
  for (double x : M) fro += x * x;
  fro = std::sqrt(fro);
  for (auto& x : r) x = -x;
  std::vector<std::vector<double>> hv;   // Householder vectors of kept columns
  std::vector<int> cols;
  for (int j = 0; j < k; ++j) {
    double* a = &M[(size_t)j * m];
    for (size_t t = 0; t < hv.size(); ++t) {   // apply earlier reflections
      const std::vector<double>& v = hv[t];
      const int64_t o = (int64_t)t;
      double d = 0.0;
      for (int64_t i = o; i < m; ++i) d += v[(size_t)(i - o)] * a[i];
      for (int64_t i = o; i < m; ++i) a[i] -= 2.0 * d * v[(size_t)(i - o)];
    }
    const int64_t o = (int64_t)hv.size();
    double nrm = 0.0;
    for (int64_t i = o; i < m; ++i) nrm += a[i] * a[i];
    nrm = std::sqrt(nrm);
    if (nrm <= 1e-12 * fro || o >= m) continue;          // dependent column
    std::vector<double> v((size_t)(m - o));
    const double alpha = a[o] > 0 ? -nrm : nrm;
    for (int64_t i = o; i < m; ++i) v[(size_t)(i - o)] = a[i];
    v[0] -= alpha;
    double vn = 0.0;
    for (double x : v) vn += x * x;
    vn = std::sqrt(vn);
    for (double& x : v) x /= vn;
    for (int64_t i = o; i < m; ++i) a[i] = i == o ? alpha : 0.0;
    hv.push_back(std::move(v));
    cols.push_back(j);
  }
  const int kk = (int)hv.size();
  for (int t = 0; t < kk; ++t) {                      // Q^T (-r)
    const std::vector<double>& v = hv[(size_t)t];
    double d = 0.0;
    for (int64_t i = t; i < m; ++i) d += v[(size_t)(i - t)] * r[(size_t)i];
    for (int64_t i = t; i < m; ++i) r[(size_t)i] -= 2.0 * d * v[(size_t)(i - t)];
  }
  std::vector<double> y((size_t)kk, 0.0);
  for (int t = kk - 1; t >= 0; --t) {                 // R y = (Q^T (-r))_{0..kk-1}
    double acc = r[(size_t)t];
    for (int u = t + 1; u < kk; ++u) acc -= M[(size_t)cols[(size_t)u] * m + t] * y[(size_t)u];
    y[(size_t)t] = acc / M[(size_t)cols[(size_t)t] * m + t];
  }
  std::vector<double> c((size_t)k, 0.0);
  for (int t = 0; t < kk; ++t) c[(size_t)cols[(size_t)t]] = y[(size_t)t];
  return c;
}

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
  const int nzc = L.nzc();
  nG = (int64_t)L.nx * nzc;
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
  pm_top = (int64_t)(L.nyp - 1) * nzc * L.nx;
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
  ff_p0 = ff.L.off_p;      // p(., 0) rows of the free-flow subsystem
  ff_v1 = ff.L.off_v;      // v(., 1) rows
  // ---- sub-solvers and device buffers
  sd_solver_opts so = *o;
  if (so.schur == SD_SCHUR_CC) so.schur = SD_SCHUR_MASS;
  sff.reset(new Solver());
  sff->setup_host(&ff, &so);
  sff->upload(alloc, s);
  spm.reset(new Solver());
  spm->setup_host(&pm, &so);
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
  std::vector<std::vector<double>> Rh, Vh;
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
      Rh.push_back(r);
      Vh.push_back(vt);
      if (Rh.size() == 1) {
        for (int64_t g = 0; g < nG; ++g) v[g] = v[g] + d.omega0 * r[g];
      } else {
        const int kc = (int)Rh.size() - 1;
        std::vector<double> dR((size_t)nG * kc), dV((size_t)nG * kc);
        for (int c = 0; c < kc; ++c)
          for (int64_t g = 0; g < nG; ++g) {
            dR[(size_t)c * nG + g] = Rh[c + 1][g] - Rh[c][g];
            dV[(size_t)c * nG + g] = Vh[c + 1][g] - Vh[c][g];
          }
        const std::vector<double> cf = lsq(dR, nG, kc, r);
        for (int64_t g = 0; g < nG; ++g) {
          double acc = vt[g];
          for (int c = 0; c < kc; ++c) acc += dV[(size_t)c * nG + g] * cf[(size_t)c];
          v[g] = acc;
        }
      }
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
