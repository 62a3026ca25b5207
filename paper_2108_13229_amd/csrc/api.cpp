// C ABI of the Stokes-Darcy library: handles, error reporting, argument checks.
#include <hip/hip_runtime.h>

#include <cmath>
#include <memory>
#include <string>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "handles.h"
#include "sd.h"
#include "solver.h"

namespace sd {
TraceRange::TraceRange(const char* name) { roctxRangePushA(name); }
TraceRange::~TraceRange() { roctxRangePop(); }
}  // namespace sd

struct sd_solver {
  std::unique_ptr<sd::Solver> s;
  sd_problem* pb = nullptr;
};

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

template <typename F>
int guarded(F&& f) {
  return sd::guarded_call(std::forward<F>(f));
}

int require_device() {
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) {
    (void)hipGetLastError();
    throw sd::Error(SD_E_DEVICE, "no HIP device available");
  }
  int d = 0;
  SD_HIP(hipGetDevice(&d));
  return d;
}

}  // namespace

void sd::set_last_error(const std::string& msg) { g_err = msg; }

extern "C" {

const char* sd_status_string(int status) {
  switch (status) {
    case SD_OK: return "SD_OK";
    case SD_E_INVALID: return "SD_E_INVALID";
    case SD_E_NOMEM: return "SD_E_NOMEM";
    case SD_E_DEVICE: return "SD_E_DEVICE";
    case SD_E_NOCONV: return "SD_E_NOCONV";
    case SD_E_BREAKDOWN: return "SD_E_BREAKDOWN";
    case SD_E_BUSY: return "SD_E_BUSY";
    case SD_E_NOTFOUND: return "SD_E_NOTFOUND";
    default: return "unknown status";
  }
}

const char* sd_last_error(void) { return g_err.c_str(); }

void sd_solver_opts_default(sd_solver_opts* o) {
  if (!o) return;
  o->krylov = SD_KRYLOV_FGMRES;
  o->restart = 30;
  o->maxit = 1000;
  o->tol = 1e-8;
  o->precond = SD_PREC_BGS;
  o->schur = SD_SCHUR_MASS;
  o->precision = SD_PRECISION_FP64;
  o->amg = SD_AMG_SMOOTHED;
  o->mis = 2;
  o->theta = 0.08;
  o->omega = 2.0 / 3.0;
  o->nu_pre = 2;
  o->nu_post = 2;
  o->coarse_max = 2048;
  o->max_levels = 20;
  o->darcy = SD_DARCY_AMG;
  o->pd_m_init = 3;
  o->pd_m_min = 3;
  o->pd_m_step = 5;
  o->pd_alpha_p = -3.0;
  o->pd_alpha_d = 5.0;
  o->stencil_slices = 1;
  o->fused_restriction = 1;
}

static int assemble_impl(const sd_grid* grid, const sd_physics* phys, const sd_bcs* bcs,
                         const double* K, const sd_forcing* forcing, bool device,
                         const sd_allocator* alloc, void* stream, sd_problem** out) {
  return guarded([&] {
    if (!out) return fail(SD_E_INVALID, "out is NULL");
    *out = nullptr;
    std::unique_ptr<sd_problem> p(new sd_problem());
    if (device) {
      p->device_id = require_device();
      p->device = true;
      if (alloc && alloc->alloc && alloc->free) {
        p->alloc = *alloc;
        p->has_alloc = true;
      }
      p->stream = (hipStream_t)stream;
    }
    sd::assemble_host(grid, phys, bcs, K, forcing, p->hp);
    *out = p.release();
    return (int)SD_OK;
  });
}

int sd_assemble(const sd_grid* grid, const sd_physics* phys, const sd_bcs* bcs, const double* K,
                const sd_forcing* forcing, const sd_allocator* allocator, void* hip_stream,
                sd_problem** out) {
  return assemble_impl(grid, phys, bcs, K, forcing, true, allocator, hip_stream, out);
}

int sd_assemble_host(const sd_grid* grid, const sd_physics* phys, const sd_bcs* bcs,
                     const double* K, const sd_forcing* forcing, sd_problem** out) {
  return assemble_impl(grid, phys, bcs, K, forcing, false, nullptr, nullptr, out);
}

int sd_problem_info(const sd_problem* pb, int64_t* N, int64_t block_off[5], int64_t* nnz) {
  if (!pb) return fail(SD_E_INVALID, "problem is NULL");
  const sd::Layout& L = pb->hp.L;
  if (N) *N = L.N;
  if (block_off) {
    block_off[0] = 0;
    block_off[1] = L.off_v;
    block_off[2] = L.off_p;
    block_off[3] = L.off_q;
    block_off[4] = L.N;
  }
  if (nnz) *nnz = pb->hp.A.nnz();
  return SD_OK;
}

int sd_problem_csr(const sd_problem* pb, const int64_t** rowptr, const int32_t** col,
                   const double** val, const double** b) {
  if (!pb) return fail(SD_E_INVALID, "problem is NULL");
  if (rowptr) *rowptr = pb->hp.A.rowptr.data();
  if (col) *col = pb->hp.A.col.data();
  if (val) *val = pb->hp.A.val.data();
  if (b) *b = pb->hp.b.data();
  return SD_OK;
}

static int setup_impl(sd_problem* pb, const sd_solver_opts* opts, bool device, sd_solver** out) {
  return guarded([&] {
    if (!pb || !out) return fail(SD_E_INVALID, "NULL argument");
    *out = nullptr;
    if (device && !pb->device)
      return fail(SD_E_INVALID, "problem was assembled without a device (sd_assemble_host)");
    std::unique_ptr<sd_solver> s(new sd_solver());
    s->pb = pb;
    s->s.reset(new sd::Solver());
    s->s->setup_host(&pb->hp, opts);
    if (device) {
      SD_HIP(hipSetDevice(pb->device_id));
      s->s->upload(pb->has_alloc ? &pb->alloc : nullptr, pb->stream);
    }
    *out = s.release();
    return (int)SD_OK;
  });
}

int sd_setup(sd_problem* pb, const sd_solver_opts* opts, sd_solver** out) {
  return setup_impl(pb, opts, true, out);
}

int sd_setup_host(sd_problem* pb, const sd_solver_opts* opts, sd_solver** out) {
  return setup_impl(pb, opts, false, out);
}

int sd_solver_levels(const sd_solver* s, int block, int* n_levels) {
  if (!s || block < 0 || block > 2 || !n_levels) return fail(SD_E_INVALID, "bad argument");
  *n_levels = (int)s->s->hh[block].levels.size();
  return SD_OK;
}

int sd_solver_level_csr(const sd_solver* s, int block, int level, int which, int64_t* n_rows,
                        int64_t* n_cols, const int64_t** rowptr, const int32_t** col,
                        const double** val) {
  if (!s || block < 0 || block > 2) return fail(SD_E_INVALID, "bad argument");
  const auto& h = s->s->hh[block];
  if (level < 0 || level >= (int)h.levels.size()) return fail(SD_E_INVALID, "bad level");
  const sd::HostLevel& L = h.levels[(size_t)level];
  const sd::HostCSR* M = which == 0 ? &L.A : which == 1 ? &L.P : which == 2 ? &L.R : nullptr;
  if (!M) return fail(SD_E_INVALID, "which must be 0, 1 or 2");
  if (which != 0 && level + 1 == (int)h.levels.size())
    return fail(SD_E_INVALID, "the coarsest level has no transfer operators");
  if (n_rows) *n_rows = M->n_rows;
  if (n_cols) *n_cols = M->n_cols;
  if (rowptr) *rowptr = M->rowptr.data();
  if (col) *col = M->col.data();
  if (val) *val = M->val.data();
  return SD_OK;
}

int sd_solver_ilu(const sd_solver* s, int lower, int64_t* n, int* n_levels,
                  const int32_t** lev, const int32_t** ord, const int32_t** col,
                  const double** val, const double** diag) {
  if (!s) return fail(SD_E_INVALID, "bad argument");
  const sd::HostIlu& f = s->s->ilu;
  if (f.n == 0) return fail(SD_E_INVALID, "the solver has no ILU(0) factors");
  if (n) *n = f.n;
  if (n_levels) *n_levels = (int)(lower ? f.lev_l.size() : f.lev_u.size()) - 1;
  if (lev) *lev = lower ? f.lev_l.data() : f.lev_u.data();
  if (ord) *ord = lower ? f.ord_l.data() : f.ord_u.data();
  if (col) *col = lower ? f.col_l.data() : f.col_u.data();
  if (val) *val = lower ? f.val_l.data() : f.val_u.data();
  if (diag) *diag = lower ? nullptr : f.diag_u.data();
  return SD_OK;
}

int sd_solver_level_agg(const sd_solver* s, int block, int level, const int32_t** agg,
                        int64_t* n) {
  if (!s || block < 0 || block > 2) return fail(SD_E_INVALID, "bad argument");
  const auto& h = s->s->hh[block];
  if (level < 0 || level + 1 >= (int)h.levels.size())
    return fail(SD_E_INVALID, "bad level (the coarsest level has no aggregates)");
  if (agg) *agg = h.levels[(size_t)level].agg.data();
  if (n) *n = (int64_t)h.levels[(size_t)level].agg.size();
  return SD_OK;
}

int sd_solver_coarse_inverse(const sd_solver* s, int block, const double** inv, int64_t* n) {
  if (!s || block < 0 || block > 2) return fail(SD_E_INVALID, "bad argument");
  if (s->s->hh[block].levels.empty()) return fail(SD_E_INVALID, "block has no hierarchy");
  if (inv) *inv = s->s->hh[block].Ainv.data();
  if (n) *n = s->s->hh[block].n_coarse;
  return SD_OK;
}

int sd_solve(sd_solver* s, const double* d_b, double* d_x, int use_x0, sd_stats* stats,
             void* hip_stream) {
  return guarded([&] {
    if (!s) return fail(SD_E_INVALID, "solver is NULL");
    SD_HIP(hipSetDevice(s->pb->device_id));
    const int rc = s->s->solve(d_b, d_x, use_x0, stats, (hipStream_t)hip_stream);
    if (rc == SD_E_NOCONV) g_err = "maximum number of iterations reached";
    if (rc == SD_E_BREAKDOWN) g_err = "non-finite value or zero pivot in the iteration";
    return rc;
  });
}

static void step_rhs_impl(sd_solver* s, const double* d_b, const double* d_x, double* d_out,
                          hipStream_t st) {
  const sd::HostProblem& hp = s->pb->hp;
  if (!(hp.mass > 0.0))
    throw sd::Error(SD_E_INVALID, "problem is stationary (assembled with phys.dt = 0)");
  if (!s->s->on_device) throw sd::Error(SD_E_INVALID, "solver has no device data");
  if (!d_x || !d_out) throw sd::Error(SD_E_INVALID, "NULL device vector");
  const sd::Layout& L = hp.L;
  sd::launch_step_rhs(d_b ? d_b : s->s->b_dev, d_x, d_out, hp.mass, (int)L.N, L.nux, L.i_first,
                      L.nx, (int)L.off_v, (int)L.n_gamma(), (int)L.off_w, (int)L.off_p, st);
  SD_HIP(hipGetLastError());
}

int sd_step_rhs(sd_solver* s, const double* d_b_data, const double* d_x_prev, double* d_b_out,
                void* hip_stream) {
  return guarded([&] {
    if (!s) return fail(SD_E_INVALID, "solver is NULL");
    SD_HIP(hipSetDevice(s->pb->device_id));
    step_rhs_impl(s, d_b_data, d_x_prev, d_b_out, (hipStream_t)hip_stream);
    return (int)SD_OK;
  });
}

int sd_advance(sd_solver* s, const double* d_b_data, double* d_x, int n_steps, sd_stats* stats,
               int* steps_done, void* hip_stream) {
  return guarded([&] {
    if (steps_done) *steps_done = 0;
    if (!s) return fail(SD_E_INVALID, "solver is NULL");
    if (n_steps < 0) return fail(SD_E_INVALID, "n_steps must be >= 0");
    SD_HIP(hipSetDevice(s->pb->device_id));
    sd::Solver& S = *s->s;
    hipStream_t st = (hipStream_t)hip_stream;
    for (int k = 0; k < n_steps; ++k) {
      step_rhs_impl(s, d_b_data, d_x, S.step_b, st);
      sd_stats one{};
      const int rc = S.solve(S.step_b, d_x, 1, &one, st);
      if (stats) stats[k] = one;
      if (rc != SD_OK) {
        if (rc == SD_E_NOCONV) g_err = "a time step reached the maximum number of iterations";
        if (rc == SD_E_BREAKDOWN) g_err = "non-finite value or zero pivot in a time step";
        return rc;
      }
      if (steps_done) *steps_done = k + 1;
    }
    return (int)SD_OK;
  });
}

int sd_apply_matrix(sd_solver* s, const double* d_x, double* d_y, void* hip_stream) {
  return guarded([&] {
    if (!s || !d_x || !d_y) return fail(SD_E_INVALID, "NULL argument");
    if (!s->s->on_device) return fail(SD_E_INVALID, "solver has no device data");
    hipStream_t st = (hipStream_t)hip_stream;
    sd::launch_spmv<double, double, double>(s->s->A64, d_x, d_y, nullptr, st);
    SD_HIP(hipGetLastError());
    SD_HIP(hipStreamSynchronize(st));
    return (int)SD_OK;
  });
}

int sd_residual(sd_solver* s, const double* d_b, const double* d_x, double* d_r,
                double* d_norms, void* hip_stream) {
  return guarded([&] {
    if (!s || !d_r || !d_norms) return fail(SD_E_INVALID, "NULL argument");
    if (!s->s->on_device) return fail(SD_E_INVALID, "solver has no device data");
    SD_HIP(hipSetDevice(s->pb->device_id));
    sd::Solver& S = *s->s;
    sd::launch_residual_norms(S.A64, d_b ? d_b : S.b_dev, d_x, d_r, S.off, S.part, d_norms,
                              (hipStream_t)hip_stream);
    SD_HIP(hipGetLastError());
    return (int)SD_OK;
  });
}

int sd_residual_noalloc(sd_solver* s, const double* d_b, const double* d_x, double* d_r,
                        double* d_norms, void* hip_stream) {
  return guarded([&] {
    if (!s || !d_r || !d_norms) return fail(SD_E_INVALID, "NULL argument");
    if (!s->s->on_device) return fail(SD_E_INVALID, "solver has no device data");
    SD_HIP(hipSetDevice(s->pb->device_id));
    sd::Solver& S = *s->s;
    sd::launch_residual_norms_noalloc(S.A64, d_b ? d_b : S.b_dev, d_x, d_r, S.off, d_norms,
                                      (hipStream_t)hip_stream);
    SD_HIP(hipGetLastError());
    return (int)SD_OK;
  });
}

int sd_apply_preconditioner(sd_solver* s, const double* d_r, double* d_z, void* hip_stream) {
  return guarded([&] {
    if (!s || !d_r || !d_z) return fail(SD_E_INVALID, "NULL argument");
    if (!s->s->on_device) return fail(SD_E_INVALID, "solver has no device data");
    hipStream_t st = (hipStream_t)hip_stream;
    s->s->prec->apply_precond(*s->s, d_r, d_z, st);
    SD_HIP(hipGetLastError());
    SD_HIP(hipStreamSynchronize(st));
    return (int)SD_OK;
  });
}

int sd_apply_vcycle(sd_solver* s, int block, const double* d_b, double* d_x, int64_t n,
                    void* hip_stream) {
  return guarded([&] {
    if (!s || !d_b || !d_x || block < 0 || block > 2) return fail(SD_E_INVALID, "bad argument");
    if (s->s->hh[block].levels.empty())
      return fail(SD_E_INVALID, "the block has no hierarchy (block 2 exists only with "
                                "SD_SCHUR_CC, block 1 not with SD_DARCY_ILU0)");
    if (!s->s->on_device) return fail(SD_E_INVALID, "solver has no device data");
    const int64_t nb = s->s->hh[block].levels[0].A.n_rows;
    if (n != nb)
      return fail(SD_E_INVALID, "vector length " + std::to_string(n) + " != block size " +
                                    std::to_string(nb));
    hipStream_t st = (hipStream_t)hip_stream;
    s->s->prec->apply_vcycle(*s->s, block, d_b, d_x, st);
    SD_HIP(hipGetLastError());
    SD_HIP(hipStreamSynchronize(st));
    return (int)SD_OK;
  });
}

int sd_set_host_threads(int n) {
  if (n < 0) return fail(SD_E_INVALID, "n must be >= 0");
  sd::set_host_threads(n);
  return SD_OK;
}

int sd_arnoldi_layout(int64_t n, int* rows_per_block, int* blocks, size_t* lds_bytes) {
  if (n < 1 || n > sd::kMaxUnknowns)
    return fail(SD_E_INVALID, "n must be in 1.." + std::to_string(sd::kMaxUnknowns));
  const int rp = sd::gs_rows_per_block((int)n, sd::kGsProjectRows);
  if (rows_per_block) *rows_per_block = rp;
  if (blocks) *blocks = (int)((n + rp - 1) / rp);
  if (lds_bytes) *lds_bytes = (size_t)2 * rp * sizeof(double);
  return SD_OK;
}

struct sd_sell {
  sd::HostSell<double> h;
};

int sd_sell_build(int64_t n_rows, int64_t n_cols, const int64_t* rowptr, const int32_t* col,
                  const double* val, int allow_csr, int stencil, sd_sell** out) {
  return guarded([&] {
    if (!out) return fail(SD_E_INVALID, "out is NULL");
    *out = nullptr;
    if (n_rows < 0 || n_cols < 0 || !rowptr || (n_rows > 0 && rowptr[n_rows] > 0 && (!col || !val)))
      return fail(SD_E_INVALID, "bad CSR arguments");
    if (rowptr[0] != 0) return fail(SD_E_INVALID, "rowptr[0] must be 0");
    for (int64_t r = 0; r < n_rows; ++r)
      if (rowptr[r + 1] < rowptr[r]) return fail(SD_E_INVALID, "rowptr must not decrease");
    sd::HostCSR A;
    A.n_rows = n_rows;
    A.n_cols = n_cols;
    A.rowptr.assign(rowptr, rowptr + n_rows + 1);
    const int64_t nnz = rowptr[n_rows];
    A.col.assign(col, col + nnz);
    A.val.assign(val, val + nnz);
    for (int32_t c : A.col)
      if (c < 0 || c >= n_cols) return fail(SD_E_INVALID, "column outside [0, n_cols)");
    std::unique_ptr<sd_sell> m(new sd_sell());
    m->h = sd::build_sell<double>(A, allow_csr != 0, 0, stencil != 0);
    *out = m.release();
    return (int)SD_OK;
  });
}

int sd_sell_view(const sd_sell* m, sd_sell_info* info) {
  if (!m || !info) return fail(SD_E_INVALID, "NULL argument");
  const sd::HostSell<double>& h = m->h;
  info->lpr = h.lpr;
  info->width = h.width;
  info->stencil = h.stencil;
  info->n_rows = h.n_rows;
  info->n_cols = h.n_cols;
  info->nnz = h.nnz;
  info->idx = h.idx;
  info->n_ptr = (int64_t)h.sptr.size();
  info->n_entries = (int64_t)h.col.size();
  info->n_doff = (int64_t)h.doff.size();
  info->sptr = h.sptr.data();
  info->col = h.col.data();
  info->val = h.val.data();
  info->doff = h.doff.empty() ? nullptr : h.doff.data();
  return SD_OK;
}

void sd_sell_destroy(sd_sell* m) { delete m; }

int sd_solver_profile(sd_solver* s, int kernel_class) {
  if (!s || kernel_class < 0 || kernel_class > 4) return fail(SD_E_INVALID, "bad argument");
  s->s->prof_class = kernel_class;
  s->s->prof_launches = 0;
  s->s->prof_seconds = 0.0;
  s->s->prof_bytes = 0.0;
  return SD_OK;
}

int sd_solver_precond_cost(sd_solver* s, double* bytes, int* launches) {
  return guarded([&] {
    if (!s) return fail(SD_E_INVALID, "solver is NULL");
    if (!s->s->on_device) return fail(SD_E_INVALID, "solver has no device data");
    s->s->prec->precond_cost(*s->s, bytes, launches);
    return (int)SD_OK;
  });
}

int sd_solver_middle_scale(const sd_solver* s, double* x) {
  if (!s || !x) return fail(SD_E_INVALID, "NULL argument");
  *x = s->s->xscale;
  return SD_OK;
}

int sd_solver_profile_read(const sd_solver* s, int64_t* launches, double* seconds,
                           double* bytes) {
  if (!s) return fail(SD_E_INVALID, "solver is NULL");
  if (launches) *launches = s->s->prof_launches;
  if (seconds) *seconds = s->s->prof_seconds;
  if (bytes) *bytes = s->s->prof_bytes;
  return SD_OK;
}

void sd_problem_destroy(sd_problem* pb) { delete pb; }

void sd_solver_destroy(sd_solver* s) {
  if (!s) return;
  if (s->pb && s->pb->device) (void)hipSetDevice(s->pb->device_id);
  delete s;
}

}  // extern "C"
