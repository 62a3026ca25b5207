// Host orchestration of the device solve: SELL upload, AMG hierarchies, the
// block preconditioner (Sec. 4) with V-cycle sub-solves (Sec. 5), and the
// flexible GMRES driver with FP64 restart residuals.
#include "solver.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <map>
#include <optional>
#include <type_traits>

namespace sd {

double wall_time() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// ------------------------------------------------------------------ memory
constexpr size_t kChunkBytes = (size_t)32 << 20;

DeviceMem::~DeviceMem() {
  for (void* p : chunks_) {
    if (has_)
      alloc_.free(p, alloc_.ctx, stream_);
    else
      (void)hipFreeAsync(p, nullptr);
  }
}

void* DeviceMem::chunk(size_t bytes) {
  void* p = nullptr;
  if (has_) {
    p = alloc_.alloc(bytes, alloc_.ctx, stream_);
    if (!p) throw Error(SD_E_NOMEM, "device allocation failed (allocator callback)");
  } else {
    if (hipMallocAsync(&p, bytes, stream_) != hipSuccess || !p) {
      (void)hipGetLastError();
      throw Error(SD_E_NOMEM, "hipMallocAsync failed");
    }
  }
  chunks_.push_back(p);
  return p;
}

void* DeviceMem::get(size_t bytes) {
  bytes = (bytes + 255) & ~(size_t)255;
  total_ += bytes;
  if (bytes > kChunkBytes / 4) return chunk(bytes);   // large arrays: a chunk of their own
  if (!cur_ || cur_off_ + bytes > cur_cap_) {
    cur_ = static_cast<char*>(chunk(kChunkBytes));
    cur_off_ = 0;
    cur_cap_ = kChunkBytes;
  }
  void* p = cur_ + cur_off_;
  cur_off_ += bytes;
  return p;
}

namespace {
std::mutex g_pinned_mu;
std::map<std::pair<size_t, bool>, std::vector<void*>> g_pinned_free;
}  // namespace

void* pinned_acquire(size_t bytes, bool mapped) {
  {
    std::lock_guard<std::mutex> lk(g_pinned_mu);
    auto& v = g_pinned_free[{bytes, mapped}];
    if (!v.empty()) {
      void* p = v.back();
      v.pop_back();
      return p;
    }
  }
  void* p = nullptr;
  SD_HIP(hipHostMalloc(&p, bytes,
                       mapped ? (hipHostMallocMapped | hipHostMallocCoherent) : hipHostMallocDefault));
  return p;
}

void pinned_release(void* p, size_t bytes, bool mapped) {
  if (!p) return;
  std::lock_guard<std::mutex> lk(g_pinned_mu);
  g_pinned_free[{bytes, mapped}].push_back(p);
}

// -------------------------------------------------------------------- SELL
// Device format choice: SELL-64 for long matrices (at least 65,536 rows)
// with at most 32 entries per row on average; CSR with 4, 8 or 16 lanes per
// row for short matrices or long rows (coarse AMG levels and transfer
// operators), when the kernels that use it allow.
[[noreturn]] void throw_launch(const char* what) { throw Error(SD_E_INVALID, what); }

static int lanes_per_row(const HostCSR& A, bool allow_csr, int force_lpr, double sell_max = 32.0) {
  if (force_lpr > 0) return force_lpr;
  if (!allow_csr || A.n_rows == 0) return 1;
  const double avg = (double)A.nnz() / (double)A.n_rows;
  if (avg <= sell_max && A.n_rows >= 65536) return 1;
  return avg <= 16.0 ? 4 : (avg <= 48.0 ? 8 : (avg <= 96.0 ? 16 : (avg <= 192.0 ? 32 : 64)));
}

// Lanes per row of a grid-transfer operator (R, P, Q): their rows gather from
// scattered aggregates, so SELL-64 pays only up to 16 entries per row (the
// first coarse velocity restriction of 1024x512, 27 per row: 12.1 us with one
// lane per row, 10.7 us with 8).
static int transfer_lanes(const HostCSR& M) { return lanes_per_row(M, true, 0, 16.0); }

// Offsets of a stencil slice (see Sell): the ascending union of col - row
// over the slice's rows, or an empty list when a row repeats a column, the
// slice has no entries or the union is longer than cap.
static std::vector<int> stencil_offsets(const HostCSR& A, int64_t sl, int64_t cap) {
  const int64_t n = A.n_rows, r0 = sl * 64, r1 = std::min(n, r0 + 64);
  std::vector<int64_t> o;                 // distinct offsets, ascending
  o.reserve((size_t)cap + 1);
  for (int64_t r = r0; r < r1; ++r) {
    for (int64_t e = A.rowptr[r]; e < A.rowptr[r + 1]; ++e) {
      if (e > A.rowptr[r] && A.col[e] <= A.col[e - 1]) return {};
      const int64_t d = (int64_t)A.col[e] - r;
      auto it = std::lower_bound(o.begin(), o.end(), d);
      if (it != o.end() && *it == d) continue;
      if ((int64_t)o.size() == cap) return {};
      o.insert(it, d);
    }
  }
  return std::vector<int>(o.begin(), o.end());
}

// A stencil slice may be widened beyond its longest row by this many
// positions (zeros) when its rows' offsets differ (layouts with per-slice
// widths only).
constexpr int64_t kStencilWiden = 8;

// SELL-C layout on the host: slices of C = 64 / lpr rows, entry k of row r of
// slice s at sptr[s] + C k + (r - C s).  A slice's width is its longest row
// rounded up to a multiple of lpr; padding has val 0 and repeats the row's
// last column (0 for an empty row).  lpr = 1 (SELL-64) unless allow_csr
// picks more lanes for matrices with few or long rows.  Hierarchy matrices
// whose slices pad to one common width at most 30 % larger get that width,
// which spares the kernels the slice pointer load.  Stencil slices (lpr == 1,
// see Sell) are used where they hold at least half of the entries; with
// per-slice widths a slice whose offsets outnumber its longest row by at most
// kStencilWiden is widened to hold them.
template <typename T>
HostSell<T> build_sell(const HostCSR& A, bool allow_csr, int force_lpr, bool stencil) {
  HostSell<T> h;
  const int64_t n = A.n_rows;
  const int lpr = lanes_per_row(A, allow_csr, force_lpr);
  const int64_t C = 64 / lpr;
  const int64_t ns = (n + C - 1) / C;
  std::vector<int64_t> width((size_t)ns, 0);
  int64_t tot = 0, wmax = 0;
  for (int64_t sl = 0; sl < ns; ++sl) {
    int64_t w = 0;
    for (int64_t r = sl * C; r < std::min(n, sl * C + C); ++r)
      w = std::max(w, A.rowptr[r + 1] - A.rowptr[r]);
    w = (w + lpr - 1) / lpr * lpr;
    width[sl] = w;
    wmax = std::max(wmax, w);
    tot += C * w;
  }
  const bool uniform = allow_csr && wmax > 0 && (double)(C * ns * wmax) <= 1.3 * (double)tot;
  if (uniform) {
    for (auto& w : width) w = wmax;
    tot = C * ns * wmax;
  }
  // stencil slices: offsets per slice (empty: the slice reads col)
  std::vector<std::vector<int>> offs;
  if (stencil && lpr == 1) {
    offs.resize((size_t)ns);
    parallel_ranges(0, ns, [&](int64_t s0, int64_t s1) {
      for (int64_t sl = s0; sl < s1; ++sl)
        offs[sl] = stencil_offsets(A, sl, uniform ? wmax : width[sl] + kStencilWiden);
    });
    int64_t covered = 0;
    for (int64_t sl = 0; sl < ns; ++sl)
      if (!offs[sl].empty()) covered += A.rowptr[std::min(n, sl * 64 + 64)] - A.rowptr[sl * 64];
    if (covered == 0 || 2 * covered < A.nnz()) {
      offs.clear();
    } else if (!uniform) {
      tot = 0;
      for (int64_t sl = 0; sl < ns; ++sl) {
        width[sl] = std::max<int64_t>(width[sl], (int64_t)offs[sl].size());
        tot += 64 * width[sl];
      }
    }
  }
  if (tot >= ((int64_t)1 << 31)) throw Error(SD_E_INVALID, "matrix too large for int32 SELL");
  h.n_rows = n;
  h.n_cols = A.n_cols;
  h.lpr = lpr;
  h.width = uniform ? (int)wmax : 0;
  h.nnz = A.nnz();
  std::vector<int>& sptr = h.sptr;
  std::vector<int>& col = h.col;
  std::vector<T>& val = h.val;
  sptr.assign((size_t)ns + 1, 0);
  for (int64_t sl = 0; sl < ns; ++sl) sptr[sl + 1] = (int)(sptr[sl] + C * width[sl]);
  col.assign((size_t)tot, 0);
  val.assign((size_t)tot, (T)0);
  std::vector<int>& doff = h.doff;
  h.idx = A.nnz();
  if (!offs.empty()) {
    // one entry per slice position, and a closing kIrregularSlice: a slice
    // of width 0 has no entry of its own, the kernels read the flag at its
    // base (the next slice's first offset, or this one) and then nothing
    doff.assign((size_t)(tot / 64 + 1), 0);
    doff.back() = kIrregularSlice;
    h.idx = (int64_t)doff.size();
    h.stencil = 2;
    for (int64_t sl = 0; sl < ns; ++sl) {
      const int64_t b = sptr[sl] / 64, w = width[sl];
      const std::vector<int>& o = offs[sl];
      if (w == 0) continue;
      if (o.empty()) {
        doff[b] = kIrregularSlice;
        h.stencil = 1;
        h.idx += A.rowptr[std::min(n, sl * 64 + 64)] - A.rowptr[sl * 64];
      } else {
        // positions past the slice's offsets repeat the last one (zeros)
        for (int64_t k = 0; k < w; ++k) doff[b + k] = o[std::min<int64_t>(k, (int64_t)o.size() - 1)];
      }
    }
  }
  parallel_ranges(0, ns, [&](int64_t s0, int64_t s1) {
    for (int64_t sl = s0; sl < s1; ++sl) {
      const int64_t w = width[sl];
      if (!offs.empty() && !offs[sl].empty()) {
        const int* o = &doff[sptr[sl] / 64];
        for (int64_t ri = 0; ri < 64; ++ri) {
          const int64_t r = sl * 64 + ri;
          int64_t e = r < n ? A.rowptr[r] : 0;
          const int64_t end = r < n ? A.rowptr[r + 1] : 0;
          for (int64_t k = 0; k < w; ++k) {
            const int64_t p = sptr[sl] + 64 * k + ri;
            // the kernels clamp the column into [0, n_cols): positions where
            // row + o_k falls outside hold zeros
            col[p] = (int)std::min<int64_t>(std::max<int64_t>(r + o[k], 0), A.n_cols - 1);
            const bool here = e < end && (int64_t)A.col[e] - r == o[k] &&
                              (k == 0 || o[k] != o[k - 1]);
            val[p] = here ? (T)A.val[e++] : (T)0;
          }
        }
        continue;
      }
      for (int64_t ri = 0; ri < C; ++ri) {
        const int64_t r = sl * C + ri;
        int64_t len = 0, beg = 0;
        if (r < n) {
          beg = A.rowptr[r];
          len = A.rowptr[r + 1] - beg;
        }
        for (int64_t k = 0; k < w; ++k) {
          const int64_t e = sptr[sl] + C * k + ri;
          if (k < len) {
            col[e] = A.col[beg + k];
            val[e] = (T)A.val[beg + k];
          } else {
            col[e] = len > 0 ? A.col[beg + len - 1] : 0;
            val[e] = (T)0;
          }
        }
      }
    }
  });
  return h;
}

template HostSell<double> build_sell<double>(const HostCSR&, bool, int, bool);
template HostSell<float> build_sell<float>(const HostCSR&, bool, int, bool);

template <typename T>
Sell<T> upload_sell(const HostCSR& A, DeviceMem& mem, hipStream_t s, bool allow_csr,
                    int force_lpr, bool stencil) {
  const HostSell<T> h = build_sell<T>(A, allow_csr, force_lpr, stencil);
  Sell<T> d;
  d.n_rows = (int)h.n_rows;
  d.n_cols = (int)h.n_cols;
  d.lpr = h.lpr;
  d.width = h.width;
  d.nnz = h.nnz;
  d.idx = h.idx;
  d.stencil = h.stencil;
  int* dp = mem.array<int>(std::max<size_t>(h.sptr.size(), 1));
  // an all-stencil matrix is never read through col: it stays on the host
  const bool need_col = h.stencil != 2;
  int* dcol = need_col ? mem.array<int>(std::max<size_t>(h.col.size(), 1)) : nullptr;
  T* dval = mem.array<T>(std::max<size_t>(h.val.size(), 1));
  if (!h.sptr.empty())
    SD_HIP(hipMemcpyAsync(dp, h.sptr.data(), h.sptr.size() * sizeof(int), hipMemcpyHostToDevice, s));
  if (need_col && !h.col.empty())
    SD_HIP(hipMemcpyAsync(dcol, h.col.data(), h.col.size() * sizeof(int), hipMemcpyHostToDevice, s));
  if (!h.val.empty())
    SD_HIP(hipMemcpyAsync(dval, h.val.data(), h.val.size() * sizeof(T), hipMemcpyHostToDevice, s));
  if (!h.doff.empty()) {
    int* dd = mem.array<int>(h.doff.size());
    SD_HIP(hipMemcpyAsync(dd, h.doff.data(), h.doff.size() * sizeof(int), hipMemcpyHostToDevice, s));
    d.doff = dd;
  }
  SD_HIP(hipStreamSynchronize(s));
  d.sptr = dp;
  d.col = dcol;
  d.val = dval;
  return d;
}

template Sell<double> upload_sell<double>(const HostCSR&, DeviceMem&, hipStream_t, bool, int, bool);
template Sell<float> upload_sell<float>(const HostCSR&, DeviceMem&, hipStream_t, bool, int, bool);

// ------------------------------------------------------------ host setup
static double diag_at(const HostCSR& A, int64_t r) {
  for (int64_t k = A.rowptr[r]; k < A.rowptr[r + 1]; ++k)
    if (A.col[k] == r) return A.val[k];
  throw Error(SD_E_INVALID, "missing diagonal entry");
}

void Solver::setup_host(HostProblem* p, const sd_solver_opts* o) {
  TraceRange trace("sd: set-up (host)");
  const double t0 = wall_time();
  pb = p;
  sd_solver_opts d;
  sd_solver_opts_default(&d);
  opts.o = o ? *o : d;
  const sd_solver_opts& so = opts.o;
  if (so.restart < 1 || so.restart > kMaxBasis - 1)
    throw Error(SD_E_INVALID, "restart must be in 1..63");
  if (!(so.tol > 0.0) || so.maxit < 1) throw Error(SD_E_INVALID, "tol > 0 and maxit >= 1 required");
  if (so.precond < SD_PREC_BJ || so.precond > SD_PREC_TD_BGS) throw Error(SD_E_INVALID, "precond");
  if (so.schur != SD_SCHUR_IDENTITY && so.schur != SD_SCHUR_MASS && so.schur != SD_SCHUR_CC)
    throw Error(SD_E_INVALID, "schur");
  if (so.schur == SD_SCHUR_CC && !(p->mass > 0.0))
    throw Error(SD_E_INVALID,
                "SD_SCHUR_CC needs a backward-Euler system (problem assembled with phys.dt > 0)");
  if (so.precision != SD_PRECISION_FP64 && so.precision != SD_PRECISION_MIXED &&
      so.precision != SD_PRECISION_MIXED32)
    throw Error(SD_E_INVALID, "precision");
  if (so.krylov != SD_KRYLOV_FGMRES && so.krylov != SD_KRYLOV_BICGSTAB &&
      so.krylov != SD_KRYLOV_PDGMRES)
    throw Error(SD_E_INVALID, "krylov");
  if (so.krylov == SD_KRYLOV_PDGMRES &&
      (so.pd_m_init < 1 || so.pd_m_min < 1 || so.pd_m_step < 0 ||
       !std::isfinite(so.pd_alpha_p) || !std::isfinite(so.pd_alpha_d)))
    throw Error(SD_E_INVALID, "PD-GMRES needs pd_m_init, pd_m_min >= 1, pd_m_step >= 0 and "
                              "finite gains");
  if (so.amg != SD_AMG_PLAIN && so.amg != SD_AMG_SMOOTHED) throw Error(SD_E_INVALID, "amg");
  if (so.stencil_slices != 0 && so.stencil_slices != 1)
    throw Error(SD_E_INVALID, "stencil_slices must be 0 or 1");
  if (so.fused_restriction != 0 && so.fused_restriction != 1)
    throw Error(SD_E_INVALID, "fused_restriction must be 0 or 1");
  if (so.darcy != SD_DARCY_AMG && so.darcy != SD_DARCY_ILU0) throw Error(SD_E_INVALID, "darcy");
  opts.amg.theta = so.theta;
  opts.amg.omega = so.omega;
  opts.amg.nu_pre = so.nu_pre;
  opts.amg.nu_post = so.nu_post;
  opts.amg.coarse_max = so.coarse_max;
  opts.amg.max_levels = so.max_levels;
  opts.amg.smoothed = so.amg == SD_AMG_SMOOTHED;
  opts.amg.mis = so.mis;

  const Layout& L = p->L;
  if (L.N > kMaxUnknowns)
    throw Error(SD_E_INVALID, "more than " + std::to_string(kMaxUnknowns) +
                                  " unknowns: beyond the row blocking of the Gram-Schmidt kernels");
  off[0] = 0;
  off[1] = L.off_v;
  off[2] = L.off_p;
  off[3] = L.off_q;
  off[4] = L.N;
  N = (int)L.N;
  HostCSR Vb = extract_block(p->A, 0, L.off_p, 0, L.off_p);
  HostCSR Db = extract_block(p->A, L.off_q, L.N, L.off_q, L.N);
  HostCSR C1 = extract_block(p->A, L.off_q, L.N, 0, L.off_p);
  HostCSR B1 = extract_block(p->A, 0, L.off_p, L.off_q, L.N);
  HostCSR Dt = darcy_interface_block(Db, C1, B1, Vb);
  std::vector<int32_t> compV((size_t)L.off_p, 0);
  for (int64_t i = L.off_v; i < L.off_w; ++i) compV[i] = 1;
  for (int64_t i = L.off_w; i < L.off_p; ++i) compV[i] = 2;   // w (3-D)
  std::vector<int32_t> compD((size_t)(L.N - L.off_q), 0);
  // a subdomain system (partitioned coupling) may have no velocity or no
  // porous block: its hierarchy then stays empty and its V-cycle is skipped
  hh[0] = HostHierarchy();
  hh[1] = HostHierarchy();
  ilu = HostIlu();
  if (L.off_p > 0) {
    TraceRange trace("sd: AMG set-up, velocity block");
    amg_setup_host(Vb, compV, false, opts.amg, hh[0]);
  }
  if (L.N > L.off_q) {
    TraceRange trace("sd: Darcy block set-up");
    if (so.darcy == SD_DARCY_ILU0) ilu0_host(Dt, ilu);
    else amg_setup_host(Dt, compD, false, opts.amg, hh[1]);
  }
  hh[2] = HostHierarchy();
  if (so.schur == SD_SCHUR_CC) {
    // L_p = B^T D^-1 B = (-C) diag(1/D) B, D = |CV|/dt on the velocity rows
    // with a time derivative and diag(V) on the others
    HostCSR Cm = extract_block(p->A, L.off_p, L.off_q, 0, L.off_p);
    for (double& v : Cm.val) v = -v;
    HostCSR Bp = extract_block(p->A, 0, L.off_p, L.off_p, L.off_q);
    std::vector<double> dinv((size_t)L.off_p);
    for (int64_t k = 0; k < L.off_p; ++k)
      dinv[(size_t)k] = 1.0 / (L.has_mass(k) ? p->mass : diag_at(Vb, k));
    HostCSR Lp = scaled_product(Cm, dinv, Bp);
    std::vector<int32_t> compP((size_t)(L.off_q - L.off_p), 0);
    amg_setup_host(Lp, compP, false, opts.amg, hh[2]);
  }
  if (so.precond == SD_PREC_BGS || so.precond == SD_PREC_TD_BGS) {
    Cf = extract_block(p->A, L.off_p, L.N, 0, L.off_p);
  } else if (so.precond == SD_PREC_TD_BJ) {
    // continuity rows keep their velocity coupling, porous rows lose theirs
    Cf = extract_block(p->A, L.off_p, L.off_q, 0, L.off_p);
    Cf.n_rows = L.N - L.off_p;
    Cf.rowptr.resize((size_t)Cf.n_rows + 1, Cf.rowptr.back());
  } else {
    Cf.n_rows = L.N - L.off_p;
    Cf.n_cols = L.off_p;
    Cf.rowptr.assign((size_t)Cf.n_rows + 1, 0);
  }
  const double dz = p->L.nz > 0 ? p->grid.Lz / (double)p->grid.nz : 1.0;
  const double vol = ((p->grid.Lx / (double)p->grid.nx) * (p->grid.H_ff / (double)p->grid.ny)) * dz;
  xscale = so.schur == SD_SCHUR_IDENTITY ? 1.0 : p->phys.mu / vol;
  if (so.precond == SD_PREC_TD_BJ || so.precond == SD_PREC_TD_BGS) {
    if (so.schur == SD_SCHUR_CC) throw Error(SD_E_INVALID, "two-domain forms use the Uzawa block");
    xscale = 1.0;   // replaced by the Uzawa relaxation once the V-cycle is on the device
  }
  t_setup = wall_time() - t0;
}

Solver::~Solver() {
  prec.reset();
  if (stream) (void)hipStreamSynchronize(stream);
  for (auto e : events) (void)hipEventDestroy(e);
  for (auto e : prof_ev) (void)hipEventDestroy(e);
  if (ev_join) (void)hipEventDestroy(ev_join);
  if (ev_state) (void)hipEventDestroy(ev_state);
  pinned_release(hs, sizeof(HostState), false);
  if (stream) (void)hipStreamDestroy(stream);
  if (stream2) {
    (void)hipStreamSynchronize(stream2);
    (void)hipStreamDestroy(stream2);
  }
  if (ev_fork) (void)hipEventDestroy(ev_fork);
  if (ev_back) (void)hipEventDestroy(ev_back);
  pinned_release((void*)hf, sizeof(HostFlags), true);
}

void Solver::upload(const sd_allocator* alloc, hipStream_t s) {
  TraceRange trace("sd: upload");
  const double t0 = wall_time();
  mem.reset(new DeviceMem(alloc, s));
  const bool stencil = opts.o.stencil_slices != 0;
  {
    TraceRange trace_a("sd: upload, coupled matrix");
    A64 = upload_sell<double>(pb->A, *mem, s, false, 0, stencil);
  }
  b_dev = mem->array<double>((size_t)N);
  if (pb->mass > 0.0) step_b = mem->array<double>((size_t)N);
  SD_HIP(hipMemcpyAsync(b_dev, pb->b.data(), (size_t)N * sizeof(double), hipMemcpyHostToDevice, s));
  ldv = ((int64_t)N + 63) / 64 * 64;
  const int m = opts.o.restart;
  V = mem->array<double>((size_t)(m + 1) * ldv);
  W = mem->array<double>((size_t)ldv);
  part = mem->array<double>(std::max((size_t)kGsPartRows * kGsMaxBlocks,
                                     (size_t)kDotBlocks * kPartStride));
  st = static_cast<DevState*>(mem->get(sizeof(DevState)));
  SD_HIP(hipMemsetAsync(st, 0, sizeof(DevState), s));
  void* h = pinned_acquire(sizeof(HostFlags), true);
  hf = static_cast<HostFlags*>(h);
  std::memset(h, 0, sizeof(HostFlags));
  void* hd = nullptr;
  SD_HIP(hipHostGetDevicePointer(&hd, h, 0));
  hf_dev = static_cast<HostFlags*>(hd);
  events.resize((size_t)kMaxBasis + 2);
  for (auto& e : events) SD_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  SD_HIP(hipEventCreateWithFlags(&ev_join, hipEventDisableTiming));
  SD_HIP(hipEventCreateWithFlags(&ev_state, hipEventDisableTiming));
  void* hsp = pinned_acquire(sizeof(HostState), false);
  hs = static_cast<HostState*>(hsp);
  std::memset(hsp, 0, sizeof(HostState));
  prof_ev.resize((size_t)2 * kMaxBasis);
  for (auto& e : prof_ev) SD_HIP(hipEventCreate(&e));
  nnz_A = pb->A.nnz();
  nnz_V0 = hh[0].levels.empty() ? 0 : hh[0].levels[0].A.nnz();
  SD_HIP(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
  if (opts.o.precond == SD_PREC_BJ) {
    SD_HIP(hipStreamCreateWithFlags(&stream2, hipStreamNonBlocking));
    SD_HIP(hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming));
    SD_HIP(hipEventCreateWithFlags(&ev_back, hipEventDisableTiming));
  }
  prec = opts.o.precision == SD_PRECISION_FP64 ? make_prec_fp64(*this, s) : make_prec_fp32(*this, s);
  SD_HIP(hipStreamSynchronize(s));
  if ((opts.o.precond == SD_PREC_TD_BJ || opts.o.precond == SD_PREC_TD_BGS) && off[2] > 0 &&
      off[3] > off[2])
    xscale = uzawa_relaxation(s);
  on_device = true;
  t_setup += wall_time() - t0;
}

// omega = 1/lambda_max of -C P_V B, P_V one V-cycle on the velocity block,
// by power iteration from the normalised ones vector (the inexact Uzawa step
// of the two-domain preconditioners).  Products with B and C run on the host,
// the V-cycle on the device.
double Solver::uzawa_relaxation(hipStream_t s) {
  const int64_t nv = off[2], np_ = off[3] - off[2];
  HostCSR Bh = extract_block(pb->A, 0, nv, nv, off[3]);
  HostCSR Ch = extract_block(pb->A, nv, off[3], 0, nv);
  double* d_in = mem->array<double>((size_t)nv);
  double* d_out = mem->array<double>((size_t)nv);
  std::vector<double> x((size_t)np_, 1.0 / std::sqrt((double)np_)), t((size_t)nv), y((size_t)np_);
  double lam = 1.0;
  for (int it = 0; it < kUzawaPowerIters; ++it) {
    for (int64_t r = 0; r < nv; ++r) {
      double acc = 0.0;
      for (int64_t k = Bh.rowptr[r]; k < Bh.rowptr[r + 1]; ++k) acc += Bh.val[k] * x[Bh.col[k]];
      t[r] = acc;
    }
    SD_HIP(hipMemcpyAsync(d_in, t.data(), (size_t)nv * 8, hipMemcpyHostToDevice, s));
    prec->apply_vcycle(*this, 0, d_in, d_out, s);
    SD_HIP(hipMemcpyAsync(t.data(), d_out, (size_t)nv * 8, hipMemcpyDeviceToHost, s));
    SD_HIP(hipStreamSynchronize(s));
    double nrm = 0.0;
    for (int64_t r = 0; r < np_; ++r) {
      double acc = 0.0;
      for (int64_t k = Ch.rowptr[r]; k < Ch.rowptr[r + 1]; ++k) acc += Ch.val[k] * t[Ch.col[k]];
      y[r] = -acc;
      nrm += y[r] * y[r];
    }
    lam = std::sqrt(nrm);
    if (!(lam > 0.0) || !std::isfinite(lam))
      throw Error(SD_E_INVALID, "Uzawa relaxation: degenerate Schur complement");
    for (int64_t r = 0; r < np_; ++r) x[r] = y[r] / lam;
  }
  return 1.0 / lam;
}

void Solver::enable_column_replay() {
  if (!on_device) throw Error(SD_E_INVALID, "solver was set up without a device");
  if (rin) return;
  const size_t tz = opts.o.precision == SD_PRECISION_FP64 ? sizeof(double) : sizeof(float);
  rin = mem->array<double>((size_t)ldv);
  sigfix = mem->array<double>(1);
  zfix = mem->get((size_t)ldv * tz + 16);
}

int pd_next_length(const sd_solver_opts& o, SolveRun& R, int m_cap) {
  const std::vector<double>& r = R.pd_res;
  const size_t k = r.size();
  int m;
  if (R.pd_m == 0 || k < 2) {
    m = R.pd_m_init;
  } else {
    const double rj = r[k - 1], rj1 = r[k - 2];
    double d = o.pd_alpha_p * rj / rj1;
    if (k >= 3) d += o.pd_alpha_d * (rj - r[k - 3]) / (2.0 * rj1);
    const double step = std::floor(d);
    m = R.pd_m + (std::isfinite(step) ? (int)std::max(-1e6, std::min(1e6, step)) : 0);
    if (m < o.pd_m_min) {
      R.pd_m_init += o.pd_m_step;
      m = R.pd_m_init;
    }
  }
  m = std::max(1, std::min(m, m_cap));
  R.pd_m = m;
  return m;
}

int Solver::solve(const double* b, double* x, int use_x0, sd_stats* stats, hipStream_t s) {
  TraceRange trace("sd: solve");
  if (!on_device) throw Error(SD_E_INVALID, "solver was set up without a device");
  if (!x) throw Error(SD_E_INVALID, "x must be a device pointer");
  if (!b) b = b_dev;
  if (opts.o.krylov == SD_KRYLOV_BICGSTAB) return prec->bicgstab(*this, b, x, use_x0, stats, s);
  return prec->fgmres(*this, b, x, use_x0, stats, s);
}

// ===================================================== precision-specific
namespace {

// Levels below these sizes are latency bound: their smoothing is fused with
// the transfers (fewer, wider launches); larger levels keep separate passes,
// whose one-lane-per-row stencil gathers are coalesced.
constexpr int64_t kFusePreRows = 196608, kFusePostRows = 65536;
// Fusion pays while the fused operators stay about as sparse as the passes
// they replace.  On the wide Galerkin stencils of 3-D hierarchies
// G = R (I - A M2) grows to 4-18x the nonzeros of Q = [R | -RA] and
// F = P - W A P to 0.75-0.8x those of A (2-D: at most 1.9x and 0.55x), so such
// levels keep separate passes; G is not even formed above an average row
// width of kFuseMaxRowWidth.
constexpr double kFuseMaxGOverQ = 3.0, kFuseMaxFOverA = 0.65;
constexpr int64_t kFuseMaxRowWidth = 64;

template <typename T>
void upload_hierarchy(const HostHierarchy& h, DevHierarchy<T>& d, double omega, int nu_pre,
                      int nu_post, bool stencil, bool fuse_restriction, DeviceMem& mem,
                      hipStream_t s) {
  d.lev.resize(h.levels.size());
  for (size_t l = 0; l < h.levels.size(); ++l) {
    const HostLevel& H = h.levels[l];
    DevLevel<T>& D = d.lev[l];
    D.n = (int)H.A.n_rows;
    D.A = upload_sell<T>(H.A, mem, s, true, 0, stencil);
    std::vector<double> w((size_t)D.n);
    for (int i = 0; i < D.n; ++i) w[i] = omega / diag_at(H.A, i);
    std::vector<T> wd((size_t)D.n);
    for (int i = 0; i < D.n; ++i) wd[i] = (T)w[i];
    D.wd = mem.array<T>((size_t)D.n);
    SD_HIP(hipMemcpyAsync(D.wd, wd.data(), wd.size() * sizeof(T), hipMemcpyHostToDevice, s));
    D.tmp = mem.array<T>((size_t)D.n);
    D.x = mem.array<T>((size_t)D.n);
    D.b = mem.array<T>((size_t)D.n);
    if (l + 1 < h.levels.size()) {
      const int64_t nnzA = H.A.nnz();
      HostCSR G, F, RA;
      std::optional<TraceRange> trace_f;
      trace_f.emplace("sd: fused transfer operators (host)");
      D.fuse_pre = fuse_restriction && nu_pre == 2 && (l > 0 || H.A.n_rows < kFusePreRows) &&
                   nnzA <= kFuseMaxRowWidth * H.A.n_rows;
      // R A serves both G and Q = [R | -R A] (nnz(Q) = nnz(R) + nnz(R A))
      if (l > 0 || D.fuse_pre) RA = sparse_product(H.R, H.A);
      if (D.fuse_pre) {
        G = presmoothed_restriction(H.A, H.R, RA, omega);
        const int64_t replaced = l > 0 ? H.R.nnz() + RA.nnz() : H.R.nnz() + nnzA;
        D.fuse_pre = (double)G.nnz() <= kFuseMaxGOverQ * (double)replaced;
      }
      D.fuse_post = nu_post >= 1 && (l > 0 || H.A.n_rows < kFusePostRows);
      if (D.fuse_post) {
        F = smoothed_correction(H.A, H.P, H.AP, omega);
        D.fuse_post = l == 0 || (double)F.nnz() <= kFuseMaxFOverA * (double)nnzA;
      }
      trace_f.reset();
      if (D.fuse_pre) {
        // the fused pre-smoothing reads A diag(w)
        HostCSR AW = H.A;
        for (size_t k = 0; k < AW.val.size(); ++k) AW.val[k] = H.A.val[k] * w[AW.col[k]];
        D.AW = upload_sell<T>(AW, mem, s, true, D.A.lpr, stencil);
        D.G = upload_sell<T>(G, mem, s, true, 64);
      } else if (l == 0) {
        D.R = upload_sell<T>(H.R, mem, s, true, transfer_lanes(H.R));
        D.r = mem.array<T>((size_t)D.n);
      } else {
        const HostCSR Qh = residual_restriction(H.A, H.R, RA);
        D.Q = upload_sell<T>(Qh, mem, s, true, transfer_lanes(Qh));
      }
      if (D.fuse_post) D.F = upload_sell<T>(F, mem, s, true, D.A.lpr);
      else D.P = upload_sell<T>(H.P, mem, s, true, transfer_lanes(H.P));
    }
    SD_HIP(hipStreamSynchronize(s));
  }
  d.n_coarse = (int)h.n_coarse;
  d.Ainv = mem.array<double>(h.Ainv.size());
  SD_HIP(hipMemcpyAsync(d.Ainv, h.Ainv.data(), h.Ainv.size() * sizeof(double),
                        hipMemcpyHostToDevice, s));
  SD_HIP(hipStreamSynchronize(s));
}

template <typename T, typename S>
static const T* upload_vec(const std::vector<S>& v, DeviceMem& mem, hipStream_t s) {
  std::vector<T> h(v.begin(), v.end());
  T* d = mem.array<T>(h.size());
  SD_HIP(hipMemcpyAsync(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
  SD_HIP(hipStreamSynchronize(s));
  return d;
}

template <typename T>
IluDev<T> upload_ilu(const HostIlu& h, DeviceMem& mem, hipStream_t s) {
  IluDev<T> d;
  d.n = (int)h.n;
  d.nlev_l = (int)h.lev_l.size() - 1;
  d.nlev_u = (int)h.lev_u.size() - 1;
  d.lev_l = upload_vec<int>(h.lev_l, mem, s);
  d.lev_u = upload_vec<int>(h.lev_u, mem, s);
  d.ord_l = upload_vec<int>(h.ord_l, mem, s);
  d.ord_u = upload_vec<int>(h.ord_u, mem, s);
  d.col_l = upload_vec<int>(h.col_l, mem, s);
  d.col_u = upload_vec<int>(h.col_u, mem, s);
  d.val_l = upload_vec<T>(h.val_l, mem, s);
  d.val_u = upload_vec<T>(h.val_u, mem, s);
  d.diag_u = upload_vec<T>(h.diag_u, mem, s);
  return d;
}

template <typename T>
class PrecImpl : public PrecBase {
 public:
  DevHierarchy<T> H[3];  // V, D~ and (Cahouet-Chabard middle block) L_p
  IluDev<T> ilu;         // ILU(0) of D~ in place of its hierarchy (SD_DARCY_ILU0)
  Sell<T> Cf;
  Sell<float> A32;       // FP32 copy of A for the Arnoldi product (MIXED32 only)
  bool arn32 = false;
  T* Z = nullptr;        // m preconditioned vectors
  T* tq = nullptr;       // porous right-hand side of the block sweep
  T* tp = nullptr;       // pressure right-hand side of the L_p V-cycle (cc only)
  T* yl = nullptr;       // its result
  bool cc = false;
  T* tmpN = nullptr;     // scratch vector of length N (apply entry points)
  int64_t ldz = 0;
  int nu_pre = 2, nu_post = 2;

  PrecImpl(Solver& S, hipStream_t s) {
    DeviceMem& mem = *S.mem;
    nu_pre = S.opts.amg.nu_pre;
    nu_post = S.opts.amg.nu_post;
    cc = !S.hh[2].levels.empty();
    static const char* const kRange[3] = {"sd: upload, velocity hierarchy",
                                          "sd: upload, Darcy hierarchy",
                                          "sd: upload, pressure-operator hierarchy"};
    for (int b = 0; b < 3; ++b)
      if (!S.hh[b].levels.empty()) {
        TraceRange trace(kRange[b]);
        upload_hierarchy<T>(S.hh[b], H[b], S.opts.amg.omega, nu_pre, nu_post,
                            S.opts.o.stencil_slices != 0, S.opts.o.fused_restriction != 0, mem,
                            s);
      }
    if (S.ilu.n > 0) ilu = upload_ilu<T>(S.ilu, mem, s);
    if (cc) {
      tp = mem.array<T>((size_t)(S.off[3] - S.off[2]));
      yl = mem.array<T>((size_t)(S.off[3] - S.off[2]));
    }
    Cf = upload_sell<T>(S.Cf, mem, s, false, 0, S.opts.o.stencil_slices != 0);
    arn32 = S.opts.o.precision == SD_PRECISION_MIXED32;
    if (arn32) A32 = upload_sell<float>(S.pb->A, mem, s, false, 0, S.opts.o.stencil_slices != 0);
    ldz = S.ldv;
    Z = mem.array<T>((size_t)S.opts.o.restart * ldz);
    tq = mem.array<T>((size_t)(S.N - S.off[3]) + 1);
    tmpN = mem.array<T>((size_t)ldz);
  }

  // One V-cycle from x = 0 on block blk, level l; b of type TB scaled by *bs.
  template <typename TB>
  void vcycle(int blk, int l, const TB* b, const double* bs, T* x, const DevState* gate,
              hipStream_t s) {
    DevHierarchy<T>& h = H[blk];
    DevLevel<T>& L = h.lev[l];
    if (l == (int)h.lev.size() - 1) {
      const T* bc = nullptr;
      if constexpr (std::is_same<TB, T>::value) {
        if (!bs) bc = b;
      }
      if (!bc) {  // scale / convert into the level's buffer first
        launch_scale_convert<TB, T>(b, bs, L.b, L.n, gate, s);
        bc = L.b;
      }
      launch_coarse<T>(h.Ainv, L.n, bc, x, gate, s);
      return;
    }
    T* cur = x;
    T* other = L.tmp;
    DevLevel<T>& C = h.lev[l + 1];
    if (L.fuse_pre) {
      launch_presmooth_restrict<T, TB>(L.AW, L.wd, L.G, b, bs, cur, C.b, gate, s);
    } else {
      if (nu_pre == 0) {
        launch_fill<T>(cur, (T)0, L.n, s);
      } else {
        launch_jacobi_zero<T, TB>(L.A, L.wd, b, bs, cur, nu_pre >= 2 ? 1 : 0, gate, s);
        for (int k = 2; k < nu_pre; ++k) {
          launch_jacobi<T, TB>(L.A, L.wd, b, bs, cur, other, gate, s);
          std::swap(cur, other);
        }
      }
      if (l == 0) {
        launch_residual<T, TB>(L.A, b, bs, cur, L.r, gate, s);
        launch_spmv<T, T, T>(L.R, L.r, C.b, gate, s);
      } else {
        launch_restrict_residual<T, TB>(L.Q, b, bs, cur, L.n, C.b, gate, s);
      }
    }
    vcycle<T>(blk, l + 1, C.b, nullptr, C.x, gate, s);
    int k0 = 0;
    if (L.fuse_post) {
      launch_prolong_smooth<T, TB>(L.A, L.F, L.wd, b, bs, cur, C.x, other, gate, s);
      std::swap(cur, other);
      k0 = 1;
    } else {
      launch_prolong<T>(L.P, C.x, cur, gate, s);
    }
    for (int k = k0; k < nu_post; ++k) {
      const bool timed = prof_jacobi_ev && blk == 0 && l == 0 && k + 1 == nu_post;
      if (timed) SD_HIP(hipEventRecord(prof_jacobi_ev[0], s));
      launch_jacobi<T, TB>(L.A, L.wd, b, bs, cur, other, gate, s);
      if (timed) SD_HIP(hipEventRecord(prof_jacobi_ev[1], s));
      std::swap(cur, other);
    }
    if (cur != x) launch_convert<T, T>(cur, x, L.n, s);
  }

  // apply() with events around the last post-smoothing sweep of the finest
  // velocity level (the same kernel and arguments as in apply()).
  void apply_profiled_jacobi(Solver& S, const double* r, const double* bs, T* z, hipStream_t s,
                             hipEvent_t* ev) {
    prof_jacobi_ev = ev;
    apply(S, r, bs, z, nullptr, s);
    prof_jacobi_ev = nullptr;
  }
  hipEvent_t* prof_jacobi_ev = nullptr;

  // z = P(bs * r): block preconditioner on a basis vector (FP64 input).  In
  // the block-Jacobi form nothing after the velocity V-cycle reads its
  // result, so the rest runs on a second stream beside it (two parallel
  // branches of the column graph); recorded columns stay in one sequence.
  void apply(Solver& S, const double* r, const double* bs, T* z, const DevState* gate,
             hipStream_t s) {
    const int64_t* o = S.off;
    const int n_p = (int)(o[3] - o[2]);
    const bool fork = S.stream2 && !launch_recording();
    hipStream_t s2 = s;
    if (fork) {
      SD_HIP(hipEventRecord(S.ev_fork, s));
      SD_HIP(hipStreamWaitEvent(S.stream2, S.ev_fork, 0));
      s2 = S.stream2;
    }
    if (!H[0].lev.empty()) vcycle<double>(0, 0, r, bs, z, gate, s);
    launch_block_sweep<T>(Cf, n_p, r + o[2], bs, z, S.xscale, z + o[2], tq, cc ? tp : nullptr,
                          gate, s2);
    if (cc) {
      vcycle<T>(2, 0, tp, nullptr, yl, gate, s2);
      launch_add<T>(yl, z + o[2], n_p, gate, s2);
    }
    if (ilu.n > 0) {
      launch_ilu0<T>(ilu, tq, z + o[3], gate, s2);
    } else if (!H[1].lev.empty()) {
      vcycle<T>(1, 0, tq, nullptr, z + o[3], gate, s2);
    }
    if (fork) {
      SD_HIP(hipEventRecord(S.ev_back, S.stream2));
      SD_HIP(hipStreamWaitEvent(s, S.ev_back, 0));
    }
  }

  void apply_precond(Solver& S, const double* r, double* z, hipStream_t s) override {
    if constexpr (std::is_same<T, double>::value) {
      apply(S, r, nullptr, z, nullptr, s);
    } else {
      apply(S, r, nullptr, tmpN, nullptr, s);
      launch_convert<T, double>(tmpN, z, S.N, s);
    }
  }

  void apply_vcycle(Solver& S, int blk, const double* b, double* x, hipStream_t s) override {
    if (H[blk].lev.empty()) throw Error(SD_E_INVALID, "block has no hierarchy");
    const int n = H[blk].lev[0].n;
    if constexpr (std::is_same<T, double>::value) {
      vcycle<double>(blk, 0, b, nullptr, x, nullptr, s);
    } else {
      vcycle<double>(blk, 0, b, nullptr, tmpN, nullptr, s);
      launch_convert<T, double>(tmpN, x, n, s);
    }
  }

  HostState read_state(Solver& S, hipStream_t s) {
    HostState h;
    SD_HIP(hipMemcpyAsync(&h, S.st, sizeof(HostState), hipMemcpyDeviceToHost, s));
    SD_HIP(hipStreamSynchronize(s));
    return h;
  }

  // ------------------------------------------------- resumable FGMRES driver
  // A solve is a state machine advanced by step(): it only enqueues work and
  // polls events, so a request loop can interleave many solves; sd_solve runs
  // the same machine with blocking waits.
  void start(Solver& S, SolveRun& R) override {
    R.phase = SolveRun::INIT;
    R.first = true;
    R.restarts = 0;
    R.status = SD_E_NOCONV;
    R.t0 = wall_time();
    R.out = sd_stats{};
    R.pd_res.clear();
    R.pd_m = 0;
    R.pd_m_init = S.opts.o.pd_m_init;
  }

  static bool ready(hipEvent_t e, bool block) {
    if (block) {
      SD_HIP(hipEventSynchronize(e));
      return true;
    }
    const hipError_t q = hipEventQuery(e);
    if (q == hipSuccess) return true;
    if (q == hipErrorNotReady) return false;
    SD_HIP(q);
    return false;
  }

  void async_state(Solver& S, hipStream_t s) {
    SD_HIP(hipMemcpyAsync(S.hs, S.st, sizeof(HostState), hipMemcpyDeviceToHost, s));
    SD_HIP(hipEventRecord(S.ev_state, s));
  }

  void finish(Solver& S, SolveRun& R, int status) {
    const HostState& hs = *S.hs;
    R.status = status;
    R.out.iters = hs.iters;
    R.out.restarts = R.restarts;
    R.out.rel_res = hs.bnorm > 0.0 ? hs.beta / hs.bnorm : 0.0;
    for (int k = 0; k < 3; ++k)
      R.out.rel_res_block[k] = hs.bnorm > 0.0 ? std::sqrt(hs.resblk[k]) / hs.bnorm : 0.0;
    R.out.t_setup = S.t_setup;
    R.out.t_solve = wall_time() - R.t0;
    R.phase = SolveRun::DONE;
  }

  bool step(Solver& S, SolveRun& R, bool block) override {
    hipStream_t s = S.stream;
    const sd_solver_opts& o = S.opts.o;
    const int n = S.N;
    const int m = o.restart;
    const double drop = arn32 ? 1e-6 : 0.0;
    const int depth = 2;
    switch (R.phase) {
      case SolveRun::INIT:
        launch_init_state(S.st, m, drop, s);
        launch_norm_b(R.b, n, o.tol, S.st, S.part, s);
        async_state(S, s);
        R.phase = SolveRun::WAIT_NORM;
        return true;
      case SolveRun::WAIT_NORM:
        if (!ready(S.ev_state, block)) return false;
        if (!(S.hs->bnorm > 0.0)) {
          launch_fill<double>(R.x, 0.0, n, s);
          SD_HIP(hipStreamSynchronize(s));
          S.hs->beta = 0.0;
          finish(S, R, std::isfinite(S.hs->bnorm) ? SD_OK : SD_E_INVALID);
          return true;
        }
        if (!R.use_x0) launch_fill<double>(R.x, 0.0, n, s);
        R.phase = SolveRun::RESTART;
        return true;
      case SolveRun::RESTART: {
        launch_restart_residual(S.A64, R.b, (R.first && !R.use_x0) ? nullptr : R.x, S.V, S.off,
                                S.st, S.part, S.hf_dev, s);
        R.first = false;
        async_state(S, s);
        R.phase = SolveRun::WAIT_RESTART;
        return true;
      }
      case SolveRun::WAIT_RESTART: {
        if (!ready(S.ev_state, block)) return false;
        const HostState& hs = *S.hs;
        if (hs.breakdown || !std::isfinite(hs.beta)) {
          finish(S, R, SD_E_BREAKDOWN);
          return true;
        }
        if (hs.converged) {
          finish(S, R, SD_OK);
          return true;
        }
        if (hs.iters >= o.maxit) {
          finish(S, R, SD_E_NOCONV);
          return true;
        }
        for (int j = 0; j <= kMaxBasis; ++j) {
          S.hf->cycle_done[j] = 0;
          S.hf->est[j] = 0.0;
        }
        R.ctarget = std::max(hs.target, drop * hs.beta);
        int len = m;
        if (o.krylov == SD_KRYLOV_PDGMRES) {
          R.pd_res.push_back(hs.beta);
          len = pd_next_length(o, R, m);
        }
        R.m_cycle = std::min(len, std::max(1, o.maxit - hs.iters));
        launch_init_cycle(S, R.m_cycle, s);
        R.j_enq = 0;
        R.completed = -1;
        R.phase = SolveRun::ITER;
        return true;
      }
      case SolveRun::ITER: {
        if (R.batched) return false;   // the request loop drives the columns
        while (R.completed + 1 < R.j_enq && ready(S.events[(size_t)(R.completed + 1)], false))
          ++R.completed;
        bool done = false;
        for (int q = 0; q <= R.completed; ++q) done = done || S.hf->cycle_done[q];
        if (done || R.j_enq == R.m_cycle) {
          // a full cycle's last column is completed by the closing step
          if (!done) launch_arnoldi_close(n, S.V, S.ldv, R.j_enq, S.st, S.part, S.hf_dev, s);
          launch_trisolve(S.st, s);
          launch_update_x<T>(R.x, Z, ldz, n, S.st, s);
          ++R.restarts;
          if (S.prof_class != 0) collect_profile(S, s);
          R.phase = SolveRun::RESTART;
          return true;
        }
        // Run ahead of the device by up to `depth` columns, except when the
        // residual estimates predict the end of the cycle within that window.
        int ahead = depth;
        if (R.completed >= 1) {
          const double e1 = S.hf->est[R.completed], e0 = S.hf->est[R.completed - 1];
          const double rho = e0 > 0.0 ? e1 / e0 : 1.0;
          if (rho > 0.0 && rho < 1.0) {
            const double need = std::log(R.ctarget / e1) / std::log(rho);
            if (need <= (double)(R.j_enq - R.completed)) ahead = 0;
          }
        }
        if (R.j_enq - 1 - R.completed <= ahead) {
          iteration(S, R.j_enq, s);
          SD_HIP(hipEventRecord(S.events[(size_t)R.j_enq], s));
          ++R.j_enq;
          return true;
        }
        if (block) {
          SD_HIP(hipEventSynchronize(S.events[(size_t)(R.completed + 1)]));
          return true;
        }
        return false;
      }
      case SolveRun::DONE:
        return false;
    }
    return false;
  }

  int fgmres(Solver& S, const double* b, double* x, int use_x0, sd_stats* stats,
             hipStream_t user) override {
    // The iteration runs on the solver's own stream (graphs cannot be captured
    // on the legacy default stream); it is ordered after the caller's stream.
    SD_HIP(hipEventRecord(S.ev_join, user));
    SD_HIP(hipStreamWaitEvent(S.stream, S.ev_join, 0));
    SolveRun R;
    R.b = b;
    R.x = x;
    R.use_x0 = use_x0;
    start(S, R);
    while (R.phase != SolveRun::DONE) step(S, R, true);
    SD_HIP(hipStreamSynchronize(S.stream));
    if (stats) *stats = R.out;
    return R.status;
  }

  // Enqueue Arnoldi step j (preconditioner + orthogonalisation) as a graph.
  std::vector<hipGraphExec_t> graphs;
  void iteration(Solver& S, int j, hipStream_t s) {
    if (S.prof_class != 0) {  // measurement mode: plain launches with events
      hipEvent_t* ev = &S.prof_ev[(size_t)2 * j];
      T* zj = Z + (size_t)j * ldz;
      if (S.prof_class == 3) {
        apply_profiled_jacobi(S, S.V + (size_t)j * S.ldv, &S.st->sigma[j], zj, s, ev);
      } else if (S.prof_class == 4) {   // the whole preconditioner application
        SD_HIP(hipEventRecord(ev[0], s));
        apply(S, S.V + (size_t)j * S.ldv, &S.st->sigma[j], zj, nullptr, s);
        SD_HIP(hipEventRecord(ev[1], s));
      } else {
        apply(S, S.V + (size_t)j * S.ldv, &S.st->sigma[j], zj, nullptr, s);
      }
      arnoldi(S, zj, j, s, S.prof_class, ev);
      return;
    }
    if (graphs.empty()) graphs.assign((size_t)kMaxBasis, nullptr);
    if (!graphs[(size_t)j]) {
      hipGraph_t g = nullptr;
      SD_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      enqueue_iteration(S, j, s);
      SD_HIP(hipStreamEndCapture(s, &g));
      hipGraphExec_t ge = nullptr;
      SD_HIP(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
      SD_HIP(hipGraphDestroy(g));
      graphs[(size_t)j] = ge;
    }
    SD_HIP(hipGraphLaunch(graphs[(size_t)j], s));
  }
  // The preconditioner kernels are gated on the cycle-done flag: a column
  // enqueued ahead of a cycle's end stores nothing (the ILU(0) substitution
  // returns at once).
  struct RecorderGuard {
    explicit RecorderGuard(std::vector<RecordedOp>* r) { set_launch_recorder(r); }
    ~RecorderGuard() { set_launch_recorder(nullptr); }
  };

  void record_column(Solver& S, std::vector<RecordedOp>& ops) override {
    if (!S.rin) throw Error(SD_E_INVALID, "column replay not enabled on this solver");
    if (S.prof_class != 0) throw Error(SD_E_INVALID, "column replay in measurement mode");
    T* zf = static_cast<T*>(S.zfix);
    ops.clear();
    RecorderGuard g(&ops);
    launch_copy_in(S.V, S.ldv, S.st, S.rin, S.sigfix, S.N, nullptr);
    apply(S, S.rin, S.sigfix, zf, S.st, nullptr);
    launch_copy_out<T>(zf, Z, ldz, S.st, S.N, nullptr);
    arnoldi(S, zf, -1, nullptr, 0, nullptr);
  }

  // Algorithmic bytes and launches of one preconditioner application (from a
  // recording of it; cached).
  double pc_bytes = -1.0;
  int pc_launches = 0;
  double precond_bytes(Solver& S) {
    if (pc_bytes < 0.0) {
      std::vector<RecordedOp> ops;
      {
        RecorderGuard g(&ops);
        apply(S, S.V, &S.st->sigma[0], Z, S.st, nullptr);
      }
      pc_bytes = 0.0;
      for (const RecordedOp& o : ops) pc_bytes += o.bytes;
      pc_launches = (int)ops.size();
    }
    return pc_bytes;
  }
  void precond_cost(Solver& S, double* bytes, int* launches) override {
    const double b = precond_bytes(S);
    if (bytes) *bytes = b;
    if (launches) *launches = pc_launches;
  }

  void end_cycle(Solver& S, SolveRun& R, bool full, hipStream_t s) override {
    if (full) launch_arnoldi_close(S.N, S.V, S.ldv, R.m_cycle, S.st, S.part, S.hf_dev, s);
    launch_trisolve(S.st, s);
    launch_update_x<T>(R.x, Z, ldz, S.N, S.st, s);
    ++R.restarts;
    R.batched = false;
    R.phase = SolveRun::RESTART;
  }

  void enqueue_iteration(Solver& S, int j, hipStream_t s) {
    T* zj = Z + (size_t)j * ldz;
    apply(S, S.V + (size_t)j * S.ldv, &S.st->sigma[j], zj, S.st, s);
    arnoldi(S, zj, j, s, 0, nullptr);
  }
  // w = A z_j with the FP64 matrix, or the FP32 copy under MIXED32
  void arnoldi(Solver& S, const T* zj, int j, hipStream_t s, int prof_class, hipEvent_t* ev) {
    if constexpr (std::is_same<T, float>::value) {
      if (arn32) {
        launch_arnoldi_step<float, float>(A32, zj, S.W, S.V, S.ldv, j, S.st, S.part, S.hf_dev, s,
                                          prof_class, ev);
        return;
      }
    }
    launch_arnoldi_step<double, T>(S.A64, zj, S.W, S.V, S.ldv, j, S.st, S.part, S.hf_dev, s,
                                   prof_class, ev);
  }
  ~PrecImpl() override {
    for (auto g : graphs)
      if (g) (void)hipGraphExecDestroy(g);
    if (bicg_graph) (void)hipGraphExecDestroy(bicg_graph);
  }

  // Add the event-timed launches of the cycle that just ran (columns
  // 0..k-1; later columns returned at once and are not counted).
  void collect_profile(Solver& S, hipStream_t s) {
    SD_HIP(hipStreamSynchronize(s));
    int k = 0;
    SD_HIP(hipMemcpy(&k, &S.st->k, sizeof(int), hipMemcpyDeviceToHost));
    const double n = (double)S.N;
    const double tz = (double)sizeof(T);
    for (int j = 0; j < k; ++j) {
      float ms = 0.0f;
      SD_HIP(hipEventElapsedTime(&ms, S.prof_ev[(size_t)2 * j], S.prof_ev[(size_t)2 * j + 1]));
      S.prof_seconds += 1e-3 * ms;
      S.prof_launches += 1;
      if (S.prof_class == 1)  // A (values + indices read), z, w, j+1 basis vectors
        S.prof_bytes += (double)S.nnz_A * (arn32 ? 4.0 : 8.0) + 4.0 * (double)S.A64.idx +
                        n * (tz + 8.0) + (j + 1) * 8.0 * n;
      else if (S.prof_class == 2)  // j basis vectors, u_j and w read; v_j, u_{j+1} written
        S.prof_bytes += (j + 4) * 8.0 * n;
      else if (S.prof_class == 4)  // every launch of the application
        S.prof_bytes += precond_bytes(S);
      else {  // V level 0: A_V (values + indices read), x_in, b, w, x_out
        const double nv = (double)S.off[2];
        const double idx = H[0].lev.empty() ? 0.0 : (double)H[0].lev[0].A.idx;
        S.prof_bytes += (double)S.nnz_V0 * tz + 4.0 * idx + nv * (3.0 * tz + 8.0);
      }
    }
  }

  void launch_init_cycle(Solver& S, int m_cycle, hipStream_t s) {
    // only the cycle length changes between cycles; counters stay zero
    launch_set_cycle_length(S.st, m_cycle, s);
  }

  // ------------------------------------------------------------ BiCGSTAB
  BicgVecs<T> bw;
  hipGraphExec_t bicg_graph = nullptr;

  void bicg_alloc(Solver& S) {
    if (bw.r) return;
    DeviceMem& mem = *S.mem;
    const size_t n = (size_t)S.ldv;
    bw.r = mem.array<double>(n);
    bw.rhat = mem.array<double>(n);
    bw.p = mem.array<double>(n);
    bw.v = mem.array<double>(n);
    bw.s = mem.array<double>(n);
    bw.t = mem.array<double>(n);
    bw.y = mem.array<T>(n);
    bw.z = mem.array<T>(n);
  }

  void bicg_enqueue_iteration(Solver& S, double* x, hipStream_t s) {
    launch_bicg_iteration_part<T>(0, S.A64, bw, x, S.st, S.part, S.hf_dev, 0, s);
    apply(S, bw.p, nullptr, bw.y, nullptr, s);
    launch_bicg_iteration_part<T>(1, S.A64, bw, x, S.st, S.part, S.hf_dev, 0, s);
    apply(S, bw.s, nullptr, bw.z, nullptr, s);
    launch_bicg_iteration_part<T>(2, S.A64, bw, x, S.st, S.part, S.hf_dev, 0, s);
  }

  int bicgstab(Solver& S, const double* b, double* x, int use_x0, sd_stats* stats,
               hipStream_t user) override {
    hipStream_t s = S.stream;
    SD_HIP(hipEventRecord(S.ev_join, user));
    SD_HIP(hipStreamWaitEvent(s, S.ev_join, 0));
    bicg_alloc(S);
    const double t0 = wall_time();
    const sd_solver_opts& o = S.opts.o;
    const int n = S.N;
    launch_init_state(S.st, o.maxit, 0.0, s);
    launch_norm_b(b, n, o.tol, S.st, S.part, s);
    HostState hs = read_state(S, s);
    sd_stats out{};
    if (!(hs.bnorm > 0.0)) {
      launch_fill<double>(x, 0.0, n, s);
      SD_HIP(hipStreamSynchronize(s));
      out.t_setup = S.t_setup;
      out.t_solve = wall_time() - t0;
      if (stats) *stats = out;
      return std::isfinite(hs.bnorm) ? SD_OK : SD_E_INVALID;
    }
    if (!use_x0) launch_fill<double>(x, 0.0, n, s);
    // the graph bakes in x; rebuild it when the caller's buffer changes
    if (bicg_graph && bicg_x != x) {
      SD_HIP(hipGraphExecDestroy(bicg_graph));
      bicg_graph = nullptr;
    }
    bool first = true;
    int status = SD_E_NOCONV, restarts = 0, breakdowns = 0, last_iters = -1;
    const int depth = 2;
    for (;;) {
      launch_bicg_restart(S.A64, b, (first && !use_x0) ? nullptr : x, bw.r, bw.rhat, bw.p,
                          bw.v, S.st, S.part, s);
      first = false;
      hs = read_state(S, s);
      if (!std::isfinite(hs.beta)) {
        status = SD_E_BREAKDOWN;
        break;
      }
      if (hs.converged) {
        status = SD_OK;
        break;
      }
      if (hs.iters >= o.maxit) {
        status = SD_E_NOCONV;
        break;
      }
      if (hs.breakdown) {  // a breakdown restarts from the true residual
        if (hs.iters == last_iters || ++breakdowns > 20) {
          status = SD_E_BREAKDOWN;
          break;
        }
        SD_HIP(hipMemsetAsync(&S.st->breakdown, 0, sizeof(int), s));
      }
      last_iters = hs.iters;
      S.hf->cycle_done[0] = 0;
      if (!bicg_graph) {
        hipGraph_t g = nullptr;
        SD_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        bicg_enqueue_iteration(S, x, s);
        SD_HIP(hipStreamEndCapture(s, &g));
        SD_HIP(hipGraphInstantiate(&bicg_graph, g, nullptr, nullptr, 0));
        SD_HIP(hipGraphDestroy(g));
        bicg_x = x;
      }
      const int cap = o.maxit - hs.iters;
      for (int it = 0; it < cap; ++it) {
        SD_HIP(hipGraphLaunch(bicg_graph, s));
        SD_HIP(hipEventRecord(S.events[(size_t)(it % (depth + 1))], s));
        if (it >= depth) {
          SD_HIP(hipEventSynchronize(S.events[(size_t)((it - depth) % (depth + 1))]));
          if (S.hf->cycle_done[0]) break;
        }
      }
      ++restarts;
    }
    // final true residual with per-block norms
    launch_restart_residual(S.A64, b, x, S.V, S.off, S.st, S.part, nullptr, s);
    HostState fin = read_state(S, s);
    out.iters = fin.iters;
    out.restarts = restarts;
    out.rel_res = fin.beta / fin.bnorm;
    for (int k = 0; k < 3; ++k) out.rel_res_block[k] = std::sqrt(fin.resblk[k]) / fin.bnorm;
    out.t_setup = S.t_setup;
    out.t_solve = wall_time() - t0;
    if (stats) *stats = out;
    return status;
  }
  double* bicg_x = nullptr;
};

}  // namespace

std::unique_ptr<PrecBase> make_prec_fp64(Solver& S, hipStream_t s) {
  return std::unique_ptr<PrecBase>(new PrecImpl<double>(S, s));
}
std::unique_ptr<PrecBase> make_prec_fp32(Solver& S, hipStream_t s) {
  return std::unique_ptr<PrecBase>(new PrecImpl<float>(S, s));
}

}  // namespace sd
