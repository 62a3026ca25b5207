// Device-side data structures and kernel launchers (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace sd {

constexpr int kMaxBasis = 64;       // FGMRES basis vectors (restart m <= 63)
constexpr int kBlock = 256;         // threads per workgroup (4 wavefronts)
constexpr int kDotBlocks = 512;     // workgroups of the fused reduction kernels
constexpr int kPartStride = kMaxBasis + 4;   // partial-sum rows (k-major, kDotBlocks each)
constexpr int kGsMaxBlocks = 4096;          // row blocks of the Gram-Schmidt kernels
constexpr int kGsProjectRows = 1024;        // preferred rows per projection workgroup
constexpr int kGsMaxRowsPerBlock = 4096;    // rows per projection workgroup (LDS: 16 B each)
// largest system the Gram-Schmidt kernels take (sd_setup rejects more)
constexpr int64_t kMaxUnknowns = (int64_t)kGsMaxBlocks * kGsMaxRowsPerBlock;
// partial-sum rows of the Gram-Schmidt kernels (kGsMaxBlocks each):
// V^T u at kGsRowA, V^T w at kGsRowB, then u.u, u.w, w.w
constexpr int kGsRowA = 0, kGsRowB = kMaxBasis, kGsRowC = 2 * kMaxBasis;
constexpr int kGsPartRows = 2 * kMaxBasis + 3;
constexpr int kIluWidth = 4;        // ILU(0): off-diagonal entries per triangle row
constexpr int kIluMaxLevels = 4096; // ILU(0): levels per substitution

// Sparse matrix on the device.  lpr == 1: sliced ELLPACK with 64-row slices
// (one wavefront per slice); entry (r, k) of slice s lives at
// sptr[s] + 64 k + (r - 64 s), padding has val = 0.  lpr > 1: CSR (sptr holds
// the n_rows + 1 row pointers) read by lpr lanes per row.
//
// Stencil slices (lpr == 1 only): the rows of a slice are stored on the
// ascending union o_0 < o_1 < ... of their offsets col - row (a grid stencil:
// the same few offsets in every row), with an explicit zero at each offset a
// row lacks, and doff[sptr[s] / 64 + k] = o_k (positions past the union
// repeat its last offset).  A wavefront takes entry k's column as row + o_k,
// clamped into [0, n_cols) (the positions that need the clamp hold zeros),
// from one wavefront-uniform load per position instead of a per-lane load of
// col.  stencil == 2: every slice is a stencil slice; stencil == 1:
// doff[sptr[s] / 64] == kIrregularSlice marks the slices read through col (a
// last kIrregularSlice closes the array; slices of width 0 have no entry).
// col stays complete for every slice (the clamped row + o_k in stencil
// slices) except with stencil == 2, where nothing reads it and it is not
// uploaded (col = nullptr).  A zero added to a row sum started at +0 leaves it unchanged, so
// both forms give the same sums.
constexpr int kIrregularSlice = -2147483647 - 1;

template <typename T>
struct Sell {
  const int* sptr = nullptr;
  const int* col = nullptr;
  const T* val = nullptr;
  const int* doff = nullptr;  // stencil offsets, or nullptr: every slice reads col
  int stencil = 0;            // 0: no stencil slices, 1: some, 2: all
  int n_rows = 0;
  int n_cols = 0;
  int lpr = 1;
  int width = 0;   // > 0: every row padded to this width (SELL: slice s at
                   // 64 * width * s; CSR: row r at width * r), sptr not read
  int64_t nnz = 0; // stored entries without padding (algorithmic bytes only)
  int64_t idx = 0; // column indices a pass reads: nnz without stencil slices,
                   // else the irregular slices' unpadded entries + doff length
};

// ILU(0) factors in level order (see HostIlu): positions q of the forward
// and the backward substitution, ELL slots k * n + q.
template <typename T>
struct IluDev {
  int n = 0;
  int nlev_l = 0, nlev_u = 0;
  const int* lev_l = nullptr;
  const int* lev_u = nullptr;
  const int* ord_l = nullptr;
  const int* ord_u = nullptr;
  const int* col_l = nullptr;
  const int* col_u = nullptr;
  const T* val_l = nullptr;
  const T* val_u = nullptr;
  const T* diag_u = nullptr;
};

// Solver scalars resident in device memory.
struct DevState {
  int j;             // Arnoldi column being built
  int k;             // columns completed in this cycle
  int cycle_done;    // iteration kernels return immediately when set
  int m;             // restart length
  int converged;     // true residual <= target
  int breakdown;     // non-finite value seen
  int iters;         // total Arnoldi steps
  int pad0;
  double bnorm, target, cycle_drop, cycle_target, beta;
  double resblk[4];
  double sigma[kMaxBasis + 1];       // preconditioner input scale of V[k]
  double H[(kMaxBasis + 1) * kMaxBasis];   // column-major, ld = kMaxBasis + 1
  double cs[kMaxBasis], sn[kMaxBasis], g[kMaxBasis + 1], y[kMaxBasis];
  double h1[kMaxBasis + 1];          // first-pass coefficients of the open column
  double sums[2 * kMaxBasis + 3];    // reduced Gram-Schmidt dot products of the step
  // BiCGSTAB scalars
  double rho, alpha, omega, bbeta, dots[8];
  unsigned int counter[8];
  int jstep;         // step of the column being replayed (request-loop graph)
};

// Rows per workgroup of the Gram-Schmidt kernels for n rows (base: the
// preferred count); n <= kMaxUnknowns gives at most kGsMaxBlocks blocks.
int gs_rows_per_block(int n, int base);

// Optional per-slot host flags written by the device (mapped pinned memory).
struct HostFlags {
  volatile int cycle_done[kMaxBasis + 2];
  volatile double est[kMaxBasis + 2];
};

// ---- launchers (stream-ordered, no synchronisation) ----

// A launch recorded instead of made: the batched form of the kernel (its
// arguments in a per-slot table, see the request loop), the argument struct
// and the launch shape of this solve.
struct RecordedOp {
  const void* fn = nullptr;
  std::vector<char> args;
  int nblocks = 0, threads = 0;
  size_t lds = 0;
  double bytes = 0.0;   // algorithmic bytes: each matrix entry (value and
                        // index, padding excluded) and each vector entry
                        // read or written once
};
// While rec is set (non-null), the launchers below called on this thread
// append to it instead of launching.
void set_launch_recorder(std::vector<RecordedOp>* rec);
// Whether launches on this thread are being recorded.
bool launch_recording();

template <typename TM, typename TX, typename TY>
void launch_spmv(const Sell<TM>& A, const TX* x, TY* y, const DevState* gate,
                 hipStream_t s);
// r = bscale * b - A x
template <typename T, typename TB>
void launch_residual(const Sell<T>& A, const TB* b, const double* bscale, const T* x,
                     T* r, const DevState* gate, hipStream_t s);
// x = w .* (bscale b) (one sweep from zero), or two sweeps from zero fused
// (A read only for two sweeps)
template <typename T, typename TB>
void launch_jacobi_zero(const Sell<T>& A, const T* wd, const TB* b, const double* bscale,
                        T* x, int two_sweeps, const DevState* gate, hipStream_t s);
// x_out = x_in + w .* (bscale b - A x_in)
template <typename T, typename TB>
void launch_jacobi(const Sell<T>& A, const T* wd, const TB* b, const double* bscale,
                   const T* x_in, T* x_out, const DevState* gate, hipStream_t s);
// bc = Q [bscale b; x] with Q = [R | -R A] (n_fine = length of b and x):
// the restricted residual R (bscale b - A x) in one pass
template <typename T, typename TB>
void launch_restrict_residual(const Sell<T>& Q, const TB* b, const double* bscale, const T* x,
                              int n_fine, T* bc, const DevState* gate, hipStream_t s);
// Two damped-Jacobi sweeps from zero (x; AW = A diag(w)) and bc = G b, one
// launch (G = R (I - A M2) from presmoothed_restriction, 64 lanes per row)
template <typename T, typename TB>
void launch_presmooth_restrict(const Sell<T>& AW, const T* wd, const Sell<T>& G, const TB* b,
                               const double* bscale, T* x, T* bc, const DevState* gate,
                               hipStream_t s);
// xout = x + w .* (bscale b - A x) + F xc (F = P - W A P, stored with A's lanes)
template <typename T, typename TB>
void launch_prolong_smooth(const Sell<T>& A, const Sell<T>& F, const T* wd, const TB* b,
                           const double* bscale, const T* x, const T* xc, T* xout,
                           const DevState* gate, hipStream_t s);
// x += P xc
template <typename T>
void launch_prolong(const Sell<T>& P, const T* xc, T* x, const DevState* gate,
                    hipStream_t s);
// xc = Ainv bc (FP64 dense)
// z = U^-1 L^-1 r with the ILU(0) factors, one workgroup (z may not alias r)
template <typename T>
void launch_ilu0(const IluDev<T>& F, const T* r, T* z, const DevState* gate, hipStream_t s);
template <typename T>
void launch_coarse(const double* Ainv, int n, const T* bc, T* xc, const DevState* gate,
                   hipStream_t s);
// Block sweep: rows of the continuity and porous blocks.
//   t = bscale * r[row] - (Cf y_v)[row]; rows < n_p: zp = xscale * t (and
//   tp = t when tp is not null); else tq = t
template <typename T>
void launch_block_sweep(const Sell<T>& Cf, int n_p, const double* r, const double* bscale,
                        const T* yv, double xscale, T* zp, T* tq, T* tp, const DevState* gate,
                        hipStream_t s);
// y += a
template <typename T>
void launch_add(const T* a, T* y, int n, const DevState* gate, hipStream_t s);
// One Arnoldi step j with delayed reorthogonalisation (FP64 basis V, leading
// dimension ldv).  On entry V[0..j-1] are orthonormal and V[j] holds u_j, the
// once-orthogonalised candidate; z = M(sigma_j u_j).  The step computes
// w = A z and, with one reduction and two passes over the basis, normalises
// v_j = (u_j - V a)/nu (a = V^T u_j), writes the candidate u_{j+1} =
// w - V b - h_jj v_j into V[j+1], completes Hessenberg column j-1, its Givens
// rotation and the residual estimate (flags for column j-1 at index j), and
// records column j's first-pass coefficients and sigma_{j+1}.
// All kernels return immediately once st->cycle_done is set.
// ev (optional, 2 events): recorded around the kernel selected by prof_class
// (1: product + projection pass, 2: update pass).
template <typename TM, typename TZ>
void launch_arnoldi_step(const Sell<TM>& A, const TZ* z, double* W, double* V, int64_t ldv,
                         int j, DevState* st, double* part, HostFlags* hf, hipStream_t s,
                         int prof_class = 0, hipEvent_t* ev = nullptr);
// j < 0 in launch_arnoldi_step: the step index comes from st->jstep, written
// by launch_copy_in, which copies u_j = V[j] (j = st->j) and sigma_j into the
// fixed buffers rin and sig; launch_copy_out stores zfix into Z[j].  The
// column kernels of such a step do nothing once the cycle is done or at
// j >= st->m.  (The request loop replays one recorded column this way.)
void launch_copy_in(const double* V, int64_t ldv, DevState* st, double* rin, double* sig, int n,
                    hipStream_t s);
template <typename T>
void launch_copy_out(const T* zfix, T* Z, int64_t ldz, const DevState* st, int n, hipStream_t s);
// Completes column j-1 = m-1 at the end of a full cycle of m = j columns.
void launch_arnoldi_close(int n, double* V, int64_t ldv, int j, DevState* st, double* part,
                          HostFlags* hf, hipStream_t s);
void launch_trisolve(DevState* st, hipStream_t s);
template <typename TZ>
void launch_update_x(double* x, const TZ* Z, int64_t ldz, int n, DevState* st,
                     hipStream_t s);
// r = b - A x into V[0]; norms; starts a cycle.  x == nullptr means x = 0.
void launch_restart_residual(const Sell<double>& A, const double* b, const double* x,
                             double* r, const int64_t* blk_off, DevState* st, double* part,
                             HostFlags* hf, hipStream_t s);
// r = b - A x (x == nullptr: x = 0) and norms[0..3] = ||r||, ||r_v||, ||r_p||,
// ||r_q|| (device); part holds 3 * kDotBlocks partial sums.
void launch_residual_norms(const Sell<double>& A, const double* b, const double* x, double* r,
                           const int64_t* blk_off, double* part, double* norms, hipStream_t s);
// The same with the partials in the library's static device scratch (no
// allocation; concurrent calls on one GPU race).  Throws sd::Error.
void launch_residual_norms_noalloc(const Sell<double>& A, const double* b, const double* x,
                                   double* r, const int64_t* blk_off, double* norms,
                                   hipStream_t s);
// ||b||, sets target = tol ||b||.
void launch_norm_b(const double* b, int n, double tol, DevState* st, double* part,
                   hipStream_t s);
void launch_init_state(DevState* st, int m, double cycle_drop, hipStream_t s);
void launch_set_cycle_length(DevState* st, int m, hipStream_t s);
// out = (T)(bscale * b)
template <typename TB, typename T>
void launch_scale_convert(const TB* b, const double* bscale, T* out, int n, const DevState* gate,
                          hipStream_t s);

// BiCGSTAB work vectors (FP64 Krylov vectors; y, z preconditioned, type T).
template <typename T>
struct BicgVecs {
  double *r = nullptr, *rhat = nullptr, *p = nullptr, *v = nullptr, *s = nullptr, *t = nullptr;
  T *y = nullptr, *z = nullptr;
};
// which: 0 = p update; 1 = v = A y, alpha, s = r - alpha v, x += alpha y,
// ||s||; 2 = t = A z, omega, x += omega z, r = s - omega t, ||r||, next rho.
template <typename T>
void launch_bicg_iteration_part(int which, const Sell<double>& A, BicgVecs<T>& w, double* x,
                                DevState* st, double* part, HostFlags* hf, int slot,
                                hipStream_t s);
// r = b - A x (x null: zero), rhat = r, p = v = 0, scalars reset.
void launch_bicg_restart(const Sell<double>& A, const double* b, const double* x, double* r,
                         double* rhat, double* p, double* v, DevState* st, double* part,
                         hipStream_t s);

// Type conversions and small vector helpers.
template <typename TA, typename TB>
void launch_convert(const TA* a, TB* b, int n, hipStream_t s);
template <typename T>
void launch_fill(T* a, T v, int n, hipStream_t s);

// Backward-Euler right-hand side: out = b + m x on the velocity rows with a
// time derivative (u rows r < off_v with 1 <= r % nux + ifirst <= nx - 1, v
// rows off_v + v_skip <= r < off_w, w rows off_w <= r < off_p), b elsewhere;
// no fused multiply-add.
void launch_step_rhs(const double* b, const double* x, double* out, double m, int n, int nux,
                     int ifirst, int nx, int off_v, int v_skip, int off_w, int off_p,
                     hipStream_t s);

}  // namespace sd
