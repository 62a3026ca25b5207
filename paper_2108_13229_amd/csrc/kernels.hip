// HIP kernels of the coupled Stokes-Darcy solver for gfx950 (CDNA4).
//
// Everything here is bandwidth-bound sparse or vector work (about 0.1 - 0.25
// flop per byte), so the kernels are organised for coalesced HBM traffic:
//   * sparse matrices are sliced ELLPACK with 64-row slices: one wavefront
//     owns a slice, lane r owns row r, and entry k of all 64 rows is one
//     contiguous 256 B (index) + 256/512 B (value) segment;
//   * workgroup indices are remapped so that each of the 8 XCDs streams a
//     contiguous range of rows (neighbouring rows share x entries in its L2);
//   * reductions are two-stage and deterministic: wavefront shuffles, then
//     LDS across the 4 wavefronts of a workgroup, then the per-workgroup
//     partials are summed in a fixed order by a one-workgroup kernel that also
//     does the scalar follow-up work (Givens rotations, scale factors).  A
//     grid-wide "last workgroup" ticket would need an agent-scope release
//     fence in every workgroup, which on this chip writes back the XCD's whole
//     L2; a kernel boundary is far cheaper.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <string>
#include <type_traits>

#include "device.h"
#include "sd_internal.h"

// Device scratch of the allocation-free residual (sd_residual_noalloc): the
// 3 x kDotBlocks block partials of its norms, 12 KiB, one copy per GPU that
// the library runs on, held until the process ends.  Host code never uses
// this name as an address: it takes each device's address once from
// hipGetSymbolAddress (noalloc_scratch below).
static __device__ __align__(256) double scratch[3 * sd::kDotBlocks];

namespace sd {

namespace {

__device__ __forceinline__ int xcd_block(int b, int nb) {
  const int q = nb >> 3, r = nb & 7, x = b & 7, k = b >> 3;
  return x * q + (x < r ? x : r) + k;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// A load that is cached normally, or (NT) non-temporally: data read once
// per iteration should not evict what the iteration reads repeatedly.
template <bool NT, typename T>
__device__ __forceinline__ T load_hint(const T* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}

// M consecutive entries e, e + step, ... of a SELL row added to acc in
// order; the M index/value loads and then the M gathers are all issued
// before the first product.  NT: the index and value loads are
// non-temporal.
template <int M, bool NT = false, typename TM, typename F>
__device__ __forceinline__ void sell_chunk(const Sell<TM>& A, int e, int step, F f, TM& acc) {
  int c[M];
  TM v[M];
#pragma unroll
  for (int i = 0; i < M; ++i) {
    c[i] = load_hint<NT>(&A.col[e + i * step]);
    v[i] = load_hint<NT>(&A.val[e + i * step]);
  }
  TM x[M];
#pragma unroll
  for (int i = 0; i < M; ++i) x[i] = f(c[i]);
#pragma unroll
  for (int i = 0; i < M; ++i) acc += v[i] * x[i];
}

template <int M, bool NT, typename TM, typename F>
__device__ __forceinline__ void sell_tail(const Sell<TM>& A, int e, int cnt, int step, F f,
                                          TM& acc) {
  if constexpr (M > 0) {
    if (cnt == M) sell_chunk<M, NT>(A, e, step, f, acc);
    else sell_tail<M - 1, NT>(A, e, cnt, step, f, acc);
  }
}

// The cnt entries e, e + step, ... of a SELL row, summed in that order: K at
// a time, then one chunk of the cnt % K left, so a row of up to K entries
// costs two dependent memory round trips (indices and values, then the
// gathers) and no load is issued for an entry the row does not have.  cnt
// is the same for all lanes of a slice, so the tail takes one branch.
template <int K, bool NT = false, typename TM, typename F>
__device__ __forceinline__ TM sell_row(const Sell<TM>& A, int e, int cnt, int step, F f) {
  TM acc = 0;
  for (; cnt >= K; cnt -= K, e += K * step) sell_chunk<K, NT>(A, e, step, f, acc);
  sell_tail<K - 1, NT>(A, e, cnt, step, f, acc);
  return acc;
}

// Read-only data that no kernel writes while it runs (slice pointers,
// stencil offsets): read through the constant address space, a
// wavefront-uniform address becomes a scalar load.
typedef const __attribute__((address_space(4))) int* const_ints;

__device__ __forceinline__ const_ints as_const(const int* p) { return (const_ints)p; }

// The same sum over a stencil slice (see Sell): entry k of the row sits at
// column row + o[k] clamped into [0, n_cols), o the slice's offsets (the
// same address in every lane), and only the values are loaded per lane.
// The entries are added in the same order as by sell_row.
template <int M, bool NT, typename TM, typename F>
__device__ __forceinline__ void stencil_chunk(const Sell<TM>& A, int e, const_ints o, int row,
                                              F f, TM& acc) {
  TM v[M];
  int c[M];
  const int last = A.n_cols - 1;
#pragma unroll
  for (int i = 0; i < M; ++i) {
    v[i] = load_hint<NT>(&A.val[e + i * 64]);
    c[i] = min(max(row + o[i], 0), last);
  }
  TM x[M];
#pragma unroll
  for (int i = 0; i < M; ++i) x[i] = f(c[i]);
#pragma unroll
  for (int i = 0; i < M; ++i) acc += v[i] * x[i];
}

template <int M, bool NT, typename TM, typename F>
__device__ __forceinline__ void stencil_tail(const Sell<TM>& A, int e, int cnt, const_ints o,
                                             int row, F f, TM& acc) {
  if constexpr (M > 0) {
    if (cnt == M) stencil_chunk<M, NT>(A, e, o, row, f, acc);
    else stencil_tail<M - 1, NT>(A, e, cnt, o, row, f, acc);
  }
}

template <int K, bool NT = false, typename TM, typename F>
__device__ __forceinline__ TM stencil_row(const Sell<TM>& A, int e, int cnt, const_ints o,
                                          int row, F f) {
  TM acc = 0;
  for (; cnt >= K; cnt -= K, e += K * 64, o += K) stencil_chunk<K, NT>(A, e, o, row, f, acc);
  stencil_tail<K - 1, NT>(A, e, cnt, o, row, f, acc);
  return acc;
}

// The offsets of the wavefront's slice whose first entry is at sbase (a
// multiple of 64), or nullptr if the slice is read through col.  Callers
// give every wavefront one slice, so sbase is uniform.
template <typename TM>
__device__ __forceinline__ const_ints stencil_of(const Sell<TM>& A, int sbase) {
  if (!A.stencil) return nullptr;
  const_ints o = as_const(A.doff) + (sbase >> 6);
  if (A.stencil == 2) return o;
  return o[0] == kIrregularSlice ? nullptr : o;
}

constexpr int kRowChunk = 6;   // entries of a SELL-64 row loaded at once

// Row `row` of a SELL-64 matrix times x.  The caller's wavefront holds the
// 64 rows of one slice (64 consecutive rows from a multiple of 64).
template <int K = kRowChunk, bool NT = false, typename TM, typename TX>
__device__ __forceinline__ TM sell_dot(const Sell<TM>& A, const TX* __restrict__ x, int row) {
  const int s = __builtin_amdgcn_readfirstlane(row >> 6);
  const int sbase = as_const(A.sptr)[s];
  const int cnt = (as_const(A.sptr)[s + 1] - sbase) >> 6;
  const auto f = [&](int c) { return (TM)x[c]; };
  if (const_ints o = stencil_of(A, sbase)) return stencil_row<K, NT>(A, sbase + (row & 63), cnt, o, row, f);
  return sell_row<K, NT>(A, sbase + (row & 63), cnt, 64, f);
}

__device__ __forceinline__ double scale_of(const double* s) { return s ? *s : 1.0; }

template <typename T, typename TB>
__device__ __forceinline__ T load_b(const TB* __restrict__ b, double s, int i) {
  return (T)((double)b[i] * s);
}

// Sum the first nv entries of acc over the workgroup into the k-major
// partial buffer: part[k * kDotBlocks + block].
template <int NV>
__device__ __forceinline__ void block_partials(const double (&acc)[NV], int nv, double* part) {
  __shared__ double red[kBlock / 64][NV];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    if (k < nv) {
      const double v = wave_sum(acc[k]);
      if (lane == 0) red[wave][k] = v;
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < nv) {
    const int k = threadIdx.x;
    part[(size_t)k * kDotBlocks + blockIdx.x] = ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k];
  }
}

// Whole workgroup: out_sh[k] = sum over b < nb of part[k * kDotBlocks + b],
// k < nv, in a fixed order (identical in every workgroup that calls it).
template <int NV>
__device__ __forceinline__ void final_sums(const double* part, int nb, int nv, double* out_sh) {
  __shared__ double red[kBlock / 64][NV];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = 0.0;
  for (int b = threadIdx.x; b < nb; b += kBlock) {
#pragma unroll
    for (int k = 0; k < NV; ++k)
      if (k < nv) acc[k] += part[(size_t)k * kDotBlocks + b];
  }
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    if (k < nv) {
      const double v = wave_sum(acc[k]);
      if (lane == 0) red[wave][k] = v;
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < nv) {
    const int k = threadIdx.x;
    out_sh[k] = ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k];
  }
  __syncthreads();
}

inline int blocks_for(int n) { return (n + kBlock - 1) / kBlock; }

inline int dot_blocks(int n) {
  const int nb = (n + kBlock - 1) / kBlock;
  return nb < kDotBlocks ? (nb > 0 ? nb : 1) : kDotBlocks;
}

// ----------------------------------------------------------------- kernels

// Row access for the V-cycle kernels: SELL-C with C = 64 / LPR rows per
// slice and LPR lanes per row.  A wavefront owns one slice; lane
// (sub, r) = (lane / C, lane % C) handles entries sub, sub + LPR, ... of row
// r, and entry k of row r lives at slice base + k C + r, so each load
// instruction reads 64 consecutive entries and the gathers of C neighbouring
// rows share cache lines.  LPR == 1 is SELL-64 (finest levels, short rows);
// LPR > 1 serves coarse levels and transfer operators, whose rows are long
// and few.  A uniform width (A.width > 0, a multiple of LPR) replaces the
// slice pointers and spares their load at the head of each load chain.
template <int LPR, typename TM, typename F>
__device__ __forceinline__ TM row_sum(const Sell<TM>& A, int row, int sub, F f) {
  constexpr int C = 64 / LPR;
  // row_of_thread gives each wavefront one slice
  const int sl = __builtin_amdgcn_readfirstlane(row / C), r = row - sl * C;
  int beg, end;
  if (A.width) {
    beg = sl * (C * A.width);
    end = beg + C * A.width;
  } else {
    beg = as_const(A.sptr)[sl];
    end = as_const(A.sptr)[sl + 1];
  }
  if constexpr (LPR == 1) {
    if (const_ints o = stencil_of(A, beg)) return stencil_row<kRowChunk>(A, beg + r, (end - beg) >> 6, o, row, f);
  }
  const int e0 = beg + sub * C + r;
  TM acc = sell_row<LPR == 1 ? kRowChunk : 4>(A, e0, (end - e0 + 63) >> 6, 64, f);
#pragma unroll
  for (int o = C; o < 64; o <<= 1) acc += __shfl_xor(acc, o, 64);
  return acc;
}

// thread -> (row, lane within the row group); consecutive wavefronts of a
// workgroup take consecutive slices, workgroups XCD-contiguous row ranges
template <int LPR>
__device__ __forceinline__ int2 row_of_thread(int block, int nblocks) {
  constexpr int C = 64 / LPR;
  const int gt = xcd_block(block, nblocks) * kBlock + threadIdx.x;
  const int lane = gt & 63;
  return make_int2((gt >> 6) * C + lane % C, lane / C);
}

// The cycle-done flag of the gated kernels, read with a vector load through
// an opaque pointer so that it is in flight together with the kernel's first
// loads (a scalar load would be waited for before them); the kernels test it
// just before their stores.
__device__ __forceinline__ int gate_flag(const DevState* gate) {
  if (!gate) return 0;
  const int* p = &gate->cycle_done;
  asm volatile("" : "+v"(p));
  return *p;
}


// ---- V-cycle and block-sweep kernels.  Each is an Op: its arguments in a
// struct and a body run(a, block, nblocks) for workgroup `block` of
// `nblocks`.  A named kernel (k_spmv, k_jacobi, ...) runs one Op over its
// grid; k_batch runs the same Op for every slot of a batch of solves (the
// request loop's shared launches), each slot with its own arguments and
// workgroup count, so a solve computes the same values in either form.

template <int LPR, typename TM, typename TX, typename TY>
struct SpmvOp {
  struct Args {
    Sell<TM> A;
    const TX* x;
    TY* y;
    const DevState* gate;
  };
  static constexpr int kThreads = kBlock;
  static __device__ __forceinline__ void run(const Args& a, int block, int nblocks) {
    const int2 rs = row_of_thread<LPR>(block, nblocks);
    if (rs.x >= a.A.n_rows) return;
    const int stop = gate_flag(a.gate);
    const TX* __restrict__ x = a.x;
    const TM v = row_sum<LPR>(a.A, rs.x, rs.y, [&](int c) { return (TM)x[c]; });
    if (rs.y == 0 && !stop) a.y[rs.x] = (TY)v;
  }
};

// r = bscale * b - A x
template <int LPR, typename T, typename TB>
struct ResidualOp {
  struct Args {
    Sell<T> A;
    const TB* b;
    const double* bscale;
    const T* x;
    T* r;
    const DevState* gate;
  };
  static constexpr int kThreads = kBlock;
  static __device__ __forceinline__ void run(const Args& a, int block, int nblocks) {
    const int2 rs = row_of_thread<LPR>(block, nblocks);
    if (rs.x >= a.A.n_rows) return;
    const int stop = gate_flag(a.gate);
    const T* __restrict__ x = a.x;
    const T ax = row_sum<LPR>(a.A, rs.x, rs.y, [&](int c) { return x[c]; });
    if (rs.y == 0 && !stop) a.r[rs.x] = load_b<T>(a.b, scale_of(a.bscale), rs.x) - ax;
  }
};

// bc = Q [bscale b; x] = R (bscale b - A x): residual and restriction in one
// product over the coarse rows (columns >= n_fine address x).
template <int LPR, typename T, typename TB>
struct RestrictResidualOp {
  struct Args {
    Sell<T> Q;
    const TB* b;
    const double* bscale;
    const T* x;
    int n_fine;
    T* bc;
    const DevState* gate;
  };
  static constexpr int kThreads = kBlock;
  static __device__ __forceinline__ void run(const Args& a, int block, int nblocks) {
    const int2 rs = row_of_thread<LPR>(block, nblocks);
    if (rs.x >= a.Q.n_rows) return;
    const int stop = gate_flag(a.gate);
    const double sc = scale_of(a.bscale);
    const TB* __restrict__ b = a.b;
    const T* __restrict__ x = a.x;
    const int n_fine = a.n_fine;
    const T v = row_sum<LPR>(a.Q, rs.x, rs.y, [&](int c) {
      return c < n_fine ? load_b<T>(b, sc, c) : x[c - n_fine];
    });
    if (rs.y == 0 && !stop) a.bc[rs.x] = v;
  }
};

// Pre-smoothing and restriction in one launch, both from b alone: the first
// nb_a workgroups run two damped-Jacobi sweeps from zero on the rows of A
// (x = (2W - W A W) b, with A passed as A diag(w)), the others compute
// bc = G b with G = R (I - A M2) (one wavefront per row: G's rows are long).
template <int LA, typename T, typename TB>
struct PresmoothRestrictOp {
  struct Args {
    Sell<T> A;
    const T* wd;
    Sell<T> G;
    const TB* b;
    const double* bscale;
    T* x;
    T* bc;
    int nb_a;
    const DevState* gate;
  };
  static constexpr int kThreads = kBlock;
  static __device__ __forceinline__ void run(const Args& a, int block, int nblocks) {
    const int stop = gate_flag(a.gate);
    const double s = scale_of(a.bscale);
    const TB* __restrict__ b = a.b;
    if (block < a.nb_a) {
      const int2 rs = row_of_thread<LA>(block, a.nb_a);
      const int row = rs.x, sub = rs.y;
      if (row >= a.A.n_rows) return;
      const T bi = load_b<T>(b, s, row);
      const T acc = row_sum<LA>(a.A, row, sub, [&](int c) { return load_b<T>(b, s, c); });
      if (sub == 0 && !stop) a.x[row] = a.wd[row] * bi + a.wd[row] * (bi - acc);
    } else {
      const int2 rs = row_of_thread<64>(block - a.nb_a, nblocks - a.nb_a);
      const int row = rs.x, sub = rs.y;
      if (row >= a.G.n_rows) return;
      const T v = row_sum<64>(a.G, row, sub, [&](int c) { return load_b<T>(b, s, c); });
      if (sub == 0 && !stop) a.bc[row] = v;
    }
  }
};

// Coarse correction and the first post-smoothing sweep in one pass:
// xout = x + W (b - A x) + F xc with F = P - W A P (F stored with A's lanes).
template <int LA, typename T, typename TB>
struct ProlongSmoothOp {
  struct Args {
    Sell<T> A, F;
    const T* wd;
    const TB* b;
    const double* bscale;
    const T* x;
    const T* xc;
    T* xout;
    const DevState* gate;
  };
  static constexpr int kThreads = kBlock;
  static __device__ __forceinline__ void run(const Args& a, int block, int nblocks) {
    const int2 rs = row_of_thread<LA>(block, nblocks);
    const int row = rs.x;
    if (row >= a.A.n_rows) return;
    const int stop = gate_flag(a.gate);
    const T* __restrict__ x = a.x;
    const T* __restrict__ xc = a.xc;
    const T ax = row_sum<LA>(a.A, row, rs.y, [&](int c) { return x[c]; });
    const T fx = row_sum<LA>(a.F, row, rs.y, [&](int c) { return xc[c]; });
    if (rs.y == 0 && !stop)
      a.xout[row] = x[row] + a.wd[row] * (load_b<T>(a.b, scale_of(a.bscale), row) - ax) + fx;
  }
};

// x = w .* b (one sweep from zero) or two sweeps from zero fused: the first
// sweep's values x1 = w .* b are recomputed at the neighbours (a gather of b
// and of w each), so the pass reads A, the matrix the residual and the
// post-sweeps read next.
template <int LPR, typename T, typename TB>
struct JacobiZeroOp {
  struct Args {
    Sell<T> A;
    const T* wd;
    const TB* b;
    const double* bscale;
    T* x;
    int two;
    const DevState* gate;
  };
  static constexpr int kThreads = kBlock;
  static __device__ __forceinline__ void run(const Args& a, int block, int nblocks) {
    const int2 rs = row_of_thread<LPR>(block, nblocks);
    const int row = rs.x;
    if (row >= a.A.n_rows) return;
    const int stop = gate_flag(a.gate);
    const double s = scale_of(a.bscale);
    const TB* __restrict__ b = a.b;
    const T bi = load_b<T>(b, s, row);
    const T x1 = a.wd[row] * bi;
    if (!a.two) {
      if (rs.y == 0 && !stop) a.x[row] = x1;
      return;
    }
    const T* __restrict__ wd = a.wd;
    const T acc = row_sum<LPR>(a.A, row, rs.y, [&](int c) { return wd[c] * load_b<T>(b, s, c); });
    if (rs.y == 0 && !stop) a.x[row] = x1 + a.wd[row] * (bi - acc);
  }
};

// x_out = x_in + w .* (bscale b - A x_in)
template <int LPR, typename T, typename TB>
struct JacobiOp {
  struct Args {
    Sell<T> A;
    const T* wd;
    const TB* b;
    const double* bscale;
    const T* xin;
    T* xout;
    const DevState* gate;
  };
  static constexpr int kThreads = kBlock;
  static __device__ __forceinline__ void run(const Args& a, int block, int nblocks) {
    const int2 rs = row_of_thread<LPR>(block, nblocks);
    const int row = rs.x;
    if (row >= a.A.n_rows) return;
    const int stop = gate_flag(a.gate);
    const T* __restrict__ xin = a.xin;
    const T ax = row_sum<LPR>(a.A, row, rs.y, [&](int c) { return xin[c]; });
    if (rs.y == 0 && !stop)
      a.xout[row] = xin[row] + a.wd[row] * (load_b<T>(a.b, scale_of(a.bscale), row) - ax);
  }
};

// x += P xc
template <int LPR, typename T>
struct ProlongOp {
  struct Args {
    Sell<T> P;
    const T* xc;
    T* x;
    const DevState* gate;
  };
  static constexpr int kThreads = kBlock;
  static __device__ __forceinline__ void run(const Args& a, int block, int nblocks) {
    const int2 rs = row_of_thread<LPR>(block, nblocks);
    if (rs.x >= a.P.n_rows) return;
    const int stop = gate_flag(a.gate);
    const T* __restrict__ xc = a.xc;
    const T v = row_sum<LPR>(a.P, rs.x, rs.y, [&](int c) { return xc[c]; });
    if (rs.y == 0 && !stop) a.x[rs.x] += v;
  }
};

constexpr int kIluThreads = 1024;

// z = U^-1 L^-1 r with the ILU(0) factors of the Darcy block, in one
// workgroup.  The rows of one level of a substitution depend only on rows of
// earlier levels, so a level is one parallel step and a barrier orders the
// levels (after it the workgroup sees its own global stores).  The forward
// result y is kept in z and overwritten by the backward pass.  A position's
// row index and slots are loaded at once, then the gathers; padded slots
// (col -1) read z[0] and add nothing.
template <typename T>
struct Ilu0Op {
  struct Args {
    IluDev<T> F;
    const T* r;
    T* z;
    const DevState* gate;
  };
  static constexpr int kThreads = kIluThreads;
  static __device__ __forceinline__ void run(const Args& a, int, int) {
    __shared__ int lev[2][kIluMaxLevels + 1];
    if (a.gate && a.gate->cycle_done) return;
    const IluDev<T>& F = a.F;
    const T* __restrict__ r = a.r;
    T* z = a.z;
    const int t = threadIdx.x;
    const size_t n = (size_t)F.n;
    for (int l = t; l <= F.nlev_l; l += kIluThreads) lev[0][l] = F.lev_l[l];
    for (int l = t; l <= F.nlev_u; l += kIluThreads) lev[1][l] = F.lev_u[l];
    __syncthreads();
    for (int lv = 0; lv < F.nlev_l; ++lv) {
      const int q1 = lev[0][lv + 1];
      for (int q = lev[0][lv] + t; q < q1; q += kIluThreads) {
        const int i = F.ord_l[q];
        int c[kIluWidth];
        T v[kIluWidth];
#pragma unroll
        for (int k = 0; k < kIluWidth; ++k) {
          c[k] = F.col_l[k * n + q];
          v[k] = F.val_l[k * n + q];
        }
        T x[kIluWidth];
#pragma unroll
        for (int k = 0; k < kIluWidth; ++k) x[k] = z[max(c[k], 0)];
        T acc = r[i];
#pragma unroll
        for (int k = 0; k < kIluWidth; ++k) acc = c[k] >= 0 ? acc - v[k] * x[k] : acc;
        z[i] = acc;
      }
      __syncthreads();
    }
    for (int lv = 0; lv < F.nlev_u; ++lv) {
      const int q1 = lev[1][lv + 1];
      for (int q = lev[1][lv] + t; q < q1; q += kIluThreads) {
        const int i = F.ord_u[q];
        int c[kIluWidth];
        T v[kIluWidth];
#pragma unroll
        for (int k = 0; k < kIluWidth; ++k) {
          c[k] = F.col_u[k * n + q];
          v[k] = F.val_u[k * n + q];
        }
        const T d = F.diag_u[q];
        T x[kIluWidth];
#pragma unroll
        for (int k = 0; k < kIluWidth; ++k) x[k] = z[max(c[k], 0)];
        T acc = z[i];
#pragma unroll
        for (int k = 0; k < kIluWidth; ++k) acc = c[k] >= 0 ? acc - v[k] * x[k] : acc;
        z[i] = acc / d;
      }
      __syncthreads();
    }
  }
};

// xc = Ainv bc, FP64 dense inverse: one workgroup per row (the coarse rows
// are few), each thread with up to eight loads in flight.
template <typename T>
struct CoarseOp {
  struct Args {
    const double* Ainv;
    int n;
    const T* bc;
    T* xc;
    const DevState* gate;
  };
  static constexpr int kThreads = kBlock;
  static __device__ __forceinline__ void run(const Args& a, int block, int) {
    __shared__ double red[kBlock / 64];
    const int stop = gate_flag(a.gate);
    const int n = a.n;
    const double* __restrict__ arow = a.Ainv + (size_t)block * n;
    const T* __restrict__ bc = a.bc;
    double sp[4] = {0.0, 0.0, 0.0, 0.0};
    for (int c0 = threadIdx.x; c0 < n; c0 += 8 * kBlock) {
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int c = c0 + u * kBlock;
        if (c < n) sp[u & 3] += arow[c] * (double)bc[c];
      }
    }
    const double v = wave_sum((sp[0] + sp[1]) + (sp[2] + sp[3]));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0 && !stop) a.xc[block] = (T)(((red[0] + red[1]) + red[2]) + red[3]);
  }
};

// Block sweep: rows of the continuity and porous blocks.
template <typename T>
struct BlockSweepOp {
  struct Args {
    Sell<T> Cf;
    int n_p;
    const double* r;
    const double* bscale;
    const T* yv;
    double xscale;
    T* zp;
    T* tq;
    T* tp;
    const DevState* gate;
  };
  static constexpr int kThreads = kBlock;
  static __device__ __forceinline__ void run(const Args& a, int block, int nblocks) {
    const int row = xcd_block(block, nblocks) * kBlock + threadIdx.x;
    if (row >= a.Cf.n_rows) return;
    const int stop = gate_flag(a.gate);
    const T t = load_b<T>(a.r, scale_of(a.bscale), row) - sell_dot(a.Cf, a.yv, row);
    if (stop) return;
    if (row < a.n_p) {
      a.zp[row] = (T)a.xscale * t;
      if (a.tp) a.tp[row] = t;     // right-hand side of the pressure-operator V-cycle
    } else {
      a.tq[row - a.n_p] = t;
    }
  }
};

// y += a (the pressure-operator V-cycle's share of the middle block).
template <typename T>
struct AddOp {
  struct Args {
    const T* a;
    T* y;
    int n;
    const DevState* gate;
  };
  static constexpr int kThreads = kBlock;
  static __device__ __forceinline__ void run(const Args& p, int block, int) {
    const int i = block * kBlock + threadIdx.x;
    if (i >= p.n) return;
    const int stop = gate_flag(p.gate);
    const T v = p.a[i];
    const T w = p.y[i];
    if (stop) return;
    p.y[i] = w + v;
  }
};

// out = (T)(bscale * b)
template <typename TB, typename T>
struct ScaleConvertOp {
  struct Args {
    const TB* b;
    const double* bscale;
    T* out;
    int n;
    const DevState* gate;
  };
  static constexpr int kThreads = kBlock;
  static __device__ __forceinline__ void run(const Args& a, int block, int) {
    const int i = block * kBlock + threadIdx.x;
    if (i >= a.n) return;
    const int stop = gate_flag(a.gate);
    const T v = load_b<T>(a.b, scale_of(a.bscale), i);
    if (!stop) a.out[i] = v;
  }
};

template <typename TA, typename TB>
struct ConvertOp {
  struct Args {
    const TA* a;
    TB* b;
    int n;
  };
  static constexpr int kThreads = kBlock;
  static __device__ __forceinline__ void run(const Args& p, int block, int) {
    const int i = block * kBlock + threadIdx.x;
    if (i < p.n) p.b[i] = (TB)p.a[i];
  }
};

template <typename T>
struct FillOp {
  struct Args {
    T* a;
    T v;
    int n;
  };
  static constexpr int kThreads = kBlock;
  static __device__ __forceinline__ void run(const Args& p, int block, int) {
    const int i = block * kBlock + threadIdx.x;
    if (i < p.n) p.a[i] = p.v;
  }
};

// Named single launches of the Ops above.
template <int LPR, typename TM, typename TX, typename TY>
__global__ __launch_bounds__(kBlock) void k_spmv(typename SpmvOp<LPR, TM, TX, TY>::Args a) {
  SpmvOp<LPR, TM, TX, TY>::run(a, blockIdx.x, gridDim.x);
}
template <int LPR, typename T, typename TB>
__global__ __launch_bounds__(kBlock) void k_residual(typename ResidualOp<LPR, T, TB>::Args a) {
  ResidualOp<LPR, T, TB>::run(a, blockIdx.x, gridDim.x);
}
template <int LPR, typename T, typename TB>
__global__ __launch_bounds__(kBlock) void k_restrict_residual(
    typename RestrictResidualOp<LPR, T, TB>::Args a) {
  RestrictResidualOp<LPR, T, TB>::run(a, blockIdx.x, gridDim.x);
}
template <int LA, typename T, typename TB>
__global__ __launch_bounds__(kBlock) void k_presmooth_restrict(
    typename PresmoothRestrictOp<LA, T, TB>::Args a) {
  PresmoothRestrictOp<LA, T, TB>::run(a, blockIdx.x, gridDim.x);
}
template <int LA, typename T, typename TB>
__global__ __launch_bounds__(kBlock) void k_prolong_smooth(
    typename ProlongSmoothOp<LA, T, TB>::Args a) {
  ProlongSmoothOp<LA, T, TB>::run(a, blockIdx.x, gridDim.x);
}
template <int LPR, typename T, typename TB>
__global__ __launch_bounds__(kBlock) void k_jacobi_zero(typename JacobiZeroOp<LPR, T, TB>::Args a) {
  JacobiZeroOp<LPR, T, TB>::run(a, blockIdx.x, gridDim.x);
}
template <int LPR, typename T, typename TB>
__global__ __launch_bounds__(kBlock) void k_jacobi(typename JacobiOp<LPR, T, TB>::Args a) {
  JacobiOp<LPR, T, TB>::run(a, blockIdx.x, gridDim.x);
}
template <int LPR, typename T>
__global__ __launch_bounds__(kBlock) void k_prolong(typename ProlongOp<LPR, T>::Args a) {
  ProlongOp<LPR, T>::run(a, blockIdx.x, gridDim.x);
}
template <typename T>
__global__ __launch_bounds__(kIluThreads) void k_ilu0(typename Ilu0Op<T>::Args a) {
  Ilu0Op<T>::run(a, blockIdx.x, gridDim.x);
}
template <typename T>
__global__ __launch_bounds__(kBlock) void k_coarse(typename CoarseOp<T>::Args a) {
  CoarseOp<T>::run(a, blockIdx.x, gridDim.x);
}
template <typename T>
__global__ __launch_bounds__(kBlock) void k_block_sweep(typename BlockSweepOp<T>::Args a) {
  BlockSweepOp<T>::run(a, blockIdx.x, gridDim.x);
}
template <typename T>
__global__ __launch_bounds__(kBlock) void k_add(typename AddOp<T>::Args a) {
  AddOp<T>::run(a, blockIdx.x, gridDim.x);
}
template <typename TB, typename T>
__global__ __launch_bounds__(kBlock) void k_scale_convert(typename ScaleConvertOp<TB, T>::Args a) {
  ScaleConvertOp<TB, T>::run(a, blockIdx.x, gridDim.x);
}
template <typename TA, typename TB>
__global__ __launch_bounds__(kBlock) void k_convert(typename ConvertOp<TA, TB>::Args a) {
  ConvertOp<TA, TB>::run(a, blockIdx.x, gridDim.x);
}
template <typename T>
__global__ __launch_bounds__(kBlock) void k_fill(typename FillOp<T>::Args a) {
  FillOp<T>::run(a, blockIdx.x, gridDim.x);
}

// ---- Arnoldi step j: classical Gram-Schmidt with one reorthogonalisation
// (CGS2), the reorthogonalisation of each vector delayed by one step so that
// it shares a pass over the basis with the projection of the next vector
// (delayed CGS2: Swirydowicz, Langou, Ananthan, Yang, Thomas, "Low
// synchronization Gram-Schmidt and GMRES algorithms", 2021).
//
// On entry to step j the basis slots 0..j-1 hold orthonormal v_0..v_{j-1},
// slot j holds u_j, the once-orthogonalised (unnormalised) candidate for v_j,
// and the preconditioner has produced z_j = M(sigma_j u_j).  Three kernels:
//   project: w = A z_j; partial sums of a = V^T u_j, b = V^T w, u_j.u_j,
//            u_j.w and w.w (one pass over the basis);
//   sum:     one workgroup per partial-sum row adds the rows' partials in
//            a fixed order;
//   update:  every workgroup derives nu = sqrt(u.u - a.a) and
//            h_jj = (u.w - a.b)/nu from the sums and writes
//            v_j = (u_j - V a)/nu, u_{j+1} = w - V b - h_jj v_j (one pass
//            over the basis); the last workgroup completes Hessenberg
//            column j-1 (first-pass coefficients + a, subdiagonal nu),
//            applies the Givens rotations and sets the convergence flag
//            (the residual estimate trails the basis by one step).
// In exact arithmetic a = 0 and the iterates are those of CGS2 FGMRES.  A
// closing step (project without the product, update without row work)
// completes the last column of a full cycle.  Layout of the projection: a
// workgroup of 8 wavefronts owns a block of rows; after the product (one
// 64-row slice per wavefront and round, w and u_j kept in LDS) the basis
// entries of the block are split evenly over the wavefronts as runs of
// (vector, slice) units, so every basis entry is read once, coalesced, with
// several loads in flight per wavefront.

constexpr int kGsThreads = 512;
constexpr int kGsWaves = kGsThreads / 64;
constexpr int kProjChunk = 8;                     // basis slices loaded at once
constexpr int kProjRowChunk = 6;                  // matrix entries per row loaded at once
                                                  // (8 would spill at 64 VGPRs)
constexpr int kSumStride = 2 * kMaxBasis + 4;

// Step index of the Arnoldi kernels: the launch's j, or (j < 0: a launch
// replayed for every column of the request loop's shared graph) the step the
// column's copy-in recorded in st->jstep.
__device__ __forceinline__ int step_of(int j, const DevState* st) {
  return j >= 0 ? j : st->jstep;
}

template <typename TM, typename TZ>
struct ArnProjectOp {
  struct Args {
    Sell<TM> A;
    const TZ* z;
    double* W;
    const double* V;
    int64_t ldv;
    int n, j, rpb, spmv;
    const DevState* st;
    double* part;
  };
  static constexpr int kThreads = kGsThreads;
  static __device__ __forceinline__ void run(const Args& a, int block, int nblocks);
};

template <typename TM, typename TZ>
__device__ __forceinline__ void ArnProjectOp<TM, TZ>::run(const Args& a, int block, int) {
  const DevState* st = a.st;
  if (st->cycle_done) return;
  const int j = step_of(a.j, st);
  if (a.j < 0 && j >= st->m) return;     // no column beyond the cycle
  const Sell<TM> A = a.A;
  const TZ* __restrict__ z = a.z;
  double* __restrict__ W = a.W;
  const double* __restrict__ V = a.V;
  const int64_t ldv = a.ldv;
  const int n = a.n, rpb = a.rpb, spmv = a.spmv;
  double* part = a.part;
  extern __shared__ double sh[];                  // w and u_j of the block's rows
  double* wt = sh;
  double* ut = sh + rpb;
  __shared__ double red3[kGsWaves][3];
  __shared__ double piece[2][kMaxBasis + kGsWaves];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r0 = block * rpb;
  const int ns = rpb / 64;                        // slices of the block (multiple of 16)
  const double* uj = V + (size_t)j * ldv;
  double cuu = 0.0, cuw = 0.0, cww = 0.0;
  for (int sl = wave; sl < ns; sl += 2 * kGsWaves) {
    const bool two = sl + kGsWaves < ns;          // a second slice for this wavefront
    const int la = sl * 64 + lane, lb = la + kGsWaves * 64;
    const int ra = r0 + la, rb = r0 + lb;
    const bool hb = two && rb < n;
    double wa = 0.0, wb = 0.0, ua = 0.0, ub = 0.0;
    if (ra < n) {
      ua = uj[ra];
      if (hb) ub = uj[rb];
      if (spmv) {
        // A is read once per iteration, the AMG hierarchies several times:
        // its loads are non-temporal so that the hierarchies stay cached
        const TM sa = sell_dot<kProjRowChunk, true>(A, z, ra);
        const TM sb = hb ? sell_dot<kProjRowChunk, true>(A, z, rb) : (TM)0;
        wa = (double)sa;
        W[ra] = wa;
        if (hb) {
          wb = (double)sb;
          W[rb] = wb;
        }
      }
    }
    wt[la] = wa;
    ut[la] = ua;
    if (two) {
      wt[lb] = wb;
      ut[lb] = ub;
    }
    cuu += ua * ua + ub * ub;
    cuw += ua * wa + ub * wb;
    cww += wa * wa + wb * wb;
  }
  __syncthreads();
  if (j > 0) {
    // The j x ns (vector, slice) units, vector-major, are cut into kGsWaves
    // runs of equal length, one per wavefront, so every wavefront streams the
    // same share of the basis whatever j is.  A run's sums over each vector
    // it touches (a piece) go to LDS slot vector + wavefront, which no other
    // piece shares; a vector's sum adds its pieces in wavefront order.
    const int per = j * (ns / kGsWaves);
    const int u0 = wave * per, u1 = u0 + per;
    const int last = n - 1;
    for (int k = u0 / ns; k * ns < u1; ++k) {
      const int sb = max(u0 - k * ns, 0), se = min(u1 - k * ns, ns);
      const double* vk = V + (size_t)k * ldv;
      double sa = 0.0, sw = 0.0;
      for (int s = sb; s < se; s += kProjChunk) {
        double x[kProjChunk];
#pragma unroll
        for (int i = 0; i < kProjChunk; ++i) {
          const int si = min(s + i, se - 1);
          // rows past n: u, w are 0.  The basis is streamed: a
          // non-temporal load keeps it from evicting the matrices and
          // hierarchies, which the iteration re-reads, from the caches
          x[i] = __builtin_nontemporal_load(&vk[min(r0 + si * 64 + lane, last)]);
        }
#pragma unroll
        for (int i = 0; i < kProjChunk; ++i) {
          const int li = min(s + i, se - 1) * 64 + lane;
          const double ta = sa + x[i] * ut[li], tw = sw + x[i] * wt[li];
          sa = s + i < se ? ta : sa;
          sw = s + i < se ? tw : sw;
        }
      }
      sa = wave_sum(sa);
      sw = wave_sum(sw);
      if (lane == 0) {
        piece[0][k + wave] = sa;
        piece[1][k + wave] = sw;
      }
    }
    __syncthreads();
    if ((int)threadIdx.x < 2 * j) {
      const int ab = (int)threadIdx.x >= j;
      const int k = threadIdx.x - ab * j;
      const int wf = (k * ns) / per, wl = ((k + 1) * ns - 1) / per;
      double t = 0.0;
      for (int w = wf; w <= wl; ++w) t += piece[ab][k + w];
      part[(size_t)((ab ? kGsRowB : kGsRowA) + k) * kGsMaxBlocks + block] = t;
    }
  }
  cuu = wave_sum(cuu);
  cuw = wave_sum(cuw);
  cww = wave_sum(cww);
  if (lane == 0) {
    red3[wave][0] = cuu;
    red3[wave][1] = cuw;
    red3[wave][2] = cww;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kGsWaves; ++w) s += red3[w][threadIdx.x];
    part[(size_t)(kGsRowC + threadIdx.x) * kGsMaxBlocks + block] = s;
  }
}

template <typename TM, typename TZ>
__global__ __launch_bounds__(kGsThreads) __attribute__((amdgpu_waves_per_eu(8, 8))) void
k_arn_project(typename ArnProjectOp<TM, TZ>::Args a) {
  ArnProjectOp<TM, TZ>::run(a, blockIdx.x, gridDim.x);
}

// Scalar part of the update kernel: complete column jc = j - 1 (if any),
// rotate it, update g and the flags; record column j's first-pass
// coefficients and the input scale of the next preconditioner application.
__device__ void arn_column(int j, int update, const double* sums, const double* sc,
                           DevState* st, HostFlags* hf, double* hc, double* rot) {
  const int t = threadIdx.x;
  const int ld = kMaxBasis + 1;
  const int jc = j - 1;
  if (j >= 1) {
    if (t < j) hc[t] = st->h1[t] + sums[t];
    if (t < jc) {
      rot[t] = st->cs[t];
      rot[kMaxBasis + t] = st->sn[t];
    }
  }
  __syncthreads();
  if (t == 0) {
    int done = 0;
    if (j >= 1) {
      const double nu = sc[2];
      hc[j] = nu;
      for (int i = 0; i < jc; ++i) {
        const double c = rot[i], s = rot[kMaxBasis + i];
        const double x = c * hc[i] + s * hc[i + 1];
        hc[i + 1] = -s * hc[i] + c * hc[i + 1];
        hc[i] = x;
      }
      const double d = hypot(hc[jc], hc[j]);
      int bad = !(d > 0.0) || !isfinite(d) || !isfinite(nu);
      const double cj = bad ? 1.0 : hc[jc] / d;
      const double sj = bad ? 0.0 : hc[j] / d;
      st->cs[jc] = cj;
      st->sn[jc] = sj;
      hc[jc] = bad ? hc[jc] : d;
      hc[j] = 0.0;
      const double gj = st->g[jc];
      st->g[j] = -sj * gj;
      st->g[jc] = cj * gj;
      const double est = fabs(sj * gj);
      bad = bad || !isfinite(est);
      st->k = j;
      st->iters += 1;
      if (bad) st->breakdown = 1;
      done = bad || !(nu > 0.0) || est <= st->cycle_target || j >= st->m || !update;
      st->cycle_done = done;
      if (hf) {
        hf->est[j] = est;
        hf->cycle_done[j] = done;
      }
    } else if (hf) {
      hf->est[0] = st->g[0];
      hf->cycle_done[0] = 0;
    }
    if (update && !done) {
      st->h1[j] = sc[3];
      st->sigma[j + 1] = sc[4];
    }
    st->j = j + 1;
    if (hf) __threadfence_system();
  }
  __syncthreads();
  if (j >= 1 && t <= j) st->H[(size_t)jc * ld + t] = hc[t];
  if (update && t < j) st->h1[t] = sums[j + t];
}

// Row work of the update kernel: v_j = inv u_j - V (inv a), u_{j+1} =
// w - V (b - t a) - t u_j.  No dot products here, so the layout is one row
// per lane, four rows per thread (rows kGsThreads apart), the coefficients
// broadcast from LDS, and each row's sums run over the basis in ascending
// order.  The basis loads are unconditional (a row past the block reloads
// the thread's first row, and its sums are dropped), so the four rows' loads
// of four basis vectors are in flight together.
__device__ __forceinline__ void arn_rows(const double* __restrict__ W, double* __restrict__ V,
                                         int64_t ldv, int n, int j, int rpb, int block,
                                         const double* cf, double inv, double tt) {
  const int t = threadIdx.x;
  double* uj = V + (size_t)j * ldv;
  double* un = V + (size_t)(j + 1) * ldv;
  const int r0 = block * rpb;
  const int r1 = min(r0 + rpb, n);
  for (int r = r0 + t; r < r1; r += 4 * kGsThreads) {
    int rr[4];
    bool ok[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      ok[q] = r + q * kGsThreads < r1;
      rr[q] = ok[q] ? r + q * kGsThreads : r;   // rows past the block reload row r
    }
    double p1[4] = {0.0, 0.0, 0.0, 0.0}, p2[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int k = 0; k < j; ++k) {
      const double* vk = V + (size_t)k * ldv;
      // streamed basis: non-temporal, as in the projection
      double x[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) x[q] = __builtin_nontemporal_load(&vk[rr[q]]);
      const double ca = cf[k], cb = cf[kMaxBasis + k];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        p1[q] += ca * x[q];
        p2[q] += cb * x[q];
      }
    }
    // u_j and w are read for the last time and v_j is next read as part of
    // the streamed basis: all non-temporal; u_{j+1}, which the
    // preconditioner reads next, is stored normally
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (ok[q]) {
        const int rq = rr[q];
        const double u = __builtin_nontemporal_load(&uj[rq]);
        __builtin_nontemporal_store(inv * u - p1[q], &uj[rq]);
        un[rq] = __builtin_nontemporal_load(&W[rq]) - p2[q] - tt * u;
      }
    }
  }
}

// One workgroup per partial-sum row (2j + 3 rows): the sum over the
// projection workgroups, in a fixed order, into st->sums.  (A replayed
// launch has 2m + 3 workgroups; those past the step's rows return.)
struct ArnSumRowsOp {
  struct Args {
    const double* part;
    int nb, j;
    DevState* st;
  };
  static constexpr int kThreads = kBlock;
  static __device__ __forceinline__ void run(const Args& a, int block, int) {
    DevState* st = a.st;
    const int stop = gate_flag(st);
    const int j = step_of(a.j, st);
    if (a.j < 0 && (j >= st->m || block >= 2 * j + 3)) return;
    __shared__ double red[kBlock / 64];
    const int i = block;
    const int row = i < j ? kGsRowA + i : (i < 2 * j ? kGsRowB + (i - j) : kGsRowC + (i - 2 * j));
    const double* p = a.part + (size_t)row * kGsMaxBlocks;
    double s = 0.0;
    for (int b = threadIdx.x; b < a.nb; b += kBlock) s += p[b];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0 && !stop) st->sums[i] = ((red[0] + red[1]) + red[2]) + red[3];
  }
};

__global__ __launch_bounds__(kBlock) void k_arn_sum_rows(ArnSumRowsOp::Args a) {
  ArnSumRowsOp::run(a, blockIdx.x, gridDim.x);
}

// Update pass of Arnoldi step j: every workgroup derives the coefficients
// from the 2j + 3 sums (same arithmetic in each), streams its rows, and the
// last workgroup completes the Hessenberg column.  With update == 0 (closing
// step, one workgroup) only the column is completed.
struct ArnUpdateOp {
  struct Args {
    const double* W;
    double* V;
    int64_t ldv;
    int n, j, rpb, update;
    DevState* st;
    HostFlags* hf;
  };
  static constexpr int kThreads = kGsThreads;
  static __device__ __forceinline__ void run(const Args& a, int block, int nblocks) {
    __shared__ double scratch[4 * kMaxBasis];
    __shared__ double sums[kSumStride];
    __shared__ double cf[2 * kMaxBasis];
    __shared__ double sc[8];
    DevState* st = a.st;
    const int j = step_of(a.j, st);
    if (a.j < 0 && j >= st->m) return;     // no column beyond the cycle
    const int update = a.update;
    const int t = threadIdx.x;
    const int nr = 2 * j + 3;
    const int stop = st->cycle_done;
    if (t < nr) sums[t] = st->sums[t];
    __syncthreads();
    if (stop) return;
    if (t == 0) {
      double aa = 0.0, ab = 0.0, bb = 0.0;
      for (int k = 0; k < j; ++k) {
        aa += sums[k] * sums[k];
        ab += sums[k] * sums[j + k];
        bb += sums[j + k] * sums[j + k];
      }
      const double uu = sums[2 * j], uw = sums[2 * j + 1], ww = sums[2 * j + 2];
      const double nu2 = uu - aa;
      const double nu = nu2 > 0.0 ? sqrt(nu2) : 0.0;
      const double inv = nu > 0.0 ? 1.0 / nu : 0.0;
      const double hjj = (uw - ab) * inv;
      const double rest = ww - bb - hjj * hjj;
      const double floor = 1e-16 * ww;
      sc[0] = inv;
      sc[1] = hjj * inv;
      sc[2] = nu;
      sc[3] = hjj;
      sc[4] = ww > 0.0 ? 1.0 / sqrt(rest > floor ? rest : floor) : 1.0;
    }
    __syncthreads();
    if (update) {
      if (t < j) {
        cf[t] = sc[0] * sums[t];
        cf[kMaxBasis + t] = sums[j + t] - sc[1] * sums[t];
      }
      __syncthreads();
      arn_rows(a.W, a.V, a.ldv, a.n, j, a.rpb, block, cf, sc[0], sc[1]);
    }
    if (block == nblocks - 1) {
      __syncthreads();
      arn_column(j, update, sums, sc, st, a.hf, scratch, scratch + 2 * kMaxBasis);
    }
  }
};

__global__ __launch_bounds__(kGsThreads) void k_arn_update(ArnUpdateOp::Args a) {
  ArnUpdateOp::run(a, blockIdx.x, gridDim.x);
}

// Copy-in and copy-out of a column of the request loop's shared graph: the
// graph is replayed for every column, so the preconditioner works on fixed
// per-solve buffers.  Copy-in records the step j = st->j in st->jstep (read by
// the later kernels of the column) and copies u_j = V[j] and sigma_j into
// them; copy-out stores the preconditioned vector into Z[j].  Neither runs
// once the cycle is done or past its last column.
struct CopyInOp {
  struct Args {
    const double* V;
    int64_t ldv;
    DevState* st;
    double* rin;
    double* sig;
    int n;
  };
  static constexpr int kThreads = kBlock;
  static __device__ __forceinline__ void run(const Args& a, int block, int) {
    DevState* st = a.st;
    if (st->cycle_done) return;
    const int j = st->j;
    const int i = block * kBlock + threadIdx.x;
    if (i == 0) {
      st->jstep = j;
      if (j < st->m) *a.sig = st->sigma[j];
    }
    if (j >= st->m || i >= a.n) return;
    a.rin[i] = a.V[(size_t)j * a.ldv + i];
  }
};

template <typename T>
struct CopyOutOp {
  struct Args {
    const T* zfix;
    T* Z;
    int64_t ldz;
    const DevState* st;
    int n;
  };
  static constexpr int kThreads = kBlock;
  static __device__ __forceinline__ void run(const Args& a, int block, int) {
    const DevState* st = a.st;
    if (st->cycle_done) return;
    const int j = st->jstep;
    const int i = block * kBlock + threadIdx.x;
    if (j >= st->m || i >= a.n) return;
    a.Z[(size_t)j * a.ldz + i] = a.zfix[i];
  }
};

__global__ __launch_bounds__(kBlock) void k_copy_in(CopyInOp::Args a) {
  CopyInOp::run(a, blockIdx.x, gridDim.x);
}
template <typename T>
__global__ __launch_bounds__(kBlock) void k_copy_out(typename CopyOutOp<T>::Args a) {
  CopyOutOp<T>::run(a, blockIdx.x, gridDim.x);
}

// Batched launch of an Op over the slots of the request loop's shared graph.
// The slot table is one device array of `stride` bytes per slot; slot s
// holds this Op's argument struct at base + s * stride + args_off and its
// workgroup count at base + s * stride + nb_off (0: an empty slot).
// Workgroup g serves slot g / cap as its local workgroup g % cap.
template <typename Op>
__device__ __forceinline__ void batch_slot(const char* __restrict__ base, int stride,
                                           int args_off, int nb_off, int cap) {
  const int slot = blockIdx.x / cap;
  const int lb = blockIdx.x - slot * cap;
  const char* reg = base + (size_t)slot * stride;
  const int nb = *reinterpret_cast<const int*>(reg + nb_off);
  if (lb >= nb) return;
  Op::run(*reinterpret_cast<const typename Op::Args*>(reg + args_off), lb, nb);
}

template <typename Op>
__global__ __launch_bounds__(Op::kThreads) void k_batch(const char* __restrict__ base, int stride,
                                                        int args_off, int nb_off, int cap) {
  batch_slot<Op>(base, stride, args_off, nb_off, cap);
}

// The projection keeps its occupancy hint in the batched form too.
template <typename TM, typename TZ>
__global__ __launch_bounds__(kGsThreads) __attribute__((amdgpu_waves_per_eu(8, 8))) void
k_batch_project(const char* __restrict__ base, int stride, int args_off, int nb_off, int cap) {
  batch_slot<ArnProjectOp<TM, TZ>>(base, stride, args_off, nb_off, cap);
}

// y = R^-1 g for the k x k upper triangle R of H (one wavefront): the
// triangle is staged in LDS, then column-oriented back substitution.
__global__ __launch_bounds__(64) void k_trisolve(DevState* st) {
  __shared__ double Rs[kMaxBasis][kMaxBasis];     // Rs[l][i] = R(i, l)
  __shared__ double sv[kMaxBasis];
  const int k = st->k;
  const int t = threadIdx.x;
  const int ld = kMaxBasis + 1;
  for (int l = 0; l < k; ++l)
    if (t <= l) Rs[l][t] = st->H[(size_t)l * ld + t];
  if (t < k) sv[t] = st->g[t];
  __syncthreads();
  for (int i = k - 1; i >= 0; --i) {
    const double yi = sv[i] / Rs[i][i];
    __syncthreads();
    if (t < i) sv[t] -= Rs[i][t] * yi;
    if (t == 0) st->y[i] = yi;
    __syncthreads();
  }
}

template <typename TZ>
__global__ __launch_bounds__(kBlock) void k_update_x(double* __restrict__ x,
                                                     const TZ* __restrict__ Z, int64_t ldz,
                                                     int n, const DevState* st) {
  const int row = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (row >= n) return;
  const int k = st->k;
  double s = x[row];
  for (int l = 0; l < k; ++l) s += st->y[l] * (double)Z[(size_t)l * ldz + row];
  x[row] = s;
}

__global__ __launch_bounds__(kBlock) void k_restart_residual(Sell<double> A,
                                                             const double* __restrict__ b,
                                                             const double* __restrict__ x,
                                                             double* __restrict__ r, int off_p,
                                                             int off_q, int R, double* part) {
  const int n = A.n_rows;
  const int G = gridDim.x * kBlock;
  const int gtid = blockIdx.x * kBlock + threadIdx.x;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int t = 0; t < R; ++t) {
    const int row = gtid + t * G;
    if (row < n) {
      const double rv = b[row] - (x ? sell_dot(A, x, row) : 0.0);
      r[row] = rv;
      const int blk = row < off_p ? 0 : (row < off_q ? 1 : 2);
      acc[blk] += rv * rv;
    }
  }
  block_partials<3>(acc, 3, part);
}

__global__ __launch_bounds__(kBlock) void k_restart_finish(const double* part, int nb,
                                                           DevState* st, HostFlags* hf) {
  __shared__ double sums[3];
  final_sums<3>(part, nb, 3, sums);
  if (threadIdx.x != 0) return;
  for (int k = 0; k < 3; ++k) st->resblk[k] = sums[k];
  const double beta = sqrt((sums[0] + sums[1]) + sums[2]);
  st->beta = beta;
  st->sigma[0] = 1.0 / beta;
  st->g[0] = beta;
  st->j = 0;
  st->k = 0;
  const int fin = isfinite(beta);
  const int conv = fin && beta <= st->target;
  st->converged = conv;
  if (!fin) st->breakdown = 1;
  st->cycle_done = conv || !fin || !(beta > 0.0);
  const double ct = st->cycle_drop * beta;
  st->cycle_target = ct > st->target ? ct : st->target;
  if (hf) {
    hf->est[kMaxBasis + 1] = beta;
    __threadfence_system();
  }
}

// norms = (||r||, ||r_v||, ||r_p||, ||r_q||) from the block partials of
// k_restart_residual, summed in a fixed order.
__global__ __launch_bounds__(kBlock) void k_residual_norms(const double* part, int nb,
                                                           double* norms) {
  __shared__ double sums[3];
  final_sums<3>(part, nb, 3, sums);
  if (threadIdx.x != 0) return;
  norms[0] = sqrt((sums[0] + sums[1]) + sums[2]);
  for (int k = 0; k < 3; ++k) norms[k + 1] = sqrt(sums[k]);
}

__global__ __launch_bounds__(kBlock) void k_norm_b(const double* __restrict__ b, int n, int R,
                                                   double* part) {
  const int G = gridDim.x * kBlock;
  const int gtid = blockIdx.x * kBlock + threadIdx.x;
  double acc[1] = {0.0};
  for (int t = 0; t < R; ++t) {
    const int row = gtid + t * G;
    if (row < n) acc[0] += b[row] * b[row];
  }
  block_partials<1>(acc, 1, part);
}

__global__ __launch_bounds__(kBlock) void k_norm_b_finish(const double* part, int nb, double tol,
                                                          DevState* st) {
  __shared__ double sums[1];
  final_sums<1>(part, nb, 1, sums);
  if (threadIdx.x == 0) {
    st->bnorm = sqrt(sums[0]);
    st->target = tol * st->bnorm;
  }
}

// ---- BiCGSTAB (right preconditioned, van der Vorst).  Vectors FP64; the
// preconditioned vectors y, z are in the preconditioner precision T.  Scalars
// live in DevState (rho, alpha, omega, bbeta); dots[] hold finished sums.
// Every kernel returns at once when st->cycle_done is set (converged,
// breakdown, or iteration cap), so enqueued iterations beyond that point
// leave x untouched.

// p = r + beta (p - omega v)
__global__ __launch_bounds__(kBlock) void k_bicg_p(int n, const double* __restrict__ r,
                                                   double* __restrict__ p,
                                                   const double* __restrict__ v,
                                                   const DevState* st) {
  if (st->cycle_done) return;
  const int i = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (i >= n) return;
  p[i] = r[i] + st->bbeta * (p[i] - st->omega * v[i]);
}

// out = A y (FP64 matrix, y in TY); partial dots: out.u1 (and out.out if two)
template <typename TY>
__global__ __launch_bounds__(kBlock) void k_bicg_spmv(Sell<double> A, const TY* __restrict__ y,
                                                      double* __restrict__ out,
                                                      const double* __restrict__ u1, int two,
                                                      int R, const DevState* st, double* part) {
  if (st->cycle_done) return;
  const int n = A.n_rows;
  const int G = gridDim.x * kBlock;
  const int gtid = blockIdx.x * kBlock + threadIdx.x;
  double acc[2] = {0.0, 0.0};
  for (int t = 0; t < R; ++t) {
    const int row = gtid + t * G;
    if (row < n) {
      const double w = sell_dot(A, y, row);
      out[row] = w;
      acc[0] += w * u1[row];
      acc[1] += w * w;
    }
  }
  block_partials<2>(acc, two ? 2 : 1, part);
}

// s = r - alpha v ; x += alpha y ; partial s.s
template <typename TY>
__global__ __launch_bounds__(kBlock) void k_bicg_s(int n, const double* __restrict__ r,
                                                   const double* __restrict__ v,
                                                   double* __restrict__ s,
                                                   double* __restrict__ x,
                                                   const TY* __restrict__ y, int R,
                                                   const DevState* st, double* part) {
  if (st->cycle_done) return;
  const int G = gridDim.x * kBlock;
  const int gtid = blockIdx.x * kBlock + threadIdx.x;
  const double al = st->alpha;
  double acc[1] = {0.0};
  for (int t = 0; t < R; ++t) {
    const int i = gtid + t * G;
    if (i < n) {
      const double si = r[i] - al * v[i];
      s[i] = si;
      x[i] += al * (double)y[i];
      acc[0] += si * si;
    }
  }
  block_partials<1>(acc, 1, part);
}

// x += omega z ; r = s - omega t ; partial r.r and rhat.r
template <typename TY>
__global__ __launch_bounds__(kBlock) void k_bicg_r(int n, const double* __restrict__ s,
                                                   const double* __restrict__ t,
                                                   double* __restrict__ r,
                                                   double* __restrict__ x,
                                                   const TY* __restrict__ z,
                                                   const double* __restrict__ rhat, int R,
                                                   const DevState* st, double* part) {
  if (st->cycle_done) return;
  const int G = gridDim.x * kBlock;
  const int gtid = blockIdx.x * kBlock + threadIdx.x;
  const double om = st->omega;
  double acc[2] = {0.0, 0.0};
  for (int q = 0; q < R; ++q) {
    const int i = gtid + q * G;
    if (i < n) {
      x[i] += om * (double)z[i];
      const double ri = s[i] - om * t[i];
      r[i] = ri;
      acc[0] += ri * ri;
      acc[1] += rhat[i] * ri;
    }
  }
  block_partials<2>(acc, 2, part);
}

// One-workgroup scalar steps.  op 0: alpha = rho / (rhat.v);
// op 1: ||s|| test; op 2: omega = (t.s)/(t.t); op 3: ||r|| test, next rho
// and beta; op 4: restart values (rho = r.r, bbeta = 0, omega = alpha = 1).
__global__ __launch_bounds__(kBlock) void k_bicg_scalar(const double* part, int nb, int op,
                                                        DevState* st, HostFlags* hf, int slot) {
  if (op != 4 && st->cycle_done) return;
  __shared__ double sums[2];
  const int nv = (op == 0 || op == 1 || op == 4) ? 1 : 2;
  final_sums<2>(part, nb, nv, sums);
  if (threadIdx.x != 0) return;
  int done = 0, bad = 0;
  if (op == 0) {
    const double den = sums[0];
    const double al = st->rho / den;
    bad = !(den != 0.0) || !isfinite(al);
    st->alpha = al;
  } else if (op == 1) {
    const double sn = sqrt(sums[0]);
    st->dots[0] = sn;
    done = sn <= st->target;
    st->converged = done;
    bad = !isfinite(sn);
  } else if (op == 2) {
    const double tt = sums[1];
    const double om = sums[0] / tt;
    bad = !(tt > 0.0) || !isfinite(om) || om == 0.0;
    st->omega = om;
  } else if (op == 3) {
    const double rn = sqrt(sums[0]);
    const double rho_new = sums[1];
    st->dots[1] = rn;
    st->iters += 1;
    done = rn <= st->target;
    st->converged = done;
    st->bbeta = (rho_new / st->rho) * (st->alpha / st->omega);
    bad = !isfinite(rn) || !(rho_new != 0.0) || !isfinite(st->bbeta);
    st->rho = rho_new;
    if (!done && st->iters >= st->m) done = 1;   // iteration cap of this cycle
  } else {
    const double rr = sums[0];
    st->rho = rr;
    st->bbeta = 0.0;
    st->alpha = 1.0;
    st->omega = 1.0;
    st->beta = sqrt(rr);
    st->converged = st->beta <= st->target;
    st->cycle_done = st->converged || !isfinite(st->beta) || !(st->beta > 0.0);
    if (!isfinite(st->beta)) st->breakdown = 1;
    return;
  }
  if (op == 1 && done) st->iters += 1;   // converged halfway through an iteration
  if (bad) st->breakdown = 1;
  if (done || bad) st->cycle_done = 1;
  if (hf && (op == 1 || op == 3)) {
    hf->cycle_done[slot] = st->cycle_done;
    __threadfence_system();
  }
}

// r = b - A x (x may be null: zero), rhat = r, p = v = 0; partial r.r
__global__ __launch_bounds__(kBlock) void k_bicg_restart(Sell<double> A,
                                                         const double* __restrict__ b,
                                                         const double* __restrict__ x,
                                                         double* __restrict__ r,
                                                         double* __restrict__ rhat,
                                                         double* __restrict__ p,
                                                         double* __restrict__ v, int R,
                                                         double* part) {
  const int n = A.n_rows;
  const int G = gridDim.x * kBlock;
  const int gtid = blockIdx.x * kBlock + threadIdx.x;
  double acc[2] = {0.0, 0.0};
  for (int t = 0; t < R; ++t) {
    const int row = gtid + t * G;
    if (row < n) {
      const double rv = b[row] - (x ? sell_dot(A, x, row) : 0.0);
      r[row] = rv;
      rhat[row] = rv;
      p[row] = 0.0;
      v[row] = 0.0;
      acc[0] += rv * rv;
    }
  }
  block_partials<2>(acc, 1, part);
}

__global__ void k_init_state(DevState* st, int m, double drop) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  st->j = 0;
  st->k = 0;
  st->cycle_done = 0;
  st->m = m;
  st->converged = 0;
  st->breakdown = 0;
  st->iters = 0;
  st->cycle_drop = drop;
}

__global__ void k_set_cycle_length(DevState* st, int m) {
  if (threadIdx.x == 0 && blockIdx.x == 0) st->m = m;
}

// Right-hand side of one backward-Euler step: out = b + m x on the rows whose
// momentum balance has a time derivative (u faces i = 1..nx-1: rows
// r < off_v with 1 <= r % nux + ifirst <= nx - 1; v faces off the interface: rows
// off_v + v_skip .. off_w - 1, v_skip = the interface faces; every w face:
// rows off_w .. off_p - 1), b on the others.  One rounded product and one
// rounded sum per row, never fused, so the result is reproducible bit for
// bit.  out may alias b or x (each thread reads its row before writing it).
__global__ __launch_bounds__(kBlock) void k_step_rhs(const double* b, const double* x,
                                                     double* out, double m, int n, int nux,
                                                     int ifirst, int nx, int off_v, int v_skip,
                                                     int off_w, int off_p) {
#pragma clang fp contract(off)
  const int r = blockIdx.x * kBlock + threadIdx.x;
  if (r >= n) return;
  const int iu = r % nux + ifirst;   // face index of a u row
  const bool has = r < off_v   ? (iu >= 1 && iu <= nx - 1)
                   : r < off_w ? r >= off_v + v_skip
                               : r < off_p;
  const double br = b[r];
  if (has) {
    const double mx = m * x[r];
    out[r] = br + mx;
  } else {
    out[r] = br;
  }
}

}  // namespace

// ---------------------------------------------------------------- launchers

[[noreturn]] void throw_launch(const char* what);

// workgroups for n rows in SELL-C slices of 64 / lpr rows, one wavefront each
inline int blocks_lpr(int n, int lpr) {
  const int64_t c = 64 / lpr, waves = ((int64_t)n + c - 1) / c;
  return (int)((waves * 64 + kBlock - 1) / kBlock);
}

// Launches go through launch_op: normally a launch of the Op's named
// kernel; while a recorder is installed on the calling thread (the request
// loop building its shared graph) the launch is recorded instead, with the
// Op's batched kernel, its arguments and its workgroup count.
thread_local std::vector<RecordedOp>* g_recorder = nullptr;

void set_launch_recorder(std::vector<RecordedOp>* rec) { g_recorder = rec; }
bool launch_recording() { return g_recorder != nullptr; }

template <typename Op, typename K, typename B>
void launch_op(K kernel, B batched, const typename Op::Args& a, int nb, size_t lds,
               hipStream_t s, double bytes = 0.0) {
  if (nb <= 0) return;
  if (g_recorder) {
    RecordedOp r;
    r.fn = reinterpret_cast<const void*>(batched);
    r.args.assign(reinterpret_cast<const char*>(&a), reinterpret_cast<const char*>(&a) + sizeof(a));
    r.nblocks = nb;
    r.threads = Op::kThreads;
    r.lds = lds;
    r.bytes = bytes;
    g_recorder->push_back(std::move(r));
    return;
  }
  kernel<<<nb, Op::kThreads, lds, s>>>(a);
}

// Algorithmic bytes of a sparse matrix pass: each stored value once, and
// each column index or stencil offset the pass reads once.
template <typename T>
double mat_bytes(const Sell<T>& A) {
  return (double)A.nnz * (double)sizeof(T) + (double)A.idx * (double)sizeof(int);
}

// Calls f with the lanes-per-row count as a compile-time constant.
template <typename F>
void by_lpr(int lpr, F&& f) {
  switch (lpr) {
    case 4: f(std::integral_constant<int, 4>{}); break;
    case 8: f(std::integral_constant<int, 8>{}); break;
    case 16: f(std::integral_constant<int, 16>{}); break;
    case 32: f(std::integral_constant<int, 32>{}); break;
    case 64: f(std::integral_constant<int, 64>{}); break;
    default: f(std::integral_constant<int, 1>{}); break;
  }
}

template <typename TM, typename TX, typename TY>
void launch_spmv(const Sell<TM>& A, const TX* x, TY* y, const DevState* gate, hipStream_t s) {
  if (A.n_rows <= 0) return;
  by_lpr(A.lpr, [&](auto L) {
    constexpr int l = decltype(L)::value;
    using Op = SpmvOp<l, TM, TX, TY>;
    launch_op<Op>(k_spmv<l, TM, TX, TY>, k_batch<Op>, typename Op::Args{A, x, y, gate},
                  blocks_lpr(A.n_rows, l), 0, s,
                  mat_bytes(A) + (double)A.n_cols * sizeof(TX) + (double)A.n_rows * sizeof(TY));
  });
}

template <typename T, typename TB>
void launch_residual(const Sell<T>& A, const TB* b, const double* bscale, const T* x, T* r,
                     const DevState* gate, hipStream_t s) {
  if (A.n_rows <= 0) return;
  by_lpr(A.lpr, [&](auto L) {
    constexpr int l = decltype(L)::value;
    using Op = ResidualOp<l, T, TB>;
    launch_op<Op>(k_residual<l, T, TB>, k_batch<Op>, typename Op::Args{A, b, bscale, x, r, gate},
                  blocks_lpr(A.n_rows, l), 0, s,
                  mat_bytes(A) + (double)A.n_rows * (sizeof(TB) + 2 * sizeof(T)));
  });
}

template <typename T, typename TB>
void launch_jacobi_zero(const Sell<T>& A, const T* wd, const TB* b, const double* bscale, T* x,
                        int two, const DevState* gate, hipStream_t s) {
  if (A.n_rows <= 0) return;
  by_lpr(A.lpr, [&](auto L) {
    constexpr int l = decltype(L)::value;
    using Op = JacobiZeroOp<l, T, TB>;
    launch_op<Op>(k_jacobi_zero<l, T, TB>, k_batch<Op>,
                  typename Op::Args{A, wd, b, bscale, x, two, gate}, blocks_lpr(A.n_rows, l), 0,
                  s, (two ? mat_bytes(A) : 0.0) + (double)A.n_rows * (sizeof(TB) + 2 * sizeof(T)));
  });
}

template <typename T, typename TB>
void launch_jacobi(const Sell<T>& A, const T* wd, const TB* b, const double* bscale,
                   const T* x_in, T* x_out, const DevState* gate, hipStream_t s) {
  if (A.n_rows <= 0) return;
  by_lpr(A.lpr, [&](auto L) {
    constexpr int l = decltype(L)::value;
    using Op = JacobiOp<l, T, TB>;
    launch_op<Op>(k_jacobi<l, T, TB>, k_batch<Op>,
                  typename Op::Args{A, wd, b, bscale, x_in, x_out, gate},
                  blocks_lpr(A.n_rows, l), 0, s,
                  mat_bytes(A) + (double)A.n_rows * (sizeof(TB) + 3 * sizeof(T)));
  });
}

template <typename T, typename TB>
void launch_restrict_residual(const Sell<T>& Q, const TB* b, const double* bscale, const T* x,
                              int n_fine, T* bc, const DevState* gate, hipStream_t s) {
  if (Q.n_rows <= 0) return;
  by_lpr(Q.lpr, [&](auto L) {
    constexpr int l = decltype(L)::value;
    using Op = RestrictResidualOp<l, T, TB>;
    launch_op<Op>(k_restrict_residual<l, T, TB>, k_batch<Op>,
                  typename Op::Args{Q, b, bscale, x, n_fine, bc, gate}, blocks_lpr(Q.n_rows, l),
                  0, s,
                  mat_bytes(Q) + (double)n_fine * (sizeof(TB) + sizeof(T)) +
                      (double)Q.n_rows * sizeof(T));
  });
}

template <typename T, typename TB>
void launch_presmooth_restrict(const Sell<T>& A, const T* wd, const Sell<T>& G, const TB* b,
                               const double* bscale, T* x, T* bc, const DevState* gate,
                               hipStream_t s) {
  if (A.n_rows <= 0) return;
  if (G.lpr != 64) throw_launch("presmooth_restrict: G must use 64 lanes per row");
  const int nb_a = blocks_lpr(A.n_rows, A.lpr);
  const int nb = nb_a + blocks_lpr(G.n_rows, 64);
  by_lpr(A.lpr, [&](auto L) {
    constexpr int l = decltype(L)::value;
    using Op = PresmoothRestrictOp<l, T, TB>;
    launch_op<Op>(k_presmooth_restrict<l, T, TB>, k_batch<Op>,
                  typename Op::Args{A, wd, G, b, bscale, x, bc, nb_a, gate}, nb, 0, s,
                  mat_bytes(A) + mat_bytes(G) + (double)A.n_rows * (sizeof(TB) + 2 * sizeof(T)) +
                      (double)G.n_rows * sizeof(T));
  });
}

template <typename T, typename TB>
void launch_prolong_smooth(const Sell<T>& A, const Sell<T>& F, const T* wd, const TB* b,
                           const double* bscale, const T* x, const T* xc, T* xout,
                           const DevState* gate, hipStream_t s) {
  if (A.n_rows <= 0) return;
  if (F.lpr != A.lpr) throw_launch("prolong_smooth: F must use A's lanes per row");
  by_lpr(A.lpr, [&](auto L) {
    constexpr int l = decltype(L)::value;
    using Op = ProlongSmoothOp<l, T, TB>;
    launch_op<Op>(k_prolong_smooth<l, T, TB>, k_batch<Op>,
                  typename Op::Args{A, F, wd, b, bscale, x, xc, xout, gate},
                  blocks_lpr(A.n_rows, l), 0, s,
                  mat_bytes(A) + mat_bytes(F) + (double)A.n_rows * (sizeof(TB) + 3 * sizeof(T)) +
                      (double)F.n_cols * sizeof(T));
  });
}

template <typename T>
void launch_prolong(const Sell<T>& P, const T* xc, T* x, const DevState* gate, hipStream_t s) {
  if (P.n_rows <= 0) return;
  by_lpr(P.lpr, [&](auto L) {
    constexpr int l = decltype(L)::value;
    using Op = ProlongOp<l, T>;
    launch_op<Op>(k_prolong<l, T>, k_batch<Op>, typename Op::Args{P, xc, x, gate},
                  blocks_lpr(P.n_rows, l), 0, s,
                  mat_bytes(P) + (double)P.n_cols * sizeof(T) + 2.0 * P.n_rows * sizeof(T));
  });
}

template <typename T>
void launch_ilu0(const IluDev<T>& F, const T* r, T* z, const DevState* gate, hipStream_t s) {
  if (F.n <= 0) return;
  using Op = Ilu0Op<T>;
  const double n = (double)F.n;
  launch_op<Op>(k_ilu0<T>, k_batch<Op>, typename Op::Args{F, r, z, gate}, 1, 0, s,
                n * (4 + 2 * kIluWidth * (4 + sizeof(T)) + sizeof(T)) + 3 * n * sizeof(T));
}

template <typename T>
void launch_coarse(const double* Ainv, int n, const T* bc, T* xc, const DevState* gate,
                   hipStream_t s) {
  if (n <= 0) return;
  using Op = CoarseOp<T>;
  launch_op<Op>(k_coarse<T>, k_batch<Op>, typename Op::Args{Ainv, n, bc, xc, gate}, n, 0, s,
                8.0 * n * n + 2.0 * n * sizeof(T));
}

template <typename T>
void launch_block_sweep(const Sell<T>& Cf, int n_p, const double* r, const double* bscale,
                        const T* yv, double xscale, T* zp, T* tq, T* tp, const DevState* gate,
                        hipStream_t s) {
  if (Cf.n_rows <= 0) return;
  using Op = BlockSweepOp<T>;
  launch_op<Op>(k_block_sweep<T>, k_batch<Op>,
                typename Op::Args{Cf, n_p, r, bscale, yv, xscale, zp, tq, tp, gate},
                blocks_for(Cf.n_rows), 0, s,
                mat_bytes(Cf) + (double)Cf.n_rows * (8 + sizeof(T)) + (double)Cf.n_cols * sizeof(T) +
                    (tp ? (double)n_p * sizeof(T) : 0.0));
}

template <typename T>
void launch_add(const T* a, T* y, int n, const DevState* gate, hipStream_t s) {
  if (n <= 0) return;
  using Op = AddOp<T>;
  launch_op<Op>(k_add<T>, k_batch<Op>, typename Op::Args{a, y, n, gate}, blocks_for(n), 0, s,
                3.0 * n * sizeof(T));
}

// Rows per workgroup: the projection kernel takes 1024 (two workgroups per
// CU overlap one's latency-bound product phase with the other's streaming),
// the update kernel 2048; both double while a launch would have more than
// 1024 workgroups, up to kGsMaxRowsPerBlock rows (64 KiB of LDS in the
// projection), and beyond that the grid grows, up to kGsMaxBlocks workgroups
// (the partial-sum capacity) at kMaxUnknowns rows.
int gs_rows_per_block(int n, int base) {
  int rpb = base;
  while ((n + rpb - 1) / rpb > 1024 && rpb < kGsMaxRowsPerBlock) rpb *= 2;
  return rpb;
}
constexpr int kUpdateRows = 2048;

template <typename TM, typename TZ>
void launch_arnoldi_step(const Sell<TM>& A, const TZ* z, double* W, double* V, int64_t ldv, int j,
                         DevState* st, double* part, HostFlags* hf, hipStream_t s, int prof_class,
                         hipEvent_t* ev) {
  const int n = A.n_rows;
  const int rp = gs_rows_per_block(n, kGsProjectRows), ru = gs_rows_per_block(n, kUpdateRows);
  const int np = (n + rp - 1) / rp, nu = (n + ru - 1) / ru;
  // j < 0: the step comes from st->jstep; the sums then get a workgroup per
  // row of the largest step the basis holds
  const int nsum = j >= 0 ? 2 * j + 3 : 2 * (kMaxBasis - 1) + 3;
  using POp = ArnProjectOp<TM, TZ>;
  if (ev && prof_class == 1) (void)hipEventRecord(ev[0], s);
  launch_op<POp>(k_arn_project<TM, TZ>, k_batch_project<TM, TZ>,
                 typename POp::Args{A, z, W, V, ldv, n, j, rp, 1, st, part}, np,
                 (size_t)2 * rp * sizeof(double), s);
  if (ev && prof_class == 1) (void)hipEventRecord(ev[1], s);
  launch_op<ArnSumRowsOp>(k_arn_sum_rows, k_batch<ArnSumRowsOp>,
                          ArnSumRowsOp::Args{part, np, j, st}, nsum, 0, s);
  if (ev && prof_class == 2) (void)hipEventRecord(ev[0], s);
  launch_op<ArnUpdateOp>(k_arn_update, k_batch<ArnUpdateOp>,
                         ArnUpdateOp::Args{W, V, ldv, n, j, ru, 1, st, hf}, nu, 0, s);
  if (ev && prof_class == 2) (void)hipEventRecord(ev[1], s);
}

void launch_arnoldi_close(int n, double* V, int64_t ldv, int j, DevState* st, double* part,
                          HostFlags* hf, hipStream_t s) {
  const int rp = gs_rows_per_block(n, kGsProjectRows);
  const int np = (n + rp - 1) / rp;
  using POp = ArnProjectOp<double, double>;
  k_arn_project<double, double><<<np, kGsThreads, (size_t)2 * rp * sizeof(double), s>>>(
      POp::Args{Sell<double>{}, nullptr, nullptr, V, ldv, n, j, rp, 0, st, part});
  k_arn_sum_rows<<<2 * j + 3, kBlock, 0, s>>>(ArnSumRowsOp::Args{part, np, j, st});
  k_arn_update<<<1, kGsThreads, 0, s>>>(
      ArnUpdateOp::Args{nullptr, V, ldv, n, j, kUpdateRows, 0, st, hf});
}

void launch_copy_in(const double* V, int64_t ldv, DevState* st, double* rin, double* sig, int n,
                    hipStream_t s) {
  launch_op<CopyInOp>(k_copy_in, k_batch<CopyInOp>,
                      CopyInOp::Args{V, ldv, st, rin, sig, n}, blocks_for(n), 0, s);
}

template <typename T>
void launch_copy_out(const T* zfix, T* Z, int64_t ldz, const DevState* st, int n, hipStream_t s) {
  launch_op<CopyOutOp<T>>(k_copy_out<T>, k_batch<CopyOutOp<T>>,
                          typename CopyOutOp<T>::Args{zfix, Z, ldz, st, n}, blocks_for(n), 0, s);
}

void launch_trisolve(DevState* st, hipStream_t s) { k_trisolve<<<1, 64, 0, s>>>(st); }

template <typename TZ>
void launch_update_x(double* x, const TZ* Z, int64_t ldz, int n, DevState* st, hipStream_t s) {
  if (n <= 0) return;
  k_update_x<TZ><<<blocks_for(n), kBlock, 0, s>>>(x, Z, ldz, n, st);
}

void launch_restart_residual(const Sell<double>& A, const double* b, const double* x, double* r,
                             const int64_t* blk_off, DevState* st, double* part, HostFlags* hf,
                             hipStream_t s) {
  const int n = A.n_rows;
  const int nb = dot_blocks(n);
  const int R = (n + nb * kBlock - 1) / (nb * kBlock);
  k_restart_residual<<<nb, kBlock, 0, s>>>(A, b, x, r, (int)blk_off[2], (int)blk_off[3], R, part);
  k_restart_finish<<<1, kBlock, 0, s>>>(part, nb, st, hf);
}

void launch_residual_norms(const Sell<double>& A, const double* b, const double* x, double* r,
                           const int64_t* blk_off, double* part, double* norms, hipStream_t s) {
  const int n = A.n_rows;
  const int nb = dot_blocks(n);
  const int R = (n + nb * kBlock - 1) / (nb * kBlock);
  k_restart_residual<<<nb, kBlock, 0, s>>>(A, b, x, r, (int)blk_off[2], (int)blk_off[3], R, part);
  k_residual_norms<<<1, kBlock, 0, s>>>(part, nb, norms);
}
namespace {
constexpr int kScratchMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch[kScratchMaxDevices] = {};
}  // namespace

// Address of the current device's copy of `scratch`, looked up on the first
// call on each device.
static double* noalloc_scratch() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    throw Error(SD_E_DEVICE, "hipGetDevice failed");
  }
  if (dev < 0 || dev >= kScratchMaxDevices)
    throw Error(SD_E_DEVICE, "device ordinal beyond the scratch table (64 devices)");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      throw Error(SD_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                   hipGetErrorString(e));
    }
    g_scratch[dev] = static_cast<double*>(p);
  }
  return g_scratch[dev];
}

void launch_residual_norms_noalloc(const Sell<double>& A, const double* b, const double* x,
                                   double* r, const int64_t* blk_off, double* norms,
                                   hipStream_t s) {
  if ((int64_t)A.n_rows > kMaxUnknowns)
    throw Error(SD_E_INVALID, "more unknowns than the allocation-free residual takes (" +
                                  std::to_string(kMaxUnknowns) + ")");
  if (dot_blocks(A.n_rows) * 3 > (int)(sizeof(scratch) / sizeof(double)))
    throw Error(SD_E_INVALID, "residual partials exceed the static scratch");
  launch_residual_norms(A, b, x, r, blk_off, noalloc_scratch(), norms, s);
}

void launch_norm_b(const double* b, int n, double tol, DevState* st, double* part,
                   hipStream_t s) {
  const int nb = dot_blocks(n);
  const int R = (n + nb * kBlock - 1) / (nb * kBlock);
  k_norm_b<<<nb, kBlock, 0, s>>>(b, n, R, part);
  k_norm_b_finish<<<1, kBlock, 0, s>>>(part, nb, tol, st);
}

template <typename T>
void launch_bicg_iteration_part(int which, const Sell<double>& A, BicgVecs<T>& w, double* x,
                                DevState* st, double* part, HostFlags* hf, int slot,
                                hipStream_t s) {
  const int n = A.n_rows;
  const int nb = dot_blocks(n);
  const int R = (n + nb * kBlock - 1) / (nb * kBlock);
  switch (which) {
    case 0:  // p update (before M p)
      k_bicg_p<<<blocks_for(n), kBlock, 0, s>>>(n, w.r, w.p, w.v, st);
      break;
    case 1:  // v = A y, alpha, s, ||s||
      k_bicg_spmv<T><<<nb, kBlock, 0, s>>>(A, w.y, w.v, w.rhat, 0, R, st, part);
      k_bicg_scalar<<<1, kBlock, 0, s>>>(part, nb, 0, st, hf, slot);
      k_bicg_s<T><<<nb, kBlock, 0, s>>>(n, w.r, w.v, w.s, x, w.y, R, st, part);
      k_bicg_scalar<<<1, kBlock, 0, s>>>(part, nb, 1, st, hf, slot);
      break;
    default:  // t = A z, omega, x, r, ||r||, next rho
      k_bicg_spmv<T><<<nb, kBlock, 0, s>>>(A, w.z, w.t, w.s, 1, R, st, part);
      k_bicg_scalar<<<1, kBlock, 0, s>>>(part, nb, 2, st, hf, slot);
      k_bicg_r<T><<<nb, kBlock, 0, s>>>(n, w.s, w.t, w.r, x, w.z, w.rhat, R, st, part);
      k_bicg_scalar<<<1, kBlock, 0, s>>>(part, nb, 3, st, hf, slot);
      break;
  }
}

void launch_bicg_restart(const Sell<double>& A, const double* b, const double* x, double* r,
                         double* rhat, double* p, double* v, DevState* st, double* part,
                         hipStream_t s) {
  const int n = A.n_rows;
  const int nb = dot_blocks(n);
  const int R = (n + nb * kBlock - 1) / (nb * kBlock);
  k_bicg_restart<<<nb, kBlock, 0, s>>>(A, b, x, r, rhat, p, v, R, part);
  k_bicg_scalar<<<1, kBlock, 0, s>>>(part, nb, 4, st, nullptr, 0);
}

template void launch_bicg_iteration_part<double>(int, const Sell<double>&, BicgVecs<double>&,
                                                 double*, DevState*, double*, HostFlags*, int,
                                                 hipStream_t);
template void launch_bicg_iteration_part<float>(int, const Sell<double>&, BicgVecs<float>&,
                                                double*, DevState*, double*, HostFlags*, int,
                                                hipStream_t);

void launch_init_state(DevState* st, int m, double cycle_drop, hipStream_t s) {
  k_init_state<<<1, 64, 0, s>>>(st, m, cycle_drop);
}

void launch_set_cycle_length(DevState* st, int m, hipStream_t s) {
  k_set_cycle_length<<<1, 64, 0, s>>>(st, m);
}

template <typename TB, typename T>
void launch_scale_convert(const TB* b, const double* bscale, T* out, int n, const DevState* gate,
                          hipStream_t s) {
  using Op = ScaleConvertOp<TB, T>;
  launch_op<Op>(k_scale_convert<TB, T>, k_batch<Op>, typename Op::Args{b, bscale, out, n, gate},
                blocks_for(n), 0, s, (double)n * (sizeof(TB) + sizeof(T)));
}

template <typename TA, typename TB>
void launch_convert(const TA* a, TB* b, int n, hipStream_t s) {
  using Op = ConvertOp<TA, TB>;
  launch_op<Op>(k_convert<TA, TB>, k_batch<Op>, typename Op::Args{a, b, n}, blocks_for(n), 0, s,
                (double)n * (sizeof(TA) + sizeof(TB)));
}

template <typename T>
void launch_fill(T* a, T v, int n, hipStream_t s) {
  using Op = FillOp<T>;
  launch_op<Op>(k_fill<T>, k_batch<Op>, typename Op::Args{a, v, n}, blocks_for(n), 0, s,
                (double)n * sizeof(T));
}

void launch_step_rhs(const double* b, const double* x, double* out, double m, int n, int nux,
                     int ifirst, int nx, int off_v, int v_skip, int off_w, int off_p,
                     hipStream_t s) {
  if (n <= 0) return;
  k_step_rhs<<<blocks_for(n), kBlock, 0, s>>>(b, x, out, m, n, nux, ifirst, nx, off_v, v_skip,
                                              off_w, off_p);
}

// ------------------------------------------------------- instantiations
#define SD_INST_T(T, TB)                                                                      \
  template void launch_residual<T, TB>(const Sell<T>&, const TB*, const double*, const T*, T*, \
                                       const DevState*, hipStream_t);                         \
  template void launch_jacobi_zero<T, TB>(const Sell<T>&, const T*, const TB*, const double*, \
                                          T*, int, const DevState*, hipStream_t);              \
  template void launch_jacobi<T, TB>(const Sell<T>&, const T*, const TB*, const double*,      \
                                     const T*, T*, const DevState*, hipStream_t);             \
  template void launch_restrict_residual<T, TB>(const Sell<T>&, const TB*, const double*,     \
                                                const T*, int, T*, const DevState*, hipStream_t); \
  template void launch_presmooth_restrict<T, TB>(const Sell<T>&, const T*, const Sell<T>&,     \
                                                 const TB*, const double*, T*, T*,             \
                                                 const DevState*, hipStream_t);                \
  template void launch_prolong_smooth<T, TB>(const Sell<T>&, const Sell<T>&, const T*,         \
                                             const TB*, const double*, const T*, const T*, T*, \
                                             const DevState*, hipStream_t);

SD_INST_T(double, double)
SD_INST_T(float, double)
SD_INST_T(float, float)

template void launch_spmv<double, double, double>(const Sell<double>&, const double*, double*,
                                                  const DevState*, hipStream_t);
template void launch_spmv<float, float, float>(const Sell<float>&, const float*, float*,
                                               const DevState*, hipStream_t);
template void launch_prolong<double>(const Sell<double>&, const double*, double*,
                                     const DevState*, hipStream_t);
template void launch_prolong<float>(const Sell<float>&, const float*, float*, const DevState*,
                                    hipStream_t);
template void launch_ilu0<double>(const IluDev<double>&, const double*, double*,
                                  const DevState*, hipStream_t);
template void launch_ilu0<float>(const IluDev<float>&, const float*, float*, const DevState*,
                                 hipStream_t);
template void launch_coarse<double>(const double*, int, const double*, double*,
                                    const DevState*, hipStream_t);
template void launch_coarse<float>(const double*, int, const float*, float*, const DevState*,
                                   hipStream_t);
template void launch_block_sweep<double>(const Sell<double>&, int, const double*,
                                         const double*, const double*, double, double*,
                                         double*, double*, const DevState*, hipStream_t);
template void launch_block_sweep<float>(const Sell<float>&, int, const double*, const double*,
                                        const float*, double, float*, float*, float*,
                                        const DevState*, hipStream_t);
template void launch_add<double>(const double*, double*, int, const DevState*, hipStream_t);
template void launch_add<float>(const float*, float*, int, const DevState*, hipStream_t);
template void launch_arnoldi_step<double, double>(const Sell<double>&, const double*, double*,
                                                  double*, int64_t, int, DevState*, double*,
                                                  HostFlags*, hipStream_t, int, hipEvent_t*);
template void launch_arnoldi_step<float, float>(const Sell<float>&, const float*, double*,
                                                double*, int64_t, int, DevState*, double*,
                                                HostFlags*, hipStream_t, int, hipEvent_t*);
template void launch_arnoldi_step<double, float>(const Sell<double>&, const float*, double*,
                                                double*, int64_t, int, DevState*, double*,
                                                HostFlags*, hipStream_t, int, hipEvent_t*);
template void launch_update_x<double>(double*, const double*, int64_t, int, DevState*,
                                      hipStream_t);
template void launch_update_x<float>(double*, const float*, int64_t, int, DevState*,
                                     hipStream_t);
template void launch_scale_convert<double, double>(const double*, const double*, double*, int,
                                                   const DevState*, hipStream_t);
template void launch_scale_convert<double, float>(const double*, const double*, float*, int,
                                                  const DevState*, hipStream_t);
template void launch_scale_convert<float, float>(const float*, const double*, float*, int,
                                                 const DevState*, hipStream_t);
template void launch_convert<float, float>(const float*, float*, int, hipStream_t);
template void launch_convert<double, float>(const double*, float*, int, hipStream_t);
template void launch_convert<float, double>(const float*, double*, int, hipStream_t);
template void launch_convert<double, double>(const double*, double*, int, hipStream_t);
template void launch_copy_out<double>(const double*, double*, int64_t, const DevState*, int,
                                      hipStream_t);
template void launch_copy_out<float>(const float*, float*, int64_t, const DevState*, int,
                                     hipStream_t);
template void launch_fill<double>(double*, double, int, hipStream_t);
template void launch_fill<float>(float*, float, int, hipStream_t);

}  // namespace sd
