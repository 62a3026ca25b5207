// Internal declarations of the Stokes-Darcy library (host side).
#pragma once

#include <cstdint>
#include <functional>
#include <stdexcept>
#include <string>
#include <utility>
#include <vector>

#include "sd.h"

namespace sd {

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

// Compressed sparse rows with ascending column indices in every row.
struct HostCSR {
  int64_t n_rows = 0, n_cols = 0;
  std::vector<int64_t> rowptr;
  std::vector<int32_t> col;
  std::vector<double> val;
  int64_t nnz() const { return (int64_t)col.size(); }
};

// Unknown numbering of the pressure-velocity block form.
// 2-D: u, v, p, q; 3-D (nz > 0): u, v, w, p, q with (row j, layer k,
// column i) order, i fastest.  In 2-D off_w = off_p (no w block).
// 2-D with a porous block of nx_pm columns under free-flow columns
// i0..i0+nx_pm-1: the interface v faces come first in the v block, then rows
// j = 1..ny-1; u faces start at i_first (0 with a traction left boundary).
struct Layout {
  int nx = 0, ny = 0, nyp = 0, nux = 0, nz = 0;
  int nx_pm = 0, i0 = 0, i_first = 1;
  int64_t off_v = 0, off_w = 0, off_p = 0, off_q = 0, N = 0;
  // the interface v faces lead the v block (false for the free-flow
  // subsystem of the partitioned coupling, which has them removed)
  bool gamma_rows = true;
  int nzc() const { return nz > 0 ? nz : 1; }
  // interface faces: the porous top layer under the free flow
  int64_t n_gamma() const { return nz > 0 ? (int64_t)nx * nz : (int64_t)(nx_pm > 0 ? nx_pm : nx); }
  // rows with a time derivative: interior u faces (1..nx-1), v faces off the
  // interface, all w faces
  bool has_mass(int64_t r) const {
    if (r < off_v) {
      const int i = (int)(r % nux) + i_first;
      return i >= 1 && i <= nx - 1;
    }
    if (r < off_w) return !gamma_rows || r >= off_v + n_gamma();
    return r < off_p;
  }
  int64_t u(int i, int j) const { return (int64_t)j * nux + (i - i_first); }
  int64_t v(int i, int j) const {
    return j == 0 ? off_v + (i - i0) : off_v + n_gamma() + (int64_t)(j - 1) * nx + i;
  }
  int64_t p(int i, int j) const { return off_p + (int64_t)j * nx + i; }
  int64_t q(int i, int k) const { return off_q + (int64_t)k * (nx_pm > 0 ? nx_pm : nx) + i; }
  int64_t u3(int i, int j, int k) const { return ((int64_t)j * nz + k) * nux + (i - 1); }
  int64_t v3(int i, int j, int k) const { return off_v + ((int64_t)j * nz + k) * nx + i; }
  int64_t w3(int i, int j, int k) const {
    return off_w + ((int64_t)j * (nz - 1) + (k - 1)) * nx + i;
  }
  int64_t p3(int i, int j, int k) const { return off_p + ((int64_t)j * nz + k) * nx + i; }
  int64_t q3(int i, int j, int k) const { return off_q + ((int64_t)j * nz + k) * nx + i; }
};

struct HostProblem {
  sd_grid grid{};
  sd_physics phys{};
  int bc[6] = {0, 0, 0, 0, 0, 0};
  Layout L;
  HostCSR A;
  std::vector<double> b;
  bool pm_singular = false;
  double mass = 0.0;           // |CV|/dt of the backward-Euler rows (0: stationary)
  std::vector<double> K;       // porous permeabilities, [ny_pm][nz][nx]
};

void assemble_host(const sd_grid* g, const sd_physics* ph, const sd_bcs* bcs,
                   const double* K, const sd_forcing* f, HostProblem& out);
// The 3-D box (g->nz > 0); assemble_host dispatches to it.
void assemble_host_3d(const sd_grid* g, const sd_physics* ph, const sd_bcs* bcs,
                      const double* K, const sd_forcing* f, HostProblem& out);

// Row builder shared by the assembly routines: entries of one row are
// collected, sorted by column and appended to A.
struct RowBuilder {
  HostCSR& A;
  std::vector<std::pair<int32_t, double>> row;
  explicit RowBuilder(HostCSR& a) : A(a) {}
  void add(int64_t c, double v) { row.emplace_back((int32_t)c, v); }
  void finish();
};

HostCSR extract_block(const HostCSR& A, int64_t r0, int64_t r1, int64_t c0,
                      int64_t c1);

// D~ = D' - C1' diag(V)^-1 B1' on the porous block.
HostCSR darcy_interface_block(const HostCSR& D, const HostCSR& C1,
                              const HostCSR& B1, const HostCSR& V);

struct AMGOpts {
  double theta = 0.08, omega = 2.0 / 3.0, min_ratio = 1.2;
  int nu_pre = 2, nu_post = 2, coarse_max = 256, max_levels = 20;
  bool smoothed = true;
  int mis = 2;
};

struct HostLevel {
  HostCSR A, P, R;             // P, R empty on the coarsest level
  HostCSR AP;                  // A P (the first Galerkin factor)
  std::vector<int32_t> agg;    // empty on the coarsest level
  std::vector<int32_t> comp;
};

struct HostHierarchy {
  std::vector<HostLevel> levels;
  std::vector<double> Ainv;    // dense row-major inverse of the coarsest A
  int64_t n_coarse = 0;
};

void amg_setup_host(const HostCSR& A, const std::vector<int32_t>& comp,
                    bool singular, const AMGOpts& o, HostHierarchy& h);

// f(a, b) over contiguous sub-ranges of [r0, r1) on up to 16 threads (or
// the calling thread's cap, below).
void parallel_ranges(int64_t r0, int64_t r1, const std::function<void(int64_t, int64_t)>& f);

// Cap on the threads the host set-up steps started from the calling thread
// use (0: up to 16).  Threads that prepare several problems at once share
// the host: each takes a share instead of 16.
void set_host_threads(int n);

// A named host-side phase (assembly, set-up, upload, solve, a request's
// preparation) as a ROCTx range, which rocprofv3 --marker-trace shows beside
// the kernels; without a tracing tool attached it costs well under a
// microsecond.  Pushed and popped on the constructing thread.
class TraceRange {
 public:
  explicit TraceRange(const char* name);
  ~TraceRange();
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};

// Q = [R | -R A] (n_c x 2n): the restricted residual R (b - A x) = Q [b; x]
// in one sparse product, so that a V-cycle level needs no residual vector.
// RA: the product R A when the caller has it (the same values as computed
// here).
HostCSR residual_restriction(const HostCSR& A, const HostCSR& R);
HostCSR residual_restriction(const HostCSR& A, const HostCSR& R, const HostCSR& RA);
// Z = X Y, each entry summed in ascending inner index.
HostCSR sparse_product(const HostCSR& X, const HostCSR& Y);

// (X diag(s)) Y: every entry of X scaled by s of its column, then the
// product, each result entry summed in ascending inner index.
HostCSR scaled_product(const HostCSR& X, const std::vector<double>& s, const HostCSR& Y);

// With W = diag(omega / a_ii) and M2 = 2W - W A W (two damped-Jacobi sweeps
// from zero):
//   G = R (I - A M2)   restricted residual after the pre-smoothing, from b;
//   F = P - W A P      coarse correction plus its share of the first
//                      post-smoothing sweep: x + P xc followed by one sweep is
//                      x + W (b - A x) + F xc.
HostCSR presmoothed_restriction(const HostCSR& A, const HostCSR& R, double omega);
HostCSR presmoothed_restriction(const HostCSR& A, const HostCSR& R, const HostCSR& RA,
                                double omega);
HostCSR smoothed_correction(const HostCSR& A, const HostCSR& P, const HostCSR& AP,
                            double omega);

// 32-bit finaliser of MurmurHash3 (public domain).
inline uint32_t fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}

double wall_time();

}  // namespace sd
