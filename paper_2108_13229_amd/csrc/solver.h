// Device-resident solver: matrices, AMG hierarchies, Krylov workspace.
#pragma once

#include <memory>
#include <vector>

#include "device.h"
#include "sd_internal.h"

namespace sd {

#define SD_HIP(expr)                                                                  \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      throw ::sd::Error(SD_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Device allocations of one handle: 256-byte aligned pieces carved from a few
// large chunks, which come from the caller's allocator or from the
// stream-ordered pool (hipMallocAsync / hipFreeAsync, no device-wide
// synchronisation, so handles can come and go while other solves run).
class DeviceMem {
 public:
  DeviceMem() = default;
  DeviceMem(const sd_allocator* a, hipStream_t s) : stream_(s) {
    if (a && a->alloc && a->free) alloc_ = *a, has_ = true;
  }
  ~DeviceMem();
  DeviceMem(const DeviceMem&) = delete;
  DeviceMem& operator=(const DeviceMem&) = delete;
  void* get(size_t bytes);
  template <typename T>
  T* array(size_t n) { return static_cast<T*>(get(n * sizeof(T) + 16)); }
  size_t bytes() const { return total_; }

 private:
  void* chunk(size_t bytes);
  sd_allocator alloc_{};
  bool has_ = false;
  hipStream_t stream_ = nullptr;
  std::vector<void*> chunks_;
  char* cur_ = nullptr;
  size_t cur_off_ = 0, cur_cap_ = 0;
  size_t total_ = 0;
};

// Pinned host blocks (mapped for device writes when asked) reused across
// solver handles; never returned to the driver before the process ends.
void* pinned_acquire(size_t bytes, bool mapped);
void pinned_release(void* p, size_t bytes, bool mapped);

template <typename T>
struct DevLevel {
  int n = 0;
  Sell<T> A, P;
  Sell<T> AW;          // A diag(w): the fused pre-smoothing + restriction reads it
  Sell<T> R;           // restriction (finest level)
  Sell<T> Q;           // [R | -R A]: restricted residual from [b; x] (coarser levels)
  Sell<T> G;           // R (I - A M2): restricted residual after pre-smoothing, from b
  Sell<T> F;           // P - W A P: correction fused with the first post-sweep
  bool fuse_pre = false, fuse_post = false;
  T* wd = nullptr;     // omega / a_ii
  T* x = nullptr;      // iterate (levels >= 1)
  T* tmp = nullptr;
  T* r = nullptr;      // residual (finest level)
  T* b = nullptr;      // right-hand side (levels >= 1)
};

template <typename T>
struct DevHierarchy {
  std::vector<DevLevel<T>> lev;
  double* Ainv = nullptr;
  int n_coarse = 0;
};

struct SolverOpts {
  sd_solver_opts o;
  AMGOpts amg;
};

class Solver;

// Solver scalars as copied to the host (prefix of DevState).
struct HostState {
  int j, k, cycle_done, m, converged, breakdown, iters, pad0;
  double bnorm, target, cycle_drop, cycle_target, beta;
  double resblk[4];
};

// Progress of one resumable FGMRES solve.
struct SolveRun {
  enum Phase { INIT, WAIT_NORM, RESTART, WAIT_RESTART, ITER, DONE };
  Phase phase = INIT;
  const double* b = nullptr;
  double* x = nullptr;
  int use_x0 = 0;
  bool first = true;
  int restarts = 0, status = SD_E_NOCONV;
  int m_cycle = 0, j_enq = 0, completed = -1;
  double ctarget = 0.0, t0 = 0.0;
  sd_stats out{};
  // PD-GMRES: true residual norms at the restarts (newest last), the last
  // cycle length (0 before the first) and the current m_init
  std::vector<double> pd_res;
  int pd_m = 0, pd_m_init = 0;
  // the request loop runs this solve's columns in its shared graph (ITER is
  // then driven by the loop, see PrecBase::end_cycle)
  bool batched = false;
};

// Restart length of the next PD-GMRES cycle (the controller documented at
// SD_KRYLOV_PDGMRES in sd.h) from R.pd_res; updates R.pd_m and R.pd_m_init.
int pd_next_length(const sd_solver_opts& o, SolveRun& R, int m_cap);

// ILU(0) of a square matrix (Meijerink & van der Vorst 1977; the Darcy
// preconditioner of the paper's P^td(Uzawa, ILU(0)) rows, Sec. 5 solver
// setup and Table 2): elimination in row order, row i finished by
//   l_ik = a_ik / u_kk for each k < i of its pattern, ascending, each
//   followed by a_ij -= l_ik u_kj for the j > k of row k's pattern that are
//   in row i's pattern, ascending;
// every update outside the pattern is dropped.  For the device
// substitution the rows are ordered by level: a row's forward level is one
// more than the largest among the rows its L part references (0 without
// any), its backward level likewise over its strict U part.  Positions
// q = 0..n-1 run through the levels in order (rows ascending within a
// level); the triangle entries of position q are stored as ELL with
// kIluWidth slots, slot k at k * n + q, in ascending column order, padded
// with col -1 and val 0.
struct HostIlu {
  int64_t n = 0;
  std::vector<int32_t> lev_l, lev_u;   // level pointers into the positions
  std::vector<int32_t> ord_l, ord_u;   // row of each position
  std::vector<int32_t> col_l, col_u;   // kIluWidth * n
  std::vector<double> val_l, val_u;    // l_ij, u_ij (j != i)
  std::vector<double> diag_u;          // u_ii of each backward position
};
// Throws SD_E_INVALID (row without a diagonal entry, a triangle row wider
// than kIluWidth, more than kIluMaxLevels levels) or SD_E_BREAKDOWN (zero
// pivot).
void ilu0_host(const HostCSR& A, HostIlu& out);

// Precision-specific part: preconditioner operators and the Arnoldi matrix.
class PrecBase {
 public:
  virtual ~PrecBase() = default;
  virtual int fgmres(Solver& S, const double* b, double* x, int use_x0, sd_stats* st,
                     hipStream_t s) = 0;
  virtual int bicgstab(Solver& S, const double* b, double* x, int use_x0, sd_stats* st,
                       hipStream_t s) = 0;
  // resumable FGMRES: start() then step() until run.phase == DONE; step()
  // returns whether it made progress (it never blocks unless block is set)
  virtual void start(Solver& S, SolveRun& run) = 0;
  virtual bool step(Solver& S, SolveRun& run, bool block) = 0;
  // One Arnoldi column of this solve in the form the request loop replays
  // for every column: copy-in of u_j and sigma_j (j read on the device),
  // the preconditioner on the fixed buffers, copy-out into Z[j], the
  // Arnoldi step with j from the device; recorded (RecordedOp) instead of
  // launched.  Needs enable_column_replay().
  virtual void record_column(Solver& S, std::vector<RecordedOp>& ops) = 0;
  // End of a cycle whose columns the request loop ran: complete the last
  // column if the cycle ran to its full length, solve for y, x += Z y; the
  // run continues at RESTART.  Enqueued on s.
  virtual void end_cycle(Solver& S, SolveRun& run, bool full, hipStream_t s) = 0;
  // Algorithmic bytes (each matrix entry and vector entry read or written
  // once, padding excluded) and kernel launches of one preconditioner
  // application.
  virtual void precond_cost(Solver& S, double* bytes, int* launches) = 0;
  virtual void apply_precond(Solver& S, const double* r, double* z, hipStream_t s) = 0;
  virtual void apply_vcycle(Solver& S, int block, const double* b, double* x,
                            hipStream_t s) = 0;
};

class Solver {
 public:
  HostProblem* pb = nullptr;        // not owned
  SolverOpts opts;
  HostHierarchy hh[3];              // 0: V, 1: Darcy block with interface correction,
                                    // 2: pressure operator L_p (SD_SCHUR_CC only)
  HostIlu ilu;                      // ILU(0) of the Darcy block (SD_DARCY_ILU0; else n = 0)
  HostCSR Cf;                       // continuity and porous rows x velocity columns
  double xscale = 1.0;
  int64_t off[5] = {0, 0, 0, 0, 0};
  int N = 0;
  bool on_device = false;
  double t_setup = 0.0;

  // device
  std::unique_ptr<DeviceMem> mem;
  Sell<double> A64;
  double* b_dev = nullptr;
  double* step_b = nullptr;         // backward-Euler right-hand side (sd_advance)
  double* V = nullptr;              // (m+1) basis slots: orthonormal vectors + the open candidate
  double* W = nullptr;
  double* part = nullptr;
  DevState* st = nullptr;
  HostFlags* hf = nullptr;          // mapped pinned memory (host view)
  HostFlags* hf_dev = nullptr;      // the same memory as seen by kernels
  int64_t ldv = 0;
  std::vector<hipEvent_t> events;
  hipEvent_t ev_join = nullptr;
  hipEvent_t ev_state = nullptr;    // marks a finished state copy to hs
  HostState* hs = nullptr;          // pinned host copy of the solver scalars
  hipStream_t stream = nullptr;     // internal non-blocking stream (default priority)
  // block-Jacobi forms: the Darcy (and middle) blocks of an application run
  // on stream2 beside the velocity V-cycle (a parallel branch in a captured
  // graph); ev_fork / ev_back order it into the application's stream
  hipStream_t stream2 = nullptr;
  hipEvent_t ev_fork = nullptr, ev_back = nullptr;
  std::unique_ptr<PrecBase> prec;
  // measurement mode: events around one kernel class (0 = off)
  int prof_class = 0;
  int64_t prof_launches = 0;
  double prof_seconds = 0.0, prof_bytes = 0.0;
  std::vector<hipEvent_t> prof_ev;   // 2 per Arnoldi column
  int64_t nnz_A = 0, nnz_V0 = 0;
  // fixed buffers of the request loop's replayed columns (enable_column_replay)
  double* rin = nullptr;            // u_j
  double* sigfix = nullptr;         // sigma_j
  void* zfix = nullptr;             // preconditioned vector (preconditioner precision)

  ~Solver();
  void setup_host(HostProblem* p, const sd_solver_opts* o);
  void upload(const sd_allocator* alloc, hipStream_t s);
  size_t device_bytes() const { return mem ? mem->bytes() : 0; }
  int solve(const double* b, double* x, int use_x0, sd_stats* stats, hipStream_t s);
  void enable_column_replay();
  double uzawa_relaxation(hipStream_t s);
};

constexpr int kUzawaPowerIters = 30;

// SELL layout of a matrix on the host, as upload_sell copies it to the
// device (fields as in Sell; doff empty without stencil slices).
template <typename T>
struct HostSell {
  int64_t n_rows = 0, n_cols = 0, nnz = 0, idx = 0;
  int lpr = 1, width = 0, stencil = 0;
  std::vector<int> sptr, col, doff;
  std::vector<T> val;
};
// stencil: use stencil slices (see Sell) where the layout is SELL-64.
template <typename T>
HostSell<T> build_sell(const HostCSR& A, bool allow_csr, int force_lpr, bool stencil);

// SELL construction on the host and upload.
template <typename T>
Sell<T> upload_sell(const HostCSR& A, DeviceMem& mem, hipStream_t s, bool allow_csr = false,
                    int force_lpr = 0, bool stencil = false);

std::unique_ptr<PrecBase> make_prec_fp64(Solver& S, hipStream_t s);
std::unique_ptr<PrecBase> make_prec_fp32(Solver& S, hipStream_t s);

}  // namespace sd
