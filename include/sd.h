/*
 * sd.h -- C ABI of the MI355X coupled Stokes-Darcy solver.
 *
 * The library assembles the monolithic system of the paper's Sec. 2 (free
 * flow: creeping Stokes in symmetric-gradient form on a staggered grid,
 * stationary or one backward-Euler step of the transient equations; porous
 * medium: Darcy's law with two-point fluxes; interface Gamma:
 * normal-stress balance, Beavers-Joseph-Saffman slip, normal mass-flux
 * continuity) in the pressure-velocity block form
 *
 *       [ V    B   B1' ] [ v^ff ]   [ g ]
 *       [ C    0   0   ] [ p^ff ] = [ 0 ]
 *       [ C1'  0   D'  ] [ p^pm ]   [ 0 ]
 *
 * and solves it with flexible GMRES (or BiCGSTAB) right-preconditioned by the
 * pressure-velocity block-Jacobi or block-Gauss-Seidel preconditioner of
 * Sec. 4, whose velocity and Darcy sub-solves are one aggregation-AMG V-cycle
 * each (Sec. 5 solver setup).  All iteration work runs in HIP kernels on one
 * GPU; FP64 throughout, or mixed precision (FP32 preconditioner and inner
 * products with an FP64 outer residual, orthogonalisation and coarse solve).
 *
 * Conventions.  Every function returns an sd_status (0 = success) unless its
 * return type says otherwise; no C++ exception crosses this boundary.  On
 * failure sd_last_error() returns a thread-local message.  Host inputs are
 * copied during the call; the caller may free them on return.  Handles are
 * owned by the caller and released by the matching *_destroy.  Device
 * pointers must be allocated on the device that is current when the handle
 * was created.  A problem/solver handle must not be used from two threads at
 * once; a server handle is thread-safe.
 *
 * Grid.  The porous medium occupies [0,Lx] x [0,H_pm], the free flow
 * [0,Lx] x [H_pm, H_pm+H_ff]; both have nx cell columns, the free flow ny
 * rows and the porous medium ny_pm rows.  Unknown ordering (the pv blocks):
 * u faces (free-flow row j major, face i = 1..nu_x minor, nu_x = nx with a
 * traction right boundary, nx-1 with a velocity one), v faces (j = 0..ny-1,
 * j = 0 on Gamma), free-flow cell pressures, porous cell pressures (row k = 0
 * at the bottom).  Dirichlet velocity faces are eliminated and lifted into b.
 * 3-D (nz > 0): the box has depth Lz with nz cell layers in z; unknowns u, v,
 * w (z faces k = 1..nz-1), p, q, each ordered (row j, layer k, column i) with
 * i fastest; the velocity block is u, v, w.  The interface conditions hold
 * for both tangential velocities.
 */
#ifndef SD_H
#define SD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SD_OK = 0,
  SD_E_INVALID = -1,    /* bad argument (sizes, NaN/Inf, K <= 0, unsupported BC) */
  SD_E_NOMEM = -2,      /* device or host allocation failed / over budget      */
  SD_E_DEVICE = -3,     /* HIP runtime error or no GPU                           */
  SD_E_NOCONV = -4,     /* maxit reached: best iterate and stats still written   */
  SD_E_BREAKDOWN = -5,  /* NaN/Inf in the iteration or a zero pivot              */
  SD_E_BUSY = -6,       /* server: result not ready                              */
  SD_E_NOTFOUND = -7    /* server: unknown ticket                                */
} sd_status;

typedef struct sd_problem sd_problem;
typedef struct sd_solver sd_solver;
typedef struct sd_server sd_server;

/* Device-memory callbacks (e.g. a framework's caching allocator).  NULL for
 * the library default (the stream-ordered pool: hipMallocAsync /
 * hipFreeAsync).  alloc returns NULL on failure; the library takes memory in
 * chunks of 32 MiB (larger arrays get their own) and returns each chunk with
 * free, on the stream it was allocated on, once the handle that owns it is
 * destroyed and its work has finished. */
typedef struct {
  void* (*alloc)(size_t bytes, void* ctx, void* hip_stream);
  void (*free)(void* ptr, void* ctx, void* hip_stream);
  void* ctx;
} sd_allocator;

typedef struct {
  int nx, ny, ny_pm;          /* cells: columns, free-flow rows, porous rows  */
  double Lx, H_ff, H_pm;      /* extents; Gamma at y = H_pm                    */
  int nz;                     /* spanwise cells (z); 0 = the 2-D problem       */
  double Lz;                  /* spanwise extent (3-D only)                    */
  int nx_pm;                  /* 2-D: porous columns (0 = nx), a block under   */
  int pm_i0;                  /* free-flow columns pm_i0..pm_i0+nx_pm-1; the
                                 free-flow bottom beside it is a no-slip wall  */
} sd_grid;

typedef struct {
  double mu;                  /* dynamic viscosity (rho = 1, nu = mu)          */
  double alpha_bj;            /* Beavers-Joseph coefficient                    */
  double dt;                  /* backward-Euler time step; 0 = stationary      */
  int bj_full;                /* 0: Beavers-Joseph-Saffman (the paper's);
                                 1: full Beavers-Joseph, the slip condition
                                 keeps the porous tangential velocity
                                 -(K_f/mu) dq/dt along Gamma (not supported by
                                 the partitioned coupling)                    */
} sd_physics;

typedef enum { SD_BC_VELOCITY = 0, SD_BC_TRACTION = 1, SD_BC_PRESSURE = 2,
               SD_BC_NOFLOW = 3 } sd_bc_type;

/* Boundary conditions.  Free-flow top: SD_BC_VELOCITY; left and right:
 * SD_BC_VELOCITY or SD_BC_TRACTION (2-D; a pressure-driven inlet or outlet is
 * a traction boundary whose normal datum is the pressure; 3-D: left
 * SD_BC_VELOCITY); porous left/right/bottom (and back/front in 3-D):
 * SD_BC_PRESSURE or SD_BC_NOFLOW.  Data arrays may be NULL (zero).  With a
 * narrow porous block (nx_pm < nx) the porous arrays have nx_pm columns.
 * 2-D shapes:
 *   ff_left_n [ny] u (velocity) or n.(pI - tau)n (traction) at x = 0
 *   ff_left_t [ny+1] v (velocity) or t.(pI - tau)n (traction), y_G + j dy
 *   ff_right_n [ny]  u (velocity) or n.(pI - tau)n (traction) at x = Lx
 *   ff_right_t [ny+1] v (velocity) or t.(pI - tau)n (traction), y_G + j dy
 *   ff_top_t [nx+1] u on the top wall at x = i dx; ff_top_n [nx] v on the top
 *   pm_left_p, pm_right_p [ny_pm], pm_bottom_p [nx] Dirichlet pressures
 * 3-D (x streamwise, y normal to Gamma, z spanwise; the z walls of the free
 * flow are velocity walls; every array row-major with x fastest):
 *   ff_left_n, ff_right_n [ny][nz]; ff_left_t, ff_right_t [ny+1][nz];
 *   ff_left_tz, ff_right_tz [ny][nz+1] (w, or t_z.(pI - tau)n for traction);
 *   ff_top_t [nz][nx+1], ff_top_n [nz][nx], ff_top_tz [nz+1][nx] (w);
 *   ff_back_* on z = 0 and ff_front_* on z = Lz: _u [ny][nx+1], _v [ny+1][nx],
 *   _n (normal w) [ny][nx];
 *   pm_left_p, pm_right_p [ny_pm][nz], pm_bottom_p [nz][nx],
 *   pm_back_p, pm_front_p [ny_pm][nx]. */
typedef struct {
  int ff_left, ff_right, ff_top, pm_left, pm_right, pm_bottom;
  const double *ff_left_n, *ff_left_t, *ff_right_n, *ff_right_t;
  const double *ff_top_t, *ff_top_n;
  const double *pm_left_p, *pm_right_p, *pm_bottom_p;
  /* 3-D only */
  const double *ff_left_tz, *ff_right_tz, *ff_top_tz;
  const double *ff_back_u, *ff_back_v, *ff_back_n;
  const double *ff_front_u, *ff_front_v, *ff_front_n;
  const double *pm_back_p, *pm_front_p;
  int pm_back, pm_front;
} sd_bcs;

/* Forcing sampled at DoF locations (NULL = 0): f_u [ny][nx+1] at all u faces,
 * f_v [ny+1][nx] at all v faces, q_pm [ny_pm][nx] porous source; in 3-D
 * f_u [ny][nz][nx+1], f_v [ny+1][nz][nx], f_w [ny][nz+1][nx],
 * q_pm [ny_pm][nz][nx]. */
typedef struct {
  const double *f_u, *f_v, *q_pm;
  const double *f_w;
} sd_forcing;

/* Assemble the coupled system (Sec. 2) on the host and upload it to the
 * current device.  K: [ny_pm][nx] (3-D: [ny_pm][nz][nx]) positive
 * permeabilities (host).  The matrix
 * is kept in FP64; its values are those of the documented stencil evaluated
 * in IEEE double without contraction.  allocator may be NULL; hip_stream may
 * be NULL (default stream). */
int sd_assemble(const sd_grid* grid, const sd_physics* phys, const sd_bcs* bcs,
                const double* K, const sd_forcing* forcing,
                const sd_allocator* allocator, void* hip_stream, sd_problem** out);

/* Same as sd_assemble without any device work (usable without a GPU); such
 * a problem can be inspected and set up with sd_setup_host only. */
int sd_assemble_host(const sd_grid* grid, const sd_physics* phys,
                     const sd_bcs* bcs, const double* K,
                     const sd_forcing* forcing, sd_problem** out);

/* N, block offsets [0, off_v, off_p, off_q, N] and nnz of the assembled A. */
int sd_problem_info(const sd_problem* pb, int64_t* N, int64_t block_off[5],
                    int64_t* nnz);

/* Read-only views of the host CSR (sorted columns) and the assembled b;
 * valid until sd_problem_destroy. */
int sd_problem_csr(const sd_problem* pb, const int64_t** rowptr,
                   const int32_t** col, const double** val, const double** b);

/* Outer Krylov methods (the solvers of the Sec. 5 setup): flexible GMRES(m)
 * with a fixed restart length; BiCGSTAB; PD-GMRES, the outer solver of every
 * iterative row of the paper's Table 2 (Cuevas Nunez, Schaerer, Bhaya 2018),
 * flexible GMRES whose restart length is set before each cycle from the
 * true residual norms r_j at the restarts:
 *   m_{j+1} = m_j + floor(alpha_p r_j/r_{j-1}
 *                         + alpha_d (r_j - r_{j-2})/(2 r_{j-1}))
 * (derivative term from the third restart on; the first cycle takes
 * pd_m_init); when m_{j+1} < pd_m_min, pd_m_init grows by pd_m_step and
 * m_{j+1} = pd_m_init; lengths are capped at restart (the basis capacity).
 * The paper fixes m_init = m_min = 3, m_step = 5; the gains (defaults
 * alpha_p = -3, alpha_d = 5) are this library's reading. */
enum { SD_KRYLOV_FGMRES = 0, SD_KRYLOV_BICGSTAB = 1, SD_KRYLOV_PDGMRES = 2 };
/* Block preconditioners (Sec. 4): the pressure-velocity block-Jacobi and
 * block-Gauss-Seidel forms P^pv_BJ / P^pv_BGS, and the two-domain forms
 * P^td_BJ / P^td_BGS whose free-flow block A' = [[V, B], [C, 0]] is
 * preconditioned by one inexact Uzawa step: y_v = P_V r_v,
 * y_p = omega (r_p - C y_v), a Richardson step on the Schur complement with
 * omega = 1/lambda_max(-C P_V B) from 30 power iterations at set-up (the
 * schur option is ignored for them).  TD_BGS then equals the pv
 * block-Gauss-Seidel form with middle block omega I; TD_BJ keeps the v -> p
 * coupling inside A' and drops the porous coupling (y_pm = P_D' r_pm). */
enum { SD_PREC_BJ = 0, SD_PREC_BGS = 1, SD_PREC_TD_BJ = 2, SD_PREC_TD_BGS = 3 };
/* Middle (free-flow pressure) block of the preconditioner: the paper's
 * identity; mu M_p^-1 (the viscous Schur complement, M_p = diag(dx dy)); or,
 * for backward-Euler systems only (phys.dt > 0), the Cahouet-Chabard form
 * mu M_p^-1 + L_p^-1 (Cahouet & Chabard 1988) with L_p = B^T D^-1 B, D the
 * velocity mass dx dy / dt on rows with a time derivative and diag(V) on the
 * others, L_p^-1 one AMG V-cycle (hierarchy block 2).  It keeps the
 * iteration count bounded when sqrt(mu dt) is small against the domain,
 * where mu M_p^-1 alone stalls. */
enum { SD_SCHUR_IDENTITY = 0, SD_SCHUR_MASS = 1, SD_SCHUR_CC = 2 };
/* MIXED: preconditioner (AMG hierarchies, smoothers, block sweeps) in FP32
 * with FP32 accumulation; Arnoldi product, basis, Hessenberg, x and the
 * restart residual in FP64 (flexible GMRES absorbs the FP32 preconditioner).
 * MIXED32: the Arnoldi product w = A z in FP32 as well; a cycle then also
 * ends once its implicit residual estimate has dropped by 1e-6, the accuracy
 * an FP32 product can support, and the FP64 restart residual refines. */
enum { SD_PRECISION_FP64 = 0, SD_PRECISION_MIXED = 1, SD_PRECISION_MIXED32 = 2 };
enum { SD_AMG_PLAIN = 0, SD_AMG_SMOOTHED = 1 };
/* Darcy sub-solve P_D' of the block preconditioners: one AMG V-cycle on
 * D~ (default), or ILU(0) of D~ (Meijerink & van der Vorst 1977), the Darcy
 * preconditioner of the paper's P^td_BJ/BGS(Uzawa, ILU(0)) rows (Sec. 5
 * solver setup, Table 2).  ILU(0) is factorised on the host at set-up
 * (elimination in row order, entries outside the pattern of D~ dropped) and
 * applied by level-scheduled forward and backward substitution in one
 * workgroup.  Set-up fails with SD_E_INVALID if a row of D~ has more than 4
 * entries on either side of its diagonal or a substitution has more than
 * 4096 levels (a 2-D grid of nx x ny porous cells has nx + ny - 1), and
 * with SD_E_BREAKDOWN on a zero pivot. */
enum { SD_DARCY_AMG = 0, SD_DARCY_ILU0 = 1 };

typedef struct {
  int krylov;        /* SD_KRYLOV_*                                            */
  int restart;       /* FGMRES restart length m (1..63), default 30; the
                        largest PD-GMRES cycle                                 */
  int maxit;         /* total iteration cap, default 1000                      */
  double tol;        /* relative true FP64 residual ||b-Ax||/||b||             */
  int precond;       /* SD_PREC_BJ | SD_PREC_BGS | SD_PREC_TD_BJ | SD_PREC_TD_BGS */
  int schur;         /* middle block: identity or mu * M_p^-1                  */
  int precision;     /* SD_PRECISION_FP64 | _MIXED | _MIXED32                  */
  int amg;           /* SD_AMG_SMOOTHED (default) | SD_AMG_PLAIN               */
  int mis;           /* root independent set distance: 1 or 2 (default 2)     */
  double theta;      /* strength threshold, default 0.08                       */
  double omega;      /* Jacobi damping, default 2/3                            */
  int nu_pre, nu_post; /* Jacobi sweeps, default 2 / 2                         */
  int coarse_max;    /* coarsest level size bound (dense inverse), default 2048 */
  int max_levels;    /* default 20                                             */
  int darcy;         /* SD_DARCY_AMG (default) | SD_DARCY_ILU0                 */
  int pd_m_init, pd_m_min, pd_m_step;   /* PD-GMRES: defaults 3, 3, 5          */
  double pd_alpha_p, pd_alpha_d;        /* PD-GMRES gains: defaults -3, 5      */
  int stencil_slices; /* 1 (default): 64-row slices of a one-lane-per-row
                        matrix whose rows share one list of column offsets
                        (a grid stencil) store those offsets once and read no
                        column indices; 0: every slice reads its indices.
                        Results are identical either way.                     */
  int fused_restriction; /* 1 (default): on the coarser AMG levels, and on
                        the finest one below 196,608 rows, the two
                        pre-smoothing sweeps and the restriction of the
                        residual are one pass through G = R (I - A M2)
                        (M2: the two sweeps from zero), formed on the host at
                        set-up and kept where G has at most 3x the nonzeros
                        of the operators it replaces; 0: separate passes and
                        no G, a cheaper set-up (a serving request spends
                        about a fifth of its host preparation on G) for a
                        few more launches per V-cycle.                        */
} sd_solver_opts;

/* Fill opts with the defaults above. */
void sd_solver_opts_default(sd_solver_opts* opts);

/* Set up the preconditioned Krylov solver of an assembled problem: the
 * aggregation-AMG hierarchies of the Sec. 5 solver setup (one V-cycle per
 * sub-solve) for the velocity block V and for the Darcy block
 * D~ = D' - C1' diag(V)^-1 B1' (built on the host, deterministically), the
 * operators of the Sec. 4 block preconditioner selected by opts (NULL = the
 * defaults of sd_solver_opts_default) and the Krylov workspace, all uploaded
 * to the problem's device through the allocator given to sd_assemble.  The
 * handle keeps a pointer to pb, which must outlive it.  SD_E_INVALID for
 * options out of range, a problem assembled by sd_assemble_host, or more
 * than 16,777,216 unknowns (the row-block limit of the Gram-Schmidt
 * kernels); SD_E_NOMEM when a device allocation fails. */
int sd_setup(sd_problem* pb, const sd_solver_opts* opts, sd_solver** out);

/* Host-only setup (no device work), for inspection. */
int sd_setup_host(sd_problem* pb, const sd_solver_opts* opts, sd_solver** out);

/* Hierarchy inspection: block 0 = V, 1 = D~, 2 = L_p (SD_SCHUR_CC only;
 * otherwise it has 0 levels).  n_levels counts the coarsest. */
int sd_solver_levels(const sd_solver* s, int block, int* n_levels);
/* which: 0 = A_l, 1 = P_l (n_l x n_{l+1}), 2 = R_l.  Host CSR views. */
int sd_solver_level_csr(const sd_solver* s, int block, int level, int which,
                        int64_t* n_rows, int64_t* n_cols, const int64_t** rowptr,
                        const int32_t** col, const double** val);
int sd_solver_level_agg(const sd_solver* s, int block, int level,
                        const int32_t** agg, int64_t* n);
/* ILU(0) inspection (SD_DARCY_ILU0 only, SD_E_INVALID otherwise): the
 * forward (lower != 0: the strict L part) or backward (the strict U part and
 * diag = u_ii) substitution in level order.  lev[0..n_levels] are level
 * pointers into the n positions; ord[q] is the Darcy-block row of position
 * q; its off-diagonal entries occupy slots k = 0..3 at col[k*n + q],
 * val[k*n + q] in ascending column order, padded with col -1 and val 0.
 * Host views, valid until sd_solver_destroy; diag may be NULL. */
int sd_solver_ilu(const sd_solver* s, int lower, int64_t* n, int* n_levels,
                  const int32_t** lev, const int32_t** ord, const int32_t** col,
                  const double** val, const double** diag);
/* Dense row-major inverse of the coarsest operator of a block. */
int sd_solver_coarse_inverse(const sd_solver* s, int block, const double** inv,
                             int64_t* n);

typedef struct {
  int iters, restarts;
  double rel_res;            /* final true FP64 relative residual           */
  double rel_res_block[3];   /* per block (v, p^ff, p^pm), relative to ||b|| */
  double t_setup, t_solve;   /* seconds                                     */
} sd_stats;

/* Solve the coupled system A x = b of Sec. 2 with the Krylov method of the
 * options (flexible GMRES(m) or BiCGSTAB, the solvers of the Sec. 5 setup),
 * right-preconditioned by the block preconditioner of Sec. 4, to the
 * relative true residual ||b - A x|| <= tol ||b|| (recomputed in FP64 at
 * every restart).  d_b: device FP64 [N], or NULL for the assembled b.  d_x:
 * device FP64 [N], the initial guess when use_x0 != 0 (else overwritten from
 * zero) and the result; both are owned by the caller and must not alias.
 * Ordered after the work already on hip_stream (NULL = default); returns
 * after the solve has finished.  SD_E_NOCONV still writes the best iterate
 * and stats; SD_E_BREAKDOWN on a non-finite value. */
int sd_solve(sd_solver* s, const double* d_b, double* d_x, int use_x0,
             sd_stats* stats, void* hip_stream);

/* Time stepping (Sec. 2: transient Stokes in the free flow, stationary Darcy
 * in the porous medium, first-order backward Euler in time).  With
 * phys.dt > 0 the assembled matrix is that of one step: every interior u and
 * v face row (not the outflow u faces, not the Gamma rows) integrates dv/dt
 * over its control volume, adding m = |CV|/dt = dx dy / dt (rho = 1) to its
 * diagonal; the assembled b is the step's data part (boundary data and
 * sources).  The step from state x^n solves A x^{n+1} = b_data + M x^n.
 *
 * sd_step_rhs: d_b_out = d_b_data + m d_x_prev on those rows and d_b_data on
 * the others (device FP64 vectors of length N; d_b_data NULL = the assembled
 * b).  Each entry is one rounded product and one rounded sum, never fused,
 * so the result is reproducible bit for bit.  d_b_out may alias either input.
 * Enqueued on hip_stream; returns without waiting.  SD_E_INVALID for a
 * stationary problem or a NULL vector. */
int sd_step_rhs(sd_solver* s, const double* d_b_data, const double* d_x_prev,
                double* d_b_out, void* hip_stream);

/* n_steps backward-Euler steps with the data part d_b_data (NULL = the
 * assembled b) held fixed: each step forms its right-hand side as
 * sd_step_rhs does and solves it with this solver's hierarchies (set up once
 * for all steps), starting from the previous state.  d_x: device FP64 [N],
 * the state at t on entry, at t + n_steps dt on return.  stats: NULL or an
 * array of n_steps entries, one per step.  steps_done: NULL or the number of
 * steps completed.  Stops at the first step that fails and returns its
 * status; d_x then holds that step's best iterate.  Returns after the last
 * step has finished. */
int sd_advance(sd_solver* s, const double* d_b_data, double* d_x, int n_steps,
               sd_stats* stats, int* steps_done, void* hip_stream);

/* Building blocks of the iteration on device vectors of the problem's
 * ordering (FP64, length N), exposed for testing and composition.
 * y = A x with the assembled FP64 matrix: */
int sd_apply_matrix(sd_solver* s, const double* d_x, double* d_y, void* hip_stream);
/* r = b - A x with the assembled FP64 matrix (the true residual the solver
 * recomputes at every restart) and its norms: d_norms[0..3] = ||r||_2 and
 * the norms of its velocity, free-flow pressure and porous pressure blocks
 * (device FP64, 4 entries).  d_b NULL = the assembled b; d_x NULL = zero;
 * d_r and d_norms are required (device, caller-owned).  Enqueued on
 * hip_stream; returns without waiting. */
int sd_residual(sd_solver* s, const double* d_b, const double* d_x, double* d_r,
                double* d_norms, void* hip_stream);
/* Allocation-free variant of sd_residual, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same kernels and results; the 3 x 512 block
 * partials of the norms live in a static 12 KiB device array of the library
 * (one per GPU, held until the process ends) instead of the solver's
 * workspace, and the call allocates nothing.  Every call on one GPU shares
 * that array: calls that overlap there (other streams or threads) race and
 * must be serialised by the caller.  Nothing in it needs clearing (each
 * partial is written before it is read).  Same arguments and errors as
 * sd_residual; SD_E_INVALID beyond 16,777,216 unknowns. */
int sd_residual_noalloc(sd_solver* s, const double* d_b, const double* d_x, double* d_r,
                        double* d_norms, void* hip_stream);
/* z = P(r), one application of the configured block preconditioner (in FP32
 * inside when the solver is mixed; input and output are FP64): */
int sd_apply_preconditioner(sd_solver* s, const double* d_r, double* d_z,
                            void* hip_stream);
/* x = one V-cycle on block (0 = V, 1 = D~, 2 = L_p) for right-hand side b
 * (device FP64 vectors of n entries; n must equal the block's size, the
 * row count of its finest level, else SD_E_INVALID): */
int sd_apply_vcycle(sd_solver* s, int block, const double* d_b, double* d_x,
                    int64_t n, void* hip_stream);

/* Host threads that the set-up steps (assembly, AMG set-up, layout builds)
 * started from the calling thread may use: n >= 1 caps them, 0 restores the
 * default (up to 16).  Applies to the calling thread only; a caller running
 * several set-ups at once gives each its share of the host.  Results do not
 * depend on the thread count.  SD_E_INVALID for n < 0. */
int sd_set_host_threads(int n);

/* Row blocking of the Gram-Schmidt projection kernel for n unknowns: rows
 * per workgroup, workgroups, and dynamic LDS bytes per workgroup (the block's
 * rows of w and u_j in FP64).  SD_E_INVALID for n < 1 or n above the limit
 * that sd_setup enforces.  Host-only inspection. */
int sd_arnoldi_layout(int64_t n, int* rows_per_block, int* blocks, size_t* lds_bytes);

/* Sparse matrix layout of the device kernels, built on the host exactly as a
 * solver uploads a matrix (host-only inspection).  Sliced ELLPACK: slices of
 * C = 64 / lpr rows; entry k of row r of slice s at sptr[s] + C k + (r - C s)
 * (with width > 0 every slice has that width and sptr[s] = C width s);
 * padding has val 0.  lpr = 1 unless allow_csr lets a matrix with few or long
 * rows take several lanes per row (the AMG hierarchy matrices).
 * Stencil slices (stencil = 1, lpr = 1 only): a slice stores its rows on the
 * ascending union o_0 < o_1 < ... of their offsets col - row (a grid
 * stencil), each row with an explicit zero at the offsets it lacks, and
 * doff[sptr[s] / 64 + k] = o_k (positions past the union repeat its last
 * offset); the kernels take column row + o_k, clamped into [0, n_cols)
 * (where the clamp acts the value is 0), and read no column indices for it.
 * A slice whose union is longer than its width is widened by up to 8
 * positions when slices have their own widths (width = 0); otherwise, or
 * when a row repeats a column, it is read through col.  info.stencil: 0 no
 * stencil slices (doff NULL, n_doff = 0; also when they would hold less than
 * half of the entries), 2 every slice, 1 some: doff[sptr[s] / 64] = INT32_MIN
 * marks the others.  One more INT32_MIN closes doff (a slice of width 0 has
 * no entry).  col is complete for every slice (the clamped row + o_k in
 * stencil slices).  idx counts the column indices or offsets a pass over the
 * matrix reads.  Input: CSR with n_rows + 1 row pointers from
 * 0 and columns in [0, n_cols); SD_E_INVALID otherwise or beyond 2^31 stored
 * entries.  The views stay valid until sd_sell_destroy. */
typedef struct sd_sell sd_sell;
typedef struct {
  int lpr, width, stencil;
  int64_t n_rows, n_cols, nnz, idx;
  int64_t n_ptr, n_entries, n_doff;   /* lengths of sptr, col / val, doff */
  const int32_t* sptr;
  const int32_t* col;
  const double* val;
  const int32_t* doff;
} sd_sell_info;
int sd_sell_build(int64_t n_rows, int64_t n_cols, const int64_t* rowptr,
                  const int32_t* col, const double* val, int allow_csr,
                  int stencil, sd_sell** out);
int sd_sell_view(const sd_sell* m, sd_sell_info* info);
void sd_sell_destroy(sd_sell* m);

/* Measurement: bracket every launch of one kernel class with HIP events
 * during subsequent sd_solve calls (those solves then launch kernels one by
 * one instead of replaying graphs).  kernel_class: 0 = off,
 * SD_PROF_ARNOLDI_SPMV (w = A z_j fused with the projection pass over the
 * basis), SD_PROF_ARNOLDI_UPDATE (the Gram-Schmidt update pass),
 * SD_PROF_JACOBI_V0 (damped-Jacobi sweep on the finest velocity level),
 * SD_PROF_PRECOND (one whole preconditioner application).
 * Resets the counters. */
enum { SD_PROF_OFF = 0, SD_PROF_ARNOLDI_SPMV = 1, SD_PROF_ARNOLDI_UPDATE = 2,
       SD_PROF_JACOBI_V0 = 3, SD_PROF_PRECOND = 4 };
int sd_solver_profile(sd_solver* s, int kernel_class);
/* One application of the block preconditioner (Sec. 4: the V-cycles of the
 * Sec. 5 setup and the block sweep; SD_PROF_PRECOND brackets it): its
 * algorithmic bytes (each matrix value and index, padding excluded, and each
 * vector entry read or written once, summed over its kernels) and its kernel
 * launches.  Host computation; no device work. */
int sd_solver_precond_cost(sd_solver* s, double* bytes, int* launches);
/* The scale X of the middle block's mu M_p^-1, identity or Uzawa term
 * (X = mu/(dx dy dz), 1, or omega). */
int sd_solver_middle_scale(const sd_solver* s, double* x);
/* Launches timed, their summed event durations (seconds) and the summed
 * algorithmic bytes of those launches (each matrix entry, vector entry and
 * index read or written once; padding excluded). */
int sd_solver_profile_read(const sd_solver* s, int64_t* launches, double* seconds,
                           double* bytes);

/* ------------------------------------------------- partitioned coupling */
/* The partitioned Dirichlet-Neumann coupling of Sec. 3: the free flow takes
 * the interface normal velocity v as Dirichlet data and returns the normal
 * stress sigma = p - 2 mu dv/dy on Gamma; the porous medium takes sigma as
 * its interface pressure, closed over the half top cell by Darcy's law
 * (transmissibility Ay K_top/(mu dy_pm/2)), and returns the interface
 * velocity.  The fixed point S_pm(S_ff(v)) = v is the monolithic solution.
 * Post-processing: Aitken relaxation, or IQN-ILS (the paper's choice: a
 * quasi-Newton step with the inverse Jacobian fitted in the least-squares
 * sense to the history of inputs and outputs, Degroote et al. 2009).  The
 * iteration stops when ||sigma_k - sigma_{k-1}|| < eps ||sigma_k|| and
 * ||vt_k - v_k|| < eps ||vt_k|| (Sec. 3).  Both subdomain systems are solved
 * on the GPU by FGMRES with the block preconditioner (the missing block left
 * out), to the tolerance in the sub-solver options, each warm-started from
 * its previous state.  With SD_SCHUR_CC on a backward-Euler problem the
 * free-flow solver keeps the Cahouet-Chabard middle block (on a stationary
 * problem, and for the porous solver, SD_SCHUR_MASS is used).  The
 * interface vectors (nx or nx nz values) are kept on the host. */
typedef struct sd_dn sd_dn;
enum { SD_DN_AITKEN = 0, SD_DN_IQN_ILS = 1 };
typedef struct {
  int accel;        /* SD_DN_AITKEN | SD_DN_IQN_ILS (default)                  */
  double eps;       /* relative interface tolerance, default 1e-8              */
  int maxit;        /* coupling iterations, default 200                         */
  double omega0;    /* first relaxation factor, default 0.5                     */
} sd_dn_opts;
typedef struct {
  int iters, converged;       /* coupling iterations; 1 if the rule was met   */
  int ff_iters, pm_iters;     /* FGMRES iterations summed over the sub-solves  */
  double t_solve;             /* seconds                                       */
  double dp_rel, dv_rel;      /* last ||dsigma||/||sigma|| and ||r||/||vt||    */
} sd_dn_stats;
void sd_dn_opts_default(sd_dn_opts* o);
/* Split an assembled device problem and set up both subdomain solvers
 * (sub: their options, NULL = defaults).  The problem must outlive the
 * handle. */
int sd_dn_setup(sd_problem* pb, const sd_solver_opts* sub, sd_dn** out);
/* Solve A x = b by the coupling iteration.  d_b: device FP64 [N] or NULL (the
 * assembled b); its interface rows must be zero, as assembled and as
 * sd_step_rhs leaves them (SD_E_INVALID otherwise).  d_x: device FP64 [N],
 * written in the monolithic ordering (the interface velocity is the last
 * input v).  Returns SD_E_NOCONV after maxit iterations (x and stats still
 * written), or a sub-solver's failure status.  Returns after the solve. */
int sd_dn_solve(sd_dn* h, const sd_dn_opts* o, const double* d_b, double* d_x,
                sd_dn_stats* stats, void* hip_stream);
void sd_dn_destroy(sd_dn* h);

/* ---------------------------------------------------------------- serving */
typedef struct {
  size_t hbm_budget;   /* bytes the server may hold (0 = 80% of free HBM)     */
  int max_slots;       /* concurrently active solves (default 8)             */
  int device;          /* HIP device ordinal                                 */
} sd_server_opts;

/* Start the request loop on opts->device (opts NULL = defaults).  allocator:
 * device memory of every request's matrices, hierarchies and Krylov state
 * (NULL = the stream-ordered pool, hipMallocAsync); its callbacks may be
 * called from the server's threads, with the device current, and must be
 * thread-safe.  It must stay valid until sd_server_destroy returns. */
int sd_server_create(const sd_server_opts* opts, const sd_allocator* allocator,
                     sd_server** out);

typedef struct {
  sd_grid grid;
  sd_physics phys;
  sd_bcs bcs;
  const double* K;     /* [ny_pm][nx] host                                  */
  sd_forcing forcing;
  sd_solver_opts opts;
} sd_request;

/* Queue a solve.  All host data is copied.  SD_E_NOMEM if the request can
 * never fit the budget; SD_E_INVALID for a 3-D grid (the request loop serves
 * 2-D problems) or SD_KRYLOV_BICGSTAB (the loop drives the restarted GMRES
 * forms). */
int sd_submit(sd_server* sv, const sd_request* req, uint64_t* ticket);

enum { SD_REQ_PENDING = 0, SD_REQ_RUNNING = 1, SD_REQ_DONE = 2, SD_REQ_FAILED = 3 };

typedef struct {
  int state;               /* SD_REQ_*                                       */
  int status;              /* sd_status of the solve when DONE/FAILED        */
  const double* x_host;    /* solution [N] (valid until sd_result_release)   */
  int64_t N;
  sd_stats stats;
  double t_submit, t_admit, t_done;   /* seconds on the server's clock      */
} sd_result;

/* Counters of the shared launches since sd_server_create: groups formed
 * (requests whose iterations have the same kernel sequence share one), graph
 * replays (each runs one Arnoldi column for every active member of a group
 * in one batched launch per kernel), columns run by them (summed over the
 * replays' members) and the most members a replay served. */
typedef struct {
  int64_t groups, replays, member_columns;
  int max_members;
} sd_batch_stats;
int sd_server_batch_stats(sd_server* sv, sd_batch_stats* out);

/* Non-blocking. */
int sd_poll(sd_server* sv, uint64_t ticket, sd_result* out);
/* Block until the ticket is DONE or FAILED (or timeout_s elapses: SD_E_BUSY). */
int sd_wait(sd_server* sv, uint64_t ticket, double timeout_s, sd_result* out);
int sd_result_release(sd_server* sv, uint64_t ticket);
int sd_cancel(sd_server* sv, uint64_t ticket);

void sd_problem_destroy(sd_problem* pb);
void sd_solver_destroy(sd_solver* s);
void sd_server_destroy(sd_server* sv);

const char* sd_status_string(int status);
const char* sd_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SD_H */
