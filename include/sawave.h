/*
 * sawave.h - C ABI of the MI355X (gfx950) solver library for sequences of sigma-transformed
 * Poisson systems with exponentially weighted subspace acceleration.
 *
 * What is computed (Sorensen, Guido, Engsig-Karup, Kressner, "Subspace Acceleration for
 * Efficient Nonlinear Water Wave Simulation"):
 *   - the mixed-stage operator A = grad^(i) . grad^(i-1) of the sigma-transformed pressure
 *     Poisson problem (Sec. 2.1 push-forward of the gradient; Sec. 3 discrete pressure
 *     equation), sixth-order first-derivative stencils (Sec. 5.2), p = 0 on the free surface,
 *     the Neumann condition n . grad^(i-1) p imposed through ghost nodes (Sec. 3 discrete
 *     Neumann equation);
 *   - left-preconditioned restarted GMRES (Sec. 3) with a fixed still-water preconditioner;
 *   - the initial guess of Alg. 2 with the basis V = Y of the EWMA sketch of Alg. 4,
 *     Y <- r Y + x omega^T after every solve (Sec. 4.1.2), or with V = X Omega of the
 *     randomized range finder of Alg. 3 over the K most recent solutions (Sec. 4.1.1).
 *
 * Grid and memory layout (all vectors of length n = ncol * (nz + 1), FP64 unless stated):
 *   node (level j, column c) has index j * ncol + c (x fastest). Level 0 is the ghost level
 *   below the bed (sigma = -1/(nz-1)), level 1 the bed (sigma = 0), level nz the free
 *   surface (sigma = 1). Periodic grids: ncol = nx - 1 columns at x = c dx, dx = L/(nx-1).
 *   Wall grids: ncol = nx + 2; columns 0 and ncol-1 are ghost columns, physical column p
 *   (x = p dx) has index p + 1. Bathymetry h and surface eta are given at the physical
 *   columns only (nx - 1 values periodic, nx values walls) and extended to ghost columns by
 *   even reflection. Row kinds: free-surface nodes and the four grid corners carry identity
 *   rows; the ghost level carries the bed condition -h_x G_x - G_z at the bed node above it;
 *   ghost columns carry -G_x (left) / +G_x (right) at the wall node next to them, where
 *   G_x = D_x p + sigma_x D_sigma p and G_z = D_sigma p / d use the previous stage's geometry.
 *
 * Errors: every function returns a status; 0 = success, > 0 = result produced but flagged,
 * < 0 = hard error, nothing produced. Functions never throw or abort across the ABI. The
 * message of the last hard error on the calling thread is available from sa_last_error().
 *
 * Ownership: the library owns every device buffer it allocates (operator data, preconditioner
 * hierarchy, Krylov basis, sketch, solution). Host input arrays are copied before return.
 * Device input pointers (mem = SA_MEM_DEVICE) are read on the problem's stream and must stay
 * valid until that stream has passed the consuming call. One problem must not be used from
 * two threads at once. All work is ordered on the hipStream_t given at creation
 * (NULL = the default stream).
 */
#ifndef SAWAVE_H
#define SAWAVE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------------------- */
enum {
  SA_OK = 0,
  SA_NOCONV = 1,     /* max_restarts reached: the last iterate is returned and stored   */
  SA_EARG = -1,      /* invalid argument                                                 */
  SA_EGEOM = -2,     /* h + eta <= 0 or non-finite surface/bathymetry                     */
  SA_ENONFINITE = -3,/* NaN/Inf in the right-hand side or during the solve               */
  SA_EOOM = -4,      /* device allocation failed                                         */
  SA_EDEVICE = -5,   /* HIP runtime error or device-side fault flag; problem unusable     */
  SA_ENOTBUILT = -6, /* no usable gfx950 device                                          */
  SA_EBUSY = -7      /* server: HBM budget exhausted, or the simulation still has work     */
};

enum { SA_PERIODIC = 0, SA_WALLS = 1 };
enum { SA_PC_NONE = 0, SA_PC_LINE = 1, SA_PC_MG = 2, SA_PC_ILU0 = 3 };
enum { SA_GUESS_COLD = 0, SA_GUESS_PREVIOUS = 1, SA_GUESS_EWMA = 2, SA_GUESS_RANGE = 3 };
enum { SA_FP64 = 0, SA_FP32_IR = 1 };
enum { SA_MEM_HOST = 0, SA_MEM_DEVICE = 1 };
enum { SA_SYNC = 0, SA_ASYNC = 1 };
enum { SA_DECAY_SOLVES = 0, SA_DECAY_TIME = 1 };

/* Grid: nx points on [0, length] (inclusive), nz sigma levels from bed to surface. */
typedef struct {
  int32_t nx, nz;
  int32_t bc;       /* SA_PERIODIC | SA_WALLS                                               */
  double length;
} sa_grid;

/* Solver options. sa_default_options() fills the defaults listed here. */
typedef struct {
  int32_t restart;      /* GMRES restart length m (1..64), default 30                      */
  int32_t max_restarts; /* default 200                                                     */
  double rtol;          /* true relative residual ||b - A x|| / ||b||, default 1e-8         */
  int32_t precond;      /* SA_PC_*, default SA_PC_MG. SA_PC_ILU0: the paper's preconditioner */
                        /* (Sec. 3): ILU(0) of the sixth-order operator at eta = 0 on its   */
                        /* structural pattern, factored on the host at creation, applied   */
                        /* by level-scheduled substitution on one workgroup (cluster forced */
                        /* to 1; FP64 only: SA_EARG with SA_FP32_IR)                        */
  int32_t nu1, nu2;     /* smoothing sweeps (MG) / sweeps (LINE: nu1), default 1, 1        */
  double omega;         /* line-Jacobi damping, default 0.5                                */
  int32_t max_levels;   /* MG levels including the finest, default 32 (as deep as possible)*/
  int32_t guess;        /* SA_GUESS_*, default SA_GUESS_EWMA                               */
  int32_t k;            /* sketch rank (1..16), default 8                                  */
  double r;             /* forgetting factor per stored solution (0..1], default 0.9       */
  uint64_t seed;        /* sketch stream seed, default 0                                   */
  int32_t n_init;       /* solves that use the previous solution before the sketch, 0      */
  double tau_drop;      /* least-squares column drop threshold, default 1e-7               */
  int32_t precision;    /* SA_FP64 | SA_FP32_IR, default SA_FP64                            */
                        /* SA_FP32_IR: FP64 iterative refinement around FP32 GMRES cycles on */
                        /* A d = r / ||r|| (operator, V-cycle, basis FP32; Gram-Schmidt sums,*/
                        /* Hessenberg, Givens FP64); candidates x + ||r|| d are checked on  */
                        /* the FP64 residual with the FP64 path's trigger rule              */
  double rtol_inner;    /* FP32 resolution: a cycle whose Arnoldi estimate has fallen to    */
                        /* this fraction of its start hands its checked candidate to the    */
                        /* next correction (SA_FP32_IR), default 1e-4                       */
  int32_t max_refine;   /* FP32 cycles cap (SA_FP32_IR), default 200; SA_NOCONV after      */
  int32_t cluster;      /* workgroups cooperating on one solve; 0 = one per 32 columns    */
                        /* of the grid, at most 256                                        */
  int32_t profile;      /* 1: accumulate per-phase device time (sa_get_phase_times), 0      */
  int32_t coarse_max;   /* MG: coarsening stops at the first grid with at most this many    */
                        /* unknowns, solved exactly there (<= 4096), default 700            */
  int32_t window;       /* SA_GUESS_RANGE: K, the solutions kept in the sliding window of   */
                        /* the randomized range finder (Alg. 3, V = X Omega with the k x K  */
                        /* Gaussian rows drawn as the solutions enter), k..32, default 16   */
  int32_t decay;        /* units of the EWMA sketch's forgetting exponent (Alg. 4):         */
                        /* SA_DECAY_SOLVES (default) Y <- r Y + x w^T per stored solution;  */
                        /* SA_DECAY_TIME Y <- r^((tau_x - tau_prev) / decay_dtau) Y + x w^T */
                        /* with the time labels of the stored solutions given by            */
                        /* sa_set_time (Alg. 4's exponent in physical time); EWMA only      */
  double decay_dtau;    /* SA_DECAY_TIME: the time unit of the exponent (> 0), default 1    */
  int32_t orthonormalize; /* SA_GUESS_RANGE: 1 takes V = Q, the orthonormal factor of the   */
                        /* sketch X Omega (Alg. 3), by a Cholesky factorisation of its      */
                        /* double-double Gram taking columns in order and dropping one whose */
                        /* projected norm (of the unit column) is below tau_drop; 0 (default)*/
                        /* takes V = X Omega                                                 */
} sa_options;

/* Per-solve report. iters counts Arnoldi steps over all cycles (FP32_IR: inner steps over
 * all refinements); refinements counts FP64 correction steps (FP32_IR only). */
typedef struct {
  int32_t iters, restarts, refinements, status;
  int32_t rank;         /* sketch columns kept by the least-squares guess                  */
  int32_t checks;       /* true-residual checks triggered by the Arnoldi estimate          */
  double relres0;       /* ||b - A x0|| / ||b||                                            */
  double relres;        /* ||b - A x|| / ||b|| of the returned solution                    */
} sa_solve_info;

typedef struct sa_problem sa_problem;

void sa_default_options(sa_options* opt);

/* Create a problem. h: bathymetry at the physical columns (host, nx-1 or nx values, > 0).
 * hip_stream: hipStream_t to order all work on (NULL = default stream). */
int sa_create(const sa_grid* grid, const double* h, const sa_options* opt, void* hip_stream,
              sa_problem** out);
void sa_destroy(sa_problem* p);

/* Number of unknowns n = ncol * (nz + 1) and number of columns ncol. */
int64_t sa_size(const sa_problem* p);
int32_t sa_ncol(const sa_problem* p);

/* Surfaces of the previous and current stage (Sec. 3: the solve at stage i uses eta^(i-1)
 * and eta^(i)), nx-1 (periodic) or nx (walls) values each. Copied (host) or read on the
 * stream (device). */
int sa_set_surface(sa_problem* p, const double* eta_prev, const double* eta_cur, int32_t mem);

/* Right-hand side b (n values). Host: copied. Device: referenced, not copied. */
int sa_push_rhs(sa_problem* p, const double* b, int32_t mem);

/* Time label tau of the system the next sa_solve solves (Alg. 4: the stage time whose
 * differences the forgetting exponent counts), for decay = SA_DECAY_TIME. Required before
 * every solve of such a problem (sa_solve returns SA_EARG without it); labels must not
 * decrease from one solve to the next (SA_EARG, the label is not taken). SA_EARG for a problem
 * with decay = SA_DECAY_SOLVES. Host-side bookkeeping only: the factor r^delta is computed on
 * the host when the solution enters the sketch (at the next solve). */
int sa_set_time(sa_problem* p, double tau);

/* Solve A(eta_prev, eta_cur) x = b from the guess selected by the options, then store x in
 * the sketch (Alg. 4). SA_SYNC: waits and fills *info (may be NULL). SA_ASYNC: enqueues only;
 * the report is kept in an on-device log read by sa_read_log. */
int sa_solve(sa_problem* p, sa_solve_info* info, int32_t flags);

/* Reports of the solves enqueued since the last call (oldest first); waits for the stream.
 * At most `max` are copied; *n_out receives the number copied. The log holds 4096 entries. */
int sa_read_log(sa_problem* p, sa_solve_info* out, int32_t max, int32_t* n_out);

/* Copy the last solution (n values) to host or device memory; waits for the stream. */
int sa_get_solution(sa_problem* p, double* x, int32_t mem);

/* Enqueue a copy of the last solution into device memory x (n values) on the problem's
 * stream and return at once (no wait): after an SA_ASYNC solve, x receives that solve's
 * solution once the stream reaches the copy. x must stay valid until then. */
int sa_get_solution_async(sa_problem* p, double* x);

/* y = A(eta_prev, eta_cur) x with the current surfaces (Sec. 3 mixed-stage operator).
 * x, y: n values in `mem` memory. */
int sa_apply_operator(sa_problem* p, const double* x, double* y, int32_t mem);

/* For callers that cannot allocate device memory (code under stream capture, tight serving
 * loops, harnesses that forbid hipMalloc): y = A(eta_prev, eta_cur) x as sa_apply_operator
 * computes it, with no problem object and no allocation. grid, h, eta_prev, eta_cur: host
 * arrays as for sa_create / sa_set_surface (copied); x, y: device arrays of n values; the work
 * is ordered on hip_stream (NULL = the default stream) and the call waits for it. The
 * operator tables, geometry and flags live in a static device array of the library, about
 * 2.1 MB per GPU and held until the process ends, so grids are limited to 32770 columns
 * (SA_EARG beyond, before any device work). Every call on one GPU reuses that array: calls
 * that overlap on one GPU (several host threads or streams) race and must be serialised by
 * the caller. */
int sa_apply_operator_static(const sa_grid* grid, const double* h, const double* eta_prev, const double* eta_cur,
                             const double* x, double* y, void* hip_stream);

/* ---- The mixed-stage operator on a three-dimensional grid -------------------------------
 * Sec. 2.1 writes the sigma-transform for (chi, gamma, sigma) with d = h + eta over the plane
 * and the push-forward grad = (d/dchi + sigma_x d/dsigma, d/dgamma + sigma_y d/dsigma,
 * sigma_z d/dsigma); Sec. 3 couples two stages through grad^(i) . grad^(i-1) with ghost-node
 * Neumann rows. The operator here is that product in composed first-derivative form (seven-point
 * sixth-order stencils), with identity rows on the free surface and on nodes beyond two
 * boundaries, the bed row n . grad^(i-1) p with n = (-h_chi, -h_gamma, -1) on the ghost level,
 * and -+ the chi (gamma) component of grad^(i-1) p on the ghost columns (rows) beyond walls.
 *
 * Grid: nx, ny points in chi and gamma with both ends included (periodic: nx - 1 distinct
 * columns, length_x = period; walls: one ghost column beyond each wall), nz sigma levels from
 * bed to surface plus one ghost level below the bed. Vectors: n = (nz + 1) * nrow * ncol values,
 * node (level j, row r, column c) at (j * nrow + r) * ncol + c, ncol = nx - 1 (periodic) or
 * nx + 2 (walls), likewise nrow. Host plane arrays (h, eta): nyp x nxp values, chi fastest,
 * physical points only (nx - 1 or nx per row). */
typedef struct {
  int32_t nx, ny;     /* points in chi and gamma, both ends included (>= 9 periodic, >= 7 walls) */
  int32_t nz;         /* sigma levels bed..surface, 6 <= nz <= 65                             */
  int32_t bc_x, bc_y; /* SA_PERIODIC | SA_WALLS per direction                                 */
  double length_x, length_y;
} sa_grid3;

typedef struct sa_op3d sa_op3d;

/* Tables and still-water depth (host h, copied) of one grid; device work is ordered on
 * hip_stream (NULL = the default stream). SA_EARG for a bad grid, SA_EGEOM for h <= 0. */
int sa_op3d_create(const sa_grid3* grid, const double* h, void* hip_stream, sa_op3d** out);
/* Surfaces of the previous and the current stage (mem: SA_MEM_HOST, copied, checked at once:
 * SA_EGEOM when h + eta <= 0 or non-finite; SA_MEM_DEVICE: read on the stream, a bad surface
 * is reported by the next host-memory apply or sa_op3d_sync). Forms the geometry of both. */
int sa_op3d_set_surface(sa_op3d* op, const double* eta_prev, const double* eta_cur, int32_t mem);
/* y = A(eta_prev, eta_cur) x. SA_MEM_HOST: staged, waits, reports SA_EGEOM; SA_MEM_DEVICE:
 * x and y are device arrays of n values, the kernel is enqueued and the call returns at once
 * (x must stay alive and y untouched until the stream reaches it). */
int sa_op3d_apply(sa_op3d* op, const double* x, double* y, int32_t mem);
/* Waits for the stream; SA_EGEOM if a device surface was invalid (the surfaces must be set again). */
int sa_op3d_sync(sa_op3d* op);
int64_t sa_op3d_size(const sa_op3d* op);
/* workgroups of one operator launch (tiles of 32 x 8 columns) */
int sa_op3d_workgroups(const sa_op3d* op);
void sa_op3d_destroy(sa_op3d* op);

/* ---- The closed loop (Sec. 3, Alg. 1) ---------------------------------------------------
 * Low-storage Runge-Kutta (LSERK45) stepping of the velocity field (u, w) and the free surface
 * of a periodic problem, whose mixed-stage pressure systems the problem then solves in sequence
 * (with its options: guess, preconditioner, tolerance). Per stage, with rho = 1, no viscosity
 * and gravity g = 9.81: the surface advances by the kinematic condition w - u D_chi eta; the
 * right-hand side is grad^(i) . Q on the PDE rows, n . Q at the bed (n = (-h_chi, -1)) and 0 on
 * the surface, Q = u / (beta_i dtau) + alpha_i K_u / dtau + F - (u . grad^(i-1)) u
 * + (sigma / d^(i-1)) (D_tau eta) D_sigma u. The problem solves for the dynamic pressure
 * p_d = p - p_s, p_s = g d^(i-1) (1 - sigma) (right-hand side rhs - A p_s), as the solver of
 * Sec. 1 does; after the solve u advances by K_u = alpha_i K_u + dtau (Q's force part -
 * grad^(i-1) (p_s + p_d)). Velocities live on every node of the
 * problem's grid (layout as sa_size), eta on its nx - 1 columns. The loop keeps a pointer to p
 * (which must outlive it) and works on p's stream. With decay = SA_DECAY_TIME the loop labels
 * the system of stage i of its n-th step (n from 0, counted since sa_loop_create) with the
 * stage time (n + c_i) dtau of LSERK45 itself. */
typedef struct sa_loop sa_loop;
int sa_loop_create(sa_problem* p, double dtau, sa_loop** out);  /* SA_EARG: p not periodic, dtau <= 0 */
/* eta (nx - 1), u, w (n values each) in `mem` memory; clears the Runge-Kutta registers; waits */
int sa_loop_set_state(sa_loop* L, const double* eta, const double* u, const double* w, int32_t mem);
/* one time step = five stages and five solves, enqueued on the stream without a wait between
 * them; infos (may be NULL) receives the five solve reports; waits for the stream once, at the
 * end. SA_NOCONV if a stage's solve did not converge (the step still runs its five stages: the
 * state is the one after them), negative codes as sa_solve. */
int sa_loop_step(sa_loop* L, sa_solve_info* infos);
int sa_loop_get_state(sa_loop* L, double* eta, double* u, double* w, int32_t mem);
void sa_loop_destroy(sa_loop* L);

/* y = M^-1 x, the fixed still-water preconditioner of the problem. */
int sa_apply_precond(sa_problem* p, const double* x, double* y, int32_t mem);

/* FP32 inner kernels of the refinement path (precision = SA_FP32_IR only, else SA_EARG):
 * y = A x with FP32 input, output and stencil arithmetic (geometry rounded to FP32), and
 * y = M^-1 x with FP32 line-solve factors, work vectors and coarsest inverse. x, y: n floats
 * in `mem` memory (host arrays are staged through the problem's FP32 work vectors). */
int sa_apply_operator_f32(sa_problem* p, const float* x, float* y, int32_t mem);
int sa_apply_precond_f32(sa_problem* p, const float* x, float* y, int32_t mem);

/* The k sketch draws of stored solution `index` (SplitMix64 counter stream + Box-Muller),
 * host only, no device needed: out[a] = omega_a, a < k (k <= 64). */
int sa_sketch_draws(uint64_t seed, int64_t index, int32_t k, double* out);

/* Checkpoint of the solver state that carries from one solve to the next (Alg. 4's sketch Y
 * or Alg. 3's window of solutions and their rows of Omega, the last solution, which the
 * next solve stores in the sketch first, and the counters: stored solutions, which is the
 * position of the sketch's random stream, solves and report-log position). buf == NULL:
 * *len receives the size in bytes. Otherwise buf (host memory, *len bytes) receives the
 * state, waiting for the problem's stream; SA_EARG with *len = the size needed when it is too
 * small. The state is a plain byte image for this library's build (host byte order). */
int sa_save_state(const sa_problem* p, void* buf, size_t* len);

/* Restore a state saved from a problem of the same grid and sketch options (guess mode, k,
 * window, r, seed, precision; SA_EARG otherwise) into p: its next solves compute exactly
 * what the saved problem's next solves would have computed, on any problem created with
 * those arguments (bathymetry and the other options are the caller's to keep equal). */
int sa_load_state(sa_problem* p, const void* buf, size_t len);

/* Copy the sketch Y (n x k, column-major: Y[a * n + i]) to host or device memory. */
int sa_get_sketch(sa_problem* p, double* y, int32_t mem);

/* Number of solutions stored in the sketch so far. */
int64_t sa_sketch_count(const sa_problem* p);

/* Bytes of device memory sa_create would allocate for these arguments (no device needed);
 * validates the arguments like sa_create. */
int sa_problem_footprint(const sa_grid* grid, const double* h, const sa_options* opt, int64_t* bytes);

/* Device time spent in each phase of the solves run so far with opt.profile = 1, in
 * milliseconds of the device's constant-rate clock, measured by the first workgroup:
 * out[0] geometry, [1] sketch guess (block operator, Gram, x0), [2] k x k solve,
 * [3] operator applications, [4] preconditioner, [5] orthogonalisation, [6] other
 * (Givens, updates, checks), [7] total; then the preconditioner in detail: [8] coarsest
 * solve, [9 + 2 l] down pass and [10 + 2 l] up pass of level l (l < 24), [56] the wait of
 * the other workgroups for the single-workgroup coarse tail. n = entries wanted (<= 57). */
int sa_get_phase_times(sa_problem* p, double* out, int32_t n);

/* ---- continuous-batching server ---------------------------------------------------------
 * Many independent simulations (each an sa_problem with its own sketch and hierarchy) on one
 * GPU. Simulations are admitted when their device arena fits the HBM budget (with
 * queue_admission, one that does not fit yet waits and is admitted, oldest first, once closed
 * simulations have freed enough); requests (the surfaces and right-hand side of a
 * simulation's next system) queue per simulation, first in first out; a tick runs the oldest
 * request of as many simulations as fit into one launch, one workgroup cluster per request;
 * up to max_inflight ticks run at once, so requests arriving while a tick runs join the next
 * one. A solve in a tick computes exactly what sa_solve computes for that simulation.
 * Thread safety: every sa_server_* call takes the server's lock, so requests may be submitted
 * and completions polled from different host threads (a waiting poll releases the lock while
 * it waits). Problems returned by sa_server_problem follow the rules of a single problem.
 * Stream ordering: device inputs are read after the work the caller had enqueued on the
 * server's stream (the one given at creation) when it submitted them; the solves themselves
 * run on the server's own streams. */
typedef struct sa_server sa_server;

typedef struct {
  int64_t hbm_budget;             /* device bytes the simulations may hold; 0 = 90% of free */
  int32_t max_inflight;           /* ticks running at once, each on its own stream (1..16),  */
                                  /* default 4 (HIP's default of 4 hardware queues per       */
                                  /* process; more ticks need GPU_MAX_HW_QUEUES raised as    */
                                  /* well, else they share queues and serialise); a tick     */
                                  /* gets capacity / max_inflight                            */
                                  /* workgroups (at least one simulation's cluster)          */
  int32_t max_batch;              /* solves per tick, 0 = as many as are co-resident          */
  int32_t unknowns_per_workgroup; /* cluster size of simulations opened with cluster = 0:    */
                                  /* ceil(n / this), 1..16, default 20000                    */
  int32_t queue_admission;        /* 1: sa_server_open of a simulation over the budget       */
                                  /* returns an id that waits for admission; 0 (default):    */
                                  /* SA_EBUSY                                                */
} sa_server_options;

typedef struct {
  uint64_t ticket;                /* from sa_server_submit                                    */
  int32_t sim;
  int32_t reserved;
  sa_solve_info info;             /* as sa_solve reports it; status < 0 for SA_EGEOM etc.;   */
                                  /* SA_EDEVICE for the requests of a simulation whose solve */
                                  /* timed out on the device, and for those still queued     */
  double t_submit_ms;             /* server clock: ms since sa_server_create                  */
  double t_launch_ms;             /* when its tick was enqueued                               */
  double t_done_ms;               /* when its tick finished on the device                     */
} sa_completion;

void sa_server_default_options(sa_server_options* opt);
int sa_server_create(const sa_server_options* opt, void* hip_stream, sa_server** out);
/* Waits for all work, destroys every open simulation. */
void sa_server_destroy(sa_server* s);
/* Admit a simulation (arguments as sa_create; opt->cluster = 0 picks the cluster size from
 * its size). SA_EBUSY (nothing allocated) when its arena would exceed the HBM budget, unless
 * queue_admission is set: then *sim is valid at once, requests may be submitted, and the
 * simulation is created when it fits (sa_server_admitted). A simulation larger than the whole
 * budget is always refused. Requests carry no time labels: opt->decay must be
 * SA_DECAY_SOLVES (SA_EARG otherwise). */
int sa_server_open(sa_server* s, const sa_grid* grid, const double* h, const sa_options* opt, int32_t* sim);
/* 1: the simulation holds its device arena; 0: waiting for admission; -1: no such simulation
 * (or its admission failed). */
int32_t sa_server_admitted(const sa_server* s, int32_t sim);
/* Free a simulation without queued or running requests (else SA_EBUSY); a simulation that
 * failed on the device can always be closed once its running tick has been harvested. Frees
 * budget for simulations waiting for admission. */
int sa_server_close(sa_server* s, int32_t sim);
/* Queue the next system of `sim`. Host inputs (eta: nphys values each, b: n values) are copied
 * before return; device inputs must stay valid until the request completes. x_out (same
 * memory kind as the inputs, n values, or NULL) receives the solution when the request's
 * completion is harvested. */
int sa_server_submit(sa_server* s, int32_t sim, const double* eta_prev, const double* eta_cur, const double* b,
                     int32_t mem, double* x_out, uint64_t* ticket);
/* Harvest finished ticks, admit waiting simulations, launch new ticks from the queues, return
 * up to `max` completions (oldest tick first). wait_us = 0: no waiting; < 0: wait until at
 * least one completion is available while a tick runs; > 0: wait at most that many
 * microseconds for one. */
int sa_server_poll(sa_server* s, sa_completion* out, int32_t max, int32_t* n_out, int32_t wait_us);
/* Requests queued, running or completed but not yet returned by sa_server_poll. */
int64_t sa_server_outstanding(const sa_server* s);
/* Device bytes held by the admitted simulations. */
int64_t sa_server_bytes_used(const sa_server* s);
/* The server's clock (ms since sa_server_create; the clock of sa_completion's times). */
double sa_server_clock_ms(const sa_server* s);
/* Counters since creation: out[0] ticks launched, [1] solves launched, [2] host ms spent
 * forming and enqueuing ticks, [3] ms from enqueue to completion summed over the ticks,
 * [4] co-resident workgroups of the solve kernels (the capacity ticks share), [5] workgroups
 * per tick (capacity / max_inflight), [6] solves that ended with SA_EDEVICE on the device.
 * Fills the first min(n, 7) entries. */
int sa_server_stats(const sa_server* s, double* out, int32_t n);
/* The problem of an admitted simulation with no request running (for sa_get_solution,
 * sa_read_log; no sa_solve on it); NULL while one of its requests is in a running tick. */
sa_problem* sa_server_problem(sa_server* s, int32_t sim);

/* Failure-handling tests: raise the problem's device abort flag, which every bounded wait of
 * its solve kernel checks, so that its next solve returns at once with SA_EDEVICE (every
 * kernel still exits normally) and the problem becomes unusable. */
int sa_debug_abort(sa_problem* p);

/* Thread-local message of the last hard error ("" if none). */
const char* sa_last_error(void);

/* Library build identification (gfx target, HIP version), static string. */
const char* sa_build_info(void);

#ifdef __cplusplus
}
#endif
#endif /* SAWAVE_H */
