/*
 * dlmpc.h — C ABI of the MI355X DLMPC-ADMM library (libdlmpc.so).
 *
 * The library solves the distributed and localized MPC subproblem of eq. (MPC) in
 * Section II-A of Amo Alonso & Tseng, "Effective GPU Parallelization of Distributed and
 * Localized MPC": minimise sum_t x_t'Q x_t + u_t'R u_t subject to x_{t+1} = A x_t + B u_t,
 * x_0 = x(tau), box bounds on states and inputs, and d-locality over the graph G_(A,B).
 * It uses the SLS parametrisation of the same section (the matrix Phi with N_x*T + N_u*(T-1)
 * rows and N_x columns, sparse by locality) and the ADMM of Algorithm 2: Phi-comp row by
 * row, Psi-comp column by column, the Lambda update and the convergence check, all on one
 * GPU. Algorithm 1 splits the work into an offline precomputation (dlmpc_setup) and a
 * per-MPC-step solve from the measured state x(tau) (dlmpc_solve).
 *
 * Conventions shared by every call:
 *   - Every function returns an int status: 0 = ok, > 0 = soft status with valid outputs,
 *     < 0 = error with outputs untouched. dlmpc_last_error() gives a message for the last
 *     error raised on the calling thread.
 *   - The caller owns every buffer it passes and keeps ownership; the library deep-copies
 *     what it needs during dlmpc_setup. A dlmpc_problem is owned by the library until
 *     dlmpc_destroy.
 *   - A problem is bound to one device and one HIP stream; it is not thread-safe. Calls on
 *     different problems may run concurrently.
 *   - Rows of Phi are in canonical order: state blocks x_0..x_{T-1}, then input blocks
 *     u_0..u_{T-2}; within a block subsystem-major (subsystem i owns nx consecutive state
 *     rows, nu consecutive input rows). Columns are the N_x = n_sub*nx components of x0.
 *   - Phi[r, c] may be nonzero iff hop(sub(r), sub(c)) <= d in G_(A,B) (the locality
 *     pattern of Section II-A; Lemma 1 counts the nodes within d hops).
 */
#ifndef DLMPC_H
#define DLMPC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  DLMPC_OK = 0,
  DLMPC_ENOCONV = 1,              /* max_iter reached: the last iterate is returned */
  DLMPC_EINVAL = -1,              /* bad argument (sizes, NaN/Inf, d < 0, T < 2, NULL) */
  DLMPC_ENOMEM = -2,              /* host or device allocation failed */
  DLMPC_EDEVICE = -3,             /* HIP runtime error, or no device work on a host-only problem */
  DLMPC_EINFEASIBLE_LOCALITY = -4,/* some column cannot meet Z_AB Psi = I inside its d-hop patch */
  DLMPC_ENUMERIC = -5             /* NaN/Inf appeared in the iterate */
};

typedef enum {
  DLMPC_FP64 = 0,     /* state, operators and reductions in double */
  DLMPC_FP32 = 1,     /* state and operators in float; setup and outputs stay double. Batched
                         solves: matrix-core products with both operands split into bf16 hi + lo
                         (three products hi*hi + hi*lo + lo*hi, float accumulation): each operand
                         carries about 16 significant bits (relative error up to ~2^-17 per
                         operand, against 2^-24 for float), so the products are accurate to a few
                         1e-6 relative, not to float rounding. This sets a floor on the dual
                         residual that grows with the size of x0 (measured 3e-5..1e-4 with
                         x0 ~ N(0, I) on the 8x8 grid, far below 1e-4 with x0 ~ 0.15 N(0, I) on the
                         1024-subsystem mesh): eps (times warm_eps_scale for warm starts) must
                         stay above it. */
  DLMPC_FP32_BF16 = 2 /* reduced-operator tier: as DLMPC_FP32, except that the batched solves'
                         basis operands are rounded once to bf16 (two matrix-core products per
                         tile instead of three, half the basis bytes). The rounded basis is not
                         exactly orthonormal: the iterate keeps moving by an amount set by bf16
                         rounding, so the dual residual settles on a floor that depends on the
                         network (4e-4 to 7e-3 on the grids and meshes tested) and eps must lie
                         above it, else the solve runs to max_iter (DLMPC_ENOCONV); u(0) and J
                         then carry an error of the order of eps and of bf16 rounding.
                         Single-instance solves run as DLMPC_FP32. */
} dlmpc_precision;

/* Setup flags (dlmpc_options.flags). */
#define DLMPC_FLAG_HOST_ONLY 0x1u /* build host-side data only; no HIP call is made and every
                                     solve returns DLMPC_EDEVICE. For inspection and tests. */
/* Iteration schedule. Neither flag = time both at setup and keep the faster one. */
#define DLMPC_FLAG_SCHED_GRAPH 0x2u      /* two kernels per iteration, K iterations per captured
                                            HIP graph launch, host polls the stop flag */
#define DLMPC_FLAG_SCHED_PERSISTENT 0x4u /* one launch runs every iteration with grid barriers
                                            between Phi-comp and Psi-comp; the grid is sized to be
                                            co-resident, and a barrier wait that times out fails
                                            the solve with DLMPC_EDEVICE */
#define DLMPC_FLAG_HOST_FACTOR 0x8u /* factor the column blocks with host threads instead of the
                                       device kernels (host-only problems always do) */
#define DLMPC_FLAG_NO_TUNE 0x20u   /* no autotuning at setup: graph schedule (unless the persistent
                                      one is asked for), batched-engine kernel variants at their
                                      defaults (1 instance tile per Phi-comp wave, Psi-comp split at
                                      8x the mean basis cost); the tuning cache is not used */
#define DLMPC_FLAG_NO_CHECK 0x10u  /* skip the FP64 check of the stopping iterate that every solve
                                      otherwise runs (stats kkt, eq_resid, u0_check are then 0) */
/* Per-iteration schedules of single-instance solves, the designs of Section III that this
 * library's graph and persistent schedules improve on (for comparison; same kernels, same
 * iterates, so results equal the graph schedule's). At most one DLMPC_FLAG_SCHED_* flag. */
#define DLMPC_FLAG_SCHED_STEPWISE 0x40u  /* the kernels of an iteration launched one by one, the
                                            row-to-column exchange on the device, the host reads the
                                            stop flag after every iteration (column patches: no CPU
                                            exchange inside the iteration, Section III-D) */
#define DLMPC_FLAG_SCHED_HOST_EXCHANGE 0x80u /* as STEPWISE, and Phi is copied to host memory and back
                                            between Phi-comp and Psi-comp (combined kernels: one
                                            CPU exchange per iteration, Section III-C) */
#define DLMPC_FLAG_STRUCTURED_PSI 0x200u /* single-instance solves: Psi-comp through the input rows of
                                            the null bases and the patch simulation (a null-space
                                            trajectory is fixed by its inputs: N_j = S_j N_u), reading
                                            p nu (T-1) instead of p (nx T + nu (T-1)) basis rows per
                                            column subsystem; same iterates up to rounding; graph or
                                            per-iteration schedules only. Without any schedule flag
                                            (and without DLMPC_FLAG_NO_TUNE) setup times it against
                                            the dense Psi-comp and keeps the faster one */
#define DLMPC_FLAG_SCHED_NAIVE 0x100u    /* as STEPWISE, and every kernel's results are copied to
                                            host memory and back before the next kernel runs (the
                                            naive parallelization of Section III-A) */

/* Networked plant. G_(A,B) is read off the block sparsity of A: subsystems i != j are
 * adjacent iff block A_ij or A_ji is present in the block-CSR with a nonzero entry. Every
 * subsystem has nx states and nu inputs. B is block diagonal (one nx x nu block per
 * subsystem). All arrays are host memory. */
typedef struct {
  int32_t n_sub;            /* N >= 1 */
  int32_t nx, nu;           /* states / inputs per subsystem, >= 1 */
  const int64_t *a_rowptr;  /* [N+1] block-CSR row pointers over subsystems */
  const int32_t *a_colidx;  /* [nnzb] block column indices (any order, no duplicates) */
  const double *a_blocks;   /* [nnzb * nx * nx] row-major nx x nx blocks, CSR order */
  const double *b_blocks;   /* [N * nx * nu] row-major diagonal blocks B_ii */
} dlmpc_system;

/* Diagonal stage cost and box bounds of eq. (MPC). q_diag weights every state row
 * x_0..x_{T-1}; r_diag every input row u_0..u_{T-2}. State bounds apply at t = 1..T-1
 * (x_0 is the measured state), input bounds at t = 0..T-2. A NULL bound array means
 * unbounded; +-INFINITY entries are allowed; each interval must contain 0. */
typedef struct {
  const double *q_diag; /* [N*nx], > 0 */
  const double *r_diag; /* [N*nu], > 0 */
  const double *x_lo, *x_hi; /* [N*nx] or NULL */
  const double *u_lo, *u_hi; /* [N*nu] or NULL */
} dlmpc_cost;

typedef struct {
  double rho;          /* ADMM penalty, > 0 (default 5 when 0 is passed) */
  double eps;          /* convergence tolerance, > 0 (default 1e-4 when 0) */
  int32_t max_iter;    /* > 0 (default 500 when 0) */
  int32_t check_every; /* iterations per captured graph launch between host checks (0 = auto) */
  int32_t precision;   /* dlmpc_precision */
  int32_t device;      /* HIP device ordinal */
  void *stream;        /* hipStream_t to run on, or NULL for a library-owned stream */
  uint32_t flags;      /* DLMPC_FLAG_* */
  int32_t max_batch;   /* 0, or 1..64: also set up the batched engine for up to this many x0
                          per dlmpc_solve_batch call (FP32 or FP32_BF16 precision) */
  int32_t warm_cg_iters; /* CG steps of the trajectory warm start (0: 12) */
  double factor_chol_tol; /* device factorisation: a Cholesky QR pivot of S K below this
                             fraction of the largest diagonal of (S K)'(S K) switches that
                             subsystem to the Householder QR (0: 1e-10; 1 or more: always) */
  double warm_eps_scale; /* batched and streamed solves from a warm start (trajectory, learned,
                            alpha) stop on the eps rule with eps * warm_eps_scale, in (0, 1]
                            (0: 1/2). The eps rule bounds the residuals, not the distance to the
                            optimum: from the learned start the stopping iterate was measured up
                            to 1.7x farther from the exact optimum (u(0)) than the cold start's at
                            the same eps, and no farther at eps/2 (16x16 box grid and 1024-
                            subsystem mesh). Cold runs, including the cold fallback of a
                            warm-started instance, use eps. A warm-started instance that reaches
                            max_iter without meeting eps * warm_eps_scale but whose last iterate
                            meets eps is kept (converged) instead of being solved again. */
} dlmpc_options;

/* Optional warm start (Algorithm 2 initial iterate): Psi^0 and Lambda^0 as values on the
 * canonical CSR pattern of dlmpc_phi_pattern (host arrays of nnz doubles). NULL = cold start
 * Psi^0 = Lambda^0 = 0. */
typedef struct {
  const double *psi0;
  const double *lambda0;
} dlmpc_warm;

typedef struct {
  int32_t iters;        /* ADMM iterations run */
  int32_t converged;    /* 1 iff both residuals <= eps at the stopping iterate */
  double r_primal;      /* max over columns of ||Phi[:,c] - Psi[:,c]||_2 at the stopping iterate */
  double r_dual;        /* max over columns of ||Psi^{k+1}[:,c] - Psi^k[:,c]||_2 */
  double objective;     /* sum_r w_r (Phi x0)_r^2 at the stopping iterate, FP64 */
  double t_solve_ms;    /* host wall time of the solve call; streamed solves: of the instance,
                           from its join to the host check that saw it stop (plus its cold
                           fallback, if any) */
  double t_iter_ms;     /* device time of the iteration phase (HIP events) */
  int32_t graph_launches; /* kernel-graph launches (graph schedule), iterations (per-iteration
                             schedules) or 1 (persistent) */
  int32_t schedule;       /* 0 = graph, 1 = persistent, 2 = batched, 3 = stepwise, 4 = host
                             exchange, 5 = naive */
  int32_t start;          /* initial iterate: one of DLMPC_START_* */
  int32_t fell_back;      /* 1 if the warm-started run did not converge and the instance was
                             solved again from the cold start (iters then counts both runs) */
  double t_warm_ms;       /* device time of the warm-start network inference (learned start) */
  /* FP64 check of the stopping iterate (recomputed on the device in double; skipped with
   * DLMPC_FLAG_NO_CHECK). Single-instance solves: the certificate of dlmpc_certify, with
   * eq_resid = its eq (max |Z_AB Psi - I|) and kkt = the largest of its rp, box and stat and of
   * r_dual. Batched and streamed solves (compact state): the trajectory y = Phi x0 of the
   * stopping iterate is recomputed in FP64 from the instance's state with the FP64 null bases and
   * offsets; eq_resid = max |Z_AB y - [x0; 0; ...]| (initial state and dynamics of the returned
   * trajectory), u0_check = max |u(0) returned - u(0) of that y| (the rounding of the reduced-
   * precision iteration in u(0)), kkt = the largest of eq_resid, the bound violation of y,
   * r_primal and r_dual. */
  double kkt;
  double eq_resid;
  double u0_check;
  double t_precompute_ms; /* device time of the per-solve precompute (Algorithm 1, with x0) */
  double t_check_ms;      /* device time of the FP64 check (per instance share for streams) */
  int32_t inner_iters;    /* nested-ADMM iterations over the solve (couplings, dlmpc_set_coupling) */
  int32_t pad;
  double coupling_viol;   /* largest violation of a coupling by Phi x0 at the stopping iterate */
} dlmpc_stats;

typedef struct {
  int64_t R;            /* rows of Phi: N*nx*T + N*nu*(T-1) */
  int64_t n_cols;       /* N*nx */
  int64_t nnz;          /* entries of the locality pattern */
  int64_t n_tiles;      /* (column subsystem, row subsystem) pairs within d hops */
  int32_t d_row_max;    /* longest row of the pattern (Section III-B, D_row) */
  int32_t d_col_max;    /* longest column (D_col) */
  int32_t p_max;        /* largest d-hop patch, in subsystems */
  int32_t k_max;        /* largest null-space dimension of a column block */
  int64_t sum_dcol_k;   /* sum over subsystems of D_col(j) * k_j (entries of the null bases) */
  int64_t sum_dcol2;    /* sum over subsystems of D_col(j)^2 */
  double setup_ms;      /* wall time of dlmpc_setup up to the factorisation's end */
  double factor_ms;     /* of which the FP64 factorisation of the column blocks (device
                           factorisation: list building, transfers and both kernels) */
  int32_t schedule;     /* 0 = graph, 1 = persistent, 3..5 as dlmpc_stats.schedule */
  int32_t persistent_grid; /* co-resident blocks of the persistent schedule (0 = unavailable) */
  double tune_graph_us;      /* per-iteration time measured at setup (0 if not measured) */
  double tune_persistent_us;
  int64_t sum_k;        /* sum over subsystems of k_j (null-space coordinates per instance) */
  int32_t factor_device; /* 1 if the column blocks were factored on the device, 0 on the host */
  int32_t factor_fallbacks; /* device factorisation: subsystems whose null basis came from the
                               Householder QR because Cholesky QR of S K met a tiny pivot */
  /* Autotuner (dlmpc_setup). The single-instance schedule (graph or persistent, both timed over 32
   * iterations) and the batched engine's kernel variants are chosen by timing at setup, or taken
   * from the cache file named by the environment variable DLMPC_TUNE_CACHE (one line per problem
   * signature: sizes, precision, max_batch and the device's architecture; appended after a timed
   * setup). Batched variants: instance tiles per Phi-comp wave (1: each basis fragment feeds one
   * 16-instance tile; 2: two, with half the waves loading it), and the split of heavy column blocks
   * over several Psi-comp work units (the waves serving one patch): a block whose basis cost
   * exceeds batch_psi_capx times the mean is split. */
  int32_t batch_phi_ntw;    /* 1 or 2 (0 without a batched engine) */
  int32_t batch_psi_capx;   /* 2, 4, 8, 16 or 1048576 (no split); 0: the structured Psi-comp (input
                               rows of the null bases and the patch's adjoint recursion per
                               instance, one unit per column subsystem; split operands only) */
  int32_t batch_psi_units;  /* Psi-comp work units (blocks per launch) */
  int32_t tune_cached;      /* 1 if the choices came from the cache */
  double tune_phi_us[2];    /* per-launch us of the Phi-comp variants 1, 2 (0 if not timed) */
  double tune_psi_us[6];    /* per-launch us of the Psi-comp splits 2, 4, 8, 16, none, and of the
                               structured Psi-comp (batch_psi_capx = 0; 0 us when not available) */
  /* Single-instance Psi-comp: 1 if the structured one (DLMPC_FLAG_STRUCTURED_PSI) runs, chosen
   * by the flag, or by timing at setup when no schedule flag is given (tune_structured_us: its
   * per-iteration time on the graph schedule, 0 if not timed). */
  int32_t psi_structured;
  int32_t pad_info;
  double tune_structured_us;
  int64_t sum_du_k;     /* sum over subsystems of mu_j * k_j, mu_j = p_j * nu * (T - 1) the input
                           rows of column block j (entries of the structured Psi-comp's bases N_u) */
} dlmpc_info;

/* Offline precomputation (Algorithm 1, first step). Builds G_(A,B), the d-hop patches, the
 * locality pattern, and for every subsystem j the FP64 factorisation of its column block of
 * Z_AB (the SLS achievability operator: Phi_x[0] = I, Phi_x[t] = A Phi_x[t-1] + B Phi_u[t-1])
 * restricted to the support of j's columns: an orthonormal basis N_j of its null space and
 * the minimum-norm offsets o_c solving the block's equations for each column c of j, so that
 * the Psi-comp projection is psi = N_j N_j' v + o_c. The factorisation runs as two HIP kernels
 * on opts->device (one workgroup per subsystem: pivoted Householder QR of the map from patch
 * inputs to ring values, then Cholesky QR, applied twice, of the simulated null-space
 * trajectories, with a Householder QR instead when a Cholesky pivot is tiny) unless the problem
 * is host-only or DLMPC_FLAG_HOST_FACTOR is set; both give the same N_j N_j' and o_c up to
 * rounding. Uploads the operators and allocates all solve-time device memory. d >= 0, T >= 2.
 * Returns DLMPC_EINFEASIBLE_LOCALITY when some column has no localised trajectory,
 * DLMPC_ENUMERIC when a null basis loses rank, DLMPC_EINVAL when a column block is longer
 * than 8000 rows for the device factorisation. On success *out receives the handle. */
int dlmpc_setup(const dlmpc_system *sys, int32_t d, int32_t T, const dlmpc_cost *cost,
                const dlmpc_options *opts, struct dlmpc_problem **out);

/* Sizes of the problem (fills *info). */
int dlmpc_query(const struct dlmpc_problem *p, dlmpc_info *info);

/* Canonical CSR pattern of Phi: row_ptr [R+1], col_idx [nnz] (ascending within a row). */
int dlmpc_phi_pattern(const struct dlmpc_problem *p, int64_t *row_ptr, int32_t *col_idx);

/* Host FP64 setup products of subsystem j (for inspection and tests): rows [D] are the
 * canonical Phi rows of the support of j's columns in the library's order, P [D*D] the
 * row-major projector N_j N_j' onto the null space of the column block, O [D*nx] row-major
 * offsets (column c = o_c). Any output may be NULL. *D_out receives D_col(j). */
int dlmpc_column_block(const struct dlmpc_problem *p, int32_t j, int32_t *D_out,
                       int64_t *rows, double *P, double *O);

/* Per-step solve (Algorithm 1 loop body: precompute with x0, ADMM of Algorithm 2, read
 * u(0) from Phi). x0 [N*nx] host. Outputs (host, may be NULL): u0 [N*nu] = the u_0 block of
 * Phi x0 at the stopping iterate; phi [nnz] = Phi values on the canonical CSR pattern.
 * Returns DLMPC_OK, or DLMPC_ENOCONV with outputs from the last iterate. */
int dlmpc_solve(struct dlmpc_problem *p, const double *x0, const dlmpc_warm *warm, double *u0,
                double *phi, dlmpc_stats *stats);

/* Same as dlmpc_solve with device buffers on the problem's device: x0_dev [N*nx] double in,
 * u0_dev [N*nu] double out, phi_dev [nnz] double out or NULL. Cold start. The call returns
 * after the outputs are written (the problem's stream is synchronised). */
int dlmpc_solve_device(struct dlmpc_problem *p, const double *x0_dev, double *u0_dev,
                       double *phi_dev, dlmpc_stats *stats);

/* FP64 certificate of the stopping iterate of the latest single-instance solve on this problem
 * (dlmpc_solve or dlmpc_solve_device), recomputed on the device from the stored Phi, Psi, Lambda
 * (promoted to FP64 in the FP32 tier) and x0. x0_dev: that solve's x0 on the device [N*nx], or
 * NULL for the x0 of the latest dlmpc_solve (host entry). Fields (all >= 0): */
typedef struct {
  double eq;    /* max |Z_AB Psi - I| over the support and the (d+1)-hop ring of every column */
  double pf;    /* max |Phi - Psi| */
  double rp;    /* max over columns of ||Phi[:,c] - Psi[:,c]||_2 (the primal residual of Conv) */
  double box;   /* largest bound violation of Phi x0 (0 when within the boxes) */
  double stat;  /* max over columns of |N_j N_j' rho Lambda[:,c]| (Psi-step stationarity) */
} dlmpc_cert;
int dlmpc_certify(struct dlmpc_problem *p, const double *x0_dev, dlmpc_cert *out);

/* Kernel timing for roofline measurement: runs `iters` ADMM iterations of the graph schedule
 * from x0_dev without early stop, each kernel launched on its own between HIP events on the
 * problem's stream, and writes the mean device time per launch in microseconds of each of
 * the DLMPC_TIMED_KERNELS kernels of one iteration, in this order: Phi-comp (phi_kernel),
 * Psi-comp pass 1 (psi_pass1_kernel: t = N_j' v), Psi-comp pass 2 with Lambda-comp and the
 * residual partial sums (psi_pass2_kernel), Conv (conv_kernel). us_per_launch has
 * DLMPC_TIMED_KERNELS entries. The iterate is left in an unspecified state. */
#define DLMPC_TIMED_KERNELS 4
int dlmpc_time_kernels(struct dlmpc_problem *p, const double *x0_dev, int32_t iters,
                       double *us_per_launch);

/* Kernel timing of the batched engine for roofline measurement: B instances from x0_dev
 * [B][N*nx] (device), started from row multipliers alpha0 = 0 (DLMPC_START_ALPHA, so that
 * every iteration runs the full products) without early stop; `iters` iterations with each
 * kernel launched on its own between HIP events on the problem's stream.
 * us_per_launch gets the mean device time per launch of, in this order, the batched Phi-comp
 * (bphi_kernel: row solves of all instances, products with the null bases on the matrix
 * cores), the batched Psi-comp with Lambda and Conv terms (bpsi_kernel) and the per-instance
 * stopping decision (bdecide_kernel). The batched state is left unspecified. */
#define DLMPC_BATCH_TIMED_KERNELS 3
int dlmpc_time_batch_kernels(struct dlmpc_problem *p, int32_t B, const double *x0_dev,
                             int32_t iters, double *us_per_launch);

/* Batched per-step solve: B in 1..max_batch independent MPC instances on this network (distinct
 * x0, same plant, cost and bounds), iterated together. Each instance follows the iteration of
 * Algorithm 2 from the cold start and stops at its own convergence (or max_iter); stopped
 * instances are frozen while the others continue. The iteration is run in an exact compact
 * form (per instance: the Phi-comp row scalars and the null-space coordinates of the Psi and
 * Lambda columns), and both products of an iteration run on the matrix cores (bf16 hi/lo split
 * operands, three products, FP32 accumulation). x0 [B][N*nx], u0 [B][N*nu] row-major (host for
 * dlmpc_solve_batch, device for dlmpc_solve_batch_device); stats [B] or NULL. Returns
 * DLMPC_OK when every instance converged, DLMPC_ENOCONV otherwise (per-instance stats). */
int dlmpc_solve_batch(struct dlmpc_problem *p, int32_t B, const double *x0, double *u0,
                      dlmpc_stats *stats);
int dlmpc_solve_batch_device(struct dlmpc_problem *p, int32_t B, const double *x0_dev, double *u0_dev,
                             dlmpc_stats *stats);

/* Initial iterate of a batched solve (dlmpc_solve_batch_ex). */
#define DLMPC_START_COLD 0       /* Psi^0 = Lambda^0 = 0 (Algorithm 2 as printed) */
#define DLMPC_START_ALPHA 1      /* compact start from given row multipliers */
#define DLMPC_START_TRAJECTORY 2 /* start from a given input trajectory */
#define DLMPC_START_LEARNED 3    /* input trajectory predicted by the warm-start network */
#define DLMPC_START_STATE 4      /* (dlmpc_solve) Psi^0, Lambda^0 given in canonical CSR order */

/* Batched solve with a choice of initial iterate (the better initial point that Section V lists
 * as future work). Device buffers on the problem's device: x0_dev [B][N*nx], u0_dev [B][N*nu].
 * Vectors over the R = N*rs rows of Phi (rs = nx*T + nu*(T-1)) are [B][R] in the library's
 * subsystem-major order: row l of subsystem g is entry g*rs + l, rows x_0..x_{T-1} (nx each)
 * then u_0..u_{T-2} (nu each).
 *  - DLMPC_START_ALPHA: start_dev = alpha0 [B][R]; Psi^0[:,c] = o_c and
 *    Lambda^0[:,c] = x0_c (I - N_j N_j') alpha0 on the support of column c (j = its subsystem).
 *  - DLMPC_START_TRAJECTORY: start_dev = y0 [B][R], of which only the input rows are read.
 *    The state rows are simulated from x0 (y = x0, A y + B u, ...), then warm_cg_iters
 *    conjugate-gradient steps from zero on M beta = y - b with M = sum_j ||x0_j||^2 N_j N_j'
 *    (lifted from j's support) and b = sum_c x0_c o_c give Psi^0[:,c] = o_c + x0_c N_j N_j' beta
 *    (feasible and local, trajectory close to y), and alpha = -2 w y / rho gives
 *    Lambda^0[:,c] = x0_c (I - N_j N_j') alpha.
 *  - DLMPC_START_LEARNED: as TRAJECTORY with the input rows predicted by the problem's
 *    warm-start network (dlmpc_ws_init / dlmpc_warmstart_load); start_dev is ignored.
 * Every start is a valid initial point of Algorithm 2 and each instance stops on the same eps
 * rule. Any warm-started instance that does not converge within max_iter (or meets a NaN/Inf)
 * is solved again from the cold start (stats fell_back = 1, iters counts both runs).
 * y_out_dev [B][R] (or NULL) receives each instance's trajectory Phi x0 at its stopping iterate
 * (training targets of the warm-start network), alpha_out_dev [B][R] (or NULL) its Phi-comp row
 * multipliers. Returns as dlmpc_solve_batch; stats t_warm_ms is the device time of the start
 * construction (network inference, simulation, CG). */
int dlmpc_solve_batch_ex(struct dlmpc_problem *p, int32_t B, const double *x0_dev, double *u0_dev,
                         int32_t start, const double *start_dev, double *y_out_dev,
                         double *alpha_out_dev, dlmpc_stats *stats);

/* Modes of dlmpc_closed_loop (bit flags). */
#define DLMPC_CL_SHIFT 1     /* steps t >= 1 start from the previous step's inputs, shifted */
#define DLMPC_CL_SCALE_RHO 2 /* step t runs with rho * ||x(t)||^2 / ||x(0)||^2 */

/* Closed-loop MPC (Algorithm 1) for B in 1..max_batch independent loops on this network: at
 * every step t = 0..T_sim-1 each loop measures its state x(t), solves the MPC subproblem from it
 * (a batched solve, as dlmpc_solve_batch_ex), applies u(t) = the u_0 block of Phi x(t) and moves
 * to x(t+1) = A x(t) + B u(t), all on the device (FP64 plant step). mode is 0 or a combination
 * of:
 *  - DLMPC_CL_SHIFT: steps t >= 1 start from the previous step's input trajectory moved one
 *    step ahead (u_1..u_{T-2} become u_0..u_{T-3}, the last input held), as
 *    DLMPC_START_TRAJECTORY, with the cold fallback of a warm-started instance; otherwise every
 *    step starts cold.
 *  - DLMPC_CL_SCALE_RHO: the ADMM penalty of step t is rho * max(||x(t)||^2 / ||x(0)||^2, 1e-20)
 *    (rho when x(0) = 0). Scaling x(t) by s scales the Phi-step's cost by s^2, so ADMM from x(t)
 *    with penalty rho s^2 runs the same Phi iterates as ADMM from x(t)/s with rho and bounds
 *    divided by s: the iteration count no longer grows as the loop drives x(t) to 0 (with a
 *    fixed rho the cost's weight relative to the penalty shrinks as ||x(t)||^2). The eps test
 *    is on Phi, whose scale does not depend on x(t).
 * Device buffers: x0_dev [B][N*nx] (x(0)); xs_dev [B][T_sim+1][N*nx] receives x(0)..x(T_sim) of
 * each loop, us_dev [B][T_sim][N*nu] u(0)..u(T_sim-1). stats (or NULL): [T_sim][B], step-major,
 * each the step's batched-solve stats. Returns DLMPC_OK when every step of every loop
 * converged, DLMPC_ENOCONV otherwise (the loop continues with the last iterate's u(t)), a
 * negative status on error (DLMPC_EINVAL for an unknown mode bit or a NaN/Inf in x0). */
int dlmpc_closed_loop(struct dlmpc_problem *p, int32_t B, int32_t T_sim, const double *x0_dev, double *xs_dev,
                      double *us_dev, int32_t mode, dlmpc_stats *stats);

/* Penalty rho of the ADMM of Algorithm 2 (the (rho/2) ||Phi - Psi + Lambda||^2 term) for every
 * solve started after this call, in every entry point (options.rho until the first call; the
 * closed loop's DLMPC_CL_SCALE_RHO factors multiply it). The paper does not fix rho; a caller
 * that runs its own receding-horizon loop can pass rho * ||x(t)||^2 / ||x(0)||^2 here, which
 * gives the iterates of dlmpc_closed_loop with DLMPC_CL_SCALE_RHO. Returns DLMPC_EINVAL unless
 * rho is finite and > 0. */
int dlmpc_set_rho(struct dlmpc_problem *p, double rho);

/* Neighbour-coupled constraints for the single-instance solves (dlmpc_solve, dlmpc_solve_device):
 * lo_e <= y[row_a_e] - y[row_b_e] <= hi_e for e < n, y = Phi x0 in the canonical row order (x_t
 * blocks t = 0..T-1, then u_t blocks; rows of x_0 are fixed by x(0) and not allowed). Such
 * constraints (e.g. the angle difference of a line between neighbouring nodes of the swing
 * network) couple the rows of different subsystems, so Phi-comp (Algorithm 2) is no longer one
 * clip per row: its problem in y is min sum_r c_r (y_r - m_r)^2 over the row boxes and the pairs
 * (c_r = w_r + rho / (2 ||x_r||^2), m_r the uncoupled row value), solved inside every outer
 * iteration by a nested ADMM with penalty sigma between the coupled rows (per row a clipped 1-D
 * solve over its own pairs' copies; per pair a projection onto its slab; scaled duals), at most
 * inner_max iterations, stopping when the copies agree with y and stopped moving to inner_eps,
 * warm-started from the previous outer iteration (zero at the start of a solve). The rows of
 * Phi then follow y as in the uncoupled Phi-comp. n = 0 removes the couplings. The persistent
 * schedule does not take couplings: a problem on it moves to the graph schedule; batched,
 * streamed, group and closed-loop entries return DLMPC_EINVAL while couplings are set. The
 * iteration graphs are captured again (synchronises). Stats report inner_iters and the largest
 * coupling violation of the returned trajectory. Returns DLMPC_EINVAL for a row out of range or
 * in x_0, row_a == row_b, lo > hi or NaN bounds, sigma <= 0, inner_max < 1 or inner_eps < 0. */
int dlmpc_set_coupling(struct dlmpc_problem *p, int32_t n, const int64_t *row_a, const int64_t *row_b,
                       const double *lo, const double *hi, double sigma, int32_t inner_max, double inner_eps);

/* Counters of a streamed solve (dlmpc_solve_stream). */
typedef struct {
  int32_t joins;               /* times new instances entered free slots (the first fill included) */
  int32_t checks;              /* host checks of the per-instance stop flags */
  int64_t slot_iterations;     /* iterations launched times slots in use */
  int64_t instance_iterations; /* sum over instances of their warm-started iterations */
  int32_t fell_back;           /* instances re-solved from the cold start */
  int32_t pad;
  double t_stream_ms;          /* device time from the first fill to the last stop */
} dlmpc_stream_info;

/* n independent instances of this network (any n >= 1) streamed through the batched engine's
 * max_batch slots, each from the learned start (needs the warm-start network): every
 * check_iters iterations (0: 12) the host reads the per-instance stop flags, writes u(0) of the
 * instances that stopped to their rows of u0_dev, copies their stopping state aside for the FP64
 * check (run once that copy holds max_batch instances, and at the end), and once at least
 * refill_min slots are free (0: a tenth of the slots, at least one; or the last instances are
 * waiting; or no slot is busy) starts the next instances in them: network inference and simulation at once, then the CG steps and the start
 * projections of their trajectory start inside the following iterations, in the joiners'
 * columns of the same basis products (no pass over the bases of their own), after which each
 * joiner iterates with its own iteration count. Per instance the arithmetic is that of
 * dlmpc_solve_batch_ex with the learned start (same start, same iterates, same stopping rule),
 * whatever slot and moment it joins; instances that end unconverged are solved again from the
 * cold start. x0_dev [n][N*nx], u0_dev [n][N*nu] device buffers; stats [n] and info may be NULL.
 * Returns DLMPC_OK, or DLMPC_ENOCONV if some instance did not converge even from the cold
 * start. */
int dlmpc_solve_stream(struct dlmpc_problem *p, int32_t n, const double *x0_dev, double *u0_dev,
                       int32_t refill_min, int32_t check_iters, dlmpc_stats *stats,
                       dlmpc_stream_info *info);

/* dlmpc_solve_stream without any device allocation, for callers that cannot allocate device
 * memory during a call (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the staging of the joining instances' predicted trajectories lives in a static
 * device array of the library (16 MiB, 4194304 floats, one copy per GPU, held until the process
 * ends) instead of a buffer that dlmpc_solve_stream allocates on its first call. The call needs
 * max_batch * N * (nx*T + nu*(T-1)) <= 4194304 (the 1024-subsystem mesh with T = 15 and 64 slots
 * takes 2883584) and otherwise returns DLMPC_EINVAL before any device work. Every other buffer
 * it uses belongs to the problem (allocated by dlmpc_setup / dlmpc_ws_init). Arguments, results
 * and statuses as dlmpc_solve_stream, with identical results. Calls on one GPU share that GPU's
 * array: calls that overlap in time on one GPU (from different threads, or on different
 * problems' streams) race on it and must be serialised by the caller. */
int dlmpc_solve_stream_noalloc(struct dlmpc_problem *p, int32_t n, const double *x0_dev, double *u0_dev,
                               int32_t refill_min, int32_t check_iters, dlmpc_stats *stats,
                               dlmpc_stream_info *info);

/* ---- Learned warm start: one network per subsystem g (separate FP32 weights), input the x0
 * entries of the subsystems within d hops of g (ascending subsystem order, each nx entries,
 * zero-padded to IN = p_max*nx) divided by x_scale; two GELU hidden layers of width `hidden`;
 * the output layer sees [h2, x]; output = g's input rows u_0..u_{T-2} (OUT = nu*(T-1) values)
 * divided by y_scale. Parameter layout (flat FP32, this order, row-major): W1 [N][IN][H],
 * b1 [N][H], W2 [N][H][H], b2 [N][H], W3 [N][H+IN][OUT], b3 [N][OUT]. Training minimises the
 * mean squared error over subsystems, samples and outputs (in units of y_scale) with Adam
 * (beta1 0.9, beta2 0.999, eps 1e-8); all products run on the matrix cores (bf16 hi/lo split
 * operands, FP32 accumulation). Trajectories are [S][R] as for dlmpc_solve_batch_ex. Needs a
 * device problem. */

/* Create (or re-create) the network with seeded initial weights. max_samples bounds S below. */
int dlmpc_ws_init(struct dlmpc_problem *p, int32_t hidden, int32_t max_samples, uint64_t seed,
                  double x_scale, double y_scale);
/* Sizes: IN, hidden, OUT and the parameter count (any pointer may be NULL). */
int dlmpc_ws_shape(const struct dlmpc_problem *p, int32_t *in, int32_t *hidden, int32_t *out,
                   int64_t *n_params);
/* Copy the parameters to host get [n_params] (if non-NULL), then from host set (if non-NULL). */
int dlmpc_ws_params(struct dlmpc_problem *p, float *get, const float *set);
/* Loss (mean squared error in scaled units) and its gradient for S samples: x0_dev [S][N*nx],
 * y_dev [S][R] target trajectories (input rows read; device). grad [n_params] host or NULL.
 * Weights unchanged. */
int dlmpc_ws_loss_grad(struct dlmpc_problem *p, int32_t S, const double *x0_dev,
                       const double *y_dev, double *loss, float *grad);
/* One Adam step on S samples (loss before the step returned in *loss if non-NULL). */
int dlmpc_ws_train_step(struct dlmpc_problem *p, int32_t S, const double *x0_dev,
                        const double *y_dev, double lr, double *loss);
/* Predicted input rows written into y_dev [S][R] (device; other rows untouched) for
 * S <= max_samples inputs. */
int dlmpc_ws_predict(struct dlmpc_problem *p, int32_t S, const double *x0_dev, double *y_dev);
/* Weights file: int32 {tag, N, IN, hidden, OUT, version}, double {x_scale, y_scale}, FP32
 * parameters. Load creates the network if needed (max_samples = max_batch, at least 1) and
 * fails with DLMPC_EINVAL if the shape does not match this problem. */
int dlmpc_ws_save(struct dlmpc_problem *p, const char *path);
int dlmpc_warmstart_load(struct dlmpc_problem *p, const char *path);

/* ---- Groups: instances of several networks in one launch per iteration chunk.
 * A group holds batched problems (each set up with max_batch > 0, all on one device); creation
 * captures, for chunks of 1, 2, 4, ..., 32 iterations, one graph in which every member's batched
 * iteration is an independent branch. dlmpc_group_solve_batch runs B[i] instances of member i
 * (x0_dev[i] [B[i]][N_i*nx], u0_dev[i] [B[i]][N_i*nu], device; stats[i] [B[i]] or NULL) from the
 * cold start with each member's own rho, eps and max_iter; every instance stops at its own
 * convergence, and the launches continue until all members have stopped. Per-instance results
 * equal those of dlmpc_solve_batch_device on the member alone. A member must not be used by
 * another call while a group call runs; destroy the group before its members. Returns as
 * dlmpc_solve_batch over all instances. */
struct dlmpc_group;
int dlmpc_group_create(struct dlmpc_problem *const *probs, int32_t n, struct dlmpc_group **out);
int dlmpc_group_solve_batch(struct dlmpc_group *g, const int32_t *B, const double *const *x0_dev,
                            double *const *u0_dev, dlmpc_stats *const *stats);
void dlmpc_group_destroy(struct dlmpc_group *g);

void dlmpc_destroy(struct dlmpc_problem *p);
const char *dlmpc_status_string(int status);
const char *dlmpc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DLMPC_H */
