// Device-side data of libdlmpc: the control block, kernel arguments and the engine interface
// the C ABI drives. Host code sees only the Engine interface.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <string>

#include "dlmpc_internal.h"

namespace dlmpc {

// Convergence/stop state of one solve, written by the last Psi-comp workgroup of every
// iteration (see psi_kernel) and polled by the host every K iterations.
struct Ctl {
  int32_t iters;
  int32_t stop;
  int32_t converged;
  int32_t numeric;
  int32_t max_iter;
  uint32_t done_count;
  int32_t pad0, pad1;
  unsigned long long rp_bits;  // max over columns of the primal residual, as ordered bits
  unsigned long long rd_bits;  // same for the dual residual
  double last_rp, last_rd;
  double eps;
  double objective;
  // persistent schedule: grid barrier and per-iteration residual slots (ping-pong)
  unsigned bar_count, bar_gen, bar_fail, pad2;
  unsigned long long slot_rp[2], slot_rd[2];
  // batched engine: instances of the current solve and its start (kernels captured in graphs
  // read these here, not from their launch arguments)
  int32_t batch, warm;
  int32_t cg_k, pad3;  // CG steps of the streamed joins' trajectory start
  double rho;          // single-instance engine: the penalty of the current solve
  int32_t inner_iters;  // single-instance engine: nested-ADMM iterations of the solve (couplings)
  int32_t pad4;
};

// Static work lists of the persistent schedule: block b runs Phi-comp for
// phi_list[phi_ptr[b] .. phi_ptr[b+1]) and Psi-comp for psi_list[psi_ptr[b] .. psi_ptr[b+1]).
struct Sched {
  const int32_t *phi_ptr, *phi_list, *psi_ptr, *psi_list;
};

// Work units of the split Psi-comp (graph schedule); p1/p2 hold (j, start) pairs.
template <typename Tf>
struct PsiUnits {
  const int32_t *p1;        // [2*n1] (column subsystem, first basis vector)
  const int32_t *p2;        // [2*n2] (column subsystem, first row)
  const int32_t *p2_first;  // [N] first pass-2 unit of each column subsystem
  const int32_t *p2_count;  // [N] number of its pass-2 units (consecutive)
  const int64_t *t_off;     // [N+1] offset of t_j (NX*k_j values)
  Tf *t;                    // N_j' v for every j
  double *part;             // [N][max_units][2*NX] residual partial sums, slot = first row / RB
  int32_t max_units;        // most pass-2 units of any column subsystem
};

template <typename Tf>
struct KArgs {
  int32_t N, nx, nu, T, rs, ts;
  const int64_t *tile_off;  // [N+1]
  const int64_t *rt_ptr;    // [N+1]
  const int64_t *rt_tile;   // [n_tiles]
  const int32_t *rt_col;    // [n_tiles]
  const int32_t *kdim;      // [N]
  const int64_t *nb_off;    // [N+1]
  const int64_t *off_ptr;   // [N+1]
  const int32_t *phi_order; // [N] launch order of the Phi-comp blocks
  const int32_t *psi_order; // [N] launch order of the Psi-comp blocks
  const Tf *nb;             // null bases, column-major per subsystem, padded leading dim
  const Tf *off;            // offsets o_c, column-major per subsystem, padded leading dim
  const Tf *w, *lb, *ub;    // [N*rs] row data, local order
  Tf *phi, *psi, *lam;      // [n_tiles * ts] packed iterates
  Tf *x0f;                  // [N*nx]
  Tf *nrm;                  // [N] ||x_r||^2 per row subsystem
  Tf *y;                    // [N*rs] (Phi x0)_r of the latest Phi-comp
  Ctl *ctl;
  // Neighbour-coupled constraints (NULL cp_slot: none): coupled-row index of each row (-1 if
  // uncoupled), and per coupled row the Phi-comp's a = v . x_r and its uncoupled row value
  int32_t *cp_slot;
  Tf *cp_a, *cp_s0;
};

// Structured Psi-comp (single-instance engine). A null-space trajectory of column subsystem j is
// fixed by its input rows: x_0 = 0 and x_t = A_PP x_{t-1} + B_P u_{t-1} inside the patch, so
// N_j = S_j N_u with N_u the input rows of N_j and S_j the patch simulation. N_j' v = N_u' (v_u +
// S_x' v_x) by an adjoint recursion, N_j t = [simulate(N_u t); N_u t]: the products read N_u
// (p nu (T-1) rows) instead of N_j (p (nx T + nu (T-1)) rows).
template <typename Tf>
struct SimArgs {
  const int64_t *nbu_off;  // [N+1] N_u of j at nbu + nbu_off[j], column-major, leading dim round4(mu_j)
  const Tf *nbu;
  const int64_t *rp0;      // [N] first row pointer of j's patch dynamics (p nx + 1 entries each)
  const int32_t *rp, *rpt; // row pointers of A_PP and of its transpose (local to j's entries)
  const int64_t *e0;       // [N] first entry of j's A_PP (and of its transpose)
  const int32_t *col, *colt;  // patch-state columns (local: member position * nx + state)
  const Tf *val, *valt;
  const Tf *bblk;          // [N][nx][nu] input blocks
  const int32_t *tile_sub; // [n_tiles] row subsystem of each tile
  const int64_t *goff;     // [N] the adjoint result g of j at g + goff[j], [nx][round4(mu_j)]
  Tf *g;
};

// Nested ADMM of the coupled Phi-step (single-instance engine): K coupled rows (library row
// index and subsystem), E pairs lo_e <= y[ka_e] - y[kb_e] <= hi_e, the pairs of every coupled
// row (CSR, entries 2 e + side), the pair copies and scaled duals, and the inner y.
template <typename Tf>
struct CoupleArgs {
  int32_t K, E, inner_max;
  double sigma, inner_eps;
  const int64_t *row;
  const int32_t *sub, *ka, *kb, *kp_ptr, *kp_ent;
  const double *lo, *hi;
  Tf *za, *zb, *la, *lb, *y;
};

class Engine {
 public:
  virtual ~Engine() = default;
  virtual int init(const HostSetup &hs, double rho, hipStream_t s, std::string &err) = 0;
  // Enqueue the per-solve precompute (cold start when wpsi == nullptr) on the stream; rho is
  // the penalty of this solve (kernels read it from the control block).
  virtual int precompute(const double *x0_dev, const double *wpsi, const double *wlam,
                         int max_iter, double eps, double rho, std::string &err) = 0;
  // Enqueue one ADMM iteration of the graph schedule (capturable), or one of its kernels
  // (0 Phi-comp, 1 Psi pass 1, 2 Psi pass 2, 3 Conv).
  virtual int iteration(std::string &err) = 0;
  virtual int launch_one(int which, std::string &err) = 0;
  // Enqueue all iterations of one solve as one launch (persistent schedule).
  virtual int run_persistent(bool tune, std::string &err) = 0;
  virtual int persistent_grid() const = 0;  // 0 when the device cannot co-schedule the grid
  virtual int output(double *u0_dev, std::string &err) = 0;
  virtual int export_phi(double *phi_dev, std::string &err) = 0;
  // Exchange through host memory (the schedules that hand the results of one step to the next
  // through the host): the arrays kernel `which` of an iteration wrote (0 Phi, 1 the pass-1
  // products, 2 Psi and Lambda, 3 the control block) are copied into the pinned buffer `host`
  // (exchange_bytes() bytes), the stream is synchronised, and they are copied back.
  virtual size_t exchange_bytes() const = 0;
  // Phi x0 of the latest Phi-comp (library row order), on the host. Synchronises.
  virtual int copy_y(std::vector<double> &out, std::string &err) = 0;
  // Structured Psi-comp (SimArgs) for the following iterations; graphs must be captured after.
  virtual int enable_structured(std::string &err) = 0;
  // Switches between the structured (after enable_structured) and the dense Psi-comp.
  virtual void set_structured(bool on) = 0;
  // Neighbour-coupled constraints on the rows of Phi x0 (library row indices o = m * rs + l):
  // lo_e <= y[row_a_e] - y[row_b_e] <= hi_e, solved inside Phi-comp by a nested ADMM (penalty
  // sigma, at most inner_max iterations, stop at inner_eps); n = 0 removes them.
  virtual int set_coupling(int n, const int64_t *row_a, const int64_t *row_b, const double *lo,
                           const double *hi, double sigma, int inner_max, double inner_eps,
                           std::string &err) = 0;
  virtual int host_exchange(int which, void *host, std::string &err) = 0;
  // FP64 certificate of the current iterate for x0_dev: out[0] = max |Z_AB Psi - I| over the
  // support and the (d+1)-hop ring of every column, out[1] = max |Phi - Psi|, out[2] = max over
  // columns of ||Phi[:,c] - Psi[:,c]||_2, out[3] = largest bound violation of Phi x0, out[4] =
  // max over columns of |N_j N_j' rho Lambda[:,c]| (Psi-step stationarity). Synchronises.
  virtual int certify(const double *x0_dev, double *out, std::string &err) = 0;
  virtual Ctl *ctl() = 0;
};

std::unique_ptr<Engine> make_engine(int precision, int nx);

// ----------------------------------------------------------------------------- batched engine
// B instances of one network (distinct x0) iterated together in the compact form of Algorithm 2:
// per instance only the Phi-comp row scalars alpha (current and previous iterate) and, per column
// subsystem j, tau_j = N_j' beta and eta_j = N_j' alpha (beta = running sum of alpha), from which
//   Psi[:,c] = o_c + x0_c N_j tau_j,  Lambda[:,c] = x0_c (I - N_j N_j') alpha   (on supp j),
// so that both products of an iteration are GEMMs over the instances with the shared N_j.

struct BCtl {  // per-instance control block
  int32_t iters, stop, converged, numeric;
  int32_t it0, pad;  // global iteration count when the instance entered its slot
  double last_rp, last_rd, objective;
  // FP64 check of the stopping iterate (bcheck kernels): trajectory y = Phi x0 recomputed in FP64
  // from the compact state; largest |Z_AB y - [x0; 0]| (dynamics and initial state), largest
  // bound violation of y, largest |u(0) returned - u(0) of y|, sum_r w_r y_r^2
  double eq_resid, box, u0dev, objective64;
};

struct BArgs {
  int32_t N, nx, nu, T, rs, Bmax;
  float rho;
  float *rho_b;  // [Bmax] penalty of each instance: rho, or rho times a per-instance factor
  const int64_t *tile_off, *rt_ptr, *rt_tile;
  const int32_t *rt_col, *kdim, *tile_rsub;
  const int64_t *koff;      // [N+1] offsets of the k-space vectors (multiples of 32)
  const int32_t *phi_order;  // [N] block -> row subsystem (Phi-comp dispatch order)
  // Psi-comp work units (heaviest first): column subsystem, row range [r0, r1), part index;
  // per column subsystem: number of parts, first part slot and offset of its partial sums
  // (split blocks only), arrival counters.
  const int32_t *pu_j, *pu_r0, *pu_r1, *pu_p;
  const int32_t *pj_n, *pj_first;
  const int64_t *pj_off;
  float *ppart;    // partial k-space sums [parts][k16][64]
  double *ppod;    // partial offset terms of the second cold iteration [parts][64][8][nx]
  int32_t *pcnt;   // [N]
  // Null bases in matrix-core fragment order, bf16 hi and lo (see BatchEngineT::init):
  const int64_t *ntf_off;   // [N+1] fragments of N_j' (Psi-comp left operand)
  const int64_t *nf_off;    // [n_tiles+1] fragments of the rows of tile (j, m) (Phi-comp)
  const __bf16 *ntf, *nf;
  // Structured Psi-comp (left operand N_u' of the input rows only, K = input rows in the order
  // the adjoint recursion produces them: step q = 0..T-2 gives u_{T-2-q} of every member) and
  // the transposed patch dynamics A_PP' per column subsystem (CSR over the patch states).
  const int64_t *ntu_off;   // [N+1]
  const __bf16 *ntu;
  const int64_t *srp0, *se0;
  const int32_t *srpt, *scolt;
  const float *svalt;
  const float *off;         // o_c, column-major per subsystem (leading dim ld4)
  const int64_t *off_ptr;
  const float *w, *lb, *ub; // [N*rs]
  const double *w64;
  const double *onorm2;     // [N*nx] ||o_c||^2
  float *alpha;             // [2][N*rs][Bmax] (iteration parity; instance index fastest)
  float *tau;               // [Ktot][Bmax] (instance index fastest)
  float *eta;               // [2][Ktot][Bmax] (iteration parity, as alpha)
  float *xn, *nrm;          // [Bmax][N] ||x0_j||^2 and ||x_r||^2 of row subsystem m
  float *bvec, *s;          // [N*rs][Bmax]
  float *x0;                // [Bmax][N*nx]
  BCtl *ictl;               // [Bmax]
  unsigned long long *slot; // [Bmax][2] residual maxima of the current iteration (ordered bits)
  Ctl *ctl;                 // shared: iteration count, all-stopped flag
  int64_t ktot;
  // Set-up passes outside the iteration (a copy of the arguments is launched with them):
  // init_pass 1: bpsi_kernel writes dst_k = N_j' src (row vectors [Bmax][N*rs]) per instance;
  // phi_mode 1: bphi_kernel writes cg_q = sum_{j in P(m)} ||x0_j||^2 N_j eta_j (rows of m).
  int32_t init_pass, phi_mode, wmode;
  // Streamed joins: phase[b] < 0 for an instance in the ADMM iteration; 0..cg_k+1 while its
  // trajectory start runs inside the iterations (its column of the products serves the start:
  // phase 0..cg_k-1 Psi-comp stages cg_p (eta = N'p, W = ||x0_j||^2 eta), 1..cg_k Phi-comp
  // writes q = M p and a CG step follows, cg_k stages beta (tau = N'beta), cg_k+1 stages
  // alpha^0 (eta, W = ||x0_j||^2 (tau + eta)); then the ADMM iteration starts).
  int32_t *phase;  // (the number of CG steps, cg_k, is ctl->cg_k)
  const float *src;
  int64_t src_bs, src_rs;   // element (b, row) of src at b * src_bs + row * src_rs
  float *dst_k;
  // Right operand of the Phi-comp products, W_j = ||x0_j||^2 (tau_j + eta_j) as bf16 hi + lo,
  // element (b, k) of subsystem j at ((koff_j + k) / 8 * Bw + b) * 8 + k % 8 with Bw = Bmax
  // rounded up to 16 (a product tile always covers 16 instances); and the
  // per-row-subsystem sums of (alpha - alpha_prev)^2 [Bmax][N].
  int32_t Bw;
  __bf16 *w_hi, *w_lo;
  double *dlm;
  // Trajectory warm start: predicted trajectory (state rows simulated), CG vectors, r'r.
  float *yhat, *cg_x, *cg_r, *cg_p, *cg_q;
  double *cg_rr, *cg_rrn;  // [Bmax] r'r at the start of the CG step, and after it
  double *cgpart;          // [Bmax][2][row ranges] partial sums of p'q and of the new r'r
  double *bpart;  // [Bmax][2][parts] partial sums of r'r (start) and of the objective (output)
  const int64_t *a_rowptr;
  const int32_t *a_colidx;
  const float *a_blk, *b_blk;  // plant blocks (row-major nx x nx, nx x nu)
  // FP64 check of the stopping iterate: null bases (column-major, leading dimension D rounded
  // up to 4, at nb64 + nb_off[j]), offsets, bounds, plant blocks, and the recomputed
  // trajectories y64 [Bmax][N*rs]
  const double *nb64, *off64, *lb64, *ub64, *a64, *b64;
  const int64_t *nb_off;
  double *y64;
  double *wchk;  // [Ktot][64] product operand of the check (W_j of each instance)
  double *chkpart;  // [Bmax][parts][4] per-part maxima (eq, box, u0) and objective sums
};

class BatchEngine {
 public:
  virtual ~BatchEngine() = default;
  // split: basis operands as bf16 hi + lo (FP32-level products); otherwise rounded once to bf16
  virtual int init(const HostSetup &hs, double rho, int bmax, bool split, hipStream_t s, std::string &err) = 0;
  // Per-solve set-up of B instances; warm != 0 selects the iteration of a warm start (one of
  // the start_* calls below must follow before the first iteration). rho_scale_dev [B] (or
  // NULL: all 1): instance b runs with the penalty rho * rho_scale_dev[b].
  virtual int precompute(const double *x0_dev, int B, int max_iter, double eps, int warm,
                         const double *rho_scale_dev, std::string &err) = 0;
  // Compact start from row multipliers alpha0 [B][N*rs]: Psi^0[:,c] = o_c,
  // Lambda^0[:,c] = x0_c (I - N_j N_j') alpha0 on supp j.
  virtual int start_alpha(const double *alpha0_dev, std::string &err) = 0;
  // Start from a trajectory: input rows from y0_dev [B][N*rs] (or, if NULL, already in
  // yhat()), state rows simulated from x0, cg_iters CG steps on M beta = y - b, then
  // Psi^0[:,c] = o_c + x0_c N_j N_j' beta and Lambda^0[:,c] = x0_c (I - N_j N_j') alpha with
  // alpha = -2 w y / rho.
  virtual int start_trajectory(const double *y0_dev, int cg_iters, std::string &err) = 0;
  virtual float *yhat() = 0;  // [Bmax][N*rs] FP32
  // Current row multipliers alpha and trajectory rows (Phi x0) of every instance, [B][N*rs].
  virtual int export_alpha(double *alpha_dev, std::string &err) = 0;
  virtual int export_y(double *y_dev, std::string &err) = 0;
  // One iteration (capturable); with `joins`, also the CG step of streamed joins.
  virtual int iteration(std::string &err, bool joins = false) = 0;
  // Kernel variants (autotuned at setup): instance tiles per Phi-comp wave (1 or 2) and the
  // Psi-comp split of heavy patches into several work units (basis cost above psi_capx times the
  // mean; one of 2, 4, 8, 16, 1 << 20). Synchronises the engine's stream.
  virtual int set_variant(int phi_ntw, int psi_capx, std::string &err) = 0;
  virtual void variant(int *phi_ntw, int *psi_capx, int *n_units) const = 0;
  // One kernel of an iteration: 0 bphi_kernel, 1 bpsi_kernel, 2 bdecide_kernel.
  virtual int launch_one(int k, std::string &err) = 0;
  virtual int output(double *u0_dev, std::string &err) = 0;
  // Base penalty of the solves started after this call (per-instance factors multiply it).
  virtual void set_rho(double rho) = 0;
  // Closed loop (Algorithm 1), FP64: x(t+1) = A x(t) + B u(t) for B instances in place in x_dev
  // [B][N*nx] (u_dev [B][N*nu]), with x(t) (at t = 0), x(t+1) and u(t) stored in the loop's
  // trajectories xs_dev [B][T_sim+1][N*nx] and us_dev [B][T_sim][N*nu]. rho_scale_dev [B] (or
  // NULL): receives ||x(t+1)||^2 / ||x(0)||^2 (at least 1e-20; 1 when x(0) = 0).
  virtual int plant_step(double *x_dev, const double *u_dev, double *xs_dev, double *us_dev, int t, int T_sim,
                         int B, double *rho_scale_dev, std::string &err) = 0;
  // Input rows of y_dev [B][N*rs] moved one step ahead (last held) into ys_dev.
  virtual int shift_inputs(const double *y_dev, double *ys_dev, int B, std::string &err) = 0;
  // FP64 check of the stopping iterate of every instance of the batch (x0_dev [B][N*nx], the
  // solve's FP64 initial states): results in the per-instance control blocks (BCtl eq_resid,
  // box, u0dev, objective64).
  virtual int check(const double *x0_dev, std::string &err) = 0;
  // Streams: the stopping state of slots[0..S) copied into stash slots to[0..S) (the slots can
  // then be refilled); the FP64 check of stash slots 0..S-1, holding the stopped instances
  // dst[0..S) of x0_dev, with its results in the stash's control blocks (stash_ictl).
  virtual int stash_slots(const int32_t *slots, const int32_t *to, int S, std::string &err) = 0;
  virtual int check_stash(const double *x0_dev, const int32_t *dst, int S, std::string &err) = 0;
  virtual BCtl *stash_ictl() = 0;
  // Streamed solves (warm starts only). Slots slots[0..S) take the instances xsrc[0..S) of
  // x0_dev ([*][N*nx]); their input-row predictions are ypred [S][N*rs] (FP32, device). first:
  // the initial fill (resets the solve, batch = S, slots 0..S-1); otherwise the slots join the
  // running solve. The joiners' trajectory start (cg_iters CG steps and the start projections)
  // then runs inside the following iterations, in their columns of the same products.
  virtual int stream_start(const double *x0_dev, const int32_t *slots, const int32_t *xsrc, int S,
                           const float *ypred, int cg_iters, bool first, int max_iter, double eps,
                           std::string &err) = 0;
  // u(0) and objective of slots[0..S) into rows dst[0..S) of u0_dev ([*][N*nu]).
  virtual int output_slots(double *u0_dev, const int32_t *slots, const int32_t *dst, int S, std::string &err) = 0;
  virtual Ctl *ctl() = 0;
  virtual BCtl *ictl() = 0;
  virtual int bmax() const = 0;
};

std::unique_ptr<BatchEngine> make_batch_engine(int nx);

// Device address of the current device's copy of the stream entry's static prediction
// staging (taken once per device) and its size in floats. Returns a DLMPC_* status.
int stream_scratch(float **ptr, size_t *cap_floats, std::string &err);

// *ok = every entry of x_dev[0..n) is finite (device check on stream s, synchronised; flag_dev
// one device int, flag_host one pinned host int). Returns a DLMPC_* status.
int device_all_finite(const double *x_dev, int64_t n, int32_t *flag_dev, int32_t *flag_host, hipStream_t s,
                      bool *ok, std::string &err);

// ----------------------------------------------------------------------------- learned warm start
// One network per subsystem g (separate weights): x = x0 of the members of P(g) in ascending
// order / xs (zero-padded to IN = p_max nx), h1 = gelu(x W1 + b1), h2 = gelu(h1 W2 + b2),
// y = [h2, x] W3 + b3, the input rows u_0..u_{T-2} of g's trajectory = ys y (OUT = nu (T-1)).
// Parameters are FP32, flat, in the order W1 [G][IN][H], b1 [G][H], W2 [G][H][H], b2 [G][H],
// W3 [G][H+IN][OUT], b3 [G][OUT]. Trajectories are [S][N*rs] in library row order.
class WarmStart {
 public:
  ~WarmStart();
  int init(const HostSetup &hs, int hidden, int max_samples, uint64_t seed, double x_scale, double y_scale,
           hipStream_t s, std::string &err);
  // Forward pass for S samples x0_dev [S][N*nx] (activations kept for backward).
  int forward(int S, const double *x0_dev, std::string &err);
  // After forward: loss against the input rows of trajectories y_dev [S][N*rs], gradient in grad.
  int backward(int S, const double *y_dev, double *loss, std::string &err);
  int adam(double lr, std::string &err);
  // Writes the predicted input rows into y [S][N*rs] (other rows untouched), FP64 or FP32.
  int predict(int S, const double *x0_dev, double *y_dev, std::string &err);
  int predict(int S, const double *x0_dev, float *y_dev, std::string &err);
  int save(const char *path, std::string &err);
  int load(const char *path, std::string &err);  // shape must match; scales are read
  static int peek(const char *path, int32_t *hidden, std::string &err);

  int G = 0, nx = 0, rs = 0, roff = 0, IN = 0, H = 0, OUT = 0, Smax = 0;
  double xs = 1.0, ys = 1.0;
  int64_t n_params = 0, step = 0;
  float *theta = nullptr, *grad = nullptr;

 private:
  static constexpr int kLossBlocks = 256;
  static constexpr int32_t kMagic = 0x57534d31;  // file tag
  int alloc_bytes(void **dst, size_t bytes, std::string &err);
  void views(float *base, float **W1, float **b1, float **W2, float **b2, float **W3, float **b3) const;
  std::vector<void *> owned_;
  hipStream_t stream_ = nullptr;
  int64_t *rt_ptr_ = nullptr;
  int32_t *rt_col_ = nullptr;
  float *mom1_ = nullptr, *mom2_ = nullptr;
  float *XA_ = nullptr;  // [G][S][H+IN]: h2 in the first H columns, x in the last IN
  float *Z1_ = nullptr, *A1_ = nullptr, *Z2_ = nullptr, *Y_ = nullptr, *T_ = nullptr, *dY_ = nullptr;
  float *dZ2_ = nullptr, *dZ1_ = nullptr;
  double *loss_part_ = nullptr;
};

}  // namespace dlmpc
