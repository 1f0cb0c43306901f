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
  Tf rho;
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
};

class Engine {
 public:
  virtual ~Engine() = default;
  virtual int init(const HostSetup &hs, double rho, hipStream_t s, std::string &err) = 0;
  // Enqueue the per-solve precompute (cold start when wpsi == nullptr) on the stream.
  virtual int precompute(const double *x0_dev, const double *wpsi, const double *wlam,
                         int max_iter, double eps, std::string &err) = 0;
  // Enqueue one ADMM iteration of the graph schedule (capturable), or one of its kernels
  // (0 Phi-comp, 1 Psi pass 1, 2 Psi pass 2, 3 Conv).
  virtual int iteration(std::string &err) = 0;
  virtual int launch_one(int which, std::string &err) = 0;
  // Enqueue all iterations of one solve as one launch (persistent schedule).
  virtual int run_persistent(bool tune, std::string &err) = 0;
  virtual int persistent_grid() const = 0;  // 0 when the device cannot co-schedule the grid
  virtual int output(double *u0_dev, std::string &err) = 0;
  virtual int export_phi(double *phi_dev, std::string &err) = 0;
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
  double last_rp, last_rd, objective;
};

struct BArgs {
  int32_t N, nx, nu, T, rs, Bmax;
  float rho;
  const int64_t *tile_off, *rt_ptr, *rt_tile;
  const int32_t *rt_col, *kdim, *tile_rsub;
  const int64_t *koff;      // [N+1] offsets of the k-space vectors (multiples of 16)
  const int64_t *ncm_off;   // [N+1] column-major copy: k16(j) columns of ld64(j) rows
  const int64_t *nrm_off;   // [N+1] row-major copy: D(j) rows of k32(j) entries
  const __bf16 *ncm_hi, *ncm_lo, *nrm_hi, *nrm_lo;
  const float *off;         // o_c, column-major per subsystem (leading dim ld4)
  const int64_t *off_ptr;
  const float *w, *lb, *ub; // [N*rs]
  const double *w64;
  const double *onorm2;     // [N*nx] ||o_c||^2
  float *alpha;             // [2][Bmax][N*rs] (iteration parity)
  float *tau, *eta;         // [Bmax][Ktot]
  float *xn, *nrm;          // [Bmax][N] ||x0_j||^2 and ||x_r||^2 of row subsystem m
  float *bvec, *s;          // [Bmax][N*rs]
  float *x0;                // [Bmax][N*nx]
  BCtl *ictl;               // [Bmax]
  unsigned long long *slot; // [Bmax][2] residual maxima of the current iteration (ordered bits)
  Ctl *ctl;                 // shared: iteration count, all-stopped flag
  int64_t ktot;
  int32_t init_pass;        // 1 while bpsi_kernel computes eta = N' alpha of the warm start
};

class BatchEngine {
 public:
  virtual ~BatchEngine() = default;
  virtual int init(const HostSetup &hs, double rho, int bmax, hipStream_t s, std::string &err) = 0;
  // alpha0_dev: NULL (cold start) or [B][N*rs] row multipliers of a compact warm start
  // (Psi^0[:,c] = o_c, Lambda^0[:,c] = x0_c (I - N_j N_j') alpha0 on supp j).
  virtual int precompute(const double *x0_dev, const double *alpha0_dev, int B, int max_iter,
                         double eps, std::string &err) = 0;
  // Current row multipliers alpha of every instance, [B][N*rs] doubles.
  virtual int export_alpha(double *alpha_dev, std::string &err) = 0;
  virtual int iteration(std::string &err) = 0;  // capturable
  virtual int output(double *u0_dev, std::string &err) = 0;
  virtual Ctl *ctl() = 0;
  virtual BCtl *ictl() = 0;
  virtual int bmax() const = 0;
};

std::unique_ptr<BatchEngine> make_batch_engine(int nx);

}  // namespace dlmpc
