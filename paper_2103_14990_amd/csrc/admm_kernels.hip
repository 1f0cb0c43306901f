// HIP kernels of the DLMPC-ADMM hot loop (Algorithm 2) for CDNA4 (gfx950).
//
// One ADMM iteration is a Phi-comp launch and a Psi-comp/Lambda/Conv phase:
//   phi_kernel  — Phi-comp, one workgroup per row subsystem m: gathers the tiles
//                 (Psi - Lambda)[rows of m, columns of P(m)], forms a_r = v_r . x_r for the
//                 rs rows of m, takes the explicit row solution (clip of
//                 rho a / (rho + 2 w ||x_r||^2) onto the row's box, Section II-A and
//                 Algorithm 2), and writes Phi = v + alpha_r x_r and y_r = (Phi x0)_r.
//   Psi-comp    — projects the nx columns of (Phi + Lambda) on the support of each column
//                 subsystem j onto the affine set of Z_AB psi = e_c with the null basis N_j
//                 (psi = N_j N_j' v + o_c), updates Lambda <- Lambda + Phi - Psi and reduces the
//                 per-column primal and dual residual norms to the stop decision (combined
//                 kernels, Section III-C). In the graph schedule this is three launches of
//                 uniform work units (psi_pass1_kernel, psi_pass2_kernel, conv_kernel); the
//                 persistent schedule runs one workgroup per column subsystem (psi_body).
// Every tile written by one step is read by exactly one workgroup of the other step, so the
// row->column exchange is a kernel boundary (or grid barrier) and no atomics touch the
// iterate. Every reduction runs in a fixed order (bitwise reproducible).
// A control block on the device carries the stop flag; once set, every later kernel of the
// captured iteration graph returns immediately, so the host only polls it every K
// iterations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>
#include <cstring>
#include <memory>
#include <string>

#include "dlmpc_device.h"

namespace dlmpc {

namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr int kNumIterKernels = 4;
constexpr unsigned long long kSpinLimit = 20000000ull;  // ~1 s of polling per barrier

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <typename T>
__device__ __forceinline__ T clip(T s, T lo, T hi) {
  return s < lo ? lo : (s > hi ? hi : s);
}

__device__ __forceinline__ unsigned long long as_bits(double v) {
  return static_cast<unsigned long long>(__double_as_longlong(v));
}

// ------------------------------------------------------------------ per-solve precompute

// Per row subsystem m: ||x_r||^2 over its d-hop patch (the same for all rows of m), x0 in the
// working precision, the cold-start Psi^0 = Lambda^0 = 0 on m's tiles, and (block 0) the
// control block reset (Algorithm 1, per-step precomputation with x(t)).
template <typename Tf, int NX>
__global__ __launch_bounds__(kBlock) void precompute_kernel(KArgs<Tf> a, const double *x0,
                                                            int cold, int max_iter, double eps,
                                                            double rho) {
  const int m = blockIdx.x;
  const int tid = threadIdx.x;
  if (tid < NX) a.x0f[m * NX + tid] = static_cast<Tf>(x0[m * NX + tid]);
  if (tid == 0) {
    double s = 0.0;
    for (int64_t q = a.rt_ptr[m]; q < a.rt_ptr[m + 1]; ++q) {
      const int j = a.rt_col[q];
#pragma unroll
      for (int c = 0; c < NX; ++c) s += x0[j * NX + c] * x0[j * NX + c];
    }
    a.nrm[m] = static_cast<Tf>(s);
  }
  if (cold) {
    for (int64_t q = a.rt_ptr[m]; q < a.rt_ptr[m + 1]; ++q) {
      const int64_t base = a.rt_tile[q] * a.ts;
      for (int e = tid; e < a.ts; e += kBlock) {
        a.psi[base + e] = Tf(0);
        a.lam[base + e] = Tf(0);
        a.phi[base + e] = Tf(0);
      }
    }
  }
  if (m == 0 && tid == 0) {
    Ctl *c = a.ctl;
    c->iters = 0;
    c->stop = 0;
    c->converged = 0;
    c->numeric = 0;
    c->max_iter = max_iter;
    c->done_count = 0u;
    c->rp_bits = 0ull;
    c->rd_bits = 0ull;
    c->last_rp = INFINITY;
    c->last_rd = INFINITY;
    c->eps = eps;
    c->rho = rho;
    c->inner_iters = 0;
    c->objective = 0.0;
    c->bar_count = 0u;
    c->bar_gen = 0u;
    c->bar_fail = 0u;
    c->slot_rp[0] = c->slot_rp[1] = 0ull;
    c->slot_rd[0] = c->slot_rd[1] = 0ull;
  }
}

// Warm start: Psi^0, Lambda^0 from canonical CSR values.
template <typename Tf>
__global__ __launch_bounds__(kBlock) void warm_kernel(Tf *psi, Tf *lam, const int64_t *map, int64_t n,
                                                      const double *wpsi, const double *wlam) {
  for (int64_t e = blockIdx.x * int64_t(kBlock) + threadIdx.x; e < n; e += int64_t(gridDim.x) * kBlock) {
    const int64_t c = map[e];
    psi[e] = static_cast<Tf>(wpsi[c]);
    lam[e] = static_cast<Tf>(wlam[c]);
  }
}

// ------------------------------------------------------------------ Phi-comp

// Phi-comp of row subsystem m. Lane l of every wave owns local row l0 + l of a 64-row chunk;
// the waves split the patch tiles (tile k goes to wave k mod kWaves), accumulate
// a_r = v_r . x_r over their tiles, combine the kWaves partial sums in LDS in a fixed order,
// and apply the explicit row solution to the tile values they still hold in registers.
constexpr int kPhiRegTiles = 16;  // tiles per wave kept in registers between the two sweeps

template <typename Tf, int NX>
__device__ __forceinline__ void phi_body(const KArgs<Tf> &a, int m, unsigned char *smem_raw) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t t0 = a.rt_ptr[m];
  const int np = int(a.rt_ptr[m + 1] - t0);
  const int rs = a.rs;
  Tf *xs = reinterpret_cast<Tf *>(smem_raw);  // [np][NX] x0 of the patch members
  Tf *part = xs + ((np * NX + 3) & ~3);       // [kWaves][64]
  Tf *alpha_s = part + kWaves * 64;           // [64]
  for (int i = tid; i < np * NX; i += kBlock) xs[i] = a.x0f[a.rt_col[t0 + i / NX] * NX + i % NX];
  __syncthreads();
  const Tf n = a.nrm[m], rho = static_cast<Tf>(a.ctl->rho);
  for (int l0 = 0; l0 < rs; l0 += 64) {
    const int l = l0 + lane;
    const bool act = l < rs;
    Tf vreg[kPhiRegTiles][NX];
    Tf acc = Tf(0);
#pragma unroll
    for (int kk = 0; kk < kPhiRegTiles; ++kk) {
      const int k = wave + kk * kWaves;
      if (act && k < np) {
        const int64_t base = a.rt_tile[t0 + k] * a.ts + int64_t(l) * NX;
#pragma unroll
        for (int c = 0; c < NX; ++c) {
          vreg[kk][c] = a.psi[base + c] - a.lam[base + c];
          acc += xs[k * NX + c] * vreg[kk][c];
        }
      }
    }
    for (int k = wave + kPhiRegTiles * kWaves; k < np; k += kWaves) {
      if (!act) break;
      const int64_t base = a.rt_tile[t0 + k] * a.ts + int64_t(l) * NX;
#pragma unroll
      for (int c = 0; c < NX; ++c) acc += xs[k * NX + c] * (a.psi[base + c] - a.lam[base + c]);
    }
    part[wave * 64 + lane] = acc;
    __syncthreads();
    if (wave == 0 && act) {
      Tf s = part[lane];
#pragma unroll
      for (int w = 1; w < kWaves; ++w) s += part[w * 64 + lane];
      const int64_t o = int64_t(m) * rs + l;
      Tf sv, al;
      if (n > Tf(0)) {
        sv = clip(rho * s / (rho + Tf(2) * a.w[o] * n), a.lb[o], a.ub[o]);
        al = (sv - s) / n;
      } else {
        sv = s;
        al = Tf(0);
      }
      alpha_s[lane] = al;
      a.y[o] = sv;
      if (a.cp_slot) {  // coupled row: the nested ADMM replaces sv (coupled_fix_kernel)
        const int k = a.cp_slot[o];
        if (k >= 0) {
          a.cp_a[k] = s;
          a.cp_s0[k] = sv;
        }
      }
    }
    __syncthreads();
    if (act) {
      const Tf al = alpha_s[lane];
#pragma unroll
      for (int kk = 0; kk < kPhiRegTiles; ++kk) {
        const int k = wave + kk * kWaves;
        if (k < np) {
          const int64_t base = a.rt_tile[t0 + k] * a.ts + int64_t(l) * NX;
#pragma unroll
          for (int c = 0; c < NX; ++c) a.phi[base + c] = vreg[kk][c] + al * xs[k * NX + c];
        }
      }
      for (int k = wave + kPhiRegTiles * kWaves; k < np; k += kWaves) {
        const int64_t base = a.rt_tile[t0 + k] * a.ts + int64_t(l) * NX;
#pragma unroll
        for (int c = 0; c < NX; ++c) a.phi[base + c] = (a.psi[base + c] - a.lam[base + c]) + al * xs[k * NX + c];
      }
    }
    __syncthreads();
  }
}

template <typename Tf, int NX>
__global__ __launch_bounds__(kBlock) void phi_kernel(KArgs<Tf> a) {
  if (a.ctl->stop) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  phi_body<Tf, NX>(a, a.phi_order[blockIdx.x], smem_raw);
}

// ------------------------------------------------------------------ coupled Phi-step

__device__ __forceinline__ double block_max1024(double v, double *red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  __syncthreads();  // red may still be read by the previous call
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double m = red[0];
#pragma unroll
  for (int w = 1; w < 16; ++w) m = fmax(m, red[w]);
  return m;
}

// Nested ADMM of the coupled Phi-step, one workgroup: the Phi-step in y = Phi x0 is
// min sum_r c_r (y_r - m_r)^2 over the row boxes and the pairs lo_e <= y_a - y_b <= hi_e, with
// c_r = w_r + rho / (2 n), m_r = rho a_r / (rho + 2 w_r n). Per inner iteration: every coupled
// row's y from its own pairs' copies and duals (a 1-D quadratic clipped to its box), then every
// pair's copies projected onto its slab and its duals updated; stop when the copies agree with
// y and stopped moving to inner_eps (max norms), or after inner_max iterations. Copies and
// duals carry over to the next outer iteration.
template <typename Tf, int NX>
__global__ __launch_bounds__(1024) void coupled_inner_kernel(KArgs<Tf> a, CoupleArgs<Tf> c) {
  if (a.ctl->stop) return;
  __shared__ double red[16];
  const int tid = threadIdx.x;
  const double rho = a.ctl->rho, sig = c.sigma;
  int it = 0;
  for (it = 1; it <= c.inner_max; ++it) {
    for (int k = tid; k < c.K; k += 1024) {
      const int64_t o = c.row[k];
      const double n = double(a.nrm[c.sub[k]]), ak = double(a.cp_a[k]);
      double y = ak;
      if (n > 0.0) {
        const double w = double(a.w[o]);
        const double cc = w + rho / (2.0 * n), mm = rho * ak / (rho + 2.0 * w * n);
        double acc_a = 0.0, acc_b = 0.0;  // first-row pairs, then second-row pairs
        const int p0 = c.kp_ptr[k], p1 = c.kp_ptr[k + 1];
        for (int p = p0; p < p1; ++p) {
          const int e = c.kp_ent[p] >> 1;
          if (c.kp_ent[p] & 1)
            acc_b += double(c.zb[e]) - double(c.lb[e]);
          else
            acc_a += double(c.za[e]) - double(c.la[e]);
        }
        y = (2.0 * cc * mm + sig * (acc_a + acc_b)) / (2.0 * cc + sig * double(p1 - p0));
        y = fmin(fmax(y, double(a.lb[o])), double(a.ub[o]));
      }
      c.y[k] = static_cast<Tf>(y);
    }
    __syncthreads();
    double rp = 0.0, dz = 0.0;
    for (int e = tid; e < c.E; e += 1024) {
      const double ya = double(c.y[c.ka[e]]), yb = double(c.y[c.kb[e]]);
      const double pa = ya + double(c.la[e]), pb = yb + double(c.lb[e]);
      const double d = pa - pb, sh = 0.5 * (fmin(fmax(d, c.lo[e]), c.hi[e]) - d);
      const double za = pa + sh, zb = pb - sh;
      dz = fmax(dz, fmax(fabs(za - double(c.za[e])), fabs(zb - double(c.zb[e]))));
      rp = fmax(rp, fmax(fabs(ya - za), fabs(yb - zb)));
      c.la[e] = static_cast<Tf>(double(c.la[e]) + ya - za);
      c.lb[e] = static_cast<Tf>(double(c.lb[e]) + yb - zb);
      c.za[e] = static_cast<Tf>(za);
      c.zb[e] = static_cast<Tf>(zb);
    }
    rp = block_max1024(rp, red);
    dz = block_max1024(dz, red);
    if (rp <= c.inner_eps && sig * dz <= c.inner_eps) break;
  }
  if (tid == 0) a.ctl->inner_iters += it > c.inner_max ? c.inner_max : it;
}

// The coupled rows' Phi-comp result with the nested ADMM's y: phi = v + ((y - a)/n) x_r, i.e.
// the uncoupled result plus ((y - s0)/n) x_r on every tile of the row's subsystem.
template <typename Tf, int NX>
__global__ __launch_bounds__(256) void coupled_fix_kernel(KArgs<Tf> a, CoupleArgs<Tf> c) {
  if (a.ctl->stop) return;
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= c.K) return;
  const int64_t o = c.row[k];
  const int m = c.sub[k], l = int(o - int64_t(m) * a.rs);
  const Tf n = a.nrm[m];
  const Tf y = c.y[k];
  if (!(n > Tf(0))) return;
  const Tf dl = (y - a.cp_s0[k]) / n;
  for (int64_t q = a.rt_ptr[m]; q < a.rt_ptr[m + 1]; ++q) {
    const int64_t base = a.rt_tile[q] * a.ts + int64_t(l) * NX;
    const Tf *xj = a.x0f + int64_t(a.rt_col[q]) * NX;
#pragma unroll
    for (int cc = 0; cc < NX; ++cc) a.phi[base + cc] += dl * xj[cc];
  }
  a.y[o] = y;
}

// ------------------------------------------------------------------ Psi/Lambda/Conv

// 16-byte vectors of the working type (4 floats or 2 doubles).
template <typename Tf>
struct VecT;
template <>
struct VecT<float> {
  typedef float type __attribute__((ext_vector_type(4)));
  static constexpr int N = 4;
};
template <>
struct VecT<double> {
  typedef double type __attribute__((ext_vector_type(2)));
  static constexpr int N = 2;
};

__device__ __forceinline__ float hsum(const VecT<float>::type &x) { return (x[0] + x[1]) + (x[2] + x[3]); }
__device__ __forceinline__ double hsum(const VecT<double>::type &x) { return x[0] + x[1]; }

// Psi-comp, Lambda-comp and the Conv residuals of column subsystem j. On return thread 0
// holds the largest primal and dual residual norm over j's columns in *rp_out / *rd_out
// (NaN propagates). Ends with the block synchronised.
//
// v = (Phi + Lambda)[support of j, columns of j] is staged in LDS; then
//   pass 1: t = N_j' v, each wave streams kUC basis vectors at a time with 16-byte loads
//           (kUC independent loads in flight per lane) and reduces them across lanes;
//   pass 2: psi = N_j t + o_c, each thread owns VN consecutive rows and streams the basis
//           vectors (coalesced over rows, t broadcast from LDS), then updates Lambda and the
//           residuals of its rows.
// N_j is read twice; the second read of each column block follows the first closely, so it
// is mostly served by the caches.
template <typename Tf, int NX>
__device__ __forceinline__ void psi_body(const KArgs<Tf> &a, int j, unsigned char *smem_raw,
                                         double *rp_out, double *rd_out) {
  using V = typename VecT<Tf>::type;
  constexpr int VN = VecT<Tf>::N;
  constexpr int kUC = 8;
  __shared__ double red[kWaves][2 * NX];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t tb = a.tile_off[j];
  const int D = int(a.tile_off[j + 1] - tb) * a.rs;
  const int ld = (D + 3) & ~3;
  const int nvec = ld / VN;
  const int k = a.kdim[j];
  const int64_t base = tb * a.ts;
  const Tf *__restrict__ Nj = a.nb + a.nb_off[j];
  const Tf *__restrict__ Oj = a.off + a.off_ptr[j];
  Tf *v = reinterpret_cast<Tf *>(smem_raw);  // [NX][ld], zero padded
  Tf *t = v + NX * ld;                       // [NX][k]

  for (int e = tid; e < ld * NX; e += kBlock) {
    const int r = e / NX, c = e - r * NX;
    v[c * ld + r] = (r < D) ? a.phi[base + e] + a.lam[base + e] : Tf(0);
  }
  __syncthreads();
  for (int i0 = wave * kUC; i0 < k; i0 += kWaves * kUC) {
    Tf acc[kUC][NX];
#pragma unroll
    for (int u = 0; u < kUC; ++u)
#pragma unroll
      for (int c = 0; c < NX; ++c) acc[u][c] = Tf(0);
    for (int q = lane; q < nvec; q += 64) {
      V nv[kUC];
#pragma unroll
      for (int u = 0; u < kUC; ++u)
        nv[u] = (i0 + u < k) ? *reinterpret_cast<const V *>(Nj + int64_t(i0 + u) * ld + q * VN) : V(0);
      V vv[NX];
#pragma unroll
      for (int c = 0; c < NX; ++c) vv[c] = *reinterpret_cast<const V *>(v + c * ld + q * VN);
#pragma unroll
      for (int u = 0; u < kUC; ++u)
#pragma unroll
        for (int c = 0; c < NX; ++c) acc[u][c] += hsum(nv[u] * vv[c]);
    }
#pragma unroll
    for (int u = 0; u < kUC; ++u)
#pragma unroll
      for (int c = 0; c < NX; ++c) {
        const Tf s = wave_sum(acc[u][c]);
        if (lane == 0 && i0 + u < k) t[c * k + i0 + u] = s;
      }
  }
  __syncthreads();
  // v is free after pass 1: stage psi (row-major, the global layout) for a coalesced epilogue
  for (int q = tid; q < nvec; q += kBlock) {
    V y[NX];
#pragma unroll
    for (int c = 0; c < NX; ++c) y[c] = V(0);
#pragma unroll 8
    for (int i = 0; i < k; ++i) {
      const V nv = *reinterpret_cast<const V *>(Nj + int64_t(i) * ld + q * VN);
#pragma unroll
      for (int c = 0; c < NX; ++c) y[c] += nv * t[c * k + i];
    }
#pragma unroll
    for (int e = 0; e < VN; ++e) {
      const int r = q * VN + e;
      if (r >= D) break;
#pragma unroll
      for (int c = 0; c < NX; ++c) v[r * NX + c] = y[c][e] + Oj[c * ld + r];
    }
  }
  __syncthreads();
  double rp[NX], rd[NX];
#pragma unroll
  for (int c = 0; c < NX; ++c) rp[c] = rd[c] = 0.0;
  for (int e = tid; e < D * NX; e += kBlock) {
    const int c = e % NX;
    const Tf psn = v[e];
    const int64_t idx = base + e;
    const Tf ph = a.phi[idx], la = a.lam[idx], pso = a.psi[idx];
    a.lam[idx] = (la + ph) - psn;
    a.psi[idx] = psn;
    const double dp = double(ph - psn), dd = double(psn - pso);
#pragma unroll
    for (int cc = 0; cc < NX; ++cc)
      if (cc == c) {
        rp[cc] += dp * dp;
        rd[cc] += dd * dd;
      }
  }
#pragma unroll
  for (int c = 0; c < NX; ++c) {
    rp[c] = wave_sum(rp[c]);
    rd[c] = wave_sum(rd[c]);
  }
  if (lane == 0) {
#pragma unroll
    for (int c = 0; c < NX; ++c) {
      red[wave][c] = rp[c];
      red[wave][NX + c] = rd[c];
    }
  }
  __syncthreads();
  if (tid == 0) {
    double mp = 0.0, md = 0.0;
#pragma unroll
    for (int c = 0; c < NX; ++c) {
      double sp = 0.0, sd = 0.0;
      for (int w = 0; w < kWaves; ++w) {
        sp += red[w][c];
        sd += red[w][NX + c];
      }
      sp = sqrt(sp);
      sd = sqrt(sd);
      mp = (sp > mp || sp != sp) ? sp : mp;
      md = (sd > md || sd != sd) ? sd : md;
    }
    *rp_out = mp;
    *rd_out = md;
  }
  __syncthreads();
}

// Stop decision from the reduced residuals of one iteration (shared by both schedules).
__device__ __forceinline__ void decide(Ctl *c, int it, double rpm, double rdm) {
  c->iters = it;
  c->last_rp = rpm;
  c->last_rd = rdm;
  if (!(rpm == rpm) || !(rdm == rdm) || isinf(rpm) || isinf(rdm)) {
    c->numeric = 1;
    c->stop = 1;
  } else if (rpm <= c->eps && rdm <= c->eps) {
    c->converged = 1;
    c->stop = 1;
  } else if (it >= c->max_iter) {
    c->stop = 1;
  }
}

// ------------------------------------------------------------------ split Psi-comp (graph schedule)
//
// Psi-comp of all column subsystems as two launches of uniform work units, so that the long
// patches do not bound the kernel time:
//   psi_pass1_kernel  unit (j, i0): t_j[i] = N_j[:, i]' v_j for kP1Cols basis vectors from i0;
//   psi_pass2_kernel  unit (j, r0): psi = N_j t_j + o_c on rows [r0, r0 + RB) with the basis
//                     split over the block's waves (partial sums combined in LDS in a fixed
//                     order), then Lambda and the residual partial sums of those rows;
//   conv_kernel       one block: per column subsystem, the residual partial sums of its units in
//                     unit order, the column norms, their maximum and the stop decision.
// Kernel boundaries order the three launches; nothing is exchanged through atomics.

constexpr int kP1Cols = kWaves * 8;  // basis vectors per pass-1 unit (8 per wave)

template <typename Tf, int NX>
__global__ __launch_bounds__(kBlock) void psi_pass1_kernel(KArgs<Tf> a, PsiUnits<Tf> pu) {
  if (a.ctl->stop) return;
  using V = typename VecT<Tf>::type;
  constexpr int VN = VecT<Tf>::N;
  constexpr int kUC = 8;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int j = pu.p1[2 * blockIdx.x], ibase = pu.p1[2 * blockIdx.x + 1];
  const int64_t tb = a.tile_off[j];
  const int D = int(a.tile_off[j + 1] - tb) * a.rs;
  const int ld = (D + 3) & ~3;
  const int nvec = ld / VN;
  const int k = a.kdim[j];
  const int64_t base = tb * a.ts;
  const Tf *__restrict__ Nj = a.nb + a.nb_off[j];
  Tf *v = reinterpret_cast<Tf *>(smem_raw);  // [NX][ld], zero padded
  for (int e = tid; e < ld * NX; e += kBlock) {
    const int r = e / NX, c = e - r * NX;
    v[c * ld + r] = (r < D) ? a.phi[base + e] + a.lam[base + e] : Tf(0);
  }
  __syncthreads();
  const int i0 = ibase + wave * kUC;
  if (i0 >= k) return;
  Tf acc[kUC][NX];
#pragma unroll
  for (int u = 0; u < kUC; ++u)
#pragma unroll
    for (int c = 0; c < NX; ++c) acc[u][c] = Tf(0);
  for (int q = lane; q < nvec; q += 64) {
    V nv[kUC];
#pragma unroll
    for (int u = 0; u < kUC; ++u)
      nv[u] = (i0 + u < k) ? *reinterpret_cast<const V *>(Nj + int64_t(i0 + u) * ld + q * VN) : V(0);
    V vv[NX];
#pragma unroll
    for (int c = 0; c < NX; ++c) vv[c] = *reinterpret_cast<const V *>(v + c * ld + q * VN);
#pragma unroll
    for (int u = 0; u < kUC; ++u)
#pragma unroll
      for (int c = 0; c < NX; ++c) acc[u][c] += hsum(nv[u] * vv[c]);
  }
  Tf *tj = pu.t + pu.t_off[j];
#pragma unroll
  for (int u = 0; u < kUC; ++u)
#pragma unroll
    for (int c = 0; c < NX; ++c) {
      const Tf s = wave_sum(acc[u][c]);
      if (lane == 0 && i0 + u < k) tj[c * k + i0 + u] = s;
    }
}

template <typename Tf, int NX>
__global__ __launch_bounds__(kBlock) void psi_pass2_kernel(KArgs<Tf> a, PsiUnits<Tf> pu) {
  if (a.ctl->stop) return;
  using V = typename VecT<Tf>::type;
  constexpr int VN = VecT<Tf>::N;
  constexpr int RB = 64 * VN;  // rows per unit
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[kWaves][2 * NX];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int j = pu.p2[2 * blockIdx.x], r0 = pu.p2[2 * blockIdx.x + 1];
  const int64_t tb = a.tile_off[j];
  const int D = int(a.tile_off[j + 1] - tb) * a.rs;
  const int ld = (D + 3) & ~3;
  const int k = a.kdim[j];
  const int64_t base = tb * a.ts;
  const Tf *__restrict__ Nj = a.nb + a.nb_off[j];
  const Tf *__restrict__ Oj = a.off + a.off_ptr[j];
  Tf *ypart = reinterpret_cast<Tf *>(smem_raw);  // [kWaves][NX][RB]
  Tf *tl = ypart + kWaves * NX * RB;             // [NX][k]
  const Tf *tj = pu.t + pu.t_off[j];
  for (int e = tid; e < NX * k; e += kBlock) tl[e] = tj[e];
  __syncthreads();
  const int kq = (k + kWaves - 1) / kWaves;
  const int ib = wave * kq, ie = min(k, ib + kq);
  const int q = r0 / VN + lane;
  V y[NX];
#pragma unroll
  for (int c = 0; c < NX; ++c) y[c] = V(0);
  if (q * VN < ld) {
#pragma unroll 8
    for (int i = ib; i < ie; ++i) {
      const V nv = *reinterpret_cast<const V *>(Nj + int64_t(i) * ld + q * VN);
#pragma unroll
      for (int c = 0; c < NX; ++c) y[c] += nv * tl[c * k + i];
    }
  }
#pragma unroll
  for (int c = 0; c < NX; ++c) *reinterpret_cast<V *>(ypart + (wave * NX + c) * RB + lane * VN) = y[c];
  __syncthreads();
  const int rows = min(RB, D - r0);
  double rp[NX], rd[NX];
#pragma unroll
  for (int c = 0; c < NX; ++c) rp[c] = rd[c] = 0.0;
  for (int e = tid; e < rows * NX; e += kBlock) {
    const int rl = e / NX, c = e - rl * NX;
    Tf ys = ypart[c * RB + rl];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) ys += ypart[(w * NX + c) * RB + rl];
    const Tf psn = ys + Oj[c * ld + r0 + rl];
    const int64_t idx = base + int64_t(r0) * NX + e;
    const Tf ph = a.phi[idx], la = a.lam[idx], pso = a.psi[idx];
    a.lam[idx] = (la + ph) - psn;
    a.psi[idx] = psn;
    const double dp = double(ph - psn), dd = double(psn - pso);
#pragma unroll
    for (int cc = 0; cc < NX; ++cc)
      if (cc == c) {
        rp[cc] += dp * dp;
        rd[cc] += dd * dd;
      }
  }
#pragma unroll
  for (int c = 0; c < NX; ++c) {
    rp[c] = wave_sum(rp[c]);
    rd[c] = wave_sum(rd[c]);
  }
  if (lane == 0) {
#pragma unroll
    for (int c = 0; c < NX; ++c) {
      red[wave][c] = rp[c];
      red[wave][NX + c] = rd[c];
    }
  }
  __syncthreads();
  if (tid < 2 * NX) {
    double s = 0.0;
    for (int w = 0; w < kWaves; ++w) s += red[w][tid];
    pu.part[(int64_t(j) * pu.max_units + r0 / RB) * 2 * NX + tid] = s;
  }
}

// ------------------------------------------------------------------ structured Psi-comp
//
// Pass 1a (one block per column subsystem j): g = v_u + S_x' v_x for v = (Phi + Lambda) on
// supp(j) by the adjoint recursion mu_t = v_{x,t} + A_PP' mu_{t+1} (mu_T = 0),
// g_{t-1} = v_{u,t-1} + B_P' mu_t. Pass 1b (the dense pass 1's units of basis vectors):
// t_j = N_u' g. Pass 2 (one block per j): w = N_u t_j, the trajectory x_0 = 0,
// x_t = A_PP x_{t-1} + B_P w_{t-1} on the patch, Psi = [x; w] + o_c, then Lambda and the
// residual partial sums as in the dense pass 2 (one unit per column subsystem).

// Pass 1a: the adjoint recursion of column subsystem j (one block per j) into sa.g.
template <typename Tf, int NX>
__global__ __launch_bounds__(kBlock) void sadj_kernel(KArgs<Tf> a, SimArgs<Tf> sa) {
  if (a.ctl->stop) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int tid = threadIdx.x;
  const int j = a.psi_order[blockIdx.x];
  const int64_t tb = a.tile_off[j];
  const int p = int(a.tile_off[j + 1] - tb), rs = a.rs, nu = a.nu, T = a.T;
  const int D = p * rs, ld = (D + 3) & ~3, nxT = NX * T, nuT = nu * (T - 1);
  const int mu = p * nuT, mul = (mu + 3) & ~3, ns = p * NX;
  const int64_t base = tb * a.ts;
  Tf *v = reinterpret_cast<Tf *>(smem_raw);  // [NX][ld]
  Tf *m0 = v + NX * ld;                       // [NX][ns] adjoint state, two buffers
  Tf *m1 = m0 + NX * ns;
  Tf *g = sa.g + sa.goff[j];                  // [NX][mul]
  for (int e = tid; e < D * NX; e += kBlock) {
    const int r = e / NX, c = e - r * NX;
    v[c * ld + r] = a.phi[base + e] + a.lam[base + e];
  }
  for (int e = tid; e < NX * (mul - mu); e += kBlock) {  // zero padding rows
    const int c = e / (mul - mu);
    g[c * mul + mu + e - c * (mul - mu)] = Tf(0);
  }
  for (int e = tid; e < NX * ns; e += kBlock) m1[e] = Tf(0);
  __syncthreads();
  const int32_t *rpt = sa.rpt + sa.rp0[j];
  const int32_t *colt = sa.colt + sa.e0[j];
  const Tf *valt = sa.valt + sa.e0[j];
  Tf *mcur = m0, *mnext = m1;  // mnext holds mu_{t+1}
  for (int t = T - 1; t >= 1; --t) {
    for (int e = tid; e < ns * NX; e += kBlock) {
      const int c = e / ns, r = e - c * ns;
      const int ti = r / NX, st = r - ti * NX;
      Tf acc = v[c * ld + ti * rs + t * NX + st];
      for (int q = rpt[r]; q < rpt[r + 1]; ++q) acc += valt[q] * mnext[c * ns + colt[q]];
      mcur[c * ns + r] = acc;
    }
    __syncthreads();
    for (int e = tid; e < p * nu * NX; e += kBlock) {
      const int c = e / (p * nu), rr = e - c * p * nu;
      const int ti = rr / nu, kk = rr - ti * nu;
      const Tf *bb = sa.bblk + int64_t(sa.tile_sub[tb + ti]) * NX * nu;
      Tf acc = v[c * ld + ti * rs + nxT + (t - 1) * nu + kk];
#pragma unroll
      for (int st = 0; st < NX; ++st) acc += bb[st * nu + kk] * mcur[c * ns + ti * NX + st];
      g[c * mul + ti * nuT + (t - 1) * nu + kk] = acc;
    }
    __syncthreads();
    Tf *tmp = mcur;
    mcur = mnext;
    mnext = tmp;
  }
}

// Pass 1b: t_j = N_u' g for kP1Cols basis vectors per unit (the dense pass 1's units).
template <typename Tf, int NX>
__global__ __launch_bounds__(kBlock) void spass1_kernel(KArgs<Tf> a, PsiUnits<Tf> pu, SimArgs<Tf> sa) {
  if (a.ctl->stop) return;
  using V = typename VecT<Tf>::type;
  constexpr int VN = VecT<Tf>::N;
  constexpr int kUC = 8;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int j = pu.p1[2 * blockIdx.x], ibase = pu.p1[2 * blockIdx.x + 1];
  const int p = int(a.tile_off[j + 1] - a.tile_off[j]);
  const int mul = (p * a.nu * (a.T - 1) + 3) & ~3, nvec = mul / VN, k = a.kdim[j];
  Tf *g = reinterpret_cast<Tf *>(smem_raw);  // [NX][mul]
  const Tf *gg = sa.g + sa.goff[j];
  for (int e = tid; e < NX * mul; e += kBlock) g[e] = gg[e];
  __syncthreads();
  const int i0 = ibase + wave * kUC;
  if (i0 >= k) return;
  const Tf *__restrict__ Nu = sa.nbu + sa.nbu_off[j];
  Tf acc[kUC][NX];
#pragma unroll
  for (int u = 0; u < kUC; ++u)
#pragma unroll
    for (int c = 0; c < NX; ++c) acc[u][c] = Tf(0);
  for (int q = lane; q < nvec; q += 64) {
    V nv[kUC];
#pragma unroll
    for (int u = 0; u < kUC; ++u)
      nv[u] = (i0 + u < k) ? *reinterpret_cast<const V *>(Nu + int64_t(i0 + u) * mul + q * VN) : V(0);
    V gv[NX];
#pragma unroll
    for (int c = 0; c < NX; ++c) gv[c] = *reinterpret_cast<const V *>(g + c * mul + q * VN);
#pragma unroll
    for (int u = 0; u < kUC; ++u)
#pragma unroll
      for (int c = 0; c < NX; ++c) acc[u][c] += hsum(nv[u] * gv[c]);
  }
  Tf *tj = pu.t + pu.t_off[j];
#pragma unroll
  for (int u = 0; u < kUC; ++u)
#pragma unroll
    for (int c = 0; c < NX; ++c) {
      const Tf sm = wave_sum(acc[u][c]);
      if (lane == 0 && i0 + u < k) tj[c * k + i0 + u] = sm;
    }
}

template <typename Tf, int NX>
__global__ __launch_bounds__(kBlock) void spsi2_kernel(KArgs<Tf> a, PsiUnits<Tf> pu, SimArgs<Tf> sa) {
  if (a.ctl->stop) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[kWaves][2 * NX];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int j = a.psi_order[a.N - 1 - blockIdx.x];  // the bases pass 1 read last come first
  const int64_t tb = a.tile_off[j];
  const int p = int(a.tile_off[j + 1] - tb), rs = a.rs, nu = a.nu, T = a.T;
  const int D = p * rs, ld = (D + 3) & ~3, nxT = NX * T, nuT = nu * (T - 1);
  const int mu = p * nuT, mul = (mu + 3) & ~3, ns = p * NX, k = a.kdim[j];
  const int64_t base = tb * a.ts;
  using V = typename VecT<Tf>::type;
  constexpr int VN = VecT<Tf>::N;
  Tf *y = reinterpret_cast<Tf *>(smem_raw);  // [NX][ld] the new Psi columns on supp(j)
  Tf *tl = y + NX * ld;                       // [NX][k]
  Tf *x0b = tl + NX * k;                      // [NX][ns] trajectory state, two buffers
  Tf *x1b = x0b + NX * ns;
  const Tf *tj = pu.t + pu.t_off[j];
  for (int e = tid; e < NX * k; e += kBlock) tl[e] = tj[e];
  for (int e = tid; e < NX * ns; e += kBlock) x0b[e] = Tf(0);
  for (int e = tid; e < NX * ld; e += kBlock) y[e] = Tf(0);  // x_0 rows stay 0
  __syncthreads();
  // w = N_u t_j into the input rows of y
  const Tf *__restrict__ Nu = sa.nbu + sa.nbu_off[j];
  for (int q = tid; q < mul / VN; q += kBlock) {
    V acc[NX];
#pragma unroll
    for (int c = 0; c < NX; ++c) acc[c] = V(0);
#pragma unroll 4
    for (int i = 0; i < k; ++i) {
      const V nv = *reinterpret_cast<const V *>(Nu + int64_t(i) * mul + q * VN);
#pragma unroll
      for (int c = 0; c < NX; ++c) acc[c] += nv * tl[c * k + i];
    }
#pragma unroll
    for (int e = 0; e < VN; ++e) {
      const int u = q * VN + e;
      if (u >= mu) break;
      const int ti = u / nuT, w = u - ti * nuT;
#pragma unroll
      for (int c = 0; c < NX; ++c) y[c * ld + ti * rs + nxT + w] = acc[c][e];
    }
  }
  __syncthreads();
  const int32_t *rpp = sa.rp + sa.rp0[j];
  const int32_t *col = sa.col + sa.e0[j];
  const Tf *val = sa.val + sa.e0[j];
  Tf *xprev = x0b, *xcur = x1b;
  for (int t = 1; t < T; ++t) {
    for (int e = tid; e < ns * NX; e += kBlock) {
      const int c = e / ns, r = e - c * ns;
      const int ti = r / NX, st = r - ti * NX;
      Tf acc = Tf(0);
      for (int q = rpp[r]; q < rpp[r + 1]; ++q) acc += val[q] * xprev[c * ns + col[q]];
      const Tf *bb = sa.bblk + int64_t(sa.tile_sub[tb + ti]) * NX * nu;
      for (int kk = 0; kk < nu; ++kk) acc += bb[st * nu + kk] * y[c * ld + ti * rs + nxT + (t - 1) * nu + kk];
      xcur[c * ns + r] = acc;
      y[c * ld + ti * rs + t * NX + st] = acc;
    }
    __syncthreads();
    Tf *tmp = xprev;
    xprev = xcur;
    xcur = tmp;
  }
  // Psi = y + o_c, Lambda, residual partial sums (as the dense pass 2, all rows of j)
  const Tf *__restrict__ Oj = a.off + a.off_ptr[j];
  double rp[NX], rd[NX];
#pragma unroll
  for (int c = 0; c < NX; ++c) rp[c] = rd[c] = 0.0;
  for (int e = tid; e < D * NX; e += kBlock) {
    const int r = e / NX, c = e - r * NX;
    const Tf psn = y[c * ld + r] + Oj[c * ld + r];
    const int64_t idx = base + e;
    const Tf ph = a.phi[idx], la = a.lam[idx], pso = a.psi[idx];
    a.lam[idx] = (la + ph) - psn;
    a.psi[idx] = psn;
    const double dp = double(ph - psn), dd = double(psn - pso);
#pragma unroll
    for (int cc = 0; cc < NX; ++cc)
      if (cc == c) {
        rp[cc] += dp * dp;
        rd[cc] += dd * dd;
      }
  }
#pragma unroll
  for (int c = 0; c < NX; ++c) {
    rp[c] = wave_sum(rp[c]);
    rd[c] = wave_sum(rd[c]);
  }
  if (lane == 0) {
#pragma unroll
    for (int c = 0; c < NX; ++c) {
      red[wave][c] = rp[c];
      red[wave][NX + c] = rd[c];
    }
  }
  __syncthreads();
  if (tid < 2 * NX) {
    double sm = 0.0;
    for (int w = 0; w < kWaves; ++w) sm += red[w][tid];
    pu.part[int64_t(j) * pu.max_units * 2 * NX + tid] = sm;
  }
}

// Input rows of every null basis, gathered into the structured Psi-comp's layout.
template <typename Tf>
__global__ __launch_bounds__(kBlock) void gather_nu_kernel(KArgs<Tf> a, SimArgs<Tf> sa) {
  const int j = blockIdx.x;
  const int p = int(a.tile_off[j + 1] - a.tile_off[j]), rs = a.rs;
  const int D = p * rs, ld = (D + 3) & ~3, nxT = a.nx * a.T, nuT = a.nu * (a.T - 1);
  const int mu = p * nuT, mul = (mu + 3) & ~3, k = a.kdim[j];
  const Tf *Nj = a.nb + a.nb_off[j];
  Tf *Nu = const_cast<Tf *>(sa.nbu) + sa.nbu_off[j];
  for (int64_t e = threadIdx.x; e < int64_t(k) * mul; e += kBlock) {
    const int i = int(e / mul), u = int(e - int64_t(i) * mul);
    Tf vv = Tf(0);
    if (u < mu) {
      const int ti = u / nuT, w = u - ti * nuT;
      vv = Nj[int64_t(i) * ld + ti * rs + nxT + w];
    }
    Nu[e] = vv;
  }
}

constexpr int kConvBlock = 1024;

template <typename Tf, int NX>
__global__ __launch_bounds__(kConvBlock) void conv_kernel(KArgs<Tf> a, PsiUnits<Tf> pu) {
  if (a.ctl->stop) return;
  constexpr int kCW = kConvBlock / 64;
  __shared__ double redp[kCW], redd[kCW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double mp = 0.0, md = 0.0;
  for (int j = tid; j < a.N; j += kConvBlock) {
    // j's pass-2 units own slots [j * max_units, (j + 1) * max_units); unused slots hold zeros
    const double *pj = pu.part + int64_t(j) * pu.max_units * 2 * NX;
#pragma unroll
    for (int c = 0; c < NX; ++c) {
      double sp = 0.0, sd = 0.0;
      for (int u = 0; u < pu.max_units; ++u) {
        sp += pj[u * 2 * NX + c];
        sd += pj[u * 2 * NX + NX + c];
      }
      sp = sqrt(sp);
      sd = sqrt(sd);
      mp = (sp > mp || sp != sp) ? sp : mp;
      md = (sd > md || sd != sd) ? sd : md;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double op = __shfl_xor(mp, o, 64), od = __shfl_xor(md, o, 64);
    mp = (op > mp || op != op) ? op : mp;
    md = (od > md || od != od) ? od : md;
  }
  if (lane == 0) {
    redp[wave] = mp;
    redd[wave] = md;
  }
  __syncthreads();
  if (tid == 0) {
    for (int w = 1; w < kCW; ++w) {
      mp = (redp[w] > mp || redp[w] != redp[w]) ? redp[w] : mp;
      md = (redd[w] > md || redd[w] != redd[w]) ? redd[w] : md;
    }
    decide(a.ctl, a.ctl->iters + 1, mp, md);
  }
}

// ------------------------------------------------------------------ persistent schedule

// Grid-wide barrier of the persistent schedule (the grid is sized to be co-resident). Sense is
// carried by a generation counter. Each block releases its writes once before arriving and
// acquires once after the generation moves; the wait itself polls with relaxed loads so that
// it does not disturb the caches of blocks still working. The wait is bounded: a block that
// times out flags the control block and reports failure, and every other block then leaves
// at its next barrier.
__device__ __forceinline__ bool grid_barrier(Ctl *c, unsigned nblocks) {
  __shared__ int ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned my_gen = __hip_atomic_load(&c->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const unsigned arrived = __hip_atomic_fetch_add(&c->bar_count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int good = 1;
    if (arrived == nblocks - 1) {
      __hip_atomic_store(&c->bar_count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(&c->bar_gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      unsigned long long n = 0;
      while (__hip_atomic_load(&c->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == my_gen) {
        if (__hip_atomic_load(&c->bar_fail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u ||
            ++n > kSpinLimit) {
          __hip_atomic_store(&c->bar_fail, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          good = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    ok = good;
  }
  __syncthreads();
  return ok != 0;
}

// All ADMM iterations of one solve in one launch: block b runs Phi-comp for the
// row subsystems of its static list, a grid barrier, Psi-comp/Lambda/Conv for its column
// subsystems, a grid barrier, then every block reads the same reduced residuals and takes
// the same stop decision (Section V: several ADMM iterations inside one kernel).
// kTune only gives the schedule-timing launches of dlmpc_setup their own symbol, so that
// kernel traces separate them from solves.
template <typename Tf, int NX, bool kTune>
__global__ __launch_bounds__(kBlock) void persistent_kernel(KArgs<Tf> a, Sched s) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  Ctl *c = a.ctl;
  const unsigned G = gridDim.x;
  const int b = blockIdx.x;
  const int max_iter = c->max_iter;
  const double eps = c->eps;
  for (int it = 0;;) {
    for (int q = s.phi_ptr[b]; q < s.phi_ptr[b + 1]; ++q) {
      phi_body<Tf, NX>(a, s.phi_list[q], smem_raw);
      __syncthreads();
    }
    if (!grid_barrier(c, G)) return;
    const int slot = it & 1;
    if (b == 0 && threadIdx.x == 0) {  // the other slot was last read before this barrier
      atomicExch(&c->slot_rp[slot ^ 1], 0ull);
      atomicExch(&c->slot_rd[slot ^ 1], 0ull);
    }
    double mp = 0.0, md = 0.0;
    for (int q = s.psi_ptr[b]; q < s.psi_ptr[b + 1]; ++q) {
      double p1 = 0.0, d1 = 0.0;
      psi_body<Tf, NX>(a, s.psi_list[q], smem_raw, &p1, &d1);
      if (threadIdx.x == 0) {
        mp = (p1 > mp || p1 != p1) ? p1 : mp;
        md = (d1 > md || d1 != d1) ? d1 : md;
      }
    }
    if (threadIdx.x == 0 && s.psi_ptr[b + 1] > s.psi_ptr[b]) {
      atomicMax(&c->slot_rp[slot], as_bits(mp));
      atomicMax(&c->slot_rd[slot], as_bits(md));
    }
    if (!grid_barrier(c, G)) return;
    __shared__ int stop_s;
    ++it;
    if (threadIdx.x == 0) {
      const double rpm = __longlong_as_double(static_cast<long long>(
          __hip_atomic_load(&c->slot_rp[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)));
      const double rdm = __longlong_as_double(static_cast<long long>(
          __hip_atomic_load(&c->slot_rd[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)));
      const bool bad = !(rpm == rpm) || !(rdm == rdm) || isinf(rpm) || isinf(rdm);
      const int stop = bad || (rpm <= eps && rdm <= eps) || it >= max_iter;
      if (b == 0 && stop) decide(c, it, rpm, rdm);
      stop_s = stop;
    }
    __syncthreads();
    if (stop_s) return;
  }
}

// ------------------------------------------------------------------ outputs

// u(0) = the u_0 rows of Phi x0 (Algorithm 1: compute u(t) from Phi) and the FP64 objective
// sum_r w_r y_r^2 at the stopping iterate. One workgroup.
template <typename Tf, int NX>
__global__ __launch_bounds__(kBlock) void output_kernel(KArgs<Tf> a, const double *w64, double *u0) {
  __shared__ double red[kWaves];
  const int tid = threadIdx.x;
  const int64_t ny = int64_t(a.N) * a.rs;
  double acc = 0.0;
  for (int64_t i = tid; i < ny; i += kBlock) {
    const double yv = double(a.y[i]);
    acc += w64[i] * yv * yv;
  }
  acc = wave_sum(acc);
  if ((tid & 63) == 0) red[tid >> 6] = acc;
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
    for (int w = 0; w < kWaves; ++w) s += red[w];
    a.ctl->objective = s;
  }
  const int nu = a.nu;
  for (int i = tid; i < a.N * nu; i += kBlock) {
    const int m = i / nu, q = i - m * nu;
    u0[i] = double(a.y[int64_t(m) * a.rs + NX * a.T + q]);
  }
}

template <typename Tf>
__global__ __launch_bounds__(kBlock) void export_kernel(const Tf *phi, const int64_t *map, int64_t n,
                                                        double *out) {
  for (int64_t e = blockIdx.x * int64_t(kBlock) + threadIdx.x; e < n; e += int64_t(gridDim.x) * kBlock)
    out[map[e]] = double(phi[e]);
}

// ------------------------------------------------------------------ engine

#define ENG_CHECK(expr)                                                   \
  do {                                                                    \
    hipError_t e_ = (expr);                                               \
    if (e_ != hipSuccess) {                                               \
      err = std::string(#expr) + ": " + hipGetErrorString(e_);            \
      return DLMPC_EDEVICE;                                               \
    }                                                                     \
  } while (0)

// ------------------------------------------------------------------ FP64 certificate

struct CertArgs {
  const int64_t *eq_ptr;    // [N+1] entries (subsystems i of the support and ring) of column j
  const int32_t *eq_sub;    // subsystem i
  const int64_t *eq_tile;   // tile (j, i), or -1 when i is in the ring
  const int64_t *eq_nptr;   // [entries+1] A neighbours of i (CSR order of A)
  const int64_t *eq_ntile;  // tile (j, k) of neighbour k, or -1
  const int64_t *eq_ablk;   // position of the block A_ik in the block-CSR arrays
  const double *a_blk, *b_blk, *x0;
  unsigned long long *out;  // [5] maxima as ordered bit patterns (all values >= 0)
};

// One block per subsystem b: Z_AB feasibility, |Phi - Psi| and Psi-step stationarity of column
// block j = b, and the bound check of the rows of row subsystem m = b, all in FP64.
template <typename Tf, int NX>
__global__ __launch_bounds__(kBlock) void cert_kernel(KArgs<Tf> a, CertArgs c) {
  extern __shared__ double tk[];  // [NX][k_j]
  __shared__ double red[kBlock / 64][NX + 4];
  const int j = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int rs = a.rs, T = a.T, nu = a.nu, ts = a.ts;
  double m_eq = 0.0, m_pf = 0.0, m_box = 0.0, m_stat = 0.0, s2[NX];
#pragma unroll
  for (int q = 0; q < NX; ++q) s2[q] = 0.0;
  // Z_AB Psi = I on the rows that can touch j's columns
  const int64_t e0 = c.eq_ptr[j], e1 = c.eq_ptr[j + 1];
  const int64_t per = int64_t(T) * NX * NX;
  for (int64_t w = tid; w < (e1 - e0) * per; w += kBlock) {
    const int64_t q = e0 + w / per;
    const int rem = int(w % per), t = rem / (NX * NX), comp = (rem / NX) % NX, col = rem % NX;
    const int i = c.eq_sub[q];
    const int64_t ti = c.eq_tile[q];
    double r = ti < 0 ? 0.0 : double(a.psi[ti * ts + (t * NX + comp) * NX + col]);
    if (t == 0) {
      if (i == j && comp == col) r -= 1.0;
    } else {
      for (int64_t n = c.eq_nptr[q]; n < c.eq_nptr[q + 1]; ++n) {
        const int64_t tk_ = c.eq_ntile[n];
        if (tk_ < 0) continue;
        const double *A = c.a_blk + c.eq_ablk[n] * NX * NX;
#pragma unroll
        for (int cc = 0; cc < NX; ++cc) r -= A[comp * NX + cc] * double(a.psi[tk_ * ts + ((t - 1) * NX + cc) * NX + col]);
      }
      if (ti >= 0)
        for (int u = 0; u < nu; ++u)
          r -= c.b_blk[(int64_t(i) * NX + comp) * nu + u] * double(a.psi[ti * ts + (NX * T + (t - 1) * nu + u) * NX + col]);
    }
    m_eq = fmax(m_eq, fabs(r));
  }
  // Phi - Psi on j's support
  const int64_t t0 = a.tile_off[j], t1 = a.tile_off[j + 1];
  for (int64_t e = tid; e < (t1 - t0) * ts; e += kBlock) {
    const int64_t idx = t0 * ts + e;
    const double d = double(a.phi[idx]) - double(a.psi[idx]);
    m_pf = fmax(m_pf, fabs(d));
    s2[e % NX] += d * d;
  }
  // N_j N_j' (rho Lambda_c): coordinates first, then the rows
  const int D = int(t1 - t0) * rs, ld = (D + 3) & ~3, k = a.kdim[j];
  const Tf *Nj = a.nb + a.nb_off[j];
  const double rho = a.ctl->rho;
  // one wave per basis vector i: lanes over the rows (coalesced column reads), wave reduction
  for (int i = wave; i < k; i += kBlock / 64) {
    double acc[NX];
#pragma unroll
    for (int col = 0; col < NX; ++col) acc[col] = 0.0;
    for (int r = lane; r < D; r += 64) {
      const double n = double(Nj[int64_t(i) * ld + r]);
#pragma unroll
      for (int col = 0; col < NX; ++col) acc[col] += n * rho * double(a.lam[t0 * ts + int64_t(r) * NX + col]);
    }
#pragma unroll
    for (int col = 0; col < NX; ++col) {
      double v = acc[col];
      for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
      if (lane == 0) tk[col * k + i] = v;
    }
  }
  __syncthreads();
  // rows over the threads (consecutive rows, consecutive addresses), four basis vectors in flight
  for (int r = tid; r < D; r += kBlock) {
    double acc[NX];
#pragma unroll
    for (int col = 0; col < NX; ++col) acc[col] = 0.0;
    int i = 0;
    for (; i + 4 <= k; i += 4) {
      double n[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) n[u] = double(Nj[int64_t(i + u) * ld + r]);
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int col = 0; col < NX; ++col) acc[col] += n[u] * tk[col * k + i + u];
    }
    for (; i < k; ++i)
#pragma unroll
      for (int col = 0; col < NX; ++col) acc[col] += double(Nj[int64_t(i) * ld + r]) * tk[col * k + i];
#pragma unroll
    for (int col = 0; col < NX; ++col) m_stat = fmax(m_stat, fabs(acc[col]));
  }
  // bounds of row subsystem m = j: y = Phi x0 recomputed from the tiles of m's row
  const int m = j;
  for (int l = tid; l < rs; l += kBlock) {
    double y = 0.0;
    for (int64_t q = a.rt_ptr[m]; q < a.rt_ptr[m + 1]; ++q) {
      const int64_t tile = a.rt_tile[q];
      const int jj = a.rt_col[q];
#pragma unroll
      for (int cc = 0; cc < NX; ++cc) y += double(a.phi[tile * ts + int64_t(l) * NX + cc]) * c.x0[jj * NX + cc];
    }
    const double lbv = double(a.lb[int64_t(m) * rs + l]), ubv = double(a.ub[int64_t(m) * rs + l]);
    m_box = fmax(m_box, fmax(lbv - y, y - ubv));
  }
  // block maxima and column sums, then the device maxima
  auto wmax = [](double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
  };
  auto wsum_ = [](double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
  };
  m_eq = wmax(m_eq);
  m_pf = wmax(m_pf);
  m_box = wmax(m_box);
  m_stat = wmax(m_stat);
#pragma unroll
  for (int q = 0; q < NX; ++q) s2[q] = wsum_(s2[q]);
  if (lane == 0) {
    red[wave][0] = m_eq;
    red[wave][1] = m_pf;
    red[wave][2] = m_box;
    red[wave][3] = m_stat;
#pragma unroll
    for (int q = 0; q < NX; ++q) red[wave][4 + q] = s2[q];
  }
  __syncthreads();
  if (tid == 0) {
    double v[4] = {0.0, 0.0, 0.0, 0.0}, cs[NX];
#pragma unroll
    for (int q = 0; q < NX; ++q) cs[q] = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) {
      for (int q = 0; q < 4; ++q) v[q] = fmax(v[q], red[w][q]);
      for (int q = 0; q < NX; ++q) cs[q] += red[w][4 + q];
    }
    double rp = 0.0;
    for (int q = 0; q < NX; ++q) rp = fmax(rp, sqrt(cs[q]));
    atomicMax(&c.out[0], as_bits(v[0]));
    atomicMax(&c.out[1], as_bits(v[1]));
    atomicMax(&c.out[2], as_bits(rp));
    atomicMax(&c.out[3], as_bits(fmax(v[2], 0.0)));
    atomicMax(&c.out[4], as_bits(v[3]));
  }
}

// dst = src converted to Tf (device arrays of n values).
template <typename Tf>
__global__ void convert_kernel(const double *__restrict__ src, Tf *__restrict__ dst, int64_t n) {
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n; e += int64_t(gridDim.x) * blockDim.x)
    dst[e] = Tf(src[e]);
}

template <typename Tf, int NX>
class EngineT final : public Engine {
 public:
  int init(const HostSetup &hs, double rho, hipStream_t s, std::string &err) override {
    hs_ = &hs;
    stream_ = s;
    KArgs<Tf> &a = args_;
    a.N = hs.N;
    a.nx = hs.nx;
    a.nu = hs.nu;
    a.T = hs.T;
    a.rs = hs.rs;
    a.ts = hs.ts;
    int rc;
    if ((rc = upload(hs.tile_off, &a.tile_off, err))) return rc;
    if ((rc = upload(hs.rt_ptr, &a.rt_ptr, err))) return rc;
    if ((rc = upload(hs.rt_tile, &a.rt_tile, err))) return rc;
    if ((rc = upload(hs.rt_col, &a.rt_col, err))) return rc;
    if ((rc = upload(hs.kdim, &a.kdim, err))) return rc;
    if ((rc = upload(hs.nb_off, &a.nb_off, err))) return rc;
    if ((rc = upload(hs.off_ptr, &a.off_ptr, err))) return rc;
    {
      // Launch order: largest patches first (they bound each kernel's duration).
      std::vector<int32_t> po(hs.N), so(hs.N);
      for (int i = 0; i < hs.N; ++i) po[i] = so[i] = i;
      std::stable_sort(po.begin(), po.end(), [&](int32_t x, int32_t y) { return hs.patch[x].size() > hs.patch[y].size(); });
      std::stable_sort(so.begin(), so.end(), [&](int32_t x, int32_t y) {
        return double(hs.patch[x].size()) * (hs.kdim[x] + 4) > double(hs.patch[y].size()) * (hs.kdim[y] + 4);
      });
      if ((rc = upload(po, &a.phi_order, err))) return rc;
      if ((rc = upload(so, &a.psi_order, err))) return rc;
    }
    if ((rc = upload(hs.csr_map, &map_, err))) return rc;
    if (hs.d_nb) {
      // bases on the device (device factorisation): convert there
      const int64_t n = hs.nb_off[hs.N];
      Tf *p = nullptr;
      if ((rc = alloc(&p, size_t(n), err))) return rc;
      hipLaunchKernelGGL(convert_kernel<Tf>, dim3(2048), dim3(256), 0, stream_, hs.d_nb, p, n);
      ENG_CHECK(hipGetLastError());
      ENG_CHECK(hipStreamSynchronize(stream_));
      a.nb = p;
    } else if ((rc = upload_conv(hs.nb, &a.nb, err))) {
      return rc;
    }
    if ((rc = upload_conv(hs.off, &a.off, err))) return rc;
    if ((rc = upload_conv(hs.w, &a.w, err))) return rc;
    if ((rc = upload_conv(hs.lb, &a.lb, err))) return rc;
    if ((rc = upload_conv(hs.ub, &a.ub, err))) return rc;
    if ((rc = upload(hs.w, &w64_, err))) return rc;
    const size_t nst = size_t(hs.n_tiles) * hs.ts;
    if ((rc = alloc(&a.phi, nst, err))) return rc;
    if ((rc = alloc(&a.psi, nst, err))) return rc;
    if ((rc = alloc(&a.lam, nst, err))) return rc;
    if ((rc = alloc(&a.x0f, size_t(hs.N) * NX, err))) return rc;
    if ((rc = alloc(&a.nrm, size_t(hs.N), err))) return rc;
    if ((rc = alloc(&a.y, size_t(hs.N) * hs.rs, err))) return rc;
    if ((rc = alloc(&a.ctl, 1, err))) return rc;
    lds_phi_ = (size_t((hs.p_max * NX + 3) & ~3) + size_t(kWaves) * 64 + 64) * sizeof(Tf);
    lds_psi_ = (size_t(NX) * padded_ld(hs.d_col_max) + size_t(NX) * hs.k_max) * sizeof(Tf);
    if (lds_phi_ > kMaxLds || lds_psi_ > kMaxLds) {
      err = "patch too large for the on-chip staging of this build (LDS " + std::to_string(lds_psi_) + " B)";
      return DLMPC_EINVAL;
    }
    int rc2 = build_units(hs, err);
    if (!rc2) rc2 = build_cert(hs, err);
    if (rc2) return rc2;
    return build_schedule(hs, err);
  }

  // Work units of the split Psi-comp, larger work first.
  int build_units(const HostSetup &hs, std::string &err) {
    constexpr int RB = 64 * VecT<Tf>::N;
    std::vector<int32_t> order(hs.N);
    for (int i = 0; i < hs.N; ++i) order[i] = i;
    auto D_of = [&](int j) { return int(hs.patch[j].size()) * hs.rs; };
    std::vector<int32_t> p1, p2, first(hs.N), count(hs.N);
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return D_of(x) > D_of(y); });
    for (int j : order)
      for (int i0 = 0; i0 < hs.kdim[j]; i0 += kP1Cols) {
        p1.push_back(j);
        p1.push_back(i0);
      }
    // Pass 2 visits the subsystems in the reverse order of pass 1, so that it starts on the
    // null bases pass 1 streamed last (the ones most likely still in the memory-side cache).
    std::reverse(order.begin(), order.end());
    for (int j : order) {
      first[j] = int32_t(p2.size() / 2);
      for (int r0 = 0; r0 < D_of(j); r0 += RB) {
        p2.push_back(j);
        p2.push_back(r0);
      }
      count[j] = int32_t(p2.size() / 2) - first[j];
    }
    n1_ = int(p1.size() / 2);
    n2_ = int(p2.size() / 2);
    std::vector<int64_t> toff(hs.N + 1, 0);
    for (int j = 0; j < hs.N; ++j) toff[j + 1] = toff[j] + int64_t(hs.kdim[j]) * NX;
    int rc;
    if ((rc = upload(p1, &pu_.p1, err))) return rc;
    if ((rc = upload(p2, &pu_.p2, err))) return rc;
    if ((rc = upload(first, &pu_.p2_first, err))) return rc;
    if ((rc = upload(count, &pu_.p2_count, err))) return rc;
    if ((rc = upload(toff, &pu_.t_off, err))) return rc;
    if ((rc = alloc(&pu_.t, size_t(toff[hs.N]), err))) return rc;
    t_len_ = size_t(toff[hs.N]);
    int max_units = 1;
    for (int j = 0; j < hs.N; ++j) max_units = std::max(max_units, count[j]);
    pu_.max_units = max_units;
    if ((rc = alloc(&pu_.part, size_t(hs.N) * max_units * 2 * NX, err))) return rc;
    ENG_CHECK(hipMemset(pu_.part, 0, sizeof(double) * size_t(hs.N) * max_units * 2 * NX));
    lds_p1_ = size_t(NX) * padded_ld(hs.d_col_max) * sizeof(Tf);
    lds_p2_ = (size_t(kWaves) * NX * RB + size_t(NX) * hs.k_max) * sizeof(Tf);
    if (lds_p1_ > kMaxLds || lds_p2_ > kMaxLds) {
      err = "patch too large for the on-chip staging of this build";
      return DLMPC_EINVAL;
    }
    return DLMPC_OK;
  }

  // Persistent schedule: as many blocks as can be co-resident (at most one per subsystem),
  // work lists by longest-processing-time-first greedy assignment of the per-subsystem work.
  int build_schedule(const HostSetup &hs, std::string &err) {
    int dev = 0, ncu = 0, per_cu = 0;
    ENG_CHECK(hipGetDevice(&dev));
    ENG_CHECK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    const size_t lds = std::max(lds_phi_, lds_psi_);
    ENG_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, persistent_kernel<Tf, NX, false>, kBlock, lds));
    // Every block must be resident at once for the grid barrier; stay below the occupancy
    // bound (one block per CU less) so that a co-scheduled kernel cannot starve the grid.
    grid_ = per_cu > 0 ? std::min(hs.N, std::max(1, per_cu * ncu - ncu)) : 0;
    lds_persist_ = lds;
    if (grid_ == 0) return DLMPC_OK;
    auto lpt = [&](const std::vector<double> &work, std::vector<int32_t> &ptr, std::vector<int32_t> &list) {
      std::vector<int32_t> order(work.size());
      for (size_t i = 0; i < order.size(); ++i) order[i] = int32_t(i);
      std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return work[x] > work[y]; });
      std::vector<double> load(grid_, 0.0);
      std::vector<std::vector<int32_t>> per(grid_);
      for (int32_t t : order) {
        const int b = int(std::min_element(load.begin(), load.end()) - load.begin());
        load[b] += work[t];
        per[b].push_back(t);
      }
      ptr.assign(grid_ + 1, 0);
      list.clear();
      for (int b = 0; b < grid_; ++b) {
        list.insert(list.end(), per[b].begin(), per[b].end());
        ptr[b + 1] = int32_t(list.size());
      }
    };
    std::vector<double> wphi(hs.N), wpsi(hs.N);
    for (int j = 0; j < hs.N; ++j) {
      const double p = double(hs.patch[j].size());
      wphi[j] = p * hs.rs * NX + 256.0;
      wpsi[j] = p * hs.rs * (2.0 * hs.kdim[j] + 8.0 * NX) + 1024.0;
    }
    std::vector<int32_t> pp, pl, sp, sl;
    lpt(wphi, pp, pl);
    lpt(wpsi, sp, sl);
    int rc;
    if ((rc = upload(pp, &sched_.phi_ptr, err))) return rc;
    if ((rc = upload(pl, &sched_.phi_list, err))) return rc;
    if ((rc = upload(sp, &sched_.psi_ptr, err))) return rc;
    if ((rc = upload(sl, &sched_.psi_list, err))) return rc;
    return DLMPC_OK;
  }

  int run_persistent(bool tune, std::string &err) override {
    if (grid_ == 0) {
      err = "device cannot co-schedule the persistent grid";
      return DLMPC_EDEVICE;
    }
    if (tune)
      hipLaunchKernelGGL((persistent_kernel<Tf, NX, true>), dim3(grid_), dim3(kBlock), lds_persist_, stream_,
                         args_, sched_);
    else
      hipLaunchKernelGGL((persistent_kernel<Tf, NX, false>), dim3(grid_), dim3(kBlock), lds_persist_, stream_,
                         args_, sched_);
    ENG_CHECK(hipGetLastError());
    return DLMPC_OK;
  }

  int persistent_grid() const override { return grid_; }

  int precompute(const double *x0_dev, const double *wpsi, const double *wlam, int max_iter,
                 double eps, double rho, std::string &err) override {
    const int cold = (wpsi == nullptr);
    hipLaunchKernelGGL((precompute_kernel<Tf, NX>), dim3(hs_->N), dim3(kBlock), 0, stream_, args_,
                       x0_dev, cold, max_iter, eps, rho);
    ENG_CHECK(hipGetLastError());
    if (cp_.E > 0) {  // nested ADMM copies and duals start at zero in every solve
      for (Tf *v : {cp_.za, cp_.zb, cp_.la, cp_.lb})
        ENG_CHECK(hipMemsetAsync(v, 0, sizeof(Tf) * size_t(cp_.E), stream_));
    }
    if (!cold) {
      const int64_t n = int64_t(hs_->n_tiles) * hs_->ts;
      const int g = int(std::min<int64_t>((n + kBlock - 1) / kBlock, 4096));
      hipLaunchKernelGGL((warm_kernel<Tf>), dim3(g), dim3(kBlock), 0, stream_, args_.psi, args_.lam,
                         map_, n, wpsi, wlam);
      ENG_CHECK(hipGetLastError());
    }
    return DLMPC_OK;
  }

  int iteration(std::string &err) override {
    for (int kk = 0; kk < kNumIterKernels; ++kk) {
      const int rc = launch_one(kk, err);
      if (rc) return rc;
    }
    return DLMPC_OK;
  }
  // Kernels of one iteration in order: 0 Phi-comp, 1 Psi pass 1, 2 Psi pass 2, 3 Conv.
  int launch_one(int which, std::string &err) override {
    switch (which) {
      case 0:
        hipLaunchKernelGGL((phi_kernel<Tf, NX>), dim3(hs_->N), dim3(kBlock), lds_phi_, stream_, args_);
        if (cp_.K > 0) {
          ENG_CHECK(hipGetLastError());
          hipLaunchKernelGGL((coupled_inner_kernel<Tf, NX>), dim3(1), dim3(1024), 0, stream_, args_, cp_);
          ENG_CHECK(hipGetLastError());
          hipLaunchKernelGGL((coupled_fix_kernel<Tf, NX>), dim3((cp_.K + 255) / 256), dim3(256), 0, stream_, args_,
                             cp_);
        }
        break;
      case 1:
        if (structured_) {
          hipLaunchKernelGGL((sadj_kernel<Tf, NX>), dim3(hs_->N), dim3(kBlock), lds_s1_, stream_, args_, sa_);
          ENG_CHECK(hipGetLastError());
          hipLaunchKernelGGL((spass1_kernel<Tf, NX>), dim3(n1_), dim3(kBlock), lds_s1b_, stream_, args_, spu_, sa_);
        } else
          hipLaunchKernelGGL((psi_pass1_kernel<Tf, NX>), dim3(n1_), dim3(kBlock), lds_p1_, stream_, args_, pu_);
        break;
      case 2:
        if (structured_)
          hipLaunchKernelGGL((spsi2_kernel<Tf, NX>), dim3(hs_->N), dim3(kBlock), lds_s2_, stream_, args_, spu_, sa_);
        else
          hipLaunchKernelGGL((psi_pass2_kernel<Tf, NX>), dim3(n2_), dim3(kBlock), lds_p2_, stream_, args_, pu_);
        break;
      default:
        hipLaunchKernelGGL((conv_kernel<Tf, NX>), dim3(1), dim3(kConvBlock), 0, stream_, args_, structured_ ? spu_ : pu_);
        break;
    }
    ENG_CHECK(hipGetLastError());
    return DLMPC_OK;
  }

  void set_structured(bool on) override { structured_ = on && struct_ready_; }

  int enable_structured(std::string &err) override {
    if (struct_ready_) {
      structured_ = true;
      return DLMPC_OK;
    }
    const HostSetup &hs = *hs_;
    const int N = hs.N, nx = hs.nx, nu = hs.nu, T = hs.T;
    const int nuT = nu * (T - 1);
    std::vector<int64_t> nbu_off(N + 1, 0), rp0(N), e0(N), goff(N + 1, 0);
    std::vector<int32_t> rp, rpt, col, colt;
    std::vector<Tf> val, valt;
    size_t lds1 = 0, lds1b = 0, lds2 = 0;
    for (int j = 0; j < N; ++j) {
      const std::vector<int32_t> &P = hs.patch[j];
      const int p = int(P.size()), ns = p * nx, mu = p * nuT, mul = (mu + 3) & ~3;
      const int ld = padded_ld(p * hs.rs);
      nbu_off[j + 1] = nbu_off[j] + int64_t(mul) * hs.kdim[j];
      goff[j + 1] = goff[j] + int64_t(nx) * mul;
      lds1 = std::max(lds1, size_t(nx) * (ld + 2 * ns) * sizeof(Tf));
      lds1b = std::max(lds1b, size_t(nx) * mul * sizeof(Tf));
      lds2 = std::max(lds2, size_t(nx) * (ld + hs.kdim[j] + 2 * ns) * sizeof(Tf));
      // A_PP: rows and columns are the patch states (member position * nx + state)
      std::vector<std::vector<std::pair<int32_t, double>>> rows(ns), cols(ns);
      for (int ti = 0; ti < p; ++ti) {
        const int m = P[ti];
        for (int64_t q = hs.a_rowptr[m]; q < hs.a_rowptr[m + 1]; ++q) {
          const auto it = std::lower_bound(P.begin(), P.end(), hs.a_colidx[q]);
          if (it == P.end() || *it != hs.a_colidx[q]) continue;  // outside the patch: state is 0
          const int tn = int(it - P.begin());
          for (int st = 0; st < nx; ++st)
            for (int s2 = 0; s2 < nx; ++s2) {
              const double v = hs.a_blocks[size_t(q) * nx * nx + st * nx + s2];
              if (v == 0.0) continue;
              rows[ti * nx + st].push_back({tn * nx + s2, v});
              cols[tn * nx + s2].push_back({ti * nx + st, v});
            }
        }
      }
      rp0[j] = int64_t(rp.size());
      e0[j] = int64_t(col.size());
      int32_t c0 = 0, c1 = 0;
      rp.push_back(0);
      rpt.push_back(0);
      for (int r = 0; r < ns; ++r) {
        for (const auto &e : rows[r]) {
          col.push_back(e.first);
          val.push_back(static_cast<Tf>(e.second));
        }
        for (const auto &e : cols[r]) {
          colt.push_back(e.first);
          valt.push_back(static_cast<Tf>(e.second));
        }
        c0 += int32_t(rows[r].size());
        c1 += int32_t(cols[r].size());
        rp.push_back(c0);
        rpt.push_back(c1);
      }
    }
    if (lds1 > kMaxLds || lds2 > kMaxLds) {
      err = "patch too large for the on-chip staging of the structured Psi-comp";
      return DLMPC_EINVAL;
    }
    std::vector<Tf> bb(hs.b_blocks.begin(), hs.b_blocks.end());
    SimArgs<Tf> x{};
    int rc;
    Tf *nbu = nullptr;
    if ((rc = upload(nbu_off, &x.nbu_off, err)) || (rc = alloc(&nbu, size_t(nbu_off[N]), err)) ||
        (rc = upload(rp0, &x.rp0, err)) || (rc = upload(rp, &x.rp, err)) || (rc = upload(rpt, &x.rpt, err)) ||
        (rc = upload(e0, &x.e0, err)) || (rc = upload(col, &x.col, err)) || (rc = upload(colt, &x.colt, err)) ||
        (rc = upload(val, &x.val, err)) || (rc = upload(valt, &x.valt, err)) || (rc = upload(bb, &x.bblk, err)) ||
        (rc = upload(hs.tile_rsub, &x.tile_sub, err)) || (rc = upload(goff, &x.goff, err)) ||
        (rc = alloc(&x.g, size_t(goff[N]), err)))
      return rc;
    x.nbu = nbu;
    hipLaunchKernelGGL(gather_nu_kernel<Tf>, dim3(N), dim3(kBlock), 0, stream_, args_, x);
    ENG_CHECK(hipGetLastError());
    ENG_CHECK(hipStreamSynchronize(stream_));
    spu_ = pu_;
    spu_.max_units = 1;
    if ((rc = alloc(&spu_.part, size_t(N) * 2 * NX, err))) return rc;
    ENG_CHECK(hipMemset(spu_.part, 0, sizeof(double) * size_t(N) * 2 * NX));
    sa_ = x;
    lds_s1_ = lds1;
    lds_s1b_ = lds1b;
    lds_s2_ = lds2;
    struct_ready_ = structured_ = true;
    return DLMPC_OK;
  }

  int set_coupling(int n, const int64_t *row_a, const int64_t *row_b, const double *lo, const double *hi,
                   double sigma, int inner_max, double inner_eps, std::string &err) override {
    ENG_CHECK(hipStreamSynchronize(stream_));
    cp_ = CoupleArgs<Tf>{};
    args_.cp_slot = nullptr;
    args_.cp_a = args_.cp_s0 = nullptr;
    if (n == 0) return DLMPC_OK;
    const int64_t R = int64_t(hs_->N) * hs_->rs;
    // coupled rows in order of first appearance; pairs of every coupled row (CSR)
    std::vector<int32_t> slot(size_t(R), -1), ka(n), kb(n);
    std::vector<int64_t> rows;
    auto idx = [&](int64_t o) {
      if (slot[o] < 0) {
        slot[o] = int32_t(rows.size());
        rows.push_back(o);
      }
      return slot[o];
    };
    for (int e = 0; e < n; ++e) {
      ka[e] = idx(row_a[e]);
      kb[e] = idx(row_b[e]);
    }
    const int K = int(rows.size());
    std::vector<int32_t> sub(K), ptr(K + 1, 0), ent(2 * size_t(n));
    for (int k = 0; k < K; ++k) sub[k] = int32_t(rows[k] / hs_->rs);
    for (int e = 0; e < n; ++e) {
      ++ptr[ka[e] + 1];
      ++ptr[kb[e] + 1];
    }
    for (int k = 0; k < K; ++k) ptr[k + 1] += ptr[k];
    std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
    // at every row: its first-row pairs in ascending order, then its second-row pairs
    for (int e = 0; e < n; ++e) ent[fill[ka[e]]++] = 2 * e;
    for (int e = 0; e < n; ++e) ent[fill[kb[e]]++] = 2 * e + 1;
    const std::vector<double> vlo(lo, lo + n), vhi(hi, hi + n);
    CoupleArgs<Tf> c{};
    c.K = K;
    c.E = n;
    c.inner_max = inner_max;
    c.sigma = sigma;
    c.inner_eps = inner_eps;
    int rc;
    int64_t *d_row = nullptr;
    int32_t *d_sub = nullptr, *d_ka = nullptr, *d_kb = nullptr, *d_ptr = nullptr, *d_ent = nullptr;
    double *d_lo = nullptr, *d_hi = nullptr;
    if ((rc = upload(rows, &d_row, err)) || (rc = upload(sub, &d_sub, err)) || (rc = upload(ka, &d_ka, err)) ||
        (rc = upload(kb, &d_kb, err)) || (rc = upload(ptr, &d_ptr, err)) || (rc = upload(ent, &d_ent, err)) ||
        (rc = upload(vlo, &d_lo, err)) || (rc = upload(vhi, &d_hi, err)) || (rc = alloc(&c.za, size_t(n), err)) ||
        (rc = alloc(&c.zb, size_t(n), err)) || (rc = alloc(&c.la, size_t(n), err)) ||
        (rc = alloc(&c.lb, size_t(n), err)) || (rc = alloc(&c.y, size_t(K), err)))
      return rc;
    c.row = d_row;
    c.sub = d_sub;
    c.ka = d_ka;
    c.kb = d_kb;
    c.kp_ptr = d_ptr;
    c.kp_ent = d_ent;
    c.lo = d_lo;
    c.hi = d_hi;
    int32_t *d_slot = nullptr;
    Tf *d_a = nullptr, *d_s0 = nullptr;
    if ((rc = upload(slot, &d_slot, err)) || (rc = alloc(&d_a, size_t(K), err)) || (rc = alloc(&d_s0, size_t(K), err)))
      return rc;
    args_.cp_slot = d_slot;
    args_.cp_a = d_a;
    args_.cp_s0 = d_s0;
    cp_ = c;
    return DLMPC_OK;
  }

  int copy_y(std::vector<double> &out, std::string &err) override {
    const size_t R = size_t(hs_->N) * hs_->rs;
    std::vector<Tf> tmp(R);
    ENG_CHECK(hipMemcpyAsync(tmp.data(), args_.y, R * sizeof(Tf), hipMemcpyDeviceToHost, stream_));
    ENG_CHECK(hipStreamSynchronize(stream_));
    out.assign(tmp.begin(), tmp.end());
    return DLMPC_OK;
  }

  size_t exchange_bytes() const override {
    return std::max(std::max(2 * size_t(hs_->n_tiles) * hs_->ts, t_len_) * sizeof(Tf), sizeof(Ctl));
  }

  int host_exchange(int which, void *host, std::string &err) override {
    const size_t nst = size_t(hs_->n_tiles) * hs_->ts;
    struct Part {
      void *dev;
      size_t bytes;
    } parts[2] = {{nullptr, 0}, {nullptr, 0}};
    switch (which) {
      case 0: parts[0] = {args_.phi, nst * sizeof(Tf)}; break;
      case 1: parts[0] = {pu_.t, t_len_ * sizeof(Tf)}; break;
      case 2:
        parts[0] = {args_.psi, nst * sizeof(Tf)};
        parts[1] = {args_.lam, nst * sizeof(Tf)};
        break;
      default: parts[0] = {args_.ctl, sizeof(Ctl)}; break;
    }
    char *h = static_cast<char *>(host);
    size_t o = 0;
    for (const Part &q : parts)
      if (q.bytes) {
        ENG_CHECK(hipMemcpyAsync(h + o, q.dev, q.bytes, hipMemcpyDeviceToHost, stream_));
        o += q.bytes;
      }
    ENG_CHECK(hipStreamSynchronize(stream_));
    o = 0;
    for (const Part &q : parts)
      if (q.bytes) {
        ENG_CHECK(hipMemcpyAsync(q.dev, h + o, q.bytes, hipMemcpyHostToDevice, stream_));
        o += q.bytes;
      }
    return DLMPC_OK;
  }

  int output(double *u0_dev, std::string &err) override {
    hipLaunchKernelGGL((output_kernel<Tf, NX>), dim3(1), dim3(kBlock), 0, stream_, args_, w64_, u0_dev);
    ENG_CHECK(hipGetLastError());
    return DLMPC_OK;
  }

  int export_phi(double *phi_dev, std::string &err) override {
    const int64_t n = int64_t(hs_->n_tiles) * hs_->ts;
    const int g = int(std::min<int64_t>((n + kBlock - 1) / kBlock, 4096));
    hipLaunchKernelGGL((export_kernel<Tf>), dim3(g), dim3(kBlock), 0, stream_, args_.phi, map_, n, phi_dev);
    ENG_CHECK(hipGetLastError());
    return DLMPC_OK;
  }

  int certify(const double *x0_dev, double *out, std::string &err) override {
    CertArgs c = cert_;
    c.x0 = x0_dev;
    ENG_CHECK(hipMemsetAsync(cert_out_, 0, 5 * sizeof(unsigned long long), stream_));
    c.out = cert_out_;
    const size_t lds = size_t(NX) * std::max(hs_->k_max, 1) * sizeof(double);
    hipLaunchKernelGGL((cert_kernel<Tf, NX>), dim3(hs_->N), dim3(kBlock), lds, stream_, args_, c);
    ENG_CHECK(hipGetLastError());
    unsigned long long h[5];
    ENG_CHECK(hipMemcpyAsync(h, cert_out_, sizeof(h), hipMemcpyDeviceToHost, stream_));
    ENG_CHECK(hipStreamSynchronize(stream_));
    for (int q = 0; q < 5; ++q) {
      double v;
      std::memcpy(&v, &h[q], sizeof(v));
      out[q] = v;
    }
    return DLMPC_OK;
  }

  // Lists for the certificate's Z_AB rows: per column subsystem j, the subsystems of its support
  // and ring with their tiles and the tiles of their A neighbours.
  int build_cert(const HostSetup &hs, std::string &err) {
    const int N = hs.N;
    std::vector<int64_t> eq_ptr(N + 1, 0), eq_tile, eq_nptr(1, 0), eq_ntile, eq_ablk;
    std::vector<int32_t> eq_sub;
    auto tile_of = [&](int j, int i) -> int64_t {
      const auto &P = hs.patch[j];
      const auto it = std::lower_bound(P.begin(), P.end(), i);
      return (it != P.end() && *it == i) ? hs.tile_off[j] + (it - P.begin()) : -1;
    };
    for (int j = 0; j < N; ++j) {
      std::vector<int32_t> rows(hs.patch[j].begin(), hs.patch[j].end());
      for (int32_t i : hs.patch[j])
        for (int64_t q = hs.a_rowptr[i]; q < hs.a_rowptr[i + 1]; ++q) rows.push_back(hs.a_colidx[q]);
      std::sort(rows.begin(), rows.end());
      rows.erase(std::unique(rows.begin(), rows.end()), rows.end());
      for (int32_t i : rows) {
        eq_sub.push_back(i);
        eq_tile.push_back(tile_of(j, i));
        for (int64_t q = hs.a_rowptr[i]; q < hs.a_rowptr[i + 1]; ++q) {
          eq_ntile.push_back(tile_of(j, hs.a_colidx[q]));
          eq_ablk.push_back(q);
        }
        eq_nptr.push_back(int64_t(eq_ntile.size()));
      }
      eq_ptr[j + 1] = int64_t(eq_sub.size());
    }
    int rc;
    if ((rc = upload(eq_ptr, &cert_.eq_ptr, err)) || (rc = upload(eq_sub, &cert_.eq_sub, err)) ||
        (rc = upload(eq_tile, &cert_.eq_tile, err)) || (rc = upload(eq_nptr, &cert_.eq_nptr, err)) ||
        (rc = upload(eq_ntile, &cert_.eq_ntile, err)) || (rc = upload(eq_ablk, &cert_.eq_ablk, err)) ||
        (rc = upload(hs.a_blocks, &cert_.a_blk, err)) || (rc = upload(hs.b_blocks, &cert_.b_blk, err)) ||
        (rc = alloc(&cert_out_, 5, err)))
      return rc;
    return DLMPC_OK;
  }

  Ctl *ctl() override { return args_.ctl; }

  ~EngineT() override {
    for (void *p : owned_) (void)hipFree(p);
  }

 private:
  static constexpr size_t kMaxLds = 64 * 1024;

  template <typename U>
  int alloc(U **dst, size_t n, std::string &err) {
    void *p = nullptr;
    const size_t bytes = std::max<size_t>(n, 1) * sizeof(U);
    if (hipMalloc(&p, bytes) != hipSuccess) {
      err = "hipMalloc of " + std::to_string(bytes) + " bytes failed";
      return DLMPC_ENOMEM;
    }
    owned_.push_back(p);
    *dst = static_cast<U *>(p);
    return DLMPC_OK;
  }
  template <typename U, typename V>
  int upload(const std::vector<U> &src, V **dst, std::string &err) {
    static_assert(sizeof(U) == sizeof(V), "upload type");
    U *p = nullptr;
    int rc = alloc(&p, src.size(), err);
    if (rc) return rc;
    if (!src.empty()) ENG_CHECK(hipMemcpy(p, src.data(), src.size() * sizeof(U), hipMemcpyHostToDevice));
    *dst = reinterpret_cast<V *>(p);
    return DLMPC_OK;
  }
  template <typename V, class Vec>
  int upload_conv(const Vec &src, V **dst, std::string &err) {
    std::vector<Tf> tmp(src.begin(), src.end());
    Tf *p = nullptr;
    int rc = alloc(&p, tmp.size(), err);
    if (rc) return rc;
    if (!tmp.empty()) ENG_CHECK(hipMemcpy(p, tmp.data(), tmp.size() * sizeof(Tf), hipMemcpyHostToDevice));
    *dst = const_cast<V *>(reinterpret_cast<const V *>(p));
    return DLMPC_OK;
  }

  const HostSetup *hs_ = nullptr;
  hipStream_t stream_ = nullptr;
  size_t t_len_ = 0;  // entries of the Psi pass-1 products t_j
  KArgs<Tf> args_{};
  CoupleArgs<Tf> cp_{};  // K = 0: no couplings
  // structured Psi-comp (enable_structured): its arguments, one residual slot per column
  // subsystem, and the on-chip staging of its two kernels
  bool structured_ = false, struct_ready_ = false;
  SimArgs<Tf> sa_{};
  PsiUnits<Tf> spu_{};
  size_t lds_s1_ = 0, lds_s1b_ = 0, lds_s2_ = 0;
  const int64_t *map_ = nullptr;
  const double *w64_ = nullptr;
  CertArgs cert_{};
  unsigned long long *cert_out_ = nullptr;
  size_t lds_phi_ = 0, lds_psi_ = 0, lds_persist_ = 0, lds_p1_ = 0, lds_p2_ = 0;
  int n1_ = 0, n2_ = 0;
  PsiUnits<Tf> pu_{};
  int grid_ = 0;
  Sched sched_{};
  std::vector<void *> owned_;
};

template <typename Tf>
std::unique_ptr<Engine> make_for_nx(int nx) {
  switch (nx) {
    case 1: return std::make_unique<EngineT<Tf, 1>>();
    case 2: return std::make_unique<EngineT<Tf, 2>>();
    case 3: return std::make_unique<EngineT<Tf, 3>>();
    case 4: return std::make_unique<EngineT<Tf, 4>>();
    default: return nullptr;
  }
}

}  // namespace

std::unique_ptr<Engine> make_engine(int precision, int nx) {
  if (precision == DLMPC_FP64) return make_for_nx<double>(nx);
  if (precision == DLMPC_FP32 || precision == DLMPC_FP32_BF16) return make_for_nx<float>(nx);
  return nullptr;
}

}  // namespace dlmpc
