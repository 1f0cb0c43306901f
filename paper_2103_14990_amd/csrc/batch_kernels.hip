// Batched DLMPC-ADMM (many x0 on one network) in the compact form of Algorithm 2, with the two
// products of an iteration on the gfx950 matrix cores.
//
// Compact form. With the cold start of Algorithm 2 (Psi^0 = Lambda^0 = 0) every iterate from
// the second one on has, per column c of subsystem j and on its support,
//   Psi[:,c]    = o_c + x0_c N_j tau_j,          tau_j = N_j' beta,  beta = sum of past alpha,
//   Lambda[:,c] = x0_c (I - N_j N_j') alpha,      eta_j = N_j' alpha,
// where alpha_r is the row scalar of the Phi-comp solution (Phi row = v + alpha_r x_r). Hence
//   Phi-comp : a_r = c_it b_r + sum_{j in P(m)} ||x0_j||^2 [N_j (tau_j + eta_j)]_r - n_r alpha_r,
//              b_r = sum_{j in P(m)} sum_c x0_c o_c[r], c_it = 0, 2, 1 for iterations 1, 2, >= 3,
//              then the explicit clipped row solution gives the new alpha and s_r = (Phi x0)_r;
//   Psi-comp : eta_j <- N_j' alpha|_{supp j}, tau_j <- tau_j + eta_j;
//   Conv     : ||Psi^{k+1} - Psi^k||_c = |x0_c| ||eta_j||,
//              ||Phi - Psi||_c^2 = x0_c^2 (||d_j||^2 - ||eta_j - eta_j^old||^2), d = alpha - alpha^old
//              (iteration 2 adds the o_c terms of Lambda^1 = -o).
// This is an exact rewriting of the iteration (same trajectory up to rounding). Per instance the
// state is alpha and the k-space vectors, and both products share N_j across the instances:
//   bphi_kernel : (rs x B) += N_j[rows of m, :] (rs x k_j) * W_j (k_j x B) for j in P(m),
//   bpsi_kernel : eta_j (k_j x B) = N_j' (k_j x D_j) * A_j (D_j x B),
// run as v_mfma_f32_16x16x32_bf16 with every FP32 operand split into bf16 hi + lo and the three
// significant partial products (hi*hi, hi*lo, lo*hi) accumulated in FP32.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "dlmpc_device.h"

namespace dlmpc {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kBMax = 64;         // instances per batch (four 16-wide MFMA tiles)
constexpr int kNT = kBMax / 16;
constexpr int kPsiThreads = 512;  // 8 waves
constexpr int kPsiWaves = kPsiThreads / 64;
constexpr int kMTW = 4;           // M tiles (16 basis vectors) per wave: k_j <= 512
constexpr int kKC = 64;           // support rows staged per chunk in bpsi_kernel
constexpr int kRPT = kKC / 8;     // staged rows per thread (8 row groups of 64 threads)
constexpr int kPhiThreads = 512;  // bphi_kernel: 4 instance tiles x 2 halves of the tile list
constexpr int kMaxPatch = 64;     // subsystems per d-hop patch (batched engine)
constexpr int kSNs = 88;          // structured Psi-comp: patch states (p nx) at most
constexpr int kSPnu = 64;         // structured Psi-comp: patch inputs per time step (p nu) at most
constexpr int kSNnz = 512;        // structured Psi-comp: nonzeros of the patch dynamics at most

__device__ __forceinline__ unsigned long long ord_bits(double v) {
  return static_cast<unsigned long long>(__double_as_longlong(v));
}

__device__ __forceinline__ void split8(const float *x, bf16x8 &hi, bf16x8 &lo) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const __bf16 h = static_cast<__bf16>(x[e]);
    hi[e] = h;
    lo[e] = static_cast<__bf16>(x[e] - static_cast<float>(h));
  }
}

// A*B with A = ah + al, B = bh + bl, dropping al*bl. hi + lo carries about 16 significant
// bits of each FP32 operand (lo is itself rounded to bf16: up to ~2^-17 relative error), so a
// product is accurate to a few 1e-6 relative; al*bl (~2^-16 of the product) is below that.
__device__ __forceinline__ f32x4 mfma3(const bf16x8 &ah, const bf16x8 &al, const bf16x8 &bh,
                                       const bf16x8 &bl, f32x4 c) {
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, c, 0, 0, 0);
  return c;
}

// A*B with A = ah (the operand rounded once to bf16), B = bh + bl.
__device__ __forceinline__ f32x4 mfma2(const bf16x8 &ah, const bf16x8 &bh, const bf16x8 &bl, f32x4 c) {
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, c, 0, 0, 0);
  return c;
}

// Values per basis fragment block: bf16 hi and lo of 64 lanes x 8 (split operands), or hi only.
template <bool SPLIT>
constexpr int frag_block() { return SPLIT ? 1024 : 512; }

__device__ __forceinline__ bf16x8 load8(const __bf16 *p) { return *reinterpret_cast<const bf16x8 *>(p); }

template <typename T>
__device__ __forceinline__ T wsum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ------------------------------------------------------------------ per-solve precompute

// Instances per bprecompute_kernel block, and the parts one instance's row sweeps are split
// into (bcg_init_kernel, boutput_kernel; their partial sums are added in part order by
// bpart_sum_kernel).
constexpr int kPreY = 16;
constexpr int kParts = 8;
constexpr int kCgParts = 32;  // row ranges of one instance's CG step

template <int NX>
__global__ __launch_bounds__(256) void bprecompute_kernel(BArgs a, const double *x0, int B, int warm,
                                                          int max_iter, double eps, const int32_t *slots,
                                                          const int32_t *xsrc, int reset, int join, int cg_k,
                                                          const double *rscale) {
  // row subsystem blockIdx.x, instances y = kPreY blockIdx.y + yy (y < B): slot slots[y] (or
  // y), initial state row xsrc[y] (or y) of x0; reset: the solve starts here (global control
  // block reset); otherwise the slots join a running one; rscale[y] (or 1): factor of the
  // instance's penalty. The patch columns of m and their x0 values are staged once per block.
  __shared__ int64_t s_base[kMaxPatch];
  __shared__ int s_ld[kMaxPatch], s_j[kMaxPatch], s_b[kPreY];
  __shared__ double s_x[kPreY][kMaxPatch][NX];
  const int m = blockIdx.x, tid = threadIdx.x;
  const int y0 = kPreY * blockIdx.y, ny = min(kPreY, B - y0);
  const int rs = a.rs;
  const int64_t nxs = int64_t(a.N) * NX;
  const int64_t q0 = a.rt_ptr[m];
  const int np = int(a.rt_ptr[m + 1] - q0);
  if (tid < np) {
    const int j = a.rt_col[q0 + tid];
    const int D = int(a.tile_off[j + 1] - a.tile_off[j]) * rs;
    s_j[tid] = j;
    s_ld[tid] = (D + 3) & ~3;
    s_base[tid] = a.off_ptr[j] + int64_t(a.rt_tile[q0 + tid] - a.tile_off[j]) * rs;
  }
  if (tid < ny) s_b[tid] = slots ? slots[y0 + tid] : y0 + tid;
  __syncthreads();
  for (int e = tid; e < ny * np * NX; e += 256) {
    const int yy = e / (np * NX), r = e - yy * np * NX, q = r / NX, c = r - q * NX;
    const int y = y0 + yy;
    s_x[yy][q][c] = x0[int64_t(xsrc ? xsrc[y] : y) * nxs + s_j[q] * NX + c];
  }
  __syncthreads();
  if (tid < ny) {
    const int y = y0 + tid, b = s_b[tid];
    const double *xb = x0 + int64_t(xsrc ? xsrc[y] : y) * nxs;
    double sm = 0.0, sn = 0.0;
#pragma unroll
    for (int c = 0; c < NX; ++c) {
      a.x0[int64_t(b) * nxs + m * NX + c] = static_cast<float>(xb[m * NX + c]);
      sm += xb[m * NX + c] * xb[m * NX + c];
    }
    for (int q = 0; q < np; ++q)
#pragma unroll
      for (int c = 0; c < NX; ++c) sn += s_x[tid][q][c] * s_x[tid][q][c];
    a.xn[int64_t(b) * a.N + m] = static_cast<float>(sm);
    a.nrm[int64_t(b) * a.N + m] = static_cast<float>(sn);
  }
  const int64_t plane = int64_t(a.Bmax) * a.N * rs;
  // row l of m for instance yy (instances fastest: neighbouring slots share a row's cache line)
  for (int e = tid; e < rs * ny; e += 256) {
    const int l = e / ny, yy = e - l * ny;
    const int64_t ri = (int64_t(m) * rs + l) * a.Bmax + s_b[yy];  // row vectors: [R][Bmax]
    double bv = 0.0;
    for (int q = 0; q < np; ++q) {
      const float *o = a.off + s_base[q] + l;
#pragma unroll
      for (int c = 0; c < NX; ++c) bv += s_x[yy][q][c] * double(o[int64_t(c) * s_ld[q]]);
    }
    a.bvec[ri] = static_cast<float>(bv);
    a.alpha[ri] = 0.f;
    a.alpha[plane + ri] = 0.f;
    a.s[ri] = 0.f;
  }
  const int64_t k0 = a.koff[m], nk = a.koff[m + 1] - k0;
  for (int64_t e = tid; e < nk * ny; e += 256) {
    const int64_t i = k0 + e / ny;
    const int b = s_b[int(e % ny)];
    a.tau[i * a.Bmax + b] = 0.f;
    a.eta[i * a.Bmax + b] = 0.f;
    a.eta[(a.ktot + i) * a.Bmax + b] = 0.f;
  }
  if (m == 0 && tid < ny) {
    const int y = y0 + tid, b = s_b[tid];
    BCtl &ic = a.ictl[b];
    ic.iters = 0;
    ic.stop = 0;
    ic.converged = 0;
    ic.numeric = 0;
    ic.it0 = reset ? 0 : a.ctl->iters;
    a.phase[b] = join ? 0 : -1;
    a.rho_b[b] = rscale ? static_cast<float>(double(a.rho) * rscale[y]) : a.rho;
    if (y == 0) a.ctl->cg_k = cg_k;
    ic.last_rp = ic.last_rd = INFINITY;
    ic.objective = 0.0;
    ic.eq_resid = ic.box = ic.u0dev = ic.objective64 = 0.0;
    a.slot[2 * b] = a.slot[2 * b + 1] = 0ull;
    if (!reset && y == 0) a.ctl->stop = 0;  // a running solve resumes with the new slots
    if (reset && y == 0) {
      Ctl *c = a.ctl;
      c->iters = 0;
      c->stop = 0;
      c->converged = 0;
      c->numeric = 0;
      c->max_iter = max_iter;
      c->eps = eps;
      c->last_rp = c->last_rd = INFINITY;
      c->batch = B;
      c->warm = warm;
    }
  }
}

// Sums of the kParts partial sums of each listed instance, in part order: which 0 gives r'r of
// the trajectory start (cg_rr), 1 the objective of the returned trajectory.
__global__ __launch_bounds__(64) void bpart_sum_kernel(BArgs a, const int32_t *slots, int S, int which) {
  for (int y = threadIdx.x; y < S; y += 64) {
    const int b = slots ? slots[y] : y;
    const double *p = a.bpart + (int64_t(b) * 2 + which) * kParts;
    double v = 0.0;
#pragma unroll
    for (int q = 0; q < kParts; ++q) v += p[q];
    if (which == 0)
      a.cg_rr[b] = a.cg_rrn[b] = v;
    else
      a.ictl[b].objective = v;
  }
}

// Compact warm start: alpha^0 into the previous-iterate plane (plane 0, read by iteration 1).
__global__ __launch_bounds__(256) void bwarm_alpha_kernel(BArgs a, const double *alpha0, int B) {
  const int64_t ny = int64_t(a.N) * a.rs;
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < int64_t(B) * ny; i += int64_t(gridDim.x) * 256)
    a.alpha[(i % ny) * a.Bmax + i / ny] = static_cast<float>(alpha0[i]);
}

__global__ __launch_bounds__(256) void bexport_alpha_kernel(BArgs a, double *out, int B) {
  const int64_t ny = int64_t(a.N) * a.rs;
  const int64_t plane = int64_t(a.Bmax) * ny;
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < int64_t(B) * ny; i += int64_t(gridDim.x) * 256) {
    const int b = int(i / ny);
    const int p = a.ictl[b].iters & 1;  // the plane the stopping iteration wrote
    out[i] = double(a.alpha[p * plane + (i - int64_t(b) * ny) * a.Bmax + b]);
  }
}

// ------------------------------------------------------------------ Phi-comp (batched)

// One block per row subsystem m (8 waves); wave w owns instances [16 nt, 16 nt + 16), nt = w % 4,
// for every other tile of m's row (half w / 4), all NRT row tiles of m; the two halves are summed
// in a fixed order. The right operand W_j = ||x0_j||^2 (tau_j + eta_j) is read pre-split (bf16
// hi/lo, written by bpsi_kernel) once per block; the rows of N_j that belong to m (fragment
// order) are the left operand. The (tile, k-step) sequence of a wave is one flat loop whose
// next step's operands are in flight while the current step's products run.
// SPLIT: basis fragments as bf16 hi + lo (three products per tile); otherwise hi only (two).
// NTW: instance tiles per wave. 1: wave w serves instance tile w % 4 and half w / 4 of the tile
// list; 2: instance tiles 2 (w % 2), 2 (w % 2) + 1 and quarter w / 2 of the tile list (each basis
// fragment loaded by half as many waves, twice the accumulators). The parts are summed in a
// fixed order.
template <int NX, int NRT, bool SPLIT, int NTW>
__global__ __launch_bounds__(kPhiThreads) void bphi_kernel(BArgs a) {
  constexpr int kFB = frag_block<SPLIT>();
  constexpr int NPART = 2 * NTW;  // parts of m's tile list
  if (a.ctl->stop) return;
  __shared__ float Ct[NPART][64][kBMax + 1];
  __shared__ double red[kPhiThreads / 64][kBMax];
  __shared__ int64_t s_fb[kMaxPatch], s_w8[kMaxPatch];
  __shared__ int s_nkt[kMaxPatch];
  const int m = a.phi_order[blockIdx.x], tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int ntg = wave & (4 / NTW - 1), half = wave / (4 / NTW);  // instance-tile group, part
  const int rs = a.rs, B = a.ctl->batch;
  const bool warm = a.ctl->warm != 0;
  const bool cgm = a.phi_mode != 0;  // set-up pass: q = sum_j ||x0_j||^2 N_j eta_j
  const int it = a.ctl->iters + 1;
  const float coef = warm ? 1.f : (it == 1 ? 0.f : (it == 2 ? 2.f : 1.f));
  const int64_t q0 = a.rt_ptr[m];
  const int pm = int(a.rt_ptr[m + 1] - q0);
  for (int t = tid; t < pm; t += kPhiThreads) {  // per-tile descriptors of m's row
    const int j = a.rt_col[q0 + t];
    s_fb[t] = a.nf_off[a.rt_tile[q0 + t]];
    s_w8[t] = a.koff[j] >> 3;
    s_nkt[t] = int(a.koff[j + 1] - a.koff[j]) >> 5;
  }
  __syncthreads();
  constexpr int nrt = NRT;
  f32x4 acc[NRT][NTW];
#pragma unroll
  for (int rt = 0; rt < NRT; ++rt)
#pragma unroll
    for (int u = 0; u < NTW; ++u) acc[rt][u] = f32x4{0.f, 0.f, 0.f, 0.f};
  // instance tiles of this wave that hold instances (wave-uniform); tiles past B are not loaded
  int ntv = 0;
#pragma unroll
  for (int u = 0; u < NTW; ++u) ntv += (ntg * NTW + u) * 16 < B;
  // from a cold start tau = eta = 0 before the third iteration
  if ((cgm || warm || it >= 3) && ntv > 0 && half < pm) {
    const int b0 = ntg * NTW * 16 + (lane & 15);
    bf16x8 wh[NTW], wl[NTW], ah[NRT], al[NRT];
    auto load_step = [&](int t, int kt, bf16x8 *ph, bf16x8 *pl, bf16x8 *qh, bf16x8 *ql) {
      const int64_t wrow = (s_w8[t] + 4 * kt + (lane >> 4)) * a.Bw;
#pragma unroll
      for (int u = 0; u < NTW; ++u) {
        if (u >= ntv) break;
        const int64_t wi = (wrow + b0 + 16 * u) * 8;
        ph[u] = load8(a.w_hi + wi);
        pl[u] = load8(a.w_lo + wi);
      }
      const int64_t fb = s_fb[t] + lane * 8 + int64_t(kt) * kFB, stride = int64_t(s_nkt[t]) * kFB;
#pragma unroll
      for (int rt = 0; rt < NRT; ++rt) {  // rows past rs are zero in the fragments
        qh[rt] = load8(a.nf + fb + rt * stride);
        if constexpr (SPLIT) ql[rt] = load8(a.nf + fb + rt * stride + 512);
      }
    };
    // two operand sets used alternately: the loads of one are in flight while the products of
    // the other run (no register copies between steps)
    // (the loads of the step after the last one repeat the last step: always issued, so that
    // the number of loads in flight is the same on every path)
    bf16x8 wh2[NTW], wl2[NTW], ah2[NRT], al2[NRT];
    int t = half, kt = 0;
    auto advance = [&]() {
      int tn = t, kn = kt + 1;
      if (kn >= s_nkt[t]) {
        tn = t + NPART;
        kn = 0;
      }
      const bool more = tn < pm;
      if (more) {
        t = tn;
        kt = kn;
      }
      return more;
    };
    auto products = [&](const bf16x8 *qh, const bf16x8 *ql, const bf16x8 *ph, const bf16x8 *pl) {
#pragma unroll
      for (int rt = 0; rt < NRT; ++rt)
#pragma unroll
        for (int u = 0; u < NTW; ++u) {
          if (u >= ntv) break;
          acc[rt][u] = SPLIT ? mfma3(qh[rt], ql[rt], ph[u], pl[u], acc[rt][u]) : mfma2(qh[rt], ph[u], pl[u], acc[rt][u]);
        }
    };
    load_step(t, kt, wh, wl, ah, al);
    while (true) {
      bool more = advance();
      load_step(t, kt, wh2, wl2, ah2, al2);
      __builtin_amdgcn_sched_barrier(0);  // keep the prefetch ahead of the products
      products(ah, al, wh, wl);
      if (!more) break;
      more = advance();
      load_step(t, kt, wh, wl, ah, al);
      __builtin_amdgcn_sched_barrier(0);
      products(ah2, al2, wh2, wl2);
      if (!more) break;
    }
  }
  // C tile: lane holds rows 16 rt + 4 (lane / 16) + e of instance column 16 (ntg NTW + u) + lane % 16
#pragma unroll
  for (int rt = 0; rt < nrt; ++rt)
#pragma unroll
    for (int u = 0; u < NTW; ++u)
#pragma unroll
      for (int e = 0; e < 4; ++e)
        Ct[half][rt * 16 + 4 * (lane >> 4) + e][(ntg * NTW + u) * 16 + (lane & 15)] = acc[rt][u][e];
  __syncthreads();
  auto csum = [&](int l, int b) {
    if constexpr (NPART == 2) return Ct[0][l][b] + Ct[1][l][b];
    else return (Ct[0][l][b] + Ct[1][l][b]) + (Ct[2][l][b] + Ct[3][l][b]);
  };
  if (cgm) {
    for (int idx = tid; idx < rs * B; idx += blockDim.x) {
      const int l = idx / B, b = idx - l * B;
      a.cg_q[int64_t(b) * a.N * rs + int64_t(m) * rs + l] = csum(l, b);
    }
    return;
  }
  // streamed joins whose start is at a CG step: this product is q = M p
  for (int idx = tid; idx < rs * B; idx += blockDim.x) {
    const int l = idx / B, b = idx - l * B;
    const int ph = a.phase[b];
    if (ph >= 1 && ph <= a.ctl->cg_k && !a.ictl[b].stop)
      a.cg_q[int64_t(b) * a.N * rs + int64_t(m) * rs + l] = csum(l, b);
  }
  // Row update: thread (instance b, row group lg) handles rows lg, lg + 8, ... of m, and the
  // sum of (alpha - alpha_prev)^2 over m's rows (the residual term Psi-comp needs) per instance.
  constexpr int kLG = kPhiThreads / 64;
  const int64_t plane = int64_t(a.Bmax) * a.N * rs;
  const int cur = it & 1, prev = cur ^ 1;
  const int b = tid & 63, lg = tid >> 6;
  double dl = 0.0;
  if (b < B && !a.ictl[b].stop && a.phase[b] < 0) {
    const float n = a.nrm[int64_t(b) * a.N + m], rho = a.rho_b[b];
    for (int l = lg; l < rs; l += kLG) {
      const int64_t o = int64_t(m) * rs + l;
      const int64_t rb = o * a.Bmax + b;  // consecutive instances: consecutive addresses
      const float ap = a.alpha[prev * plane + rb];
      const float av = coef * a.bvec[rb] + csum(l, b) - n * ap;
      float sv, al;
      if (n > 0.f) {
        sv = rho * av / (rho + 2.f * a.w[o] * n);
        sv = sv < a.lb[o] ? a.lb[o] : (sv > a.ub[o] ? a.ub[o] : sv);
        al = (sv - av) / n;
      } else {
        sv = av;
        al = 0.f;
      }
      a.alpha[cur * plane + rb] = al;
      a.s[rb] = sv;
      dl += double(al - ap) * double(al - ap);
    }
  }
  red[lg][b] = dl;
  __syncthreads();
  if (tid < B && !a.ictl[tid].stop && a.phase[tid] < 0) {
    double sum = 0.0;
#pragma unroll
    for (int g = 0; g < kLG; ++g) sum += red[g][tid];
    a.dlm[int64_t(tid) * a.N + m] = sum;
  }
}

// ------------------------------------------------------------------ Psi-comp + Conv (batched)

// One block per column subsystem j: eta_j = N_j' A_j over K-chunks of its support rows staged
// (as bf16 hi/lo) in LDS; wave w owns the M tiles w, w + 8, ... of the basis vectors.
// Two 8-wave blocks per CU (four waves per SIMD, 128 registers per lane, a few of them spilled)
// while a wave has at most 3 tiles, one block otherwise. SPLIT: basis fragments as bf16 hi + lo
// (three products per tile); otherwise hi only (two).
// STRUCT: the structured Psi-comp (one unit per column subsystem): eta_j = N_u' g with
// g = alpha_u + S_x' alpha_x from the adjoint recursion mu_t = alpha_{x,t} + A_PP' mu_{t+1},
// g_{t-1} = alpha_{u,t-1} + B_P' mu_t run per instance; the rows of g go through the staging
// buffer as they are produced and every full kKC-row chunk feeds the products.
// (two blocks per CU need MTW <= 3; the structured variant's staging also needs NX <= 2)
template <int NX, int MTW, bool SPLIT, bool STRUCT = false>
__global__ __launch_bounds__(kPsiThreads) __attribute__((amdgpu_waves_per_eu((MTW <= 3 && (!STRUCT || NX <= 2)) ? 4 : 2))) void bpsi_kernel(BArgs a) {
  constexpr int kFB = frag_block<SPLIT>();
  constexpr int kSH = STRUCT ? kKC + kSPnu + 8 : kKC + 8;
  if (a.ctl->stop) return;
  __shared__ __align__(16) __bf16 sh_hi[kBMax][kSH];
  __shared__ __align__(16) __bf16 sh_lo[kBMax][kSH];
  __shared__ float smu[STRUCT ? kBMax : 1][STRUCT ? kSNs + 1 : 1];
  // structured: the patch's transposed dynamics (CSR) and input blocks, read by every step of
  // the recursion (the same entries across a wave: staged once instead of loaded per step)
  __shared__ int16_t s_srp[STRUCT ? kSNs + 1 : 1], s_scol[STRUCT ? kSNnz : 1];
  __shared__ float s_sval[STRUCT ? kSNnz : 1], s_sbb[STRUCT ? kSPnu * NX : 1];
  __shared__ int s_rsub[kMaxPatch];
  __shared__ double red_e[kPsiWaves][kBMax], red_d[kPsiWaves][kBMax];
  __shared__ double red_od[kBMax][8][NX];
  // One work unit per block: rows [r_begin, r_end) of column subsystem j (part `part` of
  // np), units in decreasing order of work so that the heavy ones start first.
  __shared__ int s_last;
  const int u = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int j = a.pu_j[u], r_begin = a.pu_r0[u], r_end = a.pu_r1[u], part = a.pu_p[u];
  const int np = a.pj_n[j];
  const int rs = a.rs, B = a.ctl->batch;
  const bool warm = a.ctl->warm != 0;
  const int it = a.ctl->iters + 1;
  const int64_t tb = a.tile_off[j];
  const int D = int(a.tile_off[j + 1] - tb) * rs;
  const int k = a.kdim[j];
  const int kc16 = (k + 15) & ~15;
  const int ldK = (D + kKC - 1) / kKC * kKC;  // support rows padded to whole chunks
  const int ld4 = (D + 3) & ~3;
  const int64_t plane = int64_t(a.Bmax) * a.N * rs;
  const bool initp = a.init_pass != 0;
  const bool cold2 = !warm && it == 2;
  const int cur = it & 1;
  // a set-up pass stages the row vectors src; the iteration stages the current alpha
  const float *stage_src = initp ? a.src : a.alpha + cur * plane;
  // element (b, row) of the staged vectors: alpha planes are [R][Bmax], set-up sources carry
  // their own strides
  // staging: instance sb (fastest across the wave), rows 8 sub .. 8 sub + 7 of the chunk
  const int sb = tid & 63, sub = tid >> 6;
  // streamed joins (iteration passes): the lane's instance may stage its CG vector instead
  // (cg_p at phases 0..cg_k-1, beta = cg_x at phase cg_k; at cg_k + 1 alpha^0, in both planes)
  const int sph = (!initp && sb < B) ? a.phase[sb] : -1;
  const float *jsrc = (sph >= 0 && sph < a.ctl->cg_k) ? a.cg_p : a.cg_x;
  const bool jstage = sph >= 0 && sph <= a.ctl->cg_k;

  if (!warm && it == 1 && !initp) {  // alpha^1 = 0: Psi^1 = o, residuals ||o_c||, eta stays 0
    if (part == 0 && tid < B && !a.ictl[tid].stop) {
      double mx = 0.0;
#pragma unroll
      for (int c = 0; c < NX; ++c) mx = fmax(mx, sqrt(a.onorm2[j * NX + c]));
      atomicMax(&a.slot[2 * tid], ord_bits(mx));
      atomicMax(&a.slot[2 * tid + 1], ord_bits(mx));
    }
    return;
  }

  for (int t = tid; t < D / rs; t += kPsiThreads) s_rsub[t] = a.tile_rsub[tb + t];
  __syncthreads();
  const int nmt = kc16 >> 4, nkt = ldK >> 5;
  f32x4 acc[MTW][kNT];
#pragma unroll
  for (int t = 0; t < MTW; ++t)
#pragma unroll
    for (int nt = 0; nt < kNT; ++nt) acc[t][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
  double od[NX];
#pragma unroll
  for (int c = 0; c < NX; ++c) od[c] = 0.0;
  const bool sact = sb < B;
  // Staging values of instance sb for support rows r0 + 8 sub .. + 7 (zero past D): eight
  // independent loads (clamped address, then a select), the row's subsystem from LDS.
  auto fetch = [&](int r0, float *v) {
#pragma unroll
    for (int e = 0; e < kRPT; ++e) {
      const int rr = r0 + kRPT * sub + e;
      const bool ok = sact && rr < D;
      const int rc = ok ? rr : 0;
      const int ta = rc / rs, l = rc - ta * rs;
      const int64_t row = int64_t(s_rsub[ta]) * rs + l;
      const float x = jstage ? jsrc[int64_t(ok ? sb : 0) * a.N * rs + row]
                             : stage_src[int64_t(ok ? sb : 0) * a.src_bs + row * a.src_rs];
      v[e] = ok ? x : 0.f;
    }
  };
  if constexpr (STRUCT) {
    const int p = D / rs, ns = p * NX, nu = a.nu, T = a.T, pnu = p * nu, nxT = NX * a.T;
    const int nku = ((T - 1) * pnu + kKC - 1) / kKC * kKC / 32;  // K-steps of N_u (whole chunks)
    const int32_t *rpt = a.srpt + a.srp0[j];
    const int32_t *colt = a.scolt + a.se0[j];
    const float *valt = a.svalt + a.se0[j];
    // value of instance sb's row `row` of the staged vectors (library row index)
    auto src_at = [&](int64_t row) -> float {
      if (!sact) return 0.f;
      return jstage ? jsrc[int64_t(sb) * a.N * rs + row] : stage_src[int64_t(sb) * a.src_bs + row * a.src_rs];
    };
    for (int s0 = sub; s0 < kSNs + 1; s0 += 8) smu[sb][s0] = 0.f;  // mu_T = 0
    for (int e = tid; e <= ns; e += kPsiThreads) s_srp[e] = static_cast<int16_t>(rpt[e]);
    for (int e = tid; e < rpt[ns]; e += kPsiThreads) {
      s_scol[e] = static_cast<int16_t>(colt[e]);
      s_sval[e] = valt[e];
    }
    for (int e = tid; e < pnu * NX; e += kPsiThreads) {  // e = (member * nu + input) * NX + state
      const int w = e / NX, sx = e - w * NX, ti = w / nu, kk = w - ti * nu;
      s_sbb[e] = a.b_blk[int64_t(s_rsub[ti]) * NX * nu + sx * nu + kk];
    }
    int fill = 0, chunk = 0;
    auto products = [&](int nrows) {  // chunk `chunk` of the K rows: sh rows [0, nrows)
      for (int ks = 0; ks < nrows / 32; ++ks) {
        bf16x8 ah[MTW], al[MTW];
#pragma unroll
        for (int t = 0; t < MTW; ++t) {
          const int mt = min(wave + kPsiWaves * t, nmt - 1);
          const int64_t ai = a.ntu_off[j] + (int64_t(mt) * nku + 2 * chunk + ks) * kFB + lane * 8;
          ah[t] = load8(a.ntu + ai);
          if constexpr (SPLIT) al[t] = load8(a.ntu + ai + 512);
        }
        const int kr = ks * 32 + 8 * (lane >> 4);
#pragma unroll
        for (int nt = 0; nt < kNT; ++nt) {
          if (nt * 16 >= B) break;
          const bf16x8 bh = *reinterpret_cast<const bf16x8 *>(&sh_hi[nt * 16 + (lane & 15)][kr]);
          const bf16x8 bl = *reinterpret_cast<const bf16x8 *>(&sh_lo[nt * 16 + (lane & 15)][kr]);
#pragma unroll
          for (int t = 0; t < MTW; ++t) {
            if (wave + kPsiWaves * t >= nmt) break;
            acc[t][nt] = SPLIT ? mfma3(ah[t], al[t], bh, bl, acc[t][nt]) : mfma2(ah[t], bh, bl, acc[t][nt]);
          }
        }
      }
    };
    __syncthreads();
    for (int q = 0; q < T - 1; ++q) {
      const int t = T - 1 - q;
      // mu_t for this thread's states sub, sub + 8, ... (instance sb)
      float mreg[(kSNs + 7) / 8];
#pragma unroll
      for (int i = 0; i < (kSNs + 7) / 8; ++i) {
        const int st = sub + 8 * i;
        float v = 0.f;
        if (st < ns) {
          const int ti = st / NX, sx = st - ti * NX;
          v = src_at(int64_t(s_rsub[ti]) * rs + t * NX + sx);
          for (int e = s_srp[st]; e < s_srp[st + 1]; ++e) v += s_sval[e] * smu[sb][s_scol[e]];
        }
        mreg[i] = v;
      }
      __syncthreads();  // every read of mu_{t+1} is done
#pragma unroll
      for (int i = 0; i < (kSNs + 7) / 8; ++i)
        if (sub + 8 * i < ns) smu[sb][sub + 8 * i] = mreg[i];
      __syncthreads();
      // g_{t-1}: rows fill + w, w = member * nu + input
      for (int w = sub; w < pnu; w += 8) {
        const int ti = w / nu, kk = w - ti * nu;
        const int m = s_rsub[ti];
        float gv = src_at(int64_t(m) * rs + nxT + (t - 1) * nu + kk);
#pragma unroll
        for (int sx = 0; sx < NX; ++sx) gv += s_sbb[w * NX + sx] * smu[sb][ti * NX + sx];
        const __bf16 gh = static_cast<__bf16>(gv);
        sh_hi[sb][fill + w] = gh;
        sh_lo[sb][fill + w] = static_cast<__bf16>(gv - static_cast<float>(gh));
      }
      fill += pnu;
      const bool last = q == T - 2;
      if (last) {  // zero rows up to the next multiple of 32 (the basis rows there are zero too)
        const int pad = (fill + 31) & ~31;
        for (int w = fill + sub; w < pad; w += 8) {
          sh_hi[sb][w] = static_cast<__bf16>(0.f);
          sh_lo[sb][w] = static_cast<__bf16>(0.f);
        }
      }
      __syncthreads();
      while (fill >= kKC || (last && fill > 0)) {
        products(fill >= kKC ? kKC : ((fill + 31) & ~31));
        __syncthreads();  // the products read the staged rows
        if (fill > kKC) {
          for (int w = sub; w < fill - kKC; w += 8) {
            sh_hi[sb][w] = sh_hi[sb][kKC + w];
            sh_lo[sb][w] = sh_lo[sb][kKC + w];
          }
          __syncthreads();
        }
        fill = fill > kKC ? fill - kKC : 0;
        ++chunk;
        if (last && fill > 0) {
          const int pad = (fill + 31) & ~31;
          for (int w = fill + sub; w < pad; w += 8) {
            sh_hi[sb][w] = static_cast<__bf16>(0.f);
            sh_lo[sb][w] = static_cast<__bf16>(0.f);
          }
          __syncthreads();
        }
      }
    }
  } else {
  float v[kRPT];
  fetch(r_begin, v);
  for (int r0 = r_begin; r0 < r_end; r0 += kKC) {
    // this chunk's basis fragments (both k-steps) are issued before the staging barrier
    bf16x8 ah[kKC / 32][MTW], al[kKC / 32][MTW];
#pragma unroll
    for (int ks = 0; ks < kKC / 32; ++ks)
#pragma unroll
      for (int t = 0; t < MTW; ++t) {
        const int mt = min(wave + kPsiWaves * t, nmt - 1);  // tiles past nmt: loaded, unused
        const int64_t ai = a.ntf_off[j] + (int64_t(mt) * nkt + (r0 >> 5) + ks) * kFB + lane * 8;
        ah[ks][t] = load8(a.ntf + ai);
        if constexpr (SPLIT) al[ks][t] = load8(a.ntf + ai + 512);
      }
    __builtin_amdgcn_sched_barrier(0);  // fragments in flight before the staging barrier
#pragma unroll
    for (int h = 0; h < kRPT / 8; ++h) {
      bf16x8 vh, vl;
      split8(v + 8 * h, vh, vl);
      *reinterpret_cast<bf16x8 *>(&sh_hi[sb][kRPT * sub + 8 * h]) = vh;
      *reinterpret_cast<bf16x8 *>(&sh_lo[sb][kRPT * sub + 8 * h]) = vl;
    }
    __syncthreads();
    // next chunk in flight during the products (the last chunk fetches itself again, so the
    // loads in flight are the same on every path)
    fetch(r0 + kKC < r_end ? r0 + kKC : r0, v);
    __builtin_amdgcn_sched_barrier(0);  // next chunk's staging loads ahead of the products
#pragma unroll
    for (int ks = 0; ks < kKC / 32; ++ks) {
      const int kr = ks * 32 + 8 * (lane >> 4);
      // one instance tile's staged operand at a time (fewer live registers than all four)
#pragma unroll
      for (int nt = 0; nt < kNT; ++nt) {
        if (nt * 16 >= B) break;
        const bf16x8 bh = *reinterpret_cast<const bf16x8 *>(&sh_hi[nt * 16 + (lane & 15)][kr]);
        const bf16x8 bl = *reinterpret_cast<const bf16x8 *>(&sh_lo[nt * 16 + (lane & 15)][kr]);
#pragma unroll
        for (int t = 0; t < MTW; ++t) {
          if (wave + kPsiWaves * t >= nmt) break;
          acc[t][nt] = SPLIT ? mfma3(ah[ks][t], al[ks][t], bh, bl, acc[t][nt]) : mfma2(ah[ks][t], bh, bl, acc[t][nt]);
        }
      }
    }
    __syncthreads();
  }
  }
  if (cold2) {  // offset terms of the second cold iteration: sum_rows alpha o_c over the unit
    for (int r0 = r_begin; r0 < r_end; r0 += kKC) {
      float v[kRPT];
      fetch(r0, v);
#pragma unroll
      for (int e = 0; e < kRPT; ++e) {
        const int rr = r0 + kRPT * sub + e;
        if (sact && rr < D) {
#pragma unroll
          for (int c = 0; c < NX; ++c) od[c] += double(v[e]) * double(a.off[a.off_ptr[j] + int64_t(c) * ld4 + rr]);
        }
      }
    }
  }
  if (np > 1) {
    // Partial sums of a split column block: store, publish, and let the last part to finish
    // add all parts in part order (the result does not depend on which part is last).
    float *P = a.ppart + a.pj_off[j];
    double *Q = a.ppod + int64_t(a.pj_first[j]) * kBMax * 8 * NX;
#pragma unroll
    for (int t = 0; t < MTW; ++t) {
      const int mtile = wave + kPsiWaves * t;
      if (mtile * 16 >= kc16) break;
#pragma unroll
      for (int nt = 0; nt < kNT; ++nt)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int i = mtile * 16 + 4 * (lane >> 4) + e;
          P[(int64_t(part) * kc16 + i) * kBMax + nt * 16 + (lane & 15)] = acc[t][nt][e];
        }
    }
#pragma unroll
    for (int c = 0; c < NX; ++c) Q[((int64_t(part) * kBMax + sb) * 8 + sub) * NX + c] = od[c];
    __threadfence();
    __syncthreads();
    if (tid == 0) s_last = atomicAdd(&a.pcnt[j], 1) == np - 1;
    __syncthreads();
    if (!s_last) return;
    __threadfence();
#pragma unroll
    for (int t = 0; t < MTW; ++t) {
      const int mtile = wave + kPsiWaves * t;
      if (mtile * 16 >= kc16) break;
#pragma unroll
      for (int nt = 0; nt < kNT; ++nt)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int i = mtile * 16 + 4 * (lane >> 4) + e;
          float sum = 0.f;
          for (int q = 0; q < np; ++q) sum += P[(int64_t(q) * kc16 + i) * kBMax + nt * 16 + (lane & 15)];
          acc[t][nt][e] = sum;
        }
    }
#pragma unroll
    for (int c = 0; c < NX; ++c) {
      double sum = 0.0;
      for (int q = 0; q < np; ++q) sum += Q[((int64_t(q) * kBMax + sb) * 8 + sub) * NX + c];
      od[c] = sum;
    }
    if (tid == 0) a.pcnt[j] = 0;  // ready for the next launch
  }
  // eta_new, tau and the k-space residual terms; lane holds basis rows 4 (lane/16) + e of tile.
  const int64_t eplane = a.ktot * a.Bmax;
  double e2[kNT], d2[kNT];
#pragma unroll
  for (int nt = 0; nt < kNT; ++nt) e2[nt] = d2[nt] = 0.0;
#pragma unroll
  for (int t = 0; t < MTW; ++t) {
    const int mtile = wave + kPsiWaves * t;
    if (mtile * 16 >= kc16) break;
#pragma unroll
    for (int nt = 0; nt < kNT; ++nt) {
      const int b = nt * 16 + (lane & 15);
      if (b >= B || a.ictl[b].stop) continue;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int i = mtile * 16 + 4 * (lane >> 4) + e;
        if (i >= k) continue;
        const int64_t ki = (a.koff[j] + i) * a.Bmax + b;  // instance-minor: lanes b coalesce
        // eta planes by iteration parity: the current iterate's, and the previous one's
        const int64_t kc = ki + (cur ? eplane : 0), kp = ki + (cur ? 0 : eplane);
        const int64_t wi = (((a.koff[j] + i) >> 3) * a.Bw + b) * 8 + (i & 7);
        const float xj = a.xn[int64_t(b) * a.N + j];
        const float en = acc[t][nt][e];
        float wv;
        const int ph = initp ? -1 : a.phase[b];
        if (ph >= 0) {  // streamed join: the start's projections, as the set-up passes do them
          if (ph < a.ctl->cg_k) {
            a.eta[kc] = en;
            wv = xj * en;
          } else if (ph == a.ctl->cg_k) {
            a.tau[ki] = en;
            continue;
          } else {  // eta^0 into both planes: the joiner's first iteration may have either parity
            a.eta[kc] = en;
            a.eta[kp] = en;
            wv = xj * (a.tau[ki] + en);
          }
        } else if (initp) {
          a.dst_k[ki] = en;
          if (a.wmode == 0) continue;
          wv = xj * (a.wmode == 2 ? a.tau[ki] + en : en);
        } else {
          const float eo = a.eta[kp];
          const float tn = a.tau[ki] + en;
          a.eta[kc] = en;
          a.tau[ki] = tn;
          e2[nt] += double(en) * double(en);
          d2[nt] += double(en - eo) * double(en - eo);
          wv = xj * (tn + en);
        }
        const __bf16 wh = static_cast<__bf16>(wv);
        a.w_hi[wi] = wh;
        a.w_lo[wi] = static_cast<__bf16>(wv - static_cast<float>(wh));
      }
    }
  }
  if (initp) return;  // set-up pass: the k-space vectors only
#pragma unroll
  for (int nt = 0; nt < kNT; ++nt) {  // lanes l, l^16, l^32, l^48 share an instance
    e2[nt] += __shfl_xor(e2[nt], 16, 64);
    e2[nt] += __shfl_xor(e2[nt], 32, 64);
    d2[nt] += __shfl_xor(d2[nt], 16, 64);
    d2[nt] += __shfl_xor(d2[nt], 32, 64);
    if (lane < 16) {
      red_e[wave][nt * 16 + lane] = e2[nt];
      red_d[wave][nt * 16 + lane] = d2[nt];
    }
  }
#pragma unroll
  for (int c = 0; c < NX; ++c) red_od[sb][sub][c] = od[c];
  __syncthreads();
  if (tid < B && !a.ictl[tid].stop && a.phase[tid] < 0) {
    const int b = tid;
    double se = 0.0, sd = 0.0, sdl = 0.0;
    for (int w = 0; w < kPsiWaves; ++w) {
      se += red_e[w][b];
      sd += red_d[w][b];
    }
    // ||alpha - alpha_prev||^2 on the support of j: per-row-subsystem sums from bphi_kernel
    for (int64_t ta = tb; ta < a.tile_off[j + 1]; ++ta) sdl += a.dlm[int64_t(b) * a.N + a.tile_rsub[ta]];
    double mp = 0.0, md = 0.0;
#pragma unroll
    for (int c = 0; c < NX; ++c) {
      const double xc = double(a.x0[int64_t(b) * a.N * NX + j * NX + c]);
      const double rd = fabs(xc) * sqrt(se);
      double rp2;
      if (cold2) {
        double odc = 0.0;
        for (int q = 0; q < 8; ++q) odc += red_od[b][q][c];
        rp2 = a.onorm2[j * NX + c] + 2.0 * xc * odc + xc * xc * (sdl - se);
      } else {
        rp2 = xc * xc * (sdl - sd);
      }
      const double rp = sqrt(fmax(rp2, 0.0));
      mp = (rp > mp || rp != rp) ? rp : mp;
      md = (rd > md || rd != rd) ? rd : md;
    }
    atomicMax(&a.slot[2 * b], ord_bits(mp));
    atomicMax(&a.slot[2 * b + 1], ord_bits(md));
  }
}

// ------------------------------------------------------------------ decision, outputs

__global__ __launch_bounds__(64) void bdecide_kernel(BArgs a) {
  __shared__ int n_stop;
  __shared__ unsigned long long worst_p, worst_d;
  const int b = threadIdx.x;
  Ctl *c = a.ctl;
  // every value the decision reads is loaded before the first use (independent addresses, one
  // memory round trip instead of a chain of them)
  const bool own = b < a.Bmax;
  const int all_stop = c->stop, it = c->iters + 1, B = c->batch, cg_k = c->cg_k, max_iter = c->max_iter;
  const double eps = c->eps;
  const int i_stop = own ? a.ictl[b].stop : 1, i_it0 = own ? a.ictl[b].it0 : 0;
  const int ph = own ? a.phase[b] : -1;
  const unsigned long long sp = own ? a.slot[2 * b] : 0ull, sd = own ? a.slot[2 * b + 1] : 0ull;
  if (all_stop) return;
  if (b == 0) {
    n_stop = 0;
    worst_p = worst_d = 0ull;
  }
  __syncthreads();
  if (b < B) {
    BCtl &ic = a.ictl[b];
    bool stop = i_stop != 0;
    if (!stop && ph >= 0) {  // streamed join: its start runs; no decision yet
      if (ph + 1 > cg_k + 1) {
        a.phase[b] = -1;
        ic.it0 = it;  // its first ADMM iteration is the next one
      } else {
        a.phase[b] = ph + 1;
      }
    } else if (!stop) {
      const double rp = __longlong_as_double(static_cast<long long>(sp));
      const double rd = __longlong_as_double(static_cast<long long>(sd));
      const int iters = it - i_it0;
      ic.iters = iters;
      ic.last_rp = rp;
      ic.last_rd = rd;
      if (!(rp == rp) || !(rd == rd) || isinf(rp) || isinf(rd)) {
        ic.numeric = 1;
        stop = true;
      } else if (rp <= eps && rd <= eps) {
        ic.converged = 1;
        stop = true;
      } else if (iters >= max_iter) {
        stop = true;
      }
      if (stop) {
        ic.stop = 1;
      } else {
        atomicMax(&worst_p, ord_bits(rp));
        atomicMax(&worst_d, ord_bits(rd));
      }
    }
    a.slot[2 * b] = a.slot[2 * b + 1] = 0ull;
    if (stop) atomicAdd(&n_stop, 1);
  }
  __syncthreads();
  if (b == 0) {
    c->iters = it;
    c->last_rp = __longlong_as_double(static_cast<long long>(worst_p));
    c->last_rd = __longlong_as_double(static_cast<long long>(worst_d));
    if (n_stop == B) c->stop = 1;
  }
}

template <int NX>
__global__ __launch_bounds__(256) void boutput_kernel(BArgs a, double *u0, const int32_t *slots,
                                                      const int32_t *dst) {
  // slot slots[x] (or x) into row dst[x] (or x) of u0; part blockIdx.y of kParts writes its
  // share of u(0) and the partial objective of its row range (summed by bpart_sum_kernel)
  __shared__ double red[4];
  const int b = slots ? slots[blockIdx.x] : blockIdx.x, tid = threadIdx.x, part = blockIdx.y;
  const int64_t orow = dst ? dst[blockIdx.x] : blockIdx.x;
  const int64_t ny = int64_t(a.N) * a.rs, chunk = (ny + kParts - 1) / kParts;
  const int64_t r0 = part * chunk, r1 = min(ny, r0 + chunk);
  const float *sb = a.s + b;  // row i of instance b at sb[i * Bmax]
  double acc = 0.0;
  for (int64_t i = r0 + tid; i < r1; i += 256) acc += a.w64[i] * double(sb[i * a.Bmax]) * double(sb[i * a.Bmax]);
  acc = wsum(acc);
  if ((tid & 63) == 0) red[tid >> 6] = acc;
  __syncthreads();
  if (tid == 0) a.bpart[(int64_t(b) * 2 + 1) * kParts + part] = (red[0] + red[1]) + (red[2] + red[3]);
  for (int i = part * 256 + tid; i < a.N * a.nu; i += kParts * 256) {
    const int m = i / a.nu, q = i - m * a.nu;
    u0[orow * a.N * a.nu + i] = double(sb[(int64_t(m) * a.rs + NX * a.T + q) * a.Bmax]);
  }
}

// ------------------------------------------------------------------ FP64 check of the stopping iterate

// Trajectory y = Phi^{k+1} x0 of each instance recomputed in FP64 from its compact stopping
// state (the FP32 values taken as exact): with g the global stopping iteration, alpha^{k+1} in
// plane g & 1 and alpha^k in the other, eta likewise and tau = tau^{k+1}, row r of subsystem m
//   a_r = c b_r + sum_{j in P(m)} ||x0_j||^2 [N_j (tau^k + eta^k)]_r - n_r alpha^k_r,
//   tau^k = tau^{k+1} - eta^{k+1},  b_r = sum_{j in P(m)} sum_c x0_c o_c[r],
//   y_r = a_r + n_r alpha^{k+1}_r   (the Phi-comp row value, Phi row = v + alpha x_r),
// with the FP64 bases and offsets and c as in bphi_kernel. bcheck_w_kernel writes
// W_j = ||x0_j||^2 (tau^k + eta^k) for every instance of the slot list ([Ktot][64],
// zero past k_j, in wchk); bcheck_y_kernel (one block per row subsystem m) runs the products
// N_j[rows of m] (rs x k_j) W_j (k_j x S) as FP64 matrix-core products (v_mfma_f64_16x16x4: lane l
// holds A[l % 16][l / 16], B[l / 16][l % 16], and D[l / 16 + 4 v][l % 16], the output layout
// measured on gfx950); wave w owns row tile w (rs <= 64) and all instance tiles, 32 basis rows of
// A in flight per lane before their products.
typedef double f64x4 __attribute__((ext_vector_type(4)));

struct ChkInst {  // stopping state of instance bi of the slot list
  int b;          // slot
  const double *x;  // its FP64 x0
  int cur;        // plane of the stopping iterate
  double coef;    // coefficient of b_r in its last Phi-comp
  bool use_w;     // its last Phi-comp had the basis term
};

template <int NX>
__device__ __forceinline__ ChkInst chk_inst(const BArgs &a, const double *x0, const int32_t *slots,
                                            const int32_t *xsrc, int bi) {
  ChkInst c;
  c.b = slots ? slots[bi] : bi;
  c.x = x0 + int64_t(xsrc ? xsrc[bi] : bi) * a.N * NX;
  const BCtl &ic = a.ictl[c.b];
  const int g = ic.it0 + ic.iters;
  const bool warm = a.ctl->warm != 0;
  c.cur = g & 1;
  c.coef = warm ? 1.0 : (g == 1 ? 0.0 : (g == 2 ? 2.0 : 1.0));
  c.use_w = warm || g >= 3;
  return c;
}

template <int NX>
__global__ __launch_bounds__(256) void bcheck_w_kernel(BArgs a, const double *x0, const int32_t *slots,
                                                       const int32_t *xsrc, int S) {
  const int j = blockIdx.x;
  const int64_t k0 = a.koff[j];
  const int k = a.kdim[j], k32 = int(a.koff[j + 1] - k0);
  const int64_t eplane = a.ktot * a.Bmax;
  for (int e = threadIdx.x; e < k32 * kBMax; e += 256) {
    const int i = e / kBMax, bi = e - i * kBMax;
    double v = 0.0;
    if (i < k && bi < S) {
      const ChkInst c = chk_inst<NX>(a, x0, slots, xsrc, bi);
      if (c.use_w) {
        double x2 = 0.0;
#pragma unroll
        for (int q = 0; q < NX; ++q) x2 += c.x[j * NX + q] * c.x[j * NX + q];
        const int64_t ki = (k0 + i) * a.Bmax + c.b;
        v = x2 * ((double(a.tau[ki]) - double(a.eta[ki + (c.cur ? eplane : 0)])) +
                  double(a.eta[ki + (c.cur ? 0 : eplane)]));
      }
    }
    a.wchk[(k0 + i) * kBMax + bi] = v;
  }
}

template <int NX>
__global__ __launch_bounds__(256) void bcheck_y_kernel(BArgs a, const double *x0, const int32_t *slots,
                                                       const int32_t *xsrc, int S) {
  // The product operand of each step (tile of m's row, 32 basis vectors) is staged once per
  // block in LDS (two buffers, one barrier per step; the waves past rs only stage), and the
  // next step's operand and basis rows are loaded while the current step's products run.
  __shared__ __align__(16) double sW[2][32][kBMax];
  __shared__ const double *s_nj[kMaxPatch];
  __shared__ int64_t s_w[kMaxPatch];
  __shared__ int s_ld[kMaxPatch], s_k[kMaxPatch];
  const int m = blockIdx.x, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int rs = a.rs;
  const bool act = 16 * w < rs;
  const int ntl = (S + 15) >> 4;  // instance tiles in use
  const int64_t q0 = a.rt_ptr[m];
  const int pm = int(a.rt_ptr[m + 1] - q0);
  if (tid < pm) {
    const int j = a.rt_col[q0 + tid];
    const int D = int(a.tile_off[j + 1] - a.tile_off[j]) * rs;
    s_ld[tid] = (D + 3) & ~3;
    s_k[tid] = a.kdim[j];
    s_nj[tid] = a.nb64 + a.nb_off[j] + int64_t(a.rt_tile[q0 + tid] - a.tile_off[j]) * rs;
    s_w[tid] = a.koff[j] * kBMax;  // rows koff_j .. of wchk (zero past k_j up to a multiple of 32)
  }
  __syncthreads();
  f64x4 acc[kNT];
#pragma unroll
  for (int nt = 0; nt < kNT; ++nt) acc[nt] = f64x4{0.0, 0.0, 0.0, 0.0};
  const int row = 16 * w + (lane & 15);  // A operand row of this lane
  const bool rok = act && row < rs;
  // steps (tile t, first basis vector s) in the order of the tiles, 32 vectors per step
  auto next = [&](int &t, int &s) {
    s += 32;
    while (t < pm && s >= s_k[t]) {
      ++t;
      s = 0;
    }
    return t < pm;
  };
  double wv[8], avc[8], avn[8];
  auto load = [&](int t, int s, double *av) {
    const double *src = a.wchk + s_w[t] + int64_t(s) * kBMax + tid * 8;  // 32 x 64 contiguous
#pragma unroll
    for (int e = 0; e < 8; ++e) wv[e] = src[e];
    const double *nj = s_nj[t] + row;
    const int ld = s_ld[t], k = s_k[t];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = s + 4 * u + (lane >> 4);
      av[u] = (rok && i < k) ? nj[int64_t(i) * ld] : 0.0;
    }
  };
  auto stage = [&](int buf) {
    double *d = &sW[buf][0][0] + tid * 8;
#pragma unroll
    for (int e = 0; e < 8; ++e) d[e] = wv[e];
  };
  int ct = 0, cs = -32;
  bool ok = next(ct, cs);
  if (ok) {
    load(ct, cs, avc);
    stage(0);
  }
  __syncthreads();
  int buf = 0;
  while (ok) {
    int tn = ct, sn = cs;
    const bool more = next(tn, sn);
    if (more) load(tn, sn, avn);
    if (act) {
#pragma unroll
      for (int u = 0; u < 8; ++u)
#pragma unroll
        for (int nt = 0; nt < kNT; ++nt) {
          if (nt >= ntl) break;
          const double bv = sW[buf][4 * u + (lane >> 4)][16 * nt + (lane & 15)];
          acc[nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(avc[u], bv, acc[nt], 0, 0, 0);
        }
    }
    if (more) stage(buf ^ 1);  // read last in the previous step, before its barrier
    __syncthreads();
    buf ^= 1;
    ct = tn;
    cs = sn;
    ok = more;
#pragma unroll
    for (int u = 0; u < 8; ++u) avc[u] = avn[u];
  }
  if (!act) return;  // no barriers below
  // epilogue: lane holds rows 16 w + lane / 16 + 4 v of instance 16 nt + lane % 16
  const int64_t plane = int64_t(a.Bmax) * a.N * rs;
#pragma unroll
  for (int nt = 0; nt < kNT; ++nt) {
    if (nt >= ntl) break;
    const int bi = 16 * nt + (lane & 15);
    if (bi >= S) continue;
    const ChkInst c = chk_inst<NX>(a, x0, slots, xsrc, bi);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int l = 16 * w + (lane >> 4) + 4 * v;
      if (l >= rs) continue;
      double bsum = 0.0, nr = 0.0;
      for (int64_t q = a.rt_ptr[m]; q < a.rt_ptr[m + 1]; ++q) {
        const int j = a.rt_col[q];
        const int D = int(a.tile_off[j + 1] - a.tile_off[j]) * rs;
        const int ld = (D + 3) & ~3;
        const int ro = int(a.rt_tile[q] - a.tile_off[j]) * rs;
        const double *off = a.off64 + a.off_ptr[j] + ro + l;
#pragma unroll
        for (int cc = 0; cc < NX; ++cc) {
          const double xc = c.x[j * NX + cc];
          bsum += xc * off[int64_t(cc) * ld];
          nr += xc * xc;
        }
      }
      const int64_t rb = (int64_t(m) * rs + l) * a.Bmax + c.b;
      const double apv = a.alpha[(c.cur ? 0 : plane) + rb], acv = a.alpha[(c.cur ? plane : 0) + rb];
      a.y64[int64_t(c.b) * a.N * rs + int64_t(m) * rs + l] = ((c.coef * bsum + acc[nt][v]) - nr * apv) + nr * acv;
    }
  }
}

// Per instance from y64: largest |x_0 - x0| and |x_{t+1} - A x_t - B u_t| (Z_AB y - [x0; 0]),
// largest bound violation, largest |u(0) returned (the FP32 row values) - u(0) of y64|, and
// sum_r w_r y_r^2. Block (instance, part): the subsystems of part blockIdx.y of kParts; the
// parts' maxima and partial sums are combined, the sums in part order, by bcheck_fin_kernel.
template <int NX>
__global__ __launch_bounds__(256) void bcheck_red_kernel(BArgs a, const double *x0, const int32_t *slots,
                                                         const int32_t *xsrc, int S) {
  __shared__ double r_eq[4], r_box[4], r_u[4], r_j[4];
  const int bi = blockIdx.x, tid = threadIdx.x, part = blockIdx.y;
  const int b = slots ? slots[bi] : bi;
  const double *xb = x0 + int64_t(xsrc ? xsrc[bi] : bi) * a.N * NX;
  const int rs = a.rs, nu = a.nu, T = a.T;
  const double *y = a.y64 + int64_t(b) * a.N * rs;
  const int chunk = (a.N + kParts - 1) / kParts, m1 = min(a.N, (part + 1) * chunk);
  double eq = 0.0, box = 0.0, ud = 0.0, jv = 0.0;
  for (int m = part * chunk + tid; m < m1; m += 256) {
    const double *ym = y + int64_t(m) * rs;
#pragma unroll
    for (int c = 0; c < NX; ++c) eq = fmax(eq, fabs(ym[c] - xb[m * NX + c]));
    for (int t = 0; t + 1 < T; ++t) {
      double v[NX];
#pragma unroll
      for (int c = 0; c < NX; ++c) v[c] = ym[(t + 1) * NX + c];
      for (int64_t q = a.a_rowptr[m]; q < a.a_rowptr[m + 1]; ++q) {
        const double *blk = a.a64 + q * NX * NX;
        const double *xj = y + int64_t(a.a_colidx[q]) * rs + t * NX;
#pragma unroll
        for (int c = 0; c < NX; ++c)
#pragma unroll
          for (int c2 = 0; c2 < NX; ++c2) v[c] -= blk[c * NX + c2] * xj[c2];
      }
      const double *bb = a.b64 + int64_t(m) * NX * nu;
      for (int q = 0; q < nu; ++q)
#pragma unroll
        for (int c = 0; c < NX; ++c) v[c] -= bb[c * nu + q] * ym[NX * T + t * nu + q];
#pragma unroll
      for (int c = 0; c < NX; ++c) eq = fmax(eq, fabs(v[c]));
    }
    for (int l = 0; l < rs; ++l) {
      const int64_t o = int64_t(m) * rs + l;
      const double yv = ym[l];
      box = fmax(box, fmax(a.lb64[o] - yv, yv - a.ub64[o]));
      jv += a.w64[o] * yv * yv;
    }
    for (int q = 0; q < nu; ++q) {
      const int64_t o = int64_t(m) * rs + NX * T + q;
      ud = fmax(ud, fabs(double(a.s[o * a.Bmax + b]) - ym[NX * T + q]));
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    eq = fmax(eq, __shfl_xor(eq, o, 64));
    box = fmax(box, __shfl_xor(box, o, 64));
    ud = fmax(ud, __shfl_xor(ud, o, 64));
    jv += __shfl_xor(jv, o, 64);
  }
  if ((tid & 63) == 0) {
    r_eq[tid >> 6] = eq;
    r_box[tid >> 6] = box;
    r_u[tid >> 6] = ud;
    r_j[tid >> 6] = jv;
  }
  __syncthreads();
  if (tid == 0) {
    double *o = a.chkpart + (int64_t(b) * kParts + part) * 4;
    o[0] = fmax(fmax(r_eq[0], r_eq[1]), fmax(r_eq[2], r_eq[3]));
    o[1] = fmax(0.0, fmax(fmax(r_box[0], r_box[1]), fmax(r_box[2], r_box[3])));
    o[2] = fmax(fmax(r_u[0], r_u[1]), fmax(r_u[2], r_u[3]));
    o[3] = (r_j[0] + r_j[1]) + (r_j[2] + r_j[3]);
  }
}

__global__ __launch_bounds__(64) void bcheck_fin_kernel(BArgs a, const int32_t *slots, int S) {
  for (int bi = threadIdx.x; bi < S; bi += 64) {
    const int b = slots ? slots[bi] : bi;
    const double *o = a.chkpart + int64_t(b) * kParts * 4;
    double eq = 0.0, box = 0.0, ud = 0.0, jv = 0.0;
    for (int q = 0; q < kParts; ++q) {
      eq = fmax(eq, o[4 * q]);
      box = fmax(box, o[4 * q + 1]);
      ud = fmax(ud, o[4 * q + 2]);
      jv += o[4 * q + 3];
    }
    BCtl &ic = a.ictl[b];
    ic.eq_resid = eq;
    ic.box = box;
    ic.u0dev = ud;
    ic.objective64 = jv;
  }
}

// ------------------------------------------------------------------ closed loop (Algorithm 1)

// Plant step of every instance (FP64): x(t+1) = A x(t) + B u(t) with u(t) the u_0 rows just
// written to u [B][N*nu]; x(t) and u(t) are also stored in the loop's trajectories
// xs [B][T_sim+1][N*nx] (x(0) at t = 0) and us [B][T_sim][N*nu]. One block per instance.
template <int NX>
__global__ __launch_bounds__(256) void bplant_kernel(BArgs a, double *x, const double *u, double *xs, double *us,
                                                     int t, int T_sim, double *rscale) {
  const int b = blockIdx.x, tid = threadIdx.x, N = a.N, nu = a.nu;
  double *xb = x + int64_t(b) * N * NX;
  const double *ub = u + int64_t(b) * N * nu;
  double *xsb = xs + int64_t(b) * (T_sim + 1) * N * NX;
  double *usb = us + int64_t(b) * T_sim * N * nu;
  if (t == 0)
    for (int i = tid; i < N * NX; i += 256) xsb[i] = xb[i];
  for (int i = tid; i < N * nu; i += 256) usb[int64_t(t) * N * nu + i] = ub[i];
  // x(t+1) into the trajectory first (x itself is read by other threads of this block)
  double *xnext = xsb + int64_t(t + 1) * N * NX;
  for (int m = tid; m < N; m += 256) {
    double v[NX];
#pragma unroll
    for (int c = 0; c < NX; ++c) v[c] = 0.0;
    for (int64_t q = a.a_rowptr[m]; q < a.a_rowptr[m + 1]; ++q) {
      const double *blk = a.a64 + q * NX * NX;
      const double *xj = xb + int64_t(a.a_colidx[q]) * NX;
#pragma unroll
      for (int c = 0; c < NX; ++c)
#pragma unroll
        for (int c2 = 0; c2 < NX; ++c2) v[c] += blk[c * NX + c2] * xj[c2];
    }
    const double *bb = a.b64 + int64_t(m) * NX * nu;
    for (int k = 0; k < nu; ++k)
#pragma unroll
      for (int c = 0; c < NX; ++c) v[c] += bb[c * nu + k] * ub[int64_t(m) * nu + k];
#pragma unroll
    for (int c = 0; c < NX; ++c) xnext[m * NX + c] = v[c];
  }
  __syncthreads();
  double n1 = 0.0, n0 = 0.0;
  for (int i = tid; i < N * NX; i += 256) {
    xb[i] = xnext[i];
    n1 += xnext[i] * xnext[i];
    n0 += xsb[i] * xsb[i];
  }
  if (rscale) {
    // ||x(t+1)||^2 / ||x(0)||^2: the penalty factor of the next step's solve
    __shared__ double red[2][4];
    n1 = wsum(n1);
    n0 = wsum(n0);
    if ((tid & 63) == 0) {
      red[0][tid >> 6] = n1;
      red[1][tid >> 6] = n0;
    }
    __syncthreads();
    if (tid == 0) {
      const double s1 = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
      const double s0 = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
      rscale[b] = s0 > 0.0 ? fmax(s1 / s0, 1e-20) : 1.0;
    }
  }
}

// Stopping state of slots from[0..S) copied into stash slots to[0..S): what the FP64 check
// reads (both alpha and eta planes, tau, the row values s, the control block), so that streams
// refill the slots at once and check the stopped instances later, many at a time. One thread
// per row of the [rows][Bmax] arrays (alpha and s rows first, then the k-space rows).
__global__ __launch_bounds__(256) void bstash_kernel(BArgs a, BArgs st, const int32_t *from, const int32_t *to,
                                                     int S) {
  // one thread per (row, listed slot), the slots fastest (a row's entries share cache lines)
  __shared__ int s_f[kBMax], s_t[kBMax];
  if (threadIdx.x < S) {
    s_f[threadIdx.x] = from[threadIdx.x];
    s_t[threadIdx.x] = to[threadIdx.x];
  }
  __syncthreads();
  const int64_t R = int64_t(a.N) * a.rs, plane = R * a.Bmax, eplane = a.ktot * a.Bmax;
  const int64_t e = blockIdx.x * 256ll + threadIdx.x, r = e / S;
  const int y = int(e - r * S);
  if (e < S) st.ictl[s_t[e]] = a.ictl[s_f[e]];
  const int f = s_f[y], t = s_t[y];
  if (r < R) {
    const int64_t o = r * a.Bmax;
    st.alpha[o + t] = a.alpha[o + f];
    st.alpha[plane + o + t] = a.alpha[plane + o + f];
    st.s[o + t] = a.s[o + f];
  } else if (r < R + a.ktot) {
    const int64_t o = (r - R) * a.Bmax;
    st.tau[o + t] = a.tau[o + f];
    st.eta[o + t] = a.eta[o + f];
    st.eta[eplane + o + t] = a.eta[eplane + o + f];
  }
}

// Input rows of the trajectories y [B][N*rs] (library row order) moved one step ahead into ys:
// u_k <- u_{k+1} for k < T-2, u_{T-2} held (the start of the next step of the loop).
__global__ __launch_bounds__(256) void bshift_kernel(BArgs a, const double *y, double *ys, int B) {
  const int ux = a.nx * a.T, nur = a.rs - ux, nu = a.nu;
  const int64_t n = int64_t(B) * a.N * nur;
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
    const int64_t row = i / nur;  // b * N + g
    const int l = int(i - row * nur);
    const int k = l / nu;
    const int src = (k + 1 < a.T - 1) ? l + nu : l;
    ys[row * a.rs + ux + l] = y[row * a.rs + ux + src];
  }
}

// ------------------------------------------------------------------ trajectory warm start

// Input rows of y0 (FP64, [B][N*rs]) into yhat.
__global__ __launch_bounds__(256) void btraj_load_kernel(BArgs a, const double *y0, int B) {
  const int ux = a.nx * a.T, nur = a.rs - ux;
  const int64_t n = int64_t(B) * a.N * nur;
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
    const int64_t row = i / nur;  // b * N + g
    const int64_t o = row * a.rs + ux + (i - row * nur);
    a.yhat[o] = float(y0[o]);
  }
}

// State rows of yhat: x_0 = x0, x_{t+1} = sum_j A_ij x_j(t) + B_i u_i(t), one block per
// instance, one time step per barrier interval.
template <int NX>
__global__ __launch_bounds__(1024) void bsim_kernel(BArgs a, const int32_t *slots) {
  const int b = slots ? slots[blockIdx.x] : blockIdx.x, tid = threadIdx.x;
  const int rs = a.rs, nu = a.nu, N = a.N;
  float *y = a.yhat + int64_t(b) * N * rs;
  const float *x0 = a.x0 + int64_t(b) * N * NX;
  for (int i = tid; i < N; i += 1024)
#pragma unroll
    for (int c = 0; c < NX; ++c) y[int64_t(i) * rs + c] = x0[i * NX + c];
  __syncthreads();
  for (int t = 0; t + 1 < a.T; ++t) {
    for (int i = tid; i < N; i += 1024) {
      float v[NX];
#pragma unroll
      for (int c = 0; c < NX; ++c) v[c] = 0.f;
      for (int64_t q = a.a_rowptr[i]; q < a.a_rowptr[i + 1]; ++q) {
        const float *blk = a.a_blk + q * NX * NX;
        const float *xj = y + int64_t(a.a_colidx[q]) * rs + t * NX;
#pragma unroll
        for (int c = 0; c < NX; ++c)
#pragma unroll
          for (int c2 = 0; c2 < NX; ++c2) v[c] += blk[c * NX + c2] * xj[c2];
      }
      const float *u = y + int64_t(i) * rs + NX * a.T + t * nu;
      const float *bb = a.b_blk + int64_t(i) * NX * nu;
      for (int k = 0; k < nu; ++k)
#pragma unroll
        for (int c = 0; c < NX; ++c) v[c] += bb[c * nu + k] * u[k];
#pragma unroll
      for (int c = 0; c < NX; ++c) y[int64_t(i) * rs + (t + 1) * NX + c] = v[c];
    }
    __syncthreads();
  }
}

__device__ __forceinline__ double block_sum1024(double v, double *red) {
  v = wsum(v);
  __syncthreads();  // red may still be read by the previous call
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < 16; ++w) s += red[w];
  return s;
}

// r = yhat - b, p = r, x = 0, rr = r'r; alpha^0 = -2 w yhat / rho_b into plane `pl` (the one the
// next iteration reads as its previous iterate). Part blockIdx.y of kParts takes a contiguous
// row range; its share of r'r goes to the partial sums (added by bpart_sum_kernel).
__global__ __launch_bounds__(1024) void bcg_init_kernel(BArgs a, const int32_t *slots, int pl) {
  __shared__ double red[16];
  const int b = slots ? slots[blockIdx.x] : blockIdx.x, part = blockIdx.y;
  const int64_t plane = int64_t(a.Bmax) * a.N * a.rs;
  float *alpha = a.alpha + int64_t(pl < 0 ? 0 : pl) * plane;
  const int64_t ny = int64_t(a.N) * a.rs, o = int64_t(b) * ny, chunk = (ny + kParts - 1) / kParts;
  const int64_t r0 = part * chunk, r1 = min(ny, r0 + chunk);
  double acc = 0.0;
  const float rho = a.rho_b[b];
  for (int64_t i = r0 + threadIdx.x; i < r1; i += 1024) {
    const float y = a.yhat[o + i];
    const float r = y - a.bvec[i * a.Bmax + b];
    a.cg_r[o + i] = r;
    a.cg_p[o + i] = r;
    a.cg_x[o + i] = 0.f;
    const float a0 = -2.f * a.w[i] * y / rho;
    alpha[i * a.Bmax + b] = a0;
    if (pl < 0) alpha[plane + i * a.Bmax + b] = a0;  // both planes: read by whichever iteration starts
    acc += double(r) * double(r);
  }
  acc = block_sum1024(acc, red);
  if (threadIdx.x == 0) a.bpart[int64_t(b) * 2 * kParts + part] = acc;
}

// One CG step per instance after cg_q = M cg_p, in three passes over kCgParts row ranges of
// the instance (the scalars are sums of the parts' partial sums in part order, so every part
// takes the same step): bcg_pq_kernel p'q; bcg_upd_kernel x += s p, r -= s q with s = r'r / p'q,
// and r'r of the new r; bcg_dir_kernel p = r + g p with g = new r'r / r'r. r'r of the step's
// start is cg_rr; the new one goes to cg_rrn and becomes cg_rr in the next step's first pass.
// gate: inside the iteration, only instances whose Phi-comp just wrote q = M p (phase
// 1..cg_k); otherwise instances 0..gridDim.x-1.
__device__ __forceinline__ bool cg_gated(const BArgs &a, int b, int gate) {
  if (!gate) return true;
  if (a.ctl->stop || b >= a.ctl->batch || a.ictl[b].stop) return false;
  const int ph = a.phase[b];
  return ph >= 1 && ph <= a.ctl->cg_k;
}

__device__ __forceinline__ double block_sum256(double v, double *red) {
  v = wsum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

__device__ __forceinline__ double cg_part_sum(const double *p) {
  double v = 0.0;
#pragma unroll
  for (int q = 0; q < kCgParts; ++q) v += p[q];
  return v;
}

__global__ __launch_bounds__(256) void bcg_pq_kernel(BArgs a, int gate) {
  __shared__ double red[4];
  const int b = blockIdx.x, part = blockIdx.y;
  if (!cg_gated(a, b, gate)) return;
  const int64_t ny = int64_t(a.N) * a.rs, o = int64_t(b) * ny, chunk = (ny + kCgParts - 1) / kCgParts;
  const int64_t r0 = part * chunk, r1 = min(ny, r0 + chunk);
  double pq = 0.0;
  for (int64_t i = r0 + threadIdx.x; i < r1; i += 256) pq += double(a.cg_p[o + i]) * double(a.cg_q[o + i]);
  pq = block_sum256(pq, red);
  if (threadIdx.x == 0) {
    a.cgpart[int64_t(b) * 2 * kCgParts + part] = pq;
    if (part == 0) a.cg_rr[b] = a.cg_rrn[b];
  }
}

__global__ __launch_bounds__(256) void bcg_upd_kernel(BArgs a, int gate) {
  __shared__ double red[4];
  const int b = blockIdx.x, part = blockIdx.y;
  if (!cg_gated(a, b, gate)) return;
  const double rr = a.cg_rr[b], pq = cg_part_sum(a.cgpart + int64_t(b) * 2 * kCgParts);
  if (!(rr > 0.0) || !(pq > 0.0)) return;  // converged (or breakdown): keep x
  const float step = float(rr / pq);
  const int64_t ny = int64_t(a.N) * a.rs, o = int64_t(b) * ny, chunk = (ny + kCgParts - 1) / kCgParts;
  const int64_t r0 = part * chunk, r1 = min(ny, r0 + chunk);
  double rn = 0.0;
  for (int64_t i = r0 + threadIdx.x; i < r1; i += 256) {
    a.cg_x[o + i] += step * a.cg_p[o + i];
    const float r = a.cg_r[o + i] - step * a.cg_q[o + i];
    a.cg_r[o + i] = r;
    rn += double(r) * double(r);
  }
  rn = block_sum256(rn, red);
  if (threadIdx.x == 0) a.cgpart[(int64_t(b) * 2 + 1) * kCgParts + part] = rn;
}

__global__ __launch_bounds__(256) void bcg_dir_kernel(BArgs a, int gate) {
  const int b = blockIdx.x, part = blockIdx.y;
  if (!cg_gated(a, b, gate)) return;
  const double rr = a.cg_rr[b], pq = cg_part_sum(a.cgpart + int64_t(b) * 2 * kCgParts);
  if (!(rr > 0.0) || !(pq > 0.0)) return;
  const double rn = cg_part_sum(a.cgpart + (int64_t(b) * 2 + 1) * kCgParts);
  const float g = float(rn / rr);
  const int64_t ny = int64_t(a.N) * a.rs, o = int64_t(b) * ny, chunk = (ny + kCgParts - 1) / kCgParts;
  const int64_t r0 = part * chunk, r1 = min(ny, r0 + chunk);
  for (int64_t i = r0 + threadIdx.x; i < r1; i += 256) a.cg_p[o + i] = a.cg_r[o + i] + g * a.cg_p[o + i];
  if (part == 0 && threadIdx.x == 0) a.cg_rrn[b] = rn;
}

__global__ __launch_bounds__(256) void bexport_y_kernel(BArgs a, double *out, int B) {
  const int64_t n = int64_t(B) * a.N * a.rs;
  const int64_t ny = int64_t(a.N) * a.rs;
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
    const int64_t b = i / ny;
    out[i] = double(a.s[(i - b * ny) * a.Bmax + b]);
  }
}

// Rows of src ([S][ny], FP32) into rows slots[0..S) of dst ([Bmax][ny]).
__global__ __launch_bounds__(256) void bscatter_rows_kernel(const float *src, const int32_t *slots, int64_t ny,
                                                            float *dst) {
  const int y = blockIdx.x;
  const float *s = src + int64_t(y) * ny;
  float *d = dst + int64_t(slots[y]) * ny;
  for (int64_t i = int64_t(blockIdx.y) * 256 + threadIdx.x; i < ny; i += int64_t(gridDim.y) * 256) d[i] = s[i];
}

// ------------------------------------------------------------------ engine

#define BENG_CHECK(expr)                                                  \
  do {                                                                    \
    hipError_t e_ = (expr);                                               \
    if (e_ != hipSuccess) {                                               \
      err = std::string(#expr) + ": " + hipGetErrorString(e_);            \
      return DLMPC_EDEVICE;                                               \
    }                                                                     \
  } while (0)

// Null bases from the device factorisation (FP64, column-major, padded leading dimension) into
// the fragment orders ntf and nf (bf16 hi at [l*8+e], with split operands lo 512 further;
// layouts as built on the host from the same bases). Block (j, y) strides over the
// k_j x D_col(j) entries of N_j.
__global__ void bfrag_kernel(const double *__restrict__ nb, const int64_t *__restrict__ nb_off,
                             const int32_t *__restrict__ kdim, const int64_t *__restrict__ tile_off,
                             const int64_t *__restrict__ ntf_off, const int64_t *__restrict__ nf_off, int rs,
                             int split, __bf16 *__restrict__ ntf, __bf16 *__restrict__ nf) {
  const int fb = split ? 1024 : 512;
  const int j = blockIdx.x;
  const int64_t t0 = tile_off[j];
  const int D = int(tile_off[j + 1] - t0) * rs, k = kdim[j], ld = (D + 3) & ~3;
  const int nkt_c = (D + kKC - 1) / kKC * kKC / 32, nkt_r = ((k + 31) & ~31) / 32;
  const double *Nj = nb + nb_off[j];
  for (int64_t e = int64_t(blockIdx.y) * blockDim.x + threadIdx.x; e < int64_t(k) * D;
       e += int64_t(gridDim.y) * blockDim.x) {
    const int i = int(e / D), r = int(e % D);
    const float x = float(Nj[int64_t(i) * ld + r]);
    const __bf16 h = static_cast<__bf16>(x);
    const __bf16 lo = static_cast<__bf16>(x - static_cast<float>(h));
    {  // ntf: M = basis i, K = row r
      const int mt = i / 16, kt = r / 32, kk = r % 32;
      const int l = (i % 16) + 16 * (kk / 8), el = kk % 8;
      const int64_t at = ntf_off[j] + (int64_t(mt) * nkt_c + kt) * fb + l * 8 + el;
      ntf[at] = h;
      if (split) ntf[at + 512] = lo;
    }
    {  // nf: M = row of the tile, K = basis i
      const int t = r / rs, rr = r % rs;
      const int rt = rr / 16, kt = i / 32, kk = i % 32;
      const int l = (rr % 16) + 16 * (kk / 8), el = kk % 8;
      const int64_t at = nf_off[t0 + t] + (int64_t(rt) * nkt_r + kt) * fb + l * 8 + el;
      nf[at] = h;
      if (split) nf[at + 512] = lo;
    }
  }
}

// Fragments of N_u' for the structured Psi-comp: M = basis i, K = input row ku in the order of
// the adjoint recursion (step q = ku / (p nu) holds u_{T-2-q}, member-major within the step).
__global__ void bfragu_kernel(const double *__restrict__ nb, const int64_t *__restrict__ nb_off,
                              const int32_t *__restrict__ kdim, const int64_t *__restrict__ tile_off,
                              const int64_t *__restrict__ ntu_off, int rs, int nx, int nu, int T,
                              __bf16 *__restrict__ ntu) {
  const int j = blockIdx.x;
  const int p = int(tile_off[j + 1] - tile_off[j]);
  const int D = p * rs, k = kdim[j], ld = (D + 3) & ~3, pnu = p * nu, mu = (T - 1) * pnu;
  const int nku = (mu + kKC - 1) / kKC * kKC / 32;
  const double *Nj = nb + nb_off[j];
  for (int64_t e = int64_t(blockIdx.y) * blockDim.x + threadIdx.x; e < int64_t(k) * mu;
       e += int64_t(gridDim.y) * blockDim.x) {
    const int i = int(e / mu), ku = int(e % mu);
    const int q = ku / pnu, w = ku - q * pnu, ti = w / nu, kk = w - ti * nu;
    const int r = ti * rs + nx * T + (T - 2 - q) * nu + kk;
    const float x = float(Nj[int64_t(i) * ld + r]);
    const __bf16 h = static_cast<__bf16>(x);
    const int mt = i / 16, kt = ku / 32, kq = ku % 32;
    const int l = (i % 16) + 16 * (kq / 8), el = kq % 8;
    const int64_t at = ntu_off[j] + (int64_t(mt) * nku + kt) * 1024 + l * 8 + el;
    ntu[at] = h;
    ntu[at + 512] = static_cast<__bf16>(x - static_cast<float>(h));
  }
}

// Psi-comp work units: column blocks whose basis is more than capx times the mean are split into
// np row ranges of whole kKC-row chunks, so that a heavy patch is served by np blocks (more waves
// per patch) whose partial sums the last one adds; units are dispatched heaviest first.
// Candidates of the autotuner; the default 8 was the fastest on the 1024 mesh when fixed by hand
// (splitting blocks of two to four times the mean cost more in partial sums than it gained).
constexpr int kPsiCaps[] = {2, 4, 8, 16, 1 << 20};
constexpr int kPsiCapDefault = 8;

struct PsiSplit {
  std::vector<int32_t> pu_j, pu_r0, pu_r1, pu_p, pj_n, pj_first;
  std::vector<int64_t> pj_off;
  int64_t poff = 0;
  int32_t pfirst = 0;
};

PsiSplit psi_split(const HostSetup &hs, int capx) {
  const int N = hs.N;
  std::vector<int64_t> cost(N);
  int64_t csum = 0;
  for (int j = 0; j < N; ++j) {
    const int64_t D = int64_t(hs.patch[j].size()) * hs.rs;
    cost[j] = ((D + kKC - 1) / kKC * kKC) * ((hs.kdim[j] + 15) & ~15);
    csum += cost[j];
  }
  const int64_t cap = std::max<int64_t>(1, int64_t(capx) * csum / N);
  struct Unit { int32_t j, r0, r1, p; int64_t c; };
  std::vector<Unit> units;
  PsiSplit sp;
  sp.pj_n.assign(N, 1);
  sp.pj_first.assign(N, 0);
  sp.pj_off.assign(N, 0);
  for (int j = 0; j < N; ++j) {
    const int D = int(hs.patch[j].size()) * hs.rs, chunks = (D + kKC - 1) / kKC;
    const int np = int(std::min<int64_t>(chunks, (cost[j] + cap - 1) / cap));
    const int per = (chunks + np - 1) / np;
    int p = 0;
    for (int c0 = 0; c0 < chunks; c0 += per, ++p)
      units.push_back({j, kKC * c0, kKC * std::min(chunks, c0 + per), p,
                       cost[j] * (std::min(chunks, c0 + per) - c0) / chunks});
    sp.pj_n[j] = p;
    if (p > 1) {
      sp.pj_off[j] = sp.poff;
      sp.pj_first[j] = sp.pfirst;
      sp.poff += int64_t(p) * ((hs.kdim[j] + 15) & ~15) * kBMax;
      sp.pfirst += p;
    }
  }
  std::stable_sort(units.begin(), units.end(), [](const Unit &x, const Unit &y) { return x.c > y.c; });
  for (const Unit &u : units) {
    sp.pu_j.push_back(u.j);
    sp.pu_r0.push_back(u.r0);
    sp.pu_r1.push_back(u.r1);
    sp.pu_p.push_back(u.p);
  }
  return sp;
}

template <int NX>
class BatchEngineT final : public BatchEngine {
 public:
  int init(const HostSetup &hs, double rho, int bmax, bool split, hipStream_t s, std::string &err) override {
    if (bmax < 1 || bmax > kBMax) {
      err = "max_batch must be in 1..64";
      return DLMPC_EINVAL;
    }
    if (hs.k_max > kPsiWaves * kMTW * 16 || hs.rs > 64 || hs.p_max > kMaxPatch) {
      err = "batched engine needs k_j <= 512, nx*T + nu*(T-1) <= 64 and d-hop patches of <= 64 subsystems";
      return DLMPC_EINVAL;
    }
    split_ = split;
    const int64_t fb = split ? 1024 : 512;
    nrt_ = (hs.rs + 15) / 16;
    mtw_ = std::max(1, ((hs.k_max + 15) / 16 + kPsiWaves - 1) / kPsiWaves);
    hs_ = &hs;
    stream_ = s;
    BArgs &a = args_;
    a.N = hs.N;
    a.nx = hs.nx;
    a.nu = hs.nu;
    a.T = hs.T;
    a.rs = hs.rs;
    a.Bmax = bmax;
    a.rho = float(rho);
    const int N = hs.N;
    // Null bases in matrix-core fragment order (bf16 hi and lo of one fragment adjacent, fb =
    // 1024 values; hi only, fb = 512, when the operands are rounded once): a wave's load of one
    // fragment is one contiguous 1 KB block per half.
    //  ntf (left operand of N_j' alpha): fragment (M-tile mt of 16 basis vectors, K-step kt of
    //      32 support rows) of j at ntf_off[j] + (mt * nkt + kt) * fb, lane l, element e:
    //      N_j[32 kt + 8 (l / 16) + e][16 mt + l % 16];
    //  nf (left operand of N_j W_j for the rows of one tile (j, m)): fragment (row tile rt of 16
    //      rows of m, K-step kt of 32 basis vectors) at nf_off[tile] + (rt * nkt + kt) * fb:
    //      N_j[ro + 16 rt + l % 16][32 kt + 8 (l / 16) + e]; zero outside N_j.
    const int nrt = (hs.rs + 15) / 16;
    std::vector<int64_t> koff(N + 1, 0), ntf_off(N + 1, 0), nf_off(hs.n_tiles + 1, 0);
    for (int j = 0; j < N; ++j) {
      const int64_t D = int64_t(hs.patch[j].size()) * hs.rs, k = hs.kdim[j];
      const int64_t k32 = (k + 31) & ~31;
      koff[j + 1] = koff[j] + k32;
      ntf_off[j + 1] = ntf_off[j] + ((k + 15) & ~15) / 16 * ((D + kKC - 1) / kKC * kKC / 32) * fb;
      for (size_t t = 0; t < hs.patch[j].size(); ++t) {
        const int64_t tile = hs.tile_off[j] + int64_t(t);
        nf_off[tile + 1] = nf_off[tile] + int64_t(nrt) * (k32 / 32) * fb;
      }
    }
    a.ktot = koff[N];
    // Psi-comp work units (waves per patch): the default split and the largest any candidate of
    // the autotuner needs (buffers sized for it)
    PsiSplit sp = psi_split(hs, kPsiCapDefault);
    size_t max_units = 0;
    int64_t max_poff = 1;
    int32_t max_pfirst = 1;
    for (int capx : kPsiCaps) {
      const PsiSplit c = psi_split(hs, capx);
      max_units = std::max(max_units, c.pu_j.size());
      max_poff = std::max(max_poff, c.poff);
      max_pfirst = std::max(max_pfirst, c.pfirst);
    }
    // Phi-comp dispatch order: row subsystems with the most tiles first
    std::vector<int32_t> fo(N);
    for (int j = 0; j < N; ++j) fo[j] = j;
    std::stable_sort(fo.begin(), fo.end(), [&](int x, int y) { return hs.patch[x].size() > hs.patch[y].size(); });
    const __bf16 z = static_cast<__bf16>(0.f);
    int rc;
    if (hs.d_nb) {
      // bases on the device: build the fragments there
      __bf16 *d_ntf = nullptr, *d_nf = nullptr;
      const int64_t *d_nboff = nullptr, *d_ntfoff = nullptr, *d_nfoff = nullptr, *d_toff = nullptr;
      const int32_t *d_k = nullptr;
      if ((rc = al(&d_ntf, size_t(ntf_off[N]), err)) || (rc = al(&d_nf, size_t(nf_off[hs.n_tiles]), err)) ||
          (rc = up(hs.nb_off, &d_nboff, err)) || (rc = up(ntf_off, &d_ntfoff, err)) ||
          (rc = up(nf_off, &d_nfoff, err)) || (rc = up(hs.tile_off, &d_toff, err)) || (rc = up(hs.kdim, &d_k, err)))
        return rc;
      BENG_CHECK(hipMemset(d_ntf, 0, sizeof(__bf16) * std::max<int64_t>(ntf_off[N], 1)));
      BENG_CHECK(hipMemset(d_nf, 0, sizeof(__bf16) * std::max<int64_t>(nf_off[hs.n_tiles], 1)));
      hipLaunchKernelGGL(bfrag_kernel, dim3(N, 16), dim3(256), 0, nullptr, hs.d_nb, d_nboff, d_k, d_toff,
                         d_ntfoff, d_nfoff, hs.rs, int(split), d_ntf, d_nf);
      BENG_CHECK(hipGetLastError());
      BENG_CHECK(hipDeviceSynchronize());
      a.ntf = d_ntf;
      a.nf = d_nf;
    }
    std::vector<__bf16> ntf(hs.d_nb ? 0 : ntf_off[N], z), nf(hs.d_nb ? 0 : nf_off[hs.n_tiles], z);
    for (int j = 0; j < N && !hs.d_nb; ++j) {
      const int D = int(hs.patch[j].size()) * hs.rs, k = hs.kdim[j], ld = padded_ld(D);
      const int nkt_c = (D + kKC - 1) / kKC * kKC / 32, nkt_r = ((k + 31) & ~31) / 32;
      const double *Nj = hs.nb.data() + hs.nb_off[j];
      auto put = [&](std::vector<__bf16> &dst, int64_t at, double v) {
        const float x = float(v);
        const __bf16 h = static_cast<__bf16>(x);
        dst[at] = h;
        if (split) dst[at + 512] = static_cast<__bf16>(x - static_cast<float>(h));
      };
      for (int i = 0; i < k; ++i)
        for (int r = 0; r < D; ++r) {
          const double v = Nj[size_t(i) * ld + r];
          {  // ntf: M = basis i, K = row r
            const int mt = i / 16, kt = r / 32, kk = r % 32;
            const int l = (i % 16) + 16 * (kk / 8), e = kk % 8;
            put(ntf, ntf_off[j] + (int64_t(mt) * nkt_c + kt) * fb + l * 8 + e, v);
          }
          {  // nf: M = row of the tile, K = basis i
            const int t = r / hs.rs, rr = r % hs.rs;
            const int rt = rr / 16, kt = i / 32, kk = i % 32;
            const int l = (rr % 16) + 16 * (kk / 8), e = kk % 8;
            put(nf, nf_off[hs.tile_off[j] + t] + (int64_t(rt) * nkt_r + kt) * fb + l * 8 + e, v);
          }
        }
    }
    std::vector<double> on2(size_t(N) * NX, 0.0);
    for (int j = 0; j < N; ++j) {
      const int D = int(hs.patch[j].size()) * hs.rs, ld = padded_ld(D);
      for (int c = 0; c < NX; ++c)
        for (int r = 0; r < D; ++r) {
          const double o = hs.off[hs.off_ptr[j] + size_t(c) * ld + r];
          on2[size_t(j) * NX + c] += o * o;
        }
    }
    if (!hs.d_nb && ((rc = up(ntf, &a.ntf, err)) || (rc = up(nf, &a.nf, err)))) return rc;
    if ((rc = up(hs.tile_off, &a.tile_off, err)) || (rc = up(hs.rt_ptr, &a.rt_ptr, err)) ||
        (rc = up(hs.rt_tile, &a.rt_tile, err)) || (rc = up(hs.rt_col, &a.rt_col, err)) ||
        (rc = up(hs.kdim, &a.kdim, err)) || (rc = up(hs.tile_rsub, &a.tile_rsub, err)) ||
        (rc = up(koff, &a.koff, err)) || (rc = up(ntf_off, &a.ntf_off, err)) || (rc = up(nf_off, &a.nf_off, err)) ||
        (rc = up(hs.off_ptr, &a.off_ptr, err)) || (rc = up(on2, &a.onorm2, err)) ||
        (rc = up(hs.w, &a.w64, err)) || (rc = up(fo, &a.phi_order, err)))
      return rc;
    int32_t *d_pu_j = nullptr, *d_pu_r0 = nullptr, *d_pu_r1 = nullptr, *d_pu_p = nullptr;
    int32_t *d_pj_n = nullptr, *d_pj_first = nullptr;
    int64_t *d_pj_off = nullptr;
    if ((rc = al(&d_pu_j, max_units, err)) || (rc = al(&d_pu_r0, max_units, err)) ||
        (rc = al(&d_pu_r1, max_units, err)) || (rc = al(&d_pu_p, max_units, err)) ||
        (rc = al(&d_pj_n, size_t(N), err)) || (rc = al(&d_pj_first, size_t(N), err)) ||
        (rc = al(&d_pj_off, size_t(N), err)))
      return rc;
    a.pu_j = d_pu_j;
    a.pu_r0 = d_pu_r0;
    a.pu_r1 = d_pu_r1;
    a.pu_p = d_pu_p;
    a.pj_n = d_pj_n;
    a.pj_first = d_pj_first;
    a.pj_off = d_pj_off;
    if ((rc = al(&a.ppart, size_t(max_poff), err)) ||
        (rc = al(&a.ppod, size_t(max_pfirst) * kBMax * 8 * NX, err)) || (rc = al(&a.pcnt, size_t(N), err)))
      return rc;
    if ((rc = load_split(sp, kPsiCapDefault, err))) return rc;
    BENG_CHECK(hipMemset(a.pcnt, 0, sizeof(int32_t) * N));
    // structured Psi-comp (split operands, bases on the device, patches within its staging):
    // N_u fragments and the transposed patch dynamics
    struct_ok_ = false;
    {
      int ns_max = 0, pnu_max = 0;
      for (int j = 0; j < N; ++j) {
        ns_max = std::max(ns_max, int(hs.patch[j].size()) * NX);
        pnu_max = std::max(pnu_max, int(hs.patch[j].size()) * hs.nu);
      }
      if (split && hs.d_nb && ns_max <= kSNs && pnu_max <= kSPnu && hs.T >= 2) {
        int32_t nnz_max = 0;
        std::vector<int64_t> ntu_off(N + 1, 0), srp0(N), se0(N);
        std::vector<int32_t> srpt, scolt;
        std::vector<float> svalt;
        for (int j = 0; j < N; ++j) {
          const std::vector<int32_t> &P = hs.patch[j];
          const int p = int(P.size()), mu = (hs.T - 1) * p * hs.nu, ns = p * NX;
          const int64_t nku = (mu + kKC - 1) / kKC * kKC / 32, nmt = ((hs.kdim[j] + 15) & ~15) / 16;
          ntu_off[j + 1] = ntu_off[j] + nmt * nku * 1024;
          std::vector<std::vector<std::pair<int32_t, float>>> cols(ns);
          for (int ti = 0; ti < p; ++ti) {
            const int m = P[ti];
            for (int64_t q = hs.a_rowptr[m]; q < hs.a_rowptr[m + 1]; ++q) {
              const auto it = std::lower_bound(P.begin(), P.end(), hs.a_colidx[q]);
              if (it == P.end() || *it != hs.a_colidx[q]) continue;
              const int tn = int(it - P.begin());
              for (int st = 0; st < NX; ++st)
                for (int s2 = 0; s2 < NX; ++s2) {
                  const double v = hs.a_blocks[size_t(q) * NX * NX + st * NX + s2];
                  if (v != 0.0) cols[tn * NX + s2].push_back({ti * NX + st, float(v)});
                }
            }
          }
          srp0[j] = int64_t(srpt.size());
          se0[j] = int64_t(scolt.size());
          int32_t c = 0;
          srpt.push_back(0);
          for (int r = 0; r < ns; ++r) {
            for (const auto &e : cols[r]) {
              scolt.push_back(e.first);
              svalt.push_back(e.second);
            }
            c += int32_t(cols[r].size());
            srpt.push_back(c);
          }
          nnz_max = std::max(nnz_max, c);
        }
        __bf16 *d_ntu = nullptr;
        const int64_t *d_nboff = nullptr, *d_ntuoff = nullptr, *d_toff = nullptr;
        const int32_t *d_k = nullptr;
        if (nnz_max <= kSNnz) {  // otherwise the patch dynamics exceed the kernel's staging
          if ((rc = al(&d_ntu, size_t(std::max<int64_t>(ntu_off[N], 1)), err)) || (rc = up(hs.nb_off, &d_nboff, err)) ||
              (rc = up(ntu_off, &d_ntuoff, err)) || (rc = up(hs.tile_off, &d_toff, err)) || (rc = up(hs.kdim, &d_k, err)) ||
              (rc = up(srp0, &a.srp0, err)) || (rc = up(se0, &a.se0, err)) || (rc = up(srpt, &a.srpt, err)) ||
              (rc = up(scolt, &a.scolt, err)) || (rc = up(svalt, &a.svalt, err)))
            return rc;
          BENG_CHECK(hipMemset(d_ntu, 0, sizeof(__bf16) * std::max<int64_t>(ntu_off[N], 1)));
          hipLaunchKernelGGL(bfragu_kernel, dim3(N, 16), dim3(256), 0, nullptr, hs.d_nb, d_nboff, d_k, d_toff, d_ntuoff,
                             hs.rs, hs.nx, hs.nu, hs.T, d_ntu);
          BENG_CHECK(hipGetLastError());
          BENG_CHECK(hipDeviceSynchronize());
          a.ntu = d_ntu;
          a.ntu_off = d_ntuoff;
          struct_ok_ = true;
        }
      }
    }
    std::vector<float> offf(hs.off.begin(), hs.off.end()), wf(hs.w.begin(), hs.w.end()),
        lbf(hs.lb.begin(), hs.lb.end()), ubf(hs.ub.begin(), hs.ub.end());
    if ((rc = up(offf, &a.off, err)) || (rc = up(wf, &a.w, err)) || (rc = up(lbf, &a.lb, err)) ||
        (rc = up(ubf, &a.ub, err)))
      return rc;
    const size_t ny = size_t(N) * hs.rs;
    if ((rc = al(&a.alpha, 2 * size_t(bmax) * ny, err)) || (rc = al(&a.tau, size_t(bmax) * a.ktot, err)) ||
        (rc = al(&a.eta, 2 * size_t(bmax) * a.ktot, err)) || (rc = al(&a.xn, size_t(bmax) * N, err)) ||
        (rc = al(&a.nrm, size_t(bmax) * N, err)) || (rc = al(&a.bvec, size_t(bmax) * ny, err)) ||
        (rc = al(&a.s, size_t(bmax) * ny, err)) || (rc = al(&a.x0, size_t(bmax) * N * NX, err)) ||
        (rc = al(&a.ictl, size_t(bmax), err)) || (rc = al(&a.slot, 2 * size_t(bmax), err)) ||
        (rc = al(&a.ctl, 1, err)) || (rc = al(&d_slots_, size_t(bmax), err)) ||
        (rc = al(&d_xsrc_, size_t(bmax), err)) ||
        (rc = al(&d_oslots_, size_t(bmax), err)) || (rc = al(&d_odst_, size_t(bmax), err)) ||
        (rc = al(&d_cslots_, size_t(bmax), err)) || (rc = al(&d_cdst_, size_t(bmax), err)) ||
        (rc = al(&d_sfrom_, size_t(bmax), err)) || (rc = al(&d_sto_, size_t(bmax), err)) ||
        (rc = al(&sk_alpha_, 2 * size_t(bmax) * ny, err)) || (rc = al(&sk_s_, size_t(bmax) * ny, err)) ||
        (rc = al(&sk_tau_, size_t(bmax) * a.ktot, err)) || (rc = al(&sk_eta_, 2 * size_t(bmax) * a.ktot, err)) ||
        (rc = al(&sk_ictl_, size_t(bmax), err)) ||
        (rc = al(&a.phase, size_t(bmax), err)) || (rc = al(&a.rho_b, size_t(bmax), err)))
      return rc;
    {
      const std::vector<int32_t> adm(bmax, -1);  // every slot in the ADMM iteration
      BENG_CHECK(hipMemcpy(a.phase, adm.data(), sizeof(int32_t) * bmax, hipMemcpyHostToDevice));
      const std::vector<float> rb(bmax, a.rho);
      BENG_CHECK(hipMemcpy(a.rho_b, rb.data(), sizeof(float) * bmax, hipMemcpyHostToDevice));
    }

    // trajectory warm start: vectors and the plant in FP32
    a.Bw = (bmax + 15) & ~15;
    if ((rc = al(&a.w_hi, size_t(a.Bw) * a.ktot, err)) || (rc = al(&a.w_lo, size_t(a.Bw) * a.ktot, err)) ||
        (rc = al(&a.dlm, size_t(bmax) * N, err)))
      return rc;
    // padded k entries and instances of W stay zero: the products read whole 32-wide k blocks
    // of 16 instances
    BENG_CHECK(hipMemset(a.w_hi, 0, sizeof(__bf16) * size_t(a.Bw) * a.ktot));
    BENG_CHECK(hipMemset(a.w_lo, 0, sizeof(__bf16) * size_t(a.Bw) * a.ktot));
    if ((rc = al(&a.yhat, size_t(bmax) * ny, err)) || (rc = al(&a.cg_x, size_t(bmax) * ny, err)) ||
        (rc = al(&a.cg_r, size_t(bmax) * ny, err)) || (rc = al(&a.cg_p, size_t(bmax) * ny, err)) ||
        (rc = al(&a.cg_q, size_t(bmax) * ny, err)) || (rc = al(&a.cg_rr, size_t(bmax), err)) ||
        (rc = al(&a.bpart, size_t(bmax) * 2 * kParts, err)) || (rc = al(&a.cg_rrn, size_t(bmax), err)) ||
        (rc = al(&a.cgpart, size_t(bmax) * 2 * kCgParts, err)) ||
        (rc = al(&a.chkpart, size_t(bmax) * kParts * 4, err)))
      return rc;
    std::vector<float> ablk(hs.a_blocks.begin(), hs.a_blocks.end()), bblk(hs.b_blocks.begin(), hs.b_blocks.end());
    if ((rc = up(hs.a_rowptr, &a.a_rowptr, err)) || (rc = up(hs.a_colidx, &a.a_colidx, err)) ||
        (rc = up(ablk, &a.a_blk, err)) || (rc = up(bblk, &a.b_blk, err)))
      return rc;
    // FP64 check of the stopping iterate: bases (the device factorisation's, or uploaded),
    // offsets, bounds, plant blocks, trajectory scratch
    if (hs.d_nb) {
      a.nb64 = hs.d_nb;
    } else {
      double *d = nullptr;
      if ((rc = al(&d, hs.nb.size(), err))) return rc;
      if (!hs.nb.empty()) BENG_CHECK(hipMemcpy(d, hs.nb.data(), hs.nb.size() * sizeof(double), hipMemcpyHostToDevice));
      a.nb64 = d;
    }
    {
      double *d = nullptr;
      if ((rc = al(&d, hs.off.size(), err))) return rc;
      if (!hs.off.empty()) BENG_CHECK(hipMemcpy(d, hs.off.data(), hs.off.size() * sizeof(double), hipMemcpyHostToDevice));
      a.off64 = d;
    }
    if ((rc = up(hs.nb_off, &a.nb_off, err)) || (rc = up(hs.lb, &a.lb64, err)) || (rc = up(hs.ub, &a.ub64, err)) ||
        (rc = up(hs.a_blocks, &a.a64, err)) || (rc = up(hs.b_blocks, &a.b64, err)) ||
        (rc = al(&a.y64, size_t(bmax) * ny, err)) || (rc = al(&a.wchk, size_t(kBMax) * a.ktot, err)))
      return rc;
    a.init_pass = 0;
    a.wmode = 0;
    a.src_bs = 1;
    a.src_rs = bmax;
    ny_ = int64_t(N) * hs.rs;
    a.phi_mode = 0;
    a.src = nullptr;
    a.dst_k = nullptr;
    BENG_CHECK(hipMemset(a.slot, 0, sizeof(unsigned long long) * 2 * bmax));
    return DLMPC_OK;
  }

  int precompute(const double *x0_dev, int B, int max_iter, double eps, int warm, const double *rho_scale_dev,
                 std::string &err) override {
    if (B < 1 || B > args_.Bmax) {
      err = "batch size out of range";
      return DLMPC_EINVAL;
    }
    B_ = B;
    hipLaunchKernelGGL((bprecompute_kernel<NX>), dim3(hs_->N, (B + kPreY - 1) / kPreY), dim3(256), 0, stream_, args_,
                       x0_dev, B,
                       warm ? 1 : 0, max_iter, eps, nullptr, nullptr, 1, 0, 0, rho_scale_dev);
    BENG_CHECK(hipGetLastError());
    return DLMPC_OK;
  }

  // dst_k = N_j' src for every column subsystem j and instance; wmode 1 also writes the
  // product operand W = ||x0_j||^2 dst_k, wmode 2 W = ||x0_j||^2 (tau + dst_k).
  int project_t(const float *src, int64_t src_bs, int64_t src_rs, float *dst_k, int wmode, std::string &err) {
    BArgs ia = args_;
    ia.init_pass = 1;
    ia.wmode = wmode;
    ia.src = src;
    ia.src_bs = src_bs;
    ia.src_rs = src_rs;
    ia.dst_k = dst_k;
    launch_psi(ia);
    BENG_CHECK(hipGetLastError());
    return DLMPC_OK;
  }

  int start_alpha(const double *alpha0_dev, std::string &err) override {
    hipLaunchKernelGGL(bwarm_alpha_kernel, dim3(1024), dim3(256), 0, stream_, args_, alpha0_dev, B_);
    BENG_CHECK(hipGetLastError());
    return project_t(args_.alpha, 1, args_.Bmax, args_.eta, 2, err);  // plane 0: previous iterate of iteration 1
  }

  int start_trajectory(const double *y0_dev, int cg_iters, std::string &err) override {
    if (y0_dev) {
      hipLaunchKernelGGL(btraj_load_kernel, dim3(1024), dim3(256), 0, stream_, args_, y0_dev, B_);
      BENG_CHECK(hipGetLastError());
    }
    hipLaunchKernelGGL((bsim_kernel<NX>), dim3(B_), dim3(1024), 0, stream_, args_, nullptr);
    BENG_CHECK(hipGetLastError());
    hipLaunchKernelGGL(bcg_init_kernel, dim3(B_, kParts), dim3(1024), 0, stream_, args_, nullptr, 0);
    BENG_CHECK(hipGetLastError());
    hipLaunchKernelGGL(bpart_sum_kernel, dim3(1), dim3(64), 0, stream_, args_, nullptr, B_, 0);
    BENG_CHECK(hipGetLastError());
    BArgs qa = args_;
    qa.phi_mode = 1;
    int rc;
    for (int k = 0; k < cg_iters; ++k) {
      if ((rc = project_t(args_.cg_p, ny_, 1, args_.eta, 1, err))) return rc;  // eta = N' p, W = ||x0_j||^2 eta
      launch_phi(qa);  // q = M p
      BENG_CHECK(hipGetLastError());
      launch_cg_step(B_, 0);
      BENG_CHECK(hipGetLastError());
    }
    if ((rc = project_t(args_.cg_x, ny_, 1, args_.tau, 0, err))) return rc;  // tau = N' beta
    return project_t(args_.alpha, 1, args_.Bmax, args_.eta, 2, err);         // eta = N' alpha^0, W
  }

  float *yhat() override { return args_.yhat; }

  int stream_start(const double *x0_dev, const int32_t *slots, const int32_t *xsrc, int S, const float *ypred,
                   int cg_iters, bool first, int max_iter, double eps, std::string &err) override {
    const int Bm = args_.Bmax;
    if (S < 1 || S > Bm) {
      err = "stream_start: slot count out of range";
      return DLMPC_EINVAL;
    }
    // staging in the engine (the copies are ordered on the stream; the host rewrites these
    // vectors only after the stream has drained)
    st_slots_.assign(slots, slots + S);
    st_xsrc_.assign(xsrc, xsrc + S);
    st_mask_.assign(Bm, 0);
    for (int i = 0; i < S; ++i) {
      if (slots[i] < 0 || slots[i] >= Bm || st_mask_[slots[i]]) {
        err = "stream_start: bad or repeated slot";
        return DLMPC_EINVAL;
      }
      if (first && slots[i] != i) {
        err = "stream_start: the initial fill takes slots 0..S-1";
        return DLMPC_EINVAL;
      }
      st_mask_[slots[i]] = 1;
    }
    BENG_CHECK(hipMemcpyAsync(d_slots_, st_slots_.data(), sizeof(int32_t) * S, hipMemcpyHostToDevice, stream_));
    BENG_CHECK(hipMemcpyAsync(d_xsrc_, st_xsrc_.data(), sizeof(int32_t) * S, hipMemcpyHostToDevice, stream_));
    if (first) B_ = S;
    hipLaunchKernelGGL((bprecompute_kernel<NX>), dim3(hs_->N, (S + kPreY - 1) / kPreY), dim3(256), 0, stream_, args_,
                       x0_dev, S, 1,
                       max_iter, eps, d_slots_, d_xsrc_, first ? 1 : 0, 1, cg_iters, nullptr);
    BENG_CHECK(hipGetLastError());
    hipLaunchKernelGGL(bscatter_rows_kernel, dim3(S, 16), dim3(256), 0, stream_, ypred, d_slots_, ny_, args_.yhat);
    BENG_CHECK(hipGetLastError());
    hipLaunchKernelGGL((bsim_kernel<NX>), dim3(S), dim3(1024), 0, stream_, args_, d_slots_);
    BENG_CHECK(hipGetLastError());
    // the CG steps and the start projections run inside the following iterations (phases)
    hipLaunchKernelGGL(bcg_init_kernel, dim3(S, kParts), dim3(1024), 0, stream_, args_, d_slots_, -1);
    BENG_CHECK(hipGetLastError());
    hipLaunchKernelGGL(bpart_sum_kernel, dim3(1), dim3(64), 0, stream_, args_, d_slots_, S, 0);
    BENG_CHECK(hipGetLastError());
    return DLMPC_OK;
  }

  int output_slots(double *u0_dev, const int32_t *slots, const int32_t *dst, int S, std::string &err) override {
    if (S < 1 || S > args_.Bmax) {
      err = "output_slots: slot count out of range";
      return DLMPC_EINVAL;
    }
    for (int i = 0; i < S; ++i)
      if (slots[i] < 0 || slots[i] >= args_.Bmax) {
        err = "output_slots: bad slot";
        return DLMPC_EINVAL;
      }
    st_oslots_.assign(slots, slots + S);
    st_odst_.assign(dst, dst + S);
    BENG_CHECK(hipMemcpyAsync(d_oslots_, st_oslots_.data(), sizeof(int32_t) * S, hipMemcpyHostToDevice, stream_));
    BENG_CHECK(hipMemcpyAsync(d_odst_, st_odst_.data(), sizeof(int32_t) * S, hipMemcpyHostToDevice, stream_));
    hipLaunchKernelGGL((boutput_kernel<NX>), dim3(S, kParts), dim3(256), 0, stream_, args_, u0_dev, d_oslots_,
                       d_odst_);
    BENG_CHECK(hipGetLastError());
    hipLaunchKernelGGL(bpart_sum_kernel, dim3(1), dim3(64), 0, stream_, args_, d_oslots_, S, 1);
    BENG_CHECK(hipGetLastError());
    return DLMPC_OK;
  }

  int export_y(double *y_dev, std::string &err) override {
    hipLaunchKernelGGL(bexport_y_kernel, dim3(1024), dim3(256), 0, stream_, args_, y_dev, B_);
    BENG_CHECK(hipGetLastError());
    return DLMPC_OK;
  }

  int export_alpha(double *alpha_dev, std::string &err) override {
    hipLaunchKernelGGL(bexport_alpha_kernel, dim3(1024), dim3(256), 0, stream_, args_, alpha_dev, B_);
    BENG_CHECK(hipGetLastError());
    return DLMPC_OK;
  }

  int launch_one(int k, std::string &err) override {
    if (k == 0)
      launch_phi(args_);
    else if (k == 1)
      launch_psi(args_);
    else
      hipLaunchKernelGGL(bdecide_kernel, dim3(1), dim3(64), 0, stream_, args_);
    BENG_CHECK(hipGetLastError());
    return DLMPC_OK;
  }

  int iteration(std::string &err, bool joins) override {
    launch_phi(args_);
    BENG_CHECK(hipGetLastError());
    if (joins) {  // CG steps of streamed joins (a no-op for instances in the ADMM iteration)
      launch_cg_step(args_.Bmax, 1);
      BENG_CHECK(hipGetLastError());
    }
    launch_psi(args_);
    BENG_CHECK(hipGetLastError());
    hipLaunchKernelGGL(bdecide_kernel, dim3(1), dim3(64), 0, stream_, args_);
    BENG_CHECK(hipGetLastError());
    return DLMPC_OK;
  }

  int output(double *u0_dev, std::string &err) override {
    hipLaunchKernelGGL((boutput_kernel<NX>), dim3(B_, kParts), dim3(256), 0, stream_, args_, u0_dev, nullptr,
                       nullptr);
    BENG_CHECK(hipGetLastError());
    hipLaunchKernelGGL(bpart_sum_kernel, dim3(1), dim3(64), 0, stream_, args_, nullptr, B_, 1);
    BENG_CHECK(hipGetLastError());
    return DLMPC_OK;
  }

  void set_rho(double rho) override { args_.rho = float(rho); }

  int plant_step(double *x_dev, const double *u_dev, double *xs_dev, double *us_dev, int t, int T_sim, int B,
                 double *rho_scale_dev, std::string &err) override {
    hipLaunchKernelGGL((bplant_kernel<NX>), dim3(B), dim3(256), 0, stream_, args_, x_dev, u_dev, xs_dev, us_dev, t,
                       T_sim, rho_scale_dev);
    BENG_CHECK(hipGetLastError());
    return DLMPC_OK;
  }

  int shift_inputs(const double *y_dev, double *ys_dev, int B, std::string &err) override {
    hipLaunchKernelGGL(bshift_kernel, dim3(256), dim3(256), 0, stream_, args_, y_dev, ys_dev, B);
    BENG_CHECK(hipGetLastError());
    return DLMPC_OK;
  }

  int set_variant(int phi_ntw, int psi_capx, std::string &err) override {
    if (phi_ntw != 1 && phi_ntw != 2) {
      err = "Phi-comp instance tiles per wave must be 1 or 2";
      return DLMPC_EINVAL;
    }
    bool known = psi_capx == 0 && struct_ok_;  // 0: the structured Psi-comp
    for (int c : kPsiCaps) known = known || c == psi_capx;
    if (!known) {
      err = psi_capx == 0 ? "the structured Psi-comp is not available for this problem" : "unknown Psi-comp split";
      return DLMPC_EINVAL;
    }
    phi_ntw_ = phi_ntw;
    if (psi_capx != psi_capx_) {
      // the structured variant runs one unit per column subsystem
      const int rc = load_split(psi_split(*hs_, psi_capx == 0 ? (1 << 20) : psi_capx), psi_capx, err);
      bstruct_ = psi_capx == 0;
      return rc;
    }
    return DLMPC_OK;
  }
  void variant(int *phi_ntw, int *psi_capx, int *n_units) const override {
    *phi_ntw = phi_ntw_;
    *psi_capx = psi_capx_;
    *n_units = n_units_;
  }

  int check(const double *x0_dev, std::string &err) override {
    hipLaunchKernelGGL((bcheck_w_kernel<NX>), dim3(hs_->N), dim3(256), 0, stream_, args_, x0_dev, nullptr, nullptr,
                       B_);
    BENG_CHECK(hipGetLastError());
    hipLaunchKernelGGL((bcheck_y_kernel<NX>), dim3(hs_->N), dim3(256), 0, stream_, args_, x0_dev, nullptr, nullptr,
                       B_);
    BENG_CHECK(hipGetLastError());
    hipLaunchKernelGGL((bcheck_red_kernel<NX>), dim3(B_, kParts), dim3(256), 0, stream_, args_, x0_dev, nullptr, nullptr,
                       B_);
    BENG_CHECK(hipGetLastError());
    hipLaunchKernelGGL(bcheck_fin_kernel, dim3(1), dim3(64), 0, stream_, args_, nullptr, B_);
    BENG_CHECK(hipGetLastError());
    return DLMPC_OK;
  }

  int stash_slots(const int32_t *slots, const int32_t *to, int S, std::string &err) override {
    const int Bm = args_.Bmax;
    if (S < 1 || S > Bm) {
      err = "stash_slots: slot count out of range";
      return DLMPC_EINVAL;
    }
    for (int i = 0; i < S; ++i)
      if (slots[i] < 0 || slots[i] >= Bm || to[i] < 0 || to[i] >= Bm) {
        err = "stash_slots: bad slot";
        return DLMPC_EINVAL;
      }
    st_sfrom_.assign(slots, slots + S);
    st_sto_.assign(to, to + S);
    BENG_CHECK(hipMemcpyAsync(d_sfrom_, st_sfrom_.data(), sizeof(int32_t) * S, hipMemcpyHostToDevice, stream_));
    BENG_CHECK(hipMemcpyAsync(d_sto_, st_sto_.data(), sizeof(int32_t) * S, hipMemcpyHostToDevice, stream_));
    const int64_t items = (int64_t(hs_->N) * hs_->rs + args_.ktot) * S;
    hipLaunchKernelGGL(bstash_kernel, dim3(unsigned((items + 255) / 256)), dim3(256), 0, stream_, args_,
                       stash_args(), d_sfrom_, d_sto_, S);
    BENG_CHECK(hipGetLastError());
    return DLMPC_OK;
  }

  int check_stash(const double *x0_dev, const int32_t *dst, int S, std::string &err) override {
    if (S < 1 || S > args_.Bmax) {
      err = "check_stash: slot count out of range";
      return DLMPC_EINVAL;
    }
    st_cslots_.resize(S);
    for (int i = 0; i < S; ++i) st_cslots_[i] = i;
    st_cdst_.assign(dst, dst + S);
    BENG_CHECK(hipMemcpyAsync(d_cslots_, st_cslots_.data(), sizeof(int32_t) * S, hipMemcpyHostToDevice, stream_));
    BENG_CHECK(hipMemcpyAsync(d_cdst_, st_cdst_.data(), sizeof(int32_t) * S, hipMemcpyHostToDevice, stream_));
    const BArgs sa = stash_args();
    hipLaunchKernelGGL((bcheck_w_kernel<NX>), dim3(hs_->N), dim3(256), 0, stream_, sa, x0_dev, d_cslots_, d_cdst_, S);
    BENG_CHECK(hipGetLastError());
    hipLaunchKernelGGL((bcheck_y_kernel<NX>), dim3(hs_->N), dim3(256), 0, stream_, sa, x0_dev, d_cslots_, d_cdst_, S);
    BENG_CHECK(hipGetLastError());
    hipLaunchKernelGGL((bcheck_red_kernel<NX>), dim3(S, kParts), dim3(256), 0, stream_, sa, x0_dev, d_cslots_, d_cdst_,
                       S);
    BENG_CHECK(hipGetLastError());
    hipLaunchKernelGGL(bcheck_fin_kernel, dim3(1), dim3(64), 0, stream_, sa, d_cslots_, S);
    BENG_CHECK(hipGetLastError());
    return DLMPC_OK;
  }

  BCtl *stash_ictl() override { return sk_ictl_; }

  Ctl *ctl() override { return args_.ctl; }
  BCtl *ictl() override { return args_.ictl; }
  int bmax() const override { return args_.Bmax; }

  ~BatchEngineT() override {
    for (void *p : owned_) (void)hipFree(p);
  }

 private:
  template <typename U>
  int al(U **dst, size_t n, std::string &err) {
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
  int up(const std::vector<U> &src, V **dst, std::string &err) {
    static_assert(sizeof(U) == sizeof(V), "upload type");
    U *p = nullptr;
    int rc = al(&p, src.size(), err);
    if (rc) return rc;
    if (!src.empty()) BENG_CHECK(hipMemcpy(p, src.data(), src.size() * sizeof(U), hipMemcpyHostToDevice));
    *dst = reinterpret_cast<V *>(p);
    return DLMPC_OK;
  }

  // Psi-comp work units of one split into the engine's (preallocated) device arrays.
  int load_split(const PsiSplit &sp, int capx, std::string &err) {
    const size_t nu = sp.pu_j.size(), N = size_t(hs_->N);
    BENG_CHECK(hipStreamSynchronize(stream_));
    BENG_CHECK(hipMemcpy(const_cast<int32_t *>(args_.pu_j), sp.pu_j.data(), nu * 4, hipMemcpyHostToDevice));
    BENG_CHECK(hipMemcpy(const_cast<int32_t *>(args_.pu_r0), sp.pu_r0.data(), nu * 4, hipMemcpyHostToDevice));
    BENG_CHECK(hipMemcpy(const_cast<int32_t *>(args_.pu_r1), sp.pu_r1.data(), nu * 4, hipMemcpyHostToDevice));
    BENG_CHECK(hipMemcpy(const_cast<int32_t *>(args_.pu_p), sp.pu_p.data(), nu * 4, hipMemcpyHostToDevice));
    BENG_CHECK(hipMemcpy(const_cast<int32_t *>(args_.pj_n), sp.pj_n.data(), N * 4, hipMemcpyHostToDevice));
    BENG_CHECK(hipMemcpy(const_cast<int32_t *>(args_.pj_first), sp.pj_first.data(), N * 4, hipMemcpyHostToDevice));
    BENG_CHECK(hipMemcpy(const_cast<int64_t *>(args_.pj_off), sp.pj_off.data(), N * 8, hipMemcpyHostToDevice));
    BENG_CHECK(hipMemset(args_.pcnt, 0, sizeof(int32_t) * N));
    n_units_ = int(nu);
    psi_capx_ = capx;
    return DLMPC_OK;
  }

  const HostSetup *hs_ = nullptr;
  hipStream_t stream_ = nullptr;
  BArgs args_{};
  // instantiations for the row tiles of a subsystem and the basis tiles per wave
  void launch_phi(const BArgs &x) {
    if (split_)
      launch_phi_t<true>(x);
    else
      launch_phi_t<false>(x);
  }
  void launch_psi(const BArgs &x) {
    if (split_)
      launch_psi_t<true>(x);
    else
      launch_psi_t<false>(x);
  }
  template <bool SPLIT>
  void launch_phi_t(const BArgs &x) {
    if (phi_ntw_ == 2)
      launch_phi_n<SPLIT, 2>(x);
    else
      launch_phi_n<SPLIT, 1>(x);
  }
  template <bool SPLIT, int NTW>
  void launch_phi_n(const BArgs &x) {
    switch (nrt_) {
      case 1: hipLaunchKernelGGL((bphi_kernel<NX, 1, SPLIT, NTW>), dim3(hs_->N), dim3(kPhiThreads), 0, stream_, x); break;
      case 2: hipLaunchKernelGGL((bphi_kernel<NX, 2, SPLIT, NTW>), dim3(hs_->N), dim3(kPhiThreads), 0, stream_, x); break;
      case 3: hipLaunchKernelGGL((bphi_kernel<NX, 3, SPLIT, NTW>), dim3(hs_->N), dim3(kPhiThreads), 0, stream_, x); break;
      default: hipLaunchKernelGGL((bphi_kernel<NX, 4, SPLIT, NTW>), dim3(hs_->N), dim3(kPhiThreads), 0, stream_, x); break;
    }
  }
  template <bool SPLIT>
  void launch_psi_t(const BArgs &x) {
    if constexpr (SPLIT) {
      if (bstruct_) {
        switch (mtw_) {
          case 1: hipLaunchKernelGGL((bpsi_kernel<NX, 1, true, true>), dim3(n_units_), dim3(kPsiThreads), 0, stream_, x); break;
          case 2: hipLaunchKernelGGL((bpsi_kernel<NX, 2, true, true>), dim3(n_units_), dim3(kPsiThreads), 0, stream_, x); break;
          case 3: hipLaunchKernelGGL((bpsi_kernel<NX, 3, true, true>), dim3(n_units_), dim3(kPsiThreads), 0, stream_, x); break;
          default: hipLaunchKernelGGL((bpsi_kernel<NX, 4, true, true>), dim3(n_units_), dim3(kPsiThreads), 0, stream_, x); break;
        }
        return;
      }
    }
    switch (mtw_) {
      case 1: hipLaunchKernelGGL((bpsi_kernel<NX, 1, SPLIT>), dim3(n_units_), dim3(kPsiThreads), 0, stream_, x); break;
      case 2: hipLaunchKernelGGL((bpsi_kernel<NX, 2, SPLIT>), dim3(n_units_), dim3(kPsiThreads), 0, stream_, x); break;
      case 3: hipLaunchKernelGGL((bpsi_kernel<NX, 3, SPLIT>), dim3(n_units_), dim3(kPsiThreads), 0, stream_, x); break;
      default: hipLaunchKernelGGL((bpsi_kernel<NX, 4, SPLIT>), dim3(n_units_), dim3(kPsiThreads), 0, stream_, x); break;
    }
  }
  int nrt_ = 1, mtw_ = 1;
  int phi_ntw_ = 1;  // instance tiles per Phi-comp wave (autotuned)
  int psi_capx_ = kPsiCapDefault;  // Psi-comp split (autotuned)
  bool split_ = true;  // basis operands as bf16 hi + lo
  bool struct_ok_ = false, bstruct_ = false;  // structured Psi-comp available / running
  int B_ = 0;
  int64_t ny_ = 0;  // N * rs
  // streamed solves: slot lists on the device and their host staging
  int32_t *d_slots_ = nullptr, *d_xsrc_ = nullptr, *d_oslots_ = nullptr, *d_odst_ = nullptr;
  int32_t *d_cslots_ = nullptr, *d_cdst_ = nullptr, *d_sfrom_ = nullptr, *d_sto_ = nullptr;
  std::vector<int32_t> st_slots_, st_xsrc_, st_mask_, st_oslots_, st_odst_, st_cslots_, st_cdst_, st_sfrom_, st_sto_;
  // stash of stopped streamed instances awaiting their FP64 check (same layouts as the slots)
  float *sk_alpha_ = nullptr, *sk_s_ = nullptr, *sk_tau_ = nullptr, *sk_eta_ = nullptr;
  BCtl *sk_ictl_ = nullptr;
  void launch_cg_step(int nb, int gate) {
    hipLaunchKernelGGL(bcg_pq_kernel, dim3(nb, kCgParts), dim3(256), 0, stream_, args_, gate);
    hipLaunchKernelGGL(bcg_upd_kernel, dim3(nb, kCgParts), dim3(256), 0, stream_, args_, gate);
    hipLaunchKernelGGL(bcg_dir_kernel, dim3(nb, kCgParts), dim3(256), 0, stream_, args_, gate);
  }
  // the arguments of the check kernels, reading the stash in place of the slots
  BArgs stash_args() const {
    BArgs sa = args_;
    sa.alpha = sk_alpha_;
    sa.s = sk_s_;
    sa.tau = sk_tau_;
    sa.eta = sk_eta_;
    sa.ictl = sk_ictl_;
    return sa;
  }
  int n_units_ = 0;  // Psi-comp work units
  std::vector<void *> owned_;
};

// flag[0] = 1 if some entry of x[0..n) is NaN or +-Inf (flag cleared by the caller).
__global__ __launch_bounds__(256) void finite_kernel(const double *__restrict__ x, int64_t n, int32_t *flag) {
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256)
    if (!isfinite(x[i])) flag[0] = 1;
}

}  // namespace

// Prediction staging of the allocation-free stream entry (dlmpc_solve_stream_noalloc): a
// file-scope device array, one copy per device, held until the process ends. Host code never
// passes `scratch` itself to a kernel (in host code the name is a stand-in, not a device
// address): it takes the device address of each device's copy once, with that device current.
constexpr size_t kStreamScratchFloats = size_t(4) << 20;  // 16 MiB
static __device__ __align__(256) float scratch[kStreamScratchFloats];

int stream_scratch(float **ptr, size_t *cap_floats, std::string &err) {
  static std::mutex mu;
  static std::vector<float *> addr;  // per device ordinal (nullptr until taken)
  int dev = -1;
  BENG_CHECK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(mu);
  if (dev >= int(addr.size())) addr.resize(size_t(dev) + 1, nullptr);
  if (!addr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
      return DLMPC_EDEVICE;
    }
    addr[dev] = static_cast<float *>(p);
  }
  *ptr = addr[dev];
  *cap_floats = kStreamScratchFloats;
  return DLMPC_OK;
}

int device_all_finite(const double *x_dev, int64_t n, int32_t *flag_dev, int32_t *flag_host, hipStream_t s,
                      bool *ok, std::string &err) {
  BENG_CHECK(hipMemsetAsync(flag_dev, 0, sizeof(int32_t), s));
  const int grid = int(std::min<int64_t>(1024, (n + 255) / 256));
  if (n > 0) {
    hipLaunchKernelGGL(finite_kernel, dim3(std::max(grid, 1)), dim3(256), 0, s, x_dev, n, flag_dev);
    BENG_CHECK(hipGetLastError());
  }
  BENG_CHECK(hipMemcpyAsync(flag_host, flag_dev, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  BENG_CHECK(hipStreamSynchronize(s));
  *ok = flag_host[0] == 0;
  return DLMPC_OK;
}

std::unique_ptr<BatchEngine> make_batch_engine(int nx) {
  switch (nx) {
    case 1: return std::make_unique<BatchEngineT<1>>();
    case 2: return std::make_unique<BatchEngineT<2>>();
    case 3: return std::make_unique<BatchEngineT<3>>();
    case 4: return std::make_unique<BatchEngineT<4>>();
    default: return nullptr;
  }
}

}  // namespace dlmpc
