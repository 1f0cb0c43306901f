// FP64 factorisation of the column blocks on the device (Algorithm 1, offline step).
//
// Same mathematics as the host factorisation (the Psi-comp step of Algorithm 2 projects each
// column c of subsystem j onto {psi on the d-hop rows of j : Z_AB psi = e_c}). Within the
// patch P(j) a supported psi is a trajectory of the patch whose states never reach the
// (d+1)-hop ring, so it is fixed by the patch inputs U = (u_P[0..T-2]) subject to
// M U = (ring values), M the map from inputs to the ring values G x_P[t], t = 0..T-2, of the
// zero-initial-state response. Per subsystem, one workgroup:
//   phase 1: M' assembled from the sparse patch dynamics (blocks G A_PP^k B_P, Toeplitz in
//            time), then a Householder QR of M' with column pivoting, stopped at numerical rank
//            r (relative threshold kRankTol) -> k = dim null(M) = mu - r;
//   phase 2: K = Q [0; I_k] (orthonormal basis of null(M)); the minimum-norm inputs u_c solving
//            M u = -(free response of x_0 = e_c on the ring) by forward substitution with R'
//            and Q; trajectories S K and psi_c = S(e_c, u_c) by simulating the patch; N_j by
//            Cholesky QR applied twice to S K (its input rows are K itself, so its smallest
//            singular value is at least 1; GEMM-shaped, in 64-column panels), or by a second
//            pivoted Householder QR (rank k required) when a Cholesky pivot falls below a
//            set fraction of the largest diagonal; o_c = psi_c - N N' psi_c.
// The host only builds index lists (patches, ring rows, sparse A entries); every floating-point
// step runs here. Layout: every per-subsystem matrix is row-major in a global workspace, one
// thread per column, so a wave's loads of one row are contiguous (64 consecutive doubles).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <numeric>
#include <string>
#include <vector>

#include "dlmpc_internal.h"

namespace dlmpc {
namespace {

constexpr int kFT = 512;           // threads per workgroup
constexpr int kFW = kFT / 64;      // waves per workgroup (row groups of the column passes)
constexpr int kCC = 1;             // 64-column chunks per pass of reflect_cols
constexpr int kRU = 4;             // rows per lane and load round of reflect_cols
constexpr int kTS = 32 * 65;       // one staged GEMM operand: 32 inner x 64, rows padded to 65
constexpr int kLdsMin = 2 * kTS;   // doubles of dynamic LDS the GEMM and 64 x 64 Cholesky need
constexpr int kFallbackOk = 1;     // phase 2 status: done, with the Householder basis
constexpr int kMaxLdsRows = 4000;  // longest Householder vector staged in LDS (32 KB)

struct FacDesc {
  int64_t app_rp0, app_e0, g_rp0, g_e0;  // index lists
  int64_t f_off;    // M' (mu x mc) and its QR
  int64_t wa_off;   // phase 1 vectors: W ping-pong (2 ns x ni), tau (min(mu, mc)), norms (mc)
  int64_t ia_off;   // phase 1 pivots (mc)
  int64_t wb_off;   // phase 2: X (mu x ncol), S (D x ncol), Nw (D x k), tau2, nrm2 (k),
                    // ring values (mc x nx), rhs (r x nx), t (k x nx)
  int64_t ib_off;   // phase 2 pivots (k)
  int64_t nb_off, off_off;  // outputs (column-major, leading dimension ld)
  int32_t p, ng, aj, tile0;
  int32_t ld, pad;
};

struct FacArgs {
  const double *a_blocks, *b_blocks;
  const int32_t *rp, *ecol, *eidx;
  const int32_t *members;  // patch members of every j (tile order)
  const FacDesc *desc;
  const int32_t *order;    // workgroup -> subsystem
  double *ws;      // phase 1 workspace (M' factors, vectors)
  int32_t *iws;    // phase 1 pivots
  double *wsb;     // phase 2 workspace
  int32_t *iwsb;   // phase 2 pivots
  double *nb, *off;
  int32_t *rank;    // [N] phase 1 result
  int32_t *status;  // [N] phase 2 result (DLMPC_OK, kFallbackOk, or an error)
  double *resid;    // [N] ring residual of the particular solutions over their size
  int32_t nx, nu, T, rs;
  double chol_tol;  // smallest Cholesky QR pivot relative to the largest diagonal of Y'Y
};

// Largest value over the workgroup, ties to the smallest index; uniform result.
__device__ void block_argmax(double &v, int &ix, double *s_rv, int *s_ri) {
  for (int o = 32; o > 0; o >>= 1) {
    const double ov = __shfl_xor(v, o);
    const int oi = __shfl_xor(ix, o);
    if (ov > v || (ov == v && oi < ix)) {
      v = ov;
      ix = oi;
    }
  }
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    s_rv[threadIdx.x >> 6] = v;
    s_ri[threadIdx.x >> 6] = ix;
  }
  __syncthreads();
  v = s_rv[0];
  ix = s_ri[0];
  for (int w = 1; w < kFW; ++w)
    if (s_rv[w] > v || (s_rv[w] == v && s_ri[w] < ix)) {
      v = s_rv[w];
      ix = s_ri[w];
    }
}

// max(a, b) that returns NaN when either is NaN.
__device__ inline double max_nan(double a, double b) { return (b > a || b != b) ? b : a; }

__device__ double block_max(double v, double *s_rv) {
  for (int o = 32; o > 0; o >>= 1) v = max_nan(v, __shfl_xor(v, o));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) s_rv[threadIdx.x >> 6] = v;
  __syncthreads();
  double m = s_rv[0];
  for (int w = 1; w < kFW; ++w) m = max_nan(m, s_rv[w]);
  return m;
}

// Applies H = I - tau v v' (v_k = 1, v_i = s_v[i] for k < i < m) to columns [j0, j1) of C
// (row-major, leading dimension ld, rows k..m-1). The columns go 64 to a wave (one per lane,
// up to kCC chunks per pass) and the rows are split over the kFW waves; each lane keeps kRU
// rows x kCC chunks of independent loads in flight. The partial products v'C meet in LDS
// (s_part, kFW x kCC*64). With nrm2 non-null, nrm2[j] receives the squared norm of rows
// k+1..m-1 of each updated column. Ends with a barrier.
__device__ void reflect_cols(double *C, int ld, int m, int k, const double *s_v, double tau, int j0, int j1,
                             double *nrm2, double *s_part) {
  const int lane = threadIdx.x & 63, rg = threadIdx.x >> 6;
  for (int jb = j0; jb < j1; jb += kCC * 64) {
    const int ncc = min(kCC, (j1 - jb + 63) / 64);
    int col[kCC];
    bool ok[kCC];
#pragma unroll
    for (int cc = 0; cc < kCC; ++cc) {
      const int j = jb + cc * 64 + lane;
      ok[cc] = cc < ncc && j < j1;
      col[cc] = ok[cc] ? j : j0;  // idle lanes read a valid column and store nothing
    }
    double part[kCC];
#pragma unroll
    for (int cc = 0; cc < kCC; ++cc) part[cc] = 0.0;
    int i = k + rg;
    for (; i + (kRU - 1) * kFW < m; i += kRU * kFW) {
      double v[kRU], x[kRU][kCC];
#pragma unroll
      for (int u = 0; u < kRU; ++u) {
        const int iu = i + u * kFW;
        v[u] = (iu == k) ? 1.0 : s_v[iu];
        const double *r = C + int64_t(iu) * ld;
#pragma unroll
        for (int cc = 0; cc < kCC; ++cc)
          if (cc < ncc) x[u][cc] = r[col[cc]];
      }
#pragma unroll
      for (int u = 0; u < kRU; ++u)
#pragma unroll
        for (int cc = 0; cc < kCC; ++cc)
          if (cc < ncc) part[cc] += v[u] * x[u][cc];
    }
    for (; i < m; i += kFW) {
      const double v0 = (i == k) ? 1.0 : s_v[i];
      const double *r0 = C + int64_t(i) * ld;
#pragma unroll
      for (int cc = 0; cc < kCC; ++cc)
        if (cc < ncc) part[cc] += v0 * r0[col[cc]];
    }
#pragma unroll
    for (int cc = 0; cc < kCC; ++cc)
      if (cc < ncc) s_part[rg * (kCC * 64) + cc * 64 + lane] = part[cc];
    __syncthreads();
    double w[kCC];
#pragma unroll
    for (int cc = 0; cc < kCC; ++cc)
      if (cc < ncc) {
        double t = 0.0;
        for (int g = 0; g < kFW; ++g) t += s_part[g * (kCC * 64) + cc * 64 + lane];
        w[cc] = t * tau;
      }
    __syncthreads();
    double q[kCC];
#pragma unroll
    for (int cc = 0; cc < kCC; ++cc) q[cc] = 0.0;
    for (i = k + rg; i + (kRU - 1) * kFW < m; i += kRU * kFW) {
      double v[kRU], x[kRU][kCC];
#pragma unroll
      for (int u = 0; u < kRU; ++u) {
        const int iu = i + u * kFW;
        v[u] = (iu == k) ? 1.0 : s_v[iu];
        const double *r = C + int64_t(iu) * ld;
#pragma unroll
        for (int cc = 0; cc < kCC; ++cc)
          if (cc < ncc) x[u][cc] = r[col[cc]];
      }
#pragma unroll
      for (int u = 0; u < kRU; ++u) {
        const int iu = i + u * kFW;
        const double n0 = (iu == k) ? 0.0 : 1.0;
        double *r = C + int64_t(iu) * ld;
#pragma unroll
        for (int cc = 0; cc < kCC; ++cc)
          if (cc < ncc) {
            const double y = x[u][cc] - w[cc] * v[u];
            q[cc] += n0 * y * y;
            if (ok[cc]) r[col[cc]] = y;
          }
      }
    }
    for (; i < m; i += kFW) {
      const double v0 = (i == k) ? 1.0 : s_v[i];
      const double n0 = (i == k) ? 0.0 : 1.0;
      double *r0 = C + int64_t(i) * ld;
#pragma unroll
      for (int cc = 0; cc < kCC; ++cc)
        if (cc < ncc) {
          const double y = r0[col[cc]] - w[cc] * v0;
          q[cc] += n0 * y * y;
          if (ok[cc]) r0[col[cc]] = y;
        }
    }
    if (nrm2) {
#pragma unroll
      for (int cc = 0; cc < kCC; ++cc)
        if (cc < ncc) s_part[rg * (kCC * 64) + cc * 64 + lane] = q[cc];
      __syncthreads();
      if (rg == 0)
#pragma unroll
        for (int cc = 0; cc < kCC; ++cc)
          if (ok[cc]) {
            double t = 0.0;
            for (int g = 0; g < kFW; ++g) t += s_part[g * (kCC * 64) + cc * 64 + lane];
            nrm2[col[cc]] = t;
          }
    }
    __syncthreads();
  }
}

// Householder QR with column pivoting of the first n columns of F (m rows, row-major, leading
// dimension ld), stopped at the first step whose largest remaining column norm is not above
// rtol times the first pivot's. F receives R in its upper rows and the reflector vectors
// (implicit unit leading entry) below the diagonal; column k of the result is input column
// jpvt[k]. Norms of the trailing columns are recomputed in the pass that updates them.
__device__ int qr_pivoted_dev(double *F, int m, int n, int ld, double rtol, double *tau, int *jpvt,
                              double *nrm2, double *s_v, double *s_part, double *s_rv, int *s_ri) {
  const int tid = threadIdx.x;
  // Initial squared column norms: rows split over the waves, partial sums through LDS.
  {
    const int lane = tid & 63, rg = tid >> 6;
    for (int jb = 0; jb < n; jb += 64) {
      const int j = jb + lane;
      double s0 = 0.0, s1 = 0.0;
      if (j < n) {
        int i = rg;
        for (; i + kFW < m; i += 2 * kFW) {
          const double x0 = F[int64_t(i) * ld + j], x1 = F[int64_t(i + kFW) * ld + j];
          s0 += x0 * x0;
          s1 += x1 * x1;
        }
        if (i < m) {
          const double x0 = F[int64_t(i) * ld + j];
          s0 += x0 * x0;
        }
      }
      s_part[rg * 64 + lane] = s0 + s1;
      __syncthreads();
      if (rg == 0 && j < n) {
        double t = 0.0;
        for (int g = 0; g < kFW; ++g) t += s_part[g * 64 + lane];
        nrm2[j] = t;
        jpvt[j] = j;
      }
      __syncthreads();
    }
  }
  const int kmax = min(m, n);
  double first = 0.0;
  int rank = 0;
  for (int k = 0; k < kmax; ++k) {
    double best = -1.0;
    int piv = INT_MAX;
    for (int j = k + tid; j < n; j += kFT) {
      const double s = nrm2[j];
      if (s > best) {
        best = s;
        piv = j;
      }
    }
    block_argmax(best, piv, s_rv, s_ri);
    const double nrm = sqrt(best);
    if (k == 0) first = nrm;
    if (!(nrm > rtol * first) || nrm == 0.0) break;
    if (piv != k) {
      for (int i = tid; i < m; i += kFT) {
        double *row = F + int64_t(i) * ld;
        const double t = row[k];
        row[k] = row[piv];
        row[piv] = t;
      }
      if (tid == 0) {
        const double t = nrm2[k];
        nrm2[k] = nrm2[piv];
        nrm2[piv] = t;
        const int q = jpvt[k];
        jpvt[k] = jpvt[piv];
        jpvt[piv] = q;
      }
      __syncthreads();
    }
    for (int i = k + tid; i < m; i += kFT) s_v[i] = F[int64_t(i) * ld + k];
    __syncthreads();
    const double alpha = s_v[k];
    const double beta = -copysign(nrm, alpha);
    const double scale = 1.0 / (alpha - beta);
    const double tk = (beta - alpha) / beta;
    for (int i = k + 1 + tid; i < m; i += kFT) {
      const double v = s_v[i] * scale;
      s_v[i] = v;
      F[int64_t(i) * ld + k] = v;
    }
    if (tid == 0) {
      F[int64_t(k) * ld + k] = beta;
      tau[k] = tk;
    }
    __syncthreads();
    if (k + 1 < n) reflect_cols(F, ld, m, k, s_v, tk, k + 1, n, nrm2, s_part);
    rank = k + 1;
  }
  return rank;
}

// X <- H_0 H_1 ... H_{rank-1} X for the reflectors of qr_pivoted_dev held in F (m rows,
// leading dimension ldf); X is m x nc row-major with leading dimension ldx. With `unit`, X
// starts as the first nc columns of the identity: column c is then left alone by H_k, k > c
// (v_k vanishes above row k), so H_k only touches columns k..nc-1.
__device__ void apply_q_dev(const double *F, int m, int ldf, const double *tau, int rank, double *X,
                            int nc, int ldx, bool unit, double *s_v, double *s_part) {
  const int tid = threadIdx.x;
  for (int k = rank - 1; k >= 0; --k) {
    const int c0 = unit ? k : 0;
    if (c0 >= nc) continue;
    for (int i = k + 1 + tid; i < m; i += kFT) s_v[i] = F[int64_t(i) * ldf + k];
    __syncthreads();
    reflect_cols(X, ldx, m, k, s_v, tau[k], c0, nc, nullptr, s_part);
  }
}

// C (M x Nn, row-major ldc) = beta C + alpha A B' with A(i, l) and B(j, l), l < L, read as
// A[l*lda + i] and B[l*ldb + j] (TN) or A[i*lda + l] and B[j*ldb + l] (NT). 64 x 64 output
// tiles, 4 x 2 outputs per thread; 32 values of l of both operands staged in LDS (s_t, 2 kTS
// doubles) per round. lower: tiles above the diagonal are skipped and only j <= i is written.
// beta = 0 does not read C. A tile's operands are read completely before it is written, so C
// may alias A or B when Nn <= 64 (one column tile). Ends with a barrier.
template <bool TN>
__device__ void gemm_dev(int M, int Nn, int L, double alpha, const double *A, int lda, const double *B, int ldb,
                         double beta, double *C, int ldc, bool lower, double *s_t) {
  const int tid = threadIdx.x, ta = tid >> 5, tb = tid & 31;
  for (int i0 = 0; i0 < M; i0 += 64)
    for (int j0 = 0; j0 < Nn; j0 += 64) {
      if (lower && j0 > i0 + 63) continue;
      double acc[4][2];
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q][0] = acc[q][1] = 0.0;
      for (int l0 = 0; l0 < L; l0 += 32) {
#pragma unroll
        for (int u = 0; u < 2048 / kFT; ++u) {  // 64 x 32 values of each operand
          const int e = tid + kFT * u;
          const int ii = TN ? (e & 63) : (e >> 5), ll = TN ? (e >> 6) : (e & 31);
          const int i = i0 + ii, j = j0 + ii, l = l0 + ll;
          const bool lin = l < L;
          s_t[ll * 65 + ii] = (lin && i < M) ? (TN ? A[int64_t(l) * lda + i] : A[int64_t(i) * lda + l]) : 0.0;
          s_t[kTS + ll * 65 + ii] = (lin && j < Nn) ? (TN ? B[int64_t(l) * ldb + j] : B[int64_t(j) * ldb + l]) : 0.0;
        }
        __syncthreads();
#pragma unroll 4
        for (int ll = 0; ll < 32; ++ll) {
          const double *ra = s_t + ll * 65 + 4 * ta, *rb = s_t + kTS + ll * 65 + 2 * tb;
          const double a0 = ra[0], a1 = ra[1], a2 = ra[2], a3 = ra[3], b0 = rb[0], b1 = rb[1];
          acc[0][0] += a0 * b0;
          acc[0][1] += a0 * b1;
          acc[1][0] += a1 * b0;
          acc[1][1] += a1 * b1;
          acc[2][0] += a2 * b0;
          acc[2][1] += a2 * b1;
          acc[3][0] += a3 * b0;
          acc[3][1] += a3 * b1;
        }
        __syncthreads();
      }
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int w = 0; w < 2; ++w) {
          const int i = i0 + 4 * ta + q, j = j0 + 2 * tb + w;
          if (i < M && j < Nn && (!lower || j <= i)) {
            double *c = C + int64_t(i) * ldc + j;
            *c = (beta == 0.0) ? alpha * acc[q][w] : beta * *c + alpha * acc[q][w];
          }
        }
    }
  __syncthreads();
}

// Cholesky factor of the nb x nb (nb <= 64) diagonal block at (jb, jb) of G (row-major,
// leading dimension ldg; lower triangle used and overwritten with L), and the inverse of that
// factor written to Li (64 x 64 row-major, zero above the diagonal). Both triangles live packed
// in LDS (s_t: L at i(i+1)/2 + l, inverse 2080 further). Returns false, uniformly, when a pivot
// is not above tol.
__device__ bool chol_inv64(double *G, int ldg, int jb, int nb, double *Li, double tol, double *s_t) {
  const int tid = threadIdx.x;
  double *sl = s_t, *si = s_t + 2080;
  for (int e = tid; e < nb * nb; e += kFT) {
    const int i = e / nb, l = e % nb;
    if (l <= i) sl[i * (i + 1) / 2 + l] = G[int64_t(jb + i) * ldg + jb + l];
  }
  __syncthreads();
  for (int j = 0; j < nb; ++j) {
    const double pv = sl[j * (j + 1) / 2 + j];
    if (!(pv > tol) || !(pv < INFINITY)) return false;
    const double dj = sqrt(pv);
    for (int i = j + 1 + tid; i < nb; i += kFT) sl[i * (i + 1) / 2 + j] /= dj;
    __syncthreads();
    if (tid == 0) sl[j * (j + 1) / 2 + j] = dj;
    const int n = nb - j - 1;
    for (int e = tid; e < n * n; e += kFT) {
      const int i = j + 1 + e / n, l = j + 1 + e % n;
      if (l <= i) sl[i * (i + 1) / 2 + l] -= sl[i * (i + 1) / 2 + j] * sl[l * (l + 1) / 2 + j];
    }
    __syncthreads();
  }
  for (int i = 0; i < nb; ++i) {
    for (int c = tid; c <= i; c += kFT) {
      double t = (c == i) ? 1.0 : 0.0;
      for (int l = c; l < i; ++l) t -= sl[i * (i + 1) / 2 + l] * si[l * (l + 1) / 2 + c];
      si[i * (i + 1) / 2 + c] = t / sl[i * (i + 1) / 2 + i];
    }
    __syncthreads();
  }
  for (int e = tid; e < 64 * 64; e += kFT) {
    const int i = e >> 6, l = e & 63;
    Li[e] = (i < nb && l <= i) ? si[i * (i + 1) / 2 + l] : 0.0;
    if (i < nb && l <= i) G[int64_t(jb + i) * ldg + jb + l] = sl[i * (i + 1) / 2 + l];
  }
  __syncthreads();
  return true;
}

// Q (m x k, row-major ldq) = Y L^{-T}, an orthonormal basis of range(Y) for Y (m x k, row-major
// ldy) with Y'Y = L L' (Cholesky QR): Gram by gemm_dev, Cholesky in 64-column panels (panel
// factor and inverse in LDS, L21 = G21 L11^{-T} and G22 -= L21 L21' by gemm_dev), then
// Q_B = (Y_B - Q_<B L_B,<B') L_BB^{-T} panel by panel. G: k x k workspace; Lb: ceil(k/64)
// blocks of 64 x 64. Y and Q must not alias. Returns false, uniformly, when a pivot is not
// above tol times the largest diagonal entry of Y'Y.
__device__ bool cholqr_dev(const double *Y, int ldy, int m, int k, double *Q, int ldq, double *G, double *Lb,
                           double tol, double *s_t, double *s_rv) {
  const int tid = threadIdx.x;
  gemm_dev<true>(k, k, m, 1.0, Y, ldy, Y, ldy, 0.0, G, k, true, s_t);
  double md = 0.0;
  for (int i = tid; i < k; i += kFT) md = max_nan(md, G[int64_t(i) * k + i]);
  md = block_max(md, s_rv);
  if (!(md > 0.0) || !(md < INFINITY)) return false;
  for (int jb = 0; jb < k; jb += 64) {
    const int nb = min(64, k - jb), rest = k - jb - nb;
    double *Li = Lb + int64_t(jb / 64) * 4096;
    if (!chol_inv64(G, k, jb, nb, Li, tol * md, s_t)) return false;
    if (rest > 0) {
      double *G21 = G + int64_t(jb + nb) * k + jb;
      gemm_dev<false>(rest, nb, nb, 1.0, G21, k, Li, 64, 0.0, G21, k, false, s_t);
      gemm_dev<false>(rest, rest, nb, -1.0, G21, k, G21, k, 1.0, G21 + nb, k, true, s_t);
    }
  }
  for (int jb = 0; jb < k; jb += 64) {
    const int nb = min(64, k - jb);
    for (int64_t e = tid; e < int64_t(m) * nb; e += kFT) {
      const int i = int(e / nb), c = int(e % nb);
      Q[int64_t(i) * ldq + jb + c] = Y[int64_t(i) * ldy + jb + c];
    }
    __syncthreads();
    if (jb > 0) gemm_dev<false>(m, nb, jb, -1.0, Q, ldq, G + int64_t(jb) * k, k, 1.0, Q + jb, ldq, false, s_t);
    gemm_dev<false>(m, nb, nb, 1.0, Q + jb, ldq, Lb + int64_t(jb / 64) * 4096, 64, 0.0, Q + jb, ldq, false, s_t);
  }
  return true;
}

struct Patch {
  const double *A, *B;
  const int32_t *arp, *acol, *aidx;  // A_PP (CSR over patch states)
  const int32_t *grp, *gcol, *gidx;  // G (CSR over ring rows)
  const int32_t *mem;
  int p, ns, ni, ng, nx, nu, T, rs;

  // Row of state s of patch member a at time t in the local trajectory order.
  __device__ int srow(int r, int t) const { return (r / nx) * rs + t * nx + r % nx; }

  // Simulates columns [c0, c1) of S (row-major, leading dimension lds): column c starts from
  // e_{x0base + c - off0} when c >= off0 (zero state otherwise) under the inputs in column c of
  // U (row-major, leading dimension lds, rows t*ni + a*nu + q; zero inputs when U is null),
  // and every state and input row of its trajectory is written. For the columns c >= off0 the
  // ring values G x[t], t = 0..T-2, are computed, stored to ring[(t*ng+i)*ring_ld + c - off0]
  // when ring is non-null, and the largest magnitude over them (NaN if any is NaN) is
  // returned to every thread, divided by max(1, largest magnitude of those columns' entries).
  // Lanes take columns, the waves split the rows of each time step.
  __device__ double simulate(double *S, int lds, int c0, int c1, const double *U, int off0, int x0base,
                             double *ring, int ring_ld, double *s_rv) const {
    double sz = 1.0;  // size of the tracked trajectories
    const int lane = threadIdx.x & 63, rg = threadIdx.x >> 6;
    for (int cb = c0; cb < c1; cb += 64) {
      const int c = cb + lane;
      if (c >= c1) continue;
      const int x0row = (c >= off0) ? x0base + c - off0 : -1;
      for (int r = rg; r < ns; r += kFW) S[int64_t(srow(r, 0)) * lds + c] = (r == x0row) ? 1.0 : 0.0;
      for (int e = rg; e < (T - 1) * ni; e += kFW) {
        const int t = e / ni, a = (e % ni) / nu, q = e % nu;
        const double uv = U ? U[int64_t(e) * lds + c] : 0.0;
        S[int64_t(a * rs + nx * T + t * nu + q) * lds + c] = uv;
        if (c >= off0) sz = max_nan(sz, fabs(uv));
      }
    }
    __syncthreads();
    double mx = 0.0;
    for (int t = 0; t < T; ++t) {
      for (int cb = c0; cb < c1; cb += 64) {
        const int c = cb + lane;
        if (c >= c1) continue;
        if (c >= off0 && t <= T - 2)
          for (int i = rg; i < ng; i += kFW) {
            double g = 0.0;
            for (int q = grp[i]; q < grp[i + 1]; ++q) g += A[gidx[q]] * S[int64_t(srow(gcol[q], t)) * lds + c];
            if (ring) ring[int64_t(t * ng + i) * ring_ld + c - off0] = g;
            mx = max_nan(mx, fabs(g));
          }
        if (t == T - 1) continue;
        for (int r = rg; r < ns; r += kFW) {
          double v = 0.0;
          for (int q = arp[r]; q < arp[r + 1]; ++q) v += A[aidx[q]] * S[int64_t(srow(acol[q], t)) * lds + c];
          if (U) {
            const int a = r / nx, s = r % nx;
            for (int q = 0; q < nu; ++q)
              v += B[(int64_t(mem[a]) * nx + s) * nu + q] * U[int64_t(t * ni + a * nu + q) * lds + c];
          }
          S[int64_t(srow(r, t + 1)) * lds + c] = v;
          if (c >= off0) sz = max_nan(sz, fabs(v));
        }
      }
      __syncthreads();
    }
    mx = block_max(mx, s_rv);
    sz = block_max(sz, s_rv);
    return mx / sz;
  }
};

__device__ Patch make_patch(const FacArgs &a, const FacDesc &d) {
  Patch P;
  P.A = a.a_blocks;
  P.B = a.b_blocks;
  P.arp = a.rp + d.app_rp0;
  P.acol = a.ecol + d.app_e0;
  P.aidx = a.eidx + d.app_e0;
  P.grp = a.rp + d.g_rp0;
  P.gcol = a.ecol + d.g_e0;
  P.gidx = a.eidx + d.g_e0;
  P.mem = a.members + d.tile0;
  P.p = d.p;
  P.nx = a.nx;
  P.nu = a.nu;
  P.T = a.T;
  P.rs = a.rs;
  P.ns = d.p * a.nx;
  P.ni = d.p * a.nu;
  P.ng = d.ng;
  return P;
}

// Phase 1: assemble M' and factor it; rank[j] = numerical rank.
__global__ __launch_bounds__(kFT) void fac_ring_qr_kernel(FacArgs a) {
  extern __shared__ double s_v[];
  __shared__ double s_part[kFW * kCC * 64];
  __shared__ double s_rv[kFW];
  __shared__ int s_ri[kFW];
  const int j = a.order[blockIdx.x];
  const FacDesc d = a.desc[j];
  const Patch P = make_patch(a, d);
  const int T = a.T, ns = P.ns, ni = P.ni, ng = P.ng, mu = ni * (T - 1), mc = ng * (T - 1);
  const int tid = threadIdx.x;
  double *F = a.ws + d.f_off;
  double *W = a.ws + d.wa_off, *Wn = W + int64_t(ns) * ni;
  double *tau = Wn + int64_t(ns) * ni, *nrm = tau + min(mu, mc);
  int *jpvt = a.iws + d.ia_off;
  for (int64_t e = tid; e < int64_t(mu) * mc; e += kFT) F[e] = 0.0;
  for (int e = tid; e < ns * ni; e += kFT) {
    const int r = e / ni, c = e % ni, am = r / a.nx, s = r % a.nx;
    W[e] = (am == c / a.nu) ? a.b_blocks[(int64_t(P.mem[am]) * a.nx + s) * a.nu + c % a.nu] : 0.0;
  }
  __syncthreads();
  // Block (t', tau) of M is G A_PP^(t'-1-tau) B_P for tau < t' <= T-2; W = A_PP^kk B_P.
  for (int kk = 0; kk <= T - 3; ++kk) {
    for (int e = tid; e < ng * ni; e += kFT) {
      const int i = e / ni, c = e % ni;
      double g = 0.0;
      for (int q = P.grp[i]; q < P.grp[i + 1]; ++q) g += P.A[P.gidx[q]] * W[int64_t(P.gcol[q]) * ni + c];
      for (int t = 0; t + kk + 1 <= T - 2; ++t) F[int64_t(t * ni + c) * mc + (t + kk + 1) * ng + i] = g;
    }
    for (int e = tid; e < ns * ni; e += kFT) {
      const int r = e / ni, c = e % ni;
      double v = 0.0;
      for (int q = P.arp[r]; q < P.arp[r + 1]; ++q) v += P.A[P.aidx[q]] * W[int64_t(P.acol[q]) * ni + c];
      Wn[e] = v;
    }
    __syncthreads();
    double *t = W;
    W = Wn;
    Wn = t;
  }
  const int r = qr_pivoted_dev(F, mu, mc, mc, kRankTol, tau, jpvt, nrm, s_v, s_part, s_rv, s_ri);
  if (tid == 0) a.rank[j] = r;
}

// Phase 2: null basis N_j and offsets o_c from the factored M'.
__global__ __launch_bounds__(kFT) void fac_basis_kernel(FacArgs a) {
  extern __shared__ double s_v[];
  __shared__ double s_part[kFW * kCC * 64];
  __shared__ double s_rv[kFW];
  __shared__ int s_ri[kFW];
  const int j = a.order[blockIdx.x];
  const FacDesc d = a.desc[j];
  const Patch P = make_patch(a, d);
  const int T = a.T, nx = a.nx, ni = P.ni, ng = P.ng, mu = ni * (T - 1), mc = ng * (T - 1);
  const int D = d.p * a.rs, r = a.rank[j], k = mu - r, ncol = k + nx, ld = d.ld;
  const int tid = threadIdx.x;
  const double *F = a.ws + d.f_off;
  const double *tau = a.ws + d.wa_off + 2 * int64_t(P.ns) * ni;
  const int *jpvt = a.iws + d.ia_off;
  double *X = a.wsb + d.wb_off;
  double *S = X + int64_t(mu) * ncol;
  double *Nw = S + int64_t(D) * ncol;
  double *tau2 = Nw + int64_t(D) * k, *nrm2 = tau2 + k;
  double *ringv = nrm2 + k, *rhs = ringv + int64_t(mc) * nx, *tv = rhs + int64_t(r) * nx;
  double *Q2 = tv + int64_t(k) * nx, *Gk = Q2 + int64_t(D) * k, *Lb = Gk + int64_t(k) * k;
  int *jp2 = a.iwsb + d.ib_off;

  // Ring values of the free responses x_0 = e_c (scratch trajectories in the offset columns).
  P.simulate(S, ncol, k, ncol, nullptr, k, d.aj * nx, ringv, nx, s_rv);
  for (int e = tid; e < r * nx; e += kFT) {
    const int i = e / nx, c = e % nx;
    rhs[e] = -ringv[int64_t(jpvt[i]) * nx + c];
  }
  for (int64_t e = tid; e < int64_t(mu) * ncol; e += kFT) {
    const int i = int(e / ncol), c = int(e % ncol);
    X[e] = (c < k && i == r + c) ? 1.0 : 0.0;
  }
  __syncthreads();
  // R11' w = rhs (column-oriented forward substitution); w lands in X's offset columns.
  for (int i = 0; i < r; ++i) {
    const double rii = F[int64_t(i) * mc + i];
    for (int e = i + 1 + tid; e < r; e += kFT) {
      const double ril = F[int64_t(i) * mc + e];
      for (int c = 0; c < nx; ++c) rhs[int64_t(e) * nx + c] -= ril * (rhs[int64_t(i) * nx + c] / rii);
    }
    if (tid < nx) X[int64_t(i) * ncol + k + tid] = rhs[int64_t(i) * nx + tid] / rii;
    __syncthreads();
  }
  // X = Q [I_k-part | w; 0] = [K | u_c].
  apply_q_dev(F, mu, mc, tau, r, X, ncol, ncol, false, s_v, s_part);
  // Trajectories: S K (zero initial state) and psi_c (initial state e_c, inputs u_c).
  const double res = P.simulate(S, ncol, 0, ncol, X, k, d.aj * nx, nullptr, 0, s_rv);
  if (!(res <= kFeasTol)) {
    if (tid == 0) {
      a.status[j] = DLMPC_EINFEASIBLE_LOCALITY;
      a.resid[j] = res;
    }
    return;
  }
  // N_j: Cholesky QR twice (S K -> Nw -> Q2); Householder QR of S K when a pivot is too small.
  const double *Nb = Q2;
  if (k > 0) {
    bool ok = cholqr_dev(S, ncol, D, k, Nw, k, Gk, Lb, a.chol_tol, s_v, s_rv);
    if (ok) ok = cholqr_dev(Nw, k, D, k, Q2, k, Gk, Lb, a.chol_tol, s_v, s_rv);
    if (!ok) {
      const int r2 = qr_pivoted_dev(S, D, k, ncol, kBasisTol, tau2, jp2, nrm2, s_v, s_part, s_rv, s_ri);
      if (r2 != k) {
        if (tid == 0) a.status[j] = DLMPC_ENUMERIC;
        return;
      }
      for (int64_t e = tid; e < int64_t(D) * k; e += kFT) {
        const int i = int(e / k), c = int(e % k);
        Nw[e] = (i == c) ? 1.0 : 0.0;
      }
      __syncthreads();
      apply_q_dev(S, D, ncol, tau2, k, Nw, k, k, true, s_v, s_part);
      Nb = Nw;
      if (tid == 0) a.status[j] = kFallbackOk;
    }
    // t = N' psi_c
    for (int e = tid; e < k * nx; e += kFT) {
      const int c = e / nx, cc = e % nx;
      double s0 = 0.0, s1 = 0.0;
      int i = 0;
      for (; i + 1 < D; i += 2) {
        s0 += Nb[int64_t(i) * k + c] * S[int64_t(i) * ncol + k + cc];
        s1 += Nb[int64_t(i + 1) * k + c] * S[int64_t(i + 1) * ncol + k + cc];
      }
      if (i < D) s0 += Nb[int64_t(i) * k + c] * S[int64_t(i) * ncol + k + cc];
      tv[e] = s0 + s1;
    }
    __syncthreads();
  }
  // o_c = psi_c - N t_c; N to the output (column-major, leading dimension ld).
  for (int i = tid; i < D; i += kFT)
    for (int cc = 0; cc < nx; ++cc) {
      double s = 0.0;
      for (int c = 0; c < k; ++c) s += Nb[int64_t(i) * k + c] * tv[c * nx + cc];
      a.off[d.off_off + int64_t(cc) * ld + i] = S[int64_t(i) * ncol + k + cc] - s;
    }
  for (int64_t e = tid; e < int64_t(D) * k; e += kFT) {
    const int c = int(e / D), i = int(e % D);
    a.nb[d.nb_off + int64_t(c) * ld + i] = Nb[int64_t(i) * k + c];
  }
  if (tid == 0) {
    if (Nb != Nw) a.status[j] = DLMPC_OK;
    a.resid[j] = res;
  }
}

// Device buffers of one factorisation, released on every exit path.
struct DevBufs {
  std::vector<void *> ptrs;
  ~DevBufs() {
    for (void *p : ptrs) (void)hipFree(p);
  }
  template <class T>
  hipError_t alloc(T **p, size_t n) {
    *p = nullptr;
    if (n == 0) n = 1;
    const hipError_t e = hipMalloc(reinterpret_cast<void **>(p), n * sizeof(T));
    if (e == hipSuccess) ptrs.push_back(*p);
    return e;
  }
};

}  // namespace

int factor_device(HostSetup &hs, int device, double chol_tol, std::string &err) {
  const auto t0 = std::chrono::steady_clock::now();
  const int32_t N = hs.N, nx = hs.nx, nu = hs.nu, T = hs.T;
  if (hs.a_blocks.size() >= size_t(INT_MAX)) {
    err = "A has too many entries for the device factorisation (use DLMPC_FLAG_HOST_FACTOR)";
    return DLMPC_EINVAL;
  }
  FactorLists fl;
  factor_lists(hs, fl);

  std::vector<FacDesc> desc(N);
  std::vector<double> cost(N);
  int64_t f_tot = 0, wa_tot = 0, ia_tot = 0;
  int vmax = 1;
  for (int j = 0; j < N; ++j) {
    FacDesc &d = desc[j];
    const int p = int(hs.patch[j].size()), ns = p * nx, ni = p * nu, ng = fl.ng[j];
    const int64_t mu = int64_t(ni) * (T - 1), mc = int64_t(ng) * (T - 1), D = int64_t(p) * hs.rs;
    if (mu * std::max<int64_t>(mc, D) >= INT_MAX / 4 || D * (mu + nx) >= INT_MAX / 4) {
      err = "column block of subsystem " + std::to_string(j) + " too large for the device factorisation";
      return DLMPC_EINVAL;
    }
    vmax = std::max<int>(vmax, int(std::max(mu, D)));
    d.app_rp0 = fl.app_rp0[j];
    d.app_e0 = fl.app_e0[j];
    d.g_rp0 = fl.g_rp0[j];
    d.g_e0 = fl.g_e0[j];
    d.p = p;
    d.ng = ng;
    d.aj = fl.aj[j];
    d.tile0 = int32_t(hs.tile_off[j]);
    d.ld = padded_ld(int32_t(D));
    d.f_off = f_tot;
    f_tot += mu * mc;
    d.wa_off = wa_tot;
    wa_tot += 2 * int64_t(ns) * ni + std::min(mu, mc) + mc;
    d.ia_off = ia_tot;
    ia_tot += mc;
    cost[j] = double(mu) * double(mc) * double(std::min(mu, mc)) + double(D) * double(mu) * double(mu);
  }
  if (vmax > kMaxLdsRows) {
    err = "column block longer than " + std::to_string(kMaxLdsRows) +
          " rows: too long for the device factorisation (use DLMPC_FLAG_HOST_FACTOR)";
    return DLMPC_EINVAL;
  }
  std::vector<int32_t> order(N);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });

  auto hip_fail = [&](hipError_t e, const char *what) {
    err = std::string("device factorisation: ") + what + ": " + hipGetErrorString(e);
    return DLMPC_EDEVICE;
  };
#define FAC_HIP(x, what)                            \
  do {                                              \
    const hipError_t e_ = (x);                      \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)
  FAC_HIP(hipSetDevice(device), "hipSetDevice");
  hipStream_t st = nullptr;
  FAC_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking), "stream");
  struct StreamGuard {
    hipStream_t s;
    ~StreamGuard() { (void)hipStreamDestroy(s); }
  } sg{st};
  DevBufs B;
  FacArgs a{};
  double *d_A, *d_B, *ws, *d_nb, *d_off, *d_resid;
  int32_t *d_rp, *d_ecol, *d_eidx, *d_mem, *d_order, *iws, *d_rank, *d_status;
  FacDesc *d_desc;
  FAC_HIP(B.alloc(&d_A, hs.a_blocks.size()), "alloc");
  FAC_HIP(B.alloc(&d_B, hs.b_blocks.size()), "alloc");
  FAC_HIP(B.alloc(&d_rp, fl.rp.size()), "alloc");
  FAC_HIP(B.alloc(&d_ecol, fl.ecol.size()), "alloc");
  FAC_HIP(B.alloc(&d_eidx, fl.eidx.size()), "alloc");
  FAC_HIP(B.alloc(&d_mem, hs.tile_rsub.size()), "alloc");
  FAC_HIP(B.alloc(&d_order, size_t(N)), "alloc");
  FAC_HIP(B.alloc(&d_desc, size_t(N)), "alloc");
  FAC_HIP(B.alloc(&d_rank, size_t(N)), "alloc");
  FAC_HIP(B.alloc(&d_status, size_t(N)), "alloc");
  FAC_HIP(B.alloc(&d_resid, size_t(N)), "alloc");
  const int64_t wa_base = f_tot;
  for (FacDesc &d : desc) d.wa_off += wa_base;
  int64_t ws1 = f_tot + wa_tot;
  FAC_HIP(B.alloc(&ws, size_t(ws1)), "workspace");
  FAC_HIP(B.alloc(&iws, size_t(ia_tot)), "workspace");
  auto up = [&](void *dst, const void *src, size_t bytes) {
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st);
  };
  FAC_HIP(up(d_A, hs.a_blocks.data(), hs.a_blocks.size() * 8), "upload");
  FAC_HIP(up(d_B, hs.b_blocks.data(), hs.b_blocks.size() * 8), "upload");
  FAC_HIP(up(d_rp, fl.rp.data(), fl.rp.size() * 4), "upload");
  if (!fl.ecol.empty()) {
    FAC_HIP(up(d_ecol, fl.ecol.data(), fl.ecol.size() * 4), "upload");
    FAC_HIP(up(d_eidx, fl.eidx.data(), fl.eidx.size() * 4), "upload");
  }
  FAC_HIP(up(d_mem, hs.tile_rsub.data(), hs.tile_rsub.size() * 4), "upload");
  FAC_HIP(up(d_order, order.data(), size_t(N) * 4), "upload");
  FAC_HIP(up(d_desc, desc.data(), size_t(N) * sizeof(FacDesc)), "upload");
  a.a_blocks = d_A;
  a.b_blocks = d_B;
  a.rp = d_rp;
  a.ecol = d_ecol;
  a.eidx = d_eidx;
  a.members = d_mem;
  a.desc = d_desc;
  a.order = d_order;
  a.ws = ws;
  a.iws = iws;
  a.rank = d_rank;
  a.status = d_status;
  a.resid = d_resid;
  a.nx = nx;
  a.nu = nu;
  a.T = T;
  a.rs = hs.rs;
  a.chol_tol = chol_tol;
  const size_t lds = size_t(std::max(vmax, kLdsMin)) * sizeof(double);
  hipLaunchKernelGGL(fac_ring_qr_kernel, dim3(N), dim3(kFT), lds, st, a);
  FAC_HIP(hipGetLastError(), "phase 1 launch");
  std::vector<int32_t> rank(N);
  FAC_HIP(hipMemcpyAsync(rank.data(), d_rank, size_t(N) * 4, hipMemcpyDeviceToHost, st), "download");
  FAC_HIP(hipStreamSynchronize(st), "phase 1");

  // Null-space dimensions, output layout, phase 2 workspace.
  std::vector<int> ks(N);
  for (int j = 0; j < N; ++j) {
    const int64_t mu = int64_t(hs.patch[j].size()) * nu * (T - 1);
    if (rank[j] < 0 || rank[j] > mu) {
      err = "device factorisation: bad rank";
      return DLMPC_EDEVICE;
    }
    ks[j] = int(mu - rank[j]);
  }
  pack_factors(hs, ks, {}, {});
  hs.nb = BigVec();  // the bases stay on the device
  int64_t wb_tot = 0, ib_tot = 0;
  for (int j = 0; j < N; ++j) {
    FacDesc &d = desc[j];
    const int64_t mu = int64_t(hs.patch[j].size()) * nu * (T - 1), mc = int64_t(d.ng) * (T - 1);
    const int64_t D = int64_t(d.p) * hs.rs, k = ks[j], ncol = k + nx, r = rank[j];
    d.wb_off = wb_tot;
    wb_tot += mu * ncol + D * ncol + D * k + 2 * k + mc * nx + r * nx + k * nx + D * k + k * k +
              (k + 63) / 64 * 4096;
    d.ib_off = ib_tot;
    ib_tot += k;
    d.nb_off = hs.nb_off[j];
    d.off_off = hs.off_ptr[j];
  }
  double *ws2;
  int32_t *iws2;
  FAC_HIP(B.alloc(&ws2, size_t(wb_tot)), "workspace");
  FAC_HIP(B.alloc(&iws2, size_t(ib_tot)), "workspace");
  const size_t nb_len = size_t(hs.nb_off[N]);
  FAC_HIP(hipMalloc(reinterpret_cast<void **>(&d_nb), std::max<size_t>(nb_len, 1) * sizeof(double)), "alloc");
  hs.d_nb = d_nb;  // owned by hs from here on (released with the problem, or below on error)
  hs.d_nb_device = device;
  FAC_HIP(B.alloc(&d_off, hs.off.size()), "alloc");
  FAC_HIP(hipMemsetAsync(d_nb, 0, std::max<size_t>(nb_len, 1) * 8, st), "memset");
  FAC_HIP(hipMemsetAsync(d_off, 0, std::max<size_t>(hs.off.size(), 1) * 8, st), "memset");
  FAC_HIP(hipMemsetAsync(d_status, 0xff, size_t(N) * 4, st), "memset");
  FAC_HIP(up(d_desc, desc.data(), size_t(N) * sizeof(FacDesc)), "upload");
  a.wsb = ws2;
  a.iwsb = iws2;
  a.nb = d_nb;
  a.off = d_off;
  hipLaunchKernelGGL(fac_basis_kernel, dim3(N), dim3(kFT), lds, st, a);
  FAC_HIP(hipGetLastError(), "phase 2 launch");
  std::vector<int32_t> status(N);
  std::vector<double> resid(N);
  FAC_HIP(hipMemcpyAsync(status.data(), d_status, size_t(N) * 4, hipMemcpyDeviceToHost, st), "download");
  FAC_HIP(hipMemcpyAsync(resid.data(), d_resid, size_t(N) * 8, hipMemcpyDeviceToHost, st), "download");
  if (!hs.off.empty())
    FAC_HIP(hipMemcpyAsync(hs.off.data(), d_off, hs.off.size() * 8, hipMemcpyDeviceToHost, st), "download");
  FAC_HIP(hipStreamSynchronize(st), "phase 2");
#undef FAC_HIP
  hs.factor_fallbacks = 0;
  for (int j = 0; j < N; ++j) {
    if (status[j] == kFallbackOk) {
      ++hs.factor_fallbacks;
      continue;
    }
    if (status[j] == DLMPC_EINFEASIBLE_LOCALITY) {
      err = "column of subsystem " + std::to_string(j) +
            " has no trajectory inside its d-hop patch (relative ring residual " + std::to_string(resid[j]) + ")";
      return DLMPC_EINFEASIBLE_LOCALITY;
    }
    if (status[j] == DLMPC_ENUMERIC) {
      err = "null basis lost rank at subsystem " + std::to_string(j);
      return DLMPC_ENUMERIC;
    }
    if (status[j] != DLMPC_OK) {
      err = "device factorisation did not finish subsystem " + std::to_string(j);
      return DLMPC_EDEVICE;
    }
  }
  hs.factor_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  hs.factor_where = 1;
  return DLMPC_OK;
}

void free_factors_device(HostSetup &hs) {
  if (!hs.d_nb) return;
  int cur = -1;
  (void)hipGetDevice(&cur);
  if (hs.d_nb_device >= 0) (void)hipSetDevice(hs.d_nb_device);
  (void)hipFree(hs.d_nb);
  if (cur >= 0) (void)hipSetDevice(cur);
  hs.d_nb = nullptr;
  hs.d_nb_device = -1;
}

int fetch_basis(const HostSetup &hs, int32_t j, std::vector<double> &out, std::string &err) {
  const size_t len = size_t(hs.nb_off[j + 1] - hs.nb_off[j]);
  out.resize(len);
  if (len == 0) return DLMPC_OK;
  if (!hs.nb.empty()) {
    std::copy(hs.nb.begin() + hs.nb_off[j], hs.nb.begin() + hs.nb_off[j + 1], out.begin());
    return DLMPC_OK;
  }
  if (!hs.d_nb) {
    err = "no null bases";
    return DLMPC_EINVAL;
  }
  hipError_t e = hipSetDevice(hs.d_nb_device);
  if (e == hipSuccess) e = hipMemcpy(out.data(), hs.d_nb + hs.nb_off[j], len * sizeof(double), hipMemcpyDeviceToHost);
  if (e != hipSuccess) {
    err = std::string("fetching a null basis: ") + hipGetErrorString(e);
    return DLMPC_EDEVICE;
  }
  return DLMPC_OK;
}

}  // namespace dlmpc
