// Learned warm start: one small network per subsystem predicting the optimal input sequence
// u_0..u_{T-2} of that subsystem from the d-hop slice of x0; the prediction feeds the trajectory
// start of the batched engine (the better initial point that Section V lists as future work).
// Training and inference run on the project's own kernels:
//   ws_gemm_kernel   grouped C_g = op(A_g) op(B_g) on the matrix cores (v_mfma_f32_16x16x32_bf16,
//                    operands split into bf16 hi + lo, FP32 accumulation) with fused epilogues
//                    (bias + GELU forward, GELU derivative backward, plain store);
//   ws_bias_grad_kernel, ws_loss_kernel, ws_adam_kernel, and the gather / target / scatter
//   kernels between x0, trajectories and the per-subsystem sample matrices.
// Network of subsystem g: h1 = gelu(x W1 + b1), h2 = gelu(h1 W2 + b2), out = [h2, x] W3 + b3
// with gelu(z) = z (1 + erf(z / sqrt 2)) / 2, x = x0 slice / x_scale, u rows = y_scale * out;
// the loss is the mean squared error over subsystems, samples and outputs (in units of
// y_scale); the optimiser is Adam.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <fstream>
#include <random>
#include <string>
#include <vector>

#include "dlmpc_device.h"

namespace dlmpc {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr float kInvSqrt2 = 0.70710678118654752f;
constexpr float kInvSqrt2Pi = 0.39894228040143268f;

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.f + erff(z * kInvSqrt2)); }
__device__ __forceinline__ float gelu_grad(float z) {
  return 0.5f * (1.f + erff(z * kInvSqrt2)) + z * kInvSqrt2Pi * expf(-0.5f * z * z);
}

enum Epi { kStore = 0, kBiasGelu = 1, kBiasOnly = 2, kGeluGrad = 3 };

struct GemmArgs {
  int M, N, K;
  const float *A;  // element (m, k): TA ? A[k*lda + m] : A[m*lda + k]   (per group: + g*sA)
  const float *B;  // element (k, n): TB ? B[n*ldb + k] : B[k*ldb + n]   (per group: + g*sB)
  float *C;        // C[m*ldc + n] (+ g*sC)
  float *Z;        // kBiasGelu / kBiasOnly: pre-activation out; kGeluGrad: pre-activation in
  const float *bias;  // [G][N]
  int lda, ldb, ldc, ldz;
  int64_t sA, sB, sC, sZ;
};

// Grouped GEMM, one 32 x 32 tile of C per block (4 waves of 16 x 16), K in steps of 32.
template <bool TA, bool TB, int EPI>
__global__ __launch_bounds__(256) void ws_gemm_kernel(GemmArgs g) {
  const int grp = blockIdx.z, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int m0 = blockIdx.y * 32 + 16 * (wave >> 1), n0 = blockIdx.x * 32 + 16 * (wave & 1);
  const float *A = g.A + grp * g.sA;
  const float *B = g.B + grp * g.sB;
  const int am = m0 + (lane & 15), bn = n0 + (lane & 15);
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < g.K; k0 += 32) {
    bf16x8 ah, al, bh, bl;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int kk = k0 + 8 * (lane >> 4) + e;
      float av = 0.f, bv = 0.f;
      if (am < g.M && kk < g.K) av = TA ? A[int64_t(kk) * g.lda + am] : A[int64_t(am) * g.lda + kk];
      if (bn < g.N && kk < g.K) bv = TB ? B[int64_t(bn) * g.ldb + kk] : B[int64_t(kk) * g.ldb + bn];
      const __bf16 ha = static_cast<__bf16>(av), hb = static_cast<__bf16>(bv);
      ah[e] = ha;
      al[e] = static_cast<__bf16>(av - static_cast<float>(ha));
      bh[e] = hb;
      bl[e] = static_cast<__bf16>(bv - static_cast<float>(hb));
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc, 0, 0, 0);
  }
  // lane holds C rows m0 + 4 (lane / 16) + e, column n0 + lane % 16
  const int n = n0 + (lane & 15);
  if (n >= g.N) return;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int m = m0 + 4 * (lane >> 4) + e;
    if (m >= g.M) continue;
    const int64_t ci = grp * g.sC + int64_t(m) * g.ldc + n;
    float v = acc[e];
    if (EPI == kBiasGelu || EPI == kBiasOnly) {
      v += g.bias[int64_t(grp) * g.N + n];
      g.Z[grp * g.sZ + int64_t(m) * g.ldz + n] = v;
      if (EPI == kBiasGelu) v = gelu(v);
    } else if (EPI == kGeluGrad) {
      v *= gelu_grad(g.Z[grp * g.sZ + int64_t(m) * g.ldz + n]);
    }
    g.C[ci] = v;
  }
}

// db[g][n] = sum_s dZ[g][s][n]
__global__ __launch_bounds__(256) void ws_bias_grad_kernel(const float *dZ, float *db, int S, int N) {
  const int grp = blockIdx.y, n = blockIdx.x * 256 + threadIdx.x;
  if (n >= N) return;
  double s = 0.0;
  for (int i = 0; i < S; ++i) s += dZ[(int64_t(grp) * S + i) * N + n];
  db[int64_t(grp) * N + n] = float(s);
}

// dY = 2 (Y - T) / count; per-block partial sums of the squared error.
__global__ __launch_bounds__(256) void ws_loss_kernel(const float *Y, const float *T, float *dY, int64_t n,
                                                      double inv_count, double *part) {
  __shared__ double red[4];
  double acc = 0.0;
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
    const double d = double(Y[i]) - double(T[i]);
    acc += d * d;
    dY[i] = float(2.0 * d * inv_count);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(256) void ws_adam_kernel(float *th, const float *gr, float *m, float *v, int64_t n,
                                                      float lr, float c1, float c2) {
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
    const float g = gr[i];
    const float mi = 0.9f * m[i] + 0.1f * g;
    const float vi = 0.999f * v[i] + 0.001f * g * g;
    m[i] = mi;
    v[i] = vi;
    th[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + 1e-8f);
  }
}

// X[g][s][i] = x0[s][member i / nx of P(g)] / x_scale, zero-padded to IN (row stride ld).
__global__ __launch_bounds__(64) void ws_gather_kernel(const double *x0, float *X, int ld, const int64_t *rt_ptr,
                                                       const int32_t *rt_col, int N, int nx, int S, int IN,
                                                       float inv_xs) {
  const int g = blockIdx.x, s = blockIdx.y;
  const int64_t t0 = rt_ptr[g];
  const int np = int(rt_ptr[g + 1] - t0);
  for (int i = threadIdx.x; i < IN; i += 64) {
    float v = 0.f;
    if (i < np * nx) v = float(x0[int64_t(s) * N * nx + int64_t(rt_col[t0 + i / nx]) * nx + i % nx]) * inv_xs;
    X[(int64_t(g) * S + s) * ld + i] = v;
  }
}

// Targets from trajectories: T[g][s][l] = y[s][g*rs + roff + l] / y_scale.
__global__ __launch_bounds__(64) void ws_target_kernel(const double *y, float *T, int N, int rs, int roff, int OUT,
                                                       int S, float inv_ys) {
  const int g = blockIdx.x, s = blockIdx.y;
  for (int l = threadIdx.x; l < OUT; l += 64)
    T[(int64_t(g) * S + s) * OUT + l] = float(y[int64_t(s) * N * rs + int64_t(g) * rs + roff + l]) * inv_ys;
}

// Predicted input rows: y[s][g*rs + roff + l] = y_scale * Y[g][s][l].
template <typename T>
__global__ __launch_bounds__(64) void ws_scatter_kernel(T *y, const float *Y, int N, int rs, int roff, int OUT, int S,
                                                        float ys) {
  const int g = blockIdx.x, s = blockIdx.y;
  for (int l = threadIdx.x; l < OUT; l += 64)
    y[int64_t(s) * N * rs + int64_t(g) * rs + roff + l] = T(ys * Y[(int64_t(g) * S + s) * OUT + l]);
}

}  // namespace

// ------------------------------------------------------------------ host side

#define WS_CHECK(expr)                                                    \
  do {                                                                    \
    hipError_t e_ = (expr);                                               \
    if (e_ != hipSuccess) {                                               \
      err = std::string(#expr) + ": " + hipGetErrorString(e_);            \
      return DLMPC_EDEVICE;                                               \
    }                                                                     \
  } while (0)

WarmStart::~WarmStart() {
  for (void *p : owned_) (void)hipFree(p);
}

int WarmStart::alloc_bytes(void **dst, size_t bytes, std::string &err) {
  void *p = nullptr;
  if (hipMalloc(&p, std::max<size_t>(bytes, 16)) != hipSuccess) {
    err = "hipMalloc failed (warm-start network)";
    return DLMPC_ENOMEM;
  }
  owned_.push_back(p);
  *dst = p;
  return DLMPC_OK;
}

int WarmStart::init(const HostSetup &hs, int hidden, int max_samples, uint64_t seed, double x_scale,
                    double y_scale, hipStream_t s, std::string &err) {
  if (hidden < 1 || hidden > 4096 || max_samples < 1 || max_samples > 65535 || !(x_scale > 0) ||
      !(y_scale > 0) || !std::isfinite(x_scale) || !std::isfinite(y_scale)) {
    err = "warm start: need 1 <= hidden <= 4096, 1 <= max_samples <= 65535, finite positive scales";
    return DLMPC_EINVAL;
  }
  G = hs.N;
  nx = hs.nx;
  rs = hs.rs;
  roff = hs.nx * hs.T;
  IN = hs.p_max * hs.nx;
  H = hidden;
  OUT = hs.rs - roff;  // nu (T - 1) input rows
  Smax = max_samples;
  xs = x_scale;
  ys = y_scale;
  stream_ = s;
  const int64_t per = int64_t(IN) * H + H + int64_t(H) * H + H + int64_t(H + IN) * OUT + OUT;
  n_params = int64_t(G) * per;
  const size_t act = size_t(G) * Smax, F = sizeof(float);
  int rc;
  void *p[16];
  if ((rc = alloc_bytes(&p[0], F * n_params, err)) || (rc = alloc_bytes(&p[1], F * n_params, err)) ||
      (rc = alloc_bytes(&p[2], F * n_params, err)) || (rc = alloc_bytes(&p[3], F * n_params, err)) ||
      (rc = alloc_bytes(&p[4], F * act * (H + IN), err)) || (rc = alloc_bytes(&p[5], F * act * H, err)) ||
      (rc = alloc_bytes(&p[6], F * act * H, err)) || (rc = alloc_bytes(&p[7], F * act * H, err)) ||
      (rc = alloc_bytes(&p[8], F * act * OUT, err)) || (rc = alloc_bytes(&p[9], F * act * OUT, err)) ||
      (rc = alloc_bytes(&p[10], F * act * OUT, err)) || (rc = alloc_bytes(&p[11], F * act * H, err)) ||
      (rc = alloc_bytes(&p[12], F * act * H, err)) || (rc = alloc_bytes(&p[13], sizeof(double) * kLossBlocks, err)) ||
      (rc = alloc_bytes(&p[14], sizeof(int64_t) * (G + 1), err)) ||
      (rc = alloc_bytes(&p[15], sizeof(int32_t) * hs.rt_col.size(), err)))
    return rc;
  theta = static_cast<float *>(p[0]);
  grad = static_cast<float *>(p[1]);
  mom1_ = static_cast<float *>(p[2]);
  mom2_ = static_cast<float *>(p[3]);
  XA_ = static_cast<float *>(p[4]);
  Z1_ = static_cast<float *>(p[5]);
  A1_ = static_cast<float *>(p[6]);
  Z2_ = static_cast<float *>(p[7]);
  Y_ = static_cast<float *>(p[8]);
  T_ = static_cast<float *>(p[9]);
  dY_ = static_cast<float *>(p[10]);
  dZ2_ = static_cast<float *>(p[11]);
  dZ1_ = static_cast<float *>(p[12]);
  loss_part_ = static_cast<double *>(p[13]);
  rt_ptr_ = static_cast<int64_t *>(p[14]);
  rt_col_ = static_cast<int32_t *>(p[15]);
  WS_CHECK(hipMemcpy(rt_ptr_, hs.rt_ptr.data(), sizeof(int64_t) * (G + 1), hipMemcpyHostToDevice));
  WS_CHECK(hipMemcpy(rt_col_, hs.rt_col.data(), sizeof(int32_t) * hs.rt_col.size(), hipMemcpyHostToDevice));
  // Seeded He-style initialisation; biases zero. The skip block of W3 starts at zero too.
  std::vector<float> h(n_params, 0.f);
  std::mt19937_64 gen(seed);
  std::normal_distribution<float> nd(0.f, 1.f);
  float *W1, *b1, *W2, *b2, *W3, *b3;
  views(h.data(), &W1, &b1, &W2, &b2, &W3, &b3);
  const float s1 = std::sqrt(2.f / IN), s2 = std::sqrt(2.f / H), s3 = std::sqrt(1.f / H);
  for (int64_t i = 0; i < int64_t(G) * IN * H; ++i) W1[i] = s1 * nd(gen);
  for (int64_t i = 0; i < int64_t(G) * H * H; ++i) W2[i] = s2 * nd(gen);
  for (int g = 0; g < G; ++g)
    for (int64_t i = 0; i < int64_t(H) * OUT; ++i) W3[int64_t(g) * (H + IN) * OUT + i] = s3 * nd(gen);
  WS_CHECK(hipMemcpy(theta, h.data(), sizeof(float) * n_params, hipMemcpyHostToDevice));
  WS_CHECK(hipMemset(mom1_, 0, sizeof(float) * n_params));
  WS_CHECK(hipMemset(mom2_, 0, sizeof(float) * n_params));
  WS_CHECK(hipMemset(grad, 0, sizeof(float) * n_params));
  step = 0;
  return DLMPC_OK;
}

void WarmStart::views(float *base, float **W1, float **b1, float **W2, float **b2, float **W3, float **b3) const {
  *W1 = base;
  *b1 = *W1 + int64_t(G) * IN * H;
  *W2 = *b1 + int64_t(G) * H;
  *b2 = *W2 + int64_t(G) * H * H;
  *W3 = *b2 + int64_t(G) * H;
  *b3 = *W3 + int64_t(G) * (H + IN) * OUT;
}

namespace {

struct Mat {  // one operand or result: base pointer, leading dimension, per-group stride
  const float *p;
  int ld;
  int64_t sg;
};

template <bool TA, bool TB, int EPI>
int gemm(hipStream_t s, int G, int M, int N, int K, Mat A, Mat B, Mat C, Mat Z, const float *bias,
         std::string &err) {
  GemmArgs g{M,    N,    K,    A.p,  B.p,  const_cast<float *>(C.p), const_cast<float *>(Z.p), bias,
             A.ld, B.ld, C.ld, Z.ld, A.sg, B.sg,                       C.sg,                       Z.sg};
  hipLaunchKernelGGL((ws_gemm_kernel<TA, TB, EPI>), dim3((N + 31) / 32, (M + 31) / 32, G), dim3(256), 0, s, g);
  WS_CHECK(hipGetLastError());
  return DLMPC_OK;
}

}  // namespace

int WarmStart::forward(int S, const double *x0_dev, std::string &err) {
  if (S < 1 || S > Smax || !x0_dev) {
    err = "warm start: sample count out of range or NULL input";
    return DLMPC_EINVAL;
  }
  const int LX = H + IN;  // row length of XA
  hipLaunchKernelGGL(ws_gather_kernel, dim3(G, S), dim3(64), 0, stream_, x0_dev, XA_ + H, LX, rt_ptr_, rt_col_, G,
                     nx, S, IN, float(1.0 / xs));
  WS_CHECK(hipGetLastError());
  float *W1, *b1, *W2, *b2, *W3, *b3;
  views(theta, &W1, &b1, &W2, &b2, &W3, &b3);
  const int64_t sX = int64_t(S) * LX, sH = int64_t(S) * H, sO = int64_t(S) * OUT;
  const Mat X{XA_ + H, LX, sX}, XA{XA_, LX, sX}, Z1{Z1_, H, sH}, A1{A1_, H, sH}, Z2{Z2_, H, sH}, Y{Y_, OUT, sO};
  int rc;
  if ((rc = gemm<false, false, kBiasGelu>(stream_, G, S, H, IN, X, Mat{W1, H, int64_t(IN) * H}, A1, Z1, b1, err)))
    return rc;
  if ((rc = gemm<false, false, kBiasGelu>(stream_, G, S, H, H, A1, Mat{W2, H, int64_t(H) * H}, XA, Z2, b2, err)))
    return rc;
  // output layer over [h2, x]; its pre-activation is the output itself (Z = C = Y)
  return gemm<false, false, kBiasOnly>(stream_, G, S, OUT, LX, XA, Mat{W3, OUT, int64_t(LX) * OUT}, Y, Y, b3, err);
}

int WarmStart::backward(int S, const double *y_dev, double *loss, std::string &err) {
  if (S < 1 || S > Smax || !y_dev) {
    err = "warm start: sample count out of range or NULL targets";
    return DLMPC_EINVAL;
  }
  hipLaunchKernelGGL(ws_target_kernel, dim3(G, S), dim3(64), 0, stream_, y_dev, T_, G, rs, roff, OUT, S,
                     float(1.0 / ys));
  WS_CHECK(hipGetLastError());
  const int64_t nY = int64_t(G) * S * OUT;
  hipLaunchKernelGGL(ws_loss_kernel, dim3(kLossBlocks), dim3(256), 0, stream_, Y_, T_, dY_, nY, 1.0 / double(nY),
                     loss_part_);
  WS_CHECK(hipGetLastError());
  float *W1, *b1, *W2, *b2, *W3, *b3, *dW1, *db1, *dW2, *db2, *dW3, *db3;
  views(theta, &W1, &b1, &W2, &b2, &W3, &b3);
  views(grad, &dW1, &db1, &dW2, &db2, &dW3, &db3);
  const int LX = H + IN;
  const int64_t sX = int64_t(S) * LX, sH = int64_t(S) * H, sO = int64_t(S) * OUT;
  const Mat X{XA_ + H, LX, sX}, XA{XA_, LX, sX}, Z1{Z1_, H, sH}, A1{A1_, H, sH}, Z2{Z2_, H, sH};
  const Mat dY{dY_, OUT, sO}, dZ2{dZ2_, H, sH}, dZ1{dZ1_, H, sH}, none{nullptr, 0, 0};
  int rc;
  // output layer: dW3 = [h2, x]' dY, db3 = colsum dY, dZ2 = (dY W3[:H]') * gelu'(Z2)
  if ((rc = gemm<true, false, kStore>(stream_, G, LX, OUT, S, XA, dY, Mat{dW3, OUT, int64_t(LX) * OUT}, none,
                                      nullptr, err)))
    return rc;
  hipLaunchKernelGGL(ws_bias_grad_kernel, dim3((OUT + 255) / 256, G), dim3(256), 0, stream_, dY_, db3, S, OUT);
  WS_CHECK(hipGetLastError());
  if ((rc = gemm<false, true, kGeluGrad>(stream_, G, S, H, OUT, dY, Mat{W3, OUT, int64_t(LX) * OUT}, dZ2, Z2,
                                         nullptr, err)))
    return rc;
  // hidden layer 2
  if ((rc = gemm<true, false, kStore>(stream_, G, H, H, S, A1, dZ2, Mat{dW2, H, int64_t(H) * H}, none, nullptr,
                                      err)))
    return rc;
  hipLaunchKernelGGL(ws_bias_grad_kernel, dim3((H + 255) / 256, G), dim3(256), 0, stream_, dZ2_, db2, S, H);
  WS_CHECK(hipGetLastError());
  if ((rc = gemm<false, true, kGeluGrad>(stream_, G, S, H, H, dZ2, Mat{W2, H, int64_t(H) * H}, dZ1, Z1, nullptr,
                                         err)))
    return rc;
  // hidden layer 1
  if ((rc = gemm<true, false, kStore>(stream_, G, IN, H, S, X, dZ1, Mat{dW1, H, int64_t(IN) * H}, none, nullptr,
                                      err)))
    return rc;
  hipLaunchKernelGGL(ws_bias_grad_kernel, dim3((H + 255) / 256, G), dim3(256), 0, stream_, dZ1_, db1, S, H);
  WS_CHECK(hipGetLastError());
  if (loss) {
    std::vector<double> part(kLossBlocks);
    WS_CHECK(hipMemcpyAsync(part.data(), loss_part_, sizeof(double) * kLossBlocks, hipMemcpyDeviceToHost, stream_));
    WS_CHECK(hipStreamSynchronize(stream_));
    double sum = 0.0;
    for (double v : part) sum += v;
    *loss = sum / double(nY);
  }
  return DLMPC_OK;
}

int WarmStart::adam(double lr, std::string &err) {
  if (!(lr > 0) || !std::isfinite(lr)) {
    err = "warm start: learning rate must be finite and positive";
    return DLMPC_EINVAL;
  }
  ++step;
  const float c1 = float(1.0 / (1.0 - std::pow(0.9, double(step))));
  const float c2 = float(1.0 / (1.0 - std::pow(0.999, double(step))));
  hipLaunchKernelGGL(ws_adam_kernel, dim3(2048), dim3(256), 0, stream_, theta, grad, mom1_, mom2_, n_params,
                     float(lr), c1, c2);
  WS_CHECK(hipGetLastError());
  return DLMPC_OK;
}

int WarmStart::predict(int S, const double *x0_dev, double *y_dev, std::string &err) {
  int rc = forward(S, x0_dev, err);
  if (rc) return rc;
  hipLaunchKernelGGL(ws_scatter_kernel<double>, dim3(G, S), dim3(64), 0, stream_, y_dev, Y_, G, rs, roff, OUT, S,
                     float(ys));
  WS_CHECK(hipGetLastError());
  return DLMPC_OK;
}

int WarmStart::predict(int S, const double *x0_dev, float *y_dev, std::string &err) {
  int rc = forward(S, x0_dev, err);
  if (rc) return rc;
  hipLaunchKernelGGL(ws_scatter_kernel<float>, dim3(G, S), dim3(64), 0, stream_, y_dev, Y_, G, rs, roff, OUT, S,
                     float(ys));
  WS_CHECK(hipGetLastError());
  return DLMPC_OK;
}

// File: int32 {tag, G, IN, H, OUT, version}, double {x_scale, y_scale}, float theta[n_params].
int WarmStart::save(const char *path, std::string &err) {
  std::vector<float> h(n_params);
  WS_CHECK(hipMemcpy(h.data(), theta, sizeof(float) * n_params, hipMemcpyDeviceToHost));
  std::ofstream f(path, std::ios::binary);
  const int32_t hdr[6] = {kMagic, G, IN, H, OUT, 1};
  const double sc[2] = {xs, ys};
  if (f) f.write(reinterpret_cast<const char *>(hdr), sizeof(hdr));
  if (f) f.write(reinterpret_cast<const char *>(sc), sizeof(sc));
  if (f) f.write(reinterpret_cast<const char *>(h.data()), std::streamsize(sizeof(float) * n_params));
  if (!f) {
    err = std::string("cannot write ") + path;
    return DLMPC_EINVAL;
  }
  return DLMPC_OK;
}

int WarmStart::peek(const char *path, int32_t *hidden, std::string &err) {
  std::ifstream f(path, std::ios::binary);
  int32_t hdr[6];
  if (!f || !f.read(reinterpret_cast<char *>(hdr), sizeof(hdr)) || hdr[0] != kMagic) {
    err = std::string("not a warm-start weight file: ") + path;
    return DLMPC_EINVAL;
  }
  *hidden = hdr[3];
  return DLMPC_OK;
}

int WarmStart::load(const char *path, std::string &err) {
  std::ifstream f(path, std::ios::binary);
  int32_t hdr[6];
  double sc[2];
  if (!f || !f.read(reinterpret_cast<char *>(hdr), sizeof(hdr)) || !f.read(reinterpret_cast<char *>(sc), sizeof(sc)) ||
      hdr[0] != kMagic) {
    err = std::string("not a warm-start weight file: ") + path;
    return DLMPC_EINVAL;
  }
  if (hdr[1] != G || hdr[2] != IN || hdr[3] != H || hdr[4] != OUT) {
    err = "warm-start weight file does not match this problem's network shape";
    return DLMPC_EINVAL;
  }
  if (!(sc[0] > 0) || !(sc[1] > 0) || !std::isfinite(sc[0]) || !std::isfinite(sc[1])) {
    err = "warm-start weight file has invalid scales";
    return DLMPC_EINVAL;
  }
  std::vector<float> h(n_params);
  if (!f.read(reinterpret_cast<char *>(h.data()), std::streamsize(sizeof(float) * n_params))) {
    err = "truncated warm-start weight file";
    return DLMPC_EINVAL;
  }
  xs = sc[0];
  ys = sc[1];
  WS_CHECK(hipMemcpy(theta, h.data(), sizeof(float) * n_params, hipMemcpyHostToDevice));
  return DLMPC_OK;
}

}  // namespace dlmpc
