// C ABI of libdlmpc (declared in include/dlmpc.h): argument checks, the offline setup,
// device residency, the captured iteration graph and the per-step solve loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "dlmpc_device.h"

using dlmpc::Ctl;
using dlmpc::HostSetup;

struct dlmpc_problem {
  HostSetup hs;
  dlmpc_options opt{};
  bool host_only = false;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::unique_ptr<dlmpc::Engine> eng;
  // Captured graphs of 1, 2, 4, ..., 2^(kGraphs-1) iterations of the graph schedule.
  static constexpr int kGraphs = 6;
  hipGraph_t graph[kGraphs] = {};
  hipGraphExec_t gexec[kGraphs] = {};
  int K = 32;  // fixed chunk when check_every > 0; otherwise the first chunk
  int sched = 0;  // 0 = graph, 1 = persistent
  double tune_graph_us = 0.0, tune_persistent_us = 0.0;
  // batched-engine autotuning: per-launch us of the Phi-comp variants (1, 2 instance tiles per
  // wave) and of the Psi-comp splits (kPsiCaps order); 1 if the choice came from the cache
  double tune_phi_us[2] = {0, 0}, tune_psi_us[6] = {0, 0, 0, 0, 0, 0};
  int32_t tune_cached = 0;
  Ctl *h_ctl = nullptr;  // pinned, 2 slots
  void *h_xchg = nullptr;  // pinned staging of the host-exchange schedules
  hipEvent_t ev_ctl[2] = {nullptr, nullptr};
  hipEvent_t ev_t0 = nullptr, ev_t1 = nullptr;
  double *d_x0 = nullptr, *d_u0 = nullptr, *d_phi = nullptr, *d_warm = nullptr;
  // batched engine
  std::unique_ptr<dlmpc::BatchEngine> beng;
  hipGraph_t bgraph[kGraphs] = {};
  hipGraphExec_t bgexec[kGraphs] = {};
  hipGraph_t sgraph[kGraphs] = {};      // iterations with the CG step of streamed joins
  hipGraphExec_t sgexec[kGraphs] = {};
  double *d_bx0 = nullptr, *d_bu0 = nullptr;
  dlmpc::BCtl *h_bctl = nullptr;
  // learned warm start: network, predicted multipliers [Bmax][R], cold re-solve staging
  std::unique_ptr<dlmpc::WarmStart> ws;
  double *d_fx0 = nullptr, *d_fu0 = nullptr, *d_falpha = nullptr, *d_fy = nullptr;
  int cg_iters = 12;
  hipEvent_t ev_w0 = nullptr, ev_w1 = nullptr;
  float *d_sy = nullptr;  // streamed solves: predicted trajectories of the joining instances [Bmax][R]
  // closed loop: current states and inputs, stopping trajectories, shifted starts
  double *d_clx = nullptr, *d_clu = nullptr, *d_cly = nullptr, *d_clys = nullptr;
  double *d_clrs = nullptr, *d_frs = nullptr;  // penalty factors of the closed loop's instances
  // per-solve precompute and FP64 check timing; device finiteness flag of x0 (device entries)
  hipEvent_t ev_p0 = nullptr, ev_p1 = nullptr, ev_c0 = nullptr, ev_c1 = nullptr;
  int32_t *d_flag = nullptr, *h_flag = nullptr;
  double warm_eps = 1e-4;  // eps of warm-started batched and streamed runs
  double rho = 5.0;        // penalty of the solves (options.rho until dlmpc_set_rho)
  bool struct_ok = false;  // the structured Psi-comp is a candidate of the setup timing
  bool psi_structured = false;
  double tune_structured_us = 0.0;
  // neighbour-coupled constraints of the single-instance solves (library row indices)
  std::vector<int64_t> cp_a, cp_b;
  std::vector<double> cp_lo, cp_hi;
};

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

#define API_HIP(expr)                                                               \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess) return fail(DLMPC_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

void release_device(dlmpc_problem *p) {
  if (!p || p->host_only) return;
  (void)hipSetDevice(p->opt.device);
  if (p->stream) (void)hipStreamSynchronize(p->stream);
  for (int g = 0; g < dlmpc_problem::kGraphs; ++g) {
    if (p->gexec[g]) (void)hipGraphExecDestroy(p->gexec[g]);
    if (p->graph[g]) (void)hipGraphDestroy(p->graph[g]);
    if (p->bgexec[g]) (void)hipGraphExecDestroy(p->bgexec[g]);
    if (p->bgraph[g]) (void)hipGraphDestroy(p->bgraph[g]);
    if (p->sgexec[g]) (void)hipGraphExecDestroy(p->sgexec[g]);
    if (p->sgraph[g]) (void)hipGraphDestroy(p->sgraph[g]);
    p->sgexec[g] = nullptr;
    p->sgraph[g] = nullptr;
    p->gexec[g] = nullptr;
    p->graph[g] = nullptr;
    p->bgexec[g] = nullptr;
    p->bgraph[g] = nullptr;
  }
  if (p->h_bctl) (void)hipHostFree(p->h_bctl);
  for (double *d : {p->d_bx0, p->d_bu0, p->d_fx0, p->d_fu0, p->d_falpha, p->d_fy, p->d_clx, p->d_clu, p->d_cly,
                    p->d_clys, p->d_clrs, p->d_frs})
    if (d) (void)hipFree(d);
  p->d_fx0 = p->d_fu0 = p->d_falpha = p->d_fy = nullptr;
  p->d_clx = p->d_clu = p->d_cly = p->d_clys = p->d_clrs = p->d_frs = nullptr;
  if (p->d_sy) (void)hipFree(p->d_sy);
  p->d_sy = nullptr;
  for (hipEvent_t e : {p->ev_w0, p->ev_w1})
    if (e) (void)hipEventDestroy(e);
  p->ev_w0 = p->ev_w1 = nullptr;
  p->ws.reset();
  p->beng.reset();
  p->h_bctl = nullptr;
  p->d_bx0 = p->d_bu0 = nullptr;
  for (hipEvent_t e : {p->ev_ctl[0], p->ev_ctl[1], p->ev_t0, p->ev_t1, p->ev_p0, p->ev_p1, p->ev_c0, p->ev_c1})
    if (e) (void)hipEventDestroy(e);
  p->ev_p0 = p->ev_p1 = p->ev_c0 = p->ev_c1 = nullptr;
  if (p->d_flag) (void)hipFree(p->d_flag);
  if (p->h_flag) (void)hipHostFree(p->h_flag);
  p->d_flag = p->h_flag = nullptr;
  if (p->h_ctl) (void)hipHostFree(p->h_ctl);
  if (p->h_xchg) (void)hipHostFree(p->h_xchg);
  p->h_xchg = nullptr;
  for (double *d : {p->d_x0, p->d_u0, p->d_phi, p->d_warm})
    if (d) (void)hipFree(d);
  p->eng.reset();
  if (p->own_stream && p->stream) (void)hipStreamDestroy(p->stream);
  p->h_ctl = nullptr;
  p->stream = nullptr;
  dlmpc::free_factors_device(p->hs);
}

int choose_schedule(dlmpc_problem *p);

// (Re)captures the single-instance iteration graphs of 2^g iterations (synchronises).
int capture_single(dlmpc_problem *p) {
  std::string err;
  API_HIP(hipStreamSynchronize(p->stream));
  for (int g = 0; g < dlmpc_problem::kGraphs; ++g) {
    if (p->gexec[g]) (void)hipGraphExecDestroy(p->gexec[g]);
    if (p->graph[g]) (void)hipGraphDestroy(p->graph[g]);
    p->gexec[g] = nullptr;
    p->graph[g] = nullptr;
    API_HIP(hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal));
    for (int i = 0; i < (1 << g); ++i) {
      const int rc = p->eng->iteration(err);
      if (rc) {
        hipGraph_t gr = nullptr;
        (void)hipStreamEndCapture(p->stream, &gr);
        if (gr) (void)hipGraphDestroy(gr);
        return fail(rc, err);
      }
    }
    API_HIP(hipStreamEndCapture(p->stream, &p->graph[g]));
    API_HIP(hipGraphInstantiate(&p->gexec[g], p->graph[g], nullptr, nullptr, 0));
  }
  API_HIP(hipStreamSynchronize(p->stream));
  return DLMPC_OK;
}
int setup_batch(dlmpc_problem *p);

int setup_device(dlmpc_problem *p) {
  const HostSetup &hs = p->hs;
  int ndev = 0;
  API_HIP(hipGetDeviceCount(&ndev));
  if (p->opt.device < 0 || p->opt.device >= ndev) return fail(DLMPC_EINVAL, "device ordinal out of range");
  API_HIP(hipSetDevice(p->opt.device));
  if (p->opt.stream) {
    p->stream = static_cast<hipStream_t>(p->opt.stream);
  } else {
    API_HIP(hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking));
    p->own_stream = true;
  }
  p->eng = dlmpc::make_engine(p->opt.precision, hs.nx);
  if (!p->eng) return fail(DLMPC_EINVAL, "unsupported (precision, nx) combination; nx must be 1..4");
  std::string err;
  int rc = p->eng->init(hs, p->opt.rho, p->stream, err);
  if (rc) return fail(rc, err);
  {
    // structured Psi-comp: forced by its flag, or a candidate of the setup timing when no
    // schedule is given (a patch too large for its staging leaves only the dense one)
    const uint32_t f = p->opt.flags;
    const uint32_t fixed = DLMPC_FLAG_SCHED_GRAPH | DLMPC_FLAG_SCHED_PERSISTENT | DLMPC_FLAG_SCHED_STEPWISE |
                           DLMPC_FLAG_SCHED_HOST_EXCHANGE | DLMPC_FLAG_SCHED_NAIVE | DLMPC_FLAG_NO_TUNE;
    if (f & DLMPC_FLAG_STRUCTURED_PSI) {
      if ((rc = p->eng->enable_structured(err))) return fail(rc, err);
    } else if (!(f & fixed)) {
      p->struct_ok = p->eng->enable_structured(err) == DLMPC_OK;
      p->eng->set_structured(false);
    }
  }
  API_HIP(hipMalloc(&p->d_x0, sizeof(double) * size_t(hs.N) * hs.nx));
  API_HIP(hipMalloc(&p->d_u0, sizeof(double) * size_t(hs.N) * hs.nu));
  API_HIP(hipMalloc(&p->d_phi, sizeof(double) * size_t(std::max<int64_t>(hs.nnz, 1))));
  API_HIP(hipMalloc(&p->d_warm, sizeof(double) * size_t(2 * std::max<int64_t>(hs.nnz, 1))));
  API_HIP(hipHostMalloc(reinterpret_cast<void **>(&p->h_ctl), 2 * sizeof(Ctl), hipHostMallocDefault));
  std::memset(p->h_ctl, 0, 2 * sizeof(Ctl));
  for (auto *e : {&p->ev_ctl[0], &p->ev_ctl[1]}) API_HIP(hipEventCreateWithFlags(e, hipEventDisableTiming));
  API_HIP(hipEventCreate(&p->ev_t0));
  API_HIP(hipEventCreate(&p->ev_t1));
  for (auto *e : {&p->ev_p0, &p->ev_p1, &p->ev_c0, &p->ev_c1}) API_HIP(hipEventCreate(e));
  API_HIP(hipMalloc(&p->d_flag, sizeof(int32_t)));
  API_HIP(hipHostMalloc(reinterpret_cast<void **>(&p->h_flag), sizeof(int32_t), hipHostMallocDefault));
  // Iteration graphs of 2^g iterations; every launch after the device-side stop is a no-op.
  p->K = p->opt.check_every > 0 ? std::min(p->opt.check_every, p->opt.max_iter) : 32;
  if ((rc = capture_single(p))) return rc;
  if (p->opt.max_batch > 0) {
    rc = setup_batch(p);
    if (rc) return rc;
  }
  return choose_schedule(p);
}

// Autotuner cache (file named by DLMPC_TUNE_CACHE): one line per problem signature,
// "<signature>|phi_ntw=<1|2> psi_capx=<n> sched=<0|1>".
std::string tune_signature(const dlmpc_problem *p) {
  const HostSetup &h = p->hs;
  hipDeviceProp_t prop{};
  std::string arch = "unknown";
  if (hipGetDeviceProperties(&prop, p->opt.device) == hipSuccess) arch = prop.gcnArchName;
  char buf[512];
  std::snprintf(buf, sizeof(buf), "N=%d nx=%d nu=%d T=%d nnz=%lld sumk=%lld sumdk=%lld dmax=%d bmax=%d prec=%d arch=%s",
                h.N, h.nx, h.nu, h.T, static_cast<long long>(h.nnz), static_cast<long long>(h.sum_k),
                static_cast<long long>(h.sum_dcol_k), h.d_col_max, p->opt.max_batch, p->opt.precision, arch.c_str());
  return buf;
}

bool tune_cache_read(const std::string &sig, int *phi_ntw, int *psi_capx, int *sched) {
  const char *path = std::getenv("DLMPC_TUNE_CACHE");
  if (!path || !*path) return false;
  std::FILE *f = std::fopen(path, "r");
  if (!f) return false;
  char line[1024];
  bool found = false;
  while (std::fgets(line, sizeof(line), f)) {
    std::string l(line);
    const size_t bar = l.find('|');
    if (bar == std::string::npos || l.substr(0, bar) != sig) continue;
    int a = 0, b = 0, c = 0;
    if (std::sscanf(l.c_str() + bar + 1, "phi_ntw=%d psi_capx=%d sched=%d", &a, &b, &c) == 3) {
      *phi_ntw = a;
      *psi_capx = b;
      *sched = c;
      found = true;
    }
  }
  std::fclose(f);
  return found;
}

void tune_cache_write(const std::string &sig, int phi_ntw, int psi_capx, int sched) {
  const char *path = std::getenv("DLMPC_TUNE_CACHE");
  if (!path || !*path) return;
  std::FILE *f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s|phi_ntw=%d psi_capx=%d sched=%d\n", sig.c_str(), phi_ntw, psi_capx, sched);
  std::fclose(f);
}

// Times the batched-engine variants with max_batch instances from a zero-multiplier start (every
// launch does the full work; x0 = 1 everywhere) and keeps the fastest Phi-comp and Psi-comp.
int tune_batch(dlmpc_problem *p) {
  const HostSetup &hs = p->hs;
  const int B = p->beng->bmax();
  const size_t nx = size_t(B) * hs.N * hs.nx, nr = size_t(B) * hs.N * hs.rs;
  std::vector<double> ones(nx, 1.0);
  double *x = nullptr, *z = nullptr;
  API_HIP(hipMalloc(&x, sizeof(double) * nx));
  API_HIP(hipMalloc(&z, sizeof(double) * nr));
  std::string err;
  auto run = [&]() -> int {
    API_HIP(hipMemcpy(x, ones.data(), sizeof(double) * nx, hipMemcpyHostToDevice));
    API_HIP(hipMemset(z, 0, sizeof(double) * nr));
    int rc = p->beng->precompute(x, B, 1 << 20, -1.0, 1, nullptr, err);
    if (!rc) rc = p->beng->start_alpha(z, err);
    if (rc) return fail(rc, err);
    auto time_k = [&](int k, double *us) -> int {
      float best = 1e30f;
      for (int rep = 0; rep < 6; ++rep) {  // the first launch warms code and caches
        API_HIP(hipEventRecord(p->ev_t0, p->stream));
        int r = p->beng->launch_one(k, err);
        if (r) return fail(r, err);
        API_HIP(hipEventRecord(p->ev_t1, p->stream));
        API_HIP(hipEventSynchronize(p->ev_t1));
        float ms = 0.f;
        API_HIP(hipEventElapsedTime(&ms, p->ev_t0, p->ev_t1));
        if (rep > 0) best = std::min(best, ms);
      }
      *us = 1e3 * best;
      return DLMPC_OK;
    };
    int cur_ntw = 1, cur_cap = 8, nu = 0;
    p->beng->variant(&cur_ntw, &cur_cap, &nu);
    for (int v = 0; v < 2; ++v) {
      if ((rc = p->beng->set_variant(v + 1, cur_cap, err))) return fail(rc, err);
      if ((rc = time_k(0, &p->tune_phi_us[v]))) return rc;
    }
    // a candidate replaces the default only when it is faster by more than timing noise (1 %)
    const int ntw = p->tune_phi_us[1] < 0.99 * p->tune_phi_us[0] ? 2 : 1;
    // splits of heavy column blocks, and the structured Psi-comp (0) where the problem allows it
    static const int caps[6] = {2, 4, 8, 16, 1 << 20, 0};
    for (int c = 0; c < 6; ++c) {
      p->tune_psi_us[c] = 0.0;
      if (p->beng->set_variant(ntw, caps[c], err)) continue;  // not available
      if ((rc = time_k(1, &p->tune_psi_us[c]))) return rc;
    }
    int best_c = 2;  // the default split
    for (int c = 0; c < 6; ++c)
      if (p->tune_psi_us[c] > 0.0 && p->tune_psi_us[c] < 0.99 * p->tune_psi_us[best_c]) best_c = c;
    if ((rc = p->beng->set_variant(ntw, caps[best_c], err))) return fail(rc, err);
    return DLMPC_OK;
  };
  const int rc = run();
  (void)hipStreamSynchronize(p->stream);
  (void)hipFree(x);
  (void)hipFree(z);
  return rc;
}

int setup_batch(dlmpc_problem *p) {
  const HostSetup &hs = p->hs;
  std::string err;
  if (p->opt.precision != DLMPC_FP32 && p->opt.precision != DLMPC_FP32_BF16)
    return fail(DLMPC_EINVAL, "the batched engine runs in FP32 or FP32_BF16 precision");
  p->beng = dlmpc::make_batch_engine(hs.nx);
  if (!p->beng) return fail(DLMPC_EINVAL, "batched engine: nx must be 1..4");
  int rc = p->beng->init(hs, p->opt.rho, p->opt.max_batch, p->opt.precision == DLMPC_FP32, p->stream, err);
  if (rc) return fail(rc, err);
  const int B = p->opt.max_batch;
  API_HIP(hipMalloc(&p->d_bx0, sizeof(double) * size_t(B) * hs.N * hs.nx));
  API_HIP(hipMalloc(&p->d_bu0, sizeof(double) * size_t(B) * hs.N * hs.nu));
  API_HIP(hipHostMalloc(reinterpret_cast<void **>(&p->h_bctl), sizeof(dlmpc::BCtl) * B, hipHostMallocDefault));
  const size_t R = size_t(hs.N) * hs.rs;
  API_HIP(hipMalloc(&p->d_fy, sizeof(double) * size_t(B) * R));
  API_HIP(hipMalloc(&p->d_falpha, sizeof(double) * size_t(B) * R));
  p->cg_iters = p->opt.warm_cg_iters > 0 ? p->opt.warm_cg_iters : 12;
  API_HIP(hipMalloc(&p->d_fx0, sizeof(double) * size_t(B) * hs.N * hs.nx));
  API_HIP(hipMalloc(&p->d_fu0, sizeof(double) * size_t(B) * hs.N * hs.nu));
  API_HIP(hipMalloc(&p->d_clx, sizeof(double) * size_t(B) * hs.N * hs.nx));
  API_HIP(hipMalloc(&p->d_clu, sizeof(double) * size_t(B) * hs.N * hs.nu));
  API_HIP(hipMalloc(&p->d_cly, sizeof(double) * size_t(B) * R));
  API_HIP(hipMalloc(&p->d_clys, sizeof(double) * size_t(B) * R));
  API_HIP(hipMalloc(&p->d_clrs, sizeof(double) * size_t(B)));
  API_HIP(hipMalloc(&p->d_frs, sizeof(double) * size_t(B)));
  API_HIP(hipEventCreate(&p->ev_w0));
  API_HIP(hipEventCreate(&p->ev_w1));
  // kernel variants: from the tuning cache, else timed here (before the graphs are captured:
  // they record the variant and the work-unit count), unless the caller fixed the defaults
  if (!(p->opt.flags & DLMPC_FLAG_NO_TUNE)) {
    int ntw = 0, capx = 0, sched = 0;
    std::string err2;
    if (tune_cache_read(tune_signature(p), &ntw, &capx, &sched) && !p->beng->set_variant(ntw, capx, err2)) {
      p->tune_cached = 1;
    } else {
      rc = tune_batch(p);
      if (rc) return rc;
    }
  }
  for (int joins = 0; joins < 2; ++joins)
    for (int g = 0; g < dlmpc_problem::kGraphs; ++g) {
      API_HIP(hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal));
      for (int i = 0; i < (1 << g); ++i) {
        rc = p->beng->iteration(err, joins != 0);
        if (rc) {
          hipGraph_t gr = nullptr;
          (void)hipStreamEndCapture(p->stream, &gr);
          if (gr) (void)hipGraphDestroy(gr);
          return fail(rc, err);
        }
      }
      hipGraph_t &gr = joins ? p->sgraph[g] : p->bgraph[g];
      hipGraphExec_t &ex = joins ? p->sgexec[g] : p->bgexec[g];
      API_HIP(hipStreamEndCapture(p->stream, &gr));
      API_HIP(hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0));
    }
  API_HIP(hipStreamSynchronize(p->stream));
  return DLMPC_OK;
}

// Enqueues n iterations as a sum of captured power-of-two iteration graphs.
int launch_graphs(hipGraphExec_t *ex, hipStream_t s, int n) {
  constexpr int top = dlmpc_problem::kGraphs - 1;
  while (n >= (1 << top)) {
    API_HIP(hipGraphLaunch(ex[top], s));
    n -= 1 << top;
  }
  for (int g = top - 1; g >= 0; --g)
    if (n & (1 << g)) API_HIP(hipGraphLaunch(ex[g], s));
  return DLMPC_OK;
}

int launch_iterations(dlmpc_problem *p, int n) { return launch_graphs(p->gexec, p->stream, n); }

// Sizes the next chunk of iterations from the decay of the residual: least-squares slope of
// log max(r_p, r_d) over the last (up to 4) host checks, extrapolated to eps.
struct ChunkPredictor {
  double hk[4] = {0, 0, 0, 0}, hr[4] = {0, 0, 0, 0};
  int nh = 0;
  int next(int iters, double rp, double rd, double eps) {
    const double r = std::max(rp, rd);
    if (!(r > 0.0) || !std::isfinite(r)) return 8;
    for (int i = 3; i > 0; --i) {
      hk[i] = hk[i - 1];
      hr[i] = hr[i - 1];
    }
    hk[0] = iters;
    hr[0] = std::log(r);
    nh = std::min(nh + 1, 4);
    if (nh < 2) return 8;
    double mk = 0, mr = 0;
    for (int i = 0; i < nh; ++i) {
      mk += hk[i] / nh;
      mr += hr[i] / nh;
    }
    double sxy = 0, sxx = 0;
    for (int i = 0; i < nh; ++i) {
      sxy += (hk[i] - mk) * (hr[i] - mr);
      sxx += (hk[i] - mk) * (hk[i] - mk);
    }
    const double slope = sxx > 0 ? sxy / sxx : 0.0;
    if (!(slope < -1e-9)) return 8;
    const double need = (std::log(eps) - hr[0]) / slope;
    return int(std::min(64.0, std::max(1.0, std::round(need))));
  }
};

// Times n iterations of a schedule from x0 = (1, ..., 1) with the stop test disabled.
int time_schedule(dlmpc_problem *p, int sched, int n, double *us_per_iter) {
  std::string err;
  const HostSetup &hs = p->hs;
  std::vector<double> ones(size_t(hs.N) * hs.nx, 1.0);
  API_HIP(hipMemcpy(p->d_x0, ones.data(), ones.size() * sizeof(double), hipMemcpyHostToDevice));
  float best = 1e30f;
  for (int rep = 0; rep < 2; ++rep) {  // the first repetition warms code and caches
    int rc = p->eng->precompute(p->d_x0, nullptr, nullptr, n, -1.0, p->opt.rho, err);
    if (rc) return fail(rc, err);
    API_HIP(hipEventRecord(p->ev_t0, p->stream));
    if (sched == 1) {
      rc = p->eng->run_persistent(true, err);
      if (rc) return fail(rc, err);
    } else {
      rc = launch_iterations(p, n);
      if (rc) return rc;
    }
    API_HIP(hipEventRecord(p->ev_t1, p->stream));
    API_HIP(hipStreamSynchronize(p->stream));
    float ms = 0.f;
    API_HIP(hipEventElapsedTime(&ms, p->ev_t0, p->ev_t1));
    best = std::min(best, ms);
    API_HIP(hipMemcpy(&p->h_ctl[0], p->eng->ctl(), sizeof(Ctl), hipMemcpyDeviceToHost));
    if (p->h_ctl[0].bar_fail) return fail(DLMPC_EDEVICE, "persistent grid barrier timed out");
  }
  *us_per_iter = 1e3 * double(best) / n;
  return DLMPC_OK;
}

int choose_schedule(dlmpc_problem *p) {
  const uint32_t f = p->opt.flags;
  const bool can_persist = p->eng->persistent_grid() > 0;
  p->psi_structured = (f & DLMPC_FLAG_STRUCTURED_PSI) != 0;
  // the per-iteration schedules of the exchange ablation (no tuning)
  const int per_iter = (f & DLMPC_FLAG_SCHED_STEPWISE) ? 3
                       : (f & DLMPC_FLAG_SCHED_HOST_EXCHANGE) ? 4
                       : (f & DLMPC_FLAG_SCHED_NAIVE) ? 5 : 0;
  if (per_iter) {
    p->sched = per_iter;
    if (per_iter >= 4)
      API_HIP(hipHostMalloc(&p->h_xchg, p->eng->exchange_bytes(), hipHostMallocDefault));
    return DLMPC_OK;
  }
  if (f & DLMPC_FLAG_SCHED_GRAPH) {
    p->sched = 0;
    return DLMPC_OK;
  }
  if (f & DLMPC_FLAG_STRUCTURED_PSI) {  // the persistent kernel runs the dense Psi-comp only
    if (f & DLMPC_FLAG_SCHED_PERSISTENT) return fail(DLMPC_EINVAL, "the structured Psi-comp runs on the graph schedule");
    p->sched = 0;
    return DLMPC_OK;
  }
  if (f & DLMPC_FLAG_SCHED_PERSISTENT) {
    if (!can_persist) return fail(DLMPC_EDEVICE, "persistent schedule unavailable on this device");
    p->sched = 1;
    return DLMPC_OK;
  }
  if (f & DLMPC_FLAG_NO_TUNE) {
    p->sched = 0;
    return DLMPC_OK;
  }
  const std::string sig = tune_signature(p);
  int ntw = 0, capx = 0, sched = 0;
  // candidates: 0 graph schedule with the dense Psi-comp, 1 persistent, 2 graph schedule with the
  // structured Psi-comp (cached as such; p->sched is 0 for it)
  auto apply = [&](int s) -> int {
    p->sched = s == 1 ? 1 : 0;
    p->psi_structured = s == 2;
    p->eng->set_structured(s == 2);
    return capture_single(p);
  };
  if (tune_cache_read(sig, &ntw, &capx, &sched) && (sched == 0 || (sched == 1 && can_persist) ||
                                                    (sched == 2 && p->struct_ok))) {
    p->tune_cached = 1;
    return apply(sched);
  }
  const int n = 32;
  int rc = time_schedule(p, 0, n, &p->tune_graph_us);
  if (rc) return rc;
  if (can_persist) {
    rc = time_schedule(p, 1, n, &p->tune_persistent_us);
    if (rc) return rc;
  }
  if (p->struct_ok) {
    if ((rc = apply(2))) return rc;
    rc = time_schedule(p, 0, n, &p->tune_structured_us);
    if (rc) return rc;
  }
  int best = 0;
  double best_us = p->tune_graph_us;
  if (can_persist && p->tune_persistent_us < best_us) {
    best = 1;
    best_us = p->tune_persistent_us;
  }
  if (p->struct_ok && p->tune_structured_us < best_us) best = 2;
  if ((rc = apply(best))) return rc;
  int nu = 0;
  ntw = 1;
  capx = 8;
  if (p->beng) p->beng->variant(&ntw, &capx, &nu);
  tune_cache_write(sig, ntw, capx, best);
  return DLMPC_OK;
}

bool finite_all(const double *v, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

bool finite_all(const float *v, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

// The solve loop shared by the host- and device-buffer entry points. x0_dev, u0_dev on device.
int run_solve(dlmpc_problem *p, const double *x0_dev, const double *wpsi, const double *wlam,
              double *u0_dev, double *phi_dev, dlmpc_stats *stats, double t_host0_ms) {
  std::string err;
  const int max_iter = p->opt.max_iter;
  API_HIP(hipEventRecord(p->ev_p0, p->stream));
  int rc = p->eng->precompute(x0_dev, wpsi, wlam, max_iter, p->opt.eps, p->rho, err);
  if (rc) return fail(rc, err);
  API_HIP(hipEventRecord(p->ev_p1, p->stream));
  API_HIP(hipEventRecord(p->ev_t0, p->stream));
  int launched = 0, launches = 0;
  bool stopped = false;
  Ctl *d_ctl = p->eng->ctl();
  if (p->sched == 1) {
    rc = p->eng->run_persistent(false, err);
    if (rc) return fail(rc, err);
    launches = 1;
    stopped = true;
  }
  // Per-iteration schedules: the kernels of one iteration launched one by one and the stop flag
  // read after every iteration; 4 also copies Phi through host memory between Phi-comp and
  // Psi-comp (the row-to-column exchange on the host, the other steps combined on the device),
  // 5 copies each kernel's results through host memory before the next kernel runs.
  for (int it = 0; p->sched >= 3 && !stopped && it < max_iter; ++it) {
    for (int kk = 0; kk < 4; ++kk) {
      if ((rc = p->eng->launch_one(kk, err))) return fail(rc, err);
      if ((p->sched == 5 || (p->sched == 4 && kk == 0)) && (rc = p->eng->host_exchange(kk, p->h_xchg, err)))
        return fail(rc, err);
    }
    ++launches;
    API_HIP(hipMemcpyAsync(&p->h_ctl[1], d_ctl, sizeof(Ctl), hipMemcpyDeviceToHost, p->stream));
    API_HIP(hipEventRecord(p->ev_ctl[1], p->stream));
    API_HIP(hipEventSynchronize(p->ev_ctl[1]));
    stopped = p->h_ctl[1].stop != 0;
  }
  // Graph schedule: launch a chunk of iterations, read the control block, and size the next
  // chunk from the residual decay (ChunkPredictor), so that few launches land after the
  // device-side stop and few host checks are needed. With check_every > 0 the chunk is fixed.
  ChunkPredictor pred;
  int n = p->K;
  while (!stopped && p->sched == 0) {
    n = std::max(1, std::min(n, max_iter - launched));
    rc = launch_iterations(p, n);
    if (rc) return rc;
    launched += n;
    ++launches;
    API_HIP(hipMemcpyAsync(&p->h_ctl[1], d_ctl, sizeof(Ctl), hipMemcpyDeviceToHost, p->stream));
    API_HIP(hipEventRecord(p->ev_ctl[1], p->stream));
    API_HIP(hipEventSynchronize(p->ev_ctl[1]));
    const Ctl &c = p->h_ctl[1];
    if (c.stop) {
      stopped = true;
      break;
    }
    if (launched >= max_iter) break;
    if (p->opt.check_every > 0) continue;
    n = pred.next(c.iters, c.last_rp, c.last_rd, p->opt.eps);
  }
  if (!stopped) return fail(DLMPC_EDEVICE, "the iteration did not reach its stop condition");
  API_HIP(hipEventRecord(p->ev_t1, p->stream));
  rc = p->eng->output(u0_dev, err);
  if (rc) return fail(rc, err);
  if (phi_dev) {
    rc = p->eng->export_phi(phi_dev, err);
    if (rc) return fail(rc, err);
  }
  API_HIP(hipMemcpyAsync(&p->h_ctl[0], d_ctl, sizeof(Ctl), hipMemcpyDeviceToHost, p->stream));
  API_HIP(hipStreamSynchronize(p->stream));
  const Ctl &c = p->h_ctl[0];
  // FP64 certificate of the stopping iterate (synchronises)
  double cert[5] = {0, 0, 0, 0, 0};
  float mc = 0.f;
  if (!(p->opt.flags & DLMPC_FLAG_NO_CHECK) && !c.bar_fail) {
    API_HIP(hipEventRecord(p->ev_c0, p->stream));
    rc = p->eng->certify(x0_dev, cert, err);
    if (rc) return fail(rc, err);
    API_HIP(hipEventRecord(p->ev_c1, p->stream));
    API_HIP(hipEventSynchronize(p->ev_c1));
    (void)hipEventElapsedTime(&mc, p->ev_c0, p->ev_c1);
  }
  if (stats) {
    float ms = 0.f, mp = 0.f;
    (void)hipEventElapsedTime(&ms, p->ev_t0, p->ev_t1);
    (void)hipEventElapsedTime(&mp, p->ev_p0, p->ev_p1);
    stats->eq_resid = cert[0];
    stats->kkt = std::max(std::max(cert[2], cert[3]), std::max(cert[4], double(c.last_rd)));
    stats->u0_check = 0.0;
    stats->t_precompute_ms = mp;
    stats->t_check_ms = mc;
    stats->inner_iters = c.inner_iters;
    stats->coupling_viol = 0.0;
    if (!p->cp_a.empty()) {
      std::vector<double> y;
      if ((rc = p->eng->copy_y(y, err))) return fail(rc, err);
      for (size_t e = 0; e < p->cp_a.size(); ++e) {
        const double d = y[p->cp_a[e]] - y[p->cp_b[e]];
        stats->coupling_viol = std::max(stats->coupling_viol, std::max(p->cp_lo[e] - d, d - p->cp_hi[e]));
      }
    }
    stats->iters = c.iters;
    stats->converged = c.converged;
    stats->r_primal = c.last_rp;
    stats->r_dual = c.last_rd;
    stats->objective = c.objective;
    stats->t_iter_ms = ms;
    stats->graph_launches = launches;  // host checks (graph and per-iteration schedules) or 1 (persistent)
    stats->schedule = p->sched;
    stats->start = wpsi ? DLMPC_START_STATE : DLMPC_START_COLD;
    stats->fell_back = 0;
    stats->t_warm_ms = 0.0;
    const double t_now = std::chrono::duration<double, std::milli>(
                             std::chrono::steady_clock::now().time_since_epoch()).count();
    stats->t_solve_ms = t_now - t_host0_ms;
  }
  if (c.bar_fail) return fail(DLMPC_EDEVICE, "persistent grid barrier timed out");
  if (c.numeric) return fail(DLMPC_ENUMERIC, "NaN/Inf in the ADMM iterate");
  return c.converged ? DLMPC_OK : DLMPC_ENOCONV;
}

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// n initial states on the device (x0_dev [n][N*nx]) must be finite: DLMPC_EINVAL otherwise.
int check_x0_device(dlmpc_problem *p, const double *x0_dev, int64_t n) {
  std::string err;
  bool ok = false;
  const int rc = dlmpc::device_all_finite(x0_dev, n * p->hs.N * p->hs.nx, p->d_flag, p->h_flag, p->stream, &ok, err);
  if (rc) return fail(rc, err);
  return ok ? DLMPC_OK : fail(DLMPC_EINVAL, "x0 has a NaN/Inf entry");
}

}  // namespace

extern "C" {

const char *dlmpc_last_error(void) { return g_err.c_str(); }

const char *dlmpc_status_string(int s) {
  switch (s) {
    case DLMPC_OK: return "ok";
    case DLMPC_ENOCONV: return "not converged within max_iter";
    case DLMPC_EINVAL: return "invalid argument";
    case DLMPC_ENOMEM: return "out of memory";
    case DLMPC_EDEVICE: return "device error";
    case DLMPC_EINFEASIBLE_LOCALITY: return "locality constraint infeasible";
    case DLMPC_ENUMERIC: return "numerical breakdown (NaN/Inf)";
    default: return "unknown status";
  }
}

int dlmpc_setup(const dlmpc_system *sys, int32_t d, int32_t T, const dlmpc_cost *cost,
                const dlmpc_options *opts, dlmpc_problem **out) {
  if (!out) return fail(DLMPC_EINVAL, "out must be non-NULL");
  *out = nullptr;
  dlmpc_options o{};
  if (opts) o = *opts;
  if (o.rho == 0.0) o.rho = 5.0;
  if (o.eps == 0.0) o.eps = 1e-4;
  if (o.max_iter == 0) o.max_iter = 500;
  if (!(o.rho > 0.0) || !std::isfinite(o.rho) || !(o.eps > 0.0) || o.max_iter < 0 || o.check_every < 0)
    return fail(DLMPC_EINVAL, "options: need rho > 0, eps > 0, max_iter >= 0, check_every >= 0");
  if (o.precision != DLMPC_FP64 && o.precision != DLMPC_FP32 && o.precision != DLMPC_FP32_BF16)
    return fail(DLMPC_EINVAL, "unknown precision");
  if (o.max_batch < 0 || o.max_batch > 64) return fail(DLMPC_EINVAL, "max_batch must be in 0..64");
  {
    const uint32_t sf = o.flags & (DLMPC_FLAG_SCHED_GRAPH | DLMPC_FLAG_SCHED_PERSISTENT | DLMPC_FLAG_SCHED_STEPWISE |
                                   DLMPC_FLAG_SCHED_HOST_EXCHANGE | DLMPC_FLAG_SCHED_NAIVE);
    if (sf & (sf - 1)) return fail(DLMPC_EINVAL, "at most one DLMPC_FLAG_SCHED_* flag");
  }
  if (!(o.factor_chol_tol >= 0.0)) return fail(DLMPC_EINVAL, "factor_chol_tol must be >= 0");
  if (o.warm_eps_scale == 0.0) o.warm_eps_scale = 0.5;
  if (!(o.warm_eps_scale > 0.0 && o.warm_eps_scale <= 1.0))
    return fail(DLMPC_EINVAL, "warm_eps_scale must be in (0, 1]");
  auto p = std::make_unique<dlmpc_problem>();
  p->opt = o;
  p->warm_eps = o.eps * o.warm_eps_scale;
  p->rho = o.rho;
  p->host_only = (o.flags & DLMPC_FLAG_HOST_ONLY) != 0;
  std::string err;
  const auto t_setup = std::chrono::steady_clock::now();
  int rc = dlmpc::host_setup(sys, d, T, cost, p->hs, err);
  if (rc) return fail(rc, err);
  // The column blocks are factored by device kernels unless the problem is host-only or the
  // caller asks for the host factorisation.
  if (p->host_only || (o.flags & DLMPC_FLAG_HOST_FACTOR))
    rc = dlmpc::factor_host(p->hs, err);
  else
    rc = dlmpc::factor_device(p->hs, o.device, o.factor_chol_tol > 0.0 ? o.factor_chol_tol : 1e-10, err);
  if (rc) {
    dlmpc::free_factors_device(p->hs);
    return fail(rc, err);
  }
  p->hs.setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_setup).count();
  if (!p->host_only) {
    rc = setup_device(p.get());
    if (rc) {
      const std::string keep = g_err;
      release_device(p.get());
      return fail(rc, keep);
    }
  }
  *out = p.release();
  return DLMPC_OK;
}

int dlmpc_query(const dlmpc_problem *p, dlmpc_info *info) {
  if (!p || !info) return fail(DLMPC_EINVAL, "NULL argument");
  const HostSetup &h = p->hs;
  info->R = h.R;
  info->n_cols = int64_t(h.N) * h.nx;
  info->nnz = h.nnz;
  info->n_tiles = h.n_tiles;
  info->d_row_max = h.d_row_max;
  info->d_col_max = h.d_col_max;
  info->p_max = h.p_max;
  info->k_max = h.k_max;
  info->sum_dcol_k = h.sum_dcol_k;
  info->sum_k = h.sum_k;
  info->sum_dcol2 = h.sum_dcol2;
  info->setup_ms = h.setup_ms;
  info->factor_ms = h.factor_ms;
  info->factor_device = h.factor_where;
  info->factor_fallbacks = h.factor_fallbacks;
  info->schedule = p->sched;
  info->persistent_grid = (p->eng ? p->eng->persistent_grid() : 0);
  info->tune_graph_us = p->tune_graph_us;
  info->tune_persistent_us = p->tune_persistent_us;
  info->batch_phi_ntw = 0;
  info->batch_psi_capx = 0;
  info->batch_psi_units = 0;
  if (p->beng) p->beng->variant(&info->batch_phi_ntw, &info->batch_psi_capx, &info->batch_psi_units);
  for (int v = 0; v < 2; ++v) info->tune_phi_us[v] = p->tune_phi_us[v];
  for (int c = 0; c < 6; ++c) info->tune_psi_us[c] = p->tune_psi_us[c];
  info->tune_cached = p->tune_cached;
  info->psi_structured = p->psi_structured ? 1 : 0;
  info->tune_structured_us = p->tune_structured_us;
  info->sum_du_k = 0;
  for (int j = 0; j < h.N; ++j)
    info->sum_du_k += int64_t(h.patch[j].size()) * h.nu * (h.T - 1) * h.kdim[j];
  return DLMPC_OK;
}

int dlmpc_phi_pattern(const dlmpc_problem *p, int64_t *row_ptr, int32_t *col_idx) {
  if (!p || !row_ptr || !col_idx) return fail(DLMPC_EINVAL, "NULL argument");
  const HostSetup &h = p->hs;
  std::copy(h.csr_rowptr.begin(), h.csr_rowptr.end(), row_ptr);
  const int64_t Nx = int64_t(h.N) * h.nx, Nu = int64_t(h.N) * h.nu;
  for (int64_t r = 0; r < h.R; ++r) {
    const int32_t m = (r < Nx * h.T) ? int32_t((r % Nx) / h.nx) : int32_t(((r - Nx * h.T) % Nu) / h.nu);
    int64_t w = h.csr_rowptr[r];
    for (int32_t j : h.patch[m])
      for (int c = 0; c < h.nx; ++c) col_idx[w++] = j * h.nx + c;
  }
  return DLMPC_OK;
}

int dlmpc_column_block(const dlmpc_problem *p, int32_t j, int32_t *D_out, int64_t *rows, double *P,
                       double *O) {
  if (!p || j < 0 || j >= p->hs.N) return fail(DLMPC_EINVAL, "bad problem or subsystem index");
  const HostSetup &h = p->hs;
  const int32_t np = int32_t(h.patch[j].size());
  const int32_t D = np * h.rs;
  if (D_out) *D_out = D;
  if (rows)
    for (int a = 0; a < np; ++a)
      for (int l = 0; l < h.rs; ++l) rows[a * h.rs + l] = dlmpc::canon_row(h, h.patch[j][a], l);
  const int k = h.kdim[j];
  const int ld = dlmpc::padded_ld(D);
  std::vector<double> nbj;
  if (P) {
    std::string err;
    const int rc = dlmpc::fetch_basis(h, j, nbj, err);
    if (rc) return fail(rc, err);
  }
  const double *Nj = nbj.data();
  if (P)
    for (int r = 0; r < D; ++r)
      for (int c = 0; c < D; ++c) {
        double s = 0.0;
        for (int i = 0; i < k; ++i) s += Nj[size_t(i) * ld + r] * Nj[size_t(i) * ld + c];
        P[size_t(r) * D + c] = s;
      }
  if (O) {
    const double *Oj = h.off.data() + h.off_ptr[j];
    for (int r = 0; r < D; ++r)
      for (int c = 0; c < h.nx; ++c) O[size_t(r) * h.nx + c] = Oj[size_t(c) * ld + r];
  }
  return DLMPC_OK;
}

int dlmpc_solve(dlmpc_problem *p, const double *x0, const dlmpc_warm *warm, double *u0, double *phi,
                dlmpc_stats *stats) {
  const double t0 = now_ms();
  if (!p || !x0) return fail(DLMPC_EINVAL, "NULL argument");
  if (p->host_only) return fail(DLMPC_EDEVICE, "problem was set up host-only");
  const HostSetup &h = p->hs;
  const size_t nxs = size_t(h.N) * h.nx;
  if (!finite_all(x0, nxs)) return fail(DLMPC_EINVAL, "x0 has a NaN/Inf entry");
  const bool use_warm = warm && warm->psi0 && warm->lambda0;
  if (warm && (!warm->psi0) != (!warm->lambda0)) return fail(DLMPC_EINVAL, "warm start needs both psi0 and lambda0");
  if (use_warm && (!finite_all(warm->psi0, size_t(h.nnz)) || !finite_all(warm->lambda0, size_t(h.nnz))))
    return fail(DLMPC_EINVAL, "warm start has a NaN/Inf entry");
  API_HIP(hipSetDevice(p->opt.device));
  API_HIP(hipMemcpyAsync(p->d_x0, x0, nxs * sizeof(double), hipMemcpyHostToDevice, p->stream));
  const double *wpsi = nullptr, *wlam = nullptr;
  if (use_warm) {
    API_HIP(hipMemcpyAsync(p->d_warm, warm->psi0, size_t(h.nnz) * sizeof(double), hipMemcpyHostToDevice, p->stream));
    API_HIP(hipMemcpyAsync(p->d_warm + h.nnz, warm->lambda0, size_t(h.nnz) * sizeof(double),
                           hipMemcpyHostToDevice, p->stream));
    wpsi = p->d_warm;
    wlam = p->d_warm + h.nnz;
  }
  const int rc = run_solve(p, p->d_x0, wpsi, wlam, p->d_u0, phi ? p->d_phi : nullptr, stats, t0);
  if (rc < 0) return rc;
  if (u0) API_HIP(hipMemcpy(u0, p->d_u0, size_t(h.N) * h.nu * sizeof(double), hipMemcpyDeviceToHost));
  if (phi) API_HIP(hipMemcpy(phi, p->d_phi, size_t(h.nnz) * sizeof(double), hipMemcpyDeviceToHost));
  if (stats) stats->t_solve_ms = now_ms() - t0;
  return rc;
}

int dlmpc_solve_device(dlmpc_problem *p, const double *x0_dev, double *u0_dev, double *phi_dev,
                       dlmpc_stats *stats) {
  const double t0 = now_ms();
  if (!p || !x0_dev || !u0_dev) return fail(DLMPC_EINVAL, "NULL argument");
  if (p->host_only) return fail(DLMPC_EDEVICE, "problem was set up host-only");
  API_HIP(hipSetDevice(p->opt.device));
  int rc = check_x0_device(p, x0_dev, 1);
  if (rc) return rc;
  return run_solve(p, x0_dev, nullptr, nullptr, u0_dev, phi_dev, stats, t0);
}

int dlmpc_certify(dlmpc_problem *p, const double *x0_dev, dlmpc_cert *out) {
  if (!p || !out) return fail(DLMPC_EINVAL, "NULL argument");
  if (p->host_only) return fail(DLMPC_EDEVICE, "problem was set up host-only");
  API_HIP(hipSetDevice(p->opt.device));
  std::string err;
  double v[5];
  const int rc = p->eng->certify(x0_dev ? x0_dev : p->d_x0, v, err);
  if (rc) return fail(rc, err);
  out->eq = v[0];
  out->pf = v[1];
  out->rp = v[2];
  out->box = v[3];
  out->stat = v[4];
  return DLMPC_OK;
}

int dlmpc_time_kernels(dlmpc_problem *p, const double *x0_dev, int32_t iters, double *us_per_launch) {
  if (!p || !x0_dev || iters < 1 || !us_per_launch) return fail(DLMPC_EINVAL, "bad argument");
  if (p->host_only) return fail(DLMPC_EDEVICE, "problem was set up host-only");
  API_HIP(hipSetDevice(p->opt.device));
  std::string err;
  int rc = p->eng->precompute(x0_dev, nullptr, nullptr, iters, -1.0, p->rho, err);
  if (rc) return fail(rc, err);
  constexpr int nk = DLMPC_TIMED_KERNELS;
  std::vector<hipEvent_t> ev(size_t(nk) * iters + 1);
  for (auto &e : ev) API_HIP(hipEventCreate(&e));
  API_HIP(hipEventRecord(ev[0], p->stream));
  for (int i = 0; i < iters && rc == DLMPC_OK; ++i)
    for (int k = 0; k < nk && rc == DLMPC_OK; ++k) {
      rc = p->eng->launch_one(k, err);
      if (!rc) API_HIP(hipEventRecord(ev[size_t(i) * nk + k + 1], p->stream));
    }
  API_HIP(hipStreamSynchronize(p->stream));
  double sum[nk] = {};
  for (int i = 0; i < iters && rc == DLMPC_OK; ++i)
    for (int k = 0; k < nk; ++k) {
      float ms = 0.f;
      API_HIP(hipEventElapsedTime(&ms, ev[size_t(i) * nk + k], ev[size_t(i) * nk + k + 1]));
      sum[k] += ms;
    }
  for (auto &e : ev) (void)hipEventDestroy(e);
  if (rc) return fail(rc, err);
  for (int k = 0; k < nk; ++k) us_per_launch[k] = 1e3 * sum[k] / iters;
  return DLMPC_OK;
}

int dlmpc_time_batch_kernels(dlmpc_problem *p, int32_t B, const double *x0_dev, int32_t iters,
                             double *us_per_launch) {
  if (!p || !x0_dev || iters < 1 || !us_per_launch) return fail(DLMPC_EINVAL, "bad argument");
  if (p->host_only) return fail(DLMPC_EDEVICE, "problem was set up host-only");
  if (!p->beng) return fail(DLMPC_EINVAL, "problem was set up without max_batch");
  if (B < 1 || B > p->beng->bmax()) return fail(DLMPC_EINVAL, "batch size out of range");
  API_HIP(hipSetDevice(p->opt.device));
  std::string err;
  // Warm start from alpha0 = 0 (every iteration then runs the full products, unlike the
  // first two of the cold start) and no stop (eps < 0).
  const size_t nrow = size_t(B) * p->hs.N * p->hs.rs;
  double *zero = nullptr;
  API_HIP(hipMalloc(&zero, sizeof(double) * nrow));
  int rc = hipMemsetAsync(zero, 0, sizeof(double) * nrow, p->stream) == hipSuccess ? DLMPC_OK : DLMPC_EDEVICE;
  if (!rc) rc = p->beng->precompute(x0_dev, B, iters, -1.0, 1, nullptr, err);
  if (!rc) rc = p->beng->start_alpha(zero, err);
  const bool dev_ok = hipStreamSynchronize(p->stream) == hipSuccess;
  (void)hipFree(zero);
  if (!dev_ok) return fail(DLMPC_EDEVICE, "device error while preparing the timing run");
  if (rc) return fail(rc, err.empty() ? std::string("hipMemsetAsync failed") : err);
  constexpr int nk = DLMPC_BATCH_TIMED_KERNELS;
  std::vector<hipEvent_t> ev(size_t(nk) * iters + 1);
  for (auto &e : ev) API_HIP(hipEventCreate(&e));
  API_HIP(hipEventRecord(ev[0], p->stream));
  for (int i = 0; i < iters && rc == DLMPC_OK; ++i)
    for (int k = 0; k < nk && rc == DLMPC_OK; ++k) {
      rc = p->beng->launch_one(k, err);
      if (!rc) API_HIP(hipEventRecord(ev[size_t(i) * nk + k + 1], p->stream));
    }
  API_HIP(hipStreamSynchronize(p->stream));
  double sum[nk] = {};
  for (int i = 0; i < iters && rc == DLMPC_OK; ++i)
    for (int k = 0; k < nk; ++k) {
      float ms = 0.f;
      API_HIP(hipEventElapsedTime(&ms, ev[size_t(i) * nk + k], ev[size_t(i) * nk + k + 1]));
      sum[k] += ms;
    }
  for (auto &e : ev) (void)hipEventDestroy(e);
  if (rc) return fail(rc, err);
  for (int k = 0; k < nk; ++k) us_per_launch[k] = 1e3 * sum[k] / iters;
  return DLMPC_OK;
}

namespace {

// One batched run from the given start. Per-instance control blocks land in p->h_bctl;
// y_out_dev / alpha_out_dev (or NULL) get the stopping trajectories and multipliers.
// *t_warm_ms is the device time of the start construction. Returns DLMPC_OK or a negative
// status (per-instance outcomes are left to the caller).
// Device times of a batched run (ms): iteration phase, start construction, precompute, FP64 check.
struct RunTimes {
  float iter = 0.f, warm = 0.f, pre = 0.f, check = 0.f;
};

int run_batch_once(dlmpc_problem *p, int B, const double *x0_dev, int start, const double *start_dev,
                   double *u0_dev, double *y_out_dev, double *alpha_out_dev, RunTimes *times, int *checks_out,
                   const double *rscale_dev = nullptr) {
  std::string err;
  const int max_iter = p->opt.max_iter;
  const HostSetup &h = p->hs;
  const double eps = start != DLMPC_START_COLD ? p->warm_eps : p->opt.eps;
  API_HIP(hipEventRecord(p->ev_p0, p->stream));
  int rc = p->beng->precompute(x0_dev, B, max_iter, eps, start != DLMPC_START_COLD ? 1 : 0, rscale_dev, err);
  if (rc) return fail(rc, err);
  API_HIP(hipEventRecord(p->ev_p1, p->stream));
  API_HIP(hipEventRecord(p->ev_w0, p->stream));
  if (start == DLMPC_START_ALPHA) {
    rc = p->beng->start_alpha(start_dev, err);
  } else if (start == DLMPC_START_TRAJECTORY) {
    rc = p->beng->start_trajectory(start_dev, p->cg_iters, err);
  } else if (start == DLMPC_START_LEARNED) {
    const size_t nxs = size_t(h.N) * h.nx, R = size_t(h.N) * h.rs;
    for (int s0 = 0; s0 < B && !rc; s0 += p->ws->Smax) {
      const int S = std::min(p->ws->Smax, B - s0);
      rc = p->ws->predict(S, x0_dev + s0 * nxs, p->beng->yhat() + s0 * R, err);
    }
    if (!rc) rc = p->beng->start_trajectory(nullptr, p->cg_iters, err);
  }
  if (rc) return fail(rc, err);
  API_HIP(hipEventRecord(p->ev_w1, p->stream));
  API_HIP(hipEventRecord(p->ev_t0, p->stream));
  Ctl *d_ctl = p->beng->ctl();
  ChunkPredictor pred;
  int launched = 0, checks = 0, n = p->K;
  bool stopped = false;
  while (!stopped) {
    n = std::max(1, std::min(n, max_iter - launched));
    rc = launch_graphs(p->bgexec, p->stream, n);
    if (rc) return rc;
    launched += n;
    ++checks;
    API_HIP(hipMemcpyAsync(&p->h_ctl[1], d_ctl, sizeof(Ctl), hipMemcpyDeviceToHost, p->stream));
    API_HIP(hipEventRecord(p->ev_ctl[1], p->stream));
    API_HIP(hipEventSynchronize(p->ev_ctl[1]));
    const Ctl &c = p->h_ctl[1];
    if (c.stop) {
      stopped = true;
      break;
    }
    if (launched >= max_iter) break;
    n = p->opt.check_every > 0 ? p->K : pred.next(c.iters, c.last_rp, c.last_rd, eps);
  }
  if (!stopped) return fail(DLMPC_EDEVICE, "batched iteration did not reach its stop condition");
  API_HIP(hipEventRecord(p->ev_t1, p->stream));
  rc = p->beng->output(u0_dev, err);
  if (!rc && alpha_out_dev) rc = p->beng->export_alpha(alpha_out_dev, err);
  if (!rc && y_out_dev) rc = p->beng->export_y(y_out_dev, err);
  if (rc) return fail(rc, err);
  const bool check = !(p->opt.flags & DLMPC_FLAG_NO_CHECK);
  API_HIP(hipEventRecord(p->ev_c0, p->stream));
  if (check && (rc = p->beng->check(x0_dev, err))) return fail(rc, err);
  API_HIP(hipEventRecord(p->ev_c1, p->stream));
  API_HIP(hipMemcpyAsync(p->h_bctl, p->beng->ictl(), sizeof(dlmpc::BCtl) * B, hipMemcpyDeviceToHost, p->stream));
  API_HIP(hipStreamSynchronize(p->stream));
  float ms = 0.f, mw = 0.f, mp = 0.f, mc = 0.f;
  (void)hipEventElapsedTime(&ms, p->ev_t0, p->ev_t1);
  (void)hipEventElapsedTime(&mw, p->ev_w0, p->ev_w1);
  (void)hipEventElapsedTime(&mp, p->ev_p0, p->ev_p1);
  (void)hipEventElapsedTime(&mc, p->ev_c0, p->ev_c1);
  times->iter = ms;
  times->warm = start == DLMPC_START_COLD ? 0.f : mw;
  times->pre = mp;
  times->check = check ? mc : 0.f;
  *checks_out = checks;
  return DLMPC_OK;
}

// A warm-started instance is kept when it met eps * warm_eps_scale, or when it ran out of
// iterations but its last iterate meets the unscaled eps (the cold start's own rule; it is then
// marked converged); otherwise it is solved again from the cold start.
bool warm_accept(const dlmpc_problem *p, dlmpc::BCtl &ic) {
  if (ic.numeric) return false;
  if (ic.converged) return true;
  if (ic.last_rp <= p->opt.eps && ic.last_rd <= p->opt.eps) {
    ic.converged = 1;
    return true;
  }
  return false;
}

void fill_stats(dlmpc_stats &st, const dlmpc::BCtl &ic, float ms, int checks, int start, double t0) {
  st.eq_resid = ic.eq_resid;
  st.u0_check = ic.u0dev;
  st.kkt = std::max(std::max(ic.eq_resid, ic.box), std::max(ic.last_rp, ic.last_rd));
  st.iters = ic.iters;
  st.converged = ic.converged;
  st.r_primal = ic.last_rp;
  st.r_dual = ic.last_rd;
  st.objective = ic.objective;
  st.t_iter_ms = ms;
  st.graph_launches = checks;
  st.schedule = 2;
  st.start = start;
  st.fell_back = 0;
  st.t_warm_ms = 0.0;
  st.t_solve_ms = now_ms() - t0;
}

// Batched solve with the given start; warm-started instances that end unconverged (or with a
// NaN/Inf) are solved again from the cold start in one more batched run. rscale_dev [B] (or
// NULL): per-instance factors of the penalty rho.
int run_batch(dlmpc_problem *p, int B, const double *x0_dev, double *u0_dev, int start, const double *start_dev,
              double *y_out_dev, double *alpha_out_dev, dlmpc_stats *stats, double t0,
              const double *rscale_dev = nullptr) {
  const HostSetup &h = p->hs;
  const size_t nxs = size_t(h.N) * h.nx, nus = size_t(h.N) * h.nu, R = size_t(h.N) * h.rs;
  RunTimes tm;
  int checks = 0;
  int rc = run_batch_once(p, B, x0_dev, start, start_dev, u0_dev, y_out_dev, alpha_out_dev, &tm, &checks,
                          rscale_dev);
  if (rc) return rc;
  const float ms = tm.iter, mw = tm.warm;
  std::vector<dlmpc::BCtl> first(p->h_bctl, p->h_bctl + B);
  std::vector<int> redo;
  if (start != DLMPC_START_COLD)
    for (int b = 0; b < B; ++b)
      if (!warm_accept(p, first[b])) redo.push_back(b);
  for (int b = 0; b < B; ++b)
    if (stats) fill_stats(stats[b], first[b], ms, checks, start, t0);
  if (!redo.empty()) {
    const int F = int(redo.size());
    for (int f = 0; f < F; ++f) {
      API_HIP(hipMemcpyAsync(p->d_fx0 + f * nxs, x0_dev + redo[f] * nxs, nxs * sizeof(double),
                             hipMemcpyDeviceToDevice, p->stream));
      if (rscale_dev)
        API_HIP(hipMemcpyAsync(p->d_frs + f, rscale_dev + redo[f], sizeof(double), hipMemcpyDeviceToDevice,
                               p->stream));
    }
    RunTimes tm2;
    int checks2 = 0;
    rc = run_batch_once(p, F, p->d_fx0, DLMPC_START_COLD, nullptr, p->d_fu0, y_out_dev ? p->d_fy : nullptr,
                        alpha_out_dev ? p->d_falpha : nullptr, &tm2, &checks2, rscale_dev ? p->d_frs : nullptr);
    if (rc) return rc;
    const float ms2 = tm2.iter;
    tm.pre += tm2.pre;
    tm.check += tm2.check;
    for (int f = 0; f < F; ++f) {
      const int b = redo[f];
      API_HIP(hipMemcpyAsync(u0_dev + b * nus, p->d_fu0 + f * nus, nus * sizeof(double), hipMemcpyDeviceToDevice,
                             p->stream));
      if (y_out_dev)
        API_HIP(hipMemcpyAsync(y_out_dev + b * R, p->d_fy + f * R, R * sizeof(double), hipMemcpyDeviceToDevice,
                               p->stream));
      if (alpha_out_dev)
        API_HIP(hipMemcpyAsync(alpha_out_dev + b * R, p->d_falpha + f * R, R * sizeof(double),
                               hipMemcpyDeviceToDevice, p->stream));
      dlmpc::BCtl ic = p->h_bctl[f];
      ic.iters += first[b].iters;
      first[b] = ic;
      if (stats) {
        fill_stats(stats[b], ic, ms + ms2, checks + checks2, start, t0);
        stats[b].fell_back = 1;
      }
    }
    API_HIP(hipStreamSynchronize(p->stream));
  }
  bool all = true, numeric = false;
  for (int b = 0; b < B; ++b) {
    all = all && first[b].converged;
    numeric = numeric || first[b].numeric;
    if (stats) {
      stats[b].t_warm_ms = mw;
      stats[b].t_precompute_ms = tm.pre;
      stats[b].t_check_ms = tm.check;
      stats[b].t_solve_ms = now_ms() - t0;
    }
  }
  if (numeric) return fail(DLMPC_ENUMERIC, "NaN/Inf in a batched ADMM iterate");
  return all ? DLMPC_OK : DLMPC_ENOCONV;
}

int check_batch(dlmpc_problem *p, int32_t B) {
  if (!p) return fail(DLMPC_EINVAL, "NULL problem");
  if (p->host_only) return fail(DLMPC_EDEVICE, "problem was set up host-only");
  if (!p->beng) return fail(DLMPC_EINVAL, "problem was set up without max_batch");
  if (!p->cp_a.empty()) return fail(DLMPC_EINVAL, "couplings are set: only single-instance solves take them");
  if (B < 1 || B > p->beng->bmax()) return fail(DLMPC_EINVAL, "batch size out of range");
  return DLMPC_OK;
}

}  // namespace

int dlmpc_solve_batch(dlmpc_problem *p, int32_t B, const double *x0, double *u0, dlmpc_stats *stats) {
  const double t0 = now_ms();
  int rc = check_batch(p, B);
  if (rc) return rc;
  if (!x0) return fail(DLMPC_EINVAL, "NULL x0");
  const HostSetup &h = p->hs;
  const size_t nxs = size_t(B) * h.N * h.nx;
  if (!finite_all(x0, nxs)) return fail(DLMPC_EINVAL, "x0 has a NaN/Inf entry");
  API_HIP(hipSetDevice(p->opt.device));
  API_HIP(hipMemcpyAsync(p->d_bx0, x0, nxs * sizeof(double), hipMemcpyHostToDevice, p->stream));
  rc = run_batch(p, B, p->d_bx0, p->d_bu0, DLMPC_START_COLD, nullptr, nullptr, nullptr, stats, t0);
  if (rc < 0) return rc;
  if (u0) API_HIP(hipMemcpy(u0, p->d_bu0, size_t(B) * h.N * h.nu * sizeof(double), hipMemcpyDeviceToHost));
  return rc;
}

int dlmpc_solve_batch_device(dlmpc_problem *p, int32_t B, const double *x0_dev, double *u0_dev,
                             dlmpc_stats *stats) {
  const double t0 = now_ms();
  int rc = check_batch(p, B);
  if (rc) return rc;
  if (!x0_dev || !u0_dev) return fail(DLMPC_EINVAL, "NULL argument");
  API_HIP(hipSetDevice(p->opt.device));
  if ((rc = check_x0_device(p, x0_dev, B))) return rc;
  return run_batch(p, B, x0_dev, u0_dev, DLMPC_START_COLD, nullptr, nullptr, nullptr, stats, t0);
}

int dlmpc_solve_batch_ex(dlmpc_problem *p, int32_t B, const double *x0_dev, double *u0_dev, int32_t start,
                         const double *start_dev, double *y_out_dev, double *alpha_out_dev, dlmpc_stats *stats) {
  const double t0 = now_ms();
  int rc = check_batch(p, B);
  if (rc) return rc;
  if (!x0_dev || !u0_dev) return fail(DLMPC_EINVAL, "NULL argument");
  if (start != DLMPC_START_COLD && start != DLMPC_START_ALPHA && start != DLMPC_START_TRAJECTORY &&
      start != DLMPC_START_LEARNED)
    return fail(DLMPC_EINVAL, "unknown start mode");
  if ((start == DLMPC_START_ALPHA || start == DLMPC_START_TRAJECTORY) && !start_dev)
    return fail(DLMPC_EINVAL, "this start mode needs start_dev");
  if (start == DLMPC_START_LEARNED && !p->ws)
    return fail(DLMPC_EINVAL, "no warm-start network (dlmpc_ws_init or dlmpc_warmstart_load)");
  API_HIP(hipSetDevice(p->opt.device));
  if ((rc = check_x0_device(p, x0_dev, B))) return rc;
  return run_batch(p, B, x0_dev, u0_dev, start, start_dev, y_out_dev, alpha_out_dev, stats, t0);
}

namespace {

int check_stream_args(dlmpc_problem *p, int32_t n, const double *x0_dev, double *u0_dev, int32_t refill_min,
                      int32_t check_iters) {
  int rc = check_batch(p, 1);
  if (rc) return rc;
  if (!x0_dev || !u0_dev || n < 1) return fail(DLMPC_EINVAL, "need n >= 1 and non-NULL x0_dev, u0_dev");
  if (!p->ws) return fail(DLMPC_EINVAL, "no warm-start network (dlmpc_ws_init or dlmpc_warmstart_load)");
  if (check_iters < 0 || refill_min < 0) return fail(DLMPC_EINVAL, "refill_min and check_iters must be >= 0");
  return DLMPC_OK;
}

// The streamed solve; sy: staging of the joiners' predicted trajectories, max_batch * N * rs
// floats on the problem's device (the caller checked the arguments and made the device current).
int run_stream(dlmpc_problem *p, int32_t n, const double *x0_dev, double *u0_dev, int32_t refill_min,
               int32_t check_iters, dlmpc_stats *stats, dlmpc_stream_info *info, float *sy, double t0) {
  int rc = check_x0_device(p, x0_dev, n);
  if (rc) return rc;
  const bool check = !(p->opt.flags & DLMPC_FLAG_NO_CHECK);
  double t_check = 0.0, t_pre = 0.0;  // device ms over the whole stream
  const HostSetup &h = p->hs;
  const size_t nxs = size_t(h.N) * h.nx, nus = size_t(h.N) * h.nu, R = size_t(h.N) * h.rs;
  const int Bm = p->beng->bmax(), Bs = std::min<int>(Bm, n);
  if (refill_min == 0) refill_min = std::max(1, Bs / 10);
  refill_min = std::min(refill_min, Bs);
  // Every check leaves the device idle for one host round trip (stop flags read, u(0) of the
  // stopped instances written, their state stashed, joiners started), and a stopped slot idles
  // until the check that sees it: on the 1024 mesh with 64 slots, 12 iterations between checks
  // and refills at 6 free slots measured fastest among 6..16 and 2..8 (the iterates do not
  // depend on it).
  const int K = check_iters > 0 ? check_iters : 12;
  std::string err;
  std::vector<int32_t> inst(Bs, -1);  // instance in each slot (-1: free)
  std::vector<dlmpc::BCtl> fin(n);     // final control block of every instance
  std::vector<double> t_lat(n, 0.0);   // host time of the join, then latency join -> stop seen
  // Stopped instances awaiting their FP64 check: their stopping state is copied into the
  // engine's stash (stash slot c holds instance pend_i[c]) and their slots are refilled at once;
  // the check runs once the stash is full and at the end, many instances per pass over the
  // FP64 bases. stash_t: a stash copy whose device time has not been read yet.
  std::vector<int32_t> pend_i;
  bool stash_t = false;
  auto read_stash_time = [&]() {
    if (!stash_t) return;
    float mc = 0.f;
    (void)hipEventElapsedTime(&mc, p->ev_p0, p->ev_p1);
    t_check += mc;
    stash_t = false;
  };
  auto run_pending_checks = [&]() -> int {
    const int S = int(pend_i.size());
    API_HIP(hipEventRecord(p->ev_c0, p->stream));
    const int r = p->beng->check_stash(x0_dev, pend_i.data(), S, err);
    if (r) return fail(r, err);
    API_HIP(hipEventRecord(p->ev_c1, p->stream));
    API_HIP(hipMemcpyAsync(p->h_bctl, p->beng->stash_ictl(), sizeof(dlmpc::BCtl) * S, hipMemcpyDeviceToHost,
                           p->stream));
    API_HIP(hipStreamSynchronize(p->stream));
    read_stash_time();
    float mc = 0.f;
    (void)hipEventElapsedTime(&mc, p->ev_c0, p->ev_c1);
    t_check += mc;
    for (int c = 0; c < S; ++c) fin[pend_i[c]] = p->h_bctl[c];
    pend_i.clear();
    return DLMPC_OK;
  };
  int next = 0, active = 0, joins = 0, checks = 0;
  int64_t slot_iters = 0;  // slot-iterations launched (active or idle)
  // Iterations that may still hold a CG step of the latest joiners (phases 1..cg_k fall in the
  // 2nd..(cg_k+1)-th iteration after a join): those run the graphs with the CG kernels, the
  // others the plain iteration graphs.
  int cg_left = 0;
  // New instances next.. into the given slots: network inference, then the trajectory start.
  auto join = [&](std::vector<int32_t> slots, bool first) -> int {
    const int S = int(slots.size());
    std::vector<int32_t> xsrc(S);
    for (int i = 0; i < S; ++i) xsrc[i] = next + i;
    for (int s0 = 0; s0 < S; s0 += p->ws->Smax) {
      const int c = std::min(p->ws->Smax, S - s0);
      const int r = p->ws->predict(c, x0_dev + size_t(next + s0) * nxs, sy + size_t(s0) * R, err);
      if (r) return fail(r, err);
    }
    const int r = p->beng->stream_start(x0_dev, slots.data(), xsrc.data(), S, sy, p->cg_iters, first,
                                        p->opt.max_iter, p->warm_eps, err);
    if (r) return fail(r, err);
    const double tj = now_ms();
    for (int i = 0; i < S; ++i) {
      inst[slots[i]] = next + i;
      t_lat[next + i] = tj;
    }
    next += S;
    active += S;
    ++joins;
    cg_left = p->cg_iters + 2;
    return DLMPC_OK;
  };
  {
    std::vector<int32_t> s0(Bs);
    for (int b = 0; b < Bs; ++b) s0[b] = b;
    if ((rc = join(s0, true))) return rc;
  }
  API_HIP(hipEventRecord(p->ev_t0, p->stream));
  Ctl *d_ctl = p->beng->ctl();
  // Bound on the loop: every join brings at least one instance, and every instance stops
  // within max_iter iterations of its join.
  const int64_t guard = (int64_t(n) + 1) * (p->opt.max_iter + K);
  int64_t launched = 0;
  while (active > 0) {
    const int kc = std::min(K, cg_left);
    if ((rc = launch_graphs(p->sgexec, p->stream, kc)) || (rc = launch_graphs(p->bgexec, p->stream, K - kc))) return rc;
    cg_left -= kc;
    launched += K;
    slot_iters += int64_t(K) * Bs;
    ++checks;
    API_HIP(hipMemcpyAsync(&p->h_ctl[1], d_ctl, sizeof(Ctl), hipMemcpyDeviceToHost, p->stream));
    API_HIP(hipMemcpyAsync(p->h_bctl, p->beng->ictl(), sizeof(dlmpc::BCtl) * Bs, hipMemcpyDeviceToHost, p->stream));
    API_HIP(hipStreamSynchronize(p->stream));
    read_stash_time();
    std::vector<int32_t> done_s, done_i, free_s;
    for (int b = 0; b < Bs; ++b) {
      if (inst[b] >= 0 && p->h_bctl[b].stop) {
        done_s.push_back(b);
        done_i.push_back(inst[b]);
      }
    }
    if (!done_s.empty()) {
      if ((rc = p->beng->output_slots(u0_dev, done_s.data(), done_i.data(), int(done_s.size()), err)))
        return fail(rc, err);
      API_HIP(hipMemcpyAsync(p->h_bctl, p->beng->ictl(), sizeof(dlmpc::BCtl) * Bs, hipMemcpyDeviceToHost, p->stream));
      API_HIP(hipStreamSynchronize(p->stream));
      for (size_t q = 0; q < done_s.size(); ++q) {
        fin[done_i[q]] = p->h_bctl[done_s[q]];
        t_lat[done_i[q]] = now_ms() - t_lat[done_i[q]];
        inst[done_s[q]] = -1;
      }
      active -= int(done_s.size());
      if (check) {
        if (pend_i.size() + done_s.size() > size_t(Bm) && (rc = run_pending_checks())) return rc;
        std::vector<int32_t> to(done_s.size());
        for (size_t q = 0; q < done_s.size(); ++q) to[q] = int32_t(pend_i.size() + q);
        API_HIP(hipEventRecord(p->ev_p0, p->stream));
        if ((rc = p->beng->stash_slots(done_s.data(), to.data(), int(done_s.size()), err))) return fail(rc, err);
        API_HIP(hipEventRecord(p->ev_p1, p->stream));
        stash_t = true;
        pend_i.insert(pend_i.end(), done_i.begin(), done_i.end());
      }
    }
    for (int b = 0; b < Bs; ++b)
      if (inst[b] < 0) free_s.push_back(b);
    const int want = std::min<int>(int(free_s.size()), n - next);
    const bool refill = want > 0 && (int(free_s.size()) >= refill_min || active == 0 || next + want == n);
    if (refill) {
      free_s.resize(want);
      if ((rc = join(free_s, false))) return rc;
    }
    if (launched > guard) return fail(DLMPC_EDEVICE, "streamed solve did not drain");
  }
  if (!pend_i.empty() && (rc = run_pending_checks())) return rc;
  API_HIP(hipEventRecord(p->ev_t1, p->stream));
  API_HIP(hipStreamSynchronize(p->stream));
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, p->ev_t0, p->ev_t1);
  // Instances the warm start left unconverged (or with a NaN/Inf): cold batched solves.
  std::vector<int> redo;
  for (int i = 0; i < n; ++i)
    if (!warm_accept(p, fin[i])) redo.push_back(i);
  for (int i = 0; i < n; ++i)
    if (stats) {
      fill_stats(stats[i], fin[i], ms, checks, DLMPC_START_LEARNED, t0);
      stats[i].t_solve_ms = t_lat[i];
    }
  for (size_t r0 = 0; r0 < redo.size(); r0 += size_t(Bm)) {
    const int F = int(std::min(redo.size() - r0, size_t(Bm)));
    for (int f = 0; f < F; ++f)
      API_HIP(hipMemcpyAsync(p->d_fx0 + f * nxs, x0_dev + size_t(redo[r0 + f]) * nxs, nxs * sizeof(double),
                             hipMemcpyDeviceToDevice, p->stream));
    RunTimes tm2;
    int checks2 = 0;
    const double tf = now_ms();
    rc = run_batch_once(p, F, p->d_fx0, DLMPC_START_COLD, nullptr, p->d_fu0, nullptr, nullptr, &tm2, &checks2);
    if (rc) return rc;
    const double t_redo = now_ms() - tf;
    const float ms2 = tm2.iter;
    t_check += tm2.check;
    t_pre += tm2.pre;
    for (int f = 0; f < F; ++f) {
      const int i = redo[r0 + f];
      API_HIP(hipMemcpyAsync(u0_dev + size_t(i) * nus, p->d_fu0 + f * nus, nus * sizeof(double),
                             hipMemcpyDeviceToDevice, p->stream));
      dlmpc::BCtl ic = p->h_bctl[f];
      ic.iters += fin[i].iters;
      fin[i] = ic;
      if (stats) {
        fill_stats(stats[i], ic, ms + ms2, checks + checks2, DLMPC_START_LEARNED, t0);
        stats[i].fell_back = 1;
        stats[i].t_solve_ms = t_lat[i] + t_redo;
      }
    }
  }
  API_HIP(hipStreamSynchronize(p->stream));
  if (info) {
    info->joins = joins;
    info->checks = checks;
    info->slot_iterations = slot_iters;
    int64_t used = 0;
    for (int i = 0; i < n; ++i) used += fin[i].iters;
    info->instance_iterations = used;
    info->fell_back = int32_t(redo.size());
    info->t_stream_ms = ms;
  }
  int conv = 0;
  bool numeric = false;
  for (int i = 0; i < n; ++i) {
    conv += fin[i].converged;
    numeric = numeric || fin[i].numeric;
    if (stats) {
      stats[i].t_check_ms = t_check / n;
      stats[i].t_precompute_ms = t_pre / n;
    }
  }
  if (numeric) return fail(DLMPC_ENUMERIC, "NaN/Inf in a streamed ADMM iterate (also after the cold fallback)");
  return conv == n ? DLMPC_OK : DLMPC_ENOCONV;
}

}  // namespace

int dlmpc_closed_loop(dlmpc_problem *p, int32_t B, int32_t T_sim, const double *x0_dev, double *xs_dev,
                      double *us_dev, int32_t mode, dlmpc_stats *stats) {
  int rc = check_batch(p, B);
  if (rc) return rc;
  if (!x0_dev || !xs_dev || !us_dev) return fail(DLMPC_EINVAL, "NULL argument");
  if (T_sim < 1 || (mode & ~(DLMPC_CL_SHIFT | DLMPC_CL_SCALE_RHO)))
    return fail(DLMPC_EINVAL, "need T_sim >= 1 and mode a combination of DLMPC_CL_SHIFT, DLMPC_CL_SCALE_RHO");
  API_HIP(hipSetDevice(p->opt.device));
  if ((rc = check_x0_device(p, x0_dev, B))) return rc;
  const HostSetup &h = p->hs;
  const size_t nxs = size_t(h.N) * h.nx;
  const bool shift = mode & DLMPC_CL_SHIFT, scale = mode & DLMPC_CL_SCALE_RHO;
  API_HIP(hipMemcpyAsync(p->d_clx, x0_dev, sizeof(double) * B * nxs, hipMemcpyDeviceToDevice, p->stream));
  if (scale) {
    const std::vector<double> ones(B, 1.0);  // step 0 runs with rho itself
    API_HIP(hipMemcpyAsync(p->d_clrs, ones.data(), sizeof(double) * B, hipMemcpyHostToDevice, p->stream));
    API_HIP(hipStreamSynchronize(p->stream));
  }
  std::string err;
  bool all = true;
  for (int t = 0; t < T_sim; ++t) {
    const int start = (shift && t > 0) ? DLMPC_START_TRAJECTORY : DLMPC_START_COLD;
    rc = run_batch(p, B, p->d_clx, p->d_clu, start, p->d_clys, shift ? p->d_cly : nullptr, nullptr,
                   stats ? stats + size_t(t) * B : nullptr, now_ms(), scale ? p->d_clrs : nullptr);
    if (rc < 0) return rc;
    all = all && rc == DLMPC_OK;
    if ((rc = p->beng->plant_step(p->d_clx, p->d_clu, xs_dev, us_dev, t, T_sim, B, scale ? p->d_clrs : nullptr,
                                  err)))
      return fail(rc, err);
    if (shift && (rc = p->beng->shift_inputs(p->d_cly, p->d_clys, B, err))) return fail(rc, err);
  }
  API_HIP(hipStreamSynchronize(p->stream));
  return all ? DLMPC_OK : DLMPC_ENOCONV;
}

int dlmpc_set_rho(dlmpc_problem *p, double rho) {
  if (!p) return fail(DLMPC_EINVAL, "NULL problem");
  if (!(rho > 0.0) || !std::isfinite(rho)) return fail(DLMPC_EINVAL, "need a finite rho > 0");
  p->rho = rho;
  if (p->beng) p->beng->set_rho(rho);
  return DLMPC_OK;
}

int dlmpc_set_coupling(dlmpc_problem *p, int32_t n, const int64_t *row_a, const int64_t *row_b, const double *lo,
                       const double *hi, double sigma, int32_t inner_max, double inner_eps) {
  if (!p) return fail(DLMPC_EINVAL, "NULL problem");
  if (n < 0 || (n > 0 && (!row_a || !row_b || !lo || !hi))) return fail(DLMPC_EINVAL, "NULL coupling array");
  if (!(sigma > 0.0) || !std::isfinite(sigma) || inner_max < 1 || !(inner_eps >= 0.0))
    return fail(DLMPC_EINVAL, "need sigma > 0, inner_max >= 1, inner_eps >= 0");
  const HostSetup &h = p->hs;
  const int64_t Nx = int64_t(h.N) * h.nx, Nu = int64_t(h.N) * h.nu, R = Nx * h.T + Nu * (h.T - 1);
  // canonical row -> library row m * rs + l (local order x_0..x_{T-1}, then u_0..u_{T-2})
  auto lib_row = [&](int64_t r) -> int64_t {
    if (r < Nx * h.T) {
      const int64_t t = r / Nx, q = r % Nx;
      return (q / h.nx) * h.rs + t * h.nx + q % h.nx;
    }
    const int64_t r2 = r - Nx * h.T, t = r2 / Nu, q = r2 % Nu;
    return (q / h.nu) * h.rs + int64_t(h.nx) * h.T + t * h.nu + q % h.nu;
  };
  std::vector<int64_t> a(n), b(n);
  for (int32_t e = 0; e < n; ++e) {
    if (row_a[e] < Nx || row_a[e] >= R || row_b[e] < Nx || row_b[e] >= R || row_a[e] == row_b[e])
      return fail(DLMPC_EINVAL, "coupling " + std::to_string(e) + ": rows must be distinct, in range and not in x_0");
    if (std::isnan(lo[e]) || std::isnan(hi[e]) || lo[e] > hi[e])
      return fail(DLMPC_EINVAL, "coupling " + std::to_string(e) + ": need lo <= hi");
    a[e] = lib_row(row_a[e]);
    b[e] = lib_row(row_b[e]);
  }
  if (p->host_only) return fail(DLMPC_EDEVICE, "problem was set up host-only");
  API_HIP(hipSetDevice(p->opt.device));
  std::string err;
  int rc = p->eng->set_coupling(n, a.data(), b.data(), lo, hi, sigma, inner_max, inner_eps, err);
  if (rc) return fail(rc, err);
  p->cp_a = a;
  p->cp_b = b;
  p->cp_lo.assign(lo, lo + n);
  p->cp_hi.assign(hi, hi + n);
  if (p->sched == 1) p->sched = 0;  // the persistent kernel has no nested step
  return capture_single(p);
}

int dlmpc_solve_stream(dlmpc_problem *p, int32_t n, const double *x0_dev, double *u0_dev, int32_t refill_min,
                       int32_t check_iters, dlmpc_stats *stats, dlmpc_stream_info *info) {
  const double t0 = now_ms();
  int rc = check_stream_args(p, n, x0_dev, u0_dev, refill_min, check_iters);
  if (rc) return rc;
  API_HIP(hipSetDevice(p->opt.device));
  const size_t sy_len = size_t(p->beng->bmax()) * p->hs.N * p->hs.rs;
  if (!p->d_sy) API_HIP(hipMalloc(&p->d_sy, sizeof(float) * sy_len));
  return run_stream(p, n, x0_dev, u0_dev, refill_min, check_iters, stats, info, p->d_sy, t0);
}

int dlmpc_solve_stream_noalloc(dlmpc_problem *p, int32_t n, const double *x0_dev, double *u0_dev,
                               int32_t refill_min, int32_t check_iters, dlmpc_stats *stats,
                               dlmpc_stream_info *info) {
  const double t0 = now_ms();
  int rc = check_stream_args(p, n, x0_dev, u0_dev, refill_min, check_iters);
  if (rc) return rc;
  API_HIP(hipSetDevice(p->opt.device));
  const size_t sy_len = size_t(p->beng->bmax()) * p->hs.N * p->hs.rs;
  float *sy = nullptr;
  size_t cap = 0;
  std::string err;
  if ((rc = dlmpc::stream_scratch(&sy, &cap, err))) return fail(rc, err);
  if (sy_len > cap)
    return fail(DLMPC_EINVAL, "dlmpc_solve_stream_noalloc: max_batch * N * (nx*T + nu*(T-1)) = " +
                                  std::to_string(sy_len) + " exceeds the static staging of " + std::to_string(cap) +
                                  " floats");
  return run_stream(p, n, x0_dev, u0_dev, refill_min, check_iters, stats, info, sy, t0);
}

namespace {

int check_ws(dlmpc_problem *p) {
  if (!p) return fail(DLMPC_EINVAL, "NULL problem");
  if (p->host_only) return fail(DLMPC_EDEVICE, "problem was set up host-only");
  if (!p->ws) return fail(DLMPC_EINVAL, "no warm-start network (dlmpc_ws_init or dlmpc_warmstart_load)");
  return DLMPC_OK;
}

}  // namespace

int dlmpc_ws_init(dlmpc_problem *p, int32_t hidden, int32_t max_samples, uint64_t seed, double x_scale,
                  double y_scale) {
  if (!p) return fail(DLMPC_EINVAL, "NULL problem");
  if (p->host_only) return fail(DLMPC_EDEVICE, "problem was set up host-only");
  API_HIP(hipSetDevice(p->opt.device));
  API_HIP(hipStreamSynchronize(p->stream));
  p->ws.reset();
  auto ws = std::make_unique<dlmpc::WarmStart>();
  std::string err;
  const int rc = ws->init(p->hs, hidden, max_samples, seed, x_scale, y_scale, p->stream, err);
  if (rc) return fail(rc, err);
  p->ws = std::move(ws);
  return DLMPC_OK;
}

int dlmpc_ws_shape(const dlmpc_problem *p, int32_t *in, int32_t *hidden, int32_t *out, int64_t *n_params) {
  int rc = check_ws(const_cast<dlmpc_problem *>(p));
  if (rc) return rc;
  if (in) *in = p->ws->IN;
  if (hidden) *hidden = p->ws->H;
  if (out) *out = p->ws->OUT;
  if (n_params) *n_params = p->ws->n_params;
  return DLMPC_OK;
}

int dlmpc_ws_params(dlmpc_problem *p, float *get, const float *set) {
  int rc = check_ws(p);
  if (rc) return rc;
  API_HIP(hipSetDevice(p->opt.device));
  API_HIP(hipStreamSynchronize(p->stream));
  const size_t bytes = sizeof(float) * size_t(p->ws->n_params);
  if (get) API_HIP(hipMemcpy(get, p->ws->theta, bytes, hipMemcpyDeviceToHost));
  if (set) {
    if (!finite_all(set, size_t(p->ws->n_params))) return fail(DLMPC_EINVAL, "parameters have a NaN/Inf entry");
    API_HIP(hipMemcpy(p->ws->theta, set, bytes, hipMemcpyHostToDevice));
  }
  return DLMPC_OK;
}

int dlmpc_ws_loss_grad(dlmpc_problem *p, int32_t S, const double *x0_dev, const double *y_dev, double *loss,
                       float *grad) {
  int rc = check_ws(p);
  if (rc) return rc;
  API_HIP(hipSetDevice(p->opt.device));
  std::string err;
  double l = 0.0;
  if ((rc = p->ws->forward(S, x0_dev, err)) || (rc = p->ws->backward(S, y_dev, &l, err))) return fail(rc, err);
  if (loss) *loss = l;
  if (grad)
    API_HIP(hipMemcpy(grad, p->ws->grad, sizeof(float) * size_t(p->ws->n_params), hipMemcpyDeviceToHost));
  return DLMPC_OK;
}

int dlmpc_ws_train_step(dlmpc_problem *p, int32_t S, const double *x0_dev, const double *y_dev, double lr,
                        double *loss) {
  int rc = check_ws(p);
  if (rc) return rc;
  API_HIP(hipSetDevice(p->opt.device));
  std::string err;
  if ((rc = p->ws->forward(S, x0_dev, err)) || (rc = p->ws->backward(S, y_dev, loss, err)) ||
      (rc = p->ws->adam(lr, err)))
    return fail(rc, err);
  return DLMPC_OK;
}

int dlmpc_ws_predict(dlmpc_problem *p, int32_t S, const double *x0_dev, double *y_dev) {
  int rc = check_ws(p);
  if (rc) return rc;
  if (!y_dev) return fail(DLMPC_EINVAL, "NULL output");
  API_HIP(hipSetDevice(p->opt.device));
  std::string err;
  if ((rc = p->ws->predict(S, x0_dev, y_dev, err))) return fail(rc, err);
  API_HIP(hipStreamSynchronize(p->stream));
  return DLMPC_OK;
}

int dlmpc_ws_save(dlmpc_problem *p, const char *path) {
  int rc = check_ws(p);
  if (rc) return rc;
  if (!path) return fail(DLMPC_EINVAL, "NULL path");
  API_HIP(hipSetDevice(p->opt.device));
  API_HIP(hipStreamSynchronize(p->stream));
  std::string err;
  if ((rc = p->ws->save(path, err))) return fail(rc, err);
  return DLMPC_OK;
}

int dlmpc_warmstart_load(dlmpc_problem *p, const char *path) {
  if (!p || !path) return fail(DLMPC_EINVAL, "NULL argument");
  if (p->host_only) return fail(DLMPC_EDEVICE, "problem was set up host-only");
  std::string err;
  int32_t hidden = 0;
  int rc = dlmpc::WarmStart::peek(path, &hidden, err);
  if (rc) return fail(rc, err);
  const bool created = !p->ws || p->ws->H != hidden;
  if (created) {
    rc = dlmpc_ws_init(p, hidden, std::max(1, p->opt.max_batch), 0, 1.0, 1.0);
    if (rc) return rc;
  }
  API_HIP(hipSetDevice(p->opt.device));
  API_HIP(hipStreamSynchronize(p->stream));
  if ((rc = p->ws->load(path, err))) {
    if (created) p->ws.reset();  // no half-made network is left behind
    return fail(rc, err);
  }
  return DLMPC_OK;
}

void dlmpc_destroy(dlmpc_problem *p) {
  if (!p) return;
  release_device(p);
  delete p;
}

// ------------------------------------------------------------------ groups of problems

struct dlmpc_group {
  std::vector<dlmpc_problem *> p;
  hipStream_t stream = nullptr;
  hipGraph_t graph[dlmpc_problem::kGraphs] = {};
  hipGraphExec_t gexec[dlmpc_problem::kGraphs] = {};
  hipEvent_t ev_fork = nullptr, ev_done = nullptr, ev_t0 = nullptr, ev_t1 = nullptr;
  std::vector<hipEvent_t> ev_join;
  Ctl *h_ctl = nullptr;  // pinned, one per member
};

namespace {

void group_release(dlmpc_group *g) {
  if (!g) return;
  if (!g->p.empty()) (void)hipSetDevice(g->p[0]->opt.device);
  if (g->stream) (void)hipStreamSynchronize(g->stream);
  for (int k = 0; k < dlmpc_problem::kGraphs; ++k) {
    if (g->gexec[k]) (void)hipGraphExecDestroy(g->gexec[k]);
    if (g->graph[k]) (void)hipGraphDestroy(g->graph[k]);
  }
  for (hipEvent_t e : g->ev_join)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : {g->ev_fork, g->ev_done, g->ev_t0, g->ev_t1})
    if (e) (void)hipEventDestroy(e);
  if (g->h_ctl) (void)hipHostFree(g->h_ctl);
  if (g->stream) (void)hipStreamDestroy(g->stream);
}

}  // namespace

int dlmpc_group_create(dlmpc_problem *const *probs, int32_t n, dlmpc_group **out) {
  if (!probs || n < 1 || !out) return fail(DLMPC_EINVAL, "need n >= 1 problems and an output handle");
  *out = nullptr;
  for (int i = 0; i < n; ++i) {
    if (!probs[i]) return fail(DLMPC_EINVAL, "NULL problem in group");
    if (probs[i]->host_only || !probs[i]->beng) return fail(DLMPC_EINVAL, "group members need the batched engine (max_batch > 0)");
    if (!probs[i]->cp_a.empty()) return fail(DLMPC_EINVAL, "couplings are set: only single-instance solves take them");
    if (probs[i]->opt.device != probs[0]->opt.device) return fail(DLMPC_EINVAL, "group members must share one device");
    for (int k = 0; k < i; ++k)
      if (probs[k] == probs[i]) return fail(DLMPC_EINVAL, "a problem appears twice in the group");
  }
  auto g = std::make_unique<dlmpc_group>();
  g->p.assign(probs, probs + n);
  auto undo = [&](int code, const std::string &msg) {
    group_release(g.get());
    g->stream = nullptr;
    return fail(code, msg);
  };
#define GRP_HIP(expr)                                                                         \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess) return undo(DLMPC_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)
  GRP_HIP(hipSetDevice(probs[0]->opt.device));
  GRP_HIP(hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking));
  GRP_HIP(hipEventCreateWithFlags(&g->ev_fork, hipEventDisableTiming));
  GRP_HIP(hipEventCreateWithFlags(&g->ev_done, hipEventDisableTiming));
  GRP_HIP(hipEventCreate(&g->ev_t0));
  GRP_HIP(hipEventCreate(&g->ev_t1));
  g->ev_join.assign(n, nullptr);
  for (auto &e : g->ev_join) GRP_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  GRP_HIP(hipHostMalloc(reinterpret_cast<void **>(&g->h_ctl), sizeof(Ctl) * n, hipHostMallocDefault));
  for (int i = 0; i < n; ++i) GRP_HIP(hipStreamSynchronize(probs[i]->stream));
  // One graph per chunk size: fork to every member's stream, 2^k batched iterations each,
  // join back (the members' kernels are independent branches of the graph).
  for (int k = 0; k < dlmpc_problem::kGraphs; ++k) {
    GRP_HIP(hipStreamBeginCapture(g->stream, hipStreamCaptureModeThreadLocal));
    int rc = hipEventRecord(g->ev_fork, g->stream) == hipSuccess ? DLMPC_OK : DLMPC_EDEVICE;
    std::string err = rc ? "hipEventRecord failed during capture" : "";
    for (int i = 0; i < n && !rc; ++i) {
      dlmpc_problem *q = probs[i];
      if (hipStreamWaitEvent(q->stream, g->ev_fork, 0) != hipSuccess) {
        rc = DLMPC_EDEVICE;
        err = "hipStreamWaitEvent failed during capture";
        break;
      }
      for (int it = 0; it < (1 << k) && !rc; ++it) rc = q->beng->iteration(err);
      if (!rc && (hipEventRecord(g->ev_join[i], q->stream) != hipSuccess ||
                  hipStreamWaitEvent(g->stream, g->ev_join[i], 0) != hipSuccess)) {
        rc = DLMPC_EDEVICE;
        err = "event join failed during capture";
      }
    }
    hipGraph_t gr = nullptr;
    const hipError_t ec = hipStreamEndCapture(g->stream, &gr);
    if (rc || ec != hipSuccess) {
      if (gr) (void)hipGraphDestroy(gr);
      return undo(rc ? rc : DLMPC_EDEVICE, rc ? err : std::string("hipStreamEndCapture: ") + hipGetErrorString(ec));
    }
    g->graph[k] = gr;
    GRP_HIP(hipGraphInstantiate(&g->gexec[k], g->graph[k], nullptr, nullptr, 0));
  }
#undef GRP_HIP
  *out = g.release();
  return DLMPC_OK;
}

int dlmpc_group_solve_batch(dlmpc_group *g, const int32_t *B, const double *const *x0_dev,
                            double *const *u0_dev, dlmpc_stats *const *stats) {
  const double t0 = now_ms();
  if (!g || !B || !x0_dev || !u0_dev) return fail(DLMPC_EINVAL, "NULL argument");
  const int n = int(g->p.size());
  for (int i = 0; i < n; ++i) {
    int rc = check_batch(g->p[i], B[i]);
    if (rc) return rc;
    if (!x0_dev[i] || !u0_dev[i]) return fail(DLMPC_EINVAL, "NULL device buffer for a group member");
  }
  API_HIP(hipSetDevice(g->p[0]->opt.device));
  std::string err;
  int max_iter = 0;
  double eps = 0.0;
  for (int i = 0; i < n; ++i) {
    dlmpc_problem *q = g->p[i];
    int rc = q->beng->precompute(x0_dev[i], B[i], q->opt.max_iter, q->opt.eps, 0, nullptr, err);
    if (rc) return fail(rc, err);
    API_HIP(hipEventRecord(g->ev_join[i], q->stream));
    API_HIP(hipStreamWaitEvent(g->stream, g->ev_join[i], 0));
    max_iter = std::max(max_iter, q->opt.max_iter);
    eps = std::max(eps, q->opt.eps);
  }
  API_HIP(hipEventRecord(g->ev_t0, g->stream));
  ChunkPredictor pred;
  int launched = 0, checks = 0, nchunk = 32;
  bool all_stopped = false;
  while (!all_stopped) {
    nchunk = std::max(1, std::min(nchunk, max_iter - launched));
    int rc = launch_graphs(g->gexec, g->stream, nchunk);
    if (rc) return rc;
    launched += nchunk;
    ++checks;
    for (int i = 0; i < n; ++i)
      API_HIP(hipMemcpyAsync(&g->h_ctl[i], g->p[i]->beng->ctl(), sizeof(Ctl), hipMemcpyDeviceToHost, g->stream));
    API_HIP(hipStreamSynchronize(g->stream));
    all_stopped = true;
    double worst = 0.0, worst_d = 0.0;
    int iters = 0;
    for (int i = 0; i < n; ++i) {
      const Ctl &c = g->h_ctl[i];
      if (!c.stop) {
        all_stopped = false;
        if (c.last_rp > worst) worst = c.last_rp;
        if (c.last_rd > worst_d) worst_d = c.last_rd;
        iters = std::max(iters, c.iters);
      }
    }
    if (all_stopped || launched >= max_iter) break;
    nchunk = pred.next(iters, worst, worst_d, eps);
  }
  if (!all_stopped) return fail(DLMPC_EDEVICE, "grouped iteration did not reach its stop condition");
  API_HIP(hipEventRecord(g->ev_t1, g->stream));
  API_HIP(hipEventRecord(g->ev_done, g->stream));
  float ms = 0.f;
  bool all = true, numeric = false;
  for (int i = 0; i < n; ++i) {
    dlmpc_problem *q = g->p[i];
    API_HIP(hipStreamWaitEvent(q->stream, g->ev_done, 0));
    int rc = q->beng->output(u0_dev[i], err);
    if (rc) return fail(rc, err);
    if (!(q->opt.flags & DLMPC_FLAG_NO_CHECK) && (rc = q->beng->check(x0_dev[i], err))) return fail(rc, err);
    API_HIP(hipMemcpyAsync(q->h_bctl, q->beng->ictl(), sizeof(dlmpc::BCtl) * B[i], hipMemcpyDeviceToHost, q->stream));
    API_HIP(hipStreamSynchronize(q->stream));
    if (i == 0) (void)hipEventElapsedTime(&ms, g->ev_t0, g->ev_t1);
    for (int b = 0; b < B[i]; ++b) {
      const dlmpc::BCtl &ic = q->h_bctl[b];
      all = all && ic.converged;
      numeric = numeric || ic.numeric;
      if (stats && stats[i]) fill_stats(stats[i][b], ic, ms, checks, DLMPC_START_COLD, t0);
    }
  }
  if (numeric) return fail(DLMPC_ENUMERIC, "NaN/Inf in a batched ADMM iterate");
  return all ? DLMPC_OK : DLMPC_ENOCONV;
}

void dlmpc_group_destroy(dlmpc_group *g) {
  if (!g) return;
  group_release(g);
  delete g;
}

}  // extern "C"
