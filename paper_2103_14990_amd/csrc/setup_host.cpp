// Offline precomputation of DLMPC (Algorithm 1, first step), host side, FP64.
//
// For every subsystem j the Psi-comp step of Algorithm 2 projects each column c of j onto
// {psi supported on the d-hop rows of j : Z_AB psi = e_c}, where Z_AB is the SLS
// achievability operator (Section II-A): x_0 = e_c, x_{t+1} = A x_t + B u_t. Restricted to
// the patch P(j), a vector psi in the support is a state/input trajectory of the patch whose
// states stay inside the patch, so its equations are:
//   (a) the patch dynamics x_P[t+1] = A_PP x_P[t] + B_P u_P[t] (rows of patch states);
//   (b) the ring equations G x_P[t] = 0 for t = 0..T-2, G = rows of A for states outside the
//       patch that couple to it (the patch must not leak into the (d+1)-hop ring).
// Rather than factoring the whole column block (D_col rows), this parametrises (a) by the
// patch inputs U (u_P[0..T-2]) and factors only (b) as a linear map M: U -> ring values:
//   null space:  N_j = orth( S K ), K = orthonormal basis of null(M) from a Householder QR
//                with column pivoting of M', S = the simulation map U -> trajectory;
//   offsets:     o_c = (I - N_j N_j') psi_p, psi_p = trajectory from x_0 = e_c under the
//                minimum-norm input solving M U = -(free response on the ring).
// psi_p meets every equation of the block iff that solve is consistent; otherwise column c has
// no localised trajectory and setup fails with DLMPC_EINFEASIBLE_LOCALITY.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <numeric>
#include <thread>

#include "dlmpc_internal.h"

namespace dlmpc {
namespace {


// Column-major dense matrix.
struct Dense {
  int m = 0, n = 0;
  std::vector<double> a;
  Dense() = default;
  Dense(int m_, int n_) : m(m_), n(n_), a(size_t(m_) * size_t(n_), 0.0) {}
  double &operator()(int i, int j) { return a[size_t(j) * m + i]; }
  double operator()(int i, int j) const { return a[size_t(j) * m + i]; }
  double *col(int j) { return a.data() + size_t(j) * m; }
  const double *col(int j) const { return a.data() + size_t(j) * m; }
};

// C = A * B.
Dense matmul(const Dense &A, const Dense &B) {
  Dense C(A.m, B.n);
  for (int j = 0; j < B.n; ++j) {
    double *c = C.col(j);
    for (int k = 0; k < A.n; ++k) {
      const double b = B(k, j);
      if (b == 0.0) continue;
      const double *a = A.col(k);
      for (int i = 0; i < A.m; ++i) c[i] += a[i] * b;
    }
  }
  return C;
}

// Householder QR with column pivoting, stopped at numerical rank: F (m x n) is overwritten
// with R in its upper rows and the reflector vectors (unit leading entry implicit) below the
// diagonal of its first `rank` columns. Column k of the factored matrix is column jpvt[k] of
// the input. The factorisation stops at the first step whose largest remaining column norm
// is <= rtol times the first pivot's norm.
int qr_pivoted(Dense &F, std::vector<double> &tau, std::vector<int> &jpvt, double rtol) {
  const int m = F.m, n = F.n, kmax = std::min(m, n);
  tau.assign(kmax, 0.0);
  jpvt.resize(n);
  std::iota(jpvt.begin(), jpvt.end(), 0);
  double first = 0.0;
  int rank = 0;
  for (int k = 0; k < kmax; ++k) {
    int piv = k;
    double best = -1.0;
    for (int j = k; j < n; ++j) {
      const double *c = F.col(j);
      double s = 0.0;
      for (int i = k; i < m; ++i) s += c[i] * c[i];
      if (s > best) {
        best = s;
        piv = j;
      }
    }
    const double nrm = std::sqrt(best);
    if (k == 0) first = nrm;
    if (!(nrm > rtol * first) || nrm == 0.0) break;
    if (piv != k) {
      std::swap_ranges(F.col(k), F.col(k) + m, F.col(piv));
      std::swap(jpvt[k], jpvt[piv]);
    }
    double *x = F.col(k);
    const double alpha = x[k];
    const double beta = -std::copysign(nrm, alpha);
    const double scale = 1.0 / (alpha - beta);
    for (int i = k + 1; i < m; ++i) x[i] *= scale;
    x[k] = beta;
    tau[k] = (beta - alpha) / beta;
    for (int j = k + 1; j < n; ++j) {
      double *c = F.col(j);
      double s = c[k];
      for (int i = k + 1; i < m; ++i) s += x[i] * c[i];
      s *= tau[k];
      c[k] -= s;
      for (int i = k + 1; i < m; ++i) c[i] -= s * x[i];
    }
    rank = k + 1;
  }
  return rank;
}

// X <- Q X with Q = H_0 H_1 ... H_{rank-1} from qr_pivoted.
void apply_q(const Dense &F, const std::vector<double> &tau, int rank, Dense &X) {
  for (int k = rank - 1; k >= 0; --k) {
    const double *v = F.col(k);
    for (int j = 0; j < X.n; ++j) {
      double *c = X.col(j);
      double s = c[k];
      for (int i = k + 1; i < F.m; ++i) s += v[i] * c[i];
      s *= tau[k];
      c[k] -= s;
      for (int i = k + 1; i < F.m; ++i) c[i] -= s * v[i];
    }
  }
}

struct BlockRef {
  int32_t col;
  const double *blk;  // nx x nx row-major
};

// Block rows of A (pointers into hs.a_blocks) and the undirected interconnection graph
// G_(A,B): i ~ j when block A_ij or A_ji has a nonzero entry.
void block_rows(const HostSetup &hs, std::vector<std::vector<BlockRef>> &arow,
                std::vector<std::vector<int32_t>> &adj) {
  const int32_t N = hs.N, nx = hs.nx;
  for (int i = 0; i < N; ++i)
    for (int64_t q = hs.a_rowptr[i]; q < hs.a_rowptr[i + 1]; ++q) {
      const int32_t j = hs.a_colidx[q];
      const double *blk = hs.a_blocks.data() + size_t(q) * nx * nx;
      arow[i].push_back({j, blk});
      bool nz = false;
      for (int e = 0; e < nx * nx; ++e) nz |= (blk[e] != 0.0);
      if (nz && j != i) {
        adj[i].push_back(j);
        adj[j].push_back(i);
      }
    }
  for (auto &a : adj) {
    std::sort(a.begin(), a.end());
    a.erase(std::unique(a.begin(), a.end()), a.end());
  }
}

// Per-subsystem factorisation context (everything local to patch P(j)).
struct PatchFactor {
  int N, nx, nu, T, rs;
  const std::vector<std::vector<BlockRef>> *arow;  // A blocks per block row
  const double *b_blocks;
  const std::vector<std::vector<int32_t>> *adj;

  // Simulates the patch from initial states X0 (ns x K) under inputs U (mu x K); writes the
  // trajectories in local tile order into psi (D x K, may be null) and the ring values
  // G x[t], t = 0..T-2, into cons (mc x K, may be null).
  void simulate(const Dense &App, const Dense &Bp, const Dense &G, const Dense &X0,
                const Dense &U, int p, Dense *psi, Dense *cons) const {
    const int ns = p * nx, ni = p * nu, K = X0.n, ng = G.m;
    Dense X = X0;
    for (int t = 0; t < T; ++t) {
      if (psi)
        for (int k = 0; k < K; ++k)
          for (int a = 0; a < p; ++a)
            for (int s = 0; s < nx; ++s) (*psi)(a * rs + t * nx + s, k) = X(a * nx + s, k);
      if (cons && t <= T - 2 && ng > 0) {
        Dense g = matmul(G, X);
        for (int k = 0; k < K; ++k)
          for (int i = 0; i < ng; ++i) (*cons)(t * ng + i, k) = g(i, k);
      }
      if (t < T - 1) {
        Dense Ut(ni, K);
        for (int k = 0; k < K; ++k)
          for (int i = 0; i < ni; ++i) Ut(i, k) = U(t * ni + i, k);
        Dense Xn = matmul(App, X);
        Dense BU = matmul(Bp, Ut);
        for (size_t i = 0; i < Xn.a.size(); ++i) Xn.a[i] += BU.a[i];
        X = std::move(Xn);
      }
    }
    if (psi)
      for (int k = 0; k < K; ++k)
        for (int t = 0; t + 1 < T; ++t)
          for (int a = 0; a < p; ++a)
            for (int q = 0; q < nu; ++q)
              (*psi)(a * rs + nx * T + t * nu + q, k) = U(t * ni + a * nu + q, k);
    (void)ns;
  }

  // Returns 0 or a DLMPC_* error; fills N_j (D x k, column-major) and offsets (D x nx).
  int run(int j, const std::vector<int32_t> &P, std::vector<double> &nbj, int &kj,
          std::vector<double> &offj, std::string &err) const {
    const int p = int(P.size()), ns = p * nx, ni = p * nu, D = p * rs;
    std::vector<int> pos(N, -1);
    for (int a = 0; a < p; ++a) pos[P[a]] = a;

    Dense App(ns, ns), Bp(ns, ni);
    for (int a = 0; a < p; ++a) {
      const int m = P[a];
      for (const BlockRef &br : (*arow)[m]) {
        if (pos[br.col] < 0) continue;
        const int b = pos[br.col];
        for (int s = 0; s < nx; ++s)
          for (int s2 = 0; s2 < nx; ++s2) App(a * nx + s, b * nx + s2) = br.blk[s * nx + s2];
      }
      for (int s = 0; s < nx; ++s)
        for (int q = 0; q < nu; ++q) Bp(a * nx + s, a * nu + q) = b_blocks[(size_t(m) * nx + s) * nu + q];
    }
    // Ring rows: states of subsystems outside P whose A row touches a patch state.
    std::vector<int32_t> ring;
    for (int a = 0; a < p; ++a)
      for (int32_t q : (*adj)[P[a]])
        if (pos[q] < 0) ring.push_back(q);
    std::sort(ring.begin(), ring.end());
    ring.erase(std::unique(ring.begin(), ring.end()), ring.end());
    std::vector<std::vector<double>> grows;
    for (int32_t q : ring)
      for (int s = 0; s < nx; ++s) {
        std::vector<double> g(ns, 0.0);
        bool any = false;
        for (const BlockRef &br : (*arow)[q]) {
          if (pos[br.col] < 0) continue;
          for (int s2 = 0; s2 < nx; ++s2) {
            const double v = br.blk[s * nx + s2];
            g[pos[br.col] * nx + s2] = v;
            any |= (v != 0.0);
          }
        }
        if (any) grows.push_back(std::move(g));
      }
    const int ng = int(grows.size());
    Dense G(ng, ns);
    for (int i = 0; i < ng; ++i)
      for (int c = 0; c < ns; ++c) G(i, c) = grows[i][c];

    const int mu = ni * (T - 1), mc = ng * (T - 1);
    // M (mc x mu): block (t', tau) = G A_PP^{t'-1-tau} B_P for tau < t' (Toeplitz in time).
    Dense M(mc, mu);
    if (ng > 0) {
      Dense W = Bp;
      for (int k = 0; k <= T - 3; ++k) {
        Dense Mk = matmul(G, W);
        for (int tau = 0; tau + k + 1 <= T - 2; ++tau) {
          const int tp = tau + k + 1;
          for (int c = 0; c < ni; ++c)
            for (int i = 0; i < ng; ++i) M(tp * ng + i, tau * ni + c) = Mk(i, c);
        }
        W = matmul(App, W);
      }
    }
    // Rank-revealing QR of M' (mu x mc).
    Dense F(mu, mc);
    for (int i = 0; i < mc; ++i)
      for (int c = 0; c < mu; ++c) F(c, i) = M(i, c);
    std::vector<double> tau;
    std::vector<int> jpvt;
    const int r = (mc > 0) ? qr_pivoted(F, tau, jpvt, kRankTol) : 0;
    const int k = mu - r;
    // K = Q [0; I_k]: orthonormal basis of null(M).
    Dense Kb(mu, k);
    for (int i = 0; i < k; ++i) Kb(r + i, i) = 1.0;
    apply_q(F, tau, r, Kb);
    // S K, then an orthonormal basis of its range.
    Dense SK(D, k);
    {
      Dense X0(ns, k);
      simulate(App, Bp, G, X0, Kb, p, &SK, nullptr);
    }
    Dense Nj(D, k);
    if (k > 0) {
      Dense Fs = SK;
      std::vector<double> tau2;
      std::vector<int> jp2;
      const int r2 = qr_pivoted(Fs, tau2, jp2, kBasisTol);
      if (r2 != k) {
        err = "null basis lost rank at subsystem " + std::to_string(j);
        return DLMPC_ENUMERIC;
      }
      for (int i = 0; i < k; ++i) Nj(i, i) = 1.0;
      apply_q(Fs, tau2, r2, Nj);
    }
    // Particular solutions and offsets for every column c of j.
    const int aj = pos[j];
    Dense offs(D, nx);
    for (int c = 0; c < nx; ++c) {
      Dense X0(ns, 1), U0(mu, 1), cons0(std::max(mc, 1), 1);
      X0(aj * nx + c, 0) = 1.0;
      if (ng > 0) simulate(App, Bp, G, X0, U0, p, nullptr, &cons0);
      Dense u(mu, 1);
      if (r > 0) {
        // min-norm u with M u = b, b = -cons0: M' Pi = Q R  =>  R11' w = (Pi' b)[:r], u = Q [w; 0].
        std::vector<double> w(r);
        for (int i = 0; i < r; ++i) {
          double s = -cons0(jpvt[i], 0);
          for (int l = 0; l < i; ++l) s -= F(l, i) * w[l];
          w[i] = s / F(i, i);
        }
        for (int i = 0; i < r; ++i) u(i, 0) = w[i];
        apply_q(F, tau, r, u);
      }
      Dense psi(D, 1), cons(std::max(mc, 1), 1);
      simulate(App, Bp, G, X0, u, p, &psi, ng > 0 ? &cons : nullptr);
      // ring residual relative to the size of the trajectory (rounding grows with it)
      double resid = 0.0, size = 1.0;
      if (ng > 0)
        for (int i = 0; i < mc; ++i) resid = std::max(resid, std::fabs(cons(i, 0)));
      for (int rr = 0; rr < D; ++rr) size = std::max(size, std::fabs(psi(rr, 0)));
      resid /= size;
      if (!(resid <= kFeasTol)) {
        err = "column " + std::to_string(j * nx + c) + " of subsystem " + std::to_string(j) +
              " has no trajectory inside its d-hop patch (relative ring residual " + std::to_string(resid) + ")";
        return DLMPC_EINFEASIBLE_LOCALITY;
      }
      // o_c = psi - N (N' psi)
      std::vector<double> t(k, 0.0);
      for (int i = 0; i < k; ++i) {
        const double *nc = Nj.col(i);
        double s = 0.0;
        for (int rr = 0; rr < D; ++rr) s += nc[rr] * psi(rr, 0);
        t[i] = s;
      }
      for (int rr = 0; rr < D; ++rr) {
        double s = 0.0;
        for (int i = 0; i < k; ++i) s += Nj(rr, i) * t[i];
        offs(rr, c) = psi(rr, 0) - s;
      }
    }
    kj = k;
    nbj = std::move(Nj.a);
    offj = std::move(offs.a);
    return DLMPC_OK;
  }
};

bool finite_all(const double *v, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

}  // namespace

int host_setup(const dlmpc_system *sys, int32_t d, int32_t T, const dlmpc_cost *cost,
               HostSetup &hs, std::string &err) {
  const auto t_start = std::chrono::steady_clock::now();
  if (!sys || !cost) {
    err = "system and cost must be non-NULL";
    return DLMPC_EINVAL;
  }
  const int32_t N = sys->n_sub, nx = sys->nx, nu = sys->nu;
  if (N < 1 || nx < 1 || nu < 1 || d < 0 || T < 2) {
    err = "need n_sub >= 1, nx >= 1, nu >= 1, d >= 0, T >= 2";
    return DLMPC_EINVAL;
  }
  if (!sys->a_rowptr || !sys->a_colidx || !sys->a_blocks || !sys->b_blocks || !cost->q_diag ||
      !cost->r_diag) {
    err = "NULL array in system or cost";
    return DLMPC_EINVAL;
  }
  if (sys->a_rowptr[0] != 0) {
    err = "a_rowptr[0] must be 0";
    return DLMPC_EINVAL;
  }
  for (int i = 0; i < N; ++i)
    if (sys->a_rowptr[i + 1] < sys->a_rowptr[i]) {
      err = "a_rowptr must be non-decreasing";
      return DLMPC_EINVAL;
    }
  const int64_t nnzb = sys->a_rowptr[N];
  if (!finite_all(sys->a_blocks, size_t(nnzb) * nx * nx) ||
      !finite_all(sys->b_blocks, size_t(N) * nx * nu)) {
    err = "A or B has a NaN/Inf entry";
    return DLMPC_EINVAL;
  }
  const int64_t Nx = int64_t(N) * nx, Nu = int64_t(N) * nu;
  for (int64_t i = 0; i < Nx; ++i)
    if (!(cost->q_diag[i] > 0.0) || !std::isfinite(cost->q_diag[i])) {
      err = "q_diag must be finite and > 0";
      return DLMPC_EINVAL;
    }
  for (int64_t i = 0; i < Nu; ++i)
    if (!(cost->r_diag[i] > 0.0) || !std::isfinite(cost->r_diag[i])) {
      err = "r_diag must be finite and > 0";
      return DLMPC_EINVAL;
    }
  auto check_bounds = [&](const double *lo, const double *hi, int64_t n) {
    for (int64_t i = 0; i < n; ++i) {
      if (lo && (std::isnan(lo[i]) || lo[i] > 0.0)) return false;
      if (hi && (std::isnan(hi[i]) || hi[i] < 0.0)) return false;
    }
    return true;
  };
  if (!check_bounds(cost->x_lo, cost->x_hi, Nx) || !check_bounds(cost->u_lo, cost->u_hi, Nu)) {
    err = "bounds must be non-NaN with lo <= 0 <= hi";
    return DLMPC_EINVAL;
  }

  hs = HostSetup();
  hs.N = N;
  hs.nx = nx;
  hs.nu = nu;
  hs.T = T;
  hs.d = d;
  hs.rs = nx * T + nu * (T - 1);
  hs.ts = hs.rs * nx;
  hs.R = Nx * T + Nu * (T - 1);
  hs.a_rowptr.assign(sys->a_rowptr, sys->a_rowptr + N + 1);
  hs.a_colidx.assign(sys->a_colidx, sys->a_colidx + nnzb);
  hs.a_blocks.assign(sys->a_blocks, sys->a_blocks + size_t(nnzb) * nx * nx);
  hs.b_blocks.assign(sys->b_blocks, sys->b_blocks + size_t(N) * nx * nu);

  // Block rows of A and the interconnection graph G_(A,B).
  for (int i = 0; i < N; ++i) {
    std::vector<int32_t> cols(sys->a_colidx + sys->a_rowptr[i], sys->a_colidx + sys->a_rowptr[i + 1]);
    for (int32_t j : cols)
      if (j < 0 || j >= N) {
        err = "a_colidx out of range";
        return DLMPC_EINVAL;
      }
    std::sort(cols.begin(), cols.end());
    if (std::adjacent_find(cols.begin(), cols.end()) != cols.end()) {
      err = "duplicate block in a row of A";
      return DLMPC_EINVAL;
    }
  }
  std::vector<std::vector<BlockRef>> arow(N);
  std::vector<std::vector<int32_t>> adj(N);
  block_rows(hs, arow, adj);

  // d-hop patches by breadth-first search.
  hs.patch.assign(N, {});
  {
    std::vector<int32_t> dist(N, -1);
    std::vector<int32_t> seen;
    for (int s = 0; s < N; ++s) {
      std::deque<int32_t> q{s};
      dist[s] = 0;
      seen.assign(1, s);
      while (!q.empty()) {
        const int32_t u = q.front();
        q.pop_front();
        if (dist[u] == d) continue;
        for (int32_t v : adj[u])
          if (dist[v] < 0) {
            dist[v] = dist[u] + 1;
            seen.push_back(v);
            q.push_back(v);
          }
      }
      std::sort(seen.begin(), seen.end());
      hs.patch[s] = seen;
      for (int32_t v : seen) dist[v] = -1;
    }
  }

  // Tiles, row-side lists and sizes.
  hs.tile_off.assign(N + 1, 0);
  for (int j = 0; j < N; ++j) hs.tile_off[j + 1] = hs.tile_off[j] + int64_t(hs.patch[j].size());
  hs.n_tiles = hs.tile_off[N];
  hs.nnz = hs.n_tiles * hs.ts;
  hs.tile_rsub.resize(hs.n_tiles);
  for (int j = 0; j < N; ++j)
    for (size_t a = 0; a < hs.patch[j].size(); ++a) hs.tile_rsub[hs.tile_off[j] + a] = hs.patch[j][a];
  // Patches are symmetric (hop distance is), so tile (j, m) exists iff tile (m, j) does.
  hs.rt_ptr.assign(N + 1, 0);
  for (int m = 0; m < N; ++m) hs.rt_ptr[m + 1] = hs.rt_ptr[m] + int64_t(hs.patch[m].size());
  hs.rt_tile.resize(hs.n_tiles);
  hs.rt_col.resize(hs.n_tiles);
  for (int m = 0; m < N; ++m) {
    int64_t w = hs.rt_ptr[m];
    for (int32_t j : hs.patch[m]) {
      const auto &Pj = hs.patch[j];
      const auto it = std::lower_bound(Pj.begin(), Pj.end(), m);
      if (it == Pj.end() || *it != m) {
        err = "internal: asymmetric patch";
        return DLMPC_EINVAL;
      }
      hs.rt_tile[w] = hs.tile_off[j] + (it - Pj.begin());
      hs.rt_col[w] = j;
      ++w;
    }
  }
  for (int j = 0; j < N; ++j) {
    const int32_t p = int32_t(hs.patch[j].size());
    hs.p_max = std::max(hs.p_max, p);
    hs.d_row_max = std::max(hs.d_row_max, p * nx);
    hs.d_col_max = std::max(hs.d_col_max, p * hs.rs);
    hs.sum_dcol2 += int64_t(p) * hs.rs * int64_t(p) * hs.rs;
  }

  // Row data (local order).
  hs.w.resize(size_t(N) * hs.rs);
  hs.lb.resize(size_t(N) * hs.rs);
  hs.ub.resize(size_t(N) * hs.rs);
  for (int m = 0; m < N; ++m)
    for (int l = 0; l < hs.rs; ++l) {
      const size_t o = size_t(m) * hs.rs + l;
      double w, lo = -INFINITY, hi = INFINITY;
      if (l < nx * T) {
        const int t = l / nx, s = l % nx;
        const int64_t g = int64_t(m) * nx + s;
        w = cost->q_diag[g];
        if (t >= 1) {
          if (cost->x_lo) lo = cost->x_lo[g];
          if (cost->x_hi) hi = cost->x_hi[g];
        }
      } else {
        const int q = (l - nx * T) % nu;
        const int64_t g = int64_t(m) * nu + q;
        w = cost->r_diag[g];
        if (cost->u_lo) lo = cost->u_lo[g];
        if (cost->u_hi) hi = cost->u_hi[g];
      }
      hs.w[o] = w;
      hs.lb[o] = lo;
      hs.ub[o] = hi;
    }

  // Canonical CSR pattern and the tile-element -> CSR map.
  hs.csr_rowptr.assign(hs.R + 1, 0);
  for (int64_t r = 0; r < hs.R; ++r) {
    const int32_t m = (r < Nx * T) ? int32_t((r % Nx) / nx) : int32_t(((r - Nx * T) % Nu) / nu);
    hs.csr_rowptr[r + 1] = hs.csr_rowptr[r] + int64_t(hs.patch[m].size()) * nx;
  }
  hs.csr_map.resize(size_t(hs.nnz));
  for (int m = 0; m < N; ++m)
    for (int64_t q = hs.rt_ptr[m]; q < hs.rt_ptr[m + 1]; ++q) {
      const int64_t tile = hs.rt_tile[q];
      const int64_t pos_in_row = q - hs.rt_ptr[m];  // index of j in P(m)
      for (int l = 0; l < hs.rs; ++l) {
        const int64_t base = hs.csr_rowptr[canon_row(hs, m, l)] + pos_in_row * nx;
        for (int c = 0; c < nx; ++c) hs.csr_map[size_t(tile * hs.ts + l * nx + c)] = base + c;
      }
    }

  hs.setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
  return DLMPC_OK;
}

void pack_factors(HostSetup &hs, const std::vector<int> &ks, const std::vector<std::vector<double>> &nbs,
                  const std::vector<std::vector<double>> &offs) {
  const int32_t N = hs.N, nx = hs.nx;
  hs.kdim = ks;
  hs.nb_off.assign(N + 1, 0);
  hs.off_ptr.assign(N + 1, 0);
  for (int j = 0; j < N; ++j) {
    const int64_t ld = padded_ld(int32_t(hs.patch[j].size()) * hs.rs);
    hs.nb_off[j + 1] = hs.nb_off[j] + ld * ks[j];
    hs.off_ptr[j + 1] = hs.off_ptr[j] + ld * nx;
  }
  hs.nb.clear();
  hs.off.clear();
  hs.nb.resize(size_t(hs.nb_off[N]));
  hs.off.resize(size_t(hs.off_ptr[N]));
  if (!nbs.empty()) std::fill(hs.nb.begin(), hs.nb.end(), 0.0);
  if (!offs.empty()) std::fill(hs.off.begin(), hs.off.end(), 0.0);
  hs.k_max = 0;
  hs.sum_dcol_k = hs.sum_k = 0;
  for (int j = 0; j < N; ++j) {
    const int32_t D = int32_t(hs.patch[j].size()) * hs.rs, ld = padded_ld(D);
    if (!nbs.empty())
      for (int i = 0; i < ks[j]; ++i)
        std::copy(nbs[j].begin() + size_t(i) * D, nbs[j].begin() + size_t(i + 1) * D,
                  hs.nb.begin() + hs.nb_off[j] + size_t(i) * ld);
    if (!offs.empty())
      for (int c = 0; c < nx; ++c)
        std::copy(offs[j].begin() + size_t(c) * D, offs[j].begin() + size_t(c + 1) * D,
                  hs.off.begin() + hs.off_ptr[j] + size_t(c) * ld);
    hs.k_max = std::max(hs.k_max, ks[j]);
    hs.sum_dcol_k += int64_t(D) * ks[j];
    hs.sum_k += ks[j];
  }
}

int factor_host(HostSetup &hs, std::string &err) {
  const auto t_fac = std::chrono::steady_clock::now();
  const int32_t N = hs.N, nx = hs.nx, nu = hs.nu, T = hs.T;
  std::vector<std::vector<BlockRef>> arow(N);
  std::vector<std::vector<int32_t>> adj(N);
  block_rows(hs, arow, adj);
  std::vector<std::vector<double>> nbs(N), offs(N);
  std::vector<int> ks(N, 0), stat(N, DLMPC_OK);
  std::vector<std::string> errs(N);
  PatchFactor pf{N, nx, nu, T, hs.rs, &arow, hs.b_blocks.data(), &adj};
  std::atomic<int> next{0};
  unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  nth = std::min<unsigned>(nth, unsigned(N));
  auto worker = [&]() {
    for (int j; (j = next.fetch_add(1)) < N;) stat[j] = pf.run(j, hs.patch[j], nbs[j], ks[j], offs[j], errs[j]);
  };
  std::vector<std::thread> th;
  for (unsigned t = 1; t < nth; ++t) th.emplace_back(worker);
  worker();
  for (auto &t : th) t.join();
  for (int j = 0; j < N; ++j)
    if (stat[j] != DLMPC_OK) {
      err = errs[j];
      return stat[j];
    }
  pack_factors(hs, ks, nbs, offs);
  hs.factor_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_fac).count();
  hs.factor_where = 0;
  return DLMPC_OK;
}

void factor_lists(const HostSetup &hs, FactorLists &fl) {
  const int32_t N = hs.N, nx = hs.nx;
  std::vector<std::vector<BlockRef>> arow(N);
  std::vector<std::vector<int32_t>> adj(N);
  block_rows(hs, arow, adj);
  fl = FactorLists();
  fl.aj.resize(N);
  fl.ng.resize(N);
  fl.app_rp0.resize(N);
  fl.g_rp0.resize(N);
  fl.app_e0.resize(N);
  fl.g_e0.resize(N);
  std::vector<int> pos(N, -1);
  for (int j = 0; j < N; ++j) {
    const std::vector<int32_t> &P = hs.patch[j];
    const int p = int(P.size());
    for (int a = 0; a < p; ++a) pos[P[a]] = a;
    fl.aj[j] = pos[j];
    // A_PP: row a*nx+s, entries of the blocks of row P[a] whose column is in the patch.
    fl.app_rp0[j] = int64_t(fl.rp.size());
    fl.app_e0[j] = int64_t(fl.ecol.size());
    int32_t cnt = 0;
    fl.rp.push_back(0);
    for (int a = 0; a < p; ++a)
      for (int s = 0; s < nx; ++s) {
        for (const BlockRef &br : arow[P[a]]) {
          if (pos[br.col] < 0) continue;
          const int64_t base = br.blk - hs.a_blocks.data();
          for (int s2 = 0; s2 < nx; ++s2) {
            fl.ecol.push_back(pos[br.col] * nx + s2);
            fl.eidx.push_back(int32_t(base + s * nx + s2));
            ++cnt;
          }
        }
        fl.rp.push_back(cnt);
      }
    // Ring rows: states outside the patch whose A row has a nonzero entry on a patch state.
    std::vector<int32_t> ring;
    for (int a = 0; a < p; ++a)
      for (int32_t q : adj[P[a]])
        if (pos[q] < 0) ring.push_back(q);
    std::sort(ring.begin(), ring.end());
    ring.erase(std::unique(ring.begin(), ring.end()), ring.end());
    fl.g_rp0[j] = int64_t(fl.rp.size());
    fl.g_e0[j] = int64_t(fl.ecol.size());
    cnt = 0;
    int32_t ng = 0;
    fl.rp.push_back(0);
    for (int32_t q : ring)
      for (int s = 0; s < nx; ++s) {
        bool any = false;
        const size_t mark = fl.ecol.size();
        for (const BlockRef &br : arow[q]) {
          if (pos[br.col] < 0) continue;
          const int64_t base = br.blk - hs.a_blocks.data();
          for (int s2 = 0; s2 < nx; ++s2) {
            const double v = br.blk[s * nx + s2];
            any |= (v != 0.0);
            fl.ecol.push_back(pos[br.col] * nx + s2);
            fl.eidx.push_back(int32_t(base + s * nx + s2));
          }
        }
        if (!any) {
          fl.ecol.resize(mark);
          fl.eidx.resize(mark);
          continue;
        }
        cnt += int32_t(fl.ecol.size() - mark);
        fl.rp.push_back(cnt);
        ++ng;
      }
    fl.ng[j] = ng;
    for (int a = 0; a < p; ++a) pos[P[a]] = -1;
  }
}

}  // namespace dlmpc
