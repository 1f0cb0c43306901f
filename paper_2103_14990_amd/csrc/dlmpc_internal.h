// Internal data structures shared by the host setup and the HIP runtime of libdlmpc.
#pragma once

#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "../../include/dlmpc.h"

namespace dlmpc {

// Thresholds of the column-block factorisation (host and device alike).
constexpr double kRankTol = 1e-10;   // relative pivot threshold of the rank-revealing QR of the ring map
constexpr double kBasisTol = 1e-13;  // relative pivot threshold of the QR that orthonormalises S K
constexpr double kFeasTol = 1e-9;    // ring residual of a particular solution over max(1, its largest entry)

// Allocator whose resize() leaves doubles uninitialised (large arrays filled by a copy).
template <class T>
struct NoInitAlloc : std::allocator<T> {
  template <class U>
  struct rebind {
    using other = NoInitAlloc<U>;
  };
  NoInitAlloc() = default;
  template <class U>
  NoInitAlloc(const NoInitAlloc<U> &) noexcept {}
  template <class U>
  void construct(U *p) noexcept {
    ::new (static_cast<void *>(p)) U;
  }
  template <class U, class... Args>
  void construct(U *p, Args &&...args) {
    ::new (static_cast<void *>(p)) U(std::forward<Args>(args)...);
  }
};
using BigVec = std::vector<double, NoInitAlloc<double>>;

// Host-side result of the offline precomputation (Algorithm 1, first step).
//
// Packing ("tiles"): for every column subsystem j and every row subsystem m in its d-hop
// patch P(j) there is one tile holding the block Phi[rows of m, columns of j], rs x nx values
// row-major, where rs = nx*T + nu*(T-1) and the rows of m are in local order
// (x_0..x_{T-1} with nx states each, then u_0..u_{T-2} with nu inputs each). The tiles of j
// are contiguous and ordered by m ascending, so the support of j's columns (D_col(j) rows)
// is one contiguous [D_col(j) x nx] block: Psi-comp of j reads and writes exactly that
// block, Phi-comp of m gathers its p_m tiles, one from each column subsystem in P(m).
struct HostSetup {
  int32_t N = 0, nx = 0, nu = 0, T = 0, d = 0;
  int32_t rs = 0;  // rows per subsystem
  int32_t ts = 0;  // values per tile (rs * nx)
  int64_t R = 0, nnz = 0, n_tiles = 0;

  std::vector<std::vector<int32_t>> patch;  // P(j), ascending

  // The plant as given (block-CSR A with row-major nx x nx blocks, diagonal nx x nu B blocks).
  std::vector<int64_t> a_rowptr;
  std::vector<int32_t> a_colidx;
  std::vector<double> a_blocks, b_blocks;

  std::vector<int64_t> tile_off;    // [N+1] first tile of column subsystem j
  std::vector<int32_t> tile_rsub;   // [n_tiles] row subsystem m of each tile
  std::vector<int64_t> rt_ptr;      // [N+1] row-side CSR over row subsystems
  std::vector<int64_t> rt_tile;     // [n_tiles] tile (j, m) for j in P(m), j ascending
  std::vector<int32_t> rt_col;      // [n_tiles] the column subsystem j of that tile

  // Null bases: N_j is D_col(j) x k_j, column-major with leading dimension ld(j) =
  // D_col(j) rounded up to a multiple of 4 (zero rows below D_col(j)), at nb[nb_off[j]].
  std::vector<int32_t> kdim;        // [N]
  std::vector<int64_t> nb_off;      // [N+1]
  BigVec nb;                        // empty when the bases stay on the device (d_nb)
  // Offsets o_c: ld(j) x nx column-major (zero padded) at off[off_ptr[j]].
  std::vector<int64_t> off_ptr;     // [N+1]
  BigVec off;

  // Row data in local order: w (cost weight), lb/ub (bounds on (Phi x0)_r), [N * rs].
  std::vector<double> w, lb, ub;

  std::vector<int64_t> csr_rowptr;  // [R+1] canonical pattern
  std::vector<int64_t> csr_map;     // [n_tiles*ts] tile element -> canonical CSR index

  int32_t p_max = 0, k_max = 0, d_row_max = 0, d_col_max = 0;
  int64_t sum_dcol_k = 0, sum_dcol2 = 0, sum_k = 0;
  double setup_ms = 0, factor_ms = 0;
  int32_t factor_where = 0;  // 0 = host threads, 1 = device kernels
  int32_t factor_fallbacks = 0;  // device: subsystems whose basis needed the Householder QR
  // Device factorisation: the padded N_j array (same layout as nb, FP64) stays on the device
  // (owned here, released by free_factors_device); nb is then left empty.
  double *d_nb = nullptr;
  int32_t d_nb_device = -1;
};

// Index lists for factoring the column blocks elsewhere than in the host loop: for each
// subsystem j, the sparse patch dynamics A_PP (CSR over the p*nx patch states) and the ring
// map G (CSR over the ng ring state rows that couple to the patch), with entries
// (patch-state column, index into a_blocks). Row pointers are local to j's entry range.
struct FactorLists {
  std::vector<int32_t> aj;       // [N] position of j in P(j)
  std::vector<int32_t> ng;       // [N] ring rows
  std::vector<int64_t> app_rp0;  // [N] first row pointer of A_PP in rp
  std::vector<int64_t> g_rp0;    // [N] first row pointer of G in rp
  std::vector<int64_t> app_e0;   // [N] first entry of A_PP in ecol/eidx
  std::vector<int64_t> g_e0;     // [N] first entry of G
  std::vector<int32_t> rp;       // concatenated row pointers (p*nx+1 then ng+1 per j)
  std::vector<int32_t> ecol, eidx;
};

inline int32_t padded_ld(int32_t D) { return (D + 3) & ~3; }

// Canonical Phi row of local row l of subsystem m.
inline int64_t canon_row(const HostSetup &h, int32_t m, int32_t l) {
  const int64_t Nx = int64_t(h.N) * h.nx, Nu = int64_t(h.N) * h.nu;
  if (l < h.nx * h.T) return int64_t(l / h.nx) * Nx + int64_t(m) * h.nx + (l % h.nx);
  const int32_t lu = l - h.nx * h.T;
  return Nx * h.T + int64_t(lu / h.nu) * Nu + int64_t(m) * h.nu + (lu % h.nu);
}

// Builds everything above except the factorisation (kdim, nb, off) on the host. Returns a
// DLMPC_* status; err gets a message.
int host_setup(const dlmpc_system *sys, int32_t d, int32_t T, const dlmpc_cost *cost,
               HostSetup &hs, std::string &err);

// FP64 factorisation of every column block by host threads (fills kdim, nb_off, nb, off_ptr,
// off and the sums).
int factor_host(HostSetup &hs, std::string &err);

// The same factorisation by HIP kernels on `device` (one workgroup per subsystem). The
// offsets come back to hs.off; the bases stay on the device in hs.d_nb.
int factor_device(HostSetup &hs, int device, double chol_tol, std::string &err);

// Releases hs.d_nb (no-op when null).
void free_factors_device(HostSetup &hs);

// Copies N_j (D x k_j column-major, leading dimension padded_ld(D)) to host memory `out`
// from hs.nb or hs.d_nb. Returns a DLMPC_* status.
int fetch_basis(const HostSetup &hs, int32_t j, std::vector<double> &out, std::string &err);

// Index lists of the per-subsystem factorisation (graph work only).
void factor_lists(const HostSetup &hs, FactorLists &fl);

// Sets kdim, nb_off, off_ptr and the sums from ks and sizes nb/off; copies nbs/offs (D x k and
// D x nx column-major per subsystem) into the zero-padded arrays, or leaves the arrays
// uninitialised when nbs/offs are empty (the caller fills every entry).
void pack_factors(HostSetup &hs, const std::vector<int> &ks, const std::vector<std::vector<double>> &nbs,
                  const std::vector<std::vector<double>> &offs);

}  // namespace dlmpc
