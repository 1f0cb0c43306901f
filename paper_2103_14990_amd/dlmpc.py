"""Python binding of libdlmpc (ctypes). Argument marshalling only: every step of the solve
runs in the library's HIP kernels. Names follow include/dlmpc.h.

The library must have been built (``python -m paper_2103_14990_amd.build``); loading fails
loudly otherwise — there is no fallback implementation.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import sys
import weakref
from dataclasses import dataclass

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "_lib", "libdlmpc.so")

OK, ENOCONV, EINVAL, ENOMEM, EDEVICE, EINFEASIBLE_LOCALITY, ENUMERIC = 0, 1, -1, -2, -3, -4, -5
FP64, FP32, FP32_BF16 = 0, 1, 2
FLAG_HOST_ONLY = 0x1
FLAG_SCHED_GRAPH = 0x2
FLAG_SCHED_PERSISTENT = 0x4
FLAG_HOST_FACTOR = 0x8
FLAG_NO_CHECK = 0x10
FLAG_NO_TUNE = 0x20
FLAG_SCHED_STEPWISE = 0x40
FLAG_SCHED_HOST_EXCHANGE = 0x80
FLAG_SCHED_NAIVE = 0x100
FLAG_STRUCTURED_PSI = 0x200
CL_SHIFT = 1
CL_SCALE_RHO = 2
FACTORS = {"device": 0, "host": FLAG_HOST_FACTOR}
SCHEDULES = {"auto": 0, "graph": FLAG_SCHED_GRAPH, "persistent": FLAG_SCHED_PERSISTENT,
             "stepwise": FLAG_SCHED_STEPWISE, "host_exchange": FLAG_SCHED_HOST_EXCHANGE, "naive": FLAG_SCHED_NAIVE}
SCHEDULE_NAMES = {0: "graph", 1: "persistent", 2: "batched", 3: "stepwise", 4: "host_exchange", 5: "naive"}
PRECISIONS = {"fp64": FP64, "fp32": FP32, "fp32_bf16": FP32_BF16}
TIMED_KERNELS = 4
KERNEL_NAMES = ("phi_kernel", "psi_pass1_kernel", "psi_pass2_kernel", "conv_kernel")
BATCH_KERNEL_NAMES = ("bphi_kernel", "bpsi_kernel", "bdecide_kernel")
STARTS = {"cold": 0, "alpha": 1, "trajectory": 2, "learned": 3, "state": 4}

_dp = C.POINTER(C.c_double)
_i64p = C.POINTER(C.c_int64)
_i32p = C.POINTER(C.c_int32)
_fp = C.POINTER(C.c_float)


class System(C.Structure):
    _fields_ = [("n_sub", C.c_int32), ("nx", C.c_int32), ("nu", C.c_int32),
                ("a_rowptr", _i64p), ("a_colidx", _i32p), ("a_blocks", _dp), ("b_blocks", _dp)]


class Cost(C.Structure):
    _fields_ = [("q_diag", _dp), ("r_diag", _dp), ("x_lo", _dp), ("x_hi", _dp), ("u_lo", _dp),
                ("u_hi", _dp)]


class Options(C.Structure):
    _fields_ = [("rho", C.c_double), ("eps", C.c_double), ("max_iter", C.c_int32),
                ("check_every", C.c_int32), ("precision", C.c_int32), ("device", C.c_int32),
                ("stream", C.c_void_p), ("flags", C.c_uint32), ("max_batch", C.c_int32),
                ("warm_cg_iters", C.c_int32), ("factor_chol_tol", C.c_double),
                ("warm_eps_scale", C.c_double)]


class Warm(C.Structure):
    _fields_ = [("psi0", _dp), ("lambda0", _dp)]


class Stats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32), ("r_primal", C.c_double),
                ("r_dual", C.c_double), ("objective", C.c_double), ("t_solve_ms", C.c_double),
                ("t_iter_ms", C.c_double), ("graph_launches", C.c_int32), ("schedule", C.c_int32),
                ("start", C.c_int32), ("fell_back", C.c_int32), ("t_warm_ms", C.c_double),
                ("kkt", C.c_double), ("eq_resid", C.c_double), ("u0_check", C.c_double),
                ("t_precompute_ms", C.c_double), ("t_check_ms", C.c_double), ("inner_iters", C.c_int32),
                ("pad", C.c_int32), ("coupling_viol", C.c_double)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class Cert(C.Structure):
    _fields_ = [("eq", C.c_double), ("pf", C.c_double), ("rp", C.c_double), ("box", C.c_double),
                ("stat", C.c_double)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class StreamInfo(C.Structure):
    _fields_ = [("joins", C.c_int32), ("checks", C.c_int32), ("slot_iterations", C.c_int64),
                ("instance_iterations", C.c_int64), ("fell_back", C.c_int32), ("pad", C.c_int32),
                ("t_stream_ms", C.c_double)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "pad"}


class Info(C.Structure):
    _fields_ = [("R", C.c_int64), ("n_cols", C.c_int64), ("nnz", C.c_int64), ("n_tiles", C.c_int64),
                ("d_row_max", C.c_int32), ("d_col_max", C.c_int32), ("p_max", C.c_int32),
                ("k_max", C.c_int32), ("sum_dcol_k", C.c_int64), ("sum_dcol2", C.c_int64),
                ("setup_ms", C.c_double), ("factor_ms", C.c_double), ("schedule", C.c_int32),
                ("persistent_grid", C.c_int32), ("tune_graph_us", C.c_double),
                ("tune_persistent_us", C.c_double), ("sum_k", C.c_int64),
                ("factor_device", C.c_int32), ("factor_fallbacks", C.c_int32),
                ("batch_phi_ntw", C.c_int32), ("batch_psi_capx", C.c_int32), ("batch_psi_units", C.c_int32),
                ("tune_cached", C.c_int32), ("tune_phi_us", C.c_double * 2), ("tune_psi_us", C.c_double * 6),
                ("psi_structured", C.c_int32), ("pad_info", C.c_int32), ("tune_structured_us", C.c_double),
                ("sum_du_k", C.c_int64)]

    def as_dict(self) -> dict:
        out = {}
        for f, _ in self._fields_:
            v = getattr(self, f)
            out[f] = list(v) if isinstance(v, C.Array) else v
        return out


EXPORTS = {
    "dlmpc_setup": (C.c_int, [C.POINTER(System), C.c_int32, C.c_int32, C.POINTER(Cost),
                              C.POINTER(Options), C.POINTER(C.c_void_p)]),
    "dlmpc_query": (C.c_int, [C.c_void_p, C.POINTER(Info)]),
    "dlmpc_phi_pattern": (C.c_int, [C.c_void_p, _i64p, _i32p]),
    "dlmpc_column_block": (C.c_int, [C.c_void_p, C.c_int32, _i32p, _i64p, _dp, _dp]),
    "dlmpc_solve": (C.c_int, [C.c_void_p, _dp, C.POINTER(Warm), _dp, _dp, C.POINTER(Stats)]),
    "dlmpc_solve_device": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(Stats)]),
    "dlmpc_certify": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(Cert)]),
    "dlmpc_time_kernels": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, _dp]),
    "dlmpc_time_batch_kernels": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, _dp]),
    "dlmpc_solve_batch": (C.c_int, [C.c_void_p, C.c_int32, _dp, _dp, C.POINTER(Stats)]),
    "dlmpc_solve_batch_device": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.POINTER(Stats)]),
    "dlmpc_solve_stream": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32,
                                     C.c_void_p, C.c_void_p]),
    "dlmpc_set_coupling": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                     C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_double, C.c_int32,
                                     C.c_double]),
    "dlmpc_set_rho": (C.c_int, [C.c_void_p, C.c_double]),
    "dlmpc_closed_loop": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.c_int32, C.c_void_p]),
    "dlmpc_solve_stream_noalloc": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32,
                                             C.c_void_p, C.c_void_p]),
    "dlmpc_solve_batch_ex": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32,
                                       C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(Stats)]),
    "dlmpc_ws_init": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_uint64, C.c_double, C.c_double]),
    "dlmpc_ws_shape": (C.c_int, [C.c_void_p, _i32p, _i32p, _i32p, _i64p]),
    "dlmpc_ws_params": (C.c_int, [C.c_void_p, _fp, _fp]),
    "dlmpc_ws_loss_grad": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, _dp, _fp]),
    "dlmpc_ws_train_step": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_double, _dp]),
    "dlmpc_ws_predict": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "dlmpc_ws_save": (C.c_int, [C.c_void_p, C.c_char_p]),
    "dlmpc_warmstart_load": (C.c_int, [C.c_void_p, C.c_char_p]),
    "dlmpc_group_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int32, C.POINTER(C.c_void_p)]),
    "dlmpc_group_solve_batch": (C.c_int, [C.c_void_p, _i32p, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                          C.POINTER(C.POINTER(Stats))]),
    "dlmpc_group_destroy": (None, [C.c_void_p]),
    "dlmpc_destroy": (None, [C.c_void_p]),
    "dlmpc_status_string": (C.c_char_p, [C.c_int]),
    "dlmpc_last_error": (C.c_char_p, []),
}

_lib: C.CDLL | None = None
# Live handles, released at interpreter exit before the HIP runtime goes away (the hook is
# registered when the library is loaded, i.e. after torch's own exit hooks, so it runs first).
_LIVE: "weakref.WeakSet" = weakref.WeakSet()


def _close_all():
    for obj in sorted(list(_LIVE), key=lambda o: 0 if isinstance(o, Group) else 1):
        try:
            obj.close()
        except Exception:
            pass


def load(path: str | None = None) -> C.CDLL:
    """Loads the built library (raises if it is missing: there is no CPU fallback)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"libdlmpc not built at {p}; run python -m paper_2103_14990_amd.build")
    # One HIP runtime per process: torch ships its own libamdhip64.so.7, and the library must
    # bind to that one (same soname) rather than load the system copy first.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(p)
    for name, (res, args) in EXPORTS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if path is None:
        _lib = lib
        atexit.register(_close_all)
    return lib


class DlmpcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"dlmpc status {status}: {msg}")
        self.status = status


def _ptr(a: np.ndarray | None, ctype=C.c_double):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(ctype))


def _f64(a) -> np.ndarray | None:
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


@dataclass
class SolveResult:
    status: int
    u0: np.ndarray
    phi: np.ndarray | None
    stats: dict

    @property
    def converged(self) -> bool:
        return self.status == OK


class Problem:
    """One DLMPC problem resident on a device (dlmpc_setup ... dlmpc_destroy)."""

    def __init__(self, n_sub: int, nx: int, nu: int, a_rowptr, a_colidx, a_blocks, b_blocks,
                 d: int, T: int, q_diag, r_diag, x_lo=None, x_hi=None, u_lo=None, u_hi=None,
                 rho: float = 5.0, eps: float = 1e-4, max_iter: int = 500, precision: str = "fp64",
                 device: int = 0, stream: int | None = None, check_every: int = 0,
                 host_only: bool = False, schedule: str = "auto", max_batch: int = 0,
                 warm_cg_iters: int = 0, factor: str = "device", factor_chol_tol: float = 0.0,
                 warm_eps_scale: float = 0.0, check: bool = True, tune: bool = True, flags: int = 0,
                 structured_psi: bool = False):
        self._lib = load()
        self._h = C.c_void_p()
        keep = dict(rowptr=np.ascontiguousarray(a_rowptr, dtype=np.int64),
                    colidx=np.ascontiguousarray(a_colidx, dtype=np.int32),
                    ab=_f64(np.reshape(a_blocks, -1)), bb=_f64(np.reshape(b_blocks, -1)),
                    q=_f64(q_diag), r=_f64(r_diag), xl=_f64(x_lo), xh=_f64(x_hi), ul=_f64(u_lo),
                    uh=_f64(u_hi))
        sysd = System(n_sub, nx, nu, _ptr(keep["rowptr"], C.c_int64), _ptr(keep["colidx"], C.c_int32),
                      _ptr(keep["ab"]), _ptr(keep["bb"]))
        cost = Cost(_ptr(keep["q"]), _ptr(keep["r"]), _ptr(keep["xl"]), _ptr(keep["xh"]),
                    _ptr(keep["ul"]), _ptr(keep["uh"]))
        opts = Options(rho, eps, max_iter, check_every, PRECISIONS[precision], device,
                       C.c_void_p(stream) if stream else None,
                       (FLAG_HOST_ONLY if host_only else 0) | SCHEDULES[schedule] | FACTORS[factor]
                       | (0 if check else FLAG_NO_CHECK) | (0 if tune else FLAG_NO_TUNE) | flags
                       | (FLAG_STRUCTURED_PSI if structured_psi else 0), max_batch,
                       warm_cg_iters, factor_chol_tol, warm_eps_scale)
        st = self._lib.dlmpc_setup(C.byref(sysd), d, T, C.byref(cost), C.byref(opts), C.byref(self._h))
        if st != OK:
            raise DlmpcError(st, self._lib.dlmpc_last_error().decode())
        self.n_sub, self.nx, self.nu, self.d, self.T = n_sub, nx, nu, d, T
        self.precision = precision
        inf = Info()
        self._check(self._lib.dlmpc_query(self._h, C.byref(inf)))
        self.info = inf.as_dict()
        _LIVE.add(self)

    @classmethod
    def from_network(cls, net, d: int, T: int, cost, **kw) -> "Problem":
        return cls(net.n_sub, net.nx, net.nu, net.a_rowptr, net.a_colidx, net.a_blocks,
                   net.b_blocks, d, T, cost.q_diag, cost.r_diag, cost.x_lo, cost.x_hi, cost.u_lo,
                   cost.u_hi, **kw)

    def _check(self, st: int) -> int:
        if st < 0:
            raise DlmpcError(st, self._lib.dlmpc_last_error().decode())
        return st

    @property
    def nnz(self) -> int:
        return int(self.info["nnz"])

    def phi_pattern(self):
        rp = np.zeros(self.info["R"] + 1, dtype=np.int64)
        ci = np.zeros(self.nnz, dtype=np.int32)
        self._check(self._lib.dlmpc_phi_pattern(self._h, _ptr(rp, C.c_int64), _ptr(ci, C.c_int32)))
        return rp, ci

    def column_block(self, j: int, want_P: bool = True):
        D = C.c_int32()
        self._check(self._lib.dlmpc_column_block(self._h, j, C.byref(D), None, None, None))
        D = D.value
        rows = np.zeros(D, dtype=np.int64)
        P = np.zeros((D, D)) if want_P else None
        O = np.zeros((D, self.nx))
        self._check(self._lib.dlmpc_column_block(self._h, j, None, _ptr(rows, C.c_int64), _ptr(P), _ptr(O)))
        return rows, P, O

    def solve(self, x0, psi0=None, lambda0=None, want_phi: bool = False) -> SolveResult:
        x0 = _f64(x0)
        u0 = np.zeros(self.n_sub * self.nu)
        phi = np.zeros(self.nnz) if want_phi else None
        st = Stats()
        warm = None
        if psi0 is not None or lambda0 is not None:
            p0, l0 = _f64(psi0), _f64(lambda0)
            warm = Warm(_ptr(p0), _ptr(l0))
            self._keep_warm = (p0, l0)
        s = self._check(self._lib.dlmpc_solve(self._h, _ptr(x0), C.byref(warm) if warm else None,
                                              _ptr(u0), _ptr(phi), C.byref(st)))
        return SolveResult(s, u0, phi, st.as_dict())

    def solve_device(self, x0_dev: int, u0_dev: int, phi_dev: int = 0) -> tuple[int, dict]:
        """Device pointers (e.g. ``tensor.data_ptr()`` of float64 tensors on the problem's device)."""
        st = Stats()
        s = self._check(self._lib.dlmpc_solve_device(self._h, C.c_void_p(x0_dev), C.c_void_p(u0_dev),
                                                     C.c_void_p(phi_dev) if phi_dev else None,
                                                     C.byref(st)))
        return s, st.as_dict()

    def solve_batch(self, x0s) -> tuple[int, np.ndarray, list[dict]]:
        """x0s [B, N*nx] -> (status, u0 [B, N*nu], per-instance stats)."""
        x0s = np.ascontiguousarray(x0s, dtype=np.float64)
        B = x0s.shape[0]
        u0 = np.zeros((B, self.n_sub * self.nu))
        st = (Stats * B)()
        s = self._check(self._lib.dlmpc_solve_batch(self._h, B, _ptr(x0s), _ptr(u0), st))
        return s, u0, [x.as_dict() for x in st]

    def solve_batch_device(self, B: int, x0_dev: int, u0_dev: int) -> tuple[int, list[dict]]:
        st = (Stats * B)()
        s = self._check(self._lib.dlmpc_solve_batch_device(self._h, B, C.c_void_p(x0_dev),
                                                           C.c_void_p(u0_dev), st))
        return s, [x.as_dict() for x in st]

    def solve_batch_ex(self, B: int, x0_dev: int, u0_dev: int, start: str = "cold", start_dev: int = 0,
                       y_out_dev: int = 0, alpha_out_dev: int = 0) -> tuple[int, list[dict]]:
        """Batched solve from the cold start, given row multipliers (``start="alpha"``), a given
        input trajectory (``"trajectory"``) or the warm-start network (``"learned"``); device
        pointers of float64 buffers ([B][R] for start_dev, y_out_dev, alpha_out_dev)."""
        st = (Stats * B)()
        opt = lambda v: C.c_void_p(v) if v else None  # noqa: E731
        s = self._check(self._lib.dlmpc_solve_batch_ex(
            self._h, B, C.c_void_p(x0_dev), C.c_void_p(u0_dev), STARTS[start], opt(start_dev),
            opt(y_out_dev), opt(alpha_out_dev), st))
        return s, [x.as_dict() for x in st]

    def solve_stream(self, n: int, x0_dev: int, u0_dev: int, refill_min: int = 0,
                     check_iters: int = 0) -> tuple[int, list[dict], dict]:
        """n instances streamed through the batched engine's slots from the learned start
        (device pointers of float64 [n][N*nx] and [n][N*nu]); returns (status, per-instance
        stats, stream counters)."""
        st = (Stats * n)()
        info = StreamInfo()
        s = self._check(self._lib.dlmpc_solve_stream(self._h, n, C.c_void_p(x0_dev), C.c_void_p(u0_dev),
                                                      refill_min, check_iters, st, C.byref(info)))
        return s, [x.as_dict() for x in st], info.as_dict()

    def closed_loop(self, B: int, T_sim: int, x0_dev: int, xs_dev: int, us_dev: int,
                    warm: bool = False, scale_rho: bool = False) -> tuple[int, list[list[dict]]]:
        """B closed loops of T_sim steps (Algorithm 1) from x0_dev [B][N*nx]; xs_dev
        [B][T_sim+1][N*nx] and us_dev [B][T_sim][N*nu] receive the state and input trajectories
        (device pointers of float64 buffers). warm: shifted start (CL_SHIFT); scale_rho: penalty
        rho ||x(t)||^2 / ||x(0)||^2 (CL_SCALE_RHO). Returns (status, stats[t][b])."""
        st = (Stats * (B * T_sim))()
        mode = (CL_SHIFT if warm else 0) | (CL_SCALE_RHO if scale_rho else 0)
        s = self._check(self._lib.dlmpc_closed_loop(self._h, B, T_sim, C.c_void_p(x0_dev), C.c_void_p(xs_dev),
                                                     C.c_void_p(us_dev), mode, st))
        flat = [x.as_dict() for x in st]
        return s, [flat[t * B:(t + 1) * B] for t in range(T_sim)]

    def set_coupling(self, row_a, row_b, lo, hi, sigma: float = 1.0, inner_max: int = 50,
                     inner_eps: float = 1e-9) -> None:
        """Neighbour-coupled constraints lo <= y[row_a] - y[row_b] <= hi on canonical rows of
        Phi x0 for the single-instance solves (dlmpc_set_coupling); empty arrays remove them."""
        ra = np.ascontiguousarray(row_a, dtype=np.int64)
        rb = np.ascontiguousarray(row_b, dtype=np.int64)
        lo_, hi_ = _f64(lo), _f64(hi)
        n = len(ra)
        if not (len(rb) == n and len(lo_) == n and len(hi_) == n):
            raise ValueError("row_a, row_b, lo, hi must have one entry per coupling")
        self._check(self._lib.dlmpc_set_coupling(self._h, n, _ptr(ra, C.c_int64), _ptr(rb, C.c_int64), _ptr(lo_),
                                                 _ptr(hi_), float(sigma), int(inner_max), float(inner_eps)))
        self._coupling = (ra, rb, lo_, hi_)

    def set_rho(self, rho: float) -> None:
        """Penalty of every solve started after this call (dlmpc_set_rho)."""
        self._check(self._lib.dlmpc_set_rho(self._h, float(rho)))

    def solve_stream_noalloc(self, n: int, x0_dev: int, u0_dev: int, refill_min: int = 0,
                             check_iters: int = 0) -> tuple[int, list[dict], dict]:
        """solve_stream without device allocation (static staging array of the library; calls
        that overlap on one GPU race on it)."""
        st = (Stats * n)()
        info = StreamInfo()
        s = self._check(self._lib.dlmpc_solve_stream_noalloc(self._h, n, C.c_void_p(x0_dev), C.c_void_p(u0_dev),
                                                              refill_min, check_iters, st, C.byref(info)))
        return s, [x.as_dict() for x in st], info.as_dict()

    # ---- learned warm start
    def ws_init(self, hidden: int, max_samples: int, seed: int = 0, x_scale: float = 1.0,
                y_scale: float = 1.0):
        self._check(self._lib.dlmpc_ws_init(self._h, hidden, max_samples, seed, x_scale, y_scale))

    def ws_shape(self) -> dict:
        i, h, o, n = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int64()
        self._check(self._lib.dlmpc_ws_shape(self._h, C.byref(i), C.byref(h), C.byref(o), C.byref(n)))
        return dict(IN=i.value, H=h.value, OUT=o.value, n_params=n.value)

    def ws_params(self, set_to=None) -> np.ndarray:
        """Returns the current flat FP32 parameters; sets them afterwards if ``set_to`` is given."""
        out = np.zeros(self.ws_shape()["n_params"], dtype=np.float32)
        src = None if set_to is None else np.ascontiguousarray(set_to, dtype=np.float32)
        self._check(self._lib.dlmpc_ws_params(self._h, _ptr(out, C.c_float), _ptr(src, C.c_float)))
        return out

    def ws_loss_grad(self, S: int, x0_dev: int, y_dev: int, want_grad: bool = True):
        loss = C.c_double()
        g = np.zeros(self.ws_shape()["n_params"], dtype=np.float32) if want_grad else None
        self._check(self._lib.dlmpc_ws_loss_grad(self._h, S, C.c_void_p(x0_dev), C.c_void_p(y_dev),
                                                 C.byref(loss), _ptr(g, C.c_float)))
        return loss.value, g

    def ws_train_step(self, S: int, x0_dev: int, y_dev: int, lr: float) -> float:
        loss = C.c_double()
        self._check(self._lib.dlmpc_ws_train_step(self._h, S, C.c_void_p(x0_dev), C.c_void_p(y_dev),
                                                  lr, C.byref(loss)))
        return loss.value

    def ws_predict(self, S: int, x0_dev: int, y_dev: int):
        self._check(self._lib.dlmpc_ws_predict(self._h, S, C.c_void_p(x0_dev), C.c_void_p(y_dev)))

    def ws_save(self, path: str):
        self._check(self._lib.dlmpc_ws_save(self._h, os.fsencode(path)))

    def warmstart_load(self, path: str):
        self._check(self._lib.dlmpc_warmstart_load(self._h, os.fsencode(path)))

    def certify(self, x0_dev: int = 0) -> dict:
        """FP64 certificate of the latest single-instance solve (x0_dev 0: the latest host x0)."""
        c = Cert()
        self._check(self._lib.dlmpc_certify(self._h, C.c_void_p(x0_dev) if x0_dev else None, C.byref(c)))
        return c.as_dict()

    def time_kernels(self, x0_dev: int, iters: int) -> dict:
        """Mean microseconds per launch of each kernel of one iteration (no early stop)."""
        us = np.zeros(TIMED_KERNELS)
        self._check(self._lib.dlmpc_time_kernels(self._h, C.c_void_p(x0_dev), iters, _ptr(us)))
        return dict(zip(KERNEL_NAMES, us.tolist()))

    def time_batch_kernels(self, B: int, x0_dev: int, iters: int) -> dict:
        """Mean microseconds per launch of each batched-engine kernel (no early stop)."""
        us = np.zeros(len(BATCH_KERNEL_NAMES))
        self._check(self._lib.dlmpc_time_batch_kernels(self._h, B, C.c_void_p(x0_dev), iters, _ptr(us)))
        return dict(zip(BATCH_KERNEL_NAMES, us.tolist()))

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self._lib.dlmpc_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self, _finalizing=sys.is_finalizing):  # bound here: module globals may be gone at exit
        if _finalizing():  # the exit hook has closed every live handle
            return
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Group:
    """Batched problems of different networks advanced together (dlmpc_group_*)."""

    def __init__(self, problems: list):
        self._lib = load()
        self.problems = list(problems)
        arr = (C.c_void_p * len(self.problems))(*[p._h.value for p in self.problems])
        self._h = C.c_void_p()
        st = self._lib.dlmpc_group_create(arr, len(self.problems), C.byref(self._h))
        if st != OK:
            raise DlmpcError(st, self._lib.dlmpc_last_error().decode())
        _LIVE.add(self)

    def solve_batch_device(self, Bs: list[int], x0_devs: list[int], u0_devs: list[int]):
        n = len(self.problems)
        bs = (C.c_int32 * n)(*Bs)
        xs = (C.c_void_p * n)(*x0_devs)
        us = (C.c_void_p * n)(*u0_devs)
        st_arrays = [(Stats * b)() for b in Bs]
        sp = (C.POINTER(Stats) * n)(*[C.cast(a, C.POINTER(Stats)) for a in st_arrays])
        s = self._lib.dlmpc_group_solve_batch(self._h, bs, xs, us, sp)
        if s < 0:
            raise DlmpcError(s, self._lib.dlmpc_last_error().decode())
        return s, [[x.as_dict() for x in a] for a in st_arrays]

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self._lib.dlmpc_group_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self, _finalizing=sys.is_finalizing):  # bound here: module globals may be gone at exit
        if _finalizing():  # the exit hook has closed every live handle
            return
        try:
            self.close()
        except Exception:
            pass

