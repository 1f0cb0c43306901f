"""Pins of the FP64 oracle against what the mathematics fixes (no GPU).

Each pin is independent of the oracle's own code path:
* Riccati LQR (centralised, unconstrained): for generic x0 and an actuator at every node the
  localised optimum has the centralised trajectory (eq. (MPC) without bounds);
* a dense quadratic program over the supported entries of Phi, built by simulating the plant
  (not through Z_AB) and certified by its KKT conditions (sparse x0 where locality binds, and
  box-constrained instances with active bounds);
* per-step properties of Algorithm 2: the Phi-comp row solve against a brute-force scalar
  minimisation, the Psi-comp projection against the KKT system of the projection, the
  Lambda identity, feasibility of Psi, the locality pattern, the dual closed form;
* Lemma 1 bounds on the generated graphs;
* planted mistakes in the oracle must break at least one pin.
"""
import numpy as np
import pytest
from scipy.optimize import linprog, minimize_scalar

from oracle import certify as C
from oracle import dlmpc_oracle as O
from paper_2103_14990_amd import workloads as W

RHO = 5.0


def _setup(net, d, T, cost):
    return O.setup_from_network(net, d, T, cost)


@pytest.fixture(scope="module")
def chain10():
    wl = W.workload("chain10")
    return wl, _setup(wl.net, wl.d, wl.T, wl.cost)


# --------------------------------------------------------------------------- LQR pins

@pytest.mark.parametrize("seed", [1, 2, 3])
def test_chain10_matches_riccati_lqr(chain10, seed):
    wl, pb = chain10
    x0 = wl.x0(seed)
    res = O.solve(pb, x0, rho=RHO, eps=1e-10, max_iter=20000)
    assert res.converged
    u0, J, y = C.lqr_riccati(wl.net.dense_A(), wl.net.dense_B(), wl.cost.q_diag, wl.cost.r_diag,
                             wl.T, x0)
    assert np.abs(res.u0 - u0).max() <= 1e-8 * np.abs(u0).max()
    assert abs(res.J - J) <= 1e-9 * J
    assert np.abs(res.y - y).max() <= 1e-8 * np.abs(y).max()


def test_grid4_d1_matches_riccati_lqr():
    net = W.grid(4)
    cost = W.unit_cost(net)
    pb = _setup(net, 1, 6, cost)
    x0 = W.x0(net, 7)
    res = O.solve(pb, x0, rho=RHO, eps=1e-10, max_iter=50000)
    u0, J, _ = C.lqr_riccati(net.dense_A(), net.dense_B(), cost.q_diag, cost.r_diag, 6, x0)
    assert res.converged
    assert np.abs(res.u0 - u0).max() <= 1e-7 * np.abs(u0).max()
    assert abs(res.J - J) <= 1e-9 * J


def test_eps_1e4_semantics(chain10):
    """At eps = 1e-4 the stopping iterate is close to, not at, the optimum."""
    wl, pb = chain10
    x0 = wl.x0(1)
    res = O.solve(pb, x0, rho=RHO, eps=1e-4, max_iter=500)
    u0, J, _ = C.lqr_riccati(wl.net.dense_A(), wl.net.dense_B(), wl.cost.q_diag, wl.cost.r_diag,
                             wl.T, x0)
    assert res.converged and 100 < res.iters < 400
    rel = np.abs(res.u0 - u0).max() / np.abs(u0).max()
    assert 1e-6 < rel < 5e-3


# --------------------------------------------------------------------------- dense QP pins

def test_sparse_x0_locality_binds(chain10):
    """x0 = e_0: the d-local optimum differs from LQR and equals the dense localised program."""
    wl, pb = chain10
    x0 = np.zeros(wl.net.n_sub * 2)
    x0[0] = 1.0
    res = O.solve(pb, x0, rho=RHO, eps=1e-10, max_iter=50000)
    A, B = wl.net.dense_A(), wl.net.dense_B()
    qp = C.localized_qp(A, B, 10, 2, 1, wl.d, wl.T, pb.w, x0)
    _, J_lqr, _ = C.lqr_riccati(A, B, wl.cost.q_diag, wl.cost.r_diag, wl.T, x0)
    assert max(qp.kkt.values()) < 1e-9
    assert np.abs(res.y - qp.y).max() < 1e-8
    assert abs(res.J - qp.J) < 1e-9 * qp.J
    assert qp.J > J_lqr * (1 + 1e-3)  # locality costs something here


@pytest.mark.parametrize("seed,n_active_min", [(9, 5), (10, 3)])
def test_box_constrained_matches_kkt_certified_qp(seed, n_active_min):
    """|theta| <= 0.8, |u| <= 0.3, x0 = 0.4 N(0, I): several bounds active at the optimum."""
    net = W.chain(10)
    cost = W.box_cost(net, theta_max=0.8, u_max=0.3)
    pb = _setup(net, 1, 5, cost)
    x0 = W.x0(net, seed, 0.4)
    qp = C.localized_qp(net.dense_A(), net.dense_B(), 10, 2, 1, 1, 5, pb.w, x0, pb.lb, pb.ub)
    assert max(qp.kkt.values()) < 1e-9
    assert len(qp.active_lower) + len(qp.active_upper) >= n_active_min
    res = O.solve(pb, x0, rho=RHO, eps=1e-10, max_iter=50000)
    assert res.converged
    assert np.abs(res.y - qp.y).max() < 1e-7
    assert abs(res.J - qp.J) < 1e-8 * qp.J
    # the clip binds exactly on the certified active rows
    assert np.allclose(res.y[qp.active_lower], pb.lb[qp.active_lower], atol=1e-12)
    assert np.allclose(res.y[qp.active_upper], pb.ub[qp.active_upper], atol=1e-12)


def test_infeasible_constrained_instance_does_not_converge():
    """x0 ~ N(0, I) with |theta| <= 0.8: theta(1) = theta(0) + dt omega(0) is beyond any input,
    the feasible set is empty (LP certificate) and ADMM must stop at max_iter unconverged."""
    net = W.chain(10)
    cost = W.box_cost(net)
    pb = _setup(net, 1, 5, cost)
    x0 = W.x0(net, 1, 1.0)
    theta1 = x0[0::2] + W.DT * x0[1::2]
    assert np.abs(theta1).max() > 0.8
    sls = C.dense_sls(net.dense_A(), net.dense_B(), 10, 2, 1, 1, 5, x0)
    bounded = np.isfinite(pb.ub)
    A_ub = np.vstack([sls.G[bounded], -sls.G[bounded]])
    b_ub = np.concatenate([pb.ub[bounded], -pb.lb[bounded]])
    lp = linprog(np.zeros(sls.G.shape[1]), A_ub=A_ub, b_ub=b_ub, A_eq=sls.E, b_eq=sls.f,
                 bounds=(None, None), method="highs")
    assert lp.status == 2  # infeasible
    res = O.solve(pb, x0, rho=RHO, eps=1e-4, max_iter=500)
    assert not res.converged and res.iters == 500


def test_infeasible_locality_detected():
    """A node without actuation cannot localise its own column: H_j o_c != e_c."""
    net = W.chain(6)
    net.b_blocks[2] = 0.0
    pb = _setup(net, 1, 5, W.unit_cost(net))
    assert not pb.feasible
    bad = [j for j, b in enumerate(pb.blocks) if b.feas_resid > O.FEASIBILITY_TOL]
    assert 2 in bad or 1 in bad or 3 in bad


# --------------------------------------------------------------------------- step pins

def test_phi_comp_row_solve_brute_force(chain10):
    """Each row of Phi-comp minimises w (phi.x)^2 + rho/2 ||phi - v||^2 on lb <= phi.x <= ub."""
    net = W.chain(10)
    cost = W.box_cost(net, theta_max=0.5, u_max=0.4)
    pb = _setup(net, 1, 5, cost)
    rng = np.random.default_rng(3)
    x0 = rng.standard_normal(20)
    Psi = rng.standard_normal(pb.mask.shape) * pb.mask
    Lam = rng.standard_normal(pb.mask.shape) * pb.mask
    Phi, s = O.phi_comp(pb, Psi, Lam, x0, RHO)
    assert np.all(Phi[~pb.mask] == 0)
    for r in range(0, pb.lay.R, 3):
        S = np.flatnonzero(pb.mask[r])
        x, v = x0[S], (Psi - Lam)[r, S]
        n = x @ x
        f = lambda t: pb.w[r] * t * t + 0.5 * RHO * (t - v @ x) ** 2 / n  # cost along phi = v + a x
        lo, hi = max(pb.lb[r], -1e3), min(pb.ub[r], 1e3)
        best = minimize_scalar(f, bounds=(lo, hi), method="bounded", options={"xatol": 1e-12})
        assert abs(s[r] - best.x) < 1e-7
        assert abs(Phi[r, S] @ x - s[r]) < 1e-12
        # phi - v is parallel to x (the component orthogonal to x is not penalised by the cost)
        dphi = Phi[r, S] - v
        assert np.linalg.norm(dphi - (dphi @ x) / n * x) < 1e-12


def test_psi_comp_is_projection(chain10):
    wl, pb = chain10
    Z = O.build_zab(pb.A, pb.B, pb.lay.T).toarray()
    rng = np.random.default_rng(5)
    for j, blk in enumerate(pb.blocks):
        H = Z[:, blk.rows]
        keep = np.any(H != 0, axis=1)
        H = H[keep]
        for c in range(2):
            e = np.zeros(Z.shape[0])
            e[2 * j + c] = 1.0
            e = e[keep]
            v = rng.standard_normal(len(blk.rows))
            psi = blk.P @ v + blk.O[:, c]
            ref = C.projection_by_kkt(H, v, e)
            assert np.abs(psi - ref).max() < 1e-8  # KKT matrix conditioning ~ sigma_min(H)^-2
            assert np.abs(H @ psi - e).max() < 1e-12


def test_iterate_invariants(chain10):
    """Z_AB Psi = I and the locality pattern hold at every iterate; Lambda obeys its update."""
    wl, pb = chain10
    x0 = wl.x0(2)
    Z = O.build_zab(pb.A, pb.B, pb.lay.T)
    rhs = np.zeros((Z.shape[0], pb.lay.Nx))
    rhs[:pb.lay.Nx] = np.eye(pb.lay.Nx)
    Psi = np.zeros((pb.lay.R, pb.lay.Nx))
    Lam = np.zeros_like(Psi)
    for _ in range(12):
        Phi, _ = O.phi_comp(pb, Psi, Lam, x0, RHO)
        Psi = O.psi_comp(pb, Phi, Lam)
        Lam_new = O.lambda_comp(Lam, Phi, Psi)
        assert np.array_equal(Lam_new, Lam + Phi - Psi)
        Lam = Lam_new
        assert np.abs(Z @ Psi - rhs).max() < 1e-12
        for M in (Phi, Psi, Lam):
            assert np.all(M[~pb.mask] == 0)


def test_dual_closed_form_at_optimum(chain10):
    """Unconstrained optimum: rho Lambda*[r, S_r] = -2 w_r y_r x_r (stationarity of Phi-comp)."""
    wl, pb = chain10
    x0 = wl.x0(3)
    res = O.solve(pb, x0, rho=RHO, eps=1e-11, max_iter=50000)
    Xr = pb.mask * x0[None, :]
    pred = -2.0 * (pb.w * res.y)[:, None] * Xr
    assert np.abs(RHO * res.Lam - pred).max() < 1e-8
    k = O.kkt_residuals(pb, res, x0, RHO)
    assert k["eq"] < 1e-12 and k["stat"] < 1e-9 and k["pattern"] == 0.0


def test_phi_nonunique_but_trajectory_unique(chain10):
    """Phi* is not unique (the cost sees Phi only through Phi x0); y, u(0) and J are."""
    wl, pb = chain10
    x0 = wl.x0(4)
    cold = O.solve(pb, x0, rho=RHO, eps=1e-11, max_iter=50000)
    rng = np.random.default_rng(11)
    warm = O.solve(pb, x0, rho=RHO, eps=1e-11, max_iter=50000,
                   psi0=rng.standard_normal(pb.mask.shape) * pb.mask,
                   lam0=rng.standard_normal(pb.mask.shape) * pb.mask)
    assert np.abs(cold.u0 - warm.u0).max() < 1e-8
    assert np.abs(cold.Phi - warm.Phi).max() > 1e-3


def test_zero_patch_x0_row_keeps_v():
    """x0 zero on a whole d-hop patch: those rows keep phi = v (their cost vanishes)."""
    net = W.chain(10)
    pb = _setup(net, 1, 5, W.unit_cost(net))
    x0 = W.x0(net, 1)
    x0[0:6] = 0.0  # nodes 0..2 -> node 0 and node 1 have all-zero patches (d = 1)
    rng = np.random.default_rng(1)
    Psi = rng.standard_normal(pb.mask.shape) * pb.mask
    Lam = rng.standard_normal(pb.mask.shape) * pb.mask
    Phi, s = O.phi_comp(pb, Psi, Lam, x0, RHO)
    rows = np.flatnonzero(np.isin(pb.lay.sub_of_row(), [0, 1]))
    assert np.array_equal(Phi[rows], (Psi - Lam)[rows])
    assert np.all(s[rows] == 0.0)


# --------------------------------------------------------------------------- Lemma 1

@pytest.mark.parametrize("name,d,T", [("chain10", 1, 5), ("grid16", 2, 10), ("irregular", 3, 15)])
def test_lemma1_bounds(name, d, T):
    net = {"chain10": lambda: W.chain(10), "grid16": lambda: W.grid(16),
           "irregular": lambda: W.irregular_mesh(32, 32, 0)}[name]()
    adj = [set() for _ in range(net.n_sub)]
    for a, b in net.edges:
        adj[a].add(int(b))
        adj[b].add(int(a))
    dist = O.hop_distances(adj)
    lay = O.Layout(net.n_sub, 2, 1, T)
    mask = O.locality_mask(dist, d, lay)
    d_row = int(mask.sum(axis=1).max())
    d_col = int(mask.sum(axis=0).max())
    b_row, b_col = O.lemma1_bounds(adj, d, T, s=2)
    assert d_row <= b_row and d_col <= b_col
    assert mask.shape == (2 * net.n_sub * T + net.n_sub * (T - 1), 2 * net.n_sub)


# --------------------------------------------------------------------------- planted mistakes

def test_planted_mistake_dropped_boundary_rows_fails_pin(chain10, monkeypatch):
    """Deleting the (d+1)-hop boundary rows of H_j (a plausible slip) breaks the LQR pin."""
    wl, _ = chain10
    orig = O.column_blocks

    def no_boundary(Z, mask, lay):
        blocks = orig(Z, mask, lay)
        out = []
        Zc = Z.tocsc()
        for j, b in enumerate(blocks):
            H = Zc[:, b.rows].toarray()
            keep = np.any(H != 0, axis=1)
            # keep only equations whose own state row lies inside the patch
            own = np.zeros(Z.shape[0], bool)
            own[b.rows[b.rows < Z.shape[0]]] = True
            Hk = H[keep & own]
            Hp = np.linalg.pinv(Hk)
            P = np.eye(len(b.rows)) - Hp @ Hk
            E = np.zeros((Z.shape[0], 2))
            E[2 * j, 0] = 1
            E[2 * j + 1, 1] = 1
            out.append(O.ColumnBlock(b.j, b.rows, P, Hp @ E[keep & own], b.rank, 0.0))
        return out

    monkeypatch.setattr(O, "column_blocks", no_boundary)
    pb = _setup(wl.net, wl.d, wl.T, wl.cost)
    x0 = np.zeros(20)
    x0[0] = 1.0
    res = O.solve(pb, x0, rho=RHO, eps=1e-10, max_iter=20000)
    qp = C.localized_qp(wl.net.dense_A(), wl.net.dense_B(), 10, 2, 1, wl.d, wl.T, pb.w, x0)
    assert np.abs(res.y - qp.y).max() > 1e-4


def test_planted_mistake_wrong_input_weight_fails_pin(chain10, monkeypatch):
    """Halving the weight of the input rows inside the row solve (a dropped factor on R)
    moves the fixed point off the LQR optimum."""
    wl, pb = chain10
    orig = O.phi_comp
    u_rows = np.arange(pb.lay.Nx * pb.lay.T, pb.lay.R)

    def bad(pb_, Psi, Lam, x0, rho):
        w = pb_.w
        pb_.w = w.copy()
        pb_.w[u_rows] *= 0.5
        try:
            return orig(pb_, Psi, Lam, x0, rho)
        finally:
            pb_.w = w

    monkeypatch.setattr(O, "phi_comp", bad)
    x0 = wl.x0(1)
    res = O.solve(pb, x0, rho=RHO, eps=1e-10, max_iter=20000)
    u0, J, _ = C.lqr_riccati(wl.net.dense_A(), wl.net.dense_B(), wl.cost.q_diag, wl.cost.r_diag,
                             wl.T, x0)
    assert np.abs(res.u0 - u0).max() > 1e-3 * np.abs(u0).max()


def test_planted_mistake_transposed_coupling_fails_pin(chain10, monkeypatch):
    """Building Z_AB with A' instead of A (a transposed operand) breaks the LQR pin."""
    wl, _ = chain10
    orig = O.build_zab
    monkeypatch.setattr(O, "build_zab", lambda A, B, T: orig(A.T.copy(), B, T))
    pb = _setup(wl.net, wl.d, wl.T, wl.cost)
    x0 = wl.x0(1)
    res = O.solve(pb, x0, rho=RHO, eps=1e-10, max_iter=20000)
    u0, _, _ = C.lqr_riccati(wl.net.dense_A(), wl.net.dense_B(), wl.cost.q_diag, wl.cost.r_diag,
                             wl.T, x0)
    assert np.abs(res.u0 - u0).max() > 1e-3 * np.abs(u0).max()
