"""Seeded generator: determinism, topology shapes and the plant definition."""
import numpy as np
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import connected_components

from paper_2103_14990_amd import workloads as W


def test_deterministic():
    a, b = W.irregular_mesh(32, 32, 0), W.irregular_mesh(32, 32, 0)
    assert np.array_equal(a.edges, b.edges)
    assert np.array_equal(a.a_blocks, b.a_blocks)
    assert np.array_equal(W.x0(a, 5), W.x0(b, 5))
    assert not np.array_equal(W.x0(a, 5), W.x0(a, 6))


def test_grid_and_chain_edge_counts():
    assert len(W.chain(10).edges) == 9
    assert len(W.grid(16).edges) == 2 * 16 * 15
    assert len(W.grid(8).edges) == 2 * 8 * 7


def test_irregular_mesh_connected_with_chords():
    n = 1024
    net = W.irregular_mesh(32, 32, 0)
    grid_e = {tuple(e) for e in W.grid_edges(32, 32)}
    kept_grid = sum(1 for e in map(tuple, net.edges) if e in grid_e)
    chords = len(net.edges) - kept_grid
    assert kept_grid == len(grid_e) - round(0.3 * len(grid_e))
    assert chords == round(0.05 * n)
    adj = csr_matrix((np.ones(len(net.edges)), (net.edges[:, 0], net.edges[:, 1])), shape=(n, n))
    ncomp, _ = connected_components(adj, directed=False)
    assert ncomp == 1


def test_swing_plant_blocks():
    net = W.chain(4, seed=3)
    A = net.dense_A()
    dt = W.DT
    # theta row of every diagonal block is [1, dt]; coupling only enters the omega row
    for i in range(4):
        assert np.allclose(A[2 * i, 2 * i:2 * i + 2], [1.0, dt])
        others = np.delete(A[2 * i], [2 * i, 2 * i + 1])
        assert np.all(others == 0)
    # Laplacian coupling: omega row sums of the theta coefficients vanish
    assert np.allclose(A[1::2, 0::2].sum(axis=1), 0.0)
    B = net.dense_B()
    assert np.allclose(B[1::2].diagonal(), dt) and np.all(B[0::2] == 0)


def test_box_x0_first_step_inside_box():
    """On the box-constrained workloads theta_i(1) = theta_i(0) + dt omega_i(0) is beyond any
    input; every x0 the workloads hand out (bench, stored full-size values, held-out, training
    seeds) keeps it inside the box, and a passing draw is returned unchanged."""
    for name, seeds in (("irregular1024_box", list(range(1000, 1100)) + list(range(2000, 2200))
                         + list(range(2280, 7400, 7)) + list(range(10**6, 10**6 + 300))),
                        ("grid16_box", list(range(1000, 1100)) + list(range(2000, 2200)))):
        wl = W.workload(name)
        for s in seeds:
            x = wl.x0(s)
            assert not W.first_step_outside_box(wl.net, wl.cost, x), (name, s)
            th1 = x[0::2] + W.DT * x[1::2]
            assert np.abs(th1).max() <= 0.8
    wl = W.workload("irregular1024_box")
    raw = W.x0(wl.net, 4605, wl.sigma)  # the one draw of the bench range that leaves the box
    assert W.first_step_outside_box(wl.net, wl.cost, raw)
    assert not np.array_equal(wl.x0(4605), raw)
    assert np.array_equal(wl.x0(1000), W.x0(wl.net, 1000, wl.sigma))
