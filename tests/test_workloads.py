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
