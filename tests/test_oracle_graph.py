"""Pins of the oracle's BFS and SpMV: scipy routines, Graph500-style validation,
exact rational brute force, planted mistakes."""
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import shortest_path

import oracle
from paper_2504_19365_amd import gen

U = 2.0 ** -24


def _csr(scale, ef, abc=(0.57, 0.19, 0.19), seed=0):
    return gen.rmat_csr(scale, ef, *abc, seed=seed)


@pytest.mark.parametrize("scale,ef,abc", [(6, 4, (0.57, 0.19, 0.19)), (9, 8, (0.57, 0.19, 0.19)),
                                          (8, 2, (0.25, 0.25, 0.25))])
def test_bfs_levels_equal_unweighted_shortest_paths(scale, ef, abc):
    row_ptr, col, val = _csr(scale, ef, abc)
    V = row_ptr.size - 1
    src = gen.bfs_source(0, row_ptr)
    lev = oracle.bfs(row_ptr, col, src)
    A = sp.csr_matrix((np.ones(col.size), col, row_ptr), shape=(V, V))
    dist = shortest_path(A, directed=True, unweighted=True, indices=src)
    ref = np.where(np.isinf(dist), -1, dist).astype(np.int32)
    assert np.array_equal(lev, ref)
    assert oracle.bfs_validate(row_ptr, col, src, lev) == 0


def test_bfs_brute_force_tiny_graphs():
    rng = np.random.default_rng(1)
    for trial in range(20):
        V = int(rng.integers(1, 12))
        adj = rng.random((V, V)) < 0.25
        row_ptr = np.zeros(V + 1, dtype=np.int64)
        row_ptr[1:] = np.cumsum(adj.sum(axis=1))
        col = np.nonzero(adj)[1].astype(np.int32)
        src = int(rng.integers(0, V))
        # Floyd-Warshall on hop counts
        INF = 10 ** 9
        d = np.full((V, V), INF)
        np.fill_diagonal(d, 0)
        d[adj] = np.minimum(d[adj], 1)
        for k in range(V):
            d = np.minimum(d, d[:, [k]] + d[[k], :])
        ref = np.where(d[src] >= INF, -1, d[src]).astype(np.int32)
        assert np.array_equal(oracle.bfs(row_ptr, col, src), ref)


def test_bfs_validator_catches_planted_mistakes():
    row_ptr, col, _ = _csr(8, 8)
    src = gen.bfs_source(0, row_ptr)
    lev = oracle.bfs(row_ptr, col, src)
    assert oracle.bfs_validate(row_ptr, col, src, lev) == 0
    reached = np.nonzero(lev > 1)[0]
    bad = lev.copy()
    bad[src] = 1
    assert oracle.bfs_validate(row_ptr, col, src, bad) == 1
    bad = lev.copy()
    bad[reached[0]] += 1  # too deep: some in-edge violates level[v] <= level[u] + 1
    assert oracle.bfs_validate(row_ptr, col, src, bad) != 0
    bad = lev.copy()
    bad[reached[0]] = -1  # unreached although an in-neighbour is reached
    assert oracle.bfs_validate(row_ptr, col, src, bad) == 2
    bad = lev.copy()
    bad[reached[-1]] -= 1  # too shallow: no parent one level up
    assert oracle.bfs_validate(row_ptr, col, src, bad) != 0


def test_spmv_vs_scipy_fp64_within_bound():
    row_ptr, col, val = _csr(10, 16)
    V = row_ptr.size - 1
    x = gen.uniform_f32(1, gen.S_X, V, -1.0, 1.0)
    y = oracle.spmv(row_ptr, col, val, x)
    A = sp.csr_matrix((val.astype(np.float64), col, row_ptr), shape=(V, V))
    ref = A @ x.astype(np.float64)
    absA = sp.csr_matrix((np.abs(val.astype(np.float64)), col, row_ptr), shape=(V, V))
    mag = absA @ np.abs(x.astype(np.float64))
    n = np.diff(row_ptr)
    bound = (n * U / (1 - n * U)) * mag + 1e-30
    assert np.all(np.abs(y - ref) <= bound)
    part = oracle.spmv(row_ptr, col, val, x, 100, 200)
    assert np.array_equal(part, y[100:200])


def _round_f32(x: Fraction) -> float:
    if x == 0:
        return 0.0
    s = -1 if x < 0 else 1
    x = abs(x)
    e = 0
    while x >= 2 ** 24:
        x /= 2
        e += 1
    while x < 2 ** 23:
        x *= 2
        e -= 1
    m = int(x)
    r = x - m
    if r > Fraction(1, 2) or (r == Fraction(1, 2) and m % 2 == 1):
        m += 1
    return float(np.float32(s * m * 2.0 ** e))


def test_spmv_tiny_exact_rational_fma_fold():
    row_ptr, col, val = _csr(5, 4)
    V = row_ptr.size - 1
    x = gen.uniform_f32(2, gen.S_X, V, -1.0, 1.0)
    y = oracle.spmv(row_ptr, col, val, x)
    for i in range(V):
        acc = 0.0
        for k in range(row_ptr[i], row_ptr[i + 1]):
            acc = _round_f32(Fraction(float(val[k])) * Fraction(float(x[col[k]])) +
                             Fraction(acc))
        assert y[i] == np.float32(acc), i
