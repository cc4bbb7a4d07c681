"""Input generators: published test vectors, closed forms and distribution properties."""
import math
import os

import numpy as np
import pytest

from paper_2504_19365_amd import gen


def test_splitmix64_published_vectors(golden_dir):
    rows = [l.split() for l in open(os.path.join(golden_dir, "splitmix64_seed0.txt"))
            if l.strip() and not l.startswith("#")]
    for i, h in rows:
        assert gen.u64(0, 0, int(i)) == int(h, 16)


def test_streams_and_seeds_differ():
    a = [gen.u64(3, gen.S_ZIPF, i) for i in range(4)]
    b = [gen.u64(3, gen.S_BAGLEN, i) for i in range(4)]
    c = [gen.u64(4, gen.S_ZIPF, i) for i in range(4)]
    assert len(set(a) | set(b) | set(c)) == 12


def test_table_values_closed_form():
    t = gen.table(257, 8, seed=5)
    k = (t.astype(np.float64) + 1.0) * 2.0 ** 23
    assert np.all(k == np.floor(k)) and k.min() >= 0 and k.max() < 2 ** 24
    assert t.min() >= -1.0 and t.max() < 1.0
    # element (r, d) uses draw r*dim + d of (seed, values stream): check one explicitly
    h = gen.u64(5, gen.S_VALUES, 100 * 8 + 3)
    assert t[100, 3] == np.float32((h >> 40) * 2.0 ** -23 - 1.0)
    # row-range fills agree with the whole-table fill
    part = np.empty((10, 8), dtype=np.float32)
    gen.fill_table(part.ctypes.data, 200, 10, 8, 5)
    assert np.array_equal(part, t[200:210])


def test_zipf_cdf_closed_form_and_picks():
    n, a = 1000, 1.05
    cum = gen.zipf_cum(n, a)
    ref = np.cumsum(np.arange(1, n + 1, dtype=np.float64) ** -a)
    assert np.allclose(cum, ref, rtol=1e-12, atol=0)
    assert gen.zipf_pick(cum, 0.0) == 0
    assert gen.zipf_pick(cum, np.nextafter(1.0, 0.0)) == n - 1
    # boundary: u exactly at cum[k]/total picks k+1
    assert gen.zipf_pick(cum, cum[3] / cum[-1]) >= 3


def test_zipf_frequencies_match_probabilities():
    n, a, m = 8, 1.05, 200_000
    cum = gen.zipf_cum(n, a)
    rows = gen.zipf_rows(cum, seed=11, count=m)
    p = np.arange(1, n + 1, dtype=np.float64) ** -a
    p /= p.sum()
    cnt = np.bincount(rows, minlength=n)
    sigma = np.sqrt(m * p * (1 - p))
    assert np.all(np.abs(cnt - m * p) < 5 * sigma)


def test_bag_lengths_and_batch_layout():
    cum = gen.zipf_cum(4096, 1.05)
    off, idx = gen.embbag_batch(cum, B=256, T=4, len_lo=1, len_hi=80, seed=9)
    lens = np.diff(off)
    assert off[0] == 0 and lens.min() >= 1 and lens.max() <= 80
    assert abs(lens.mean() - 40.5) < 2.0
    assert idx.size == off[-1] and idx.min() >= 0 and idx.max() < 4096
    ints = gen.uniform_int(9, gen.S_BAGLEN, 1024, 1, 80)
    assert np.array_equal(ints, lens)


def test_normal_moments():
    g = gen.normal_f32(31, 200_000).astype(np.float64)
    assert abs(g.mean()) < 0.01 and abs(g.var() - 1.0) < 0.02


def test_rmat_csr_shape_and_skew():
    scale, ef = 12, 16
    row_ptr, col, val = gen.rmat_csr(scale, ef, 0.57, 0.19, 0.19, seed=0)
    V = 1 << scale
    assert row_ptr[0] == 0 and row_ptr[-1] == V * ef and col.size == V * ef
    assert np.all(np.diff(row_ptr) >= 0)
    assert col.min() >= 0 and col.max() < V
    for v in range(0, V, 97):
        seg = col[row_ptr[v]:row_ptr[v + 1]]
        assert np.all(np.diff(seg) >= 0)
    deg = np.diff(row_ptr)
    assert deg.max() > 20 * deg.mean()  # RMAT skew
    assert val.min() >= 0 and val.max() < 1
    # uniform quadrants give a near-Poisson degree distribution
    rp2, _, _ = gen.rmat_csr(scale, ef, 0.25, 0.25, 0.25, seed=0)
    d2 = np.diff(rp2)
    assert d2.max() < 3 * d2.mean()
    # deterministic regardless of threads
    row_ptr_b, col_b, _ = gen.rmat_csr(scale, ef, 0.57, 0.19, 0.19, seed=0)
    assert np.array_equal(row_ptr, row_ptr_b) and np.array_equal(col, col_b)
    src = gen.bfs_source(0, row_ptr)
    assert 0 <= src < V and deg[src] >= 1


def test_requests_stream():
    t, n = gen.requests(40, 50_000, rate=20_000.0, max_log2=12)
    assert np.all(np.diff(t) > 0)
    assert abs(t[-1] / 50_000 - 1 / 20_000) < 0.03 / 20_000 * 5
    assert n.min() >= 1 and n.max() <= 4096
    lg = np.log2(n)
    assert abs(lg.mean() - 6.0) < 0.1


def test_uniform_blocks():
    b = gen.uniform_blocks(7, 100_000, 1000)
    assert b.min() >= 0 and b.max() < 1000
    assert abs(np.bincount(b, minlength=1000).std() - math.sqrt(100)) < 3
