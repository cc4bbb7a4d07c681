"""Pins of the CPU oracle's core functions against closed forms, library routines,
hand-worked traces and brute force (never against the oracle itself)."""
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import protocol_model as pm
from paper_2504_19365_amd import gen

U = 2.0 ** -24  # unit roundoff of fp32


def gamma(n):
    return n * U / (1 - n * U)


# ---------------------------------------------------------------- f_K (Sec. 4.2 compute)
@pytest.mark.parametrize("K", [0, 1, 7, 64, 512, 5000])
def test_fK_closed_form(K):
    a, b = float(np.float32(0.999)), float(np.float32(0.001))
    c = b / (1.0 - a)  # fixed point of v -> a v + b
    vs = gen.table(4, 64, seed=1).ravel()[:200]
    for v in vs:
        exact = c + a ** K * (float(v) - c)
        got = oracle.fK(float(v), K)
        # each step rounds once (<= U * |v_k| <= U * 2) and earlier errors decay by a
        bound = 2 * U * min(K, 2000) + 1e-30
        assert abs(got - exact) <= bound, (K, v, got, exact)
    assert oracle.fK(0.25, 0) == 0.25


def test_fK_single_step_exact_rounding():
    # one step is one correctly rounded fma: compare with exact rational arithmetic
    for v in gen.table(2, 32, seed=2).ravel():
        exact = Fraction(float(v)) * Fraction(float(np.float32(0.999))) + \
            Fraction(float(np.float32(0.001)))
        assert oracle.fK(float(v), 1) == _round_f32(exact)


def _round_f32(x: Fraction) -> float:
    """Round an exact rational to the nearest fp32 (ties to even)."""
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


# ---------------------------------------------------------------- gather
def test_gather_matches_numpy_view():
    rows, dim = 4096, 64
    tab = gen.table(rows, dim, seed=0)
    image = tab.view(np.uint8).ravel()
    idx = gen.zipf_rows(gen.zipf_cum(rows, 1.05), seed=0, count=1000)
    out = oracle.gather(image, dim * 4, idx)
    assert np.array_equal(out.view(np.float32).reshape(-1, dim), tab[idx])


# ---------------------------------------------------------------- embedding-bag forward
def _tables_image(rows, dim, T, seed0):
    tabs = [gen.table(rows, dim, seed=seed0 + t) for t in range(T)]
    return tabs, np.concatenate([t.ravel() for t in tabs]).view(np.uint8)


@pytest.mark.parametrize("K", [0, 3, 64])
def test_embbag_forward_vs_fp64_within_higham_bound(K):
    rows, dim, T, B = 2048, 16, 3, 40
    tabs, image = _tables_image(rows, dim, T, 20)
    off, idx = gen.embbag_batch(gen.zipf_cum(rows, 1.05), B, T, 1, 80, seed=3)
    got = oracle.embbag_forward(image, rows, dim, T, idx, off, B, K)
    a, b = float(np.float32(0.999)), float(np.float32(0.001))
    c = b / (1.0 - a)
    for g in range(B * T):
        t = g % T
        vals = tabs[t][idx[off[g]:off[g + 1]]].astype(np.float64)
        terms = c + a ** K * (vals - c)
        ref = terms.sum(axis=0)
        n = max(off[g + 1] - off[g], 1)
        bound = gamma(n) * np.abs(terms).sum(axis=0) + n * (2 * U * min(K, 2000)) * 1.01
        assert np.all(np.abs(got[g] - ref) <= bound + 1e-30), g


def test_embbag_forward_tiny_brute_force_bit_exact():
    rows, dim, T, B = 64, 8, 2, 6
    tabs, image = _tables_image(rows, dim, T, 7)
    off, idx = gen.embbag_batch(gen.zipf_cum(rows, 1.05), B, T, 1, 10, seed=4)
    got = oracle.embbag_forward(image, rows, dim, T, idx, off, B, 0)
    for g in range(B * T):
        acc = np.zeros(dim, dtype=np.float32)
        for j in range(off[g], off[g + 1]):
            acc = (acc + tabs[g % T][idx[j]]).astype(np.float32)
        assert np.array_equal(got[g], acc)
    sub = oracle.embbag_forward(image, rows, dim, T, idx, off, B, 0, bags=[5, 0, 7])
    assert np.array_equal(sub, got[[5, 0, 7]])


def test_embbag_forward_empty_bags():
    rows, dim = 16, 4
    _, image = _tables_image(rows, dim, 1, 0)
    off = np.array([0, 0, 2, 2], dtype=np.int64)
    idx = np.array([3, 3], dtype=np.int64)
    got = oracle.embbag_forward(image, rows, dim, 1, idx, off, 3, 0)
    assert np.all(got[0] == 0) and np.all(got[2] == 0)


# ---------------------------------------------------------------- backward + SGD
def test_backward_sgd_vs_dense_transpose_product():
    rows, dim, T, B, lr = 512, 8, 2, 128, 0.01
    tabs, image = _tables_image(rows, dim, T, 30)
    off, idx = gen.embbag_batch(gen.zipf_cum(rows, 1.1), B, T, 1, 40, seed=5)
    g = gen.normal_f32(31, B * T * dim).reshape(B * T, dim)
    upd = image.copy()
    uniq = oracle.embbag_backward_sgd(upd, rows, dim, T, idx, off, B, g, lr)
    # dense incidence A[g, t*rows + r] = multiplicity; grad = A^T g in fp64
    A = np.zeros((B * T, T * rows))
    for gb in range(B * T):
        for j in range(off[gb], off[gb + 1]):
            A[gb, (gb % T) * rows + idx[j]] += 1
    grad = A.T @ g.astype(np.float64)
    absg = np.abs(A).T @ np.abs(g.astype(np.float64))
    W0 = np.concatenate([t for t in tabs]).astype(np.float64)
    W1 = upd.view(np.float32).reshape(T * rows, dim).astype(np.float64)
    touched = A.sum(axis=0) > 0
    assert uniq == int(touched.sum())
    assert np.array_equal(W1[~touched], W0[~touched])
    m = A.sum(axis=0).max()
    bound = lr * gamma(int(m)) * absg + 2 * U * np.abs(W0 - lr * grad) + 1e-12
    assert np.all(np.abs(W1 - (W0 - lr * grad)) <= bound)


def test_backward_sgd_tiny_brute_force_bit_exact():
    # The update of every touched row is pinned bit for bit: the gradient summed in fp32
    # from +0.0f over the row's occurrences in ascending lookup position, then one
    # correctly rounded fused multiply-add w' = round(w - lr * g), here from exact
    # rationals.  The data are chosen so that a plausible slip is caught: summing the
    # occurrences in another order, or rounding the product before the add, changes at
    # least one element.
    rows, dim, T, B = 64, 8, 2, 24
    tabs, image = _tables_image(rows, dim, T, 11)
    off, idx = gen.embbag_batch(gen.zipf_cum(rows, 1.1), B, T, 1, 12, seed=6)
    g = gen.normal_f32(33, B * T * dim).reshape(B * T, dim)
    lr = np.float32(0.01)
    upd = image.copy()
    uniq = oracle.embbag_backward_sgd(upd, rows, dim, T, idx, off, B, g, float(lr))
    occ = {}
    for gb in range(B * T):
        for j in range(off[gb], off[gb + 1]):
            occ.setdefault((gb % T, int(idx[j])), []).append((j, gb))
    assert uniq == len(occ)
    got = upd.view(np.float32).reshape(T, rows, dim)
    expect = np.stack(tabs).copy()
    order_sensitive = rounding_sensitive = False
    for (t, r), lst in occ.items():
        lst.sort()
        acc = np.zeros(dim, dtype=np.float32)
        for _, gb in lst:
            acc = (acc + g[gb]).astype(np.float32)
        rev = np.zeros(dim, dtype=np.float32)
        for _, gb in reversed(lst):
            rev = (rev + g[gb]).astype(np.float32)
        order_sensitive |= bool(np.any(rev != acc))
        for d in range(dim):
            w = Fraction(float(tabs[t][r, d]))
            exact = w - Fraction(float(lr)) * Fraction(float(acc[d]))
            expect[t, r, d] = np.float32(_round_f32(exact))
            two = np.float32(np.float32(tabs[t][r, d]) - np.float32(lr * acc[d]))
            rounding_sensitive |= bool(two != expect[t, r, d])
    assert order_sensitive and rounding_sensitive
    assert np.array_equal(got.view(np.uint32), expect.view(np.uint32))


def test_backward_matches_central_finite_differences():
    # L(W) = sum_g sum_d gout[g,d] * pooled[g,d] is linear in W, so the central
    # difference of L equals dL/dW up to the rounding of the fp32 pooled values.
    rows, dim, B = 256, 8, 64
    tab = gen.table(rows, dim, seed=0)
    image = tab.view(np.uint8).ravel().copy()
    off, idx = gen.embbag_batch(gen.zipf_cum(rows, 1.1), B, 1, 1, 40, seed=0)
    gout = gen.normal_f32(31, B * dim).reshape(B, dim)
    lr = 1.0
    upd = image.copy()
    oracle.embbag_backward_sgd(upd, rows, dim, 1, idx, off, B, gout, lr)
    grad = (image.view(np.float32) - upd.view(np.float32)).reshape(rows, dim).astype(np.float64)
    # the update used fmaf(-1, g, w): w - fl(w - g) recovers g up to rounding of w - g
    W = image.view(np.float32).reshape(rows, dim)

    def loss(img):
        p = oracle.embbag_forward(img, rows, dim, 1, idx, off, B, 0)
        return float((gout.astype(np.float64) * p.astype(np.float64)).sum())

    rng = np.random.default_rng(0)
    used = np.unique(idx)
    picks = [(int(r), int(d)) for r in rng.choice(used, 24) for d in rng.choice(dim, 1)]
    picks += [(int(r), 0) for r in np.setdiff1d(np.arange(rows), used)[:4]]
    for r, d in picks:
        w = W[r, d]
        wp, wm = np.float32(w + np.float32(1e-3)), np.float32(w - np.float32(1e-3))
        ip, im = image.copy(), image.copy()
        ip.view(np.float32)[r * dim + d] = wp
        im.view(np.float32)[r * dim + d] = wm
        fd = (loss(ip) - loss(im)) / (float(wp) - float(wm))
        gr = grad[r, d]
        assert abs(fd - gr) <= 1e-3 * max(1.0, abs(gr)) + 4 * U * (abs(w) + abs(gr)), (r, d)


# ---------------------------------------------------------------- Eq. 1
def test_eq1_hand_worked_points(golden_dir):
    for line in open(os.path.join(golden_dir, "eq1_points.txt")):
        if line.strip() and not line.startswith("#"):
            ctc, s = map(float, line.split())
            assert abs(oracle.eq1(ctc) - s) < 1e-12
    # continuous at CTC = 1 and maximal there
    assert abs(oracle.eq1(1 - 1e-9) - oracle.eq1(1 + 1e-9)) < 1e-8
    xs = np.linspace(0, 5, 501)
    assert max(oracle.eq1(x) for x in xs) == oracle.eq1(1.0) == 2.0


# ---------------------------------------------------------------- clock simulator
def _load_traces(golden_dir):
    traces, cur = [], None
    for line in open(os.path.join(golden_dir, "clock_traces.txt")):
        p = line.split()
        if not p or p[0].startswith("#"):
            continue
        if p[0] == "trace":
            cur = dict(name=p[1], sets=int(p[2]), assoc=int(p[3]), acc=[], final={},
                       flush=None)
        elif p[0] == "a":
            cur["acc"].append((int(p[1]), p[2] == "W", int(p[3]), int(p[4])))
        elif p[0] == "flush":
            cur["flush"] = int(p[1])
        elif p[0] == "final":
            cur["final"][int(p[1])] = [int(x) for x in p[2:]]
        elif p[0] == "counts":
            cur["counts"] = [int(x) for x in p[1:]]
        elif p[0] == "end":
            traces.append(cur)
    return traces


def test_clock_hand_worked_traces(golden_dir):
    traces = _load_traces(golden_dir)
    assert len(traces) == 3
    for tr in traces:
        c = oracle.Clock(tr["sets"], tr["assoc"])
        for line, w, hit, way in tr["acc"]:
            assert c.access(line, w) == (bool(hit), way), tr["name"]
        if tr["flush"] is not None:
            assert c.flush() == tr["flush"]
        tags, dirty = c.state()
        for s, exp in tr["final"].items():
            assert list(tags[s]) == exp, tr["name"]
        cnt = c.counters()
        assert [cnt["hits"], cnt["misses"], cnt["wb_evict"], cnt["wb_flush"]] == tr["counts"]
        if tr["flush"] is not None:
            assert dirty.sum() == 0


def test_clock_invariants_on_zipf_trace():
    lines = gen.zipf_rows(gen.zipf_cum(4096, 1.05), seed=0, count=20_000) // 16
    c = oracle.Clock(32, 8)
    hit, way = c.run(lines)
    cnt = c.counters()
    assert cnt["hits"] + cnt["misses"] == lines.size
    assert cnt["misses"] >= np.unique(lines).size
    tags, _ = c.state()
    valid = tags[tags >= 0]
    assert valid.size == np.unique(valid).size
    assert np.all(tags[tags >= 0] % 32 == np.nonzero(tags >= 0)[0])
    # a cache at least as large as the working set misses exactly once per line
    big = oracle.Clock(1, 256)
    big.run(lines)
    assert big.counters()["misses"] == np.unique(lines).size


# ---------------------------------------------------------------- queue protocol model
@pytest.mark.parametrize("depth,window,reqs", [
    (2, 2, (1, 2)), (4, 2, (3, 2)), (4, 4, (2, 2, 1)), (2, 1, (3,)), (4, 2, (5,)),
])
def test_protocol_model_agile_has_no_deadlock(depth, window, reqs):
    n, dead = pm.explore("agile", depth, reqs, window=window)
    assert dead is None, dead
    assert n > 10


def test_protocol_model_ringing_only_after_all_writes_deadlocks():
    # a wave whose third command needs the slot of its own first command
    n, dead = pm.explore("agile_ring_last", 2, (3,), window=1)
    assert dead is not None
    n, dead = pm.explore("agile", 2, (3,), window=1)
    assert dead is None


def test_protocol_model_all_or_nothing_completion_posting_deadlocks():
    # a controller that posts its executed commands all at once (or none) can wait for
    # CQ room that only a full polling window frees
    n, dead = pm.explore("agile_batch_post", 4, (3, 2), window=4)
    assert dead is not None
    n, dead = pm.explore("agile", 4, (3, 2), window=4)
    assert dead is None


def test_protocol_model_naive_deadlocks_as_in_fig1():
    # Fig. 1: two threads each holding SQ entries, both spinning on a full queue
    n, dead = pm.explore("naive", 2, (2, 2))
    assert dead is not None
    # with enough room for everyone the naive design completes
    n, dead = pm.explore("naive", 4, (2, 2))
    assert dead is None


@pytest.mark.parametrize("controllers,total", [(2, 4), (3, 5)])
def test_protocol_model_shared_fetch_reads_fetch_pointer_first(controllers, total):
    # several controller wavefronts claim runs of one SQ with a compare-and-swap on its
    # fetch pointer; a doorbell read before the fetch pointer can be stale by then
    n, bad = pm.explore_fetch("db_first", controllers=controllers, total=total)
    assert bad is not None
    for order, guard in (("fetch_first", False), ("fetch_first", True), ("db_first", True)):
        n, bad = pm.explore_fetch(order, controllers=controllers, total=total, guard=guard)
        assert bad is None, (order, guard, bad)
        assert n > 100


# ---------------------------------------------------------------- all-cores CPU baseline
def test_parallel_forward_equals_oracle_bit_for_bit():
    rows, dim, T, B = 1024, 32, 4, 96
    _, image = _tables_image(rows, dim, T, 40)
    off, idx = gen.embbag_batch(gen.zipf_cum(rows, 1.05), B, T, 1, 80, seed=8)
    for K in (0, 5):
        a = oracle.embbag_forward(image, rows, dim, T, idx, off, B, K)
        b = oracle.embbag_forward_par(image, rows, dim, T, idx, off, B, K)
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    assert oracle.par_threads() >= 1
