"""GPU parity of the next-batch prefetch forward (Sec. 4.3's asynchronous DLRM mode):
every batch of a sequence computed while the next one is prefetched equals the oracle
bit for bit, whatever the cache keeps of the prefetch (a cache that holds everything, a
cache so small that prefetched lines are evicted and full sets drop requests, an emulated
latency and IOPS cap); once a call has completed, the next batch's lines are resident
(the next call misses nothing) and nothing is pinned or in flight; the call that only
prefetches (B = 0) and the call that prefetches nothing (B_next = 0) behave as
documented."""
import numpy as np
import pytest

import oracle
from paper_2504_19365_amd import agile, gen

from gpu_helpers import check_quiescent_invariants, cuda, table_store

pytestmark = pytest.mark.gpu


def _batch(rows, T, B, seed, lo=1, hi=80, empty=()):
    off, idx = gen.embbag_batch(gen.zipf_cum(rows, 1.05), B, T, lo, hi, seed=seed)
    if empty:
        lens = np.diff(off)
        keep = np.ones(idx.size, dtype=bool)
        for b in empty:
            keep[off[b]:off[b + 1]] = False
            lens[b] = 0
        off = np.zeros(off.size, dtype=np.int64)
        np.cumsum(lens, out=off[1:])
        idx = idx[keep]
    return off, idx


def _lines(off, idx, T, rows, dim, line_bytes=4096):
    """Distinct cache lines of a batch (the index-to-block mapping of the store layout)."""
    t = np.repeat(np.arange(off.size - 1, dtype=np.int64) % T, np.diff(off))
    byte = (t * rows + idx) * (dim * 4)
    return np.unique(byte // line_bytes)


def _run_sequence(ctx, buf, rows, dim, T, B, K, seeds, check_resident):
    import torch
    tb = ctx.tables(rows, dim, T)
    batches = [_batch(rows, T, B, s, empty=(1, B * T - 2)) for s in seeds]
    dev = [(cuda(i), cuda(o)) for o, i in batches]
    for n, (off, idx) in enumerate(batches):
        out = torch.full((B * T, dim), float("nan"), device="cuda")
        if n + 1 < len(batches):
            ni, no = dev[n + 1]
            ctx.embbag_forward_prefetch(tb, dev[n][0], dev[n][1], B, K, out, ni, no, B)
        else:
            ctx.embbag_forward_prefetch(tb, dev[n][0], dev[n][1], B, K, out, None, None, 0)
        ctx.sync()
        ref = oracle.embbag_forward(buf.array, rows, dim, T, idx, off, B, K)
        got = out.cpu().numpy()
        assert np.array_equal(got.view(np.uint32), ref.view(np.uint32)), f"batch {n}"
        if check_resident and n + 1 < len(batches):
            tags = check_quiescent_invariants(ctx, ctx.info()["assoc"])[0]
            want = _lines(batches[n + 1][0], batches[n + 1][1], T, rows, dim)
            assert np.isin(want, tags).all(), f"batch {n + 1} not resident after the prefetch"


def test_prefetch_sequence_large_cache_next_batch_resident():
    rows, dim, T, B = 65536, 64, 4, 256
    buf = table_store(rows, dim, [1, 2, 3, 4])
    ctx = agile.Context(cache_bytes=64 << 20, line_bytes=4096, assoc=8, num_qp=8, qp_depth=256,
                        timeout_ns=int(10e9))
    try:
        ctx.open_store(buf)
        _run_sequence(ctx, buf, rows, dim, T, B, 0, [11, 12, 13, 14], check_resident=True)
    finally:
        ctx.close_store()
        ctx.shutdown()
        buf.free()


def test_prefetched_batch_misses_nothing():
    import torch
    rows, dim, T, B = 65536, 128, 2, 300
    buf = table_store(rows, dim, [5, 6])
    ctx = agile.Context(cache_bytes=64 << 20, line_bytes=4096, assoc=16, num_qp=4, qp_depth=256,
                        timeout_ns=int(10e9))
    try:
        ctx.open_store(buf)
        tb = ctx.tables(rows, dim, T)
        off, idx = _batch(rows, T, B, 21)
        di, do = cuda(idx), cuda(off)
        # B = 0: only the prefetch (no output, no offsets of a current batch)
        ctx.embbag_forward_prefetch(tb, None, None, 0, 0, None, di, do, B)
        ctx.sync()
        s0 = ctx.stats(reset=True)
        assert s0["read_cmds"] == _lines(off, idx, T, rows, dim).size
        out = torch.empty((B * T, dim), device="cuda")
        ctx.embbag_forward(tb, di, do, B, 3, out, mode=agile.MODE_SYNC)
        ctx.sync()
        s = ctx.stats(reset=True)
        assert s["misses"] == 0 and s["read_cmds"] == 0
        assert s["requests"] == idx.size and s["hits"] == idx.size
        ref = oracle.embbag_forward(buf.array, rows, dim, T, idx, off, B, 3)
        assert np.array_equal(out.cpu().numpy().view(np.uint32), ref.view(np.uint32))
        check_quiescent_invariants(ctx, 16)
    finally:
        ctx.close_store()
        ctx.shutdown()
        buf.free()


@pytest.mark.parametrize("dim", [32, 64, 256])
def test_prefetch_sequence_tiny_cache(dim):
    # 256 KiB, 4-way: each batch touches many times the cache, so the prefetch evicts lines
    # the current batch still needs, sets fill with lines in flight, requests are dropped
    rows, T, B = 32768, 3, 200
    buf = table_store(rows, dim, [7, 8, 9])
    ctx = agile.Context(cache_bytes=256 << 10, line_bytes=4096, assoc=4, num_qp=2, qp_depth=64,
                        timeout_ns=int(10e9))
    try:
        ctx.open_store(buf)
        _run_sequence(ctx, buf, rows, dim, T, B, 5, [31, 32, 33], check_resident=False)
        check_quiescent_invariants(ctx, 4)
    finally:
        ctx.close_store()
        ctx.shutdown()
        buf.free()


def test_prefetch_with_latency_and_cap_and_no_prefetch_call():
    import torch
    rows, dim, T, B = 65536, 64, 4, 512
    buf = table_store(rows, dim, [1, 3, 5, 7])
    ctx = agile.Context(cache_bytes=8 << 20, line_bytes=4096, assoc=16, num_qp=8, qp_depth=512,
                        latency_ns=20000, iops_cap=2_000_000, timeout_ns=int(10e9))
    try:
        ctx.open_store(buf)
        _run_sequence(ctx, buf, rows, dim, T, B, 64, [41, 42, 43], check_resident=False)
        # B_next = 0 is the plain asynchronous forward
        tb = ctx.tables(rows, dim, T)
        off, idx = _batch(rows, T, B, 44)
        a = torch.empty((B * T, dim), device="cuda")
        b = torch.empty((B * T, dim), device="cuda")
        ctx.invalidate()
        ctx.embbag_forward_prefetch(tb, cuda(idx), cuda(off), B, 2, a, None, None, 0)
        ctx.invalidate()
        ctx.embbag_forward(tb, cuda(idx), cuda(off), B, 2, b, mode=agile.MODE_ASYNC)
        ctx.sync()
        assert np.array_equal(a.cpu().numpy().view(np.uint32), b.cpu().numpy().view(np.uint32))
        check_quiescent_invariants(ctx, 16)
    finally:
        ctx.close_store()
        ctx.shutdown()
        buf.free()


def test_prefetch_next_batch_all_empty_and_rows_outside_store():
    import torch
    rows, dim, T, B = 4096, 64, 2, 64
    buf = table_store(rows, dim, [2, 4])
    ctx = agile.Context(cache_bytes=4 << 20, line_bytes=4096, assoc=8, num_qp=2, qp_depth=128,
                        timeout_ns=int(10e9))
    try:
        ctx.open_store(buf)
        tb = ctx.tables(rows, dim, T)
        off, idx = _batch(rows, T, B, 51)
        out = torch.empty((B * T, dim), device="cuda")
        # every next bag empty: the next lookups are never read (NULL indices)
        empty_off = np.zeros(B * T + 1, dtype=np.int64)
        ctx.embbag_forward_prefetch(tb, cuda(idx), cuda(off), B, 0, out, None, cuda(empty_off), B)
        ctx.sync()
        ref = oracle.embbag_forward(buf.array, rows, dim, T, idx, off, B, 0)
        assert np.array_equal(out.cpu().numpy().view(np.uint32), ref.view(np.uint32))
        # a prefetch of rows past the store is a hint: skipped, no error
        bad_idx = np.array([rows + 5, 3, 2 * rows], dtype=np.int64)
        bad_off = np.zeros(B * T + 1, dtype=np.int64)
        bad_off[-2] = 0
        bad_off[-1] = 3
        ctx.embbag_forward_prefetch(tb, cuda(idx), cuda(off), B, 0, out, cuda(bad_idx), cuda(bad_off), B)
        ctx.sync()
        assert np.array_equal(out.cpu().numpy().view(np.uint32), ref.view(np.uint32))
        check_quiescent_invariants(ctx, 8)
    finally:
        ctx.close_store()
        ctx.shutdown()
        buf.free()


def test_prefetch_finds_bags_across_runs_of_empty_bags():
    """The prefetch finds a lookup's bag (its table) 64 lookups at a time; a run of
    hundreds of empty bags inside a chunk, and empty bags at both ends, still give every
    lookup its own table: after a call that only prefetches, every distinct line of the
    batch is resident, each was read once, and computing the batch misses nothing."""
    import torch
    rows, dim, T, B = 65536, 64, 4, 256
    buf = table_store(rows, dim, [1, 2, 3, 4])
    ctx = agile.Context(cache_bytes=64 << 20, line_bytes=4096, assoc=8, num_qp=8, qp_depth=256,
                        timeout_ns=int(10e9))
    try:
        ctx.open_store(buf)
        tb = ctx.tables(rows, dim, T)
        empty = [0, 1] + list(range(5, 301)) + list(range(600, 700)) + [B * T - 1]
        off, idx = _batch(rows, T, B, 71, lo=1, hi=6, empty=tuple(empty))
        di, do = cuda(idx), cuda(off)
        ctx.embbag_forward_prefetch(tb, None, None, 0, 0, None, di, do, B)
        ctx.sync()
        want = _lines(off, idx, T, rows, dim)
        assert ctx.stats(reset=True)["read_cmds"] == want.size
        tags = check_quiescent_invariants(ctx, 8)[0]
        assert np.isin(want, tags).all()
        out = torch.empty((B * T, dim), device="cuda")
        ctx.embbag_forward(tb, di, do, B, 0, out, mode=agile.MODE_SYNC)
        ctx.sync()
        assert ctx.stats()["misses"] == 0
        ref = oracle.embbag_forward(buf.array, rows, dim, T, idx, off, B, 0)
        assert np.array_equal(out.cpu().numpy().view(np.uint32), ref.view(np.uint32))
    finally:
        ctx.close_store()
        ctx.shutdown()
        buf.free()


def test_prefetch_entry_points_edge_cases():
    """Serialized contexts prefetch nothing and still compute the batch exactly; a next
    batch without offsets is rejected before anything runs; the backward with no lookups
    only prefetches (its batch is then resident)."""
    import torch
    rows, dim, T, B = 4096, 64, 2, 64
    buf = table_store(rows, dim, [3, 5])
    try:
        off, idx = _batch(rows, T, B, 81)
        off2, idx2 = _batch(rows, T, B, 82)
        ref = oracle.embbag_forward(buf.array, rows, dim, T, idx, off, B, 0)
        # serialized: one lane in program order, no prefetch
        ctx = agile.Context(cache_bytes=4 << 20, line_bytes=4096, assoc=8, num_qp=1, qp_depth=64,
                            timeout_ns=int(10e9), flags=agile.F_SERIALIZED)
        try:
            ctx.open_store(buf)
            tb = ctx.tables(rows, dim, T)
            out = torch.empty((B * T, dim), device="cuda")
            ctx.embbag_forward_prefetch(tb, cuda(idx), cuda(off), B, 0, out, cuda(idx2), cuda(off2), B)
            ctx.sync()
            assert np.array_equal(out.cpu().numpy().view(np.uint32), ref.view(np.uint32))
            st = ctx.stats()
            assert st["read_cmds"] == _lines(off, idx, T, rows, dim).size  # this batch's only
        finally:
            ctx.close_store()
            ctx.shutdown()
        ctx = agile.Context(cache_bytes=4 << 20, line_bytes=4096, assoc=8, num_qp=2, qp_depth=128,
                            timeout_ns=int(10e9))
        try:
            ctx.open_store(buf)
            tb = ctx.tables(rows, dim, T)
            out = torch.empty((B * T, dim), device="cuda")
            with pytest.raises(agile.AgileError) as e:
                ctx.embbag_forward_prefetch(tb, cuda(idx), cuda(off), B, 0, out, cuda(idx2), None, B)
            assert e.value.status == agile.EINVAL
            with pytest.raises(agile.AgileError) as e:
                ctx.embbag_backward_sgd_prefetch(tb, cuda(idx), cuda(off), B,
                                                 torch.zeros((B * T, dim), device="cuda"), 0.01,
                                                 cuda(idx2), None, B)
            assert e.value.status == agile.EINVAL
            # no lookups to update: the call only prefetches the next batch
            ctx.stats(reset=True)
            empty_off = torch.zeros(B * T + 1, dtype=torch.int64, device="cuda")
            ctx.embbag_backward_sgd_prefetch(tb, torch.empty(0, dtype=torch.int64, device="cuda"),
                                             empty_off, B, torch.zeros((B * T, dim), device="cuda"),
                                             0.01, cuda(idx2), cuda(off2), B)
            ctx.sync()
            assert ctx.stats()["read_cmds"] == _lines(off2, idx2, T, rows, dim).size
            ctx.stats(reset=True)
            ctx.embbag_forward(tb, cuda(idx2), cuda(off2), B, 0, out, mode=agile.MODE_SYNC)
            ctx.sync()
            assert ctx.stats()["read_cmds"] == 0
            ref2 = oracle.embbag_forward(buf.array, rows, dim, T, idx2, off2, B, 0)
            assert np.array_equal(out.cpu().numpy().view(np.uint32), ref2.view(np.uint32))
            check_quiescent_invariants(ctx, 8)
        finally:
            ctx.close_store()
            ctx.shutdown()
    finally:
        buf.free()
