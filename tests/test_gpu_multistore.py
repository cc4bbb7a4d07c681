"""GPU parity over several emulated devices (Sec. 4.3: request i goes to device i mod n):
a store striped line by line over 2 and 3 pinned images gives the oracle's results over
the logical image for the embedding-bag forward, the ticket reads, the write-through of
whole lines and the backward's write-backs; afterwards each device image equals the
oracle's split of the expected logical image.  Three fp32 tables of 65,536 x 64 (48 MiB,
12,288 lines of 4 KiB)."""
import ctypes as C

import numpy as np
import pytest

import oracle
from paper_2504_19365_amd import agile, gen

from gpu_helpers import (check_quiescent_invariants, cuda, device_bytes, dump_meta,
                         striped_store)

pytestmark = pytest.mark.gpu

ROWS, DIM, T = 65536, 64, 3
LINE = 4096


@pytest.fixture(scope="module")
def logical():
    tb = ROWS * DIM * 4
    x = np.empty(T * tb, dtype=np.uint8)
    for t in range(T):
        gen.fill_table(x.ctypes.data + t * tb, 0, ROWS, DIM, 40 + t)
    return x


def _ctx(**kw):
    cfg = dict(cache_bytes=1 << 20, line_bytes=LINE, assoc=8, num_qp=6, qp_depth=256,
               timeout_ns=int(10e9))
    cfg.update(kw)
    return agile.Context(**cfg)


def _open(ctx, x, n):
    bufs = striped_store(x, n, LINE)
    ctx.open_store_striped(bufs)
    return bufs


def _free(bufs):
    for b in bufs:
        b.free()


def _devices_equal(bufs, expected_logical, n):
    ref = oracle.stripe_split(expected_logical, n, LINE)
    return all(np.array_equal(b.array, r) for b, r in zip(bufs, ref))


@pytest.mark.parametrize("mode", [agile.MODE_SYNC, agile.MODE_ASYNC])
@pytest.mark.parametrize("n", [2, 3])
def test_forward_over_devices_equals_oracle(logical, n, mode):
    import torch
    ctx = _ctx()
    bufs = _open(ctx, logical, n)
    try:
        B, K = 512, 16
        off, idx = gen.embbag_batch(gen.zipf_cum(ROWS, 1.05), B, T, 1, 40, seed=5)
        out = torch.empty((B * T, DIM), dtype=torch.float32, device="cuda")
        ctx.stats(reset=True)
        ctx.embbag_forward(ctx.tables(ROWS, DIM, T), cuda(idx), cuda(off), B, K, out, mode=mode)
        ctx.sync()
        ref = oracle.embbag_forward(logical, ROWS, DIM, T, idx, off, B, K)
        assert np.array_equal(out.cpu().numpy().view(np.uint32), ref.view(np.uint32))
        st = ctx.stats()
        assert st["read_cmds"] > 0 and st["submitted"] == st["completed"]
        assert _devices_equal(bufs, logical, n)  # reads leave the images alone
        check_quiescent_invariants(ctx, 8)
    finally:
        ctx.close_store()
        ctx.shutdown()
        _free(bufs)


@pytest.mark.parametrize("n", [2, 3])
def test_prefetch_forward_over_devices_equals_oracle(logical, n):
    """A batch computed while the next is prefetched, over a store striped on n devices
    (each prefetched line goes to its own device's queue pairs): every batch equals the
    oracle, and a call that only prefetches a batch leaves all of its lines resident."""
    import torch
    ctx = _ctx(cache_bytes=48 << 20)
    bufs = _open(ctx, logical, n)
    try:
        B, K = 384, 8
        tb = ctx.tables(ROWS, DIM, T)
        cum = gen.zipf_cum(ROWS, 1.05)
        host = [gen.embbag_batch(cum, B, T, 1, 40, seed=60 + k) for k in range(3)]
        dev = [(cuda(o), cuda(i)) for o, i in host]
        for k in range(2):
            out = torch.empty((B * T, DIM), dtype=torch.float32, device="cuda")
            ctx.embbag_forward_prefetch(tb, dev[k][1], dev[k][0], B, K, out, dev[k + 1][1],
                                        dev[k + 1][0], B)
            ctx.sync()
            ref = oracle.embbag_forward(logical, ROWS, DIM, T, host[k][1], host[k][0], B, K)
            assert np.array_equal(out.cpu().numpy().view(np.uint32), ref.view(np.uint32)), k
        # batch 2 was prefetched by the last call: computing it reads nothing
        ctx.stats(reset=True)
        out = torch.empty((B * T, DIM), dtype=torch.float32, device="cuda")
        ctx.embbag_forward(tb, dev[2][1], dev[2][0], B, K, out, mode=agile.MODE_SYNC)
        ctx.sync()
        assert ctx.stats()["read_cmds"] == 0
        ref = oracle.embbag_forward(logical, ROWS, DIM, T, host[2][1], host[2][0], B, K)
        assert np.array_equal(out.cpu().numpy().view(np.uint32), ref.view(np.uint32))
        assert _devices_equal(bufs, logical, n)
        check_quiescent_invariants(ctx, 8)
    finally:
        ctx.close_store()
        ctx.shutdown()
        _free(bufs)


@pytest.mark.parametrize("n", [2, 3])
def test_ticket_reads_over_devices(logical, n):
    import torch
    ctx = _ctx(cache_bytes=16 << 20, num_qp=12, qp_depth=64)
    bufs = _open(ctx, logical, n)
    try:
        nblocks = logical.size // 4096
        blocks = gen.uniform_blocks(11, 200, nblocks)
        tk = torch.empty(blocks.size, dtype=torch.int64, device="cuda")
        ptr = torch.empty(blocks.size, dtype=torch.int64, device="cuda")
        ctx.async_read(cuda(blocks), tk)
        s = ctx.wait(tk, ptr)
        assert s == agile.OK
        info = ctx.info()
        cache = device_bytes(info["cache_base"], info["num_lines"] * 4096).cpu().numpy()
        p = ptr.cpu().numpy().view(np.uint64)
        for i, b in enumerate(blocks):
            off = int(p[i] - info["cache_base"])
            assert np.array_equal(cache[off:off + 4096], logical[int(b) * 4096:(int(b) + 1) * 4096]), i
        ctx.release(tk)
        ctx.sync()
        check_quiescent_invariants(ctx, 8)
    finally:
        ctx.close_store()
        ctx.shutdown()
        _free(bufs)


def _read_lines(ctx, lines, batch):
    """The cached content of each line, through the ticket calls (4 KiB lines), `batch`
    lines per call (one at a time when the cache is too small to hold a batch)."""
    import torch
    info = ctx.info()
    got = []
    for i in range(0, lines.size, batch):
        part = lines[i:i + batch]
        tk = torch.empty(part.size, dtype=torch.int64, device="cuda")
        ptr = torch.empty(part.size, dtype=torch.int64, device="cuda")
        ctx.async_read(cuda(part.astype(np.uint64).view(np.int64)), tk)
        assert ctx.wait(tk, ptr) == agile.OK
        cache = device_bytes(info["cache_base"], info["num_lines"] * 4096).cpu().numpy()
        for q in ptr.cpu().numpy().view(np.uint64):
            o = int(q - info["cache_base"])
            got.append(cache[o:o + 4096].copy())
        ctx.release(tk)
        ctx.sync()
    return np.stack(got)


@pytest.mark.parametrize("cache_kw", [dict(), dict(cache_bytes=8 * LINE, assoc=2)])
@pytest.mark.parametrize("n", [1, 2, 3])
def test_write_through_over_devices(logical, n, cache_kw):
    """Distinct random lines written through the cache (with a 1 MiB cache, and with an
    8-line cache where writes wait for ways), then 64 entries in one wavefront that name
    some lines twice (the later entry wins): the device images equal the oracle's split
    of the written logical image, the cache reads back the new bytes before and after an
    invalidate, and every distinct line cost one WRITE."""
    import torch
    ctx = _ctx(**cache_kw)
    bufs = _open(ctx, logical, n)
    try:
        nlines = logical.size // LINE
        rng = np.random.default_rng(20 + n)
        lines = rng.choice(nlines, 300, replace=False).astype(np.uint64)
        src = rng.integers(0, 256, (300, LINE), dtype=np.uint8)
        ctx.stats(reset=True)
        ctx.write(cuda(lines.view(np.int64)), cuda(src))
        st = ctx.stats()
        assert st["write_cmds"] == 300 and st["read_cmds"] == 0
        exp = oracle.write_units(logical, LINE, lines, src)
        assert _devices_equal(bufs, exp, n)
        batch = 40 if not cache_kw else 1
        assert np.array_equal(_read_lines(ctx, lines[:40], batch), src[:40])
        # duplicates inside one wavefront: the later entry is the one written
        dup = np.concatenate([lines[:32], lines[:32]])
        src2 = rng.integers(0, 256, (64, LINE), dtype=np.uint8)
        ctx.write(cuda(dup.view(np.int64)), cuda(src2))
        exp = oracle.write_units(exp, LINE, dup, src2)
        assert _devices_equal(bufs, exp, n)
        ctx.invalidate()
        assert np.array_equal(_read_lines(ctx, lines[:40], batch),
                              exp.reshape(-1, LINE)[lines[:40].astype(np.int64)])
        check_quiescent_invariants(ctx, cache_kw.get("assoc", 8))
    finally:
        ctx.close_store()
        ctx.shutdown()
        _free(bufs)


@pytest.mark.parametrize("n", [2, 3])
def test_backward_write_backs_over_devices(logical, n):
    """The backward's dirty lines go back to their own devices, on eviction (16-line
    cache) and at the flush."""
    ctx = _ctx(cache_bytes=16 * LINE, assoc=4)
    bufs = _open(ctx, logical, n)
    try:
        ref = logical.copy()
        tb = ctx.tables(ROWS, DIM, T)
        B, lr = 256, 0.01
        off, idx = gen.embbag_batch(gen.zipf_cum(ROWS, 1.1), B, T, 1, 40, seed=31)
        g = gen.normal_f32(32, B * T * DIM).reshape(B * T, DIM)
        ctx.stats(reset=True)
        ctx.embbag_backward_sgd(tb, cuda(idx), cuda(off), B, cuda(g), lr)
        ctx.sync()
        oracle.embbag_backward_sgd(ref, ROWS, DIM, T, idx, off, B, g, lr)
        assert ctx.stats()["wb_evict"] > 0
        ctx.flush()
        assert _devices_equal(bufs, ref, n)
        check_quiescent_invariants(ctx, 4)
    finally:
        ctx.close_store()
        ctx.shutdown()
        _free(bufs)


def test_striped_store_arguments(logical):
    bufs = striped_store(logical[:12 * LINE], 3, LINE)
    try:
        L = agile.lib()

        def open_raw(ctx, ptrs, n, nbytes):
            arr = (C.c_void_p * max(len(ptrs), 1))(*ptrs)
            h = C.c_void_p()
            return L.agile_open_store_striped(ctx.h, arr, n, nbytes, 4096, 0, C.byref(h))

        ptrs = [b.ptr for b in bufs]
        ctx = _ctx(num_qp=4)
        try:
            assert open_raw(ctx, ptrs, 0, 4 * LINE) == agile.EINVAL
            assert open_raw(ctx, ptrs * 3, 9, 4 * LINE) == agile.EINVAL
            assert open_raw(ctx, ptrs, 3, 4 * LINE) == agile.EINVAL  # 4 queue pairs, 3 devices
        finally:
            ctx.shutdown()
        ctx = _ctx(line_bytes=8192, num_qp=3)
        try:
            assert open_raw(ctx, ptrs, 3, 4 * LINE + 4096) == agile.EINVAL  # not whole lines
            assert open_raw(ctx, ptrs, 3, 4 * LINE) == agile.OK
        finally:
            ctx.shutdown()
    finally:
        _free(bufs)
