"""GPU parity of reads into user buffers and the Share Table (Sec. 3.4.1): every buffer
(or the holder's buffer a request shares) ends up holding its block's bytes of the store
image, whether the block was resident, being filled (the pending list, drained by the
completion service) or had to wait for a way; sharing gives one owner per live block;
released blocks get a new owner; the owner's writeback reaches the store after a flush.
Expected bytes come from the image itself and from the oracle's ordered unit writes."""
import numpy as np
import pytest

import oracle
from paper_2504_19365_amd import agile, gen

from gpu_helpers import check_quiescent_invariants, cuda, table_store

pytestmark = pytest.mark.gpu

ROWS, DIM = 65536, 64
NBLK = ROWS * DIM * 4 // 4096


@pytest.fixture(scope="module")
def image():
    buf = table_store(ROWS, DIM, [0])
    yield buf
    buf.free()


def _ctx(image, **kw):
    cfg = dict(cache_bytes=1 << 20, line_bytes=4096, assoc=8, num_qp=4, qp_depth=256,
               latency_ns=20_000, timeout_ns=int(10e9))
    cfg.update(kw)
    ctx = agile.Context(**cfg)
    ctx.open_store(image)
    return ctx


def _issue(ctx, blocks, share=False):
    import torch
    n = blocks.size
    pool = torch.zeros((n, 4096), dtype=torch.uint8, device="cuda")
    bufs = torch.arange(n, dtype=torch.int64, device="cuda") * 4096 + pool.data_ptr()
    ptrs = torch.zeros(n, dtype=torch.int64, device="cuda")
    status = torch.zeros(n, dtype=torch.int32, device="cuda")
    d_blocks = cuda(blocks.astype(np.uint64).view(np.int64))
    ctx.async_issue(d_blocks, bufs, ptrs, status, share=share)
    return pool, bufs, ptrs, status, d_blocks


def _held_bytes(pool, bufs, ptrs):
    """The 4 KiB each request's pointer designates (a pointer into the pool)."""
    base = pool.data_ptr()
    idx = ((ptrs - base) // 4096).cpu().numpy()
    assert np.all((ptrs.cpu().numpy() - base) % 4096 == 0)
    return pool.cpu().numpy()[idx]


def _expected(image, blocks):
    return image.array.reshape(-1, 4096)[blocks.astype(np.int64)]


@pytest.mark.parametrize("cache_kw", [dict(), dict(cache_bytes=8 * 4096, assoc=2)])
def test_private_copies_cold_then_warm(image, cache_kw):
    ctx = _ctx(image, **cache_kw)
    try:
        blocks = gen.uniform_blocks(5, 600, NBLK)  # repeats included
        for _ in range(2):  # cold (fills, pending lists), then resident
            pool, bufs, ptrs, status, _ = _issue(ctx, blocks)
            assert np.all(status.cpu().numpy() == agile.Context.BUF_PRIVATE)
            assert np.array_equal(ptrs.cpu().numpy(), bufs.cpu().numpy())
            assert np.array_equal(pool.cpu().numpy(), _expected(image, blocks))
        check_quiescent_invariants(ctx, cache_kw.get("assoc", 8))
    finally:
        ctx.close_store()
        ctx.shutdown()


def test_pending_lists_many_requests_per_line(image):
    """2,560 requests on 8 blocks with 100 us fills: most requests find their line being
    filled and wait on its pending list."""
    ctx = _ctx(image, latency_ns=100_000)
    try:
        rng = np.random.default_rng(3)
        blocks = rng.choice(rng.choice(NBLK, 8, replace=False), 2560).astype(np.uint64)
        pool, bufs, ptrs, status, _ = _issue(ctx, blocks)
        assert np.array_equal(pool.cpu().numpy(), _expected(image, blocks))
        st = ctx.stats()
        assert st["read_cmds"] == 8
        check_quiescent_invariants(ctx, 8)
    finally:
        ctx.close_store()
        ctx.shutdown()


def test_share_table_owner_sharers_release(image):
    ctx = _ctx(image)
    try:
        rng = np.random.default_rng(4)
        distinct = rng.choice(NBLK, 64, replace=False)
        blocks = rng.choice(distinct, 512).astype(np.uint64)
        pool, bufs, ptrs, status, d_blocks = _issue(ctx, blocks, share=True)
        s = status.cpu().numpy()
        p = ptrs.cpu().numpy()
        b = bufs.cpu().numpy()
        assert set(np.unique(s)) <= {agile.Context.BUF_OWNER, agile.Context.BUF_SHARED}
        for blk in np.unique(blocks):
            sel = np.nonzero(blocks == blk)[0]
            owners = sel[s[sel] == agile.Context.BUF_OWNER]
            assert owners.size == 1  # one owner per live block
            assert np.all(p[sel] == b[owners[0]])  # everyone points at the owner's buffer
        assert np.array_equal(_held_bytes(pool, bufs, ptrs), _expected(image, blocks))
        # while held, a second issue shares the same buffers
        pool2, bufs2, ptrs2, status2, d2 = _issue(ctx, blocks[:32], share=True)
        assert np.all(status2.cpu().numpy() == agile.Context.BUF_SHARED)
        assert np.all(np.isin(ptrs2.cpu().numpy(), b))
        ctx.buffers_release(d2, status2)
        ctx.buffers_release(d_blocks, status)
        # nothing held: the next requests own their blocks again, in their own buffers
        pool3, bufs3, ptrs3, status3, d3 = _issue(ctx, distinct.astype(np.uint64), share=True)
        assert np.all(status3.cpu().numpy() == agile.Context.BUF_OWNER)
        assert np.array_equal(ptrs3.cpu().numpy(), bufs3.cpu().numpy())
        assert np.array_equal(pool3.cpu().numpy(), _expected(image, distinct.astype(np.uint64)))
        ctx.buffers_release(d3, status3)
        check_quiescent_invariants(ctx, 8)
        # releasing again is more often than held
        with pytest.raises(agile.AgileError) as e:
            ctx.buffers_release(d3, status3)
        assert e.value.status == agile.ESTATE
    finally:
        ctx.shutdown()


def test_owner_writeback_reaches_the_store(image):
    import torch
    ctx = _ctx(image, cache_bytes=16 * 4096, assoc=4)  # small: written lines get evicted too
    try:
        ref = image.array.copy()
        rng = np.random.default_rng(6)
        blocks = rng.choice(NBLK, 200, replace=False).astype(np.uint64)
        pool, bufs, ptrs, status, d_blocks = _issue(ctx, blocks, share=True)
        new = rng.integers(0, 256, (blocks.size, 4096), dtype=np.uint8)
        pool.copy_(torch.from_numpy(new).cuda())  # the owners modify their buffers
        ctx.buffers_writeback(d_blocks, ptrs)
        ctx.flush()
        exp = oracle.write_units(ref, 4096, blocks, new)
        assert np.array_equal(image.array, exp)
        ctx.buffers_release(d_blocks, status)
        # and reads see the new bytes
        blocks2 = blocks[:50]
        pool2, _, _, _, _ = _issue(ctx, blocks2)
        assert np.array_equal(pool2.cpu().numpy(), exp.reshape(-1, 4096)[blocks2.astype(np.int64)])
        check_quiescent_invariants(ctx, 4)
    finally:
        ctx.close_store()
        ctx.shutdown()
        image.array[:] = ref  # the module's image back for the other tests
