"""GPU parity for the tiny plain-method configuration: one 65,536 x 64 fp32 table (16 MiB
store, 4 KiB blocks) in pinned memory, a 1 MiB HBM cache of 256 lines (8-way), one queue
pair of depth 64, no emulated latency; 4,096 Zipf(1.05) lookups from seed 0.  Expected
values come from the oracle and from direct reads of the store image."""
import numpy as np
import pytest

import oracle
from paper_2504_19365_amd import agile, gen

from gpu_helpers import (check_quiescent_invariants, cuda, device_bytes, dump_meta,
                         table_store)

pytestmark = pytest.mark.gpu

ROWS, DIM = 65536, 64


@pytest.fixture(scope="module")
def image():
    buf = table_store(ROWS, DIM, [0])
    yield buf
    buf.free()


@pytest.fixture(scope="module")
def lookups():
    return gen.zipf_rows(gen.zipf_cum(ROWS, 1.05), seed=0, count=4096)


def make_ctx(image, **kw):
    cfg = dict(cache_bytes=1 << 20, line_bytes=4096, assoc=8, num_qp=1, qp_depth=64,
               timeout_ns=int(5e9))
    cfg.update(kw)
    ctx = agile.Context(**cfg)
    ctx.open_store(image)
    return ctx


@pytest.mark.parametrize("mode", [agile.MODE_SYNC, agile.MODE_ASYNC])
def test_gather_bit_exact(image, lookups, mode):
    import torch
    ctx = make_ctx(image)
    try:
        idx = cuda(lookups)
        out = torch.empty((lookups.size, DIM), dtype=torch.float32, device="cuda")
        ctx.stats(reset=True)
        ctx.gather(ctx.tables(ROWS, DIM), idx, out, mode=mode)
        ctx.sync()
        got = out.cpu().numpy()
        ref = oracle.gather(image.array, DIM * 4, lookups).view(np.float32).reshape(-1, DIM)
        assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))
        # brute force: the image itself
        assert np.array_equal(got, image.array[:ROWS * DIM * 4].view(np.float32)
                              .reshape(ROWS, DIM)[lookups])
        st = ctx.stats()
        assert st["consumed"] == lookups.size
        # a lookup is presented again when its unpinned line changed tenant while it was
        # read, or when its prefetched chunk was dropped after an EAGAIN
        assert st["requests"] >= lookups.size
        assert st["hits"] + st["misses"] == st["requests"]
        distinct_lines = np.unique(lookups // 16).size
        assert distinct_lines <= st["read_cmds"] <= st["misses"]
        assert st["ctrl_cmds"] >= st["read_cmds"] and st["write_cmds"] == 0
        assert st["submitted"] == st["completed"]
        check_quiescent_invariants(ctx, 8)
    finally:
        ctx.close_store()
        ctx.shutdown()


@pytest.mark.parametrize("K", [0, 64])
@pytest.mark.parametrize("mode", [agile.MODE_SYNC, agile.MODE_ASYNC])
def test_pooled_bags_bit_exact(image, lookups, mode, K):
    import torch
    ctx = make_ctx(image)
    try:
        off = np.arange(0, 4097, 64, dtype=np.int64)
        out = torch.empty((64, DIM), dtype=torch.float32, device="cuda")
        ctx.embbag_forward(ctx.tables(ROWS, DIM), cuda(lookups), cuda(off), 64, K, out,
                           mode=mode)
        ctx.sync()
        ref = oracle.embbag_forward(image.array, ROWS, DIM, 1, lookups, off, 64, K)
        assert np.array_equal(out.cpu().numpy().view(np.uint32), ref.view(np.uint32))
        # a second pass over a warm cache gives the same bits
        ctx.embbag_forward(ctx.tables(ROWS, DIM), cuda(lookups), cuda(off), 64, K, out,
                           mode=mode)
        ctx.sync()
        assert np.array_equal(out.cpu().numpy().view(np.uint32), ref.view(np.uint32))
    finally:
        ctx.close_store()
        ctx.shutdown()


def test_serialized_trace_equals_clock_simulator(image, lookups):
    import torch
    ctx = make_ctx(image)
    try:
        lines = (lookups // 16).astype(np.uint64)
        rng = np.random.default_rng(3)
        writes = (rng.random(lines.size) < 0.1).astype(np.uint8)
        hit = torch.empty(lines.size, dtype=torch.uint8, device="cuda")
        way = torch.empty(lines.size, dtype=torch.int32, device="cuda")
        ctx.stats(reset=True)
        ctx.debug_trace(cuda(lines.astype(np.int64)), cuda(writes), hit, way)
        sim = oracle.Clock(32, 8)
        ehit, eway = sim.run(lines, writes)
        assert np.array_equal(hit.cpu().numpy(), ehit)
        assert np.array_equal(way.cpu().numpy(), eway)
        tags, st, rc = dump_meta(ctx)
        etags, edirty = sim.state()
        assert np.array_equal(tags.reshape(32, 8), etags)
        assert np.array_equal((st == 3).reshape(32, 8), edirty.astype(bool))
        s = ctx.stats()
        cnt = sim.counters()
        assert s["wb_evict"] == cnt["wb_evict"]
        assert s["read_cmds"] == cnt["misses"]
        ndirty = int(edirty.sum())
        ctx.flush()
        assert ctx.stats()["wb_flush"] == ndirty == sim.flush()
        check_quiescent_invariants(ctx, 8)
        tags, st, rc = dump_meta(ctx)
        assert not np.any(st == 3)
        # write-backs carried unchanged rows: the image is untouched
        ref = gen.table(ROWS, DIM, 0)
        assert np.array_equal(image.array[:ROWS * DIM * 4].view(np.float32).reshape(ROWS, DIM),
                              ref)
    finally:
        ctx.close_store()
        ctx.shutdown()


def test_ticket_api_read_wait_release(image):
    import torch
    ctx = make_ctx(image)
    try:
        nblocks = ROWS * DIM * 4 // 4096
        blocks = gen.uniform_blocks(7, 300, nblocks)  # duplicates and full sets included
        tk = torch.empty(blocks.size, dtype=torch.int64, device="cuda")
        ptr = torch.empty(blocks.size, dtype=torch.int64, device="cuda")
        ctx.async_read(cuda(blocks), tk)
        s = ctx.wait(tk, ptr)
        t = tk.cpu().numpy().view(np.uint64)
        p = ptr.cpu().numpy().view(np.uint64)
        status = (t >> np.uint64(40)) & np.uint64(0xFF)
        ok = status == 0
        assert s == (agile.OK if ok.all() else agile.EAGAIN)
        assert np.all(p[~ok] == 0)
        info = ctx.info()
        cache = device_bytes(info["cache_base"], info["num_lines"] * 4096).cpu().numpy()
        img = image.array
        for i in np.nonzero(ok)[0]:
            off = int(p[i] - info["cache_base"])
            b = int(blocks[i])
            assert np.array_equal(cache[off:off + 4096], img[b * 4096:(b + 1) * 4096]), i
        tags, st, rc = dump_meta(ctx)
        # every ok ticket holds one pin
        assert rc.sum() == ok.sum()
        ctx.release(tk)
        ctx.sync()
        assert dump_meta(ctx)[2].sum() == 0
        # the EAGAIN ones succeed once the pins are gone
        if (~ok).any():
            rb = blocks[~ok]
            tk2 = torch.empty(rb.size, dtype=torch.int64, device="cuda")
            p2 = torch.empty(rb.size, dtype=torch.int64, device="cuda")
            ctx.async_read(cuda(rb), tk2)
            assert ctx.wait(tk2, p2) in (agile.OK, agile.EAGAIN)
            ctx.release(tk2)
            ctx.sync()
        check_quiescent_invariants(ctx, 8)
    finally:
        ctx.close_store()
        ctx.shutdown()


def test_ticket_pin_limit_per_line(image):
    """300,000 tickets for one block: a line holds at most 262,144 pins, so at most that
    many tickets succeed and the others carry EAGAIN with nothing pinned (the pin count
    never reaches the generation bits); every successful ticket names the same line with
    the block's bytes, and after the release nothing is pinned."""
    import torch
    ctx = make_ctx(image)
    try:
        n = 300_000
        blocks = np.full(n, 5, dtype=np.uint64)
        tk = torch.empty(n, dtype=torch.int64, device="cuda")
        ctx.async_read(cuda(blocks), tk)
        ctx.sync()
        t = tk.cpu().numpy().view(np.uint64)
        status = (t >> np.uint64(40)) & np.uint64(0xFF)
        ok = status == 0
        assert np.all((status == 0) | (status == 1))
        assert 200_000 <= ok.sum() <= 262_144
        lines = np.unique(t[ok] & np.uint64(0xFFFFFFFF))
        gens = np.unique((t[ok] >> np.uint64(32)) & np.uint64(0xFF))
        assert lines.size == 1 and gens.size == 1
        tags, st, rc = dump_meta(ctx)
        assert rc[int(lines[0])] == ok.sum() and rc.sum() == ok.sum()
        assert tags[int(lines[0])] == 5 and st[int(lines[0])] == 2
        ptr = torch.empty(64, dtype=torch.int64, device="cuda")
        first = torch.from_numpy(t[ok][:64].view(np.int64)).cuda()
        assert ctx.wait(first, ptr) == agile.OK
        info = ctx.info()
        off = int(ptr[0].item()) - info["cache_base"]
        cache = device_bytes(info["cache_base"], info["num_lines"] * 4096).cpu().numpy()
        assert np.array_equal(cache[off:off + 4096], image.array[5 * 4096:6 * 4096])
        ctx.release(tk)
        ctx.sync()
        check_quiescent_invariants(ctx, 8)
    finally:
        ctx.close_store()
        ctx.shutdown()


@pytest.mark.parametrize("mode", [agile.MODE_SYNC, agile.MODE_ASYNC])
def test_cache_deadlock_case_one_set_four_ways(image, lookups, mode):
    """Sec. 2.3.2: waves that pin lines while asking for more must not deadlock; with one
    set of four ways every chunk needs more lines than the set holds."""
    import torch
    ctx = make_ctx(image, cache_bytes=4 * 4096, assoc=4)
    try:
        idx = cuda(lookups)
        out = torch.empty((lookups.size, DIM), dtype=torch.float32, device="cuda")
        ctx.gather(ctx.tables(ROWS, DIM), idx, out, mode=mode)
        ctx.sync()
        ref = oracle.gather(image.array, DIM * 4, lookups).view(np.float32).reshape(-1, DIM)
        assert np.array_equal(out.cpu().numpy(), ref)
        assert ctx.stats()["eagain"] > 0
        check_quiescent_invariants(ctx, 4)
    finally:
        ctx.close_store()
        ctx.shutdown()


def test_queue_deadlock_case_one_shallow_queue(image):
    """Sec. 2.3.1 / Fig. 1: one queue pair of depth 64 shared by every wave, far more
    outstanding misses than slots."""
    import torch
    ctx = make_ctx(image)
    try:
        rows = gen.uniform_int(5, gen.S_BLOCKS, 65536, 0, ROWS - 1)
        out = torch.empty((rows.size, DIM), dtype=torch.float32, device="cuda")
        ctx.gather(ctx.tables(ROWS, DIM), cuda(rows), out, mode=agile.MODE_ASYNC)
        ctx.sync()
        ref = image.array[:ROWS * DIM * 4].view(np.float32).reshape(ROWS, DIM)[rows]
        assert np.array_equal(out.cpu().numpy(), ref)
        st = ctx.stats()
        assert st["submitted"] == st["completed"] and st["read_cmds"] > 64 * 10
        check_quiescent_invariants(ctx, 8)
    finally:
        ctx.close_store()
        ctx.shutdown()


def test_multi_block_lines_and_many_queues(image, lookups):
    import torch
    ctx = make_ctx(image, line_bytes=16384, assoc=4, num_qp=4, qp_depth=128)
    try:
        off = np.arange(0, 4097, 64, dtype=np.int64)
        out = torch.empty((64, DIM), dtype=torch.float32, device="cuda")
        ctx.embbag_forward(ctx.tables(ROWS, DIM), cuda(lookups), cuda(off), 64, 3, out,
                           mode=agile.MODE_ASYNC)
        ctx.sync()
        ref = oracle.embbag_forward(image.array, ROWS, DIM, 1, lookups, off, 64, 3)
        assert np.array_equal(out.cpu().numpy(), ref)
        check_quiescent_invariants(ctx, 4)
    finally:
        ctx.close_store()
        ctx.shutdown()


def test_empty_inputs(image):
    import torch
    ctx = make_ctx(image)
    try:
        e = torch.empty(0, dtype=torch.int64, device="cuda")
        out = torch.empty((0, DIM), dtype=torch.float32, device="cuda")
        ctx.gather(ctx.tables(ROWS, DIM), e, out)
        off = torch.zeros(3, dtype=torch.int64, device="cuda")  # two empty bags
        pooled = torch.full((2, DIM), 7.0, device="cuda")
        ctx.embbag_forward(ctx.tables(ROWS, DIM), e, off, 2, 0, pooled)
        ctx.sync()
        assert torch.all(pooled == 0)
    finally:
        ctx.close_store()
        ctx.shutdown()
