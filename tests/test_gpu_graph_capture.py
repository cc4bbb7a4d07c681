"""The embedding-bag forward step captured once in a HIP graph and replayed.

A launch carries no host-side running totals (its work and completion counters start at
zero on the device and are cleared by the launch's last service wavefront), so one
captured launch can be replayed.  Each replay is checked against the oracle, with eager
launches, cache invalidations and stream synchronisations between the replays; the
counters must show that every replay did the whole batch."""
import numpy as np
import pytest

import oracle
from paper_2504_19365_amd import agile, gen

from gpu_helpers import cuda, table_store

pytestmark = pytest.mark.gpu

ROWS, DIM = 65536, 64


@pytest.fixture(scope="module")
def image():
    buf = table_store(ROWS, DIM, [0])
    yield buf
    buf.free()


def batch(seed, B):
    cum = gen.zipf_cum(ROWS, 1.05)
    return gen.embbag_batch(cum, B, 1, 1, 80, seed)


@pytest.mark.parametrize("mode", [agile.MODE_SYNC, agile.MODE_ASYNC])
@pytest.mark.parametrize("geom", [dict(cache_bytes=1 << 20, assoc=8, num_qp=1, qp_depth=64),
                                  dict(cache_bytes=16 << 20, assoc=16, num_qp=8, qp_depth=256)])
def test_captured_forward_replays_match_oracle(image, mode, geom):
    import torch
    ctx = agile.Context(line_bytes=4096, timeout_ns=int(10e9), **geom)
    try:
        ctx.open_store(image)
        tb = ctx.tables(ROWS, DIM)
        B, K = 512, 16
        off, idx = batch(7, B)
        off2, idx2 = batch(8, B)
        ref = oracle.embbag_forward(image.array, ROWS, DIM, 1, idx, off, B, K)
        ref2 = oracle.embbag_forward(image.array, ROWS, DIM, 1, idx2, off2, B, K)
        d_off, d_idx = cuda(off), cuda(idx)
        d_off2, d_idx2 = cuda(off2), cuda(idx2)
        out = torch.zeros((B, DIM), dtype=torch.float32, device="cuda")
        out2 = torch.empty((B, DIM), dtype=torch.float32, device="cuda")

        # eager launch first (the library caches its occupancy queries outside capture)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            ctx.embbag_forward(tb, d_idx, d_off, B, K, out, mode=mode)
        torch.cuda.current_stream().wait_stream(side)
        ctx.sync()
        assert np.array_equal(out.cpu().numpy().view(np.uint32), ref.view(np.uint32))

        g = torch.cuda.CUDAGraph()
        out.zero_()
        with torch.cuda.graph(g):
            ctx.embbag_forward(tb, d_idx, d_off, B, K, out, mode=mode)
        torch.cuda.synchronize()

        for rep in range(4):
            if rep % 2:
                ctx.invalidate()  # the replay must fetch everything again
            out.zero_()
            ctx.stats(reset=True)
            g.replay()
            torch.cuda.synchronize()
            st = ctx.stats()
            got = out.cpu().numpy()
            assert np.array_equal(got.view(np.uint32), ref.view(np.uint32)), rep
            assert st["consumed"] == idx.size, (rep, st)
            assert st["submitted"] == st["completed"]
            # eager work between replays
            ctx.embbag_forward(tb, d_idx2, d_off2, B, K, out2, mode=mode)
            ctx.sync()
            assert np.array_equal(out2.cpu().numpy().view(np.uint32), ref2.view(np.uint32)), rep
        del g
    finally:
        ctx.close_store()
        ctx.shutdown()


@pytest.mark.parametrize("geom", [dict(cache_bytes=16 << 20, assoc=16, num_qp=8, qp_depth=256),
                                  dict(cache_bytes=64 << 20, assoc=16, num_qp=8, qp_depth=256)])
def test_captured_prefetch_forward_replays_match_oracle(image, geom):
    """agile_embbag_forward_prefetch (one launch: this batch computed while the next is
    prefetched) captured once and replayed, with invalidations and eager calls between the
    replays: every replay equals the oracle, completes every command it submits, and
    leaves the next batch resident (a forward of it then reads nothing)."""
    import torch
    ctx = agile.Context(line_bytes=4096, timeout_ns=int(10e9), **geom)
    try:
        ctx.open_store(image)
        tb = ctx.tables(ROWS, DIM)
        B, K = 512, 16
        off, idx = batch(7, B)
        off2, idx2 = batch(8, B)
        ref = oracle.embbag_forward(image.array, ROWS, DIM, 1, idx, off, B, K)
        ref2 = oracle.embbag_forward(image.array, ROWS, DIM, 1, idx2, off2, B, K)
        d_off, d_idx = cuda(off), cuda(idx)
        d_off2, d_idx2 = cuda(off2), cuda(idx2)
        out = torch.zeros((B, DIM), dtype=torch.float32, device="cuda")
        out2 = torch.empty((B, DIM), dtype=torch.float32, device="cuda")

        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            ctx.embbag_forward_prefetch(tb, d_idx, d_off, B, K, out, d_idx2, d_off2, B)
        torch.cuda.current_stream().wait_stream(side)
        ctx.sync()
        assert np.array_equal(out.cpu().numpy().view(np.uint32), ref.view(np.uint32))

        g = torch.cuda.CUDAGraph()
        out.zero_()
        with torch.cuda.graph(g):
            ctx.embbag_forward_prefetch(tb, d_idx, d_off, B, K, out, d_idx2, d_off2, B)
        torch.cuda.synchronize()

        for rep in range(4):
            if rep % 2:
                ctx.invalidate()
            out.zero_()
            ctx.stats(reset=True)
            g.replay()
            torch.cuda.synchronize()
            st = ctx.stats()
            assert np.array_equal(out.cpu().numpy().view(np.uint32), ref.view(np.uint32)), rep
            assert st["submitted"] == st["completed"]
            if rep % 2:
                assert st["read_cmds"] > 0, rep  # the invalidated cache was read again
            if geom["cache_bytes"] >= 64 << 20:
                # the whole store fits: the prefetched batch is resident after the replay
                ctx.stats(reset=True)
                ctx.embbag_forward(tb, d_idx2, d_off2, B, K, out2, mode=agile.MODE_SYNC)
                ctx.sync()
                assert ctx.stats()["read_cmds"] == 0, rep
            else:
                ctx.embbag_forward(tb, d_idx2, d_off2, B, K, out2, mode=agile.MODE_ASYNC)
                ctx.sync()
            assert np.array_equal(out2.cpu().numpy().view(np.uint32), ref2.view(np.uint32)), rep
        del g
    finally:
        ctx.close_store()
        ctx.shutdown()
