"""The emulated NVMe device keeps its two performance parameters: every command completes
no earlier than the configured latency after it was fetched, and commands execute at no
more than the configured IOPS cap (the device model behind Eq. 1 and the throughput
figures of the evaluation).  Host wall-clock time around a synchronised call bounds both
from above; the lower bounds are the properties under test."""
import time

import numpy as np
import pytest

from paper_2504_19365_amd import agile

from gpu_helpers import cuda, table_store

pytestmark = pytest.mark.gpu

ROWS, DIM = 262144, 64          # 64 MiB store, 16 rows per 4 KiB block
ROWS_PER_BLOCK = 4096 // (DIM * 4)


@pytest.fixture(scope="module")
def image():
    buf = table_store(ROWS, DIM, [3])
    yield buf
    buf.free()


def timed_gather(ctx, rows):
    import torch
    out = torch.empty((rows.size, DIM), dtype=torch.float32, device="cuda")
    idx = cuda(rows)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.gather(ctx.tables(ROWS, DIM), idx, out, mode=agile.MODE_ASYNC)
    ctx.sync()
    return time.perf_counter() - t0, out


@pytest.mark.parametrize("iops", [100_000, 400_000])
def test_iops_cap_bounds_miss_throughput(image, iops):
    nblk = 16384                                    # every block of the store once
    rows = np.arange(nblk, dtype=np.int64) * ROWS_PER_BLOCK
    ctx = agile.Context(cache_bytes=128 << 20, line_bytes=4096, assoc=8, num_qp=16,
                        qp_depth=1024, latency_ns=0, iops_cap=iops, timeout_ns=int(10e9))
    try:
        ctx.open_store(image)
        timed_gather(ctx, rows[:64])                # first launch outside the timing
        ctx.invalidate()
        ctx.stats(reset=True)
        el, out = timed_gather(ctx, rows)
        st = ctx.stats()
        assert st["read_cmds"] == nblk
        floor = (nblk - 64) / iops                  # no burst allowance beyond one fetch
        assert el >= 0.97 * floor, (el, floor)
        assert el <= 2.0 * nblk / iops + 0.25, (el, nblk / iops)
        ref = image.array[:ROWS * DIM * 4].view(np.float32).reshape(ROWS, DIM)[rows]
        assert np.array_equal(out.cpu().numpy(), ref)
    finally:
        ctx.close_store()
        ctx.shutdown()


def test_latency_bounds_every_miss(image):
    lat_ns = 40_000_000                             # 40 ms per command
    ctx = agile.Context(cache_bytes=4 << 20, line_bytes=4096, assoc=8, num_qp=1,
                        qp_depth=64, latency_ns=lat_ns, iops_cap=0, timeout_ns=int(10e9))
    try:
        ctx.open_store(image)
        for rows in (np.array([5 * ROWS_PER_BLOCK], dtype=np.int64),
                     np.arange(64, dtype=np.int64) * ROWS_PER_BLOCK + 7):
            ctx.invalidate()
            el, out = timed_gather(ctx, rows)
            assert el >= lat_ns * 1e-9 * 0.99, el
            assert el <= lat_ns * 1e-9 * 4 + 0.25, el
            ref = image.array[:ROWS * DIM * 4].view(np.float32).reshape(ROWS, DIM)[rows]
            assert np.array_equal(out.cpu().numpy(), ref)
        # a second pass over the same rows hits: no command, far below one latency
        el, _ = timed_gather(ctx, rows)
        assert el < lat_ns * 1e-9 * 0.5, el
    finally:
        ctx.close_store()
        ctx.shutdown()
