"""GPU parity of the kernel-only embedding-bag forward (the tables resident in device
memory, no cache or queues): bit-identical to the oracle and to the cached forward, for
each row width the kernels specialise (1, 2 and 4 floats per lane, and a row narrower
than the wavefront), with empty and long bags; a row out of range raises the sticky
error."""
import numpy as np
import pytest

import oracle
from paper_2504_19365_amd import agile, gen

from gpu_helpers import cuda, table_store

pytestmark = pytest.mark.gpu


def _bags(rows, T, B, seed):
    off, idx = gen.embbag_batch(gen.zipf_cum(rows, 1.05), B, T, 1, 150, seed=seed)
    # make a few bags empty: drop their lookups
    lens = np.diff(off)
    keep = np.ones(idx.size, dtype=bool)
    for b in (0, 5, B * T - 1):
        keep[off[b]:off[b + 1]] = False
        lens[b] = 0
    off2 = np.zeros(off.size, dtype=np.int64)
    np.cumsum(lens, out=off2[1:])
    return off2, idx[keep]


@pytest.mark.parametrize("dim", [16, 64, 128, 256])
@pytest.mark.parametrize("K", [0, 16])
def test_resident_forward_equals_oracle_and_cached(dim, K):
    import torch
    rows, T, B = 16384, 3, 300
    buf = table_store(rows, dim, [3, 4, 5])
    ctx = agile.Context(cache_bytes=1 << 20, line_bytes=4096, assoc=8, num_qp=4, qp_depth=256,
                        timeout_ns=int(10e9))
    try:
        ctx.open_store(buf)
        tb = ctx.tables(rows, dim, T)
        off, idx = _bags(rows, T, B, seed=7 + dim)
        img = torch.from_numpy(buf.array).cuda()
        out_r = torch.full((B * T, dim), float("nan"), device="cuda")
        ctx.embbag_forward_resident(img, buf.nbytes, tb, cuda(idx), cuda(off), B, K, out_r)
        out_c = torch.empty((B * T, dim), device="cuda")
        ctx.embbag_forward(tb, cuda(idx), cuda(off), B, K, out_c, mode=agile.MODE_ASYNC)
        ctx.sync()
        ref = oracle.embbag_forward(buf.array, rows, dim, T, idx, off, B, K)
        got = out_r.cpu().numpy()
        assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))
        assert np.array_equal(got.view(np.uint32), out_c.cpu().numpy().view(np.uint32))
        assert np.all(got[0] == 0) and np.all(got[5] == 0)
    finally:
        ctx.close_store()
        ctx.shutdown()
        buf.free()


def test_resident_forward_rejects_rows_out_of_range():
    import torch
    rows, dim = 4096, 64
    buf = table_store(rows, dim, [0])
    ctx = agile.Context(cache_bytes=1 << 20, timeout_ns=int(5e9))
    try:
        tb = ctx.tables(rows, dim, 1)
        img = torch.from_numpy(buf.array).cuda()
        idx = np.array([1, rows, 2], dtype=np.int64)
        off = np.array([0, 3], dtype=np.int64)
        out = torch.empty((1, dim), device="cuda")
        ctx.embbag_forward_resident(img, buf.nbytes, tb, cuda(idx), cuda(off), 1, 0, out)
        with pytest.raises(agile.AgileError) as e:
            ctx.sync()
        assert e.value.status == agile.ESTATE
    finally:
        ctx.shutdown()
        buf.free()
