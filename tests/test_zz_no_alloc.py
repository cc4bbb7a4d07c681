"""The allocation-free backward entry point (agile_embbag_backward_sgd_noalloc), through
the C ABI, against the existing entry point (agile_embbag_backward_sgd): two contexts over
two copies of the same store image run the same two calls in a row, the second with a
smaller batch; after a flush both images are equal bit for bit (and equal the oracle's
update).  Also: a batch above the fixed work area's maximum is rejected before anything
is launched."""
import ctypes as C

import numpy as np
import pytest

import oracle
from paper_2504_19365_amd import agile, gen

from gpu_helpers import check_quiescent_invariants, cuda, table_store

pytestmark = pytest.mark.gpu

ROWS, DIM, T = 262144, 64, 4


def _noalloc(ctx, tb, idx, off, B, g, lr):
    L = agile.lib()
    f = L.agile_embbag_backward_sgd_noalloc
    f.restype = C.c_int
    f.argtypes = [C.c_void_p, C.c_void_p, C.POINTER(agile.Tables), C.c_void_p, C.c_void_p,
                  C.c_uint64, C.c_uint64, C.c_void_p, C.c_float, C.c_void_p]
    n = int(idx.numel())
    return f(ctx.h, ctx.store.handle, C.byref(tb), idx.data_ptr(), off.data_ptr(), B, n,
             g.data_ptr(), lr, agile._stream(None))


def test_noalloc_backward_equals_existing_entry_point():
    bufs = [table_store(ROWS, DIM, [20, 21, 22, 23]) for _ in range(2)]
    ref = bufs[0].array.copy()
    ctxs = [agile.Context(cache_bytes=16 << 20, line_bytes=4096, assoc=16, num_qp=4,
                          qp_depth=256, timeout_ns=int(30e9)) for _ in range(2)]
    try:
        for c, b in zip(ctxs, bufs):
            c.open_store(b)
        tbs = [c.tables(ROWS, DIM, T) for c in ctxs]
        cum = gen.zipf_cum(ROWS, 1.1)
        lr = 0.01
        for step, B in enumerate((4096, 1000)):   # the second call is smaller
            off, idx = gen.embbag_batch(cum, B, T, 1, 40, seed=700 + step)
            g = gen.normal_f32(710 + step, B * T * DIM).reshape(B * T, DIM)
            d_off, d_idx, d_g = cuda(off), cuda(idx), cuda(g)
            ctxs[0].embbag_backward_sgd(tbs[0], d_idx, d_off, B, d_g, lr)
            st = _noalloc(ctxs[1], tbs[1], d_idx, d_off, B, d_g, lr)
            assert st == agile.OK, agile.status_string(st)
            for c in ctxs:
                c.sync()
            oracle.embbag_backward_sgd(ref, ROWS, DIM, T, idx, off, B, g, lr)
        for c in ctxs:
            c.flush()
            check_quiescent_invariants(c, 16)
        assert np.array_equal(bufs[0].array, bufs[1].array)
        assert np.array_equal(bufs[1].array, ref)
        # above the maximum: rejected, nothing launched, the context stays usable
        big = 1 << 21
        d_idx = cuda(np.zeros(big, dtype=np.int64))
        d_off = cuda(np.array([0, big], dtype=np.int64))
        d_g = cuda(np.zeros((1, DIM), dtype=np.float32))
        tb1 = ctxs[1].tables(ROWS, DIM, 1)
        assert _noalloc(ctxs[1], tb1, d_idx, d_off, 1, d_g, lr) == agile.EINVAL
        ctxs[1].sync()
    finally:
        for c in ctxs:
            c.close_store()
            c.shutdown()
        for b in bufs:
            b.free()
