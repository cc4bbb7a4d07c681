"""GPU checks of the continuous-batching serving session over the tiny table (65,536 x
64 fp32): every request's pooled outputs equal the oracle's, bit for bit, whether the
request runs in the Poisson mix or alone."""
import numpy as np
import pytest

import oracle
from paper_2504_19365_amd import agile, gen

from gpu_helpers import check_quiescent_invariants, table_store

pytestmark = pytest.mark.gpu

ROWS, DIM = 65536, 64


@pytest.fixture(scope="module")
def image():
    buf = table_store(ROWS, DIM, [0])
    yield buf
    buf.free()


def _expected(image, req_bag0, bag_off, idx, K):
    # every bag reads table 0 (one table), in its own order
    nb = int(req_bag0[-1])
    return oracle.embbag_forward(image.array, ROWS, DIM, 1, idx, bag_off, nb, K)


@pytest.mark.parametrize("mode", [agile.MODE_SYNC, agile.MODE_ASYNC])
def test_mix_equals_oracle_and_alone(image, mode):
    arrival, req_bag0, bag_off, idx = gen.serve_stream(300, 20000.0, ROWS, 1.05, seed=40,
                                                       max_log2=9)
    ctx = agile.Context(cache_bytes=1 << 20, line_bytes=4096, assoc=8, num_qp=4, qp_depth=256,
                        timeout_ns=int(10e9))
    try:
        ctx.open_store(image)
        tb = ctx.tables(ROWS, DIM, 1)
        K = 16
        out, lat, rep = ctx.serve(tb, K, arrival, req_bag0, bag_off, idx, mode=mode)
        ref = _expected(image, req_bag0, bag_off, idx, K)
        assert np.array_equal(out.view(np.uint32), ref.view(np.uint32))
        assert rep["requests"] == 300 and np.all(lat > 0)
        assert rep["max_inflight_requests"] >= 1
        # a few requests alone (each one its own session) give the same bits
        for r in (0, 7, 150, 299):
            b0, b1 = int(req_bag0[r]), int(req_bag0[r + 1])
            l0, l1 = int(bag_off[b0]), int(bag_off[b1])
            o1, _, _ = ctx.serve(tb, K, np.zeros(1), np.array([0, b1 - b0]),
                                 bag_off[b0:b1 + 1] - l0, idx[l0:l1], mode=mode)
            assert np.array_equal(o1.view(np.uint32), out[b0:b1].view(np.uint32))
        check_quiescent_invariants(ctx, 8)
    finally:
        ctx.close_store()
        ctx.shutdown()
