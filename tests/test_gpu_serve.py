"""GPU checks of the continuous-batching serving session over the tiny table (65,536 x
64 fp32, 1 MiB cache): every request's pooled outputs equal the oracle's, bit for bit,
whether the request runs in the Poisson mix or alone, over the full request range of the
serving workload (1..4096 lookups, log-uniform) and in the geometries the measurements
use (the default and the one the committed tuning run chose)."""
import numpy as np
import pytest

import oracle
from paper_2504_19365_amd import agile, gen, tune

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


def _geometry(name):
    if name == "small":
        return dict(line_bytes=4096, assoc=8, num_qp=4, qp_depth=256), {}
    if name == "default":
        return dict(line_bytes=4096, assoc=8, num_qp=16, qp_depth=1024), {}
    return tune.split_point(tune.load_chosen(tune.SUMMARY_PATH))


def _check_session(image, geom, opts, mode, K, nreq, rate, max_log2, alone=(0, 7)):
    arrival, req_bag0, bag_off, idx = gen.serve_stream(nreq, rate, ROWS, 1.05, seed=40,
                                                       max_log2=max_log2)
    ctx = agile.Context(cache_bytes=1 << 20, timeout_ns=int(10e9), **geom)
    try:
        ctx.open_store(image)
        tb = ctx.tables(ROWS, DIM, 1)
        out, lat, rep = ctx.serve(tb, K, arrival, req_bag0, bag_off, idx, mode=mode, **opts)
        ref = _expected(image, req_bag0, bag_off, idx, K)
        assert np.array_equal(out.view(np.uint32), ref.view(np.uint32))
        assert rep["requests"] == nreq and np.all(lat > 0)
        assert rep["lookups"] == idx.size
        st = ctx.stats()
        assert st["consumed"] == idx.size
        # a few requests alone (each one its own session) give the same bits
        for r in alone:
            b0, b1 = int(req_bag0[r]), int(req_bag0[r + 1])
            l0, l1 = int(bag_off[b0]), int(bag_off[b1])
            o1, _, _ = ctx.serve(tb, K, np.zeros(1), np.array([0, b1 - b0]),
                                 bag_off[b0:b1 + 1] - l0, idx[l0:l1], mode=mode, **opts)
            assert np.array_equal(o1.view(np.uint32), out[b0:b1].view(np.uint32))
        check_quiescent_invariants(ctx, geom["assoc"])
        return rep, idx
    finally:
        ctx.close_store()
        ctx.shutdown()


@pytest.mark.parametrize("mode", [agile.MODE_SYNC, agile.MODE_ASYNC])
def test_mix_equals_oracle_and_alone(image, mode):
    geom, opts = _geometry("small")
    rep, _ = _check_session(image, geom, opts, mode, 16, 300, 20000.0, 9, alone=(0, 7, 150, 299))
    assert rep["max_inflight_requests"] >= 1


@pytest.mark.timeout(300)
@pytest.mark.parametrize("geometry", ["default", "tuned"])
def test_full_request_range_equals_oracle(image, geometry):
    """Requests of 1..4096 lookups at the offered 20k requests/s, in the geometry the
    serving measurements run."""
    geom, opts = _geometry(geometry)
    rep, idx = _check_session(image, geom, opts, agile.MODE_ASYNC, 0, 300, 20000.0, 12,
                              alone=(0, 7, 299))
    # the stream does reach the large end of the range
    assert idx.size > 300 * 200


@pytest.mark.timeout(300)
@pytest.mark.parametrize("waves", [1, 3, 7])
def test_fewer_waves_than_work_partitions(image, waves):
    """With fewer user wavefronts than work partitions, requests published over time (a
    slow Poisson stream, so most bags are claimed before their request is published) and
    an admission cap of two requests in flight, every request completes and equals the
    oracle."""
    geom, _ = _geometry("small")
    opts = dict(user_waves=waves, max_inflight_requests=2)
    _check_session(image, geom, opts, agile.MODE_ASYNC, 0, 40, 2000.0, 8, alone=(3,))
