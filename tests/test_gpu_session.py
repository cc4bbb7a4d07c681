"""GPU checks of the serving session calls (open, submit, poll, close): requests
submitted while the persistent kernel runs, in bursts with idle gaps between them and
collected in an order of their own, give the oracle's pooled outputs bit for bit; the
request, lookup and bag rings wrap many times; the largest request, empty bags and the
argument and state errors behave as the header states.  Tiny table (65,536 x 64 fp32),
1 MiB cache."""
import time

import numpy as np
import pytest

import oracle
from paper_2504_19365_amd import agile, gen

from gpu_helpers import check_quiescent_invariants, table_store

pytestmark = pytest.mark.gpu

ROWS, DIM = 65536, 64
GEOM = dict(line_bytes=4096, assoc=8, num_qp=4, qp_depth=256)


@pytest.fixture(scope="module")
def image():
    buf = table_store(ROWS, DIM, [0])
    yield buf
    buf.free()


def _context(image):
    ctx = agile.Context(cache_bytes=1 << 20, timeout_ns=int(10e9), **GEOM)
    ctx.open_store(image)
    return ctx


def _expected(image, bag_off, idx, K):
    return oracle.embbag_forward(image.array, ROWS, DIM, 1, idx, bag_off, bag_off.size - 1, K)


def _request(req_bag0, bag_off, idx, r):
    b0, b1 = int(req_bag0[r]), int(req_bag0[r + 1])
    l0, l1 = int(bag_off[b0]), int(bag_off[b1])
    return bag_off[b0:b1 + 1] - l0, idx[l0:l1]


@pytest.mark.timeout(300)
@pytest.mark.parametrize("mode", [agile.MODE_SYNC, agile.MODE_ASYNC])
def test_submit_while_running(image, mode):
    """600 requests of 1..4096 lookups (about 300k lookups: the lookup ring of 131,072
    slots wraps twice, the request ring of 8 slots every 8 requests) submitted in bursts
    of 1..24 with idle gaps of up to 20 ms, polled in shuffled order."""
    K = 16
    nreq = 600
    _, req_bag0, bag_off, idx = gen.serve_stream(nreq, 20000.0, ROWS, 1.05, seed=41,
                                                 max_log2=12)
    assert idx.size > 2 * 131072
    ref = _expected(image, bag_off, idx, K)
    rng = np.random.default_rng(7)
    ctx = _context(image)
    try:
        tb = ctx.tables(ROWS, DIM, 1)
        got = [None] * nreq
        ids = {}
        with ctx.open_session(tb, K, mode=mode, max_inflight_requests=4) as se:
            # other calls are refused while the session owns the device
            with pytest.raises(agile.AgileError) as e:
                ctx.stats()
            assert e.value.status == agile.ESTATE
            with pytest.raises(agile.AgileError) as e:
                ctx.open_session(tb, K)
            assert e.value.status == agile.ESTATE
            pending = []
            nxt = 0
            t_end = time.monotonic() + 240
            while nxt < nreq or pending:
                assert time.monotonic() < t_end
                burst = int(rng.integers(1, 25))
                for _ in range(burst):
                    if nxt == nreq:
                        break
                    bo, ix = _request(req_bag0, bag_off, idx, nxt)
                    r = se.submit(bo, ix)
                    if r is None:
                        break  # full: collect first
                    ids[r] = nxt
                    pending.append(r)
                    nxt += 1
                rng.shuffle(pending)
                keep = []
                for r in pending:
                    q = ids[r]
                    o = se.poll(r, int(req_bag0[q + 1] - req_bag0[q]))
                    if o is None:
                        keep.append(r)
                    else:
                        got[q] = o
                pending = keep
                if rng.random() < 0.2:
                    time.sleep(float(rng.uniform(0.0, 0.02)))  # an idle gap
        assert sorted(ids) == list(range(nreq))  # numbered in submission order
        out = np.concatenate(got)
        assert np.array_equal(out.view(np.uint32), ref.view(np.uint32))
        st = ctx.stats()
        assert st["consumed"] == idx.size
        check_quiescent_invariants(ctx, GEOM["assoc"])
    finally:
        ctx.close_store()
        ctx.shutdown()


@pytest.mark.timeout(300)
def test_largest_requests_empty_bags_and_errors(image):
    """Requests of 65,536 bags (a third of them empty, the rest one lookup: three of them
    wrap the bag ring of 131,072 slots) and of one bag of 65,536 lookups equal the
    oracle; a request beyond the maximum, a row out of range, bad offsets, a second poll
    and calls on the context while the session is open are refused; after close the
    context works as before."""
    rng = np.random.default_rng(3)
    ctx = _context(image)
    try:
        tb = ctx.tables(ROWS, DIM, 1)
        reqs = []
        for _ in range(3):
            lens = (rng.random(65536) >= 1 / 3).astype(np.int64)
            bo = np.zeros(65537, dtype=np.int64)
            np.cumsum(lens, out=bo[1:])
            reqs.append((bo, rng.integers(0, ROWS, int(bo[-1]), dtype=np.int64)))
        reqs.append((np.array([0, 65536], dtype=np.int64),
                     rng.integers(0, ROWS, 65536, dtype=np.int64)))
        reqs.append((np.array([0, 0, 0], dtype=np.int64), np.zeros(0, dtype=np.int64)))
        with ctx.open_session(tb, 0, mode=agile.MODE_ASYNC) as se:
            for bo, ix in [(np.array([0, 65537]), np.zeros(65537, dtype=np.int64)),
                           (np.array([0, 2]), np.array([0, ROWS])),
                           (np.array([0, 2, 1]), np.array([0, 1])),
                           (np.array([1, 2]), np.array([0, 1]))]:
                with pytest.raises(agile.AgileError) as e:
                    se.submit(bo, ix)
                assert e.value.status == agile.EINVAL
            with pytest.raises(agile.AgileError) as e:
                ctx.embbag_forward(tb, None, None, 0, 0, None)
            assert e.value.status == agile.ESTATE
            assert ctx.close_store() == agile.ESTATE and ctx.store is not None
            for bo, ix in reqs:
                r = None
                t_end = time.monotonic() + 120
                while r is None:
                    assert time.monotonic() < t_end
                    r = se.submit(bo, ix)
                o = None
                while o is None:
                    assert time.monotonic() < t_end
                    o = se.poll(r, bo.size - 1)
                ref = _expected(image, bo, ix, 0)
                assert np.array_equal(o.view(np.uint32), ref.view(np.uint32))
                with pytest.raises(agile.AgileError) as e:
                    se.poll(r, bo.size - 1)
                assert e.value.status == agile.EINVAL
        # the context takes ordinary calls again
        bo, ix = reqs[3]
        out, _, _ = ctx.serve(tb, 0, np.zeros(1), np.array([0, 1]), bo, ix)
        assert np.array_equal(out.view(np.uint32), _expected(image, bo, ix, 0).view(np.uint32))
        check_quiescent_invariants(ctx, 8)
    finally:
        ctx.close_store()
        ctx.shutdown()
