"""GPU checks of the lock-chain debugging mode (AGILE_F_LOCKCHAIN, after Sec. 3.5's
lock-chain debugger): the device walker, run on planted wait states, follows a set lock
to its holder and on to what the holder waits for, stops at a wait on no wave or at a
running holder, and reports a cycle; and a wait that times out for real (a store whose
latency far exceeds the context's timeout, so every kernel ends through its own bounded
waits) puts the recorded chain into the error text."""
import numpy as np
import pytest

from paper_2504_19365_amd import agile

from gpu_helpers import cuda, table_store

pytestmark = pytest.mark.gpu

W = agile.Context


def _ctx(**kw):
    cfg = dict(cache_bytes=1 << 20, line_bytes=4096, assoc=8, num_qp=4, qp_depth=256,
               timeout_ns=int(5e9), flags=agile.F_LOCKCHAIN)
    cfg.update(kw)
    return agile.Context(**cfg)


def wi(kind, obj):
    return (kind << 56) | obj


def test_walker_follows_a_set_lock_to_a_fill():
    ctx = _ctx()
    try:
        sets = ctx.info()["num_sets"]
        line = 1000
        waits = {0: wi(W.W_SETLOCK, line), 2: wi(W.W_FILL, 7)}
        msg = ctx.debug_lockchain(waits, {line % sets: 2 + 2}, 0, waits[0])
        assert msg.startswith(f"lock chain: wave 0 waits for the set lock of store line {line}, held by wave 2")
        assert "wave 2 waits for the fill of cache line 7" in msg
        assert "cycle" not in msg
    finally:
        ctx.shutdown()


def test_walker_reports_a_cycle():
    ctx = _ctx()
    try:
        sets = ctx.info()["num_sets"]
        a, b = 10, 11  # two lines in two different sets
        waits = {0: wi(W.W_SETLOCK, a), 1: wi(W.W_SETLOCK, b)}
        msg = ctx.debug_lockchain(waits, {a % sets: 1 + 2, b % sets: 0 + 2}, 0, waits[0])
        assert "wave 0 waits for the set lock of store line 10, held by wave 1" in msg
        assert "wave 1 waits for the set lock of store line 11, held by wave 0" in msg
        assert msg.endswith("a cycle back to wave 0")
    finally:
        ctx.shutdown()


def test_walker_stops_at_a_running_holder_and_a_free_lock():
    ctx = _ctx()
    try:
        sets = ctx.info()["num_sets"]
        waits = {0: wi(W.W_SETLOCK, 5)}
        msg = ctx.debug_lockchain(waits, {5 % sets: 7 + 2}, 0, waits[0])
        assert "held by wave 7" in msg and "wave 7 waits for nothing (running)" in msg
        # the state was cleared: the same lock now reads free
        msg = ctx.debug_lockchain(waits, {}, 0, waits[0])
        assert msg == "lock chain: wave 0 waits for the set lock of store line 5 (free now)"
    finally:
        ctx.shutdown()


@pytest.mark.parametrize("flags", [agile.F_LOCKCHAIN, 0])
def test_timeout_reports_the_chain(flags):
    """Fills take 200 ms, the context gives up after 20 ms: the forward ends with a
    timeout whose text (in lock-chain mode only) names what the first wave waited for."""
    import torch
    rows, dim = 65536, 64
    buf = table_store(rows, dim, [0])
    ctx = _ctx(latency_ns=200_000_000, timeout_ns=20_000_000, flags=flags)
    try:
        ctx.open_store(buf)
        idx = np.arange(64, dtype=np.int64) * 16  # 64 lookups on 64 lines, 2 per set
        off = np.array([0, 64], dtype=np.int64)
        out = torch.empty((1, dim), device="cuda")
        with pytest.raises(agile.AgileError) as e:
            ctx.embbag_forward(ctx.tables(rows, dim), cuda(idx), cuda(off), 1, 0, out)
            ctx.sync()
        assert e.value.status == agile.ETIMEDOUT
        text = str(e.value)
        if flags:
            assert "lock chain: wave " in text
            assert "waits for the fill of cache line" in text
        else:
            assert "lock chain" not in text
    finally:
        ctx.shutdown()
        buf.free()
