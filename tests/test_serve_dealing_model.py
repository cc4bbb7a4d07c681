"""A model of how the serving kernel's waves deal out an unbounded stream of bags
(static rounds, then one counter per work partition, a wave starting in partition
u mod P, holding its next claimed bag while it works on the current one, and waiting on
a claimed bag until the host has published it).  With P = min(8, waves) partitions every
published bag is served for any wave count; with the earlier P = 8 fewer than 8 waves
left partitions with no wave, and requests whose bags fell there never finished."""
import pytest

STATIC_ROUNDS = 2
WORK_PARTS = 8


def serve_model(A: int, parts: int, publish, steps: int = 10_000):
    """Waves 0..A-1 over an unbounded bag stream; publish[t] = bags published before step t
    (non-decreasing).  Returns the set of bags served."""
    counters = [0] * parts
    dealt = [0] * A
    cur = [None] * A
    held = [None] * A
    done = set()

    def claim(u):
        if dealt[u] < STATIC_ROUNDS:
            b = u + dealt[u] * A
            dealt[u] += 1
            return b
        p = u % parts  # the stream never ends, so a wave never leaves its partition
        v = counters[p]
        counters[p] += 1
        return STATIC_ROUNDS * A + v * parts + p

    for t in range(steps):
        pub = publish(t)
        for u in range(A):
            if held[u] is None:
                held[u] = claim(u)
            if cur[u] is None and held[u] < pub:
                cur[u], held[u] = held[u], claim(u)
            if cur[u] is not None:
                done.add(cur[u])
                cur[u] = None
    return done


def staged(total, every):
    # the host publishes `every` more bags each step until `total`
    return lambda t: min(total, (t + 1) * every)


@pytest.mark.parametrize("A", list(range(1, 20)))
def test_every_published_bag_is_served(A):
    parts = min(WORK_PARTS, A)
    total = 500
    done = serve_model(A, parts, staged(total, 3), steps=2000)
    assert set(range(total)) <= done


@pytest.mark.parametrize("A", [1, 3, 7])
def test_eight_partitions_with_fewer_waves_leave_bags_unserved(A):
    # the rule the model replaces: some partitions have no wave
    done = serve_model(A, WORK_PARTS, staged(200, 3), steps=2000)
    assert not set(range(200)) <= done


def test_bags_are_dealt_once():
    for A in range(1, 20):
        parts = min(WORK_PARTS, A)
        counters = [0] * parts
        seen = set()
        for u in range(A):
            for r in range(STATIC_ROUNDS):
                seen.add(u + r * A)
        for p in range(parts):
            for v in range(50):
                b = STATIC_ROUNDS * A + v * parts + p
                assert b not in seen
                seen.add(b)
        assert seen == set(range(STATIC_ROUNDS * A + 50 * parts))
