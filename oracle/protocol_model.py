"""Explicit-state model of the queue-pair protocol (TEST INFRASTRUCTURE).

Two small models are explored exhaustively (every interleaving of atomic steps) for
tiny queue depths and thread counts:

* ``agile``: submitters never touch completion queues.  A submitting wave reserves its
  tickets with one atomic, writes each command into its slot once the slot's previous
  lap is EMPTY, marks it UPDATED, and rings the doorbell by scanning UPDATED slots in
  order and marking them ISSUED (Sec. 3.3.1, Alg. 2).  An emulated controller fetches
  issued commands, may complete them in any order, and posts phase-tagged completion
  entries when the completion queue has room.  A separate completion service checks a
  window of entries against the expected phase, frees each command's slot for the next
  lap, and advances the completion head when the window is full (Sec. 3.2, Alg. 1).
* ``naive``: the design of Fig. 1 (Sec. 2.3.1): a submitter holds each slot it filled
  until it has itself consumed the matching completion, and it spins for a free slot
  before it ever looks at the completion queue.

``explore`` returns the number of reachable states and the first deadlocked state found
(a state where some thread has not finished and no step is enabled).  The agile model
must have none; the naive model must reach one (the Fig. 1 scenario) once the threads
together want more slots than the queue holds.

``agile_ring_last`` is ``agile`` with one change: a wave rings the doorbell only after
all of its commands are written.  The search shows that this variant deadlocks when a
wave's later command needs the slot of one of its own earlier commands, which is why
the submission loop rings while it still waits for slots.

``agile_batch_post`` is ``agile`` with a controller that posts all of its executed
commands at once or none of them.  It deadlocks: the completion queue's room frees only
when the polling window is full, and the window may need some of the very entries the
controller holds back.  The controller therefore posts as many as fit.

``explore_fetch`` models several controller wavefronts that share one submission
queue: each claims a run of issued commands by reading the queue's fetch pointer and
its doorbell and then advancing the fetch pointer with a compare-and-swap, while
submitters keep ringing the doorbell.  With the doorbell read first, a controller can
pair a stale doorbell with a fetch pointer that others have already moved past it; the
unsigned difference wraps and the claim reaches beyond the doorbell.  Reading the fetch
pointer first (the doorbell can only have grown since), or rejecting differences larger
than the queue, keeps every claim behind the doorbell.
"""
from __future__ import annotations

from collections import deque

EMPTY, UPDATED, ISSUED = 0, 1, 2


def _agile_init(depth, window, reqs):
    slots = tuple((s, EMPTY) for s in range(depth))
    cq = tuple((0, -1) for _ in range(depth))  # (phase bit in memory, cid)
    threads = tuple((0, -1, 0) for _ in reqs)  # (pc, base ticket, written mask)
    # ticket, db, head, inflight(frozenset of slot), cq_tail, cq_head, offset, mask, done
    return (0, 0, 0, frozenset(), 0, 0, 0, 0, frozenset(), slots, cq, threads)


def _agile_succ(state, depth, window, reqs, ring_early=True, batch_post=False):
    (ticket, db, head, infl, cq_tail, cq_head, off, mask, done, slots, cq, threads) = state
    out = []
    for t, (pc, base, wr) in enumerate(threads):
        n = reqs[t]
        if pc == 0:  # one atomic reservation for the whole wave
            th = list(threads)
            th[t] = (1, ticket, 0)
            out.append((ticket + n, db, head, infl, cq_tail, cq_head, off, mask, done, slots, cq,
                        tuple(th)))
        elif pc == 1:
            for i in range(n):
                if wr >> i & 1:
                    continue
                T = base + i
                s = T % depth
                if slots[s] == (T, EMPTY):
                    sl = list(slots)
                    sl[s] = (T, UPDATED)
                    nwr = wr | (1 << i)
                    th = list(threads)
                    th[t] = (2 if nwr == (1 << n) - 1 else 1, base, nwr)
                    out.append((ticket, db, head, infl, cq_tail, cq_head, off, mask, done,
                                tuple(sl), cq, tuple(th)))
        if pc == 2 or (pc == 1 and ring_early):
            # a wave rings for what it has written while it still waits for slots of
            # its own later commands (ringing only after all writes can deadlock)
            p = db
            sl = list(slots)
            while sl[p % depth] == (p, UPDATED):
                sl[p % depth] = (p, ISSUED)
                p += 1
            if p != db:
                out.append((ticket, p, head, infl, cq_tail, cq_head, off, mask, done,
                            tuple(sl), cq, threads))
        if pc == 2:
            if db >= base + n:
                th = list(threads)
                th[t] = (3, base, wr)
                out.append((ticket, db, head, infl, cq_tail, cq_head, off, mask, done, slots,
                            cq, tuple(th)))
        elif pc == 3:
            if all((base + i) in done for i in range(n)):
                th = list(threads)
                th[t] = (4, base, wr)
                out.append((ticket, db, head, infl, cq_tail, cq_head, off, mask, done, slots,
                            cq, tuple(th)))
    # controller: fetch
    if head < db:
        out.append((ticket, db, head + 1, infl | {head % depth}, cq_tail, cq_head, off, mask,
                    done, slots, cq, threads))
    # controller: complete any fetched command (out of order) when the CQ has room
    if batch_post and infl:
        # all-or-nothing: every fetched command is posted at once, or none
        if cq_tail - cq_head + len(infl) <= depth:
            c = list(cq)
            t = cq_tail
            for s in sorted(infl):
                c[t % depth] = (((t // depth) & 1) ^ 1, s)
                t += 1
            out.append((ticket, db, head, frozenset(), t, cq_head, off, mask, done, slots,
                        tuple(c), threads))
    elif cq_tail - cq_head < depth:
        for s in infl:
            c = list(cq)
            phase = ((cq_tail // depth) & 1) ^ 1
            c[cq_tail % depth] = (phase, s)
            out.append((ticket, db, head, infl - {s}, cq_tail + 1, cq_head, off, mask, done,
                        slots, tuple(c), threads))
    # completion service lanes
    for i in range(window):
        if mask >> i & 1:
            continue
        pos = off + i
        exp = ((pos // depth) & 1) ^ 1
        ph, cid = cq[pos % depth]
        if ph == exp:
            T, st = slots[cid]
            assert st == ISSUED, "completion for a slot that was not issued"
            assert T not in done, "command completed twice"
            sl = list(slots)
            sl[cid] = (T + depth, EMPTY)
            out.append((ticket, db, head, infl, cq_tail, cq_head, off, mask | (1 << i),
                        done | {T}, tuple(sl), cq, threads))
    if mask == (1 << window) - 1:
        out.append((ticket, db, head, infl, cq_tail, off + window, off + window, 0, done, slots,
                    cq, threads))
    return out


def _agile_finished(state):
    return all(pc == 4 for pc, _, _ in state[-1])


def _naive_init(depth, reqs):
    slots = tuple(-1 for _ in range(depth))  # owner thread or -1
    threads = tuple((0, 0, frozenset()) for _ in reqs)  # (pc, issued count, held slots)
    return (0, frozenset(), frozenset(), slots, threads)  # db-less: (dummy, inflight, posted)


def _naive_succ(state, depth, reqs):
    (_, infl, posted, slots, threads) = state
    out = []
    for t, (pc, k, held) in enumerate(threads):
        n = reqs[t]
        if pc == 0:  # need a free SQE for request k (spins while the SQ is full)
            for s in range(depth):
                if slots[s] == -1:
                    sl = list(slots)
                    sl[s] = t
                    th = list(threads)
                    th[t] = (1 if k + 1 == n else 0, k + 1, held | {s})
                    out.append((0, infl | {s}, posted, tuple(sl), tuple(th)))
                    break
        elif pc == 1:  # consume own completions, releasing the held SQEs
            for s in held:
                if s in posted:
                    sl = list(slots)
                    sl[s] = -1
                    nh = held - {s}
                    th = list(threads)
                    th[t] = (2 if not nh else 1, k, nh)
                    out.append((0, infl, posted - {s}, tuple(sl), tuple(th)))
    for s in infl:
        out.append((0, infl - {s}, posted | {s}, slots, threads))
    return out


def _naive_finished(state):
    return all(pc == 2 for pc, _, _ in state[-1])


def explore(model: str, depth: int, reqs, window: int = None, limit: int = 2_000_000):
    """Breadth-first search of all interleavings.  Returns (states, deadlock or None)."""
    if model in ("agile", "agile_ring_last", "agile_batch_post"):
        window = window or depth
        assert depth % window == 0
        start = _agile_init(depth, window, reqs)
        early = model != "agile_ring_last"
        batch = model == "agile_batch_post"
        succ = lambda s: _agile_succ(s, depth, window, reqs, early, batch)  # noqa: E731
        fin = _agile_finished
    elif model == "naive":
        start = _naive_init(depth, reqs)
        succ = lambda s: _naive_succ(s, depth, reqs)  # noqa: E731
        fin = _naive_finished
    else:
        raise ValueError(model)
    seen = {start}
    q = deque([start])
    while q:
        s = q.popleft()
        nxt = succ(s)
        if not nxt and not fin(s):
            return len(seen), s
        for n in nxt:
            if n not in seen:
                seen.add(n)
                if len(seen) > limit:
                    raise RuntimeError("state limit exceeded")
                q.append(n)
    return len(seen), None


def explore_fetch(order: str, controllers: int = 2, total: int = 4, depth: int = 2,
                  nfree: int = 2, guard: bool = False, limit: int = 2_000_000):
    """Shared fetch of one SQ by several controllers (32-bit pointers).

    order: "db_first" or "fetch_first".  guard: skip a claim whose difference exceeds the
    depth.  Returns (states, violating state or None); a violation is a successful claim
    whose end lies beyond the doorbell at the moment of the claim."""
    M = 1 << 32
    first_db = order == "db_first"
    if order not in ("db_first", "fetch_first"):
        raise ValueError(order)
    start = (0, 0, tuple((0, 0, 0) for _ in range(controllers)))  # db, fetch, (pc, r1, r2)
    seen = {start}
    q = deque([start])
    while q:
        st = q.popleft()
        db, fetch, cs = st
        nxt = []
        # submitters ring one more command while the queue has a free slot (fetched
        # commands complete at once, so the slots behind the fetch pointer are free)
        if db < total and db - fetch < depth:
            nxt.append((db + 1, fetch, cs))
        for i, (pc, r1, r2) in enumerate(cs):
            c = list(cs)
            if pc == 0:
                c[i] = (1, db if first_db else fetch, 0)
                nxt.append((db, fetch, tuple(c)))
            elif pc == 1:
                c[i] = (2, r1, fetch if first_db else db)
                nxt.append((db, fetch, tuple(c)))
            else:
                r_db, r_f = (r1, r2) if first_db else (r2, r1)
                avail = (r_db - r_f) % M
                c[i] = (0, 0, 0)
                if avail == 0 or (guard and avail > depth):
                    nxt.append((db, fetch, tuple(c)))
                    continue
                k = min(avail, nfree)
                if fetch == r_f:
                    if r_f + k > db:
                        return len(seen), (db, fetch, cs, i)
                    nxt.append((db, r_f + k, tuple(c)))
                else:
                    nxt.append((db, fetch, tuple(c)))
        for n in nxt:
            if n not in seen:
                seen.add(n)
                if len(seen) > limit:
                    raise RuntimeError("state limit exceeded")
                q.append(n)
    return len(seen), None
