"""Autotuner for the block-I/O path's geometry.

Staged coordinate descent over line size, associativity, queue-pair count, queue depth,
the number of emulated-controller wavefronts, the number of user wavefronts the
serving kernel runs and the admission budget of cache lines (0 = as many as the cache
holds).  Each trial builds a context with the candidate
geometry over the same store, runs a short closed-loop serving session (every request
available at once, so the session measures sustainable throughput) and scores it in
lookups per second.  Points the library rejects (for example fewer lines than ways) are
skipped.  The result is a JSON-serialisable dict: the chosen geometry and every trial.
"""
from __future__ import annotations

import json
import os
import time

import numpy as np

from . import agile, gen

SPACE = {
    "line_bytes": [4096, 8192, 16384, 32768, 65536],
    "assoc": [4, 8, 16, 32],
    "num_qp": [4, 8, 16, 32, 64],
    "qp_depth": [256, 512, 1024, 2048, 4096],
    "ctrl_waves": [16, 32, 64, 128],
    "user_waves": [16, 32, 64, 128, 256, 512, 1024],
    "max_inflight_lines": [0, 256, 512, 768, 1024, 2048],
}
START = {"line_bytes": 4096, "assoc": 8, "num_qp": 16, "qp_depth": 1024, "ctrl_waves": 64,
         "user_waves": 16, "max_inflight_lines": 0}


def _config(point: dict, cache_bytes: int, latency_ns: int, iops_cap: int) -> dict:
    return dict(cache_bytes=cache_bytes, line_bytes=point["line_bytes"], assoc=point["assoc"],
                num_qp=point["num_qp"], qp_depth=point["qp_depth"],
                ctrl_waves=point["ctrl_waves"], latency_ns=latency_ns,
                iops_cap=iops_cap, timeout_ns=int(20e9))


def feasible(point: dict, cache_bytes: int) -> bool:
    lines = cache_bytes // point["line_bytes"]
    return lines >= point["assoc"] and lines % point["assoc"] == 0


def serve_trial(image, rows: int, dim: int, point: dict, stream, cache_bytes: int, K: int = 0,
                latency_ns: int = 0, iops_cap: int = 0, mode: int = agile.MODE_ASYNC) -> dict:
    """One closed-loop serving session; returns lookups/s and latency percentiles."""
    arrival, req_bag0, bag_off, idx = stream
    ctx = agile.Context(**_config(point, cache_bytes, latency_ns, iops_cap))
    try:
        ctx.open_store(image)
        tb = ctx.tables(rows, dim, 1)
        _, lat, rep = ctx.serve(tb, K, np.zeros_like(arrival), req_bag0, bag_off, idx, mode=mode,
                                user_waves=point.get("user_waves", 0),
                                max_inflight_lines=point.get("max_inflight_lines", 0))
        ctx.close_store()
    finally:
        ctx.shutdown()
    return {"lookups_per_s": rep["lookups"] / rep["elapsed_s"], "p50_s": float(np.median(lat)),
            "p99_s": float(np.percentile(lat, 99)), "elapsed_s": rep["elapsed_s"]}


def tune(image, rows: int, dim: int, cache_bytes: int = 1 << 20, requests: int = 2000,
         seed: int = 40, rounds: int = 2, K: int = 0, latency_ns: int = 0, iops_cap: int = 0,
         space: dict | None = None, start: dict | None = None, log=print) -> dict:
    space = space or SPACE
    point = dict(start or START)
    stream = gen.serve_stream(requests, 20000.0, rows, 1.05, seed)
    trials = []
    cache = {}

    def score(p):
        key = tuple(sorted(p.items()))
        if key in cache:
            return cache[key]
        if not feasible(p, cache_bytes):
            cache[key] = None
            return None
        t0 = time.perf_counter()
        try:
            r = serve_trial(image, rows, dim, p, stream, cache_bytes, K, latency_ns, iops_cap)
        except agile.AgileError as e:  # rejected configuration
            log(f"  skip {p}: {e}")
            cache[key] = None
            return None
        r["trial_s"] = time.perf_counter() - t0
        trials.append({"point": dict(p), **r})
        log(f"  {p} -> {r['lookups_per_s'] / 1e6:.3f} M lookups/s p99 {r['p99_s'] * 1e3:.2f} ms")
        cache[key] = r["lookups_per_s"]
        return cache[key]

    best = score(point)
    for _ in range(rounds):
        improved = False
        for axis, values in space.items():
            for v in values:
                if v == point[axis]:
                    continue
                cand = dict(point)
                cand[axis] = v
                sc = score(cand)
                if sc is not None and (best is None or sc > best * 1.02):
                    best, point, improved = sc, cand, True
        if not improved:
            break
    return {"best": point, "best_lookups_per_s": best, "trials": trials,
            "cache_bytes": cache_bytes}


# The committed summary of the tuning run whose chosen point the serving measurements use.
SUMMARY_PATH = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                            "profiles", "serve_autotune_tiny_table.md")

# Geometry keys that go to the context (agile_init); the others are serving options.
CONTEXT_KEYS = ("line_bytes", "assoc", "num_qp", "qp_depth", "ctrl_waves")
CHOSEN_PREFIX = "chosen: "


def split_point(point: dict):
    """(context geometry, serving options) of a tuned point."""
    geom = {k: point[k] for k in CONTEXT_KEYS if k in point}
    opts = {k: v for k, v in point.items() if k not in CONTEXT_KEYS and v}
    return geom, opts


def summary_markdown(res: dict, command: str) -> str:
    """A short text summary of a tuning run: the command, the chosen point on one
    machine-readable line, and every trial."""
    lines = ["# Serving autotuner: tiny table (65,536 x 64 fp32), 1 MiB cache", "",
             f"command: `{command}`", "",
             f"requests per trial: {res['requests']} (Poisson stream of the serving "
             f"workload, all available at once: a closed loop that measures sustainable "
             f"throughput); trials: {len(res['trials'])}", "",
             CHOSEN_PREFIX + json.dumps(res["best"], sort_keys=True),
             f"best_lookups_per_s: {res['best_lookups_per_s']:.1f}", "",
             "| # | " + " | ".join(SPACE) + " | M lookups/s | p50 ms | p99 ms |",
             "|---" * (len(SPACE) + 4) + "|"]
    for i, t in enumerate(res["trials"]):
        p = t["point"]
        lines.append(f"| {i} | " + " | ".join(str(p.get(k, "")) for k in SPACE) +
                     f" | {t['lookups_per_s'] / 1e6:.3f} | {t['p50_s'] * 1e3:.2f} | "
                     f"{t['p99_s'] * 1e3:.2f} |")
    return "\n".join(lines) + "\n"


def load_chosen(path: str) -> dict:
    """The chosen point of a committed tuning summary (see summary_markdown)."""
    with open(path) as f:
        for line in f:
            if line.startswith(CHOSEN_PREFIX):
                return json.loads(line[len(CHOSEN_PREFIX):])
    raise ValueError(f"{path}: no '{CHOSEN_PREFIX.strip()}' line")


def main(argv=None) -> None:
    import argparse
    import sys
    ap = argparse.ArgumentParser(description="tune the serving geometry on the tiny table")
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--rounds", type=int, default=2)
    ap.add_argument("--out", default="", help="write the markdown summary here")
    args = ap.parse_args(argv)
    rows, dim = 65536, 64
    buf = agile.PinnedBuffer(rows * dim * 4)
    gen.fill_table(buf.ptr, 0, rows, dim, 0)
    res = tune(buf, rows, dim, requests=args.requests, rounds=args.rounds,
               log=lambda *a: print(*a, flush=True))
    buf.free()
    res["requests"] = args.requests
    cmd = "python -m paper_2504_19365_amd.tune " + " ".join(argv if argv is not None else sys.argv[1:])
    text = summary_markdown(res, cmd.strip())
    if args.out:
        with open(args.out, "w") as f:
            f.write(text)
    print(text)


if __name__ == "__main__":
    main()
