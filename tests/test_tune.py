"""CPU checks of the serving autotuner's search and of its committed summary format (no
GPU: the trial function is replaced by a synthetic score)."""
import numpy as np

from paper_2504_19365_amd import tune


def _fake_trial(score_of, calls):
    def trial(image, rows, dim, point, stream, cache_bytes, K=0, latency_ns=0, iops_cap=0,
              mode=1):
        calls.append(dict(point))
        s = score_of(point)
        return {"lookups_per_s": s, "p50_s": 1e-3, "p99_s": 2e-3, "elapsed_s": 0.1}
    return trial


def test_coordinate_descent_finds_separable_optimum(monkeypatch):
    # a separable score with one best value per axis; the descent must land on it
    best = {"line_bytes": 8192, "assoc": 16, "num_qp": 32, "qp_depth": 512,
            "ctrl_waves": 32, "user_waves": 256, "max_inflight_lines": 768}

    def score(p):
        s = 1e6
        for k, v in p.items():
            vals = tune.SPACE[k]
            s *= 1.0 + 0.1 * (len(vals) - abs(vals.index(v) - vals.index(best[k])))
        return s

    calls = []
    monkeypatch.setattr(tune, "serve_trial", _fake_trial(score, calls))
    monkeypatch.setattr(tune.gen, "serve_stream", lambda *a, **k: None)
    res = tune.tune(None, 65536, 64, cache_bytes=1 << 20, rounds=3, log=lambda *a: None)
    assert res["best"] == best
    # every trial was feasible and scored once
    keys = [tuple(sorted(c.items())) for c in calls]
    assert len(keys) == len(set(keys))
    for c in calls:
        assert tune.feasible(c, 1 << 20)


def test_infeasible_points_are_skipped(monkeypatch):
    calls = []
    monkeypatch.setattr(tune, "serve_trial", _fake_trial(lambda p: 1e6 * p["assoc"], calls))
    monkeypatch.setattr(tune.gen, "serve_stream", lambda *a, **k: None)
    # a 128 KiB cache holds 2 lines of 64 KiB: no associativity of 4 or more fits there
    res = tune.tune(None, 65536, 64, cache_bytes=128 << 10, rounds=2, log=lambda *a: None)
    for c in calls:
        assert (128 << 10) // c["line_bytes"] >= c["assoc"]
    assert res["best"]["assoc"] == 32 and res["best"]["line_bytes"] <= 4096


def test_summary_round_trip(tmp_path):
    res = {"best": {"line_bytes": 4096, "assoc": 4, "num_qp": 64, "qp_depth": 1024,
                    "ctrl_waves": 16, "user_waves": 512, "max_inflight_lines": 512},
           "best_lookups_per_s": 3.6e6, "requests": 2000,
           "trials": [{"point": dict(tune.START), "lookups_per_s": 1.2e6, "p50_s": 0.01,
                       "p99_s": 0.02}]}
    p = tmp_path / "s.md"
    p.write_text(tune.summary_markdown(res, "python -m paper_2504_19365_amd.tune"))
    got = tune.load_chosen(str(p))
    assert got == res["best"]
    geom, opts = tune.split_point(got)
    assert geom == {"line_bytes": 4096, "assoc": 4, "num_qp": 64, "qp_depth": 1024,
                    "ctrl_waves": 16}
    assert opts == {"user_waves": 512, "max_inflight_lines": 512}
    assert np.isfinite(res["best_lookups_per_s"])
