"""The autotuner's search and cache on the host, with a synthetic cost in
place of GPU timing (the GPU test checks that tuned parameters leave results
unchanged)."""
import json

from paper_1101_4127_amd import autotune as A
from paper_1101_4127_amd import workloads as W


def separable_cost(cfg):
    """Minimum at run_len 1024, refill_min 24, blocks_per_cu 2 (tiled) and
    brick 2, chunk 256, refill 8, bpcu 4 (per-packet), the per-packet one
    slower overall."""
    if cfg.get("direct"):
        return 50.0 + abs(cfg["brick_log2"] - 2) + abs(cfg["wave_chunk"] - 256) / 256 \
            + abs(cfg["refill_min"] - 8) / 4 + abs(cfg["blocks_per_cu"] - 4)
    return 10.0 + abs(cfg["run_len"] - 1024) / 512 + abs(cfg["refill_min"] - 24) / 8 \
        + abs(cfg["blocks_per_cu"] - 2)


def test_coordinate_descent_finds_the_separable_minimum():
    best, t, log = A.coordinate_descent(separable_cost, A.DEFAULT_TILED, A.SPACE_TILED)
    assert best == {"direct": False, "run_len": 1024, "refill_min": 24, "blocks_per_cu": 2}
    assert t == 10.0
    assert len(log) == len({json.dumps(c, sort_keys=True) for c, _ in log})    # nothing timed twice


def test_tune_picks_the_faster_kind_and_caches(tmp_path):
    w = W.small_mixed(n=8, n_src=2, packets=2000)
    cache = str(tmp_path / "tune.json")
    calls = []

    def cost(cfg):
        calls.append(cfg)
        return separable_cost(cfg)
    r = A.tune(w, fp64=False, cache=cache, measure=cost)
    assert r["config"]["direct"] is False and r["march_ms"] == 10.0
    n = len(calls)
    again = A.tune(w, fp64=False, cache=cache, measure=cost)
    assert len(calls) == n and again["config"] == r["config"]             # served from the cache
    other = A.tune(w, fp64=True, cache=cache, measure=cost)                  # another signature
    assert len(calls) > n and other["signature"] != r["signature"]
    table = json.load(open(cache))
    assert set(table) == {r["signature"], other["signature"]}


def test_signature_depends_on_the_shape_only():
    a = W.small_mixed(n=8, n_src=2, packets=2000)
    b = W.small_mixed(n=8, n_src=2, packets=2000, seed=9)
    c = W.small_mixed(n=12, n_src=2, packets=2000)
    assert A.signature(a, False) == A.signature(b, False)
    assert A.signature(a, False) != A.signature(c, False)
    assert A.signature(a, False) != A.signature(a, True)
