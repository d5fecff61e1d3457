"""Host logic of the launch-shape autotuner: size buckets, cache keys and
the JSON cache (no GPU)."""
import json

from paper_2605_02726_amd import autotune as at
from paper_2605_02726_amd import workloads as wl


def test_size_bucket_rounds_sides_up_to_256():
    assert at.size_bucket(512, 768) == "512x768"
    assert at.size_bucket(513, 1) == "768x256"
    assert at.size_bucket(256, 255) == "256x256"


def test_cache_key_separates_device_precision_decoder_and_bucket():
    hop, mop = wl.config_hop(), wl.config_preset("MOP")
    k = at.cache_key(hop, "bf16", 512, 768, "devA")
    assert k == at.cache_key(hop, "bf16", 500, 700, "devA")
    others = {at.cache_key(hop, "fp32", 512, 768, "devA"), at.cache_key(mop, "bf16", 512, 768, "devA"),
              at.cache_key(hop, "bf16", 512, 1024, "devA"), at.cache_key(hop, "bf16", 512, 768, "devB")}
    assert k not in others and len(others) == 4


def test_shape_cache_round_trip(tmp_path):
    path = str(tmp_path / "shapes.json")
    mc = wl.config_hop()
    c = at.ShapeCache(path)
    assert c.get(mc, "bf16", 512, 768, "dev") is None
    shape = {"arm_wgs": 96, "syn_chunks_per_wg": 12, "res_tiles_per_wg": 2}
    c.put(mc, "bf16", 512, 768, shape, 0.3, "dev")
    d = at.ShapeCache(path)
    assert d.get(mc, "bf16", 400, 600, "dev") == shape
    assert d.get(mc, "fp32", 512, 768, "dev") is None
    with open(path) as f:
        e = json.load(f)
    assert list(e.values())[0]["ms_per_step"] == 0.3
    m = at.ShapeCache(None)
    m.put(mc, "bf16", 64, 64, shape, 1.0, "dev")
    assert m.get(mc, "bf16", 64, 64, "dev") == shape


def test_search_is_coordinate_descent_with_a_minimum_gain():
    # separable cost: the best value of each knob wins when it gains > 1%
    cost = {"a": {1: 1.0, 2: 0.9, 3: 0.95}, "b": {10: 0.5, 20: 0.496, 30: 0.3}}
    calls = []

    def measure(shape):
        calls.append(dict(shape))
        return cost["a"][shape["a"]] + cost["b"][shape["b"]]
    best, ms, start_ms, trials = at.search({"a": 1, "b": 10}, [("a", (1, 2, 3)), ("b", (10, 20, 30))],
                                           measure, min_gain=0.01)
    assert best == {"a": 2, "b": 30}
    assert start_ms == 1.5 and abs(ms - 1.2) < 1e-12
    # the start once, then every other candidate of a knob with the others at their best
    assert calls == [{"a": 1, "b": 10}, {"a": 2, "b": 10}, {"a": 3, "b": 10},
                     {"a": 2, "b": 20}, {"a": 2, "b": 30}]
    assert len(trials) == len(calls)
    # a gain below min_gain keeps the earlier shape
    best, _, _, _ = at.search({"a": 1, "b": 10}, [("b", (20,))], measure, min_gain=0.01)
    assert best == {"a": 1, "b": 10}


def test_search_rounds_revisit_knobs_that_interact():
    """With a knob whose best value depends on another, a second sweep from
    the first sweep's best finds the joint optimum; shapes timed once are not
    timed again, and a round that changes nothing ends the search."""
    cost = {(1, 10): 1.0, (2, 10): 0.995, (1, 20): 0.99, (2, 20): 0.80, (3, 10): 1.2, (3, 20): 1.2}
    calls = []

    def measure(shape):
        calls.append((shape["a"], shape["b"]))
        return cost[(shape["a"], shape["b"])]
    knobs = [("a", (1, 2, 3)), ("b", (10, 20))]
    best, ms, _, _ = at.search({"a": 1, "b": 10}, knobs, measure, min_gain=0.01, rounds=1)
    assert best == {"a": 1, "b": 10}          # (2, 10) and (1, 20) each gain < 1%
    calls.clear()
    best, ms, _, trials = at.search({"a": 1, "b": 10}, knobs, measure, min_gain=0.005, rounds=3)
    assert best == {"a": 2, "b": 20} and ms == 0.80
    assert len(calls) == len(set(calls)) == len(trials)
