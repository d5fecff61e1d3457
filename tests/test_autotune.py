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
