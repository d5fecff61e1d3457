"""Launch shapes chosen by the autotuner change how workgroups split the
work, not the result: losses, latent gradients and ARM gradients stay
bitwise the same (the ARM's partial sums are per band whatever the number
of workgroups), synthesis and residual weight gradients change only by the
order of their partial sums; a batch mixing shapes equals each state run
alone; ``tune`` returns a valid shape and the server applies cached ones."""
import numpy as np
import pytest
import torch

from paper_2605_02726_amd import workloads as wl

pytestmark = pytest.mark.gpu

H, W = 128, 192


def _enc(mc, precision, seed=61, shape=None):
    from paper_2605_02726_amd.encoder import Encoder
    e = Encoder(mc, torch.from_numpy(wl.synth_image(H, W, seed)), 1e-3, seed,
                wl.random_latents(mc, H, W, seed), wl.init_params(mc, seed, arm_out_zero=False),
                precision=precision)
    if shape:
        e.set_launch_shape(**shape)
    return e


def _split(mc, g):
    n_lat = wl.n_latents(mc, H, W)
    spec = wl.param_spec(mc)
    n_arm = sum(1 for n, _, _ in spec if n.startswith("arm."))
    assert all(n.startswith("arm.") for n, _, _ in spec[:n_arm])      # ARM tensors come first
    arm = sum(int(np.prod(s)) for _, s, _ in spec[:n_arm])
    return g[:n_lat], g[n_lat:n_lat + arm], g[n_lat + arm:]


SHAPES = [dict(arm_wgs=7, syn_chunks_per_wg=6, res_tiles_per_wg=1),
          dict(arm_wgs=1, syn_chunks_per_wg=24, res_tiles_per_wg=4),
          dict(arm_wgs=0, syn_chunks_per_wg=64, res_tiles_per_wg=16)]


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("which", range(len(SHAPES)))
def test_launch_shape_changes_only_the_weight_sum_order(precision, which):
    from paper_2605_02726_amd.encoder import schedule
    mc = wl.config_hop()
    a = _enc(mc, precision)
    b = _enc(mc, precision, shape=SHAPES[which])
    got = b.launch_shape()
    for k, v in SHAPES[which].items():
        if v:
            assert got[k] == v
    for t in range(1, 4):
        lr, T, s = schedule(t, 20)
        ra, rb = a.step(t, lr, T, s), b.step(t, lr, T, s)
        ga, gb = a.grad(), b.grad()
        if t == 1:
            assert ra == rb
            la, aa, da = _split(mc, ga)
            lb, ab, db = _split(mc, gb)
            assert np.array_equal(la, lb)
            assert np.array_equal(aa, ab)
            scale = np.abs(da).max()
            assert np.max(np.abs(da - db)) <= 1e-5 * scale, np.max(np.abs(da - db)) / scale
        else:
            assert abs(ra[0] - rb[0]) <= 1e-5 * abs(ra[0])


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_batch_mixing_launch_shapes_equals_alone(precision):
    from paper_2605_02726_amd.encoder import schedule, step_batch, step_params
    mc = wl.config_hop()
    alone = [_enc(mc, precision, 70 + i, SHAPES[i]) for i in range(3)]
    batch = [_enc(mc, precision, 70 + i, SHAPES[i]) for i in range(3)]
    for t in range(1, 4):
        lr, T, s = schedule(t, 20)
        ra = [e.step(t, lr, T, s) for e in alone]
        rb = step_batch(batch, [step_params(t, lr, T, s)] * 3)
        assert ra == rb
    for x, y in zip(alone, batch):
        sx, sy = x.get_state(), y.get_state()
        for k in ("latents", "params", "m", "v"):
            assert np.array_equal(sx[k], sy[k]), k


def test_out_of_range_shapes_are_rejected():
    from paper_2605_02726_amd._lib import CCError
    mc = wl.config_hop()
    e = _enc(mc, "bf16")
    bands = e.launch_shape()["arm_bands"]
    for bad in (dict(arm_wgs=bands + 1), dict(syn_chunks_per_wg=3), dict(syn_chunks_per_wg=65),
                dict(res_tiles_per_wg=17), dict(res_tiles_per_wg=-1)):
        with pytest.raises(CCError):
            e.set_launch_shape(**bad)
    assert e.launch_shape()["arm_bands"] == bands


def test_tune_caches_a_valid_shape_and_the_server_applies_it(tmp_path):
    from paper_2605_02726_amd import autotune as at
    from paper_2605_02726_amd.serve import Job, Server
    mc = wl.config_hop()
    cache = at.ShapeCache(str(tmp_path / "shapes.json"))
    r = at.tune(mc, 256, 256, "bf16", steps=3, cache=cache)
    shape = r["shape"]
    assert shape["syn_chunks_per_wg"] in at.SYN_CHUNKS + (r["trials"][0][0]["syn_chunks_per_wg"],)
    assert r["ms_per_step"] <= r["default_ms_per_step"]
    assert at.ShapeCache(cache.path).get(mc, "bf16", 256, 256) == shape
    srv = Server(mc, "bf16", shapes=cache)
    srv.t0 = srv.clock()
    srv.submit(Job(rid=0, image=wl.synth_image(256, 256, 5), lam=1e-3, seed=5, n_iter=3,
                   params=wl.init_params(mc, 5)))
    srv._admit()
    got = srv.active[0][1].launch_shape()
    got.pop("arm_bands")
    assert got == shape
    # a smaller image of the same size bucket has fewer ARM bands: the cached
    # workgroup count is clamped to them
    cache.put(mc, "bf16", 256, 256, dict(shape, arm_wgs=10 ** 6), 1.0)
    srv.submit(Job(rid=1, image=wl.synth_image(192, 128, 6), lam=1e-3, seed=6, n_iter=3,
                   params=wl.init_params(mc, 6)))
    srv._admit()
    small = srv.active[1][1].launch_shape()
    assert small["arm_wgs"] == small["arm_bands"]
