"""The C-ABI library loads on the host, exports every function that
include/coolchic.h declares, and its host-only size/shape logic agrees with
the documented layouts.  No device calls."""
import ctypes as C
import os
import re

import pytest

from paper_2605_02726_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_2605_02726_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2605_02726_amd import build
        build.build()
    return _lib


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names.update(re.findall(r"\b(cc_\w+)\s*\(", text))
    return sorted(names)


def test_every_declared_function_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 14
    so = C.CDLL(lib.LIB_PATH)
    missing = [n for n in names if not hasattr(so, n)]
    assert not missing, missing
    # and the binding covers all of them
    assert set(names) <= set(lib.EXPORTED)


@pytest.mark.parametrize("mk", [wl.config_small, wl.config_hop, wl.config_tiny])
def test_param_and_latent_counts(lib, mk):
    mc = mk()
    cfg = lib.make_config(mc)
    L = lib.lib()
    assert L.cc_n_params(C.byref(cfg)) == wl.n_params(mc)
    assert L.cc_n_latents(C.byref(cfg), 512, 768) == wl.n_latents(mc, 512, 768)
    assert L.cc_state_bytes(C.byref(cfg), 512, 768) > 0


def test_rejects_bad_shapes(lib):
    L = lib.lib()
    mc = wl.config_hop()
    cfg = lib.make_config(mc)
    assert L.cc_config_supported(C.byref(cfg), 512, 768) == 1
    assert L.cc_config_supported(C.byref(cfg), 500, 768) == 0       # not a multiple of 64
    assert "multiples" in L.cc_last_error().decode()
    assert L.cc_state_bytes(C.byref(cfg), 0, 768) == 0
    bad = lib.make_config(mc)
    bad.n_spatial = 23                                              # shape not compiled in
    assert L.cc_config_supported(C.byref(bad), 512, 768) == 0
    bad = lib.make_config(mc)
    bad.p_min = 0.0
    assert L.cc_config_supported(C.byref(bad), 512, 768) == 0


def test_state_calls_reject_null(lib):
    L = lib.lib()
    assert L.cc_rd_eval(None, None, None) == lib.CC_ESTATE
    assert L.cc_encode_step(None, None, None, None) == lib.CC_ESTATE
    out = C.c_void_p()
    cfg = lib.make_config(wl.config_small())
    rc = L.cc_init_state(C.byref(cfg), 64, 64, None, 1e-3, 1, None, None, None, 0, None,
                         C.byref(out))
    assert rc == lib.CC_EINVAL and not out.value


@pytest.mark.parametrize("name", ["LOP", "MOP", "HOP", "VHOP"])
def test_table2_presets_are_supported(lib, name):
    """Every decoder preset of Table II is compiled in (parameter counts in
    the table: 0.5k, 1.0k, 1.9k, 2.7k)."""
    mc = wl.config_preset(name)
    cfg = lib.make_config(mc)
    L = lib.lib()
    assert L.cc_config_supported(C.byref(cfg), 512, 768) == 1, L.cc_last_error()
    n = L.cc_n_params(C.byref(cfg))
    assert n == wl.n_params(mc)
    target = {"LOP": 500, "MOP": 1000, "HOP": 1900, "VHOP": 2700}[name]
    assert abs(n - target) <= 0.25 * target


def test_fused_arm_covers_the_workload_and_the_presets(lib):
    """The BF16 form runs the MFMA ARM kernel for the 512x768 workload's
    decoder (with and without hyperlatents) and every Table II preset."""
    L = lib.lib()
    for mk in (wl.config_hop, wl.config_hop_hyper, wl.config_small,
               *[lambda n=n: wl.config_preset(n) for n in ("LOP", "MOP", "HOP", "VHOP")]):
        cfg = lib.make_config(mk(), lib.CC_BF16_FUSED)
        assert L.cc_arm_fused_available(C.byref(cfg)) == 1


@pytest.mark.parametrize("mk,H,W", [(wl.config_hop, 512, 768), (wl.config_hop_hyper, 512, 768),
                                    (wl.config_hop, 2048, 2048), (wl.config_small, 64, 64),
                                    (wl.config_hop, 320, 1088)])
def test_arm_band_packing(lib, mk, H, W):
    """Every band on exactly one workgroup, ascending within a workgroup, no
    workgroup empty; the packing (longest first onto the least loaded) keeps
    the largest load within one band of the even share; by default one band
    per workgroup (at most 512 workgroups)."""
    mc = mk()
    cfg = lib.make_config(mc, lib.CC_BF16_FUSED)
    nb, nd = C.c_int(0), C.c_int(0)
    assert lib.lib().cc_arm_band_plan(C.byref(cfg), H, W, 0, C.byref(nb), C.byref(nd), None, None) == 0
    levels = wl.grid_levels(mc)
    loads = []
    for k in levels:
        h, w = H >> k, W >> k
        loads += [min(2, h - y) * w + 256 for y in range(0, h, 2)]
    assert nb.value == len(loads)
    big = max(loads)
    for nw in sorted({1, 7, nd.value, nb.value, max(1, nb.value // 3)}):
        wbeg = (C.c_int * (nw + 1))()
        blist = (C.c_int * nb.value)()
        assert lib.lib().cc_arm_band_plan(C.byref(cfg), H, W, nw, None, None, wbeg, blist) == 0
        assert wbeg[0] == 0 and wbeg[nw] == nb.value
        assert sorted(blist) == list(range(nb.value))
        per = [list(blist[wbeg[i]:wbeg[i + 1]]) for i in range(nw)]
        assert all(p and p == sorted(p) for p in per)
        mx = max(sum(loads[b] for b in p) for p in per)
        assert mx <= sum(loads) / nw + big
        if nw == nd.value and nw < 512:
            assert nw == nb.value and mx <= big
    assert nd.value == min(nb.value, 512)
    with pytest.raises(AssertionError):
        assert lib.lib().cc_arm_band_plan(C.byref(cfg), H, W, nb.value + 1, None, None,
                                          (C.c_int * (nb.value + 2))(), None) == 0


def test_batch_sizes_outside_the_limit_are_rejected(lib):
    """Empty and oversized batches fail on the host (no device call)."""
    L = lib.lib()
    p = (lib.cc_step_params * 40)()
    states = (C.c_void_p * 40)()
    for n in (0, -1, lib.CC_MAX_BATCH + 1):
        assert L.cc_encode_step_batch(states, n, p, None, None) == lib.CC_EINVAL
    # a batch whose states are not initialised
    assert L.cc_encode_step_batch(states, 1, p, None, None) != lib.CC_OK
