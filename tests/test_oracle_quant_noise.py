"""Pins of the oracle's noise generator and quantisation proxy.

The quantisation proxy follows Section IV-C (eq. q-train, eq. softround);
the noise generator is Philox4x32-10 (Salmon et al., SC'11) with Box-Muller.
"""
import math

import numpy as np
import pytest
import torch

from oracle import philox
from oracle.coolchic_ref import softround, q_train, q_hard


# Known-answer vectors published with the Random123 library for
# Philox4x32-10: (counter, key) -> output.
KAT = [
    ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF, 0xFFFFFFFF),
     (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
]


@pytest.mark.parametrize("ctr,key,expect", KAT)
def test_philox_known_answers(ctr, key, expect):
    out = philox.philox4x32_10(*ctr, *key)
    assert tuple(int(x) for x in out) == expect


def test_philox_vectorised_matches_scalar():
    i = np.arange(50, dtype=np.uint64)
    vec = philox.philox4x32_10(7, 3, i, 0, 11, 12)
    for j in (0, 1, 17, 49):
        sc = philox.philox4x32_10(7, 3, j, 0, 11, 12)
        assert all(int(v[j]) == int(s) for v, s in zip(vec, sc))


def test_box_muller_closed_form():
    # r0 = 0xffffffff -> u1 = (2^24 - 1 + 1/2) 2^-24 ; r1 = 0 -> u2 = 0, cos = 1
    u1 = (2 ** 24 - 0.5) / 2 ** 24
    z = philox.box_muller(np.array([0xFFFFFFFF], np.uint32), np.array([0], np.uint32))
    assert z[0] == pytest.approx(math.sqrt(-2 * math.log(u1)), rel=1e-15)
    # u2 = 1/2 -> cos(pi) = -1 ; r0 >> 8 = 0 -> u1 = 2^-25
    z = philox.box_muller(np.array([0], np.uint32), np.array([0x80000000], np.uint32))
    assert z[0] == pytest.approx(-math.sqrt(2 * 25 * math.log(2)), rel=1e-14)


def test_latent_noise_moments_and_independence():
    n = philox.latent_noise(seed=123, t=5, k=0, n=400_000)
    assert abs(n.mean()) < 0.01
    assert abs(n.var() - 1.0) < 0.01
    # kurtosis of a Gaussian is 3
    assert abs(np.mean(n ** 4) / n.var() ** 2 - 3.0) < 0.05
    m = philox.latent_noise(seed=123, t=6, k=0, n=400_000)
    assert abs(np.corrcoef(n, m)[0, 1]) < 0.01
    assert not np.array_equal(philox.latent_noise(123, 5, 1, 10), n[:10])


T_VALUES = [0.05, 0.08, 0.2, 0.35, 1.0]


@pytest.mark.parametrize("T", T_VALUES)
def test_softround_fixes_integers_and_half_integers(T):
    n = torch.arange(-5, 6, dtype=torch.float64)
    assert torch.allclose(softround(n, T), n, atol=1e-14)
    assert torch.allclose(softround(n + 0.5, T), n + 0.5, atol=1e-14)


def test_softround_limits():
    x = torch.linspace(-3.3, 3.3, 97, dtype=torch.float64)
    x = x[(x - torch.floor(x) - 0.5).abs() > 0.05]
    # T -> 0: hard rounding
    assert torch.allclose(softround(x, 1e-3), torch.round(x), atol=1e-9)
    # T -> infinity: identity (tanh(a) ~ a)
    assert torch.allclose(softround(x, 1e4), x, atol=1e-6)


@pytest.mark.parametrize("T", T_VALUES)
def test_softround_is_c1_at_integers(T):
    eps = 1e-7
    for n in (-2.0, 0.0, 3.0):
        lo = softround(torch.tensor(n - eps, dtype=torch.float64), T)
        hi = softround(torch.tensor(n + eps, dtype=torch.float64), T)
        assert abs(float(hi - lo)) < 1e-5
        x = torch.tensor([n - 1e-9, n + 1e-9], dtype=torch.float64, requires_grad=True)
        softround(x, T).sum().backward()
        d = x.grad
        # closed form of the slope at an integer: (1 - tanh^2(1/2T)) / (2T tanh(1/2T))
        a = math.tanh(1 / (2 * T))
        expect = (1 - a * a) / (2 * T * a)
        assert float(d[0]) == pytest.approx(expect, rel=1e-6)
        assert float(d[1]) == pytest.approx(expect, rel=1e-6)


def test_softround_monotone_and_odd_symmetric():
    x = torch.linspace(-4, 4, 2001, dtype=torch.float64)
    s = softround(x, 0.2)
    assert torch.all(s[1:] >= s[:-1])
    assert torch.allclose(softround(-x, 0.2), -s, atol=1e-12)


def test_q_train_noise_free_is_double_softround():
    y = torch.linspace(-2, 2, 41, dtype=torch.float64)
    assert torch.allclose(q_train(y, 0.3, 0.0, torch.zeros_like(y)),
                          softround(softround(y, 0.3), 0.3))
    # integer latents stay put with zero noise
    n = torch.arange(-3, 4, dtype=torch.float64)
    assert torch.allclose(q_train(n, 0.3, 0.5, torch.zeros_like(n)), n, atol=1e-14)


def test_q_hard_rounds_half_to_even_with_identity_gradient():
    y = torch.tensor([-1.5, -0.5, 0.5, 1.5, 2.5, 0.49, -0.51], dtype=torch.float64,
                     requires_grad=True)
    out = q_hard(y)
    assert out.tolist() == [-2.0, -0.0, 0.0, 2.0, 2.0, 0.0, -1.0]
    out.sum().backward()
    assert torch.all(y.grad == 1.0)
