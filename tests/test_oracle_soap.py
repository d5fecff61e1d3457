"""Pins of the SOAP oracle (oracle/soap.py) against what the algorithm and
linear algebra fix: eigenbases at the first call, the closed form of a
one-dimensional tensor under a constant gradient, the reduction to
elementwise Adam when every gradient is diagonal, equivariance under
orthogonal changes of basis, the refresh as a power iteration towards the
eigenvectors, and mode products against einsum.  CPU only."""
import numpy as np
import pytest

from oracle import coolchic_ref as R
from oracle import soap as S
from paper_2605_02726_amd import workloads as wl


class One:
    """SoapState restricted to one tensor of a given shape."""

    def __init__(self, shape):
        self.st = S.SoapState.__new__(S.SoapState)
        self.st.layout = [("t", tuple(shape), 0)]
        self.st.n = int(np.prod(shape))
        self.st.s = 0
        self.st.started = False
        self.st.m = {"t": np.zeros(shape)}
        self.st.v = {"t": np.zeros(shape)}
        self.st.p = {"t": [None] * len(shape)}
        self.st.q = {"t": [None] * len(shape)}

    def step(self, theta, g, lr):
        return self.st.step(theta.reshape(-1), g.reshape(-1), lr).reshape(theta.shape)


def test_layout_matches_the_parameter_vector():
    for mk in (wl.config_hop, wl.config_small, wl.config_tiny):
        mc = mk()
        lay = S.tensors(mc.as_dict())
        assert [(n, tuple(s)) for n, s, _ in lay] == [(n, tuple(s)) for n, s, _ in wl.param_spec(mc)]
        assert lay[-1][2] + int(np.prod(lay[-1][1])) == wl.n_params(mc)


def test_first_call_moves_nothing_and_sets_eigenbases():
    rng = np.random.default_rng(0)
    o = One((5, 7))
    th = rng.normal(size=(5, 7))
    g = rng.normal(size=(5, 7))
    assert np.array_equal(o.step(th, g, 1e-2), th)
    for d, ref in ((0, g @ g.T), (1, g.T @ g)):
        p, q = o.st.p["t"][d], o.st.q["t"][d]
        assert np.allclose(p, (1 - S.PRECOND_BETA) * ref, rtol=1e-13, atol=1e-15)
        assert np.allclose(q.T @ q, np.eye(q.shape[0]), atol=1e-12)
        lam = q.T @ p @ q
        assert np.allclose(lam - np.diag(np.diag(lam)), 0.0, atol=1e-12)
        w = np.diag(lam)
        assert np.all(np.diff(w) <= 1e-12)                 # descending
        assert np.allclose(np.sort(w)[::-1], np.sort(np.linalg.eigvalsh(p))[::-1], atol=1e-12)


def test_one_dimensional_tensor_under_a_constant_gradient():
    """m_s = g (1 - b1^s), v_s = g^2 (1 - b2^s), so each update is
    lr g sqrt(1 - b2^s) / (|g| sqrt(1 - b2^s) + eps)."""
    o = One((3,))
    g = np.array([0.5, -2.0, 1e-3])
    th = np.zeros(3)
    lr = 1e-2
    th = o.step(th, g, lr)
    for s in range(1, 8):
        new = o.step(th, g, lr)
        c = np.sqrt(1 - S.BETA2 ** s)
        assert np.allclose(th - new, lr * g * c / (np.abs(g) * c + S.EPS), rtol=1e-12)
        th = new


@pytest.mark.parametrize("shape", [(4, 4), (4, 6), (6, 4)])
def test_diagonal_gradients_reduce_to_elementwise_adam(shape):
    """With every gradient diagonal (distinct magnitudes, fixed order) the
    factors stay diagonal, the bases are the coordinate axes (the extra
    axes of a rectangular tensor never see a gradient) and SOAP is Adam, in
    its step form, on the diagonal; nothing else moves."""
    rng = np.random.default_rng(1)
    n = 4
    o = One(shape)
    th = rng.normal(size=shape)
    th0 = th.copy()
    m = np.zeros(n)
    v = np.zeros(n)
    lr = 1e-2
    for t in range(30):
        a = np.array([4.0, 2.0, 1.0, 0.5]) * (1.0 + 0.3 * np.sin(t + np.arange(n)))
        a *= np.where(rng.random(n) < 0.5, -1.0, 1.0)
        g = np.zeros(shape)
        g[np.arange(n), np.arange(n)] = a
        th = o.step(th, g, lr)
        if t == 0:
            continue
        m = S.BETA1 * m + (1 - S.BETA1) * a
        v = S.BETA2 * v + (1 - S.BETA2) * a * a
        s = t
        th0[np.arange(n), np.arange(n)] -= lr * np.sqrt(1 - S.BETA2 ** s) / (1 - S.BETA1 ** s) * \
            m / (np.sqrt(v) + S.EPS)
    assert np.allclose(th, th0, rtol=1e-10, atol=1e-12)


def _orth(rng, n):
    q, r = np.linalg.qr(rng.normal(size=(n, n)))
    return q * np.sign(np.diag(r))


@pytest.mark.parametrize("shape", [(5, 5), (3, 3)])
def test_equivariance_under_orthogonal_change_of_basis(shape):
    """Running SOAP on U A_t V^T from U theta_0 V^T gives U theta_t V^T at
    every step, through basis refreshes.  Square shapes: both factors have
    full rank and distinct eigenvalues from the first call on, so the bases
    are unique up to sign (a rectangular gradient leaves a null space whose
    basis, and so the first updates along it, no rule fixes)."""
    rng = np.random.default_rng(2)
    m, n = shape
    U, V = _orth(rng, m), _orth(rng, n)
    a = One(shape)
    b = One(shape)
    th_a = rng.normal(size=shape)
    th_b = U @ th_a @ V.T
    for t in range(27):
        g = rng.normal(size=shape) * np.linspace(1.0, 2.0, n)[None, :]
        th_a = a.step(th_a, g, 1e-2)
        th_b = b.step(th_b, U @ g @ V.T, 1e-2)
        assert np.allclose(th_b, U @ th_a @ V.T, rtol=1e-8, atol=1e-10), t


def test_refresh_converges_to_the_eigenvectors():
    rng = np.random.default_rng(3)
    n = 6
    Qt = _orth(rng, n)
    lam = np.array([9.0, 5.0, 3.0, 2.0, 1.0, 0.5])
    P = Qt @ np.diag(lam) @ Qt.T
    q = _orth(rng, n)
    v = np.zeros((n, 2))
    for _ in range(300):
        q, v = S.refresh(P, q, v, 0)
    ref = S.eig_desc(P)
    assert np.allclose(np.abs(q.T @ ref), np.eye(n), atol=1e-8)


def test_refresh_permutes_the_second_moment_with_the_basis():
    n = 3
    P = np.diag([1.0, 3.0, 2.0])
    q = np.eye(n)
    v = np.arange(6.0).reshape(n, 2)
    q2, v2 = S.refresh(P, q, v, 0)
    assert np.array_equal(v2, v[[1, 2, 0]])
    assert np.allclose(np.abs(q2), np.eye(n)[:, [1, 2, 0]])


def test_mode_products_against_einsum():
    rng = np.random.default_rng(4)
    x = rng.normal(size=(3, 4, 2, 5))
    qs = [_orth(rng, k) for k in x.shape]
    ref = np.einsum("abcd,ai,bj,ck,dl->ijkl", x, *qs)
    assert np.allclose(S.rotate(x, qs), ref, atol=1e-12)
    assert np.allclose(S.rotate_back(S.rotate(x, qs), qs), x, atol=1e-12)
    g = rng.normal(size=(3, 3, 3, 3))
    assert np.allclose(S.unfold_outer(g, 2), np.einsum("abcd,abed->ce", g, g), atol=1e-12)


def test_encoder_with_soap_keeps_latent_adam_and_skips_first_parameter_update():
    mc = wl.config_tiny()
    H = W = 16
    img = wl.synth_image(H, W, 3)
    par = wl.init_params(mc, 3, arm_out_zero=False)
    lat = wl.random_latents(mc, H, W, 3, scale=1.0)
    a = R.OracleState(mc.as_dict(), H, W, img, 1e-2, 3, lat, par)
    b = R.OracleState(mc.as_dict(), H, W, img, 1e-2, 3, lat, par, optimizer="soap")
    a.step(1, 1e-2, 0.3, 0.2)
    b.step(1, 1e-2, 0.3, 0.2)
    n = a.n_lat
    assert np.array_equal(a.theta[:n], b.theta[:n])             # same latent Adam
    assert np.array_equal(b.theta[n:], par.astype(np.float64))  # no parameter update yet
    losses = [b.step(t, 1e-2, 0.3, 0.2)[0] for t in range(2, 40)]
    assert losses[-1] < losses[0]


def test_gram_schmidt_qr_is_the_library_qr_on_full_rank_input():
    rng = np.random.default_rng(5)
    for n in (3, 7, 24):
        z = rng.normal(size=(n, n)) @ np.diag(np.linspace(1.0, 3.0, n))
        assert np.allclose(S.qr_gs(z), S.qr_pos(z), atol=1e-10)


def test_gram_schmidt_qr_on_rank_deficient_input():
    """Rank r: the first r columns span the range of z, every column is a
    unit vector orthogonal to the others, and the replaced columns are the
    unit vectors' orthogonalised remainders (a fixed rule, not rounding)."""
    rng = np.random.default_rng(6)
    n, r = 6, 3
    z = rng.normal(size=(n, r)) @ rng.normal(size=(r, n))
    q = S.qr_gs(z)
    assert np.allclose(q.T @ q, np.eye(n), atol=1e-12)
    u, _, _ = np.linalg.svd(z)
    rng_basis = u[:, :r]
    assert np.allclose(rng_basis @ (rng_basis.T @ q[:, :r]), q[:, :r], atol=1e-10)
    # the rule is deterministic: scaling z does not change the result
    assert np.allclose(S.qr_gs(3.0 * z), q, atol=1e-10)
