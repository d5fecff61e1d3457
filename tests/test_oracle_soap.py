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


def _replaced(z, q, tol=S.QR_TOL):
    """Columns k of z that lie within tol of the span of q's first k columns."""
    out = []
    for k in range(z.shape[1]):
        nz = np.linalg.norm(z[:, k])
        res = z[:, k] - q[:, :k] @ (q[:, :k].T @ z[:, k])
        if nz == 0.0 or np.linalg.norm(res) <= tol * nz:
            out.append(k)
    return out


def _is_qr_within_tol(z, q, tol=S.QR_TOL):
    """What any QR of z with completed columns satisfies, whatever rule picks
    the completion: q orthonormal, and z + E = q R with R upper triangular
    and every column of E at most tol of the column of z (R = q^T z, so E's
    column k is the part of z_k outside the span of q's first k+1 columns);
    R's diagonal is positive where the column was not completed, and above
    -tol |z_k| where it was (the dropped remainder may point either way)."""
    n = z.shape[1]
    assert np.abs(q.T @ q - np.eye(n)).max() <= 1e-12
    r = q.T @ z
    rep = _replaced(z, q, tol)
    for k in range(n):
        nz = np.linalg.norm(z[:, k])
        assert np.linalg.norm(r[k + 1:, k]) <= tol * nz * (1 + 1e-6) + 1e-300
        assert r[k, k] >= -tol * nz * (1 + 1e-6) if k in rep else r[k, k] > 0.0


def test_gram_schmidt_completion_spans_the_complement_of_the_range():
    """Rank r with independent leading columns (the order a refresh produces
    when the eigenvalue estimates put the range first): the first r columns
    are the Householder QR of z's first r columns (numpy's LAPACK routine,
    signs made positive), which is unique, and the completed columns span
    the orthogonal complement of z's range, taken from the SVD.  Neither
    check uses the completion rule."""
    rng = np.random.default_rng(16)
    for n, r in ((6, 3), (24, 22), (30, 22), (40, 25), (5, 1)):
        a = rng.normal(size=(n, r))
        b = np.concatenate([np.eye(r), rng.normal(size=(r, n - r))], axis=1)
        z = a @ b
        q = S.qr_gs(z)
        _is_qr_within_tol(z, q)
        assert _replaced(z, q) == list(range(r, n))
        lib, _ = np.linalg.qr(z[:, :r])
        lib = lib * np.sign(np.diag(lib.T @ z[:, :r]))[None, :]
        assert np.abs(q[:, :r] - lib).max() <= 1e-10
        u = np.linalg.svd(z)[0]
        comp = u[:, r:] @ u[:, r:].T
        assert np.abs(q[:, r:] @ q[:, r:].T - comp).max() <= 1e-10
    # nothing to span: every column is completed, and the basis is orthonormal
    q0 = S.qr_gs(np.zeros((4, 4)))
    _is_qr_within_tol(np.zeros((4, 4)), q0)


def test_gram_schmidt_with_dependent_middle_columns_is_a_qr_within_tolerance():
    """A zero column first, a copy of an earlier column in the middle and a
    near-copy (within 1e-7 of it) further on: the result is still a QR of a
    matrix within tol of z, column by column, and z's range lies in the span
    of the columns that were not completed plus those completed before the
    last new direction."""
    rng = np.random.default_rng(17)
    n = 8
    z = rng.normal(size=(n, n))
    z[:, 0] = 0.0
    z[:, 3] = z[:, 1]
    z[:, 6] = 2.0 * z[:, 2] + 1e-7 * rng.normal(size=n)
    q = S.qr_gs(z)
    _is_qr_within_tol(z, q)
    rep = _replaced(z, q)
    assert rep[:2] == [0, 3] and 6 in rep
    u, s, _ = np.linalg.svd(z)
    rk = int(np.sum(s > 1e-6 * s[0]))
    assert n - rk <= len(rep)


def test_refresh_of_rank_deficient_soap_factors():
    """The refreshes of an 11-step oracle run (64x128, first refresh at the
    tenth update) include rank-deficient factors: the ARM output layer's
    input factor and the synthesis factors collect fewer gradient directions
    than their size.  For every refresh input z = P Q_sorted: the result is a
    QR of z within tol; its columns up to the first completed one equal the
    Householder QR of the same columns; every completed column is orthogonal
    to z's range within tol of |z|."""
    calls = []
    orig = S.qr_gs

    def spy(z, tol=S.QR_TOL):
        q = orig(z, tol)
        calls.append((z.copy(), q.copy()))
        return q

    mc = wl.config_hop()
    H, W, seed = 64, 128, 31
    ora = R.OracleState(mc.as_dict(), H, W, wl.synth_image(H, W, seed), 1e-3, seed,
                        wl.random_latents(mc, H, W, seed, scale=1.5),
                        wl.init_params(mc, seed, arm_out_zero=False), optimizer="soap")
    S.qr_gs = spy
    try:
        for t in range(1, 12):
            ora.step(t, *R.schedule(t, 200))
    finally:
        S.qr_gs = orig
    assert ora.soap.s == 10 and calls
    n_completed = 0
    for z, q in calls:
        _is_qr_within_tol(z, q)
        rep = _replaced(z, q)
        k0 = rep[0] if rep else z.shape[1]
        lib, _ = np.linalg.qr(z[:, :k0])
        lib = lib * np.sign(np.diag(lib.T @ z[:, :k0]))[None, :]
        assert np.abs(q[:, :k0] - lib).max() <= 1e-9
        zn = np.linalg.norm(z, 2)
        for k in rep:
            assert np.linalg.norm(z.T @ q[:, k]) <= S.QR_TOL * zn
        n_completed += len(rep)
    assert n_completed >= 10
