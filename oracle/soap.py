"""SOAP for the decoder parameters (Section IV-B), FP64 numpy.

TEST INFRASTRUCTURE ONLY.  Only the tests, the package's smoke check and the
benchmark's CPU-baseline leg may use this module; the product path never
does, and it shares no code with the GPU library.

The paper trains the ~2,000 decoder parameters with SOAP (Vyas et al., 2024:
Adam run in the eigenbasis of Shampoo's Kronecker-factored preconditioner)
and the latents with Adam, without stating SOAP's settings.  Readings:
  * SOAP's published defaults: beta1 = beta2 = 0.95, preconditioner average
    beta 0.95, eps 1e-8, basis refresh every 10 updates, bias correction, no
    weight decay; the learning rate follows the latents' schedule;
  * every parameter tensor of two or more dimensions gets one Kronecker
    factor per dimension d of size at most 48 (SOAP's bound on
    preconditioned dimensions, lowered to the sizes these decoders have),
    P_d <- b P_d + (1 - b) G_(d) G_(d)^T with G_(d) the mode-d unfolding of
    the gradient (for a matrix: G G^T and G^T G); one-dimensional tensors
    (biases, upsampling taps) get no factor and so run Adam in SOAP's step
    form;
  * the first call only sets the factors to (1 - b) G_(d) G_(d)^T and each
    basis Q_d to the eigenvectors of its factor, by descending eigenvalue;
    no parameter moves;
  * every later call, per tensor: rotate the gradient into the bases
    (G' = G x_d Q_d^T for every d), update the first moment M (kept in the
    original coordinates, rotated for use) and the second moment V (kept in
    the rotated coordinates, V <- b2 V + (1 - b2) G'^2), take
    N = rotate_back(rotate(M) / (sqrt(V) + eps)) and step
    theta <- theta - lr sqrt(1 - b2^s) / (1 - b1^s) N, s counting the updates;
    then update the factors with the same gradient and, when s is a multiple
    of 10, refresh every basis: order its columns by the estimated
    eigenvalues diag(Q^T P Q), descending (V is permuted along that dimension
    in the same way), then one power step Q <- qr(P Q) with the diagonal of R
    made positive;
  * that QR is Gram-Schmidt with one re-orthogonalisation pass, column by
    column; when P Q is rank-deficient the factorisation is not unique and
    its trailing columns would be set by rounding, so a column whose norm
    after orthogonalisation is below 1e-5 of its norm before is replaced by
    the first unit vector e_k, e_(k+1), ... (cyclic) that survives the same
    orthogonalisation.  For a full-rank, well-conditioned P Q this is the
    QR with a positive diagonal.
"""
from __future__ import annotations

from typing import Dict, List, Tuple

import numpy as np
import torch

from .coolchic_ref import n_params, unpack_params

BETA1 = 0.95
BETA2 = 0.95
PRECOND_BETA = 0.95
EPS = 1e-8
REFRESH = 10
MAX_PRECOND_DIM = 48


def tensors(cfg: Dict) -> List[Tuple[str, Tuple[int, ...], int]]:
    """(name, shape, offset in the decoder-parameter vector), layout order."""
    out, pos = [], 0
    for name, t in unpack_params(cfg, torch.zeros(n_params(cfg), dtype=torch.float64)).items():
        out.append((name, tuple(t.shape), pos))
        pos += int(t.numel())
    return out


def rotate(x: np.ndarray, qs: List[np.ndarray]) -> np.ndarray:
    """x' = x x_0 Q_0^T x_1 Q_1^T ...: x'[..i_d..] = sum_j Q_d[j, i_d] x[..j..]."""
    for d, q in enumerate(qs):
        if q is not None:
            x = np.moveaxis(np.tensordot(q, x, axes=([0], [d])), 0, d)
    return x


def rotate_back(x: np.ndarray, qs: List[np.ndarray]) -> np.ndarray:
    """Inverse of rotate: x[..i_d..] = sum_j Q_d[i_d, j] x'[..j..]."""
    for d, q in enumerate(qs):
        if q is not None:
            x = np.moveaxis(np.tensordot(q, x, axes=([1], [d])), 0, d)
    return x


def unfold_outer(g: np.ndarray, d: int) -> np.ndarray:
    """G_(d) G_(d)^T: sum over every other dimension."""
    other = [a for a in range(g.ndim) if a != d]
    return np.tensordot(g, g, axes=(other, other))


def eig_desc(p: np.ndarray) -> np.ndarray:
    """Eigenvectors of a symmetric matrix, columns by descending eigenvalue."""
    w, q = np.linalg.eigh(p)
    return q[:, np.argsort(-w, kind="stable")]


def qr_pos(z: np.ndarray) -> np.ndarray:
    """Q of the QR factorisation with a non-negative diagonal of R (library)."""
    q, r = np.linalg.qr(z)
    s = np.sign(np.diag(r))
    s[s == 0] = 1.0
    return q * s[None, :]


QR_TOL = 1e-5


def qr_gs(z: np.ndarray, tol: float = QR_TOL) -> np.ndarray:
    """Q of the QR factorisation of a square z: Gram-Schmidt with one
    re-orthogonalisation pass in column order (R's diagonal positive); a
    column that falls below tol of its norm is replaced by a unit vector."""
    n = z.shape[1]
    q = np.zeros_like(z, dtype=np.float64)
    for k in range(n):
        cands = [z[:, k]] + [np.eye(n)[:, (k + i) % n] for i in range(n)]
        for v0 in cands:
            v = np.array(v0, dtype=np.float64)
            n0 = np.linalg.norm(v)
            for _ in range(2):
                v = v - q[:, :k] @ (q[:, :k].T @ v)
            nv = np.linalg.norm(v)
            if n0 > 0 and nv > tol * n0:
                break
        q[:, k] = v / nv
    return q


def refresh(p: np.ndarray, q: np.ndarray, v: np.ndarray, d: int):
    """One basis refresh along dimension d: returns (new Q, permuted V)."""
    est = np.diag(q.T @ p @ q)
    order = np.argsort(-est, kind="stable")
    return qr_gs(p @ q[:, order]), np.take(v, order, axis=d)


class SoapState:
    """SOAP state of every decoder-parameter tensor of one image."""

    def __init__(self, cfg: Dict):
        self.layout = tensors(cfg)
        self.n = sum(int(np.prod(s)) for _, s, _ in self.layout)
        self.s = 0                   # updates done
        self.started = False
        self.m = {n: np.zeros(s) for n, s, _ in self.layout}
        self.v = {n: np.zeros(s) for n, s, _ in self.layout}
        self.p = {n: [None] * len(s) for n, s, _ in self.layout}
        self.q = {n: [None] * len(s) for n, s, _ in self.layout}

    def preconditioned(self, name: str) -> bool:
        return any(p is not None for p in self.p[name])

    def step(self, theta: np.ndarray, grad: np.ndarray, lr: float) -> np.ndarray:
        """One call with the gradient of the decoder parameters; returns the
        new parameter vector (unchanged on the first call)."""
        theta = np.array(theta, dtype=np.float64, copy=True)
        grad = np.asarray(grad, dtype=np.float64)
        if not self.started:
            for name, shape, off in self.layout:
                if len(shape) < 2:
                    continue
                g = grad[off:off + int(np.prod(shape))].reshape(shape)
                for d in range(len(shape)):
                    if shape[d] <= MAX_PRECOND_DIM:
                        self.p[name][d] = (1.0 - PRECOND_BETA) * unfold_outer(g, d)
                        self.q[name][d] = eig_desc(self.p[name][d])
            self.started = True
            return theta
        self.s += 1
        scale = lr * np.sqrt(1.0 - BETA2 ** self.s) / (1.0 - BETA1 ** self.s)
        for name, shape, off in self.layout:
            n = int(np.prod(shape))
            g = grad[off:off + n].reshape(shape)
            self.m[name] = BETA1 * self.m[name] + (1.0 - BETA1) * g
            if self.preconditioned(name):
                qs = self.q[name]
                gr, mr = rotate(g, qs), rotate(self.m[name], qs)
            else:
                gr, mr = g, self.m[name]
            self.v[name] = BETA2 * self.v[name] + (1.0 - BETA2) * gr * gr
            upd = mr / (np.sqrt(self.v[name]) + EPS)
            if self.preconditioned(name):
                upd = rotate_back(upd, self.q[name])
            theta[off:off + n] -= scale * upd.reshape(-1)
            if self.preconditioned(name):
                for d in range(len(shape)):
                    if self.p[name][d] is not None:
                        self.p[name][d] = PRECOND_BETA * self.p[name][d] + \
                            (1.0 - PRECOND_BETA) * unfold_outer(g, d)
                if self.s % REFRESH == 0:
                    for d in range(len(shape)):
                        if self.p[name][d] is not None:
                            self.q[name][d], self.v[name] = refresh(self.p[name][d], self.q[name][d],
                                                                    self.v[name], d)
        return theta

    # flat export / import, in the layout order, for comparisons with the GPU
    def export(self) -> Dict[str, np.ndarray]:
        m = np.concatenate([self.m[n].reshape(-1) for n, _, _ in self.layout])
        v = np.concatenate([self.v[n].reshape(-1) for n, _, _ in self.layout])
        p = [self.p[n][d].reshape(-1) for n, s, _ in self.layout if len(s) >= 2
             for d in range(len(s)) if self.p[n][d] is not None]
        q = [self.q[n][d].reshape(-1) for n, s, _ in self.layout if len(s) >= 2
             for d in range(len(s)) if self.q[n][d] is not None]
        return dict(m=m, v=v, p=np.concatenate(p) if p else np.zeros(0),
                    q=np.concatenate(q) if q else np.zeros(0), s=self.s, started=self.started)

    def load(self, st: Dict[str, np.ndarray]):
        pm = pp = 0
        for name, shape, _ in self.layout:
            n = int(np.prod(shape))
            self.m[name] = np.asarray(st["m"][pm:pm + n], np.float64).reshape(shape)
            self.v[name] = np.asarray(st["v"][pm:pm + n], np.float64).reshape(shape)
            pm += n
            if len(shape) >= 2:
                for d, k in enumerate(shape):
                    if k > MAX_PRECOND_DIM:
                        continue
                    self.p[name][d] = np.asarray(st["p"][pp:pp + k * k], np.float64).reshape(k, k)
                    self.q[name][d] = np.asarray(st["q"][pp:pp + k * k], np.float64).reshape(k, k)
                    pp += k * k
        self.s = int(st["s"])
        self.started = bool(st["started"])
