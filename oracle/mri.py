"""Oracle of Algorithm 1 on the MRI-shaped operator A = S C Psi^T.

TEST INFRASTRUCTURE ONLY.

A dense N x N coupling matrix in FP64 (N = 16384: 2 GB, 0.5 GFLOP per
replica-step) is out of reach for a host oracle, so this module applies the
same couplings in factored form.  With G = A^T A and J = -G o R R^T with a
zero diagonal,

    (J x)_r = -R_r (A^T A (R o x))_r + R_r^2 G_rr x_r,

which is the definition of J x with the diagonal term removed exactly.  A
and A^T are applied with the orthonormal 2-D DCT-II (scipy) and an
independently written orthonormal Haar transform.  The rest of Algorithm 1
(fields, Euler step, pump and threshold schedules, Jacobi CDP, FP64 refit) is
the dense oracle's, step for step.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import fft as sfft

from . import mfcim as O
from . import rng as _rng


def _haar(img, levels):
    out = np.array(img, dtype=float, copy=True)
    s = out.shape[-1]
    c = 1.0 / math.sqrt(2.0)
    for _ in range(levels):
        blk = out[..., :s, :s]
        even, odd = blk[..., :, 0::2], blk[..., :, 1::2]
        blk = np.concatenate([(even + odd) * c, (even - odd) * c], axis=-1)
        even, odd = blk[..., 0::2, :], blk[..., 1::2, :]
        out[..., :s, :s] = np.concatenate([(even + odd) * c, (even - odd) * c], axis=-2)
        s //= 2
    return out


def _ihaar(coef, levels):
    out = np.array(coef, dtype=float, copy=True)
    n = out.shape[-1]
    c = 1.0 / math.sqrt(2.0)
    for lev in reversed(range(levels)):
        s = n >> lev
        h = s // 2
        blk = out[..., :s, :s].copy()
        tmp = np.empty_like(blk)
        tmp[..., 0::2, :] = (blk[..., :h, :] + blk[..., h:, :]) * c
        tmp[..., 1::2, :] = (blk[..., :h, :] - blk[..., h:, :]) * c
        blk[..., :, 0::2] = (tmp[..., :, :h] + tmp[..., :, h:]) * c
        blk[..., :, 1::2] = (tmp[..., :, :h] - tmp[..., :, h:]) * c
        out[..., :s, :s] = blk
    return out


class MriOperator:
    """A = S C Psi^T on (size x size) images, sampled flat frequencies `freqs`."""

    def __init__(self, size: int, freqs, levels: int = 3, A=None):
        self.size = size
        self.N = size * size
        self.freqs = np.asarray(freqs, np.int64)
        self.levels = levels
        # G_rr = sum_k A_kr^2: from the dense matrix when given, otherwise one
        # column at a time through the operator
        self.colnorm2 = np.einsum("kr,kr->r", A, A) if A is not None else self._column_norms()

    def A(self, v):
        v = np.atleast_2d(v)
        img = _ihaar(v.reshape(-1, self.size, self.size), self.levels)
        return sfft.dctn(img, axes=(1, 2), norm="ortho").reshape(v.shape[0], self.N)[:, self.freqs]

    def AT(self, u):
        u = np.atleast_2d(u)
        full = np.zeros((u.shape[0], self.N))
        full[:, self.freqs] = u
        img = sfft.idctn(full.reshape(-1, self.size, self.size), axes=(1, 2), norm="ortho")
        return _haar(img, self.levels).reshape(u.shape[0], self.N)

    def gram_apply(self, v):
        return self.AT(self.A(v))

    def _column_norms(self, chunk: int = 1024):
        out = np.empty(self.N)
        for s in range(0, self.N, chunk):
            e = np.zeros((min(chunk, self.N - s), self.N))
            e[np.arange(e.shape[0]), np.arange(s, s + e.shape[0])] = 1.0
            out[s:s + e.shape[0]] = np.sum(self.A(e) ** 2, axis=1)
        return out


def coupling_apply(op: MriOperator, R, X):
    """J X for every row of X (replicas), J = -(A^T A) o R R^T, zero diagonal."""
    X = np.atleast_2d(X)
    return -R * op.gram_apply(R * X) + (R * R * op.colnorm2) * X


def scaled_field(op, R, z, c, prm: O.CimParams):
    st = math.sqrt(prm.tau)
    c = np.atleast_2d(c)
    if prm.field == O.CN:
        return coupling_apply(op, R, (c + st) / 4.0) + (st / 2.0) * z
    return (st / 2.0) * (coupling_apply(op, R, (c > 0).astype(float)) + z)


def mfcim_run(op, R, z, eta, c0, e0, prm: O.CimParams, trace_steps: int = 0):
    """The Euler integration of the dense oracle's mfcim_run with the field
    taken through the factored couplings.  Returns (c, e, trace), trace[k] =
    (c, e) after k + 1 steps for k < trace_steps (None when trace_steps = 0)."""
    c = np.array(np.atleast_2d(c0), float)
    e = np.array(np.atleast_2d(e0), float)
    trace = np.empty((trace_steps, 2) + c.shape) if trace_steps else None
    for k in range(prm.n_steps):
        p = O.pump(k * prm.dt, prm)
        phi = scaled_field(op, R, z, c, prm)
        c, e = O.euler_step(c, e, phi, p, eta, prm)
        if k < trace_steps:
            trace[k, 0] = c
            trace[k, 1] = e
    return c, e, trace


def ising_energy(op, R, z, sigma, lam):
    s = np.atleast_2d(sigma).astype(float)
    Js = coupling_apply(op, R, s)
    return -0.5 * np.sum(s * Js, axis=1) - s @ z + lam * s.sum(axis=1)


def cdp_jacobi(op, b, sigma, R, dtc, iters):
    D = op.colnorm2
    tiny = D < 1e-12
    Dsafe = np.where(tiny, 1.0, D)
    R = np.array(R, float)
    R[tiny] = 0.0
    sm = np.asarray(sigma, float)
    for _ in range(iters):
        s = sm * R
        off = op.gram_apply(s)[0] - D * s
        R = R + dtc * ((b - off) / Dsafe - R)
        R[tiny] = 0.0
    return R, (O.ST_TINY_DIAG if tiny.any() else 0)


def refit(A, y, sigma):
    """FP64 least squares on the support from the columns of the dense A:
    G_SS = A_S^T A_S and b_S = A_S^T y formed in FP64, then the dense
    oracle's Cholesky solve with its ridge rule.  Returns (S, R_S, status)."""
    S = np.flatnonzero(sigma)
    A_S = np.asarray(A, float)[:, S]
    R_S, st = O.support_lstsq(A_S.T @ A_S, A_S.T @ np.asarray(y, float))
    return S, R_S, st


def solve(op: MriOperator, y, cim: O.CimParams, outer: O.OuterParams, progress=None):
    """Algorithm 1 with the factored couplings; returns (sigma, R, history).

    The same steps as the dense oracle's solve: R_init = b / diag(G), then per
    alternation eta_i (eq. 22), z = R o b, the counter-generator start, the
    MFZ-CIM run, the lowest-energy replica (eq. 4) and the Jacobi CDP.
    history[i] holds eta, support size, H, replica, the R the run used
    (R_in) and the selected sigma."""
    b = op.AT(y)[0]
    D = op.colnorm2
    R = np.where(D < 1e-12, 0.0, b / np.where(D < 1e-12, 1.0, D))
    P, N = outer.replicas, op.N
    sigma = np.zeros(N, np.uint8)
    hist = []
    for i in range(outer.n_outer):
        eta = O.eta_schedule(i, outer)
        lam = O.lam_from_eta(eta)
        z = R * b
        c0, e0 = _rng.initial_state(outer.seed, i, P, N, cim.c0_std)
        c, e, _ = mfcim_run(op, R, z, eta, c0, e0, cim)
        sig = O.threshold(c)
        H = ising_energy(op, R, z, sig, lam)
        q = int(np.argmin(H))
        sigma = sig[q]
        R_in = R
        R, _ = cdp_jacobi(op, b, sigma, R, outer.dtc, outer.cdp_iters)
        hist.append(dict(eta=eta, support=int(sigma.sum()), H=float(H[q]), replica=q,
                         R_in=R_in, sigma=sigma.copy()))
        if progress:
            progress(i, {k: v for k, v in hist[-1].items() if k not in ("R_in", "sigma")})
    return sigma, R, hist
