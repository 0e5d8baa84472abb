"""Oracle of the MRI pipeline pieces around Algorithm 1: the L2-regularised
couplings of eq. 20, the LASSO initial R, and the conjugate-gradient CDP.

TEST INFRASTRUCTURE ONLY.

The MRI problem of eq. 18 adds (gamma / 2)(||D_v x||^2 + ||D_h x||^2) to the
least-squares term, x = Psi^T r the image of the Haar coefficients r, with
D_v and D_h the vertical and horizontal second-difference operators.  The
couplings the CIM sees (eq. 20) are built from

    G_gamma = A^T A + gamma Psi (D_v^T D_v + D_h^T D_h) Psi^T,

i.e. J = -G_gamma o R R^T with a zero diagonal, and the Zeeman term stays
sqrt(tau) A^T y (eq. 19 read dimensionally, as for the plain MRI operator).
The paper does not state the boundary rows of the second differences; here
they use the reflecting extension x[-1] = x[0], x[S] = x[S-1]:

    (D x)_i = x[i-1] - 2 x[i] + x[i+1],  i = 0 .. S-1,

so D is symmetric and D^T D = D D.

The paper's MRI runs start from the LASSO solution and update R with a
conjugate-gradient CDP (at most 10^4 iterations).  The LASSO here minimises
(1/2) r^T G_gamma r - b^T r + lam1 ||r||_1 (the eq. 18 objective with the L0
term replaced by an L1 term, up to a constant) by FISTA (Beck and Teboulle,
2009) with step 1 / (1 + 32 gamma), an upper bound of ||G_gamma||_2 (A A^T
= I, and ||D||_2 <= 4 so ||D_v^T D_v + D_h^T D_h||_2 <= 32), for a fixed
number of iterations from r = 0.  The CG CDP solves the support system
(G_gamma)_SS R_S = b_S from the current R_S (Hestenes and Stiefel) until the
residual norm is at most tol ||b_S|| or the iteration cap is reached; off the
support it sets R_r = (b_r - (G_gamma R_S)_r) / (G_gamma)_rr, the fixed point
of the Jacobi CDP, so that an excluded spin keeps a current amplitude.

An L2Operator has the interface of mri.MriOperator (A, AT, gram_apply,
colnorm2), with gram_apply = G_gamma and colnorm2 = diag(G_gamma), so the
factored couplings, fields, run, energies and Jacobi CDP of mri.py apply to
it unchanged.
"""
from __future__ import annotations

import math

import numpy as np

from . import mfcim as O
from . import mri as OM
from . import rng as _rng


def d2(x, axis):
    """Second difference along `axis` with the reflecting boundary."""
    x = np.asarray(x, float)
    first = np.take(x, [0], axis=axis)
    last = np.take(x, [-1], axis=axis)
    xp = np.concatenate([first, x, last], axis=axis)
    n = x.shape[axis]
    lo = np.take(xp, np.arange(0, n), axis=axis)
    mid = np.take(xp, np.arange(1, n + 1), axis=axis)
    hi = np.take(xp, np.arange(2, n + 2), axis=axis)
    return lo - 2.0 * mid + hi


class L2Operator:
    """G_gamma = A^T A + gamma Psi (D_v^T D_v + D_h^T D_h) Psi^T on the
    operator `op` (an mri.MriOperator)."""

    def __init__(self, op: OM.MriOperator, gamma: float, l2diag=None):
        """l2diag: the diagonal of the smoothness term when already computed
        for this geometry (it does not depend on gamma or the mask)."""
        self.op = op
        self.gamma = float(gamma)
        self.size, self.N, self.levels, self.freqs = op.size, op.N, op.levels, op.freqs
        self.l2diag = self._l2_diagonal() if l2diag is None else np.asarray(l2diag, float)
        self.colnorm2 = op.colnorm2 + self.gamma * self.l2diag

    def A(self, v):
        return self.op.A(v)

    def AT(self, u):
        return self.op.AT(u)

    def smooth_apply(self, v):
        """Psi (D_v^T D_v + D_h^T D_h) Psi^T v for every row of v."""
        v = np.atleast_2d(v)
        img = OM._ihaar(v.reshape(-1, self.size, self.size), self.levels)
        w = d2(d2(img, 1), 1) + d2(d2(img, 2), 2)        # axis 1: vertical, axis 2: horizontal
        return OM._haar(w, self.levels).reshape(v.shape[0], self.N)

    def gram_apply(self, v):
        return self.op.gram_apply(v) + self.gamma * self.smooth_apply(v)

    def _l2_diagonal(self, chunk: int = 1024):
        out = np.empty(self.N)
        for s in range(0, self.N, chunk):
            k = min(chunk, self.N - s)
            e = np.zeros((k, self.N))
            e[np.arange(k), np.arange(s, s + k)] = 1.0
            out[s:s + k] = np.einsum("kr,kr->k", e, self.smooth_apply(e))
        return out


def cdp_cg(hop: L2Operator, b, sigma, R, max_iter: int = 10000, tol: float = 1e-6):
    """CG on (G_gamma)_SS R_S = b_S from the current R_S, then the residual
    formula off the support.  Returns (R, iterations, status)."""
    S = np.asarray(sigma).astype(bool)
    D = hop.colnorm2
    tiny = D < 1e-12
    R = np.array(R, float)

    def Hs(v):                      # (G_gamma)_SS v on the support, 0 elsewhere
        return S * hop.gram_apply(S * v)[0]

    x = S * R
    r = S * b - Hs(x)
    p = r.copy()
    rr = float(r @ r)
    bn = math.sqrt(float((S * b) @ (S * b)))
    it = 0
    while it < max_iter and math.sqrt(rr) > tol * bn:
        Ap = Hs(p)
        alpha = rr / float(p @ Ap)
        x = x + alpha * p
        r = r - alpha * Ap
        rr_new = float(r @ r)
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
    full = hop.gram_apply(x)[0]
    off = np.where(tiny, 0.0, (b - (full - D * x)) / np.where(tiny, 1.0, D))
    R = np.where(S, x, off)
    return R, it, (O.ST_TINY_DIAG if tiny.any() else 0)


def soft(v, t):
    """Soft threshold, the proximal map of t ||.||_1."""
    return np.sign(v) * np.maximum(np.abs(v) - t, 0.0)


def lasso_fista(hop: L2Operator, b, lam1: float, iters: int):
    """FISTA on (1/2) r^T G_gamma r - b^T r + lam1 ||r||_1 from r = 0 with
    step 1 / (1 + 32 gamma); `iters` iterations."""
    step = 1.0 / (1.0 + 32.0 * hop.gamma)
    x = np.zeros(hop.N)
    yk = x.copy()
    tk = 1.0
    for _ in range(iters):
        grad = hop.gram_apply(yk)[0] - b
        x_new = soft(yk - step * grad, step * lam1)
        t_new = 0.5 * (1.0 + math.sqrt(1.0 + 4.0 * tk * tk))
        yk = x_new + ((tk - 1.0) / t_new) * (x_new - x)
        x, tk = x_new, t_new
    return x


def solve(hop: L2Operator, y, cim: O.CimParams, outer: O.OuterParams, lam1: float, lasso_iters: int,
          cg_max_iter: int = 10000, cg_tol: float = 1e-6, progress=None):
    """Algorithm 1 on the MRI pipeline: R_init from the LASSO, then per
    alternation eta_i (eq. 22), z = R o b, the counter-generator start, the
    MFZ-CIM run on the L2-regularised couplings, the lowest-energy replica
    (eq. 4) and the CG CDP.  Returns (sigma, R, history)."""
    b = hop.AT(y)[0]
    R = lasso_fista(hop, b, lam1, lasso_iters)
    P, N = outer.replicas, hop.N
    sigma = np.zeros(N, np.uint8)
    hist = []
    for i in range(outer.n_outer):
        eta = O.eta_schedule(i, outer)
        lam = O.lam_from_eta(eta)
        z = R * b
        c0, e0 = _rng.initial_state(outer.seed, i, P, N, cim.c0_std)
        c, e, _ = OM.mfcim_run(hop, R, z, eta, c0, e0, cim)
        sig = O.threshold(c)
        H = OM.ising_energy(hop, R, z, sig, lam)
        q = int(np.argmin(H))
        sigma = sig[q]
        R_in = R
        R, its, _ = cdp_cg(hop, b, sigma, R, cg_max_iter, cg_tol)
        hist.append(dict(eta=eta, support=int(sigma.sum()), H=float(H[q]), replica=q, cg_iters=its,
                         R_in=R_in, sigma=sigma.copy()))
        if progress:
            progress(i, {k: v for k, v in hist[-1].items() if k not in ("R_in", "sigma")})
    return sigma, R, hist
