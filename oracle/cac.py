"""Oracle of the CAC-CIM (Positive-P) support estimation, eq. 5-11, inside
Algorithm 1 -- the stochastic model the paper compares the mean-field CIM
against.

TEST INFRASTRUCTURE ONLY.

Per spin r and replica: the normalised mean amplitude mu (eq. 5), the
quantum-fluctuation variances n = <da^+ da> (eq. 6) and m = <da^2> (eq. 7),
and the error variable e of the amplitude control (eq. 9).  The measured
amplitude (eq. 10) carries the same real white noise W as eq. 5, and the
local field (eq. 11) is built from the measured amplitudes of the other
spins.  With the couplings in the R-scaled form of the mean-field oracle
(J = -G o R R^T with a zero diagonal, z = R o b), eq. 11 times R_r is

    R_r h_r = 1/2 (J (mu~ + sqrt(tau)))_r + sqrt(tau) z_r.

The paper gives the continuous-time equations only.  Reading (the same as
for the mean-field model plus the noise): forward Euler-Maruyama with the
time increment dt, every right-hand side evaluated at step k, one standard
normal xi per spin, replica and step (rng.step_normals), the white noise of
the step represented by its step average W = xi / sqrt(dt), so that the noise
increment of eq. 5 is sqrt(j g^2)(m + n) xi sqrt(dt):

    mu~ = mu + sqrt(g^2 / (4 j)) xi / sqrt(dt)                              (10)
    inj = j e (R h - sqrt(tau) eta^2 / 4)                                     (8)
    mu' = mu + dt [-(1 - p + j) mu - mu (mu^2 + 2 g^2 n + g^2 m) + K inj]
             + sqrt(j g^2) (m + n) xi sqrt(dt)                                (5)
    n'  = n + dt [-2 (1 + j) n + 2 p m - 2 mu^2 (2 n + m) - j (m + n)^2]      (6)
    m'  = m + dt [-2 (1 + j) m + 2 p n - 2 mu^2 (2 m + n) + p - (mu^2 + g^2 m)
                  - j (m + n)^2]                                              (7)
    e'  = e + dt [-beta (mu~^2 - tau) e]                                      (9)

with the pump p of eq. 21 at t = k dt.  Every run starts from mu = n = m = 0
and e = 1 (Algorithm 1), and the support it returns is sigma = H(mu) of the
mean amplitude at the last step.  Algorithm 1 is otherwise the mean-field
oracle's: eta schedule (eq. 22), replica choice by the eq. 4 energy, Jacobi
CDP with warm start.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import mfcim as O
from . import rng as _rng


@dataclass(frozen=True)
class CacParams:
    """Constants of the CAC-CIM (eq. 5-11, 21)."""

    dt: float = 0.02
    n_steps: int = 1000
    p_thr: float = 1.0
    d: float = 0.4
    t_c: float = 4.0
    t_w: float = 2.0
    K: float = 1.0            # feedback strength, 1 for random data
    j: float = 0.2            # out-coupling rate (no printed value)
    beta: float = 0.3         # CAC rate (no printed value)
    tau: float = 0.21         # target amplitude: 0.21 at noise 0.05, 0.15 at 0.1
    g2: float = 1e-7          # saturation parameter g^2


def pump(t, prm: CacParams):
    """eq. 21."""
    return (prm.p_thr - prm.d) + 2.0 * prm.d / (1.0 + math.exp(-(t - prm.t_c) / prm.t_w))


def measured(mu, xi, prm: CacParams):
    """eq. 10 with the step-averaged white noise xi / sqrt(dt)."""
    return mu + math.sqrt(prm.g2 / (4.0 * prm.j)) * xi / math.sqrt(prm.dt)


def scaled_field(J, z, mu_m, prm: CacParams):
    """R_r h_r of eq. 11 for every replica (rows of mu_m, measured amplitudes)."""
    st = math.sqrt(prm.tau)
    return 0.5 * (np.atleast_2d(mu_m) + st) @ J.T + st * z


def sde_step(mu, n, m, e, mu_m, xi, phi, p, eta, prm: CacParams):
    """One Euler-Maruyama step of eq. 5-9 from the step-k values."""
    j, g2, dt = prm.j, prm.g2, prm.dt
    inj = j * e * (phi - math.sqrt(prm.tau) * eta * eta / 4.0)
    mu2 = mu * mu
    dmu = -(1.0 - p + j) * mu - mu * (mu2 + 2.0 * g2 * n + g2 * m) + prm.K * inj
    dn = -2.0 * (1.0 + j) * n + 2.0 * p * m - 2.0 * mu2 * (2.0 * n + m) - j * (m + n) ** 2
    dm = (-2.0 * (1.0 + j) * m + 2.0 * p * n - 2.0 * mu2 * (2.0 * m + n) + p - (mu2 + g2 * m)
          - j * (m + n) ** 2)
    de = -prm.beta * (mu_m * mu_m - prm.tau) * e
    mu_new = mu + dt * dmu + math.sqrt(j * g2) * (m + n) * xi * math.sqrt(dt)
    return mu_new, n + dt * dn, m + dt * dm, e + dt * de


def cac_run(J, z, eta, seed: int, alt: int, P: int, prm: CacParams, trace_steps: int = 0, xi_fn=None):
    """Integrate eq. 5-11 for prm.n_steps steps from mu = n = m = 0, e = 1.

    xi_fn(k) -> (P, N) normals of step k (default: the counter generator keyed
    by (seed, alt)).  Returns (mu, n, m, e, trace); trace[k] = (mu, n, m, e)
    after k + 1 steps for k < trace_steps."""
    N = len(z)
    mu = np.zeros((P, N))
    n = np.zeros((P, N))
    m = np.zeros((P, N))
    e = np.ones((P, N))
    trace = np.empty((trace_steps, 4, P, N)) if trace_steps else None
    if xi_fn is None:
        xi_fn = lambda k: _rng.step_normals(seed, alt, k, P, N)
    for k in range(prm.n_steps):
        xi = xi_fn(k)
        mu_m = measured(mu, xi, prm)
        phi = scaled_field(J, z, mu_m, prm)
        mu, n, m, e = sde_step(mu, n, m, e, mu_m, xi, phi, pump(k * prm.dt, prm), eta, prm)
        if k < trace_steps:
            trace[k] = (mu, n, m, e)
    return mu, n, m, e, trace


def solve(A, y, prm: CacParams, outer: O.OuterParams, keep_history: bool = True) -> O.SolveResult:
    """Algorithm 1 with the CAC-CIM as the sigma-minimiser: per alternation
    eta_i (eq. 22), J and z from R, P replicas of cac_run, sigma = H(mu), the
    lowest eq. 4 energy, Jacobi CDP (warm start); R_init = b / diag(G)."""
    A = np.asarray(A, float)
    y = np.asarray(y, float)
    G, b = O.gram(A, y)
    D = np.diag(G)
    R = np.where(D < 1e-12, 0.0, b / np.where(D < 1e-12, 1.0, D))
    P, N = outer.replicas, A.shape[1]
    status = 0
    hist = []
    sigma = np.zeros(N, np.uint8)
    H_sel = 0.0
    lam = O.lam_from_eta(O.eta_schedule(0, outer))
    for i in range(outer.n_outer):
        eta = O.eta_schedule(i, outer)
        lam = O.lam_from_eta(eta)
        J, z = O.couplings(G, b, R)
        mu, n, m, e, _ = cac_run(J, z, eta, outer.seed, i, P, prm)
        status |= O.run_status(mu, e)
        sig = O.threshold(mu)
        q, H = O.select_replica(J, z, sig, lam)
        sigma = sig[q]
        H_sel = float(H[q])
        R_in = R
        R, st = O.cdp_jacobi(G, b, sigma, R, outer.dtc, outer.cdp_iters)
        status |= st
        if keep_history:
            hist.append(dict(eta=eta, support=int(sigma.sum()), H=H_sel, replica=q, R_in=R_in, sigma=sigma.copy()))
    if outer.refit:
        R, st = O.chol_refit(G, b, sigma)
        status |= st
    E = O.l0_objective(A, y, sigma, R, lam)
    return O.SolveResult(sigma, R, status, hist, H_sel, E)
