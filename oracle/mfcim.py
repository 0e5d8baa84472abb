"""Plain FP64 oracle of the mean-field CIM with chaotic amplitude control and
classical digital processing (CAC-MFZ-CDP) for L0RBCS.

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the CPU-baseline
leg of the benchmark may import this module; the GPU product path never does.

Everything here is written from the paper's equations, in its notation, with
no blocking, fusion or reordering beyond what the equations state.  Library
primitives (a matrix product, a Cholesky factorisation) serve as single steps.

Sections of the paper followed:
  * eq. 3 / eq. 4   : L0RBCS objective and its Ising form; the couplings
                      J~ = -A^T A and the Zeeman term h^z = sqrt(tau) A^T y
                      (stated after eq. 11 and again after eq. 15);
  * eq. 12 - 14     : MFZ amplitude equation, injection field, CAC feedback;
  * eq. 15 / eq. 16 : continuous (CN) and binarised (BN) local fields;
  * eq. 21 / eq. 22 : pump and threshold schedules;
  * Algorithm 1     : alternating minimisation (CIM for sigma, CDP for R);
  * Numerical experiments, parameter paragraph: Delta t = 0.02, 20 photon
    lifetimes, Jacobi CDP with Delta t_c = 0.1 and 100 iterations.

Readings where the paper is silent (each also listed in the design notes):
  * j and beta have no printed value: parameters, defaults j = 0.2, beta = 0.3;
  * forward Euler, c and e updated together from the step-k values, p
    evaluated at t_k = k dt, t restarting at 0 every alternation;
  * sigma = H(c) with H(0) = 0 (strict c > 0);
  * the returned configuration is the one at the last Euler step;
  * R_init = b / diag(G) when none is given;
  * the Jacobi CDP updates every r synchronously (damped Jacobi with step
    dt_c); its fixed point is the least-squares R on the support and the
    residual correlation off it;
  * the couplings have a zero diagonal exactly as eq. 4 writes them;
  * with P > 1 independent replicas the one with the lowest Ising energy
    (eq. 4) is kept, lowest index on ties.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, replace

import numpy as np

from . import rng as _rng

# status bits (same meaning as the GPU library reports them)
ST_NONFINITE = 1 << 0     # non-finite amplitude or error variable
ST_BLOWUP = 1 << 1        # |c| > 1e3
ST_CHOL_RIDGE = 1 << 2    # Cholesky pivot too small, ridge added
ST_TINY_DIAG = 1 << 3     # G_rr < 1e-12, R_r held at 0

CN = "CN"
BN = "BN"


@dataclass(frozen=True)
class CimParams:
    """Constants of the MFZ-CIM dynamics (eq. 12-16, 21)."""

    dt: float = 0.02          # Euler increment
    n_steps: int = 1000       # 20 photon lifetimes at dt = 0.02
    field: str = CN           # CN (eq. 15) or BN (eq. 16)
    p_thr: float = 1.0        # pump threshold (eq. 21)
    d: float = 0.4            # pump swing: 0.4 random data, 0.6 MRI
    t_c: float = 4.0          # sigmoid centre
    t_w: float = 2.0          # sigmoid width
    K: float = 1.0            # feedback strength: 1 random data, 0.1 MRI
    j: float = 0.2            # out-coupling rate (no printed value)
    beta: float = 0.3         # CAC rate (no printed value)
    tau: float = 1.0          # target amplitude
    c0_std: float = 1e-2      # vacuum-noise std of the initial amplitudes
    linear_j: bool = False    # SI variant: linear term (-1 + p - j - c^2)


@dataclass(frozen=True)
class OuterParams:
    """Alternating-minimisation schedule (Algorithm 1, eq. 22) and CDP."""

    eta_init: float = 0.8
    eta_end: float = 0.18
    velo: int = 51
    n_outer: int = 51
    dtc: float = 0.1          # Jacobi time increment
    cdp_iters: int = 100      # Jacobi iterations per alternation
    replicas: int = 1
    seed: int = 0
    refit: bool = False       # final FP64 least-squares refit on the support


# ----------------------------------------------------------------------------
# Schedules
# ----------------------------------------------------------------------------

def pump(t, prm: CimParams):
    """Pump rate, eq. 21: (p_thr - d) + 2d / (1 + exp(-(t - t_c)/t_w))."""
    return (prm.p_thr - prm.d) + 2.0 * prm.d / (1.0 + np.exp(-(np.asarray(t, float) - prm.t_c) / prm.t_w))


def eta_schedule(i: int, outer: OuterParams) -> float:
    """Threshold at alternation i, eq. 22: max(eta_init (1 - i/velo), eta_end)."""
    return max(outer.eta_init * (1.0 - i / outer.velo), outer.eta_end)


def lam_from_eta(eta: float) -> float:
    """eta = sqrt(2 lambda)  (stated with eq. 11 and again after eq. 15)."""
    return 0.5 * eta * eta


# ----------------------------------------------------------------------------
# Problem data in Ising form
# ----------------------------------------------------------------------------

def gram(A: np.ndarray, y: np.ndarray):
    """G = A^T A and b = A^T y: minus the coupling J~ and the Zeeman term
    divided by sqrt(tau)."""
    A = np.asarray(A, float)
    return A.T @ A, A.T @ np.asarray(y, float)


def couplings(G: np.ndarray, b: np.ndarray, R: np.ndarray):
    """R-scaled couplings and Zeeman term.

    J_rr' = -G_rr' R_r R_r' for r != r', J_rr = 0;  z_r = R_r b_r.
    With these, R_r h_r of eq. 15 is  (J (c + sqrt(tau)) / 4)_r + (sqrt(tau)/2) z_r
    and R_r h^BN_r of eq. 16 is  (sqrt(tau)/2) ((J sigma)_r + z_r)."""
    R = np.asarray(R, float)
    J = -G * np.outer(R, R)
    np.fill_diagonal(J, 0.0)
    return J, R * b


def scaled_field(J: np.ndarray, z: np.ndarray, c: np.ndarray, prm: CimParams):
    """R_r h_r for every replica (rows of c), eq. 15 (CN) or eq. 16 (BN)."""
    st = math.sqrt(prm.tau)
    c = np.atleast_2d(c)
    if prm.field == CN:
        X = (c + st) / 4.0
        return X @ J.T + (st / 2.0) * z
    if prm.field == BN:
        X = (c > 0).astype(float)
        return (st / 2.0) * (X @ J.T + z)
    raise ValueError(prm.field)


# ----------------------------------------------------------------------------
# The MFZ-CIM run (sigma minimisation)
# ----------------------------------------------------------------------------

def euler_step(c, e, phi, p, eta, prm: CimParams):
    """One forward-Euler step of eq. 12-14 from the step-k values.

    inj = j e (R h - eta^2 sqrt(tau) / 4)                       (eq. 13)
    dc  = (-1 + p - c^2) c + K inj                              (eq. 12)
    de  = -beta (c^2 - tau) e                                   (eq. 14)"""
    inj = prm.j * e * (phi - eta * eta * math.sqrt(prm.tau) / 4.0)
    lin = -1.0 + p - (prm.j if prm.linear_j else 0.0)
    dc = (lin - c * c) * c + prm.K * inj
    de = -prm.beta * (c * c - prm.tau) * e
    return c + prm.dt * dc, e + prm.dt * de


def mfcim_run(J, z, eta, c0, e0, prm: CimParams, trace_steps: int = 0):
    """Integrate the MFZ-CIM for prm.n_steps steps from (c0, e0).

    c0, e0: (P, N).  Returns (c, e, trace) where trace[k] = (c, e) after
    k + 1 steps for k < trace_steps (shape (trace_steps, 2, P, N))."""
    c = np.array(np.atleast_2d(c0), float)
    e = np.array(np.atleast_2d(e0), float)
    trace = np.empty((trace_steps, 2) + c.shape) if trace_steps else None
    for k in range(prm.n_steps):
        p = pump(k * prm.dt, prm)
        phi = scaled_field(J, z, c, prm)
        c, e = euler_step(c, e, phi, p, eta, prm)
        if k < trace_steps:
            trace[k, 0] = c
            trace[k, 1] = e
    return c, e, trace


def threshold(c) -> np.ndarray:
    """sigma = H(c) with H(0) = 0."""
    return (np.asarray(c) > 0).astype(np.uint8)


def run_status(c, e) -> int:
    st = 0
    if not (np.all(np.isfinite(c)) and np.all(np.isfinite(e))):
        st |= ST_NONFINITE
    elif np.any(np.abs(c) > 1e3):
        st |= ST_BLOWUP
    return st


# ----------------------------------------------------------------------------
# Energies (eq. 3, eq. 4)
# ----------------------------------------------------------------------------

def ising_energy(J, z, sigma, lam) -> np.ndarray:
    """eq. 4 in coupling form: -1/2 s^T J s - z^T s + lam 1^T s, per replica."""
    s = np.atleast_2d(sigma).astype(float)
    return -0.5 * np.einsum("qi,ij,qj->q", s, J, s) - s @ z + lam * s.sum(axis=1)


def l0_objective(A, y, sigma, R, lam) -> float:
    """eq. 3: 1/2 ||y - A (sigma * R)||^2 + lam ||sigma||_0."""
    res = np.asarray(y, float) - np.asarray(A, float) @ (np.asarray(sigma, float) * R)
    return 0.5 * float(res @ res) + lam * float(np.count_nonzero(sigma))


def select_replica(J, z, sigmas, lam):
    """Index of the replica with the lowest eq. 4 energy (first on ties)."""
    H = ising_energy(J, z, sigmas, lam)
    return int(np.argmin(H)), H


# ----------------------------------------------------------------------------
# CDP: R minimisation
# ----------------------------------------------------------------------------

def cdp_jacobi(G, b, sigma, R, dtc: float, iters: int):
    """Jacobi relaxation with time increment dt_c, all r updated together:

    R_r <- R_r + dt_c [ (b_r - sum_{r' != r} G_rr' sigma_r' R_r') / G_rr - R_r ].

    Spins with G_rr < 1e-12 are held at R_r = 0.  Returns (R, status)."""
    G = np.asarray(G, float)
    D = np.diag(G).copy()
    tiny = D < 1e-12
    Dsafe = np.where(tiny, 1.0, D)
    s_mask = np.asarray(sigma, float)
    R = np.array(R, float)
    R[tiny] = 0.0
    for _ in range(iters):
        s = s_mask * R
        off = G @ s - D * s
        R = R + dtc * ((b - off) / Dsafe - R)
        R[tiny] = 0.0
    return R, (ST_TINY_DIAG if tiny.any() else 0)


def support_lstsq(G_SS, b_S):
    """R_S = G_SS^{-1} b_S in FP64 through a Cholesky factor, forward then back
    substitution.  If a pivot is <= 1e-12 * max diag(G_SS) (or the matrix is
    not positive definite) a ridge of 1e-10 * tr(G_SS) / |S| is added and the
    status bit ST_CHOL_RIDGE is returned.  Returns (R_S, status)."""
    G_SS = np.asarray(G_SS, float)
    k = G_SS.shape[0]
    if k == 0:
        return np.zeros(0), 0
    st = 0
    dmax = float(np.max(np.diag(G_SS)))
    try:
        L = np.linalg.cholesky(G_SS)
        ok = float(np.min(np.diag(L))) ** 2 > 1e-12 * dmax
    except np.linalg.LinAlgError:
        ok = False
    if not ok:
        st |= ST_CHOL_RIDGE
        L = np.linalg.cholesky(G_SS + (1e-10 * float(np.trace(G_SS)) / k) * np.eye(k))
    w = np.linalg.solve(L, np.asarray(b_S, float))   # forward substitution
    return np.linalg.solve(L.T, w), st                 # back substitution


def chol_refit(G, b, sigma):
    """Least squares on the support, in FP64 through a Cholesky factor:
    R_S = G_SS^{-1} b_S (support_lstsq, with its ridge rule); off the support
    R_r = (b_r - G_rS R_S) / G_rr.  Returns (R, status)."""
    G = np.asarray(G, float)
    S = np.flatnonzero(np.asarray(sigma))
    D = np.diag(G)
    R = np.zeros(G.shape[0])
    R[S], st = support_lstsq(G[np.ix_(S, S)], b[S])
    tiny = D < 1e-12
    if tiny.any():
        st |= ST_TINY_DIAG
    off = np.setdiff1d(np.arange(G.shape[0]), S)
    R[off] = np.where(tiny[off], 0.0, (b[off] - G[np.ix_(off, S)] @ R[S]) / np.where(tiny[off], 1.0, D[off]))
    return R, st


# ----------------------------------------------------------------------------
# Algorithm 1
# ----------------------------------------------------------------------------

@dataclass
class SolveResult:
    sigma: np.ndarray
    R: np.ndarray
    status: int
    history: list            # per alternation: dict(eta, support, H, replica)
    H: float                 # eq. 4 energy of the returned sigma at the last R used by the CIM
    E: float                 # eq. 3 objective of (sigma, R)


def solve(A, y, cim: CimParams, outer: OuterParams, R_init=None, c0_list=None,
          keep_history: bool = True, j_format: str | None = None) -> SolveResult:
    """Alternating minimisation, Algorithm 1.

    For i = 0 .. n_outer-1:
      eta_i from eq. 22, lambda_i = eta_i^2 / 2;
      J, z from the current R;
      every replica runs the MFZ-CIM from c0 ~ N(0, c0_std^2), e = 1;
      sigma = H(c) at the last step (lowest-energy replica when P > 1);
      R <- Jacobi CDP on that sigma (warm start).
    c0_list, if given, supplies the (P, N) initial amplitudes of every
    alternation; otherwise they come from the counter-based generator.
    j_format ('bf16' or 'fp8'), if given, runs the CIM on the couplings as the
    narrow storage represents them (per-row scale times the rounded value,
    the rounding decided in FP32 as the device decides it)."""
    A = np.asarray(A, float)
    y = np.asarray(y, float)
    G, b = gram(A, y)
    D = np.diag(G)
    status = 0
    if R_init is None:
        R = np.where(D < 1e-12, 0.0, b / np.where(D < 1e-12, 1.0, D))
    else:
        R = np.array(R_init, float)
    P = outer.replicas
    N = A.shape[1]
    hist = []
    sigma = np.zeros(N, np.uint8)
    H_sel = 0.0
    lam = lam_from_eta(eta_schedule(0, outer))
    for i in range(outer.n_outer):
        eta = eta_schedule(i, outer)
        lam = lam_from_eta(eta)
        J, z = couplings(G, b, R)
        if j_format is not None:
            from . import quant as _quant
            f = lambda v: np.asarray(v, float).astype(np.float32)
            J32, _ = _quant.couplings_f32(f(G), f(b), f(R))
            J = _quant.dequantized(*_quant.quantize_rows(J32, j_format))
        if c0_list is not None:
            c0 = np.atleast_2d(np.asarray(c0_list[i], float))
            e0 = np.ones_like(c0)
        else:
            c0, e0 = _rng.initial_state(outer.seed, i, P, N, cim.c0_std)
        c, e, _ = mfcim_run(J, z, eta, c0, e0, cim)
        status |= run_status(c, e)
        sig = threshold(c)
        q, H = select_replica(J, z, sig, lam)
        sigma = sig[q]
        H_sel = float(H[q])
        R_in = R
        R, st = cdp_jacobi(G, b, sigma, R, outer.dtc, outer.cdp_iters)
        status |= st
        if keep_history:
            hist.append(dict(eta=eta, support=int(sigma.sum()), H=H_sel, replica=q,
                             R_in=R_in, sigma=sigma.copy()))
    if outer.refit:
        R, st = chol_refit(G, b, sigma)
        status |= st
    E = l0_objective(A, y, sigma, R, lam)
    return SolveResult(sigma, R, status, hist, H_sel, E)


# ----------------------------------------------------------------------------
# Reporting metrics
# ----------------------------------------------------------------------------

def rmse(sigma, R, x, xi) -> float:
    """sqrt(1/N sum_r (R_r sigma_r - x_r xi_r)^2)  (Results, random data)."""
    d = np.asarray(R, float) * np.asarray(sigma, float) - np.asarray(x, float) * np.asarray(xi, float)
    return float(np.sqrt(np.mean(d * d)))


def hamming_loss(sigma, xi) -> float:
    """1/N sum_r |sigma_r - xi_r|  (Discussion, r = 1..N)."""
    return float(np.mean(np.abs(np.asarray(sigma, int) - np.asarray(xi, int))))


def with_params(prm, **kw):
    return replace(prm, **kw)
