"""Exhaustive references for tiny problems (N <= 16).

TEST INFRASTRUCTURE ONLY.

* ``best_support``: the global L0RBCS optimum of eq. 3 over all 2^N supports,
  with R the least-squares fit on each support (the inner argmin of eq. 3 is
  an ordinary least-squares problem once sigma is fixed).
* ``qubo_ground_state``: the minimum of the Ising energy eq. 4 over all 2^N
  configurations at a fixed R, written as the literal double sum of eq. 4.
"""
from __future__ import annotations

import itertools

import numpy as np


def best_support(A, y, lam):
    """argmin over sigma of min_R 1/2||y - A(sigma*R)||^2 + lam ||sigma||_0."""
    A = np.asarray(A, float)
    y = np.asarray(y, float)
    M, N = A.shape
    best = (0.5 * float(y @ y), np.zeros(N, np.uint8), np.zeros(N))
    for k in range(1, N + 1):
        for S in itertools.combinations(range(N), k):
            AS = A[:, S]
            RS, *_ = np.linalg.lstsq(AS, y, rcond=None)
            res = y - AS @ RS
            val = 0.5 * float(res @ res) + lam * k
            if val < best[0] - 1e-15:
                sig = np.zeros(N, np.uint8)
                sig[list(S)] = 1
                R = np.zeros(N)
                R[list(S)] = RS
                best = (val, sig, R)
    return best


def ising_energy_literal(A, y, R, sigma, lam) -> float:
    """eq. 4 as printed: sum_{r<r'} sum_k A_r^k A_r'^k R_r R_r' s_r s_r'
    - sum_r sum_k y^k A_r^k R_r s_r + lam sum_r s_r."""
    A = np.asarray(A, float)
    M, N = A.shape
    h = 0.0
    for r in range(N):
        for rp in range(r + 1, N):
            for k in range(M):
                h += A[k, r] * A[k, rp] * R[r] * R[rp] * sigma[r] * sigma[rp]
    for r in range(N):
        for k in range(M):
            h -= y[k] * A[k, r] * R[r] * sigma[r]
    return h + lam * float(np.sum(sigma))


def qubo_ground_state(J, z, lam):
    """Brute-force minimum of -1/2 s^T J s - z^T s + lam 1^T s over {0,1}^N."""
    N = J.shape[0]
    best = (np.inf, None)
    for bits in itertools.product((0, 1), repeat=N):
        s = np.array(bits, float)
        v = -0.5 * s @ J @ s - z @ s + lam * s.sum()
        if v < best[0] - 1e-15:
            best = (v, np.array(bits, np.uint8))
    return best
