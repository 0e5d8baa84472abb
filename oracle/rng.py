"""Counter-based normal draws for the initial amplitudes (oracle side).

TEST INFRASTRUCTURE ONLY: nothing in the product path may import this module.

The paper starts every CIM run from c_r ~ N(0, 1e-4) and e_r = 1 (the
paragraph after eq. 16, and Algorithm 1).  The solver draws these numbers
itself, so the oracle and the GPU path each implement the same published
generator independently:

  * SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
    generators", OOPSLA 2014).  Its n-th output (n = 1, 2, ...) for seed s is
    mix64(s + n * GAMMA mod 2^64), so it is counter-based by construction.
  * Two 53-bit uniforms per draw, turned into one standard normal with the
    Box-Muller transform (Box and Muller, 1958): sqrt(-2 ln(1-u1)) cos(2 pi u2).

Counter of the draw for alternation i, replica q, spin r:
    ctr = (i << 40) | (q << 24) | r      (i < 2^24, q < 2^16, r < 2^24)
the two uniforms use outputs n = 2 ctr + 1 and n = 2 ctr + 2.
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output finaliser (variant 13 of Stafford's mixers)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def splitmix64(seed: int, n: np.ndarray) -> np.ndarray:
    """n-th output (n >= 1) of the SplitMix64 stream started at `seed`."""
    n = np.asarray(n, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return mix64(np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + n * GAMMA)


def uniform53(bits: np.ndarray) -> np.ndarray:
    """Top 53 bits of a 64-bit word as a double in [0, 1)."""
    return (np.asarray(bits, np.uint64) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def counters(i: int, P: int, N: int) -> np.ndarray:
    if not (0 <= i < 1 << 24 and 0 < P <= 1 << 16 and 0 < N <= 1 << 24):
        raise ValueError("counter fields out of range")
    q = np.arange(P, dtype=np.uint64)[:, None]
    r = np.arange(N, dtype=np.uint64)[None, :]
    return (np.uint64(i) << np.uint64(40)) | (q << np.uint64(24)) | r


def standard_normals(seed: int, i: int, P: int, N: int) -> np.ndarray:
    """(P, N) standard normal draws for alternation i."""
    ctr = counters(i, P, N)
    with np.errstate(over="ignore"):
        u1 = uniform53(splitmix64(seed, np.uint64(2) * ctr + np.uint64(1)))
        u2 = uniform53(splitmix64(seed, np.uint64(2) * ctr + np.uint64(2)))
    return np.sqrt(-2.0 * np.log1p(-u1)) * np.cos(2.0 * np.pi * u2)


def initial_state(seed: int, i: int, P: int, N: int, std: float):
    """(c0, e0) for alternation i: c0 = std * normal draws, e0 = 1."""
    c0 = std * standard_normals(seed, i, P, N)
    return c0, np.ones((P, N))


# ----------------------------------------------------------------------------
# Per-step noise of the CAC-CIM stochastic differential equations
# ----------------------------------------------------------------------------
#
# The Positive-P CAC-CIM (eq. 5-11) is driven by a real white noise W_r(t),
# drawn once per Euler step, spin and replica.  Its normals come from a second
# SplitMix64 stream whose seed is the finaliser of the solve seed XOR a fixed
# tag, so that it never overlaps the stream of the initial amplitudes:
#     s_noise = mix64(seed ^ NOISE_TAG)
# and the counter of the draw for alternation i, Euler step k, replica q,
# spin r is
#     ctr = (i << 52) | (k << 32) | (q << 24) | r
#     (i < 2^11, k < 2^20, q < 2^8, r < 2^24),
# with the two uniforms at outputs 2 ctr + 1 and 2 ctr + 2, Box-Muller as above.

NOISE_TAG = 0x6E6F6973655F7764     # "noise_wd" as ASCII bytes


def noise_seed(seed: int) -> int:
    return int(mix64(np.uint64((seed ^ NOISE_TAG) & 0xFFFFFFFFFFFFFFFF)))


def step_normals(seed: int, i: int, k: int, P: int, N: int) -> np.ndarray:
    """(P, N) standard normals of Euler step k of alternation i."""
    if not (0 <= i < 1 << 11 and 0 <= k < 1 << 20 and 0 < P <= 1 << 8 and 0 < N <= 1 << 24):
        raise ValueError("noise counter fields out of range")
    q = np.arange(P, dtype=np.uint64)[:, None]
    r = np.arange(N, dtype=np.uint64)[None, :]
    ctr = (np.uint64(i) << np.uint64(52)) | (np.uint64(k) << np.uint64(32)) | (q << np.uint64(24)) | r
    s = noise_seed(seed)
    with np.errstate(over="ignore"):
        u1 = uniform53(splitmix64(s, np.uint64(2) * ctr + np.uint64(1)))
        u2 = uniform53(splitmix64(s, np.uint64(2) * ctr + np.uint64(2)))
    return np.sqrt(-2.0 * np.log1p(-u1)) * np.cos(2.0 * np.pi * u2)
