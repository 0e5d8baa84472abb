"""Seeded synthetic inputs for the L0-regularised compressed-sensing (L0RBCS) solver.

This module only draws problem data.  It holds none of the solver's arithmetic
(no couplings, fields, dynamics or R-updates), so that both the FP64 oracle and
the GPU path can take their inputs from it without sharing any solver code.

Observation model (paper, eq. 17 and the paragraph after it):
  * A is M x N with iid N(0, 1/M) entries,
  * the true signal x is iid N(0, 1),
  * the support xi in {0,1}^N marks the non-zero positions (density a),
  * y = A (xi * x) + w with w iid N(0, nu^2).

Every generator takes an integer seed and draws from numpy's PCG64 in a fixed
order (A, then xi, then x, then w) so that an instance is a pure function of
its seed and sizes.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Instance:
    """One L0RBCS problem: y = A (xi * x) + w."""

    A: np.ndarray          # (M, N) float64
    y: np.ndarray          # (M,)   float64
    x: np.ndarray          # (N,)   float64, true amplitudes (also off-support draws)
    xi: np.ndarray         # (N,)   uint8, true support
    seed: int
    meta: dict = field(default_factory=dict)

    @property
    def M(self) -> int:
        return self.A.shape[0]

    @property
    def N(self) -> int:
        return self.A.shape[1]

    def rounded_f32(self) -> "Instance":
        """The same instance with A and y rounded to float32 (kept as float64).

        Parity runs feed the GPU float32 data and the oracle the *same* values,
        so that any difference measures arithmetic, not input rounding."""
        return Instance(self.A.astype(np.float32).astype(np.float64),
                        self.y.astype(np.float32).astype(np.float64),
                        self.x.copy(), self.xi.copy(), self.seed, dict(self.meta))


def gaussian_instance(seed: int, N: int, M: int, a: float, nu: float,
                      support: str = "bernoulli") -> Instance:
    """Random-data instance of eq. 17.

    support="bernoulli": xi_r iid Bernoulli(a) (the benchmark workloads);
    support="exact":     exactly round(a*N) positions set, chosen uniformly
                         (the paper's own recipe for its random data)."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((M, N)) / math.sqrt(M)
    if support == "bernoulli":
        xi = (rng.random(N) < a).astype(np.uint8)
    elif support == "exact":
        k = int(round(a * N))
        xi = np.zeros(N, np.uint8)
        xi[rng.choice(N, size=k, replace=False)] = 1
    else:
        raise ValueError(f"unknown support law {support!r}")
    x = rng.standard_normal(N)
    w = rng.standard_normal(M) * nu
    y = A @ (xi * x) + w
    return Instance(A, y, x, xi, seed, dict(N=N, M=M, a=a, nu=nu, support=support))


def small_gaussian(seed: int) -> Instance:
    """N = 64, M = 32, Bernoulli(0.1) support, noise std 0.01."""
    return gaussian_instance(seed, 64, 32, 0.1, 0.01)


def plain_gaussian(seed: int) -> Instance:
    """N = 2000, M = 1000 (alpha = 0.5), Bernoulli(0.1) support, noise std 0.01."""
    return gaussian_instance(seed, 2000, 1000, 0.1, 0.01)


def well_separated_instance(seed: int, N: int, k: int = 3, nu: float = 0.0,
                            alpha: float = 0.75) -> Instance:
    """Small instance for exhaustive checks: exactly k non-zeros whose
    magnitudes are at least 0.5 (x_r = +-(0.5 + |N(0,1)|)), M = alpha*N."""
    rng = np.random.default_rng(seed)
    M = int(round(alpha * N))
    A = rng.standard_normal((M, N)) / math.sqrt(M)
    xi = np.zeros(N, np.uint8)
    xi[rng.choice(N, size=k, replace=False)] = 1
    sign = np.where(rng.random(N) < 0.5, -1.0, 1.0)
    x = sign * (0.5 + np.abs(rng.standard_normal(N)))
    w = rng.standard_normal(M) * nu
    y = A @ (xi * x) + w
    return Instance(A, y, x, xi, seed, dict(N=N, M=M, k=k, nu=nu))


def initial_amplitudes(seed: int, P: int, N: int, std: float = 1e-2) -> np.ndarray:
    """Explicit initial amplitudes c0 ~ N(0, std^2), shape (P, N), float64.

    Used where a run takes its starting state as an input (the vacuum-noise
    initial condition stated after eq. 16: variance 1e-4, i.e. std 1e-2)."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0xC0]))
    return rng.standard_normal((P, N)) * std


def random_r(seed: int, N: int, scale: float = 1.0) -> np.ndarray:
    """An arbitrary signal estimate R for kernel-level tests."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0x52]))
    return rng.standard_normal(N) * scale


def random_support(seed: int, N: int, density: float) -> np.ndarray:
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0x5A]))
    return (rng.random(N) < density).astype(np.uint8)


# ----------------------------------------------------------------------------
# Batched and serving workloads: many instances of uneven size.
# ----------------------------------------------------------------------------

@dataclass
class InstanceSpec:
    N: int
    M: int
    a: float
    nu: float
    seed: int

    def build(self) -> Instance:
        return gaussian_instance(self.seed, self.N, self.M, self.a, self.nu)


def batch_specs(seed: int, count: int = 256, n_lo: int = 256, n_hi: int = 4096,
                alpha=(0.3, 0.7), a=(0.05, 0.2), nu: float = 0.01) -> list[InstanceSpec]:
    """Sizes for a batch of uneven instances: N log-uniform in [n_lo, n_hi],
    alpha ~ U(alpha), M = round(alpha N), sparsity ~ U(a)."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0xBA7C]))
    out = []
    for k in range(count):
        N = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        al = rng.uniform(*alpha)
        M = max(1, int(round(al * N)))
        ak = rng.uniform(*a)
        out.append(InstanceSpec(N, M, ak, nu, seed * 100003 + k))
    return out


def serving_specs(seed: int, count: int = 2000, n_lo: int = 512, n_hi: int = 8192,
                  alpha=(0.2, 0.6), a=(0.05, 0.2), nu: float = 0.01) -> list[InstanceSpec]:
    """Request sizes for the serving stream (same laws, wider N range)."""
    return batch_specs(seed, count, n_lo, n_hi, alpha, a, nu)


def poisson_arrivals(seed: int, count: int, rate: float) -> np.ndarray:
    """Arrival times (seconds) of a Poisson process with the given rate."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0xA771]))
    return np.cumsum(rng.exponential(1.0 / rate, size=count))


def gaussian_instance_device(seed: int, N: int, M: int, a: float, nu: float, device):
    """The same law as gaussian_instance (A iid N(0, 1/M), Bernoulli(a)
    support, N(0, 1) values, noise std nu), drawn with torch's counter-based
    generator on `device` so that thousands of requests can be made quickly.
    Returns FP32 tensors (A, y, x, xi); the draws differ from the NumPy ones."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    A = torch.randn(M, N, generator=g, device=device, dtype=torch.float32) / math.sqrt(M)
    xi = (torch.rand(N, generator=g, device=device) < a).to(torch.uint8)
    x = torch.randn(N, generator=g, device=device, dtype=torch.float32)
    w = torch.randn(M, generator=g, device=device, dtype=torch.float32) * nu
    y = torch.mv(A, x * xi) + w
    return A, y, x, xi
