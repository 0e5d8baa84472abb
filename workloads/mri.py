"""MRI-shaped synthetic L0RBCS instances (stand-in for the paper's brain MRI).

The paper reconstructs Haar-sparse brain images from undersampled Fourier
data (Numerical experiments; eq. 18-20).  Its image comes from a public MRI
dataset that is not available here, so this module draws a synthetic
stand-in with the same structure:

  * image: size x size random-ellipse phantom on [-1, 1]^2 (a background
    ellipse of intensity 1 plus 9 ellipses with centres U[-0.7, 0.7]^2,
    semi-axes U[0.05, 0.5], angles U[0, pi), intensities U[-0.3, 1]) with a
    low-pass noise texture of std 0.03 inside the head, clipped to [0, 1];
  * sparsity: 3-level orthonormal 2-D Haar transform (Mallat layout), keeping
    the round(sparseness * N) largest coefficients (0.178 at 128 x 128, the
    paper's sparseness for that size) that are not exactly zero;
  * measurements: round(alpha * N) rows (0.3 at 128 x 128, the paper's
    count 4915) of the orthonormal 2-D DCT-II, drawn without replacement with
    variable-density weights 1 / (1 + (rho/16)^2), rho = |frequency|, the DC
    term always included; noise std 1e-3.
A = S C Psi^T (rows of the DCT of Haar basis images), so A A^T = I.

Only input data are produced here; none of the solver's arithmetic.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import fft as sfft

from . import Instance


def phantom(seed: int, size: int = 128, n_ellipses: int = 10) -> np.ndarray:
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0xE111]))
    g = (np.arange(size) + 0.5) / size * 2.0 - 1.0
    X, Y = np.meshgrid(g, g, indexing="xy")
    img = np.zeros((size, size))
    for k in range(n_ellipses):
        if k == 0:
            cx, cy, a, b, th, val = 0.0, 0.0, 0.85, 0.95, 0.0, 1.0
        else:
            cx, cy = rng.uniform(-0.7, 0.7, 2)
            a, b = rng.uniform(0.05, 0.5, 2)
            th = rng.uniform(0.0, math.pi)
            val = rng.uniform(-0.3, 1.0)
        ct, s = math.cos(th), math.sin(th)
        u = (X - cx) * ct + (Y - cy) * s
        v = -(X - cx) * s + (Y - cy) * ct
        img[(u / a) ** 2 + (v / b) ** 2 <= 1.0] += val
    # tissue texture: low-pass Gaussian noise (std 0.03) inside the head
    noise = rng.standard_normal((size, size))
    f = np.fft.fftfreq(size)
    lp = (np.abs(f)[:, None] < 0.125) & (np.abs(f)[None, :] < 0.125)
    tex = np.real(np.fft.ifft2(np.fft.fft2(noise) * lp))
    tex *= 0.03 / max(tex.std(), 1e-30)
    head = (X / 0.85) ** 2 + (Y / 0.95) ** 2 <= 1.0
    img[head] += tex[head]
    return np.clip(img, 0.0, 1.0)


def haar2(img: np.ndarray, levels: int = 3) -> np.ndarray:
    """Orthonormal 2-D Haar analysis, Mallat layout (batched over leading axes)."""
    out = np.array(img, dtype=float, copy=True)
    s = out.shape[-1]
    r2 = 1.0 / math.sqrt(2.0)
    for _ in range(levels):
        blk = out[..., :s, :s]
        a, b = blk[..., :, 0::2], blk[..., :, 1::2]
        blk = np.concatenate([(a + b) * r2, (a - b) * r2], axis=-1)
        a, b = blk[..., 0::2, :], blk[..., 1::2, :]
        out[..., :s, :s] = np.concatenate([(a + b) * r2, (a - b) * r2], axis=-2)
        s //= 2
    return out


def ihaar2(coef: np.ndarray, levels: int = 3) -> np.ndarray:
    """Inverse of haar2."""
    out = np.array(coef, dtype=float, copy=True)
    n = out.shape[-1]
    r2 = 1.0 / math.sqrt(2.0)
    sizes = [n >> l for l in range(levels)][::-1]
    for s in sizes:
        blk = out[..., :s, :s].copy()
        h = s // 2
        lo, hi = blk[..., :h, :], blk[..., h:, :]
        tmp = np.empty_like(blk)
        tmp[..., 0::2, :] = (lo + hi) * r2
        tmp[..., 1::2, :] = (lo - hi) * r2
        lo, hi = tmp[..., :, :h], tmp[..., :, h:]
        blk[..., :, 0::2] = (lo + hi) * r2
        blk[..., :, 1::2] = (lo - hi) * r2
        out[..., :s, :s] = blk
    return out


def sample_frequencies(seed: int, size: int, M: int) -> np.ndarray:
    """M distinct flat DCT frequency indices, variable density, DC first."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0x5A3]))
    u, v = np.meshgrid(np.arange(size), np.arange(size), indexing="ij")
    rho = np.sqrt(u ** 2 + v ** 2).ravel()
    w = 1.0 / (1.0 + (rho / 16.0) ** 2)
    w[0] = 0.0
    rest = rng.choice(size * size, size=M - 1, replace=False, p=w / w.sum())
    return np.concatenate([[0], np.sort(rest)]).astype(np.int64)


def measurement_matrix(freqs: np.ndarray, size: int, levels: int = 3, chunk: int = 512) -> np.ndarray:
    """A = S C Psi^T: row i is the Haar analysis of the DCT basis image of freqs[i]."""
    N = size * size
    A = np.empty((len(freqs), N))
    for s in range(0, len(freqs), chunk):
        f = freqs[s:s + chunk]
        unit = np.zeros((len(f), size, size))
        unit.reshape(len(f), N)[np.arange(len(f)), f] = 1.0
        basis = sfft.idctn(unit, axes=(1, 2), norm="ortho")
        A[s:s + chunk] = haar2(basis, levels).reshape(len(f), N)
    return A


def mri_instance(seed: int, size: int = 128, sparseness: float = 0.178, alpha: float = 0.3,
                 nu: float = 1e-3, levels: int = 3) -> Instance:
    N = size * size
    img = phantom(seed, size)
    coef = haar2(img, levels).ravel()
    k = int(round(sparseness * N))
    keep = np.argsort(-np.abs(coef), kind="stable")[:k]
    xi = np.zeros(N, np.uint8)
    xi[keep] = 1
    xi[np.abs(coef) <= 1e-12] = 0   # exactly flat regions have no coefficient to keep
    x = coef * xi
    M = int(round(alpha * N))
    freqs = sample_frequencies(seed, size, M)
    A = measurement_matrix(freqs, size, levels)
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0x401]))
    y = A @ x + rng.standard_normal(M) * nu
    return Instance(A, y, x, xi, seed, dict(N=N, M=M, size=size, sparseness=sparseness, alpha=alpha, nu=nu,
                                            freqs=freqs, image=img))
