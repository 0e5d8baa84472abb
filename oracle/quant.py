"""Reference rounding of the couplings to BF16 and FP8 (e4m3) with per-row scales.

TEST INFRASTRUCTURE ONLY.

The precision form stores J in a narrow format with one FP32 scale per row:
  s_r = max_r' |J_rr'| / Q_max   (Q_max = 448 for e4m3, 1 for bf16; s_r = 1 for
                                  an all-zero row),
  q_rr' = RNE(J_rr' / s_r)       (saturating at +-448 for e4m3),
and the local field uses s_r * sum_r' q_rr' x_r'.  The quantised code is an
integer decision taken from floating point, so this reference takes it in the
same precision as the device: J, the scale and the quotient are FP32.

Formats (OCP 8-bit floating point specification, and bfloat16):
  * e4m3: 1 sign, 4 exponent bits (bias 7), 3 mantissa bits; largest finite
    448 = 1.75 * 2^8; smallest normal 2^-6; subnormal step 2^-9; no infinity.
  * bf16: the upper 16 bits of an FP32 word, rounded to nearest even.
"""
from __future__ import annotations

import numpy as np

E4M3_MAX = 448.0


def couplings_f32(G32, b32, R32):
    """J and z evaluated in FP32 exactly as the definition orders the
    operations: J_rr' = -(G_rr' * (R_r * R_r')), J_rr = 0, z_r = R_r * b_r."""
    G32 = np.asarray(G32, np.float32)
    R32 = np.asarray(R32, np.float32)
    RR = (R32[:, None] * R32[None, :]).astype(np.float32)
    J = (-(G32 * RR)).astype(np.float32)
    np.fill_diagonal(J, np.float32(0))
    z = (R32 * np.asarray(b32, np.float32)).astype(np.float32)
    return J, z


def round_bf16(v32) -> np.ndarray:
    """Nearest-even rounding of FP32 values to bf16, returned as FP32."""
    u = np.asarray(v32, np.float32).view(np.uint32).astype(np.uint64)
    bias = np.uint64(0x7FFF) + ((u >> np.uint64(16)) & np.uint64(1))
    r = ((u + bias) >> np.uint64(16)) << np.uint64(16)
    return r.astype(np.uint32).view(np.float32)


def round_e4m3(v32) -> np.ndarray:
    """Nearest-even rounding of FP32 values to OCP e4m3 (saturating), as FP32."""
    v = np.asarray(v32, np.float32).astype(np.float64)
    a = np.minimum(np.abs(v), E4M3_MAX)
    # exponent of the binade (normals from 2^-6); below that the step is 2^-9
    with np.errstate(divide="ignore"):
        e = np.floor(np.log2(np.where(a > 0, a, 1.0)))
    e = np.maximum(e, -6.0)
    step = np.exp2(e - 3.0)
    q = np.round(a / step) * step          # numpy rounds halves to even
    q = np.minimum(q, E4M3_MAX)
    return (np.sign(v) * q).astype(np.float32)


def quantize_rows(J32, fmt: str):
    """Per-row scales and rounded values: returns (q as FP32 values, s_r FP32)."""
    J32 = np.asarray(J32, np.float32)
    qmax = np.float32(E4M3_MAX if fmt == "fp8" else 1.0)
    amax = np.max(np.abs(J32), axis=1).astype(np.float32)
    scale = np.where(amax > 0, (amax / qmax).astype(np.float32), np.float32(1.0)).astype(np.float32)
    ratio = (J32 / scale[:, None]).astype(np.float32)
    if fmt == "fp8":
        ratio = np.clip(ratio, -qmax, qmax).astype(np.float32)
        q = round_e4m3(ratio)
    elif fmt == "bf16":
        q = round_bf16(ratio)
    else:
        raise ValueError(fmt)
    return q, scale


def dequantized(q, scale) -> np.ndarray:
    """The couplings the narrow format represents: s_r * q_rr' (FP64)."""
    return np.asarray(q, np.float64) * np.asarray(scale, np.float64)[:, None]
