"""Pins of the oracle's narrow-format rounding (precision form of the couplings)."""
import numpy as np
import pytest
import torch

from oracle import quant as Q


def test_e4m3_rounding_matches_torch_conversion():
    """torch.float8_e4m3fn is the OCP e4m3 format with round-to-nearest-even."""
    rng = np.random.default_rng(0)
    v = np.concatenate([rng.uniform(-448, 448, 20000), rng.uniform(-1, 1, 20000) * 2.0 ** -5,
                        rng.uniform(-1, 1, 2000) * 2.0 ** -9]).astype(np.float32)
    ref = torch.from_numpy(v).to(torch.float8_e4m3fn).float().numpy()
    np.testing.assert_array_equal(Q.round_e4m3(v), ref)


def test_e4m3_special_values():
    v = np.array([448.0, 449.0, 1e6, -500.0, 0.0, 2.0 ** -9, 2.0 ** -10, 3 * 2.0 ** -10,
                  1.0625, 1.1875, 240.0, 232.0], np.float32)
    # saturation at 448; half of the smallest subnormal rounds to 0 (even);
    # 1.5 steps rounds to 2 steps; ties 1.0625 -> 1.0 and 1.1875 -> 1.25 (even mantissa);
    # 232 lies between 224 and 240 (step 16): tie -> 224 (mantissa 110 is even? 224=1.75*128 -> 110)
    out = Q.round_e4m3(v)
    assert out.tolist() == [448.0, 448.0, 448.0, -448.0, 0.0, 2.0 ** -9, 0.0, 2.0 ** -8,
                            1.0, 1.25, 240.0, 224.0]


def test_bf16_rounding_matches_torch_conversion():
    rng = np.random.default_rng(1)
    v = (rng.standard_normal(50000) * np.exp(rng.uniform(-20, 20, 50000))).astype(np.float32)
    ref = torch.from_numpy(v).to(torch.bfloat16).float().numpy()
    np.testing.assert_array_equal(Q.round_bf16(v), ref)


@pytest.mark.parametrize("fmt", ["fp8", "bf16"])
def test_row_scales_and_dequantised_error(fmt):
    rng = np.random.default_rng(2)
    J = rng.standard_normal((50, 80)).astype(np.float32)
    J[7] = 0.0
    q, s = Q.quantize_rows(J, fmt)
    assert s[7] == 1.0 and np.all(q[7] == 0)
    qmax = 448.0 if fmt == "fp8" else 1.0
    np.testing.assert_array_equal(s[:7], (np.abs(J[:7]).max(axis=1) / np.float32(qmax)).astype(np.float32))
    assert np.all(np.abs(q) <= qmax)
    rel = 2.0 ** -4 if fmt == "fp8" else 2.0 ** -8     # half an ulp of the narrow mantissa
    err = np.abs(Q.dequantized(q, s) - J)
    assert np.all(err <= rel * np.abs(J).max(axis=1, keepdims=True) + 1e-30)
