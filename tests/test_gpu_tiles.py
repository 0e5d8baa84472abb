"""Every tile shape of the matrix-core Euler step (rows of J per workgroup,
16 * RB) gives the same bits: each row's sum runs over the same four column
ranges, in the same chunk order, whatever the shape.  One shape is also
checked against the oracle's trace (normwise 1e-5 per step, FP32 state).
Sizes are ragged for every shape: n = 1203 ends inside a 16-row panel and
inside every 32- to 128-row tile."""
import numpy as np
import pytest
import torch

import paper_2405_00366_amd as L
import workloads as W
from oracle import mfcim as O, quant as Q

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    return torch.device("cuda:0")


def f32(x):
    return np.asarray(x, np.float64).astype(np.float32).astype(np.float64)


def normwise(got, ref):
    den = np.max(np.abs(ref))
    return float(np.max(np.abs(got - ref)) / (den if den > 0 else 1.0))


def valid_rows(P):
    qb = 1 if P <= 16 else (2 if P <= 32 else 4)
    return [16 * rb for rb in (1, 2, 4, 8) if rb * qb <= 16]


FORMATS = {L.F32: None, L.BF16: "bf16", L.FP8E4M3: "fp8"}


@pytest.mark.parametrize("P,field,jdt", [(5, "CN", L.F32), (40, "BN", L.F32), (20, "BN", L.BF16),
                                         (64, "BN", L.BF16), (64, "BN", L.FP8E4M3), (64, "CN", L.FP8E4M3),
                                         (30, "CN", L.BF16)])
def test_every_tile_shape_same_bits(dev, P, field, jdt):
    n, steps, eta = 1203, 12, 0.6
    inst = W.gaussian_instance(77, n, 600, 0.1, 0.01).rounded_f32()
    G, b = O.gram(inst.A, inst.y)
    G32, b32 = f32(G), f32(b)
    R = f32(b / np.diag(G))
    fmt = FORMATS[jdt]
    if fmt is None:
        Jo, zo = O.couplings(G32, b32, R)
        Jo, zo = f32(Jo), f32(zo)
        Jdev = torch.tensor(Jo, dtype=torch.float32, device=dev)
        rs = None
    else:
        J32, z32 = Q.couplings_f32(G32, b32, R)
        q, s = Q.quantize_rows(J32, fmt)
        Jo, zo = Q.dequantized(q, s), z32.astype(np.float64)
        Jdev = torch.tensor(q, dtype=torch.float32, device=dev).to(
            torch.float8_e4m3fn if fmt == "fp8" else torch.bfloat16)
        rs = torch.tensor(s, dtype=torch.float32, device=dev)
    zd = torch.tensor(zo, dtype=torch.float32, device=dev)
    c0 = f32(W.initial_amplitudes(5, P, n))
    prm = L.cim_params(n_steps=steps, field=field, launch=L.LAUNCH_MATRIX)
    traces, sigs = [], []
    try:
        for rows in valid_rows(P):
            L.l0cim_matrix_tile_set(n, P, jdt, field, rows)
            c = torch.tensor(c0, dtype=torch.float32, device=dev)
            e = torch.ones_like(c)
            tr = torch.empty((steps, 2, P, n), dtype=torch.float32, device=dev)
            sig = L.l0cim_mfcim_run(Jdev, zd, eta, prm, c, e, trace=tr, trace_steps=steps, row_scale=rs)
            torch.cuda.synchronize()
            assert L.l0cim_matrix_tile_get(n, P, jdt, field) == rows
            traces.append(tr.cpu().numpy())
            sigs.append(sig.cpu().numpy())
    finally:
        L.l0cim_matrix_tile_set(n, P, jdt, field, 0)
    for k in range(1, len(traces)):
        assert np.array_equal(traces[k].view(np.uint32), traces[0].view(np.uint32)), valid_rows(P)[k]
        assert np.array_equal(sigs[k], sigs[0])
    _, _, tro = O.mfcim_run(Jo, zo, eta, c0, np.ones((P, n)), O.CimParams(n_steps=steps, field=field),
                            trace_steps=steps)
    got = traces[0].astype(np.float64)
    for k in range(steps):
        assert normwise(got[k, 0], tro[k, 0]) <= 1e-5, f"c, step {k}"
        assert normwise(got[k, 1], tro[k, 1]) <= 1e-5, f"e, step {k}"
