"""Support agreement of the precision form, separated from the rounding of
the couplings (GPU, through the C ABI).

Workload: the plain Gaussian shape (N = 2000, M = 1000, Bernoulli(0.1),
noise 0.01, inputs rounded to FP32), 16 replicas, eta 0.8 -> 0.18 over 30
alternations of 1000 steps, final FP64 refit, seeds 0-9.  The FP64 oracle's
results are stored three ways (tests/golden/oracle_supports_prec_*.txt):
with the exact couplings, and with the couplings as BF16 and as FP8 e4m3
rows with per-row scales represent them.  Measured with the oracle alone:
BF16 couplings leave its support unchanged on 10/10 seeds, FP8 changes it
on 7/10 (1-2 spins): the FP8 difference is the method's, not the device's.

Measured on MI355X: the device's solve equals the oracle run on the same
couplings on 10/10 (FP32), 9/10 (BF16) and 10/10 (FP8) seeds, and the
exact-couplings oracle on 10/10, 9/10 and 3/10; every |RMSE - RMSE_oracle|
<= 5.9e-4.  So the device follows the method it is given: the FP8 misses
against the exact couplings are the FP8 rounding's, and one BF16 seed parts
after the bifurcation.  Gates: those rates, and the 1e-3 RMSE bound.
"""
import os

import numpy as np
import pytest
import torch

import paper_2405_00366_amd as L
import workloads as W
from oracle import mfcim as O

pytestmark = pytest.mark.gpu
HERE = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    return torch.device("cuda:0")


def _golden(name):
    out = {}
    for line in open(os.path.join(HERE, f"oracle_supports_{name}.txt")):
        if line.strip() and line[0] != "#":
            k, sz, rm, hx = line.split()
            out[int(k)] = (int(hx, 16), int(sz), float(rm))
    return out


def _mask(v, n):
    return np.array([(v >> r) & 1 for r in range(n)], np.uint8)


def test_precision_form_agreement_by_coupling_format(dev):
    gold = {f: _golden(f"prec_{f}") for f in ("f64", "bf16", "fp8")}
    seeds = sorted(gold["f64"])
    assert len(seeds) == 10
    codes = {"f32": L.F32, "bf16": L.BF16, "fp8": L.FP8E4M3}
    same_fmt = {k: 0 for k in codes}
    same_exact = {k: 0 for k in codes}
    worst = 0.0
    cim = L.cim_params(n_steps=1000)
    for s in seeds:
        inst = W.plain_gaussian(s).rounded_f32()
        A = torch.tensor(inst.A, dtype=torch.float32, device=dev)
        y = torch.tensor(inst.y, dtype=torch.float32, device=dev)
        for fmt, code in codes.items():
            sp = L.solve_params(eta_init=0.8, eta_end=0.18, velo=30, n_outer=30, replicas=16, seed=s,
                                j_dtype=code, final_refit_f64=1)
            R, sig, stats = L.l0cim_solve(A, y, cim, sp)
            torch.cuda.synchronize()
            assert L.read_stats(stats).status_bits == 0
            sg = sig.cpu().numpy()
            ref = gold["f64" if fmt == "f32" else fmt][s]
            same_fmt[fmt] += int(np.array_equal(sg, _mask(ref[0], 2000)))
            same_exact[fmt] += int(np.array_equal(sg, _mask(gold["f64"][s][0], 2000)))
            rm = O.rmse(sg, R.double().cpu().numpy(), inst.x, inst.xi)
            worst = max(worst, abs(rm - ref[2]))
    print(f"device support identical to the oracle on the same couplings: {same_fmt}; "
          f"to the exact-couplings oracle: {same_exact}; max |RMSE - RMSE_oracle| {worst:.2e}")
    assert same_fmt["f32"] >= 10 and same_fmt["bf16"] >= 9 and same_fmt["fp8"] >= 10
    assert same_exact["f32"] >= 10 and same_exact["bf16"] >= 9
    assert worst <= 1e-3
