"""GPU parity of the CAC-CIM (Positive-P) form against the oracle
(oracle/cac.py, eq. 5-11), through the C ABI.

Both sides draw the same counter-based normals (each from its own code), start
from mu = n = m = 0, e = 1 and take the same J and z (FP32-rounded where the
device computes in FP32).  Gates:
  * trace: normwise relative error per Euler step over the first 200 steps,
    1e-5 for FP32 and 1e-12 for FP64, for mu, n, m and e;
  * sigma = H(mu) of the device's own final state, and the eq. 4 energy of
    that sigma (1e-5 relative);
  * Algorithm 1 (l0cim_cac_solve) on small FP64 instances: the oracle's
    support in every alternation on every seed.
"""
import numpy as np
import pytest
import torch

import paper_2405_00366_amd as L
import workloads as W
from oracle import cac as C, mfcim as O

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


def _problem(seed, n, dtype):
    inst = W.gaussian_instance(seed, n, n // 2, 0.15, 0.01)
    if dtype == torch.float32:
        inst = inst.rounded_f32()
    G, b = O.gram(inst.A, inst.y)
    R = b / np.diag(G)
    J, z = O.couplings(G, b, R)
    if dtype == torch.float32:
        J, z = f32(J), f32(z)
    return J, z


# n = 2100 in FP64 (8 replicas' amplitudes above 128 KB) takes the form that reads them from memory;
# the others stage them in LDS
@pytest.mark.parametrize("n,P,dtype,steps,tau", [(300, 2, torch.float64, 200, 0.21), (300, 3, torch.float32, 200, 0.21),
                                                  (2000, 1, torch.float32, 200, 0.15), (777, 2, torch.float32, 600, 0.21),
                                                  (2100, 2, torch.float64, 200, 0.21), (500, 11, torch.float32, 200, 0.21)])
def test_cac_run_trace_parity(dev, n, P, dtype, steps, tau):
    seed, alt, eta = 11, 3, 0.4
    J, z = _problem(seed + n, n, dtype)
    prm_o = C.CacParams(n_steps=steps, tau=tau)
    mu_o, n_o, m_o, e_o, tr_o = C.cac_run(J, z, eta, seed, alt, P, prm_o, trace_steps=min(steps, 200))
    Jd = torch.tensor(J, dtype=dtype, device=dev)
    zd = torch.tensor(z, dtype=dtype, device=dev)
    ts = min(steps, 200)
    tr = torch.empty((ts, 4, P, n), dtype=dtype, device=dev)
    H = torch.empty(P, dtype=torch.float64, device=dev)
    st = torch.zeros(1, dtype=torch.int32, device=dev)
    mu, nv, mv, e, sig = L.l0cim_cac_run(Jd, zd, eta, L.cac_params(n_steps=steps, tau=tau), seed, alt, P, H=H,
                                         trace=tr, trace_steps=ts, status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    got = tr.double().cpu().numpy()
    tol = 1e-12 if dtype == torch.float64 else 1e-5
    worst = max(normwise(got[k, v], tr_o[k, v]) for k in range(ts) for v in range(4))
    assert worst <= tol, f"worst normwise error over {ts} steps: {worst:.3g}"
    mu_h = mu.double().cpu().numpy()
    sg = sig.cpu().numpy()
    assert np.array_equal(sg, (mu_h > 0).astype(np.uint8))
    Hs = O.ising_energy(J, z, sg, 0.5 * eta * eta)
    np.testing.assert_allclose(H.cpu().numpy(), Hs, rtol=1e-5, atol=1e-8)
    if dtype == torch.float64 and steps == ts:
        np.testing.assert_array_equal(sg, O.threshold(mu_o))


@pytest.mark.parametrize("seed", range(6))
def test_cac_solve_matches_oracle(dev, seed):
    """N = 64, M = 32, FP64, 4 replicas, 1000 steps x 8 alternations, eta
    0.8 -> 0.2: the oracle's selected support in every alternation (through
    the final one) and its R to 1e-9."""
    inst = W.small_gaussian(seed)
    prm = C.CacParams(n_steps=1000)
    outer = O.OuterParams(eta_init=0.8, eta_end=0.2, velo=8, n_outer=8, replicas=4, seed=seed)
    ref = C.solve(inst.A, inst.y, prm, outer)
    A = torch.tensor(inst.A, dtype=torch.float64, device=dev)
    y = torch.tensor(inst.y, dtype=torch.float64, device=dev)
    sp = L.solve_params(eta_init=0.8, eta_end=0.2, velo=8, n_outer=8, replicas=4, seed=seed)
    R, sig, stats = L.l0cim_cac_solve(A, y, L.cac_params(n_steps=1000), sp)
    torch.cuda.synchronize()
    st = L.read_stats(stats)
    assert st.status_bits == ref.status
    np.testing.assert_array_equal(sig.cpu().numpy(), ref.sigma)
    np.testing.assert_allclose(R.cpu().numpy(), ref.R, rtol=1e-9, atol=1e-11)
    assert st.selected_replica == ref.history[-1]["replica"]


def test_cac_rejects_bad_arguments(dev):
    lib = L.lib()
    J = torch.zeros((8, 8), dtype=torch.float32, device=dev)
    p = L.cac_params(n_steps=1 << 20)
    with pytest.raises(L.L0cimError):
        L.l0cim_cac_run(J, J[0], 0.3, p, 0, 0, 1)
    with pytest.raises(L.L0cimError):
        L.l0cim_cac_run(J, J[0], 0.3, L.cac_params(), 0, 2048, 1)
    with pytest.raises(L.L0cimError):
        L.l0cim_cac_run(J, J[0], 0.3, L.cac_params(), 0, 0, 257)
    assert lib.l0cim_cac_run_workspace_bytes(L.BF16, 8, 1) == 0


def _golden_cac():
    import os
    out = {}
    for line in open(os.path.join(os.path.dirname(__file__), "golden", "oracle_supports_cac.txt")):
        if line.strip() and line[0] != "#":
            k, sz, rm, hx = line.split()
            out[int(k)] = (int(hx, 16), int(sz), float(rm))
    return out


def test_cac_solve_plain_shape_against_stored_oracle(dev):
    """l0cim_cac_solve in FP32 at the plain shape (N = 2000, M = 1000, 8
    replicas, default CAC parameters, 30 alternations of 1000 steps, eta
    0.8 -> 0.18) on the ten seeds whose FP64 oracle results are stored
    (tests/golden/oracle_supports_cac.txt): the final support and RMSE.
    Measured on MI355X: 10/10 identical, max |dRMSE| 1.5e-7.  Gate: all ten,
    and |dRMSE| <= 1e-3."""
    gold = _golden_cac()
    assert len(gold) == 10
    same, worst = 0, 0.0
    for sd in sorted(gold):
        inst = W.plain_gaussian(sd)
        A = torch.tensor(inst.A, dtype=torch.float32, device=dev)
        y = torch.tensor(inst.y, dtype=torch.float32, device=dev)
        sp = L.solve_params(eta_init=0.8, eta_end=0.18, velo=30, n_outer=30, replicas=8, seed=sd)
        R, sig, st = L.l0cim_cac_solve(A, y, L.cac_params(n_steps=1000), sp)
        torch.cuda.synchronize()
        assert L.read_stats(st).status_bits == 0
        sg = sig.cpu().numpy()
        so = np.array([(gold[sd][0] >> r) & 1 for r in range(inst.N)], np.uint8)
        same += int(np.array_equal(sg, so))
        worst = max(worst, abs(O.rmse(sg, R.double().cpu().numpy(), inst.x, inst.xi) - gold[sd][2]))
    print(f"CAC-CIM at N = 2000: {same}/10 supports identical to the FP64 oracle, max |dRMSE| {worst:.2e}")
    assert same == 10
    assert worst <= 1e-3
