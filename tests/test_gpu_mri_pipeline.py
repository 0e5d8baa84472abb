"""GPU parity of the MRI pipeline pieces in factored form against the
oracle's (oracle/mri_l2.py, oracle/mri.py), through the C ABI:

  * the diagonal of the L2-regularised Gram matrix (eq. 20), bit-for-bit up
    to the FP32 rounding of the FP64 value;
  * the CIM run on the L2-regularised couplings: normwise 1e-5 per Euler step
    over 200 steps (continuous field), as for the plain factored couplings;
  * the LASSO start (FISTA): the device's FP32 iterate against the oracle's
    FP64 one after the same number of iterations;
  * the CG CDP: the device's FP32 CG solution of the support system against
    the exact solution, within what its stopping rule allows;
  * the Jacobi CDP in factored form against the oracle's, sweep for sweep.

Inputs are the seed-0 MRI-shaped instance with FP32-rounded D, b and R.
"""
import numpy as np
import pytest
import torch

import paper_2405_00366_amd as L
import workloads as W
from oracle import mfcim as O, mri as MRI, mri_l2 as L2

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


@pytest.fixture(scope="module")
def case():
    from workloads import mri as WM
    inst = WM.mri_instance(0)
    A = f32(inst.A)
    D = f32(np.einsum("kr,kr->r", A, A))
    b = f32(A.T @ f32(inst.y))
    mask = np.zeros(128 * 128, np.uint8)
    mask[inst.meta["freqs"]] = 1
    return dict(inst=inst, freqs=inst.meta["freqs"], D=D, b=b, mask=mask)


_L2DIAG = {}


def _hop(case, gamma, levels=3, D=None):
    op = MRI.MriOperator(128, case["freqs"], levels=levels, A=np.zeros((1, 128 * 128)))
    op.colnorm2 = case["D"]
    hop = L2.L2Operator(op, gamma, _L2DIAG.get(levels))
    _L2DIAG[levels] = hop.l2diag
    if D is not None:
        hop.colnorm2 = D
    return hop


def t(x, dev, dt=torch.float32):
    return torch.tensor(np.asarray(x), dtype=dt, device=dev)


@pytest.mark.parametrize("levels", [0, 1, 2, 3, 4])
def test_l2_diagonal(dev, case, levels):
    hop = _hop(case, 1.0, levels)
    out = torch.empty(128 * 128, dtype=torch.float32, device=dev)
    L.l0cim_mri_l2_diag(128, levels, 1.0, t(np.zeros(128 * 128), dev), out)
    torch.cuda.synchronize()
    np.testing.assert_allclose(out.double().cpu().numpy(), hop.l2diag, rtol=2 ** -23, atol=0)
    # D_in + gamma diag(L), D_in read with a stride
    Dm = torch.zeros((128 * 128, 2), dtype=torch.float32, device=dev)
    Dm[:, 0] = t(case["D"], dev)
    L.l0cim_mri_l2_diag(128, levels, 1e-4, Dm[:, 0], out)
    torch.cuda.synchronize()
    np.testing.assert_allclose(out.double().cpu().numpy(), f32(case["D"] + 1e-4 * hop.l2diag), rtol=2 ** -23)


@pytest.mark.parametrize("field,gamma,P", [("CN", 1e-2, 2), ("CN", 1e-4, 1), ("BN", 1e-2, 2)])
def test_l2_run_trace_parity(dev, case, field, gamma, P):
    steps, eta, seed, n = 200, 0.1, 5, 128 * 128
    hop0 = _hop(case, gamma)
    D = f32(hop0.colnorm2)
    hop = _hop(case, gamma, D=D)
    R = f32(W.random_r(seed, n, 0.3))
    b = case["b"]
    z = f32(R * b)
    c0 = f32(W.initial_amplitudes(seed, P, n))
    prm = O.CimParams(n_steps=steps, field=field, K=1.0, d=0.6)
    c, e = t(c0, dev), torch.ones((P, n), dtype=torch.float32, device=dev)
    tr = torch.empty((steps, 2, P, n), dtype=torch.float32, device=dev)
    H = torch.empty(P, dtype=torch.float64, device=dev)
    st = torch.zeros(1, dtype=torch.int32, device=dev)
    sig = L.l0cim_mri_mfcim_run(128, 3, t(case["mask"], dev, torch.uint8), t(R, dev), t(D, dev), t(b, dev), eta,
                                L.cim_params(n_steps=steps, field=field, K=1.0, d=0.6), c, e, H=H, trace=tr,
                                trace_steps=steps, status=st, gamma=gamma)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    got = tr.double().cpu().numpy()
    worst = 0.0
    cp, ep = c0, np.ones_like(c0)
    for k in range(steps):
        phi = MRI.scaled_field(hop, R, z, cp, prm)
        cn, en = O.euler_step(cp, ep, phi, O.pump(k * prm.dt, prm), eta, prm)
        worst = max(worst, normwise(got[k, 0], cn), normwise(got[k, 1], en))
        # continuous field: the free-running trajectories; binarised: each
        # device step from the device's previous state
        cp, ep = (cn, en) if field == "CN" else (got[k, 0], got[k, 1])
    assert worst <= 1e-5, f"worst normwise error {worst:.3g}"
    sg = sig.cpu().numpy()
    Hs = MRI.ising_energy(hop, R, z, sg, 0.5 * eta * eta)
    np.testing.assert_allclose(H.cpu().numpy(), Hs, rtol=1e-5, atol=1e-6)


@pytest.mark.parametrize("gamma,lam1,iters", [(1e-4, 3e-4, 200), (1e-2, 1e-2, 60), (0.0, 3e-4, 100)])
def test_lasso_parity(dev, case, gamma, lam1, iters):
    hop = _hop(case, gamma)
    b = case["b"]
    ref = L2.lasso_fista(hop, b, lam1, iters)
    R = torch.empty(128 * 128, dtype=torch.float32, device=dev)
    L.l0cim_mri_lasso(128, 3, gamma, t(case["mask"], dev, torch.uint8), t(b, dev), lam1, iters, R)
    torch.cuda.synchronize()
    got = R.double().cpu().numpy()
    err = normwise(got, ref)
    print(f"LASSO gamma={gamma} lam1={lam1} iters={iters}: normwise {err:.3g}, "
          f"non-zeros {int(np.sum(got != 0))} (oracle {int(np.sum(ref != 0))})")
    assert err <= 1e-4


def _support(case, seed=0):
    import os
    here = os.path.join(os.path.dirname(__file__), "golden")
    for line in open(os.path.join(here, "oracle_supports_mri.txt")):
        if line.strip() and line[0] != "#" and int(line.split()[0]) == seed:
            v = int(line.split()[3], 16)
            return np.array([(v >> r) & 1 for r in range(128 * 128)], np.uint8)
    raise AssertionError("no stored support")


@pytest.mark.parametrize("gamma", [1e-4, 0.0])
def test_cg_cdp_parity(dev, case, gamma):
    """The CG CDP on the oracle's seed-0 support (|S| = 1074) from R = b / D:
    R_S within 1e-4 (normwise) of the exact solution (the oracle's CG run to a
    1e-12 residual), the iteration count within the cap.  The off-support rows
    R_r = (b_r - (G R_S)_r) / D_r are a residual, small beside R_S: their
    error is that of G (R_S - R_S*) and is bounded in the units of R_S,
    max |dR_off| <= 1e-4 max |R_S*|."""
    hop0 = _hop(case, gamma)
    D = f32(hop0.colnorm2)
    hop = _hop(case, gamma, D=D)
    b = case["b"]
    sig = _support(case)
    R0 = f32(b / D)
    ref, its_ref, _ = L2.cdp_cg(hop, b, sig, R0, max_iter=10000, tol=1e-12)
    R = t(R0, dev)
    its = torch.zeros(1, dtype=torch.int32, device=dev)
    st = torch.zeros(1, dtype=torch.int32, device=dev)
    L.l0cim_mri_update_r(128, 3, gamma, t(case["mask"], dev, torch.uint8), t(D, dev), t(b, dev),
                         t(sig, dev, torch.uint8), R, cdp=L.CDP_CG, cg_max_iter=10000, cg_tol=1e-6,
                         iters_out=its, status=st)
    torch.cuda.synchronize()
    got = R.double().cpu().numpy()
    S = sig.astype(bool)
    e_on = normwise(got[S], ref[S])
    e_off = float(np.max(np.abs(got[~S] - ref[~S])) / np.max(np.abs(ref[S])))
    print(f"CG gamma={gamma}: {int(its.item())} iterations (oracle to 1e-12: {its_ref}); "
          f"normwise on the support {e_on:.3g}, off it {e_off:.3g}")
    assert int(st.item()) == 0 and 0 < int(its.item()) < 10000
    assert e_on <= 1e-4 and e_off <= 1e-4


def test_factored_jacobi_parity(dev, case):
    hop = _hop(case, 1e-4, D=f32(_hop(case, 1e-4).colnorm2))
    b = case["b"]
    sig = _support(case)
    R0 = f32(b / hop.colnorm2)
    ref, _ = MRI.cdp_jacobi(hop, b, sig, R0, 0.1, 100)
    R = t(R0, dev)
    L.l0cim_mri_update_r(128, 3, 1e-4, t(case["mask"], dev, torch.uint8), t(hop.colnorm2, dev), t(b, dev),
                         t(sig, dev, torch.uint8), R, cdp=L.CDP_JACOBI, dtc=0.1, iters=100)
    torch.cuda.synchronize()
    assert normwise(R.double().cpu().numpy(), ref) <= 1e-5


def _golden(name):
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", f"oracle_supports_{name}.txt")
    out = {}
    if os.path.exists(path):
        for line in open(path):
            if line.strip() and line[0] != "#":
                k, sz, rm, hx = line.split()
                out[int(k)] = (int(hx, 16), int(sz), float(rm))
    return out


def _mri_solve(dev, seed, mp, refit):
    from workloads import mri as WM
    inst = WM.mri_instance(seed)
    mask = np.zeros(128 * 128, np.uint8)
    mask[inst.meta["freqs"]] = 1
    cim = L.cim_params(n_steps=1000, field="BN", K=1.0, d=0.6)
    sp = L.solve_params(eta_init=0.8, eta_end=0.03, velo=11, n_outer=11, replicas=64, seed=seed,
                        final_refit_f64=refit)
    R, sig, stats = L.l0cim_mri_solve(mp, t(f32(inst.A), dev), t(f32(inst.y), dev), t(mask, dev, torch.uint8), cim, sp)
    torch.cuda.synchronize()
    return inst, R.double().cpu().numpy(), sig.cpu().numpy(), L.read_stats(stats)


def test_mri_solve_matches_oracle_supports(dev):
    """l0cim_mri_solve (factored couplings, gamma = 0, Jacobi CDP in factored
    form, FP64 refit) on the ten seeds with a stored FP64 oracle result.
    Measured on MI355X: identical supports on 7 of 10 (seeds 0, 3 and 4
    differ on 0.7-1.2% of the spins, after the bifurcation of 64 chaotic
    replicas at N = 16384), every |RMSE - RMSE_oracle| <= 1e-3 (the three
    that differ are 0.1-0.9e-3 lower).  Gate: at least the measured 7 of 10,
    and the RMSE bound on all."""
    gold = _golden("mri")
    assert len(gold) == 10
    same, rows = 0, []
    for seed in sorted(gold):
        inst, R, sg, st = _mri_solve(dev, seed, L.mri_params(), 1)
        mask_o, k_o, rm_o = gold[seed]
        so = np.array([(mask_o >> r) & 1 for r in range(128 * 128)], np.uint8)
        rm = O.rmse(sg, R, inst.x, inst.xi)
        same += int(np.array_equal(sg, so))
        rows.append((seed, int(sg.sum()), k_o, float(np.mean(sg != so)), rm, rm_o))
        assert st.status_bits == 0
        assert abs(rm - rm_o) <= 1e-3, (seed, rm, rm_o)
    for r in rows:
        print("seed %d: |S| %d (oracle %d), Hamming %.4f, RMSE %.5f (oracle %.5f)" % r)
    print(f"identical supports: {same}/{len(rows)}")
    assert same >= 7


def test_mri_pipeline_solve_against_oracle(dev):
    """The MRI pipeline around the path (gamma = 1e-4 L2 term, LASSO start,
    CG CDP) through l0cim_mri_solve, against the oracle's stored results where
    they exist: no status bits, RMSE within 1e-3 of the oracle's."""
    gold = _golden("mri_l2")
    mp = L.mri_params(gamma=1e-4, lasso_iters=200, lasso_lam1=3e-4, cdp=L.CDP_CG, cg_max_iter=10000, cg_tol=1e-5)
    for seed in sorted(gold) or [0]:
        inst, R, sg, st = _mri_solve(dev, seed, mp, 0)
        rm = O.rmse(sg, R, inst.x, inst.xi)
        msg = f"pipeline seed {seed}: |S| {int(sg.sum())}, RMSE {rm:.5f}"
        if seed in gold:
            so = np.array([(gold[seed][0] >> r) & 1 for r in range(128 * 128)], np.uint8)
            msg += f" (oracle |S| {gold[seed][1]}, RMSE {gold[seed][2]:.5f}, Hamming {np.mean(sg != so):.4f})"
            assert abs(rm - gold[seed][2]) <= 1e-3
        print(msg)
        assert st.status_bits == 0
