"""GPU parity of the MF-CIM run with the MRI-shaped couplings applied in
factored form (l0cim_mri_mfcim_run) against the oracle's factored operator.

The couplings are J = -(A^T A) o R R^T with a zero diagonal for A = S C Psi^T
(the sampled rows of the orthonormal 2-D DCT-II of the image of the 3-level
Haar synthesis).  The oracle applies J with scipy's DCT and its own Haar
transform in FP64; the device with FFT-based DCTs and its Haar transform in
FP32.  Both sides get the same FP32 R, D = diag(A^T A), b = A^T y and c0 (z = R o b
rounded to FP32, as the device forms it).
Gates: for the continuous field, normwise relative 1e-5 per Euler step over
the first 200 steps for c and e (as for the dense couplings).  For the
binarised field X = H(c) jumps where an amplitude crosses zero, and a
rounding-level difference can move a crossing by one step, after which the
two trajectories differ by more than rounding; there every device step is
checked against the oracle's step taken from the device's previous state
(normwise 1e-5), and crossings that land on different steps than in the
oracle's own trajectory are counted, not gated.  Always: sigma = H(c) of the
device's own final state, and the eq. 4 energy of that sigma to 1e-5
relative.
"""
import numpy as np
import pytest
import torch

import paper_2405_00366_amd as L
import workloads as W
from oracle import mfcim as O, mri as MRI

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
def mri_case():
    """The seed-0 MRI-shaped instance (128 x 128 phantom, 30% of the DCT
    frequencies): FP32 D, b, R = b / D, and the sampling mask."""
    from workloads import mri as WM
    inst = WM.mri_instance(0)
    A = f32(inst.A)
    D = f32(np.einsum("kr,kr->r", A, A))
    b = f32(A.T @ f32(inst.y))
    R = f32(b / D)
    mask = np.zeros(128 * 128, np.uint8)
    mask[inst.meta["freqs"]] = 1
    return dict(freqs=inst.meta["freqs"], D=D, b=b, R=R, mask=mask)


def oracle_trace(op, R, z, c0, eta, prm, steps):
    c = np.array(c0, float)
    e = np.ones_like(c)
    out = np.empty((steps, 2) + c.shape)
    for k in range(steps):
        phi = MRI.scaled_field(op, R, z, c, prm)
        c, e = O.euler_step(c, e, phi, O.pump(k * prm.dt, prm), eta, prm)
        out[k, 0], out[k, 1] = c, e
    return out


@pytest.mark.parametrize("field,P,levels,Rkind", [("CN", 2, 3, "ls"), ("BN", 2, 3, "ls"),
                                                  ("CN", 1, 1, "random"), ("BN", 3, 3, "random"),
                                                  ("CN", 1, 0, "random"), ("CN", 1, 2, "random"),
                                                  ("CN", 1, 4, "random"), ("CN", 1, 7, "random")])
def test_mri_run_trace_parity(dev, mri_case, field, P, levels, Rkind):
    steps, eta, seed, n = 200, 0.022, 4, 128 * 128
    R = mri_case["R"] if Rkind == "ls" else f32(W.random_r(seed, n, 0.3))
    D, b = mri_case["D"], mri_case["b"]
    z = f32(R * b)
    op = MRI.MriOperator(128, mri_case["freqs"], levels=levels, A=np.zeros((1, n)))
    op.colnorm2 = D
    c0 = f32(W.initial_amplitudes(seed, P, n))
    prm = O.CimParams(n_steps=steps, field=field, K=0.1, d=0.6)
    ref = oracle_trace(op, R, z, c0, eta, prm, steps)

    t = lambda x, dt=torch.float32: torch.tensor(np.asarray(x), dtype=dt, device=dev)
    c = t(c0)
    e = torch.ones_like(c)
    tr = torch.empty((steps, 2, P, n), dtype=torch.float32, device=dev)
    H = torch.empty(P, dtype=torch.float64, device=dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    sig = L.l0cim_mri_mfcim_run(128, levels, t(mri_case["mask"], torch.uint8), t(R), t(D), t(b), eta,
                                L.cim_params(n_steps=steps, field=field, K=0.1, d=0.6), c, e, H=H, trace=tr,
                                trace_steps=steps, status=status)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    got = tr.double().cpu().numpy()
    if field == "CN":
        worst = max(normwise(got[k, v], ref[k, v]) for k in range(steps) for v in range(2))
    else:
        worst = 0.0
        cp, ep = c0, np.ones_like(c0)
        for k in range(steps):
            phi = MRI.scaled_field(op, R, z, cp, prm)
            cn, en = O.euler_step(cp, ep, phi, O.pump(k * prm.dt, prm), eta, prm)
            worst = max(worst, normwise(got[k, 0], cn), normwise(got[k, 1], en))
            cp, ep = got[k, 0], got[k, 1]
        flips = sum(int(np.sum((got[k, 0] > 0) != (ref[k, 0] > 0))) for k in range(steps))
        print(f"binarised field: {flips} spin-steps on the other side of zero than in the oracle's trajectory")
        # measured on MI355X: 0 (P = 2, least-squares R) and 44 of 9.8e6 (P = 3, random R); an FP32
        # amplitude within rounding of zero may take the other side, and the bound allows 2e-5 of them
        assert flips <= 2e-5 * steps * n * P, f"{flips} binarised spin-steps differ"
    assert worst <= 1e-5, f"worst normwise error {worst:.3g}"
    cf = c.double().cpu().numpy()
    sg = sig.cpu().numpy()
    assert np.array_equal(sg, (cf > 0).astype(np.uint8))
    Hs = MRI.ising_energy(op, R, z, sg, 0.5 * eta * eta)
    np.testing.assert_allclose(H.cpu().numpy(), Hs, rtol=1e-5, atol=1e-6)


def test_mri_run_zero_steps_energy(dev, mri_case):
    """n_steps = 0 returns the initial state; the energy of its support is one
    application of the factored couplings (a direct check of G v)."""
    n, P = 128 * 128, 4
    R, D, b = mri_case["R"], mri_case["D"], mri_case["b"]
    z = f32(R * b)
    op = MRI.MriOperator(128, mri_case["freqs"], levels=3, A=np.zeros((1, n)))
    op.colnorm2 = D
    rng = np.random.default_rng(9)
    c0 = f32(rng.standard_normal((P, n)) * np.array([[0.1], [1.0], [1.0], [1.0]]))
    c0[3] = -np.abs(c0[3])   # an empty support
    t = lambda x, dt=torch.float32: torch.tensor(np.asarray(x), dtype=dt, device=dev)
    c = t(c0)
    e = torch.ones_like(c)
    H = torch.empty(P, dtype=torch.float64, device=dev)
    sig = L.l0cim_mri_mfcim_run(128, 3, t(mri_case["mask"], torch.uint8), t(R), t(D), t(b), 0.05,
                                L.cim_params(n_steps=0), c, e, H=H)
    torch.cuda.synchronize()
    sg = sig.cpu().numpy()
    assert np.array_equal(sg, (c0 > 0).astype(np.uint8))
    assert np.array_equal(c.double().cpu().numpy(), c0)
    Hs = MRI.ising_energy(op, R, z, sg, 0.5 * 0.05 ** 2)
    np.testing.assert_allclose(H.cpu().numpy(), Hs, rtol=1e-5, atol=1e-6)
    assert H.cpu().numpy()[3] == 0.0


def test_mri_run_reads_the_gram_diagonal_in_place(dev, mri_case):
    """D given as G itself (stride ldg + 1 over its diagonal) gives the same
    bits as the diagonal copied out as a vector."""
    from workloads import mri as WM
    n, P = 128 * 128, 2
    inst = WM.mri_instance(0)
    A = torch.tensor(f32(inst.A), dtype=torch.float32, device=dev)
    y = torch.tensor(f32(inst.y), dtype=torch.float32, device=dev)
    G, b = L.l0cim_gram(A, y)
    R = L.l0cim_init_r(G, b)
    Dv = torch.diagonal(G).contiguous()
    mask = torch.tensor(mri_case["mask"], dtype=torch.uint8, device=dev)
    c0 = torch.tensor(f32(W.initial_amplitudes(2, P, n)), dtype=torch.float32, device=dev)
    prm = L.cim_params(n_steps=50, field="BN", K=1.0, d=0.6)
    outs = []
    for D in (G, Dv):
        c, e = c0.clone(), torch.ones_like(c0)
        H = torch.empty(P, dtype=torch.float64, device=dev)
        L.l0cim_mri_mfcim_run(128, 3, mask, R, D, b, 0.1, prm, c, e, H=H)
        torch.cuda.synchronize()
        outs.append((c.cpu().numpy(), e.cpu().numpy(), H.cpu().numpy()))
    for u, v in zip(*outs):
        assert np.array_equal(u, v)
