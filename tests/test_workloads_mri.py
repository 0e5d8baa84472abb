"""Pins of the MRI-shaped measurement operator (input generator)."""
import math

import numpy as np
import pytest
from scipy import fft as sfft

import workloads as W
from workloads import mri


def _dct_matrix(n):
    """Orthonormal DCT-II matrix written from its definition."""
    C = np.zeros((n, n))
    for k in range(n):
        a = math.sqrt(1.0 / n) if k == 0 else math.sqrt(2.0 / n)
        for i in range(n):
            C[k, i] = a * math.cos(math.pi * (2 * i + 1) * k / (2 * n))
    return C


def test_scipy_dct_is_the_orthonormal_dct_ii():
    C = _dct_matrix(8)
    x = np.random.default_rng(0).standard_normal((8, 8))
    np.testing.assert_allclose(sfft.dctn(x, norm="ortho"), C @ x @ C.T, atol=1e-13)


def test_haar_is_orthonormal_and_inverted():
    rng = np.random.default_rng(1)
    for size, levels in ((16, 3), (8, 2), (32, 3)):
        N = size * size
        Psi = np.stack([mri.haar2(e.reshape(size, size), levels).ravel() for e in np.eye(N)], axis=1)
        np.testing.assert_allclose(Psi @ Psi.T, np.eye(N), atol=1e-12)
        x = rng.standard_normal((size, size))
        np.testing.assert_allclose(mri.ihaar2(mri.haar2(x, levels), levels), x, atol=1e-12)


def test_haar_one_level_values():
    """One level on a 2 x 2 block: [[a, b], [c, d]] -> LL = (a+b+c+d)/2,
    HL = (a-b+c-d)/2, LH = (a+b-c-d)/2, HH = (a-b-c+d)/2."""
    x = np.array([[1.0, 2.0], [3.0, 4.0]])
    y = mri.haar2(x, 1)
    np.testing.assert_allclose(y, [[5.0, -1.0], [-2.0, 0.0]], atol=1e-14)


def test_measurement_rows_are_orthonormal():
    size = 16
    freqs = mri.sample_frequencies(3, size, 77)
    assert freqs[0] == 0 and len(set(freqs.tolist())) == 77
    A = mri.measurement_matrix(freqs, size)
    np.testing.assert_allclose(A @ A.T, np.eye(77), atol=1e-12)
    # A x equals the sampled DCT of the image whose Haar coefficients are x
    x = np.random.default_rng(4).standard_normal(size * size)
    img = mri.ihaar2(x.reshape(size, size))
    np.testing.assert_allclose(A @ x, sfft.dctn(img, norm="ortho").ravel()[freqs], atol=1e-12)


def test_small_instance_shapes_and_sparsity():
    inst = mri.mri_instance(5, size=32, sparseness=0.2, alpha=0.3)
    assert inst.A.shape == (round(0.3 * 1024), 1024)
    assert 0 < int(inst.xi.sum()) <= round(0.2 * 1024)
    assert np.all(inst.x[inst.xi == 1] != 0)
    assert np.all(inst.x[inst.xi == 0] == 0)
    img = inst.meta["image"]
    assert img.min() >= 0.0 and img.max() <= 1.0


def test_factored_couplings_equal_dense_couplings():
    """The MRI oracle's factored J x equals the dense coupling form of the
    general oracle (J = -G o R R^T, zero diagonal) on a 16 x 16 instance, and
    so do its fields, energies and Jacobi sweeps."""
    from oracle import mfcim as O
    from oracle import mri as OM

    inst = mri.mri_instance(2, size=16, sparseness=0.2, alpha=0.4)
    op = OM.MriOperator(16, inst.meta["freqs"])
    G, b = O.gram(inst.A, inst.y)
    np.testing.assert_allclose(op.colnorm2, np.diag(G), atol=1e-12)
    np.testing.assert_allclose(op.AT(inst.y)[0], b, atol=1e-12)
    rng = np.random.default_rng(3)
    R = rng.standard_normal(256)
    J, z = O.couplings(G, b, R)
    X = rng.standard_normal((3, 256))
    np.testing.assert_allclose(OM.coupling_apply(op, R, X), X @ J.T, atol=1e-11)
    for field in ("CN", "BN"):
        prm = O.CimParams(field=field)
        np.testing.assert_allclose(OM.scaled_field(op, R, z, X, prm), O.scaled_field(J, z, X, prm), atol=1e-11)
    sig = (rng.random((2, 256)) < 0.2).astype(np.uint8)
    np.testing.assert_allclose(OM.ising_energy(op, R, z, sig, 0.01), O.ising_energy(J, z, sig, 0.01), atol=1e-10)
    Ra, _ = OM.cdp_jacobi(op, b, sig[0], R, 0.1, 20)
    Rb, _ = O.cdp_jacobi(G, b, sig[0], R, 0.1, 20)
    np.testing.assert_allclose(Ra, Rb, atol=1e-10)


def test_stored_oracle_refit_matches_the_stored_support():
    """The stored oracle refit (tests/golden/oracle_refit_mri.txt) is the
    oracle's least squares on the stored seed-0 support, and that support's
    stored RMSE is the RMSE of that refit against the ground truth."""
    import os
    from oracle import mfcim as O, mri as OM
    here = os.path.join(os.path.dirname(__file__), "golden")
    sup = [l.split() for l in open(os.path.join(here, "oracle_supports_mri.txt")) if l.strip() and l[0] != "#"]
    ref = [l.split() for l in open(os.path.join(here, "oracle_refit_mri.txt")) if l.strip() and l[0] != "#"]
    seed, k, rm, hx = next(r for r in sup if r[0] == "0")
    R_S = np.array([float(v) for v in next(r for r in ref if r[0] == "0")[2:]])
    inst = mri.mri_instance(0)
    n = inst.A.shape[1]
    v = int(hx, 16)
    sigma = np.array([(v >> r) & 1 for r in range(n)], np.uint8)
    assert int(sigma.sum()) == int(k) == len(R_S)
    S, R_new, _st = OM.refit(inst.A, inst.y, sigma)
    np.testing.assert_allclose(R_new, R_S, rtol=1e-9, atol=1e-12)
    R = np.zeros(n)
    R[S] = R_S
    assert abs(O.rmse(sigma, R, inst.x, inst.xi) - float(rm)) <= 1e-9 * float(rm)


def _mri16(seed=2):
    from oracle import mri as OM
    inst = mri.mri_instance(seed, size=16, sparseness=0.2, alpha=0.4)
    return inst, OM.MriOperator(16, inst.meta["freqs"])


@pytest.mark.parametrize("field", ["CN", "BN"])
def test_factored_run_trace_equals_dense_run(field):
    """The MRI oracle's Euler integration (factored couplings) follows the
    dense oracle's mfcim_run step for step on a 16 x 16 instance: 400 steps,
    three replicas, a random R, both fields."""
    from oracle import mfcim as O
    from oracle import mri as OM

    inst, op = _mri16()
    G, b = O.gram(inst.A, inst.y)
    R = np.random.default_rng(7).standard_normal(256)
    J, z = O.couplings(G, b, R)
    prm = O.CimParams(n_steps=400, field=field, K=1.0, d=0.6)
    c0 = W.initial_amplitudes(11, 3, 256)
    e0 = np.ones_like(c0)
    cd, ed, trd = O.mfcim_run(J, z, 0.3, c0, e0, prm, trace_steps=400)
    cf, ef, trf = OM.mfcim_run(op, R, z, 0.3, c0, e0, prm, trace_steps=400)
    for k in range(400):
        for v in range(2):
            err = np.max(np.abs(trf[k, v] - trd[k, v])) / np.max(np.abs(trd[k, v]))
            assert err <= 1e-10, (k, v, err)
    np.testing.assert_array_equal(O.threshold(cf), O.threshold(cd))


@pytest.mark.parametrize("field", ["CN", "BN"])
def test_factored_solve_equals_dense_solve(field):
    """Algorithm 1 in the MRI oracle (R warm start, eta schedule, counter
    generator, replica choice by eq. 4, Jacobi CDP) equals the dense oracle's
    solve on the same 16 x 16 instance and seed: the same selected sigma in
    every alternation and the same R to 1e-10."""
    from oracle import mfcim as O
    from oracle import mri as OM

    inst, op = _mri16(3)
    cim = O.CimParams(n_steps=1000, field=field, K=1.0, d=0.6)
    outer = O.OuterParams(eta_init=0.8, eta_end=0.03, velo=3, n_outer=3, replicas=4, seed=5)
    ref = O.solve(inst.A, inst.y, cim, outer)
    sig, R, hist = OM.solve(op, inst.y, cim, outer)
    assert len(hist) == len(ref.history) == 3
    for i, (h, hr) in enumerate(zip(hist, ref.history)):
        assert h["replica"] == hr["replica"], i
        np.testing.assert_array_equal(h["sigma"], hr["sigma"], err_msg=f"alternation {i}")
        np.testing.assert_allclose(h["R_in"], hr["R_in"], rtol=0, atol=1e-10)
        assert h["H"] == pytest.approx(hr["H"], rel=1e-9, abs=1e-12)
    assert 0 < int(sig.sum()) < 256
    np.testing.assert_array_equal(sig, ref.sigma)
    np.testing.assert_allclose(R, ref.R, rtol=0, atol=1e-10)


def test_factored_refit_equals_dense_refit_and_ridge():
    """The MRI oracle's refit (G_SS and b_S formed from the columns of A)
    equals the dense oracle's Cholesky refit on the same support, and on a
    support larger than M (G_SS singular: A A^T = I, so rank(G) = M) it takes
    the ridge rule and raises the ridge status bit, as the dense one does."""
    from oracle import mfcim as O
    from oracle import mri as OM

    inst, _ = _mri16(4)
    G, b = O.gram(inst.A, inst.y)
    sig = inst.xi.copy()
    S, R_S, st = OM.refit(inst.A, inst.y, sig)
    R_ref, st_ref = O.chol_refit(G, b, sig)
    assert st == 0 and st_ref == 0
    np.testing.assert_allclose(R_S, R_ref[S], rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(R_S, np.linalg.lstsq(inst.A[:, S], inst.y, rcond=None)[0], rtol=1e-8, atol=1e-10)
    big = np.zeros(256, np.uint8)
    big[: inst.A.shape[0] + 20] = 1
    S, R_S, st = OM.refit(inst.A, inst.y, big)
    _, st_ref = O.chol_refit(G, b, big)
    assert st & O.ST_CHOL_RIDGE and st_ref & O.ST_CHOL_RIDGE
    assert np.all(np.isfinite(R_S))
