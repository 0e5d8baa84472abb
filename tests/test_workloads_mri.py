"""Pins of the MRI-shaped measurement operator (input generator)."""
import math

import numpy as np
from scipy import fft as sfft

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
    S, R_new = OM.refit(inst.A, inst.y, sigma)
    np.testing.assert_allclose(R_new, R_S, rtol=1e-9, atol=1e-12)
    R = np.zeros(n)
    R[S] = R_S
    assert abs(O.rmse(sigma, R, inst.x, inst.xi) - float(rm)) <= 1e-9 * float(rm)
