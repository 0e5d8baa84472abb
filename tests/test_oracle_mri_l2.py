"""CPU pins of the MRI pipeline oracle (oracle/mri_l2.py): the L2-regularised
couplings of eq. 20, the LASSO initial R and the conjugate-gradient CDP.

Every pin is a fact fixed outside the oracle's own code: the spectrum of the
reflecting second difference (the orthonormal DCT-II diagonalises it), the
Gram form of the regularised matrix (an augmented observation matrix), the
dense oracle's Algorithm 1 on that augmented matrix, the exact solution of
the support system, the Jacobi fixed point, and the LASSO optimality
conditions plus an independent coordinate-descent LASSO solver.
"""
import math

import numpy as np
import pytest
from scipy import fft as sfft

import workloads as W
from workloads import mri


def _op16(seed=2, gamma=1e-2):
    from oracle import mri as OM
    from oracle import mri_l2 as L2
    inst = mri.mri_instance(seed, size=16, sparseness=0.2, alpha=0.4)
    op = OM.MriOperator(16, inst.meta["freqs"])
    return inst, op, L2.L2Operator(op, gamma)


def _dense(f, n):
    return np.stack([f(e)[0] for e in np.eye(n)], axis=1)


def test_second_difference_spectrum():
    """The orthonormal DCT-II diagonalises the second difference with the
    reflecting boundary: C D C^T = diag(-4 sin^2(pi k / 2S)).  A wrong
    boundary row or sign breaks it.  Constants are in its null space and a
    quadratic has second difference 2 away from the boundary."""
    from oracle import mri_l2 as L2
    S = 16
    D = np.stack([L2.d2(e, 0) for e in np.eye(S)], axis=1)
    C = sfft.dct(np.eye(S), axis=0, norm="ortho")
    lam = -4.0 * np.sin(np.pi * np.arange(S) / (2 * S)) ** 2
    np.testing.assert_allclose(C @ D @ C.T, np.diag(lam), atol=1e-13)
    np.testing.assert_allclose(L2.d2(np.ones(S), 0), 0.0, atol=1e-15)
    q = np.arange(S, dtype=float) ** 2
    np.testing.assert_allclose(L2.d2(q, 0)[1:-1], 2.0)


def test_smoothness_term_in_the_dct_domain():
    """Psi (D_v^T D_v + D_h^T D_h) Psi^T equals Psi C^T diag(lam_r^2 + lam_c^2) C Psi^T
    (2-D orthonormal DCT-II, lam_k = 4 sin^2(pi k / 2S)), and its diagonal is
    the one the operator stores."""
    inst, op, hop = _op16()
    S = 16
    lam = 4.0 * np.sin(np.pi * np.arange(S) / (2 * S)) ** 2
    wgt = lam[:, None] ** 2 + lam[None, :] ** 2
    from oracle import mri as OM
    v = np.random.default_rng(1).standard_normal((3, S * S))
    img = OM._ihaar(v.reshape(-1, S, S), 3)
    spec = sfft.idctn(wgt * sfft.dctn(img, axes=(1, 2), norm="ortho"), axes=(1, 2), norm="ortho")
    ref = OM._haar(spec, 3).reshape(3, -1)
    np.testing.assert_allclose(hop.smooth_apply(v), ref, atol=1e-11)
    Ld = _dense(hop.smooth_apply, S * S)
    np.testing.assert_allclose(hop.l2diag, np.diag(Ld), atol=1e-12)
    np.testing.assert_allclose(Ld, Ld.T, atol=1e-12)


def test_regularised_gram_is_the_gram_of_an_augmented_matrix():
    """G_gamma = A~^T A~ with A~ = [A; sqrt(gamma) D_v Psi^T; sqrt(gamma) D_h Psi^T],
    built from the dense A and explicit difference and synthesis matrices."""
    from oracle import mri_l2 as L2
    inst, op, hop = _op16(gamma=3e-3)
    n, S = 256, 16
    Psi_T = np.stack([mri.ihaar2(e.reshape(S, S), 3).ravel() for e in np.eye(n)], axis=1)
    Dv = _dense(lambda e: L2.d2(e.reshape(1, S, S), 1).reshape(1, -1), n)
    Dh = _dense(lambda e: L2.d2(e.reshape(1, S, S), 2).reshape(1, -1), n)
    At = np.vstack([inst.A, math.sqrt(3e-3) * Dv @ Psi_T, math.sqrt(3e-3) * Dh @ Psi_T])
    np.testing.assert_allclose(_dense(hop.gram_apply, n), At.T @ At, atol=1e-11)
    np.testing.assert_allclose(hop.colnorm2, np.einsum("kr,kr->r", At, At), atol=1e-12)


@pytest.mark.parametrize("field", ["CN", "BN"])
def test_regularised_solve_equals_dense_solve_on_augmented_matrix(field):
    """Algorithm 1 with the factored L2-regularised couplings (the MRI
    oracle's run, energies and Jacobi CDP on an L2Operator) equals the dense
    oracle's solve on the augmented observation matrix (y padded with zeros):
    the same sigma in every alternation and R to 1e-10."""
    from oracle import mfcim as O
    from oracle import mri as OM
    from oracle import mri_l2 as L2
    gamma, S, n = 2e-3, 16, 256
    inst, op, hop = _op16(3, gamma)
    Psi_T = np.stack([mri.ihaar2(e.reshape(S, S), 3).ravel() for e in np.eye(n)], axis=1)
    Dv = _dense(lambda e: L2.d2(e.reshape(1, S, S), 1).reshape(1, -1), n)
    Dh = _dense(lambda e: L2.d2(e.reshape(1, S, S), 2).reshape(1, -1), n)
    At = np.vstack([inst.A, math.sqrt(gamma) * Dv @ Psi_T, math.sqrt(gamma) * Dh @ Psi_T])
    yt = np.concatenate([inst.y, np.zeros(At.shape[0] - inst.A.shape[0])])
    cim = O.CimParams(n_steps=1000, field=field, K=1.0, d=0.6)
    outer = O.OuterParams(eta_init=0.8, eta_end=0.03, velo=3, n_outer=3, replicas=4, seed=5)
    ref = O.solve(At, yt, cim, outer)
    sig, R, hist = OM.solve(hop, inst.y, cim, outer)
    for i, (h, hr) in enumerate(zip(hist, ref.history)):
        np.testing.assert_array_equal(h["sigma"], hr["sigma"], err_msg=f"alternation {i}")
        np.testing.assert_allclose(h["R_in"], hr["R_in"], rtol=0, atol=1e-10)
    np.testing.assert_allclose(R, ref.R, rtol=0, atol=1e-10)


def test_cg_cdp_solves_the_support_system():
    """The CG CDP returns the exact solution of (G_gamma)_SS R_S = b_S (to its
    tolerance) and, off the support, the Jacobi CDP's fixed point; the empty
    support leaves R_r = b_r / (G_gamma)_rr; a tolerance of 0 stops at the
    iteration cap."""
    from oracle import mri as OM
    from oracle import mri_l2 as L2
    inst, op, hop = _op16(4, 1e-2)
    n = 256
    b = hop.AT(inst.y)[0]
    sig = inst.xi.copy()
    S = np.flatnonzero(sig)
    G = _dense(hop.gram_apply, n)
    R0 = np.random.default_rng(3).standard_normal(n)
    R, its, st = L2.cdp_cg(hop, b, sig, R0, max_iter=10000, tol=1e-13)
    assert st == 0 and 0 < its <= len(S) + 5
    np.testing.assert_allclose(R[S], np.linalg.solve(G[np.ix_(S, S)], b[S]), rtol=1e-9, atol=1e-11)
    Rj, _ = OM.cdp_jacobi(hop, b, sig, R, 0.1, 3000)
    np.testing.assert_allclose(R, Rj, rtol=1e-8, atol=1e-10)
    Re, its_e, _ = L2.cdp_cg(hop, b, np.zeros(n, np.uint8), R0, tol=1e-6)
    np.testing.assert_allclose(Re, b / np.diag(G), rtol=1e-12)
    _, its_cap, _ = L2.cdp_cg(hop, b, sig, R0, max_iter=7, tol=0.0)
    assert its_cap == 7


def _lasso_cd(G, b, lam1, sweeps):
    """Cyclic coordinate descent on (1/2) x^T G x - b^T x + lam1 ||x||_1."""
    x = np.zeros(len(b))
    g = -b.copy()                       # gradient G x - b
    for _ in range(sweeps):
        for r in range(len(b)):
            z = x[r] - g[r] / G[r, r]
            xn = np.sign(z) * max(abs(z) - lam1 / G[r, r], 0.0)
            if xn != x[r]:
                g += G[:, r] * (xn - x[r])
                x[r] = xn
    return x


def test_lasso_fista_optimality_and_independent_solver():
    """FISTA's LASSO iterate satisfies the optimality conditions (gradient
    -lam1 sign(x_r) on the non-zeros, |gradient| <= lam1 elsewhere) and
    equals a coordinate-descent solution of the same strictly convex problem;
    with lam1 = 0 it is G_gamma^-1 b."""
    from oracle import mri_l2 as L2
    inst, op, hop = _op16(5, 5e-2)
    n = 256
    b = hop.AT(inst.y)[0]
    G = _dense(hop.gram_apply, n)
    lam1 = 0.02
    x = L2.lasso_fista(hop, b, lam1, 4000)
    g = G @ x - b
    nz = np.abs(x) > 1e-9
    assert 0 < nz.sum() < n
    np.testing.assert_allclose(g[nz], -lam1 * np.sign(x[nz]), atol=1e-7)
    assert np.all(np.abs(g[~nz]) <= lam1 + 1e-7)
    np.testing.assert_allclose(x, _lasso_cd(G, b, lam1, 3000), atol=1e-7)
    x0 = L2.lasso_fista(hop, b, 0.0, 4000)
    np.testing.assert_allclose(x0, np.linalg.solve(G, b), rtol=1e-6, atol=1e-8)
    # the step is within the Lipschitz bound: ||G_gamma||_2 <= 1 + 32 gamma
    assert np.max(np.linalg.eigvalsh(G)) <= 1.0 + 32 * hop.gamma + 1e-12


def test_pipeline_solve_runs_lasso_then_cg():
    """The pipeline solve starts from the LASSO iterate and applies the CG CDP
    each alternation: its first R_in is lasso_fista's output, and after each
    alternation R on the support solves that support's system."""
    from oracle import mfcim as O
    from oracle import mri_l2 as L2
    inst, op, hop = _op16(6, 1e-2)
    b = hop.AT(inst.y)[0]
    cim = O.CimParams(n_steps=600, field=O.BN, K=1.0, d=0.6)
    outer = O.OuterParams(eta_init=0.6, eta_end=0.05, velo=3, n_outer=3, replicas=4, seed=2)
    sig, R, hist = L2.solve(hop, inst.y, cim, outer, lam1=0.01, lasso_iters=200, cg_tol=1e-12)
    np.testing.assert_allclose(hist[0]["R_in"], L2.lasso_fista(hop, b, 0.01, 200), atol=0)
    G = _dense(hop.gram_apply, 256)
    S = np.flatnonzero(sig)
    np.testing.assert_allclose(R[S], np.linalg.solve(G[np.ix_(S, S)], b[S]), rtol=1e-8, atol=1e-10)
