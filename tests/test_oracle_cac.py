"""CPU pins of the CAC-CIM (Positive-P) oracle, oracle/cac.py (eq. 5-11).

Each pin ties the oracle to a fact outside its own code:
  * with g^2 = 0 the model has no noise and no fluctuation feedback, and eq. 5
    with the eq. 11 field is the mean-field amplitude equation with the
    linear loss (-1 + p - j) and twice the couplings, so the run equals the
    mean-field oracle's run from c = 0 (already pinned) step for step;
  * with mu = 0 and a constant pump the variances follow a linear ODE
    (j -> 0), whose matrix-exponential solution the Euler iterate approaches
    at first order in dt;
  * the noise: the first step of e from mu = 0 has mean 1 - beta g^2 / (4 j)
    (eq. 9 with the eq. 10 variance g^2 / (4 j dt)), and the spread of mu
    grows as the variance recursion of the eq. 5 noise increment says;
  * the step normals are standard normal and differ between steps, spins and
    replicas.
"""
import math

import numpy as np
import pytest
from scipy import linalg, stats

import workloads as W


def _couplings(seed, n=40, m=20):
    from oracle import mfcim as O
    inst = W.gaussian_instance(seed, n, m, 0.2, 0.01)
    G, b = O.gram(inst.A, inst.y)
    R = b / np.diag(G)
    return O.couplings(G, b, R)


def test_noiseless_cac_equals_mean_field_with_linear_loss_and_double_couplings():
    from oracle import cac as C
    from oracle import mfcim as O
    J, z = _couplings(3)
    prm = C.CacParams(g2=0.0, tau=0.21, n_steps=400)
    mu, n, m, e, tr = C.cac_run(J, z, 0.3, seed=1, alt=0, P=2, prm=prm, trace_steps=400)
    mprm = O.CimParams(n_steps=400, field=O.CN, tau=0.21, linear_j=True, j=prm.j, beta=prm.beta, K=prm.K)
    c, ee, trm = O.mfcim_run(2 * J, 2 * z, 0.3, np.zeros((2, 40)), np.ones((2, 40)), mprm, trace_steps=400)
    np.testing.assert_allclose(tr[:, 0], trm[:, 0], rtol=0, atol=1e-12)
    np.testing.assert_allclose(tr[:, 3], trm[:, 1], rtol=0, atol=1e-12)
    assert np.max(np.abs(mu)) > 0.1        # the run left the origin


def test_variances_follow_the_linear_ode_at_first_order():
    from oracle import cac as C
    p = 0.6
    M = np.array([[-2.0, 2 * p], [2 * p, -2.0]])
    f = np.array([0.0, p])
    T = 2.0
    exact = linalg.expm(M * T) @ np.zeros(2) + np.linalg.solve(M, (linalg.expm(M * T) - np.eye(2)) @ f)
    errs = []
    for dt in (0.02, 0.01, 0.005):
        prm = C.CacParams(g2=0.0, K=0.0, j=1e-12, p_thr=p, d=0.0, dt=dt, n_steps=int(round(T / dt)))
        J = np.zeros((3, 3))
        mu, n, m, e, _ = C.cac_run(J, np.zeros(3), 0.0, 0, 0, 1, prm)
        assert np.all(mu == 0.0)
        errs.append(max(abs(n[0, 0] - exact[0]), abs(m[0, 0] - exact[1])))
    assert 1.8 < errs[0] / errs[1] < 2.2 and 1.8 < errs[1] / errs[2] < 2.2
    assert errs[2] < 2e-3


def test_measurement_noise_enters_the_amplitude_control():
    """From mu = 0: e after one step is 1 - dt beta (mu~^2 - tau) with
    mu~ = sqrt(g^2/(4j)) xi / sqrt(dt), so its mean over many spins is
    1 - beta g^2 / (4 j) + dt beta tau."""
    from oracle import cac as C
    prm = C.CacParams(g2=4e-3, j=0.5, beta=0.7, tau=0.1, K=0.0, n_steps=1)
    N = 200000
    xi = np.random.default_rng(0).standard_normal((1, N))
    mu, n, m, e, _ = C.cac_run(_ZeroJ(N), np.zeros(N), 0.0, 0, 0, 1, prm, xi_fn=lambda k: xi)
    want = 1.0 - prm.beta * prm.g2 / (4 * prm.j) + prm.dt * prm.beta * prm.tau
    sem = prm.beta * prm.g2 / (4 * prm.j) * math.sqrt(2.0 / N)
    assert abs(float(np.mean(e)) - want) < 5 * sem


class _ZeroJ:
    """A zero coupling matrix of order N that does not store N^2 zeros."""

    __array_ufunc__ = None          # numpy defers X @ J to __rmatmul__

    def __init__(self, N):
        self.shape = (N, N)
        self.T = self

    def __rmatmul__(self, X):
        return np.zeros_like(np.asarray(X, float))


def test_amplitude_spread_follows_the_noise_recursion():
    """K = 0: mu is driven by the eq. 5 noise increment sqrt(j g^2)(m + n) xi
    sqrt(dt) alone (the mu^3 and g^2 n, g^2 m terms are ~1e-8 of the linear
    one here), so Var(mu) follows v' = (1 - dt a)^2 v + j g^2 (m + n)^2 dt,
    a = 1 - p + j, with the deterministic n, m of the oracle."""
    from oracle import cac as C
    N, steps = 40000, 300
    prm = C.CacParams(K=0.0, n_steps=steps)
    mu, n, m, e, tr = C.cac_run(_ZeroJ(N), np.zeros(N), 0.0, 5, 0, 1, prm, trace_steps=steps)
    v = 0.0
    for k in range(steps):
        nn = 0.0 if k == 0 else float(np.mean(tr[k - 1, 1]))
        mm = 0.0 if k == 0 else float(np.mean(tr[k - 1, 2]))
        a = 1.0 - C.pump(k * prm.dt, prm) + prm.j
        v = (1.0 - prm.dt * a) ** 2 * v + prm.j * prm.g2 * (mm + nn) ** 2 * prm.dt
    # n, m are (up to the mu^2 terms, ~1e-8) the same for every spin
    assert np.ptp(tr[-1, 1]) < 1e-5 * np.max(tr[-1, 1]) and np.ptp(tr[-1, 2]) < 1e-5 * np.max(tr[-1, 2])
    got = float(np.var(mu))
    assert abs(got / v - 1.0) < 4 * math.sqrt(2.0 / N)


def test_step_normals_are_standard_normal_and_fresh():
    from oracle import rng
    x = rng.step_normals(7, 2, 11, 4, 5000)
    assert stats.kstest(x.ravel(), "norm").pvalue > 1e-3
    bound = 5.0 / math.sqrt(x.size)              # five standard errors of a sample correlation
    y = rng.step_normals(7, 2, 12, 4, 5000)
    z = rng.step_normals(7, 3, 11, 4, 5000)
    assert abs(np.corrcoef(x.ravel(), y.ravel())[0, 1]) < bound
    assert abs(np.corrcoef(x.ravel(), z.ravel())[0, 1]) < bound
    assert abs(np.corrcoef(x[0], x[1])[0, 1]) < 5.0 / math.sqrt(x.shape[1])
    c0 = rng.standard_normals(7, 2, 4, 5000)    # the initial-amplitude stream of the same seed
    assert abs(np.corrcoef(x.ravel(), c0.ravel())[0, 1]) < bound
    with pytest.raises(ValueError):
        rng.step_normals(7, 1 << 11, 0, 1, 1)


def test_cac_solve_recovers_noiseless_supports():
    """Algorithm 1 with the CAC-CIM on the exhaustive set used for the
    mean-field oracle (N = M = 12, 3 well-separated non-zeros, noiseless,
    where the brute-force optimum of eq. 3 is the true support): the CAC-CIM
    finds the true support on most seeds (a heuristic; threshold set from the
    measured count)."""
    from oracle import cac as C
    from oracle import mfcim as O
    found = 0
    for seed in range(12):
        inst = W.well_separated_instance(seed, 12, k=3, nu=0.0, alpha=1.0)
        res = C.solve(inst.A, inst.y, C.CacParams(),
                      O.OuterParams(eta_init=0.8, eta_end=0.2, velo=8, n_outer=10, seed=seed))
        found += int(np.array_equal(res.sigma, inst.xi))
    print(f"CAC-CIM noiseless recovery: {found}/12")
    assert found >= 10
