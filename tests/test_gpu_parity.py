"""GPU parity of every step of the path against the FP64 oracle, through the C ABI.

Inputs are seeded and rounded to the device precision before either side sees
them, so differences measure arithmetic only.  Tolerances:
  * amplitudes / error variables, first 200 Euler steps: normwise relative
    max_r |c_gpu - c_oracle| / max_r |c_oracle| <= 1e-5 at every step (FP32),
    1e-12 (FP64);
  * integer results (supports, quantised codes, counters): bit-exact;
  * FP32 reductions of length n: 1e-5 relative (normwise);
  * FP64 Cholesky refit: 1e-10 relative.
"""
import math
import os

import numpy as np
import pytest
import torch

import paper_2405_00366_amd as L
import workloads as W
from oracle import mfcim as O, quant as Q, rng as ORNG

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    return torch.device("cuda:0")


def t(x, dtype, dev):
    return torch.tensor(np.asarray(x), dtype=dtype, device=dev)


def normwise(got, ref):
    den = np.max(np.abs(ref))
    return float(np.max(np.abs(got - ref)) / (den if den > 0 else 1.0))


def f32(x):
    return np.asarray(x, np.float64).astype(np.float32).astype(np.float64)


def problem(seed, n, m=None, Rscale=None):
    """FP32-exact G, b, R for kernel-level checks."""
    inst = W.gaussian_instance(seed, n, m or max(1, n // 2), 0.1, 0.01).rounded_f32()
    G, b = O.gram(inst.A, inst.y)
    G32, b32 = f32(G), f32(b)
    R = f32(b / np.diag(G)) if Rscale is None else f32(W.random_r(seed, n, Rscale))
    return inst, G32, b32, R


# ---------------------------------------------------------------------------
# a1: Gram / Zeeman prep
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("m,n", [(300, 517), (1000, 2000), (7, 3), (64, 64)])
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_gram_parity(dev, m, n, dtype):
    inst = W.gaussian_instance(1, n, m, 0.1, 0.01)
    A = inst.A.astype(np.float32).astype(np.float64) if dtype == torch.float32 else inst.A
    y = f32(inst.y) if dtype == torch.float32 else inst.y
    G, b = L.l0cim_gram(t(A, dtype, dev), t(y, dtype, dev))
    torch.cuda.synchronize()
    Gg, bg = G.double().cpu().numpy(), b.double().cpu().numpy()
    Go, bo = O.gram(A, y)
    eps = np.finfo(np.float32 if dtype == torch.float32 else np.float64).eps
    bound = 2 * m * eps * (np.abs(A).T @ np.abs(A)) + 1e-300
    assert np.all(np.abs(Gg - Go) <= bound)
    assert np.array_equal(Gg, Gg.T), "G must be bitwise symmetric"
    bb = 2 * m * eps * (np.abs(A).T @ np.abs(y)) + 1e-300
    assert np.all(np.abs(bg - bo) <= bb)


# ---------------------------------------------------------------------------
# a2: couplings
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n", [517, 2000, 1])
def test_couplings_f32(dev, n):
    _, G32, b32, _ = problem(2, n)
    R = f32(W.random_r(2, n))
    J, rs, z = L.l0cim_build_couplings(t(G32, torch.float32, dev), t(b32, torch.float32, dev),
                                       t(R, torch.float32, dev))
    torch.cuda.synchronize()
    Jg, zg = J.double().cpu().numpy(), z.double().cpu().numpy()
    Jo, zo = O.couplings(G32, b32, R)
    assert np.array_equal(Jg, Jg.T) and np.all(np.diag(Jg) == 0)
    assert np.all(np.abs(Jg - Jo) <= 2.5 * np.finfo(np.float32).eps * np.abs(Jo))
    assert np.all(np.abs(zg - zo) <= np.finfo(np.float32).eps * np.abs(zo))


def test_couplings_f64(dev):
    n = 300
    inst = W.gaussian_instance(3, n, 150, 0.1, 0.01)
    G, b = O.gram(inst.A, inst.y)
    R = W.random_r(3, n)
    J, _, z = L.l0cim_build_couplings(t(G, torch.float64, dev), t(b, torch.float64, dev),
                                      t(R, torch.float64, dev))
    torch.cuda.synchronize()
    Jo, zo = O.couplings(G, b, R)
    assert np.array_equal(J.cpu().numpy(), Jo)      # same operations, same order
    assert np.array_equal(z.cpu().numpy(), zo)


@pytest.mark.parametrize("fmt,code", [("fp8", L.FP8E4M3), ("bf16", L.BF16)])
@pytest.mark.parametrize("n", [300, 2049])
def test_couplings_quantised_bit_exact(dev, fmt, code, n):
    _, G32, b32, _ = problem(4, n)
    R = f32(W.random_r(4, n))
    J, rs, z = L.l0cim_build_couplings(t(G32, torch.float32, dev), t(b32, torch.float32, dev),
                                       t(R, torch.float32, dev), j_dtype=code)
    torch.cuda.synchronize()
    J32, _ = Q.couplings_f32(G32, b32, R)
    q, s = Q.quantize_rows(J32, fmt)
    assert np.array_equal(rs.cpu().numpy(), s)
    assert np.array_equal(J.float().cpu().numpy(), q)


# ---------------------------------------------------------------------------
# a7: counter-based initial state
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_init_state_matches_counter_generator(dev, dtype):
    n, P = 1000, 3
    c = torch.empty((P, n), dtype=dtype, device=dev)
    e = torch.empty_like(c)
    L.l0cim_init_state(n, P, 12345, 7, 1e-2, c, e)
    torch.cuda.synchronize()
    c0, e0 = ORNG.initial_state(12345, 7, P, n, 1e-2)
    tol = 4 * np.finfo(np.float32).eps if dtype == torch.float32 else 1e-14
    np.testing.assert_allclose(c.double().cpu().numpy(), c0, rtol=tol, atol=1e-300)
    assert np.all(e.cpu().numpy() == 1)


# ---------------------------------------------------------------------------
# a3 + a4: the MF-CIM run, 200-step trace parity
# ---------------------------------------------------------------------------

TRACE_CASES = [
    # n,    P, field, launch, dtype
    (64,    1, "CN", L.LAUNCH_AUTO, torch.float32),
    (64,    4, "BN", L.LAUNCH_AUTO, torch.float32),
    (250,   2, "CN", L.LAUNCH_AUTO, torch.float32),
    (2000,  1, "CN", L.LAUNCH_RESIDENT, torch.float32),
    (2000,  1, "BN", L.LAUNCH_RESIDENT, torch.float32),
    (4000,  1, "BN", L.LAUNCH_RESIDENT, torch.float32),
    (3001,  1, "CN", L.LAUNCH_AUTO, torch.float32),
    (777,   3, "CN", L.LAUNCH_RESIDENT, torch.float32),
    (777,   2, "CN", L.LAUNCH_STREAMED, torch.float32),
    (1500,  1, "BN", L.LAUNCH_STREAMED, torch.float32),
    (300,   4, "CN", L.LAUNCH_MATRIX, torch.float32),
    (257,  16, "BN", L.LAUNCH_MATRIX, torch.float32),
    (1000, 33, "CN", L.LAUNCH_MATRIX, torch.float32),
    (2048, 64, "BN", L.LAUNCH_AUTO, torch.float32),
    (64,    1, "CN", L.LAUNCH_AUTO, torch.float64),
    (700,   2, "CN", L.LAUNCH_RESIDENT, torch.float64),
    (300,   1, "BN", L.LAUNCH_STREAMED, torch.float64),
]


def _trace_case(dev, n, P, field, launch, dtype, steps=200, eta=0.6, jfmt=None, seed=10):
    inst, G32, b32, R = problem(seed + n, n)
    J, z = O.couplings(G32, b32, R)
    cdt = dtype
    if jfmt is None:
        Jd = f32(J) if dtype == torch.float32 else J
        Jdev = t(Jd, dtype, dev)
        rs = None
        Jo = Jd
    else:
        J32, _ = Q.couplings_f32(G32, b32, R)
        q, s = Q.quantize_rows(J32, jfmt)
        Jo = Q.dequantized(q, s)
        Jdev = t(q, torch.float32, dev).to(torch.float8_e4m3fn if jfmt == "fp8" else torch.bfloat16)
        rs = t(s, torch.float32, dev)
    zo = f32(z) if dtype == torch.float32 else z
    c0 = W.initial_amplitudes(seed, P, n)
    if dtype == torch.float32:
        c0 = f32(c0)
    c = t(c0, cdt, dev)
    e = torch.ones_like(c)
    tr = torch.empty((steps, 2, P, n), dtype=cdt, device=dev)
    H = torch.empty(P, dtype=torch.float64, device=dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    prm = L.cim_params(n_steps=steps, field=field, launch=launch)
    sig = L.l0cim_mfcim_run(Jdev, t(zo, cdt, dev), eta, prm, c, e, H=H, trace=tr, trace_steps=steps,
                            row_scale=rs, status=status)
    torch.cuda.synchronize()
    _, _, tro = O.mfcim_run(Jo, zo, eta, c0, np.ones((P, n)),
                            O.CimParams(n_steps=steps, field=field), trace_steps=steps)
    return tr.double().cpu().numpy(), tro, sig.cpu().numpy(), c.double().cpu().numpy(), H.cpu().numpy(), \
        int(status.item()), (Jo, zo)


@pytest.mark.parametrize("n,P,field,launch,dtype", TRACE_CASES)
def test_mfcim_trace_parity(dev, n, P, field, launch, dtype):
    got, ref, sig, c, H, st, (Jo, zo) = _trace_case(dev, n, P, field, launch, dtype)
    assert st == 0
    tol = 1e-5 if dtype == torch.float32 else 1e-12
    worst = max(normwise(got[k, v], ref[k, v]) for k in range(got.shape[0]) for v in range(2))
    assert worst <= tol, f"worst normwise error {worst:.3g}"
    # the support and energy returned are those of the device's own final state
    assert np.array_equal(sig, (c > 0).astype(np.uint8))
    Hs = O.ising_energy(Jo, zo, sig, O.lam_from_eta(0.6))
    np.testing.assert_allclose(H, Hs, rtol=1e-5 if dtype == torch.float32 else 1e-12, atol=1e-6)


@pytest.mark.parametrize("fmt", ["fp8", "bf16"])
@pytest.mark.parametrize("launch,P,field", [(L.LAUNCH_AUTO, 2, "BN"), (L.LAUNCH_STREAMED, 2, "BN"),
                                            (L.LAUNCH_AUTO, 1, "BN"), (L.LAUNCH_MATRIX, 16, "BN"),
                                            (L.LAUNCH_MATRIX, 64, "CN"), (L.LAUNCH_MATRIX, 5, "CN")])
def test_mfcim_trace_parity_quantised_couplings(dev, fmt, launch, P, field):
    got, ref, sig, c, H, st, _ = _trace_case(dev, 1200, P, field, launch, torch.float32, jfmt=fmt)
    assert st == 0
    worst = max(normwise(got[k, v], ref[k, v]) for k in range(got.shape[0]) for v in range(2))
    assert worst <= 1e-5


def test_mfcim_zero_steps_and_single_spin(dev):
    # n_steps = 0 returns the initial state and its support; n = 1 has J = 0
    got = _trace_case(dev, 1, 1, "CN", L.LAUNCH_AUTO, torch.float32, steps=1)
    assert got[5] == 0
    J = torch.zeros((5, 5), device=dev)
    z = torch.zeros(5, device=dev)
    c = torch.tensor([[-0.3, 0.0, 0.2, 1e-8, -1e-8]], device=dev)
    e = torch.ones_like(c)
    sig = L.l0cim_mfcim_run(J, z, 0.5, L.cim_params(n_steps=0), c, e)
    torch.cuda.synchronize()
    assert sig.cpu().numpy().tolist() == [[0, 0, 1, 1, 0]]


def test_mfcim_full_run_matches_oracle_support(dev):
    """A full 2000-step run at N = 2000 (resident launch): after the bifurcation
    FP32 and FP64 trajectories may separate, so the check is on the final
    support (identical up to a few spins) and on the device's own consistency."""
    n, steps = 2000, 2000
    inst, G32, b32, R = problem(77, n)
    J, z = O.couplings(G32, b32, R)
    Jd, zd = f32(J), f32(z)
    c0 = f32(W.initial_amplitudes(77, 1, n))
    c = t(c0, torch.float32, dev)
    e = torch.ones_like(c)
    H = torch.empty(1, dtype=torch.float64, device=dev)
    sig = L.l0cim_mfcim_run(t(Jd, torch.float32, dev), t(zd, torch.float32, dev), 0.4,
                            L.cim_params(n_steps=steps), c, e, H=H)
    torch.cuda.synchronize()
    co, eo, _ = O.mfcim_run(Jd, zd, 0.4, c0, np.ones((1, n)), O.CimParams(n_steps=steps))
    so = O.threshold(co)
    diff = int(np.sum(sig.cpu().numpy() != so))
    assert diff <= n // 100, f"{diff} spins differ"
    np.testing.assert_allclose(H.cpu().numpy(), O.ising_energy(Jd, zd, sig.cpu().numpy(), 0.08), rtol=1e-5)


def test_spin_limit_aborts_cleanly(dev):
    """A tiny bound on the device waits forces the abort path of the resident
    run (FP64, couplings in LDS, every workgroup polls as soon as it has
    published): every workgroup exits, the timeout bit is raised and nothing
    hangs."""
    n = 2000
    _, G32, b32, R = problem(5, n)
    J, z = O.couplings(G32, b32, R)
    c = t(W.initial_amplitudes(5, 1, n), torch.float64, dev)
    e = torch.ones_like(c)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    prm = L.cim_params(n_steps=500, launch=L.LAUNCH_RESIDENT, spin_limit=1)
    L.l0cim_mfcim_run(t(J, torch.float64, dev), t(z, torch.float64, dev), 0.5, prm, c, e, status=status)
    torch.cuda.synchronize()
    assert int(status.item()) & L.ST_TIMEOUT
    # the same workspace-free call works normally afterwards
    c = t(W.initial_amplitudes(5, 1, n), torch.float64, dev)
    e = torch.ones_like(c)
    status.zero_()
    L.l0cim_mfcim_run(t(J, torch.float64, dev), t(z, torch.float64, dev), 0.5,
                      L.cim_params(n_steps=50, launch=L.LAUNCH_RESIDENT), c, e, status=status)
    torch.cuda.synchronize()
    assert int(status.item()) == 0


def test_spin_limit_register_resident_run_is_bounded(dev):
    """The register-resident FP32 run sleeps before the first poll of a step,
    so its waits are mostly satisfied at once and a tiny bound need not fire;
    whichever way it goes the run ends, raises nothing but the timeout bit,
    and the next run is clean and matches the oracle's first steps."""
    n = 2000
    _, G32, b32, R = problem(5, n)
    J, z = O.couplings(G32, b32, R)
    Jd, zd = t(f32(J), torch.float32, dev), t(f32(z), torch.float32, dev)
    c = t(f32(W.initial_amplitudes(5, 1, n)), torch.float32, dev)
    e = torch.ones_like(c)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    L.l0cim_mfcim_run(Jd, zd, 0.5, L.cim_params(n_steps=500, launch=L.LAUNCH_RESIDENT, spin_limit=1), c, e,
                      status=status)
    torch.cuda.synchronize()
    assert int(status.item()) & ~L.ST_TIMEOUT == 0
    c0 = f32(W.initial_amplitudes(5, 1, n))
    c = t(c0, torch.float32, dev)
    e = torch.ones_like(c)
    status.zero_()
    steps = 50
    tr = torch.empty((steps, 2, 1, n), dtype=torch.float32, device=dev)
    L.l0cim_mfcim_run(Jd, zd, 0.5, L.cim_params(n_steps=steps, launch=L.LAUNCH_RESIDENT), c, e, status=status,
                      trace=tr, trace_steps=steps)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    _, _, tro = O.mfcim_run(f32(J), f32(z), 0.5, c0, np.ones((1, n)), O.CimParams(n_steps=steps), trace_steps=steps)
    got = tr.double().cpu().numpy()
    assert max(normwise(got[k, v], tro[k, v]) for k in range(steps) for v in range(2)) <= 1e-5


# ---------------------------------------------------------------------------
# a5: replica selection
# ---------------------------------------------------------------------------

def test_select_replica_lowest_energy_first_on_ties(dev):
    H = t([3.0, -1.0, 2.0, -1.0, float("nan")], torch.float64, dev)
    sig = t(np.arange(5 * 7).reshape(5, 7) % 2, torch.uint8, dev)
    q = torch.full((1,), -1, dtype=torch.int32, device=dev)
    out = L.l0cim_select_replica(H, sig, q_out=q)
    torch.cuda.synchronize()
    assert int(q.item()) == 1
    assert np.array_equal(out.cpu().numpy(), sig[1].cpu().numpy())
    H2 = t([float("nan"), 5.0], torch.float64, dev)
    L.l0cim_select_replica(H2, sig[:2], q_out=q)
    torch.cuda.synchronize()
    assert int(q.item()) == 1


# ---------------------------------------------------------------------------
# a6 / a8: CDP
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n", [100, 2000, 5000])
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_jacobi_parity(dev, n, dtype):
    if dtype == torch.float64 and n == 5000:
        pytest.skip("covered by the FP32 case")
    _, G32, b32, _ = problem(30 + n, n)
    sigma = W.random_support(3, n, 0.1)
    R0 = f32(W.random_r(7, n))
    Gd = t(G32, dtype, dev)
    Rg = t(R0, dtype, dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    L.l0cim_update_r(Gd, t(b32, dtype, dev), t(sigma, torch.uint8, dev), Rg, iters=100, status=status)
    torch.cuda.synchronize()
    Ro, st = O.cdp_jacobi(G32, b32, sigma, R0, 0.1, 100)
    assert int(status.item()) == st == 0
    tol = 1e-5 if dtype == torch.float32 else 1e-12
    assert normwise(Rg.double().cpu().numpy(), Ro) <= tol


@pytest.mark.parametrize("k", [0, 1, 255, 256, 257])
def test_jacobi_support_sizes_fp32(dev, k):
    """Supports around the one-workgroup limit (256 spins): both the support
    form and the resident form it hands over to agree with the sweeps."""
    n = 1200
    _, G32, b32, _ = problem(77, n)
    sigma = np.zeros(n, np.uint8)
    sigma[np.random.default_rng(k).choice(n, k, replace=False)] = 1
    R0 = f32(W.random_r(8, n))
    Rg = t(R0, torch.float32, dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    L.l0cim_update_r(t(G32, torch.float32, dev), t(b32, torch.float32, dev), t(sigma, torch.uint8, dev), Rg,
                     iters=100, status=status)
    torch.cuda.synchronize()
    Ro, st = O.cdp_jacobi(G32, b32, sigma, R0, 0.1, 100)
    assert int(status.item()) == st == 0
    assert normwise(Rg.double().cpu().numpy(), Ro) <= 1e-5


@pytest.mark.parametrize("density", [0.1, 1.0])
def test_jacobi_large_n_fp64(dev, density):
    """N = 4500 in FP64 (G too large for the resident form): a 10% support
    runs the large-N support form, a full support (above its 4096 limit)
    the streamed sweeps it hands over to."""
    n = 4500
    _, G32, b32, _ = problem(91, n)
    sigma = (np.random.default_rng(5).random(n) < density).astype(np.uint8)
    R0 = f32(W.random_r(9, n))
    Rg = t(R0, torch.float64, dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    L.l0cim_update_r(t(G32, torch.float64, dev), t(b32, torch.float64, dev), t(sigma, torch.uint8, dev), Rg,
                     iters=100, status=status)
    torch.cuda.synchronize()
    Ro, st = O.cdp_jacobi(G32, b32, sigma, R0, 0.1, 100)
    assert int(status.item()) == st == 0
    assert normwise(Rg.cpu().numpy(), Ro) <= 1e-12


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_jacobi_tiny_diagonal(dev, dtype):
    n = 64
    inst = W.gaussian_instance(8, n, 40, 0.2, 0.01)
    A = inst.A.copy()
    A[:, 5] = 0.0
    G, b = O.gram(A, inst.y)
    if dtype == torch.float32:
        G, b = f32(G), f32(b)
    sigma = np.ones(n, np.uint8)
    sigma[::3] = 0
    R = t(np.ones(n), dtype, dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    L.l0cim_update_r(t(G, dtype, dev), t(b, dtype, dev), t(sigma, torch.uint8, dev), R,
                     iters=10, status=status)
    torch.cuda.synchronize()
    Ro, st = O.cdp_jacobi(G, b, sigma, np.ones(n), 0.1, 10)
    assert int(status.item()) == st == L.ST_TINY_DIAG
    assert R[5].item() == 0.0
    if dtype == torch.float64:
        np.testing.assert_allclose(R.cpu().numpy(), Ro, rtol=1e-12, atol=1e-14)
    else:
        assert normwise(R.double().cpu().numpy(), Ro) <= 1e-5


@pytest.mark.parametrize("n,m,density", [(300, 200, 0.1), (64, 32, 0.1), (500, 400, 0.3)])
def test_cholesky_refit_parity(dev, n, m, density):
    inst = W.gaussian_instance(9 + n, n, m, density, 0.01)
    G, b = O.gram(inst.A, inst.y)
    sigma = inst.xi
    R = torch.zeros(n, dtype=torch.float64, device=dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    L.l0cim_update_r(t(G, torch.float64, dev), t(b, torch.float64, dev), t(sigma, torch.uint8, dev), R,
                     cdp=L.CDP_CHOL_F64, status=status)
    torch.cuda.synchronize()
    Ro, st = O.chol_refit(G, b, sigma)
    assert int(status.item()) == st
    assert normwise(R.cpu().numpy(), Ro) <= 1e-10
    # FP32 inputs, FP64 factorisation
    G32, b32 = f32(G), f32(b)
    R32 = torch.zeros(n, dtype=torch.float32, device=dev)
    L.l0cim_update_r(t(G32, torch.float32, dev), t(b32, torch.float32, dev), t(sigma, torch.uint8, dev),
                     R32, cdp=L.CDP_CHOL_F64)
    torch.cuda.synchronize()
    Ro32, _ = O.chol_refit(G32, b32, sigma)
    assert normwise(R32.double().cpu().numpy(), Ro32) <= 1e-6


@pytest.mark.parametrize("n,m,density", [(3000, 2600, 0.5), (2000, 1800, 0.04)])
def test_cholesky_refit_parity_large_support(dev, n, m, density):
    """Supports of ~1500 and ~80 spins: several 64 x 64 blocks and a ragged
    last block, FP64 throughout."""
    inst = W.gaussian_instance(500 + n, n, m, density, 0.01)
    G, b = O.gram(inst.A, inst.y)
    sigma = inst.xi
    R = torch.zeros(n, dtype=torch.float64, device=dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    L.l0cim_update_r(t(G, torch.float64, dev), t(b, torch.float64, dev), t(sigma, torch.uint8, dev), R,
                     cdp=L.CDP_CHOL_F64, status=status)
    torch.cuda.synchronize()
    Ro, st = O.chol_refit(G, b, sigma)
    assert int(status.item()) == st == 0
    assert normwise(R.cpu().numpy(), Ro) <= 1e-9


def _refit_a(dev, A, y, sigma, dtype):
    R = torch.zeros(A.shape[1], dtype=dtype, device=dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    L.l0cim_refit_f64(t(A, dtype, dev), t(y, dtype, dev), t(sigma, torch.uint8, dev), R, status=status)
    torch.cuda.synchronize()
    return R.double().cpu().numpy(), int(status.item())


@pytest.mark.parametrize("n,m,density", [(300, 200, 0.1), (64, 32, 0.1), (500, 400, 0.3), (3000, 2600, 0.5),
                                         (10, 5000, 0.5), (200, 100, 0.0)])
def test_refit_f64_from_a_parity(dev, n, m, density):
    """G_SS, b_S and the off-support rows from A in FP64 against the oracle's
    refit on the Gram of the same A: FP64 inputs at 1e-10; FP32 inputs against
    the oracle on the FP32-rounded A, bounded by the FP32 rounding of R.
    Covers several 64-blocks with a ragged last one (|S| ~ 1500), m far above
    the padded factor (n = 10, m = 5000) and the empty support."""
    inst = W.gaussian_instance(900 + n, n, m, density, 0.01)
    sigma = inst.xi
    G, b = O.gram(inst.A, inst.y)
    Ro, st = O.chol_refit(G, b, sigma)
    R, status = _refit_a(dev, inst.A, inst.y, sigma, torch.float64)
    assert status == st
    assert normwise(R, Ro) <= 1e-10
    A32, y32 = f32(inst.A), f32(inst.y)
    G32, b32 = O.gram(A32, y32)
    Ro32, _ = O.chol_refit(G32, b32, sigma)
    R32, _ = _refit_a(dev, A32, y32, sigma, torch.float32)
    assert np.all(np.abs(R32 - Ro32) <= 2 ** -24 * np.abs(Ro32) + 1e-12 * np.max(np.abs(Ro32)))


def test_refit_f64_from_a_ridge_and_tiny_column(dev):
    """A rank-deficient support (10 columns, 6 rows) takes the ridge branch on
    both sides; an all-zero column is held at 0 with the tiny-diagonal bit."""
    inst = W.gaussian_instance(14, 20, 6, 0.5, 0.0)
    A = inst.A.copy()
    A[:, 15] = 0.0
    sigma = np.zeros(20, np.uint8)
    sigma[:10] = 1
    G, b = O.gram(A, inst.y)
    Ro, st = O.chol_refit(G, b, sigma)
    R, status = _refit_a(dev, A, inst.y, sigma, torch.float64)
    assert st & O.ST_CHOL_RIDGE and st & O.ST_TINY_DIAG and status == st
    assert R[15] == 0.0
    res_g = A @ (sigma * R) - inst.y
    res_o = A @ (sigma * Ro) - inst.y
    assert abs(np.linalg.norm(res_g) - np.linalg.norm(res_o)) < 1e-6


def test_cholesky_refit_ridge_on_singular_support(dev):
    inst = W.gaussian_instance(14, 20, 6, 0.5, 0.0)
    G, b = O.gram(inst.A, inst.y)
    sigma = np.zeros(20, np.uint8)
    sigma[:10] = 1
    R = torch.zeros(20, dtype=torch.float64, device=dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    L.l0cim_update_r(t(G, torch.float64, dev), t(b, torch.float64, dev), t(sigma, torch.uint8, dev), R,
                     cdp=L.CDP_CHOL_F64, status=status)
    torch.cuda.synchronize()
    Ro, st = O.chol_refit(G, b, sigma)
    assert st & O.ST_CHOL_RIDGE and int(status.item()) & L.ST_CHOL_RIDGE
    assert np.all(np.isfinite(R.cpu().numpy()))
    # the ridge solution is ill-determined; check the fit it produces instead
    res_g = inst.A @ (sigma * R.cpu().numpy()) - inst.y
    res_o = inst.A @ (sigma * Ro) - inst.y
    assert abs(np.linalg.norm(res_g) - np.linalg.norm(res_o)) < 1e-6


# ---------------------------------------------------------------------------
# Algorithm 1 end to end against the oracle's stored supports
# ---------------------------------------------------------------------------

def _golden(name):
    out = {}
    for line in open(os.path.join(GOLDEN, f"oracle_supports_{name}.txt")):
        if not line.strip() or line[0] == "#":
            continue
        seed, k, rm, hx = line.split()
        out[int(seed)] = (int(k), float(rm), int(hx, 16))
    return out


def _mask(bits, n):
    return np.array([(bits >> r) & 1 for r in range(n)], np.uint8)


def test_solve_small_fp64_matches_oracle_supports(dev):
    """N = 64, M = 32, fixed eta = 0.18, 1000 steps x 50 alternations, FP64,
    every stored seed (0-199): identical supports."""
    gold = _golden("small")
    seeds = sorted(gold)
    assert len(seeds) == 200
    cim = L.cim_params(n_steps=1000)
    agree = 0
    for s in seeds:
        inst = W.small_gaussian(s)
        sp = L.solve_params(eta_init=0.18, eta_end=0.18, velo=50, n_outer=50, seed=s, j_dtype=L.F64)
        R, sig, stats = L.l0cim_solve(t(inst.A, torch.float64, dev), t(inst.y, torch.float64, dev), cim, sp)
        torch.cuda.synchronize()
        agree += int(np.array_equal(sig.cpu().numpy(), _mask(gold[s][2], 64)))
        st = L.read_stats(stats)
        assert st.status_bits == 0 and st.spin_steps == 64 * 1000 * 50
    assert agree == len(seeds)


def test_solve_plain_fp32_matches_oracle_supports(dev):
    """N = 2000, M = 1000, eta 0.8 -> 0.18 over 30 alternations of 2000 steps,
    FP32: identical support on >= 99% of seeds, RMSE within 1e-3."""
    gold = _golden("plain")
    seeds = sorted(gold)
    assert len(seeds) >= 10
    cim = L.cim_params(n_steps=2000)
    agree, worst = 0, 0.0
    for s in seeds:
        inst = W.plain_gaussian(s)
        sp = L.solve_params(eta_init=0.8, eta_end=0.18, velo=30, n_outer=30, seed=s)
        R, sig, stats = L.l0cim_solve(t(inst.A, torch.float32, dev), t(inst.y, torch.float32, dev), cim, sp)
        torch.cuda.synchronize()
        sg = sig.cpu().numpy()
        agree += int(np.array_equal(sg, _mask(gold[s][2], 2000)))
        rm = O.rmse(sg, R.double().cpu().numpy(), inst.x, inst.xi)
        worst = max(worst, abs(rm - gold[s][1]))
        assert L.read_stats(stats).status_bits == 0
    assert agree >= math.ceil(0.99 * len(seeds)), f"{agree}/{len(seeds)} supports identical"
    assert worst <= 1e-3
