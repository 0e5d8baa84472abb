"""The CIM run that allocates nothing (l0cim_mfcim_run_noalloc) against the
run on a caller workspace (l0cim_mfcim_run), through the C ABI.

Both take the same launch form for these problems (the register-resident
single-replica run, the LDS-resident multi-workgroup run, the one-workgroup
run), so c, e, sigma, the eq. 4 energies and the 200-step trace must be
bitwise equal.  Two no-alloc calls in a row share the library's scratch; the
second is the smaller one, so a stale exchange word or abort word left by the
first would show.  Sizes beyond the scratch are refused on the host.
"""
import numpy as np
import pytest
import torch

import paper_2405_00366_amd as L
import workloads as W
from oracle import mfcim as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    return torch.device("cuda:0")


def _problem(seed, n, dtype, dev):
    inst = W.gaussian_instance(seed, n, n // 2, 0.1, 0.01).rounded_f32()
    G, b = O.gram(inst.A, inst.y)
    R = b / np.diag(G)
    J, z = O.couplings(G, b, R)
    return (torch.tensor(J, dtype=dtype, device=dev), torch.tensor(z, dtype=dtype, device=dev))


def _run(fn, J, z, c0, prm, eta, steps, dev, **kw):
    c = c0.clone()
    e = torch.ones_like(c)
    P, n = c.shape
    sigma = torch.empty((P, n), dtype=torch.uint8, device=dev)
    H = torch.empty(P, dtype=torch.float64, device=dev)
    tr = torch.empty((steps, 2, P, n), dtype=c.dtype, device=dev)
    st = torch.zeros(1, dtype=torch.int32, device=dev)
    fn(J, z, eta, prm, c, e, sigma=sigma, H=H, trace=tr, trace_steps=steps, status=st, **kw)
    torch.cuda.synchronize()
    return [x.cpu() for x in (c, e, sigma, H, tr, st)]


CASES = [  # (seed, n, P, field, dtype, steps): register-resident, LDS-resident, one workgroup (FP64)
    (3, 2000, 1, "CN", torch.float32, 300),
    (4, 700, 2, "BN", torch.float32, 200),
    (5, 200, 3, "CN", torch.float64, 200),
]


def test_noalloc_run_equals_workspace_run_two_calls(dev):
    for seed, n, P, field, dtype, steps in CASES:
        print(f"no-alloc case seed={seed} n={n} P={P} field={field} dtype={dtype}", flush=True)
        J, z = _problem(seed, n, dtype, dev)
        c0 = torch.tensor(W.initial_amplitudes(seed, P, n), dtype=dtype, device=dev)
        prm = L.cim_params(n_steps=steps, field=field)
        ref = _run(L.l0cim_mfcim_run, J, z, c0, prm, 0.6, steps, dev)
        got = _run(L.l0cim_mfcim_run_noalloc, J, z, c0, prm, 0.6, steps, dev)
        for name, a, b in zip(("c", "e", "sigma", "H", "trace", "status"), ref, got):
            assert torch.equal(a, b), f"{name} differs (n={n}, P={P})"
        assert int(got[5].item()) == 0


def test_noalloc_refuses_what_does_not_fit(dev):
    lib = L.lib()
    assert lib.l0cim_noalloc_scratch_bytes() == 8 << 20
    n, P = 1 << 18, 8
    J = torch.empty((1, 1), dtype=torch.float32, device=dev)   # never read: the call is refused first
    c = torch.empty((1, 1), dtype=torch.float32, device=dev)
    prm = L.cim_params(n_steps=10)
    st = lib.l0cim_mfcim_run_noalloc(L.F32, n, P, L.F32, L._ptr(J), n, None, L._ptr(c), 0.5, L.ctypes.byref(prm),
                                     L._ptr(c), L._ptr(c), L._ptr(c), None, None, 0, None, None)
    assert st == 3 and "scratch" in lib.l0cim_last_error().decode()
    prm = L.cim_params(n_steps=10, launch=L.LAUNCH_MATRIX)
    st = lib.l0cim_mfcim_run_noalloc(L.F32, 64, 2, L.F32, L._ptr(J), 64, None, L._ptr(c), 0.5, L.ctypes.byref(prm),
                                     L._ptr(c), L._ptr(c), L._ptr(c), None, None, 0, None, None)
    assert st == 5
