"""l0cim_mri_solve_many (GPU, through the C ABI): Algorithm 1 on several
MRI-shaped instances in lock step, their factored CIM runs in one launch of
count x replicas workgroups and their LASSO starts and CDPs in one launch
each.  Every instance's result must equal, bit for bit, what l0cim_mri_solve
gives it alone (which the oracle tests pin): R, the support, and the stats.

Cases: three instances with their own operators (seeds 0-2, Jacobi CDP in
factored form, FP64 refit); two with the pipeline around the path (L2 term,
LASSO start, CG CDP); and two slices measured through one shared operator
(A and the mask passed once, stride 0).  Short runs (4 alternations of 300
steps, 64 replicas) keep the test quick; the kernels are those of the full
runs.
"""
import numpy as np
import pytest
import torch

import paper_2405_00366_amd as L

pytestmark = pytest.mark.gpu
N = 128 * 128


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def insts():
    from workloads import mri as WM
    return [WM.mri_instance(s) for s in range(3)]


def _mask(inst):
    m = np.zeros(N, np.uint8)
    m[inst.meta["freqs"]] = 1
    return m


def _t(x, dev, dt=torch.float32):
    return torch.tensor(np.asarray(x), dtype=dt, device=dev)


def _params(pipeline, seed=0):
    mp = (L.mri_params(gamma=1e-4, lasso_iters=50, lasso_lam1=3e-4, cdp=L.CDP_CG, cg_max_iter=2000, cg_tol=1e-5)
          if pipeline else L.mri_params())
    cim = L.cim_params(n_steps=300, field="BN", K=1.0, d=0.6)
    sp = L.solve_params(eta_init=0.8, eta_end=0.03, velo=4, n_outer=4, replicas=64, seed=seed,
                        final_refit_f64=0 if pipeline else 1)
    return mp, cim, sp


def _check_equal_to_singles(dev, A, y, masks, seeds, pipeline, shared=False):
    mp, cim, sp = _params(pipeline)
    L.l0cim_profile_begin()
    R, sig, stats = L.l0cim_mri_solve_many(mp, A, y, masks, seeds, cim, sp)
    torch.cuda.synchronize()
    _, launches = L.l0cim_profile_end()
    assert launches == sp.n_outer, "one factored CIM launch per alternation for all instances"
    many = L.read_stats_array(stats, len(seeds))
    for k, sd in enumerate(seeds):
        mp1, cim1, sp1 = _params(pipeline, sd)
        Ak = A if shared else A[k]
        mk = masks if shared else masks[k]
        R1, s1, st1 = L.l0cim_mri_solve(mp1, Ak, y[k].contiguous(), mk, cim1, sp1)
        torch.cuda.synchronize()
        one = L.read_stats(st1)
        assert torch.equal(s1, sig[k]), f"instance {k}: support differs"
        assert torch.equal(R1, R[k]), f"instance {k}: R differs"
        assert (one.status_bits, one.selected_replica, one.support_size) == (
            many[k].status_bits, many[k].selected_replica, many[k].support_size)
        assert one.H == many[k].H and one.E == many[k].E
        print(f"instance {k} (seed {sd}): |S| {int(s1.sum())}, status {one.status_bits}")


@pytest.mark.parametrize("pipeline,count", [(False, 3), (True, 2)])
def test_mri_solve_many_equals_single_solves(dev, insts, pipeline, count):
    use = insts[:count]
    A = _t(np.stack([i.A for i in use]), dev)
    y = _t(np.stack([i.y for i in use]), dev)
    masks = _t(np.stack([_mask(i) for i in use]), dev, torch.uint8)
    _check_equal_to_singles(dev, A, y, masks, [100 + k for k in range(count)], pipeline)


def test_mri_solve_many_shared_operator(dev, insts):
    """Two slices through one operator (seed 0's A and mask, stride 0): the
    second slice's measurements are A x of the seed-1 image's coefficients
    plus noise of the same level."""
    A0 = insts[0].A
    rng = np.random.default_rng(7)
    y1 = A0 @ insts[1].x + rng.standard_normal(A0.shape[0]) * insts[0].meta["nu"]
    A = _t(A0, dev)
    y = _t(np.stack([insts[0].y, y1]), dev)
    mask = _t(_mask(insts[0]), dev, torch.uint8)
    _check_equal_to_singles(dev, A, y, mask, [5, 6], False, shared=True)
