"""Write the FP64 oracle's final supports for the seeded benchmark workloads.

Calls only ``oracle`` and ``workloads``: every stored value is the oracle's.
Usage:  python tests/golden/make_oracle_supports.py {small|plain|mri} FIRST LAST [JOBS]

  small : N = 64,   M = 32,   fixed eta = 0.18, 1000 steps x 50 alternations,
          FP64 inputs.
  plain : N = 2000, M = 1000, eta 0.8 -> 0.18 over 30 alternations,
          2000 steps each, inputs rounded to FP32 (what the GPU receives).

  mri   : 128 x 128 synthetic phantom, 3-level Haar, 30% variable-density DCT-II
          rows (N = 16384, M = 4915), noise 1e-3, 64 replicas, K = 1, d = 0.6,
          eta 0.8 -> 0.03 over 11 alternations of 1000 steps, binarised field,
          FP64 couplings applied in factored form, FP64 refit.

  mri_f32in : the mri workload with A and y rounded to FP32 before the oracle
          sees them (the device's inputs), to measure how far input rounding
          alone moves the oracle's own final support.

  mri_l2 : the MRI pipeline around the path on the same phantom instances:
          couplings from G_gamma = A^T A + gamma Psi (D_v^T D_v + D_h^T D_h) Psi^T
          (eq. 20, gamma = 1e-4, reflecting second differences), R_init from
          the LASSO (FISTA, lam1 = 3e-4, 200 iterations), CG CDP (at most 10^4
          iterations, relative residual 1e-5); 64 replicas, K = 1, d = 0.6,
          eta 0.8 -> 0.03 over 11 alternations of 1000 steps, binarised field;
          RMSE of the last CG solution on the final support.

  batched : 16 of the 256 instances of the batched workload (batch seed 7: N
          log-uniform in [256, 4096], alpha U[0.3, 0.7], sparsity U[0.05, 0.2],
          noise 0.01), instances 0, 16, ..., 240; 16 replicas, eta 0.8 -> 0.18
          over 30 alternations of 1000 steps, inputs rounded to FP32.
          FIRST/LAST index the sample (0..15); the key is the instance index.
  serving : 50 of the first 200 requests of the serving stream (stream seed 0:
          N log-uniform in [512, 8192], alpha U[0.2, 0.6], sparsity U[0.05,
          0.2], noise 0.01), requests 0, 4, ..., 196; 8 replicas, eta 0.8 ->
          0.18 over 30 alternations of 1000 steps, inputs rounded to FP32.
          FIRST/LAST index the sample (0..49); the key is the request index.

  cac   : the CAC-CIM (Positive-P, eq. 5-11) as the sigma-minimiser at the
          plain shape (N = 2000, M = 1000, inputs rounded to FP32), default
          CAC parameters, 8 replicas, eta 0.8 -> 0.18 over 30 alternations of
          1000 steps, Jacobi CDP, no refit.

  prec_f64 | prec_bf16 | prec_fp8 : the precision-form study at the plain
          shape (N = 2000, M = 1000, Bernoulli(0.1), noise 0.01, inputs rounded
          to FP32), 16 replicas, eta 0.8 -> 0.18 over 30 alternations of 1000
          steps, final FP64 refit; the CIM runs on the exact couplings
          (prec_f64) or on the couplings as BF16 / FP8 e4m3 rows with per-row
          scales represent them (oracle solve with j_format), so that a
          device-vs-oracle difference can be told apart from the change the
          narrow couplings make to the method.  Key = seed.

Each output line:  key  support_size  rmse  hex(support bitmask, spin r = bit r)
(key = seed for small / plain / mri, the instance or request index otherwise)

Usage:  python tests/golden/make_oracle_supports.py mri-refit
  writes oracle_refit_mri.txt: for every seed of oracle_supports_mri.txt, the
  oracle's final FP64 refit on its stored support (the R of its x_hat = sigma R),
  one line per seed:  seed  support_size  R_S in increasing spin order.
"""
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402
from oracle import mfcim as O  # noqa: E402

WORKLOADS = {
    "small": dict(make=W.small_gaussian, f32=False,
                  cim=O.CimParams(n_steps=1000),
                  outer=O.OuterParams(eta_init=0.18, eta_end=0.18, velo=50, n_outer=50)),
    "plain": dict(make=W.plain_gaussian, f32=True,
                  cim=O.CimParams(n_steps=2000),
                  outer=O.OuterParams(eta_init=0.8, eta_end=0.18, velo=30, n_outer=30)),
}


def bitmask_hex(sigma) -> str:
    v = 0
    for r in np.flatnonzero(sigma):
        v |= 1 << int(r)
    return format(v, "x")


MRI_CIM = O.CimParams(n_steps=1000, field=O.BN, K=1.0, d=0.6)
MRI_OUTER = O.OuterParams(eta_init=0.8, eta_end=0.03, velo=11, n_outer=11, replicas=64)


def one_mri(seed, f32_inputs=False):
    from oracle import mri as OM
    from workloads import mri as WM
    inst = WM.mri_instance(seed)
    if f32_inputs:
        inst = inst.rounded_f32()
    op = OM.MriOperator(128, inst.meta["freqs"], A=inst.A)
    t = time.perf_counter()
    sigma, R, hist = OM.solve(op, inst.y, MRI_CIM, O.with_params(MRI_OUTER, seed=seed),
                              progress=lambda i, h: print(f"  seed {seed} alternation {i}: {h}", flush=True))
    S, R_S, _st = OM.refit(inst.A, inst.y, sigma)
    Rf = np.zeros(op.N)
    Rf[S] = R_S
    dt = time.perf_counter() - t
    return seed, int(sigma.sum()), O.rmse(sigma, Rf, inst.x, inst.xi), bitmask_hex(sigma), dt


MRI_L2 = dict(gamma=1e-4, lam1=3e-4, lasso_iters=200, cg_max_iter=10000, cg_tol=1e-5)


def one_mri_l2(seed):
    from oracle import mri as OM
    from oracle import mri_l2 as L2
    from workloads import mri as WM
    inst = WM.mri_instance(seed)
    hop = L2.L2Operator(OM.MriOperator(128, inst.meta["freqs"], A=inst.A), MRI_L2["gamma"])
    t = time.perf_counter()
    sigma, R, hist = L2.solve(hop, inst.y, MRI_CIM, O.with_params(MRI_OUTER, seed=seed), MRI_L2["lam1"],
                              MRI_L2["lasso_iters"], MRI_L2["cg_max_iter"], MRI_L2["cg_tol"],
                              progress=lambda i, h: print(f"  seed {seed} alternation {i}: {h}", flush=True))
    dt = time.perf_counter() - t
    return seed, int(sigma.sum()), O.rmse(sigma, R, inst.x, inst.xi), bitmask_hex(sigma), dt


BATCH_SEED, BATCH_COUNT, BATCH_SAMPLE = 7, 256, list(range(0, 256, 16))
SERVE_SEED, SERVE_COUNT, SERVE_SAMPLE = 0, 200, list(range(0, 200, 4))
PREC_CIM = O.CimParams(n_steps=1000)
PREC_OUTER = O.OuterParams(eta_init=0.8, eta_end=0.18, velo=30, n_outer=30, replicas=16, refit=True)
PREC_FORMATS = {"prec_f64": None, "prec_bf16": "bf16", "prec_fp8": "fp8"}


def one_prec(name, seed):
    inst = W.plain_gaussian(seed).rounded_f32()
    t = time.perf_counter()
    res = O.solve(inst.A, inst.y, PREC_CIM, O.with_params(PREC_OUTER, seed=seed), keep_history=False,
                  j_format=PREC_FORMATS[name])
    dt = time.perf_counter() - t
    return seed, int(res.sigma.sum()), O.rmse(res.sigma, res.R, inst.x, inst.xi), bitmask_hex(res.sigma), dt


MULTI = {
    "batched": dict(specs=lambda: W.batch_specs(BATCH_SEED, BATCH_COUNT), sample=BATCH_SAMPLE, replicas=16),
    "serving": dict(specs=lambda: W.serving_specs(SERVE_SEED, SERVE_COUNT), sample=SERVE_SAMPLE, replicas=8),
}


def one_multi(name, key):
    """One sampled instance of the batched or serving workload: FP32-rounded
    inputs, 16 (batched) or 8 (serving) replicas keyed by the instance's
    seed, 1000 steps x 30 alternations, eta 0.8 -> 0.18 (velo 30)."""
    w = MULTI[name]
    spec = w["specs"]()[key]
    inst = spec.build().rounded_f32()
    cim = O.CimParams(n_steps=1000)
    outer = O.OuterParams(eta_init=0.8, eta_end=0.18, velo=30, n_outer=30, replicas=w["replicas"], seed=spec.seed)
    t = time.perf_counter()
    res = O.solve(inst.A, inst.y, cim, outer, keep_history=False)
    dt = time.perf_counter() - t
    return key, int(res.sigma.sum()), O.rmse(res.sigma, res.R, inst.x, inst.xi), bitmask_hex(res.sigma), dt


CAC_OUTER = O.OuterParams(eta_init=0.8, eta_end=0.18, velo=30, n_outer=30, replicas=8)


def one_cac(seed):
    from oracle import cac as C
    inst = W.plain_gaussian(seed).rounded_f32()
    t = time.perf_counter()
    res = C.solve(inst.A, inst.y, C.CacParams(n_steps=1000), O.with_params(CAC_OUTER, seed=seed), keep_history=False)
    dt = time.perf_counter() - t
    return seed, int(res.sigma.sum()), O.rmse(res.sigma, res.R, inst.x, inst.xi), bitmask_hex(res.sigma), dt


def one(args):
    name, seed = args
    if name == "cac":
        return one_cac(seed)
    if name == "mri":
        return one_mri(seed)
    if name == "mri_f32in":
        return one_mri(seed, f32_inputs=True)
    if name == "mri_l2":
        return one_mri_l2(seed)
    if name in PREC_FORMATS:
        return one_prec(name, seed)
    if name in MULTI:
        return one_multi(name, seed)
    w = WORKLOADS[name]
    inst = w["make"](seed)
    if w["f32"]:
        inst = inst.rounded_f32()
    t = time.perf_counter()
    res = O.solve(inst.A, inst.y, w["cim"], O.with_params(w["outer"], seed=seed), keep_history=False)
    dt = time.perf_counter() - t
    return seed, int(res.sigma.sum()), O.rmse(res.sigma, res.R, inst.x, inst.xi), bitmask_hex(res.sigma), dt


def mri_refit():
    from oracle import mri as OM
    from workloads import mri as WM
    src = os.path.join(HERE, "oracle_supports_mri.txt")
    out = os.path.join(HERE, "oracle_refit_mri.txt")
    with open(out, "w") as f:
        f.write("# FP64 oracle final refit on its stored MRI-shaped supports (see make_oracle_supports.py)\n")
        f.write("# seed support_size R_S (spins in increasing order)\n")
        for line in open(src):
            if not line.strip() or line[0] == "#":
                continue
            seed, k, _rm, hx = line.split()
            inst = WM.mri_instance(int(seed))
            v = int(hx, 16)
            sigma = np.array([(v >> r) & 1 for r in range(inst.A.shape[1])], np.uint8)
            assert int(sigma.sum()) == int(k)
            S, R_S, _st = OM.refit(inst.A, inst.y, sigma)
            f.write(f"{seed} {len(S)} " + " ".join(f"{x:.12e}" for x in R_S) + "\n")
            print(f"seed {seed}: |S| = {len(S)}", flush=True)


def main():
    if sys.argv[1] == "mri-refit":
        mri_refit()
        return
    name, first, last = sys.argv[1], int(sys.argv[2]), int(sys.argv[3])
    jobs = int(sys.argv[4]) if len(sys.argv) > 4 else 1
    out = os.path.join(HERE, f"oracle_supports_{name}.txt")
    done = set()
    if os.path.exists(out):
        done = {int(l.split()[0]) for l in open(out) if l.strip() and l[0] != "#"}
    if name in MULTI:
        keys = MULTI[name]["sample"][first:last + 1]
        specs = MULTI[name]["specs"]()
        keys = sorted(keys, key=lambda k: -specs[k].N)     # largest first: the pool drains evenly
    else:
        keys = list(range(first, last + 1))
    todo = [(name, s) for s in keys if s not in done]
    if not os.path.exists(out):
        with open(out, "w") as f:
            f.write(f"# FP64 oracle final supports, workload '{name}' (see make_oracle_supports.py)\n")
            f.write("# seed support_size rmse_vs_truth support_bitmask_hex\n")
    with ProcessPoolExecutor(jobs) as ex:
        for seed, k, rm, hx, dt in ex.map(one, todo):
            with open(out, "a") as f:
                f.write(f"{seed} {k} {rm:.9e} {hx}\n")
            print(f"seed {seed}: |S|={k} rmse={rm:.4g} ({dt:.1f} s)", flush=True)


if __name__ == "__main__":
    main()
