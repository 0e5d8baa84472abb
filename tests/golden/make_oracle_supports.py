"""Write the FP64 oracle's final supports for the seeded benchmark workloads.

Calls only ``oracle`` and ``workloads``: every stored value is the oracle's.
Usage:  python tests/golden/make_oracle_supports.py {small|plain} FIRST LAST [JOBS]

  small : N = 64,   M = 32,   fixed eta = 0.18, 1000 steps x 50 alternations,
          FP64 inputs.
  plain : N = 2000, M = 1000, eta 0.8 -> 0.18 over 30 alternations,
          2000 steps each, inputs rounded to FP32 (what the GPU receives).

Each output line:  seed  support_size  rmse  hex(support bitmask, spin r = bit r)
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


def one(args):
    name, seed = args
    w = WORKLOADS[name]
    inst = w["make"](seed)
    if w["f32"]:
        inst = inst.rounded_f32()
    t = time.perf_counter()
    res = O.solve(inst.A, inst.y, w["cim"], O.with_params(w["outer"], seed=seed), keep_history=False)
    dt = time.perf_counter() - t
    return seed, int(res.sigma.sum()), O.rmse(res.sigma, res.R, inst.x, inst.xi), bitmask_hex(res.sigma), dt


def main():
    name, first, last = sys.argv[1], int(sys.argv[2]), int(sys.argv[3])
    jobs = int(sys.argv[4]) if len(sys.argv) > 4 else 1
    out = os.path.join(HERE, f"oracle_supports_{name}.txt")
    done = set()
    if os.path.exists(out):
        done = {int(l.split()[0]) for l in open(out) if l.strip() and l[0] != "#"}
    todo = [(name, s) for s in range(first, last + 1) if s not in done]
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
