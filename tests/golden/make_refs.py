"""Write the stored oracle reconstructions used by the GPU parity tests.

Calls only ``oracle`` (FP64 CPU reference) and ``synth`` (seeded inputs).
Each case feeds the oracle the float32-rounded sinogram the GPU receives.

    python tests/golden/make_refs.py            # all cases (several minutes)
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402

CASES = {
    # name: (workload, seed, Bregman iterations or None for the workload's own)
    "c2_fan_512_720_seed0": ("c2", 0, None),
    "c2_fan_512_180_seed0": ("c2_25", 0, None),
    "c5_fan_1024_2304_seed0_outer2": ("c5", 0, 2),
}


def make(name: str):
    wname, seed, n_outer = CASES[name]
    w = synth.workload(wname) if n_outer is None else synth.workload(wname, n_outer=n_outer)
    case = synth.make_case(w, seed)
    y32 = case["y"].astype(np.float32)
    g = oracle.Geom(w.geom)
    t = time.time()
    x, resid = oracle.solve(g, y32.astype(np.float64), w.lam, w.mu, w.n_outer, w.n_cg)
    dt = time.time() - t
    path = os.path.join(HERE, name + ".npz")
    np.savez_compressed(path, x=x.astype(np.float32), resid=resid, seconds=dt, threads=oracle.num_threads())
    print(f"{name}: {dt:.1f} s on {oracle.num_threads()} threads -> {path}", flush=True)


if __name__ == "__main__":
    oracle.build(force=False)
    for name in (sys.argv[1:] or CASES):
        make(name)
