"""Expected values for the 256 x 256 Wilson-like 2-spin workload, computed by the
CPU oracle only (test-vector aggregation hierarchy built by the oracle itself,
sparse-direct solves, dense inverse of the coarsest level).

Workload: U(1) phases theta ~ N(0, 0.5^2) (gauge seed 1), m0 tuned so that the
smallest eigenvalue modulus is 1e-2, 3 levels of 4 x 4 aggregates carrying 8
test vectors (20 setup sweeps, setup seed 1), Z4 probes.  Written: 16 samples of
each level difference (Remark 4.3 form) with their two quadratic forms, and
tr(A_3^{-1}) (Remark 4.2).

Run from the repository root:  python tests/golden/make_wilson256.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import hierarchy, mlmc  # noqa: E402
from workloads import gauge_field  # noqa: E402
from workloads.generate import wilson_mass  # noqa: E402

N, LEVELS, BLOCK, NVEC, SWEEPS, SETUP_SEED = 256, 3, 4, 8, 20, 1
SEED, COUNT = 5, 16


def main():
    t0 = time.time()
    m0 = wilson_mass(N)
    theta = gauge_field(N, sigma=0.5, seed=1)
    A, P = hierarchy.wilson_hierarchy(N, theta, m0, LEVELS, block=BLOCK, n_vec=NVEC,
                                      sweeps=SWEEPS, seed=SETUP_SEED)
    print("hierarchy %.1fs" % (time.time() - t0), flush=True)
    smp = mlmc.LevelSampler(A, P, complex_probe=True)
    out = dict(N=N, levels=LEVELS, block=BLOCK, n_vec=NVEC, setup_sweeps=SWEEPS,
               setup_seed=SETUP_SEED, m0=m0, gauge_seed=1, theta_sigma=0.5, seed=SEED,
               samples={})
    for level in range(1, LEVELS):
        a, b = smp.sample_parts(level, SEED, 0, COUNT)
        s = a - b
        out["samples"][str(level)] = dict(
            s=[[float(v.real), float(v.imag)] for v in s],
            a=[[float(v.real), float(v.imag)] for v in a],
            b=[[float(v.real), float(v.imag)] for v in b])
        print("level %d done %.1fs" % (level, time.time() - t0), flush=True)
    ct = smp.coarse()
    out["coarse_trace"] = [float(ct.real), float(ct.imag)]
    with open(os.path.join(HERE, "wilson256_samples.json"), "w") as f:
        json.dump(out, f, indent=1)
    print("done %.1fs" % (time.time() - t0), flush=True)


if __name__ == "__main__":
    main()
