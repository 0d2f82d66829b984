"""Tune m0 of the synthetic Wilson workloads so that the smallest |eigenvalue|
of D is about 1e-2 (shift steps on m0; eigenvalues from shift-invert Arnoldi
of the CPU oracle's operator).  Writes workloads/wilson_mass.json.

Run:  python workloads/tune_wilson_mass.py 256 512:-0.1876
"""
import json
import os
import sys

import numpy as np
import scipy.sparse.linalg as spla

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

from oracle.operators import wilson2d  # noqa: E402
from workloads.generate import gauge_field  # noqa: E402

TARGET = 1e-2


def smallest_eig(D):
    """Eigenvalue of smallest modulus: Arnoldi on D^-1 (sparse LU, minimum-degree
    ordering of the symmetric pattern), largest-modulus eigenvalues inverted."""
    lu = spla.splu(D.tocsc(), permc_spec="MMD_AT_PLUS_A")
    op = spla.LinearOperator(D.shape, matvec=lu.solve, dtype=np.complex128)
    vals = 1.0 / spla.eigs(op, k=4, which="LM", return_eigenvectors=False, tol=1e-8, ncv=40)
    return vals[np.argmin(np.abs(vals))]


def tune(N, sigma=0.5, seed=1, max_steps=8, start=None):
    """m0 at which the smallest-modulus eigenvalue of D has modulus TARGET (and a
    positive real part).  The mass only shifts the spectrum, D(m) = D(m') +
    (m - m') I, so each step moves m0 by TARGET - Re(lambda_min): exact when the
    same eigenvalue stays the one nearest to zero, a few steps otherwise.
    Starts from `start` (e.g. the value tuned on a smaller lattice of the same
    field distribution, where the eigenvalue nearest zero is well separated) or
    from the free field, where lambda_min = m0."""
    theta = gauge_field(N, sigma, seed)
    m = TARGET if start is None else float(start)
    lam = None
    for _ in range(max_steps):
        lam = smallest_eig(wilson2d(N, theta, m))
        print("N=%d m0=%.7f lambda_min=%s" % (N, m, lam), flush=True)
        if abs(abs(lam) / TARGET - 1.0) < 0.02 and lam.real > 0:
            return m, abs(lam)
        m += TARGET - lam.real
    raise RuntimeError("m0 tuning did not settle for N=%d" % N)


if __name__ == "__main__":
    path = os.path.join(HERE, "wilson_mass.json")
    table = json.load(open(path)) if os.path.exists(path) else {}
    for arg in sys.argv[1:]:
        # "N" or "N:start"
        N, _, start = arg.partition(":")
        N = int(N)
        m0, f = tune(N, start=float(start) if start else None)
        table[str(N)] = {"m0": m0, "min_abs_eig": f, "theta_sigma": 0.5, "gauge_seed": 1}
        with open(path, "w") as fh:
            json.dump(table, fh, indent=1)
        print("N=%d m0=%.6f" % (N, m0), flush=True)
