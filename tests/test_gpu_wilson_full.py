"""The 256 x 256 Wilson-like workload at full size and its launch width (128
right-hand sides): properties the oracle checks column by column.  A sparse
direct factorisation of the 131,072-unknown operator does not fit the test's
time, so the oracle instead (a) regenerates the Z4 probes bit for bit, (b)
builds its own test-vector hierarchy (same RNG start) and compares the
restriction, (c) recomputes every FP64 residual x - A y of the returned
solutions with its own operators, and (d) recomputes each sample's two
quadratic forms from those solutions."""
import numpy as np
import pytest

from oracle import hierarchy, philox
from tests.gpu_util import from_dev, require_gpu
from workloads import gauge_field, wilson_mass

pytestmark = pytest.mark.gpu

N, LEVELS, BLK, NVEC, SWEEPS, SEED, COUNT = 256, 3, 4, 8, 20, 5, 16


@pytest.fixture(scope="module")
def setup():
    require_gpu()
    import paper_2108_11281_amd as m
    m0 = wilson_mass(N)
    th = gauge_field(N, sigma=0.5, seed=1)
    est = m.TraceEstimator("wilson2d", N, LEVELS, LEVELS, mass=m0, field=th, block=BLK,
                           n_vec=NVEC, setup_sweeps=SWEEPS, setup_seed=1,
                           precision="fp32_ir64", nb=128, nu_pre=2, nu_post=2, solve_tol=1e-10)
    A, P = hierarchy.wilson_hierarchy(N, th, m0, LEVELS, block=BLK, n_vec=NVEC, sweeps=SWEEPS,
                                      seed=1)
    return est, A, P


def _rel_res(A, x, y):
    return np.linalg.norm(x - A @ y) / np.linalg.norm(x)


@pytest.mark.parametrize("level", [1, 2])
def test_full_size_solves_and_samples(setup, level):
    est, A, P = setup
    n = est.level_size(level)
    X = est.probes(level, SEED, 0, COUNT)
    x = from_dev(X, complex_=True)
    for k in range(COUNT):
        assert np.array_equal(x[k], philox.z4(n, SEED, k, level))
    Y, rel = est.solve(level, X)
    assert np.all(rel <= 1e-10), np.max(rel)
    y = from_dev(Y, complex_=True)
    Xc = est.restrict(level, X)
    xc = from_dev(Xc, complex_=True)
    R = P[level - 1].conj().T
    xc_ref = (R @ x.T).T
    assert np.max(np.abs(xc - xc_ref)) <= 1e-10 * np.max(np.abs(xc_ref))
    Z, relz = est.solve(level + 1, Xc)
    assert np.all(relz <= 1e-10)
    z = from_dev(Z, complex_=True)
    s = est.sample_level(level, SEED, 0, COUNT)
    for k in range(COUNT):
        # the oracle's own operators: FP64 residuals of the returned solutions
        assert _rel_res(A[level - 1], x[k], y[k]) <= 2e-10
        assert _rel_res(A[level], xc_ref[k], z[k]) <= 1e-8
        a, b = np.vdot(x[k], y[k]), np.vdot(xc_ref[k], z[k])
        assert abs(s[k] - (a - b)) <= 1e-8 * (abs(a) + abs(b)), k
    # gamma5-hermiticity makes every level difference real in expectation; the
    # per-sample imaginary parts are not zero, but their mean is within noise
    assert abs(np.mean(s.imag)) <= 5 * np.std(s.imag) / np.sqrt(COUNT) + 1e-12
