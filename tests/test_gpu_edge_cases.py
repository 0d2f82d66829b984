"""Smallest hierarchies of every operator kind (two levels, the coarsest a
handful of unknowns) with one-column batches, in both precisions: per-sample
values against the oracle and the estimator's result against the exact trace."""
import numpy as np
import pytest

from oracle import hierarchy, mlmc
from tests.gpu_util import quad_scale, require_gpu
from workloads import gauge_field, varcoef_faces

pytestmark = pytest.mark.gpu


def _check(est, orc, exact, complex_=False):
    s = est.sample_level(1, 17, 0, 3)
    ref = orc.sample(1, 17, 0, 3)
    scale = quad_scale(orc.sample_parts(1, 17, 0, 3))
    assert np.all(np.abs(s - ref) <= 1e-8 * scale), np.max(np.abs(s - ref) / scale)
    assert abs(est.coarse_trace() - orc.coarse()) <= 1e-9 * abs(orc.coarse())
    r = est.trace(5e-2, 3)
    assert abs(r["trace"] - exact) <= 5 * r["rmsd"] + 1e-9 * abs(exact)


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir64"])
@pytest.mark.parametrize("N", [2, 8])
def test_poisson_two_levels(precision, N):
    require_gpu()
    import paper_2108_11281_amd as m
    est = m.TraceEstimator("poisson2d", N, 2, 2, precision=precision, nb=1, solve_tol=1e-12)
    A, P = hierarchy.poisson_hierarchy(N, 2)
    orc = mlmc.LevelSampler(A, P, complex_probe=False)
    _check(est, orc, np.trace(np.linalg.inv(A[0].toarray())))


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir64"])
def test_varcoef_two_levels(precision):
    require_gpu()
    import paper_2108_11281_amd as m
    N = 4
    k = varcoef_faces(N, seed=1001)
    est = m.TraceEstimator("varcoef3d", N, 2, 2, shift=1e-3, field=k, precision=precision, nb=1,
                           solve_tol=1e-12)
    A, P = hierarchy.varcoef_hierarchy(N, k, 1e-3, 2)
    orc = mlmc.LevelSampler(A, P, complex_probe=False)
    _check(est, orc, np.trace(np.linalg.inv(A[0].toarray())))


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir64"])
@pytest.mark.parametrize("kind", ["wilson2d", "gauge2d"])
def test_lattice_two_levels(precision, kind):
    require_gpu()
    import paper_2108_11281_amd as m
    N, nv = 8, 2
    th = gauge_field(N, sigma=0.3, seed=4)
    mass = 0.2 if kind == "wilson2d" else 0.0
    est = m.TraceEstimator(kind, N, 2, 2, mass=mass, field=th, block=4, n_vec=nv,
                           setup_sweeps=4, setup_seed=1, precision=precision, nb=1,
                           solve_tol=1e-12)
    if kind == "wilson2d":
        A, P = hierarchy.wilson_hierarchy(N, th, mass, 2, block=4, n_vec=nv, sweeps=4, seed=1)
    else:
        A, P = hierarchy.gauge_hierarchy(N, th, mass, 2, block=4, n_vec=nv, sweeps=4, seed=1)
    orc = mlmc.LevelSampler(A, P, complex_probe=True)
    _check(est, orc, np.trace(np.linalg.inv(A[0].toarray())), complex_=True)
