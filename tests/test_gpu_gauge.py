"""GPU parity of the gauge Laplacian path (Example 4.2: one unknown per site,
U(1) links, test-vector aggregation, block Gauss-Seidel V-cycle, FGMRES in
complex128 refinement) against the oracle, through the C ABI."""
import numpy as np
import pytest

from oracle import hierarchy, mlmc, philox
from tests.gpu_util import from_dev, quad_scale, require_gpu, to_dev
from workloads import gauge_field

pytestmark = pytest.mark.gpu

N, LEVELS, BLK, NVEC, SWEEPS, MASS, SIGMA = 32, 3, 4, 4, 6, 0.0, 0.3


@pytest.fixture(scope="module")
def oracle_h():
    th = gauge_field(N, sigma=SIGMA, seed=1)
    A, P = hierarchy.gauge_hierarchy(N, th, MASS, LEVELS, block=BLK, n_vec=NVEC, sweeps=SWEEPS,
                                     seed=1)
    return th, A, P, mlmc.LevelSampler(A, P, complex_probe=True)


def _est(th, precision="fp64", nb=16, **kw):
    require_gpu()
    import paper_2108_11281_amd as m
    kw.setdefault("solve_tol", 1e-12)
    return m.TraceEstimator("gauge2d", N, LEVELS, LEVELS, mass=MASS, field=th, block=BLK,
                            n_vec=NVEC, setup_sweeps=SWEEPS, setup_seed=1, precision=precision,
                            nb=nb, nu_pre=1, nu_post=1, **kw)


def test_probes_operators_and_prolongation(oracle_h):
    th, A, P, orc = oracle_h
    est = _est(th)
    assert [est.level_size(l) for l in (1, 2, 3)] == [N * N, 8 * 8 * NVEC, 2 * 2 * NVEC]
    for level in (1, 2):
        n = est.level_size(level)
        got = from_dev(est.probes(level, 99, 3, 4), complex_=True)
        for j in range(4):
            assert np.array_equal(got[j], philox.z4(n, 99, 3 + j, level))
    for level in (1, 2):
        q = est.export_prolongation(level, NVEC)
        Pd = P[level - 1].toarray()
        ref = np.zeros((q.shape[0], NVEC), dtype=complex)
        for i in range(q.shape[0]):
            S = np.nonzero(Pd[i])[0][0] // NVEC
            ref[i] = Pd[i, S * NVEC:(S + 1) * NVEC]
        assert np.max(np.abs(q - ref)) < 1e-10, np.max(np.abs(q - ref))
    rng = np.random.default_rng(3)
    for level in (1, 2, 3):
        n = est.level_size(level)
        X = rng.standard_normal((3, n)) + 1j * rng.standard_normal((3, n))
        Y = from_dev(est.apply(level, to_dev(X)), complex_=True)
        ref = (A[level - 1] @ X.T).T
        tol = 1e-14 if level == 1 else 1e-9
        assert np.max(np.abs(Y - ref)) <= tol * np.max(np.abs(ref)), level
    Ad = est.export_coarse(0)
    assert np.max(np.abs(Ad - A[-1].toarray())) <= 1e-9 * np.max(np.abs(Ad))
    assert abs(est.coarse_trace() - orc.coarse()) <= 1e-9 * abs(orc.coarse())


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir64"])
def test_sweeps_match_oracle(oracle_h, precision):
    th, A, _, _ = oracle_h
    est = _est(th, precision=precision)
    rng = np.random.default_rng(5)
    tol = 1e-13 if precision == "fp64" else 1e-5
    for level, dof, side in ((1, 1, N), (2, NVEC, N // BLK)):
        n = est.level_size(level)
        B = rng.standard_normal((4, n)) + 1j * rng.standard_normal((4, n))
        X = rng.standard_normal((4, n)) + 1j * rng.standard_normal((4, n))
        colour = np.repeat(hierarchy.site_coloring(side), dof)
        for rev in (False, True):
            got = from_dev(est.smooth(level, to_dev(B), to_dev(X), 2, rev), complex_=True)
            for k in range(4):
                ref = hierarchy.rbgs_sweeps(A[level - 1], B[k], X[k], colour, 2, rev)
                err = np.max(np.abs(got[k] - ref))
                assert err <= max(tol, 1e-9 if level > 1 else 0) * np.max(np.abs(ref)), (level,
                                                                                       rev, k)


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir64"])
def test_samples_match_oracle(oracle_h, precision):
    th, _, _, orc = oracle_h
    est = _est(th, precision=precision)
    for level, first, count in [(1, 0, 12), (2, 30, 6)]:
        s, err = est.sample_level(level, 9, first, count, with_error=True)
        ref = orc.sample(level, 9, first, count)
        scale = quad_scale(orc.sample_parts(level, 9, first, count))
        assert np.all(np.abs(s - ref) <= 1e-8 * scale), np.max(np.abs(s - ref) / scale)
        assert np.all(err <= 1e-8)


def test_trace_matches_oracle_driver_and_exact(oracle_h):
    th, A, _, orc = oracle_h
    est = _est(th, precision="fp32_ir64", nb=32, alloc="giles")
    got = est.trace(2e-2, 6)
    ref = mlmc.mlmc_trace(orc, 2e-2, 6, nb=32, alloc=mlmc.ALLOC_GILES)
    assert got["n_samples"] == ref["n_samples"]
    assert abs(got["trace"] - ref["trace"]) <= 1e-8 * abs(ref["trace"])
    exact = np.trace(np.linalg.inv(A[0].toarray()))
    assert abs(got["trace"] - exact) <= 4 * got["rmsd"]
