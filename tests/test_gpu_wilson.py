"""GPU parity of the Wilson-like 2-spin operator path (test-vector aggregation,
block Gauss-Seidel V-cycle, flexible GMRES in FP64 refinement) against the CPU
oracle, through the C ABI."""
import numpy as np
import pytest

from oracle import hierarchy, mlmc, philox
from tests.gpu_util import from_dev, quad_scale, require_gpu, to_dev
from workloads import gauge_field

pytestmark = pytest.mark.gpu

N, LEVELS, BLK, NVEC, SWEEPS, M0 = 32, 3, 4, 8, 6, 0.1


@pytest.fixture(scope="module")
def oracle_h():
    th = gauge_field(N, seed=1)
    A, P = hierarchy.wilson_hierarchy(N, th, M0, LEVELS, block=BLK, n_vec=NVEC, sweeps=SWEEPS,
                                      seed=1)
    return th, A, P, mlmc.LevelSampler(A, P, complex_probe=True)


def _est(th, precision="fp64", nb=16, m0=M0, levels=LEVELS, **kw):
    require_gpu()
    import paper_2108_11281_amd as m
    kw.setdefault("solve_tol", 1e-12)
    kw.setdefault("nu_pre", 2)
    kw.setdefault("nu_post", 2)
    return m.TraceEstimator("wilson2d", N, levels, levels, mass=m0, field=th, block=BLK,
                            n_vec=NVEC, setup_sweeps=SWEEPS, setup_seed=1, precision=precision,
                            nb=nb, **kw)


def test_probes_z4_bit_exact(oracle_h):
    th = oracle_h[0]
    est = _est(th)
    for level in (1, 2):
        n = est.level_size(level)
        got = from_dev(est.probes(level, 99, 3, 5), complex_=True)
        for j in range(5):
            assert np.array_equal(got[j], philox.z4(n, 99, 3 + j, level))


def test_prolongation_matches_oracle(oracle_h):
    th, A, P, _ = oracle_h
    est = _est(th)
    for level in (1, 2):
        q = est.export_prolongation(level, NVEC)
        Pd = P[level - 1].toarray()
        # row i of q holds the coefficients of unknown i in its aggregate's basis
        n = q.shape[0]
        cols = Pd.shape[1]
        ref = np.zeros((n, NVEC), dtype=complex)
        for i in range(n):
            nz = np.nonzero(Pd[i])[0]
            assert len(nz) <= NVEC
            ref[i, :] = Pd[i, (nz[0] // NVEC) * NVEC:(nz[0] // NVEC) * NVEC + NVEC]
        assert cols % NVEC == 0
        assert np.max(np.abs(q - ref)) < 1e-10, np.max(np.abs(q - ref))


def test_operators_match_oracle(oracle_h):
    th, A, P, _ = oracle_h
    est = _est(th)
    rng = np.random.default_rng(3)
    for level in (1, 2, 3):
        n = est.level_size(level)
        X = rng.standard_normal((3, n)) + 1j * rng.standard_normal((3, n))
        Y = from_dev(est.apply(level, to_dev(X)), complex_=True)
        ref = (A[level - 1] @ X.T).T
        tol = 1e-13 if level == 1 else 1e-9
        assert np.max(np.abs(Y - ref)) <= tol * np.max(np.abs(ref)), level
        if level < 3:
            Xc = from_dev(est.restrict(level, to_dev(X)), complex_=True)
            refc = (P[level - 1].conj().T @ X.T).T
            assert np.max(np.abs(Xc - refc)) <= 1e-9 * np.max(np.abs(refc))
    Ad = est.export_coarse(0)
    assert np.max(np.abs(Ad - A[-1].toarray())) <= 1e-9 * np.max(np.abs(Ad))


def test_coarse_trace(oracle_h):
    th, A, P, orc = oracle_h
    est = _est(th)
    ref = orc.coarse()
    assert abs(est.coarse_trace() - ref) <= 1e-9 * abs(ref)


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir64"])
def test_solves_match_exact(precision, oracle_h):
    th, A, P, orc = oracle_h
    est = _est(th, precision=precision)
    rng = np.random.default_rng(5)
    for level in (1, 2, 3):
        n = est.level_size(level)
        B = rng.standard_normal((4, n)) + 1j * rng.standard_normal((4, n))
        Y, rel = est.solve(level, to_dev(B))
        assert np.all(rel <= 1e-12), rel
        ref = orc.solver(level).solve(B.T).T
        assert np.max(np.abs(from_dev(Y, complex_=True) - ref)) <= 1e-8 * np.max(np.abs(ref))


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir64"])
def test_samples_match_oracle(precision, oracle_h):
    th, A, P, orc = oracle_h
    est = _est(th, precision=precision, nb=16)
    for level, first, count in [(1, 0, 18), (2, 7, 5)]:
        s, err = est.sample_level(level, 21, first, count, with_error=True)
        ref = orc.sample(level, 21, first, count)
        scale = quad_scale(orc.sample_parts(level, 21, first, count))
        assert np.all(np.abs(s - ref) <= 1e-8 * scale), np.max(np.abs(s - ref) / scale)
        assert np.all(err <= 1e-8)


def test_mlmc_trace_matches_oracle_driver(oracle_h):
    th, A, P, orc = oracle_h
    est = _est(th, precision="fp32_ir64", nb=32)
    got = est.trace(2e-2, 4)
    ref = mlmc.mlmc_trace(orc, 2e-2, 4, nb=32)
    assert got["n_samples"] == ref["n_samples"]
    assert abs(got["trace"] - ref["trace"]) <= 1e-8 * abs(ref["trace"])
    exact = np.trace(np.linalg.inv(A[0].toarray()))
    assert abs(got["trace"] - exact) <= 4 * got["rmsd"]
    # eigenvalues in conjugate pairs: the exact trace is real
    assert abs(exact.imag) < 1e-10 * abs(exact.real)


def test_near_critical_mass_converges():
    from workloads import wilson_mass
    m0 = wilson_mass(N)
    if m0 is None:
        pytest.skip("tuned mass table missing")
    th = gauge_field(N, seed=1)
    est = _est(th, precision="fp32_ir64", nb=8, m0=m0, solve_tol=1e-10)
    rng = np.random.default_rng(8)
    B = rng.standard_normal((8, est.level_size(1))) + 1j * rng.standard_normal((8, est.level_size(1)))
    Y, rel = est.solve(1, to_dev(B))
    assert np.all(rel <= 1e-10)
