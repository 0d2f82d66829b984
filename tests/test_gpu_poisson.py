"""GPU parity of the 2D Poisson path against the CPU oracle (through the C ABI)."""
import numpy as np
import pytest

from oracle import hierarchy, mlmc, operators, philox
from tests.gpu_util import from_dev, quad_scale, require_gpu, to_dev

pytestmark = pytest.mark.gpu


def _est(N, L, **kw):
    require_gpu()
    import paper_2108_11281_amd as m
    kw.setdefault("nb", 32)
    kw.setdefault("solve_tol", 1e-12)
    return m.TraceEstimator("poisson2d", N, L, L, **kw)


@pytest.fixture(scope="module")
def c0_oracle():
    A, P = hierarchy.poisson_hierarchy(64, 3)
    return mlmc.LevelSampler(A, P, complex_probe=False)


@pytest.mark.parametrize("level,first,count", [(1, 0, 3), (2, 5, 33), (3, 2**33 + 1, 2)])
def test_probes_bit_exact(level, first, count):
    est = _est(64, 3)
    n = est.level_size(level)
    for stream in (0, 1, 3):
        got = from_dev(est.probes(level, 1234567, first, count, stream))
        for j in range(count):
            ref = philox.rademacher(n, 1234567, first + j, level, stream)
            assert np.array_equal(got[j], ref), (stream, j)


@pytest.mark.parametrize("N,L", [(64, 3), (20, 2), (96, 4)])
def test_apply_restrict_prolong(N, L):
    est = _est(N, L)
    A, P = hierarchy.poisson_hierarchy(N, L)
    rng = np.random.default_rng(1)
    for l in range(1, L + 1):
        X = rng.standard_normal((5, A[l - 1].shape[0]))
        Y = from_dev(est.apply(l, to_dev(X)))
        ref = (A[l - 1] @ X.T).T
        assert np.max(np.abs(Y - ref)) <= 1e-14 * np.max(np.abs(ref))
        if l < L:
            Xc = from_dev(est.restrict(l, to_dev(X)))
            assert np.max(np.abs(Xc - (P[l - 1].T @ X.T).T)) <= 1e-15 * np.max(np.abs(X)) * 2
            E = rng.standard_normal((3, A[l].shape[0]))
            Xf = from_dev(est.prolong(l, to_dev(E)))
            assert np.array_equal(Xf, (P[l - 1] @ E.T).T)


def test_coarse_operator_and_trace(c0_oracle):
    est = _est(64, 3)
    Ad = est.export_coarse(0)
    assert np.array_equal(Ad, c0_oracle.A[-1].toarray())
    ct = est.coarse_trace()
    ref = c0_oracle.coarse()
    assert abs(ct - ref) <= 1e-12 * abs(ref)
    # closed form 4 T(16) (Example 4.1 eigenvalues, A_3 = L^16/4)
    assert abs(ct.real - 4 * operators.poisson2d_trace_inverse(16)) < 1e-10 * abs(ref)


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir64"])
def test_solve_matches_exact(precision, c0_oracle):
    est = _est(64, 3, precision=precision)
    rng = np.random.default_rng(2)
    for l in (1, 2, 3):
        B = rng.standard_normal((7, est.level_size(l)))
        Y, rel = est.solve(l, to_dev(B))
        assert np.all(rel <= 1e-12)
        if l == 1:
            # the aggregation V-cycle (with its dense coarsest solve) is a good
            # preconditioner: a broken coarse solve or smoother shows up here
            iters, refine = est.counters()[:2]
            assert iters <= 60, (iters, refine)
        ref = c0_oracle.solver(l).solve(B.T).T
        assert np.max(np.abs(from_dev(Y) - ref)) <= 1e-9 * np.max(np.abs(ref))
    # right-hand sides of FP32 numbers (entries +-1/2, as the probes and their
    # restrictions): the FP32 refinement reads them from an exact FP32 copy,
    # the normal ones above through the FP64 path; both meet the exact solve
    for l in (1, 2):
        B = 0.5 * np.sign(rng.standard_normal((5, est.level_size(l))))
        Y, rel = est.solve(l, to_dev(B))
        assert np.all(rel <= 1e-12)
        ref = c0_oracle.solver(l).solve(B.T).T
        assert np.max(np.abs(from_dev(Y) - ref)) <= 1e-9 * np.max(np.abs(ref))


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir64"])
def test_samples_match_oracle(precision, c0_oracle):
    est = _est(64, 3, precision=precision, nb=32)
    for level, first, count in [(1, 0, 35), (2, 100, 9)]:
        s, err = est.sample_level(level, 11, first, count, with_error=True)
        ref = c0_oracle.sample(level, 11, first, count)
        scale = quad_scale(c0_oracle.sample_parts(level, 11, first, count))
        assert np.all(np.abs(s - ref) <= 1e-8 * scale), np.max(np.abs(s - ref) / scale)
        assert np.all(err <= 1e-8)


def test_level_L_not_sampleable():
    import paper_2108_11281_amd as m
    est = _est(32, 3)
    with pytest.raises(m.MLMCError) as e:
        est.sample_level(3, 1, 0, 2)
    assert e.value.code == -1


@pytest.mark.parametrize("alloc", ["equal", "giles"])
def test_mlmc_trace_matches_oracle_driver(alloc, c0_oracle):
    est = _est(64, 3, precision="fp32_ir64", nb=64, alloc=alloc)
    got = est.trace(1e-2, 3)
    ref = mlmc.mlmc_trace(c0_oracle, 1e-2, 3, nb=64,
                          alloc={"equal": mlmc.ALLOC_EQUAL, "giles": mlmc.ALLOC_GILES}[alloc])
    assert got["n_samples"] == ref["n_samples"]
    assert abs(got["trace"] - ref["trace"]) <= 1e-8 * abs(ref["trace"])
    assert abs(got["tau"] - ref["tau"]) <= 1e-8 * ref["tau"]
    exact = operators.poisson2d_trace_inverse(64)
    assert abs(got["trace"].real - exact) <= 4 * got["rmsd"]


def test_hutchinson_matches_oracle(c0_oracle):
    est = _est(64, 3, nb=64)
    got = est.hutchinson(3e-2, 2)
    ref = mlmc.hutchinson_trace(c0_oracle, 3e-2, 2, nb=64)
    assert got["n_samples"][0] == ref["n_samples"]
    assert abs(got["trace"] - ref["trace"]) <= 1e-8 * abs(ref["trace"])


def test_run_to_run_bitwise_repeatable():
    est = _est(64, 3, nb=16)
    a = est.sample_level(1, 5, 0, 16)
    b = est.sample_level(1, 5, 0, 16)
    assert np.array_equal(a, b)


def test_invalid_setup_is_rejected():
    import paper_2108_11281_amd as m
    require_gpu()
    with pytest.raises(m.MLMCError):
        m.TraceEstimator("poisson2d", 30, 4, 4)   # 30 -> 15 -> not divisible
    with pytest.raises(m.MLMCError):
        m.TraceEstimator("poisson2d", 64, 3, 4)   # L > L_s


def test_exit_handler_closes_live_estimators():
    # estimators still open at interpreter exit are closed by an exit handler
    # (while the allocator callbacks are intact), not by __del__ during
    # finalization
    import paper_2108_11281_amd as m
    est = _est(64, 3)
    assert est in m._live and est._ctx
    m._close_live()
    assert not est._ctx
    est.close()  # idempotent


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir64"])
def test_top_level_w_cycle_samples_and_iterations(precision):
    # two coarse-grid V-cycles below each solve's top level (top_cycles = 2) keep
    # the samples (same FP64 tolerance) and take fewer Krylov iterations than the
    # plain V-cycle on a 6-level 256^2 hierarchy with 2 + 2 sweeps
    N, L = 256, 6
    A, P = hierarchy.poisson_hierarchy(N, L)
    orc = mlmc.PoissonDSTSampler(N, L)
    its = {}
    for cyc in (1, 2):
        est = _est(N, L, precision=precision, nb=16, top_cycles=cyc, nu_pre=2, nu_post=2)
        s, err = est.sample_level(1, 5, 0, 16, with_error=True)
        ref = orc.sample(1, 5, 0, 16)
        scale = quad_scale(orc.sample_parts(1, 5, 0, 16))
        assert np.all(np.abs(s - ref) <= 1e-8 * scale), (cyc, np.max(np.abs(s - ref) / scale))
        assert np.all(err <= 1e-8)
        its[cyc] = est.counters()[0]
    assert its[2] < 0.8 * its[1], its
