"""GPU parity of the general decomposition of Sec. 4.1 (given prolongations,
R = P^T, finest-level probes, coarsest term tr(A_L^-1 Rhat_L Phat_L)) on
Example 4.1's hierarchy: the 2D Laplacian with bilinear interpolation and
Galerkin coarse operators, through the csr kind."""
import numpy as np
import pytest

from oracle import hierarchy, mlmc, operators
from tests.gpu_util import from_dev, quad_scale, require_gpu, to_dev
from workloads import bilinear_prolongations, laplace_matrix

pytestmark = pytest.mark.gpu

N, LS = 63, 4          # 63^2 -> 31^2 -> 15^2 -> 7^2


def _est(L, **kw):
    require_gpu()
    import paper_2108_11281_amd as m
    kw.setdefault("nb", 16)
    kw.setdefault("solve_tol", 1e-12)
    # the library's inputs come from the workload generators; the oracle builds
    # its own hierarchy, so the comparison also checks the two against each other
    return m.TraceEstimator("csr", 0, LS, L, matrix=laplace_matrix(N),
                            prolongations=bilinear_prolongations(N, LS), **kw)


_ORC = {}


def _oracle(L):
    if L not in _ORC:
        A, P = hierarchy.laplace_bilinear_hierarchy(N, LS)
        _ORC[L] = mlmc.GeneralLevelSampler(A[:L], P[:L - 1], complex_probe=False)
    return _ORC[L]


def test_hierarchy_transfers_and_coarse_term():
    A, P = hierarchy.laplace_bilinear_hierarchy(N, LS)
    for L in (3, 4):
        est = _est(L)
        for l in range(1, LS + 1):
            Al, agg, col = est.export_csr(l)
            ref = A[l - 1]
            assert np.array_equal(Al.indptr, ref.indptr) and np.array_equal(Al.indices, ref.indices)
            assert np.max(np.abs(Al.data - ref.data)) <= 1e-14 * np.max(np.abs(ref.data)), l
            assert agg is None
            assert np.array_equal(col, hierarchy.first_fit_coloring(ref))
        rng = np.random.default_rng(1)
        for l in range(1, LS):
            X = rng.standard_normal((5, A[l - 1].shape[0]))
            got = from_dev(est.restrict(l, to_dev(X)))
            ref = (P[l - 1].T @ X.T).T
            assert np.max(np.abs(got - ref)) <= 1e-14 * np.max(np.abs(ref)), l
            E = rng.standard_normal((3, A[l].shape[0]))
            got = from_dev(est.prolong(l, to_dev(E)))
            ref = (P[l - 1] @ E.T).T
            assert np.max(np.abs(got - ref)) <= 1e-14 * np.max(np.abs(ref)), l
        want = _oracle(L).coarse().real
        assert abs(est.coarse_trace().real - want) <= 1e-11 * abs(want), L


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir64"])
def test_sweeps_and_solves(precision):
    A, _ = hierarchy.laplace_bilinear_hierarchy(N, LS)
    est = _est(3, precision=precision)
    rng = np.random.default_rng(2)
    tol = 1e-13 if precision == "fp64" else 1e-5
    for l in (2, 3):     # 9-point Galerkin levels, four colour classes
        col = hierarchy.first_fit_coloring(A[l - 1])
        assert col.max() == 3
        B = rng.standard_normal((4, A[l - 1].shape[0]))
        X = rng.standard_normal((4, A[l - 1].shape[0]))
        for rev in (False, True):
            got = from_dev(est.smooth(l, to_dev(B), to_dev(X), 2, rev))
            for k in range(4):
                ref = hierarchy.multicolour_gs_sweeps(A[l - 1], B[k], X[k], col, 2, rev)
                assert np.max(np.abs(got[k] - ref)) <= tol * np.max(np.abs(ref)), (l, rev, k)
    for l in (1, 2, 3):
        B = rng.standard_normal((6, A[l - 1].shape[0]))
        Y, rel = est.solve(l, to_dev(B))
        assert np.all(rel <= 1e-12), (l, rel)
        ref = _oracle(3).solver(l).solve(B.T).T
        assert np.max(np.abs(from_dev(Y) - ref)) <= 1e-8 * np.max(np.abs(ref))


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir64"])
def test_samples_match_oracle(precision):
    for L in (3, 4):
        est = _est(L, precision=precision)
        orc = _oracle(L)
        for level, first, count in [(1, 0, 9), (L - 1, 30, 7)]:
            s, err = est.sample_level(level, 13, first, count, with_error=True)
            ref = orc.sample(level, 13, first, count)
            scale = quad_scale(orc.sample_parts(level, 13, first, count))
            assert np.all(np.abs(s - ref) <= 1e-8 * scale), (L, level,
                                                            np.max(np.abs(s - ref) / scale))
            assert np.all(err <= 1e-8)


def test_trace_matches_oracle_driver_and_closed_form():
    est = _est(3, precision="fp32_ir64", nb=32, alloc="giles")
    orc = _oracle(3)
    got = est.trace(2e-2, 4)
    ref = mlmc.mlmc_trace(orc, 2e-2, 4, nb=32, alloc=mlmc.ALLOC_GILES)
    assert got["n_samples"] == ref["n_samples"]
    assert abs(got["trace"] - ref["trace"]) <= 1e-8 * abs(ref["trace"])
    exact = operators.poisson2d_trace_inverse(N)
    assert abs(got["trace"].real - exact) <= 4 * got["rmsd"]


def test_prolongations_are_validated():
    require_gpu()
    import paper_2108_11281_amd as m
    A, P = laplace_matrix(N), bilinear_prolongations(N, LS)
    with pytest.raises(m.MLMCError):          # P_2 given where P_1 belongs
        m.TraceEstimator("csr", 0, 2, 2, matrix=A, prolongations=[P[1]])
    with pytest.raises(ValueError):           # one matrix per level below the coarsest
        m.TraceEstimator("csr", 0, LS, LS, matrix=A, prolongations=P[:1])
    with pytest.raises(m.MLMCError):          # aggregates and prolongations together
        m.TraceEstimator("csr", 0, 2, 2, matrix=A, prolongations=P[:1],
                         agg=[np.zeros(N * N, dtype=np.int32)])


def test_narrow_batches_in_fp64():
    # FP32 + refinement with batches of up to 8 columns solved in plain FP64:
    # a batch of 5 takes the FP64 path, a batch of 12 the FP32 one; both give the
    # oracle's samples
    est = _est(3, precision="fp32_ir64", nb=16, narrow_fp64=8)
    orc = _oracle(3)
    for count in (5, 12):
        s, err = est.sample_level(1, 21, 0, count, with_error=True)
        ref = orc.sample(1, 21, 0, count)
        scale = quad_scale(orc.sample_parts(1, 21, 0, count))
        assert np.all(np.abs(s - ref) <= 1e-8 * scale), (count, np.max(np.abs(s - ref) / scale))
        assert np.all(err <= 1e-8)
