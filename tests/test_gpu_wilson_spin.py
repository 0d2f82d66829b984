"""GPU parity of the spin-structure-preserving aggregation of the Wilson-like
operator (Example 4.3: test vectors split by spin, 2 n_vec coarse unknowns per
aggregate) against the oracle, and the spin symmetry J A = A^* J of the
library's own coarse operators."""
import numpy as np
import pytest

from oracle import hierarchy, mlmc
from tests.gpu_util import from_dev, quad_scale, require_gpu, to_dev
from workloads import gauge_field

pytestmark = pytest.mark.gpu

N, LEVELS, BLK, NVEC, SWEEPS, M0 = 32, 3, 4, 4, 6, 0.1
NC = 2 * NVEC


@pytest.fixture(scope="module")
def oracle_h():
    th = gauge_field(N, seed=1)
    A, P = hierarchy.wilson_hierarchy(N, th, M0, LEVELS, block=BLK, n_vec=NVEC, sweeps=SWEEPS,
                                      seed=1, spin_split=True)
    return th, A, P, mlmc.LevelSampler(A, P, complex_probe=True)


def _est(th, precision="fp64", nb=16, **kw):
    require_gpu()
    import paper_2108_11281_amd as m
    kw.setdefault("solve_tol", 1e-12)
    return m.TraceEstimator("wilson2d", N, LEVELS, LEVELS, mass=M0, field=th, block=BLK,
                            n_vec=NVEC, setup_sweeps=SWEEPS, setup_seed=1, spin_split=True,
                            precision=precision, nb=nb, nu_pre=2, nu_post=2, **kw)


def test_prolongation_and_coarse_operators(oracle_h):
    th, A, P, _ = oracle_h
    est = _est(th)
    for level in (1, 2):
        q = est.export_prolongation(level, NC)
        Pd = P[level - 1].toarray()
        # row i of q: unknown i's coefficients in its aggregate's 2 n_vec columns
        # (zero in the n_vec columns of the other spin)
        ref = np.zeros((q.shape[0], NC), dtype=complex)
        for i in range(q.shape[0]):
            S = np.nonzero(Pd[i])[0][0] // NC
            ref[i] = Pd[i, S * NC:(S + 1) * NC]
        assert np.max(np.abs(q - ref)) < 1e-10, np.max(np.abs(q - ref))
    rng = np.random.default_rng(3)
    for level in (2, 3):
        n = est.level_size(level)
        assert n == (N // BLK ** (level - 1)) ** 2 * NC
        X = rng.standard_normal((3, n)) + 1j * rng.standard_normal((3, n))
        Y = from_dev(est.apply(level, to_dev(X)), complex_=True)
        ref = (A[level - 1] @ X.T).T
        assert np.max(np.abs(Y - ref)) <= 1e-9 * np.max(np.abs(ref)), level
    # the library's coarsest operator keeps the spin symmetry
    Ad = est.export_coarse(0)
    J = hierarchy.spin_sign((N // BLK ** 2) ** 2, NC).toarray()
    assert np.max(np.abs(J @ Ad @ J - Ad.conj().T)) <= 1e-12 * np.max(np.abs(Ad))
    ct = est.coarse_trace()
    assert abs(ct.imag) <= 1e-10 * abs(ct)
    assert abs(ct - oracle_h[3].coarse()) <= 1e-9 * abs(ct)


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir64"])
def test_samples_match_oracle(oracle_h, precision):
    th, _, _, orc = oracle_h
    est = _est(th, precision=precision)
    for level, first, count in [(1, 0, 12), (2, 20, 6)]:
        s, err = est.sample_level(level, 7, first, count, with_error=True)
        ref = orc.sample(level, 7, first, count)
        scale = quad_scale(orc.sample_parts(level, 7, first, count))
        assert np.all(np.abs(s - ref) <= 1e-8 * scale), np.max(np.abs(s - ref) / scale)
        assert np.all(err <= 1e-8)


def test_sweeps_on_the_split_levels(oracle_h):
    th, A, _, _ = oracle_h
    est = _est(th, precision="fp32_ir64")
    rng = np.random.default_rng(5)
    n = est.level_size(2)
    B = rng.standard_normal((4, n)) + 1j * rng.standard_normal((4, n))
    X = rng.standard_normal((4, n)) + 1j * rng.standard_normal((4, n))
    colour = np.repeat(hierarchy.site_coloring(N // BLK), NC)
    for rev in (False, True):
        got = from_dev(est.smooth(2, to_dev(B), to_dev(X), 1, rev), complex_=True)
        for k in range(4):
            ref = hierarchy.rbgs_sweeps(A[1], B[k], X[k], colour, 1, rev)
            assert np.max(np.abs(got[k] - ref)) <= 1e-5 * np.max(np.abs(ref)), (rev, k)


def test_unsupported_site_size_is_rejected():
    require_gpu()
    import paper_2108_11281_amd as m
    th = gauge_field(N, seed=1)
    with pytest.raises(m.MLMCError):     # 2 x 16 coarse unknowns per site
        m.TraceEstimator("wilson2d", N, 2, 2, mass=M0, field=th, block=BLK, n_vec=16,
                         spin_split=True)
