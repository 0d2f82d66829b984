"""Pins for the oracle's samples, coarsest trace and MLMC driver (Secs. 2-5)."""
import itertools
import math

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import hierarchy, mlmc, operators, philox


def _enumerate_rademacher(n):
    for bits in itertools.product((1.0, -1.0), repeat=n):
        yield np.array(bits)


def test_hutchinson_mean_and_variance_by_enumeration_rademacher():
    # Theorem hutchinson / Cor. variance: E = tr(A), V = 1/2 ||offdiag(A + A^T)||_F^2
    rng = np.random.default_rng(3)
    A = rng.standard_normal((9, 9))
    vals = [mlmc.quad(x, A @ x) for x in _enumerate_rademacher(9)]
    m = np.mean(vals)
    v = np.mean(np.abs(np.array(vals) - m) ** 2)
    S = A + A.T
    off = S - np.diag(np.diag(S))
    assert abs(m - np.trace(A)) < 1e-12
    assert abs(v - 0.5 * np.sum(off ** 2)) < 1e-10


def test_hutchinson_variance_by_enumeration_z4():
    # Cor. variance, second case: V = ||offdiag(A)||_F^2 for Z4 probes
    rng = np.random.default_rng(4)
    A = rng.standard_normal((6, 6)) + 1j * rng.standard_normal((6, 6))
    vals = []
    for digits in itertools.product(range(4), repeat=6):
        x = np.array([1, 1j, -1, -1j])[list(digits)]
        vals.append(mlmc.quad(x, A @ x))
    vals = np.array(vals)
    m = vals.mean()
    v = np.mean(np.abs(vals - m) ** 2)
    off = A - np.diag(np.diag(A))
    assert abs(m - np.trace(A)) < 1e-12
    assert abs(v - np.sum(np.abs(off) ** 2)) < 1e-10


def test_mean_and_var_is_bessel_corrected():
    rng = np.random.default_rng(5)
    s = rng.standard_normal(17) + 1j * rng.standard_normal(17)
    m, v = mlmc.mean_and_var(s)
    assert abs(m - s.mean()) < 1e-14
    assert abs(v - (np.var(s.real, ddof=1) + np.var(s.imag, ddof=1))) < 1e-13


def _tiny_poisson():
    A, P = hierarchy.poisson_hierarchy(4, 2)
    return mlmc.LevelSampler(A, P, complex_probe=False), A, P


def test_sample_value_against_dense_difference_operator():
    # s = x^T (A_1^-1 - P A_2^-1 R) x (Remark 4.3)
    smp, A, P = _tiny_poisson()
    P = P[0]
    D = np.linalg.inv(A[0].toarray()) - P.toarray() @ np.linalg.inv(A[1].toarray()) @ P.T.toarray()
    s = smp.sample(1, 7, 0, 4)
    X = smp.probes(1, 7, 0, 4)
    for j in range(4):
        assert abs(s[j] - X[:, j] @ D @ X[:, j]) < 1e-13


def test_level_difference_unbiased_by_enumeration():
    # E over all 2^16 probes equals tr(A_1^-1) - tr(P A_2^-1 R) exactly
    A, P = hierarchy.poisson_hierarchy(4, 2)
    P = P[0]
    D = np.linalg.inv(A[0].toarray()) - P.toarray() @ np.linalg.inv(A[1].toarray()) @ P.T.toarray()
    X = np.array(list(_enumerate_rademacher(16))).T          # 16 x 65536
    s = np.einsum("ik,ij,jk->k", X, D, X)
    assert abs(s.mean() - np.trace(D)) < 1e-12
    off = D - np.diag(np.diag(D))
    assert abs(np.mean((s - s.mean()) ** 2) - 2.0 * np.sum(off ** 2)) < 1e-10
    # closed form: A_l = 2^{1-l} L^{N_l}, so tr(D) = T(4) - 2 T(2)
    assert abs(np.trace(D) - (operators.poisson2d_trace_inverse(4)
                              - 2.0 * operators.poisson2d_trace_inverse(2))) < 1e-12


def test_telescoping_and_closed_form_level_means_poisson64():
    # eq. tr_ml_dec with R P = I: sum_l [tr(A_l^-1) - tr(P A_{l+1}^-1 R)] + tr(A_L^-1)
    N, L = 64, 3
    A, P = hierarchy.poisson_hierarchy(N, L)
    T = operators.poisson2d_trace_inverse
    tot = 0.0
    for l in range(L - 1):
        Ainv = np.linalg.inv(A[l].toarray())
        Acinv = np.linalg.inv(A[l + 1].toarray())
        Pd = P[l].toarray()
        diff = np.trace(Ainv) - np.trace(Pd @ Acinv @ Pd.T)
        Nl = N >> l
        closed = 2.0 ** l * T(Nl) - 2.0 ** (l + 1) * T(Nl // 2)
        assert abs(diff - closed) < 1e-9 * abs(closed)
        tot += diff
    coarse = mlmc.coarse_trace(A[-1]).real
    assert abs(coarse - 2.0 ** (L - 1) * T(N >> (L - 1))) < 1e-10 * coarse
    assert abs(tot + coarse - T(N)) < 1e-9 * T(N)


def test_exact_solver_sparse_path_matches_dst():
    N = 72                                  # n = 5184 > DENSE_MAX -> sparse LU path
    A = operators.poisson2d(N, 2.0, 0.5)
    s = mlmc.ExactSolver(A)
    assert s.splu is not None
    B = np.stack([philox.rademacher(N * N, 1, k, 1) for k in range(3)], axis=1)
    Y = s.solve(B)
    ref = operators.poisson2d_solve_dst(N, B, 2.0, 0.5)
    assert np.max(np.abs(Y - ref)) < 1e-12 * np.max(np.abs(ref))


def test_giles_allocation_algebra():
    # Sec. 2: N_l = mu sqrt(V_l/C_l) minimises sum N_l C_l s.t. sum V_l/N_l = eps^2,
    # with total cost eps^-2 (sum sqrt(V_l C_l))^2.
    V = [36321.25, 9052.56, 2500.0]
    C = [5120.0, 1280.0, 320.0]
    eps2 = 4.0
    w = mlmc.level_weights(mlmc.ALLOC_GILES, 4, V, C)
    assert abs(sum(w) - 1.0) < 1e-15
    N = [V[l] / (w[l] * eps2) for l in range(3)]      # N_l = V_l / rho_l^2
    assert abs(sum(V[l] / N[l] for l in range(3)) - eps2) < 1e-9
    ratios = [N[l] / math.sqrt(V[l] / C[l]) for l in range(3)]
    assert max(ratios) - min(ratios) < 1e-9 * max(ratios)
    cost = sum(N[l] * C[l] for l in range(3))
    assert abs(cost - (sum(math.sqrt(v * c) for v, c in zip(V, C))) ** 2 / eps2) < 1e-6 * cost
    # any other feasible allocation costs more
    rng = np.random.default_rng(0)
    for _ in range(20):
        w2 = rng.dirichlet(np.ones(3))
        N2 = [V[l] / (w2[l] * eps2) for l in range(3)]
        assert sum(N2[l] * C[l] for l in range(3)) >= cost * (1 - 1e-12)


def test_equal_and_given_weights():
    assert mlmc.level_weights(mlmc.ALLOC_EQUAL, 5, None, None) == [0.25] * 4
    w = mlmc.level_weights(mlmc.ALLOC_WEIGHTS, 4, None, None, [0.4, 0.55, 0.05])
    assert np.allclose(w, [0.4, 0.55, 0.05])


@pytest.fixture(scope="module")
def c0_sampler():
    A, P = hierarchy.poisson_hierarchy(64, 3)
    return mlmc.LevelSampler(A, P, complex_probe=False)


def test_c0_level_variances_match_exact(c0_sampler):
    # V_l = 2 sum_{i != j} (D_l)_ij^2 for Rademacher probes and symmetric D_l
    A, P = c0_sampler.A, c0_sampler.P
    Ainv = [np.linalg.inv(a.toarray()) for a in A]
    for l, n in [(1, 256), (2, 256)]:
        D = Ainv[l - 1] - P[l - 1].toarray() @ Ainv[l] @ P[l - 1].T.toarray()
        off = D - np.diag(np.diag(D))
        V = 2.0 * np.sum(off ** 2)
        s = c0_sampler.sample(l, 42, 0, n)
        m, v = mlmc.mean_and_var(s)
        # sample variance of n draws: relative sd about sqrt(2/(n-1)) (+ kurtosis)
        assert abs(v / V - 1.0) < 0.35
        assert abs(m - np.trace(D)) < 4.0 * math.sqrt(V / n)


def test_c0_mlmc_trace_within_error(c0_sampler):
    exact = operators.poisson2d_trace_inverse(64)
    z = []
    for seed in [1, 2, 3]:
        r = mlmc.mlmc_trace(c0_sampler, 1e-2, seed, nb=128)
        assert r["rmsd"] <= 1e-2 * r["tau"] * (1 + 1e-12)
        assert all(n >= 5 for n in r["n_samples"])
        z.append((r["trace"].real - exact) / r["rmsd"])
    assert max(abs(v) for v in z) < 4.0


def test_minimum_five_samples_at_loose_tolerance(c0_sampler):
    # Example 4.1: at eps = 1e-1 only the minimum of five estimates is done
    r = mlmc.mlmc_trace(c0_sampler, 1e-1, 1, nb=128)
    assert r["n_samples"] == [5, 5]
    assert r["rounds"] == 0


def test_cost_scales_like_eps_minus_two(c0_sampler):
    # Example 4.1: quadratic dependence on 1/eps for small eps (same seed, same tau)
    tau = operators.poisson2d_trace_inverse(64)
    n1 = sum(mlmc.mlmc_trace(c0_sampler, 4e-3, 1, tau=tau)["n_samples"])
    n2 = sum(mlmc.mlmc_trace(c0_sampler, 2e-3, 1, tau=tau)["n_samples"])
    assert 3.0 < n2 / n1 < 5.5


def test_hutchinson_driver(c0_sampler):
    exact = operators.poisson2d_trace_inverse(64)
    r = mlmc.hutchinson_trace(c0_sampler, 2e-2, 1)
    assert abs(r["trace"].real - exact) < 4 * r["rmsd"]


def test_dst_sampler_matches_sparse_sampler():
    A, P = hierarchy.poisson_hierarchy(32, 3)
    ref = mlmc.LevelSampler(A, P, complex_probe=False)
    dst = mlmc.PoissonDSTSampler(32, 3)
    for l in (1, 2):
        assert np.allclose(dst.sample(l, 3, 5, 4), ref.sample(l, 3, 5, 4), rtol=1e-12, atol=1e-12)
    assert abs(dst.coarse() - ref.coarse()) < 1e-12 * abs(ref.coarse())
    assert np.allclose(dst.hutchinson(1, 0, 3), ref.hutchinson(1, 0, 3), rtol=1e-12)


def _gaussian_regime_sampler(n=400, scale=0.2, seed=11):
    """A = I + G with G a scaled symmetric Gaussian matrix (no dominant off-diagonal
    direction), so x^T A^{-1} x for Rademacher x is close to normally distributed
    (a second-order Rademacher chaos over a matrix with a spread-out spectrum)."""
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n, n))
    G = (G + G.T) * (scale / math.sqrt(2 * n))
    A = sp.csr_matrix(np.eye(n) + G)
    smp = mlmc.LevelSampler([A, A], [sp.identity(n, format="csr")], complex_probe=False)
    return smp, float(np.trace(np.linalg.inv(A.toarray())))


def test_pilot_tau_is_a_one_sided_t4_bound():
    # Sec. 5: tau = mean of five pilot estimates minus their RMSD (the standard error
    # sqrt(s^2/5)).  For Gaussian estimates, (mean - T)/sqrt(s^2/5) follows Student's
    # t with 4 degrees of freedom, so P(tau <= T) = F_t4(1) = 0.8130.  The standard
    # deviation in place of the standard error gives F_t4(sqrt 5) = 0.96, no
    # subtraction 0.5: both fall outside the window (800 seeds: binomial sd 0.014).
    # (C0's Hutchinson samples are too skewed, skewness ~1.4, for the t4 level.)
    import scipy.stats as st
    smp, T = _gaussian_regime_sampler()
    y = smp.hutchinson(1, 0, 2000, stream=philox.STREAM_PILOT).real
    assert abs(st.skew(y)) < 0.3          # the Gaussian regime the t4 level needs
    cover, stat = [], []
    for seed in range(800):
        tau, yp = mlmc.pilot_tau(smp, seed)
        m = float(np.mean(yp.real))
        cover.append(tau <= T)
        stat.append((m - T) / (m - tau))  # (mean - T) / standard error
    assert abs(st.t.cdf(1.0, 4) - 0.8130) < 1e-4
    assert 0.77 <= np.mean(cover) <= 0.86
    # the studentised mean is t4 distributed (a scaled statistic is rejected)
    assert st.kstest(stat, st.t(4).cdf).pvalue > 1e-3
    assert st.kstest(np.array(stat) * math.sqrt(5.0), st.t(4).cdf).pvalue < 1e-6


def test_pilot_samples_independent_of_estimator_samples():
    # Sec. 5 (reading): the five pilot estimates come from their own probe stream and
    # are not reused by the estimator or by plain Hutchinson.  Over many seeds the pilot
    # mean must be uncorrelated with the first five level-1 quadratic forms and with
    # the first five plain-Hutchinson samples (a reused stream gives correlation 1).
    smp, _ = _gaussian_regime_sampler()
    pil, lev, hut = [], [], []
    for seed in range(300):
        _, yp = mlmc.pilot_tau(smp, seed)
        pil.append(np.mean(yp.real))
        a, _ = smp.sample_parts(1, seed, 0, 5)
        lev.append(np.mean(a.real))
        hut.append(np.mean(smp.hutchinson(seed, 0, 5).real))
    for other in (lev, hut):
        r = np.corrcoef(pil, other)[0, 1]
        assert abs(r) < 4.0 / math.sqrt(300)
