"""Pins for the deflated Hutchinson oracle (Sec. 4.2, eqs. orth_proj and defl;
the comparison method of Sec. 5)."""
import itertools
import math

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import deflation, hierarchy, mlmc

C0_EXACT = 2763.642668185497   # tr((L^64)^-1), the closed form of Example 4.1
C0_PLAIN_VAR = 152291.26       # plain Hutchinson variance 2 sum_{i != j} (A^-1)_ij^2 at C0


def _closed_form_eigs(N):
    # eigenvalues of the 5-point Dirichlet Laplacian 4I - neighbours on N x N:
    # 4 sin^2(j pi / 2(N+1)) + 4 sin^2(k pi / 2(N+1)), j, k = 1..N
    s = 4.0 * np.sin(np.arange(1, N + 1) * np.pi / (2 * (N + 1))) ** 2
    return np.sort((s[:, None] + s[None, :]).ravel())


def test_eigenpairs_and_direct_term_match_closed_form():
    N, k = 24, 30
    A, _ = hierarchy.poisson_hierarchy(N, 2)
    lam, U = deflation.smallest_eigenpairs(A[0], k)
    ref = _closed_form_eigs(N)[:k]
    assert np.max(np.abs(lam - ref)) < 1e-12
    assert np.allclose(U.T @ U, np.eye(k), atol=1e-12)
    smp = deflation.DeflatedSampler(A[0], U)
    # with exact eigenvectors tr(A^-1 Pi) = sum 1/lambda_i (Sec. 5)
    assert abs(smp.direct().real - np.sum(1.0 / ref)) < 1e-10 * np.sum(1.0 / ref)


def _enumerate(n):
    for bits in itertools.product((1.0, -1.0), repeat=n):
        yield np.array(bits)


def test_deflated_sample_mean_and_variance_by_enumeration():
    # all 2^n Rademacher probes: the sample mean is tr(A^-1 (I - Pi)) exactly, for
    # exact eigenvectors that is tr(A^-1) - sum_{i<=k} 1/lambda_i, and the variance
    # is that of Cor. (variance) for B = A^-1 (I - Pi): 1/2 ||offdiag(B + B^T)||_F^2
    rng = np.random.default_rng(3)
    n, k = 10, 3
    G = rng.standard_normal((n, n))
    A = G @ G.T + n * np.eye(n)
    lam_all = np.linalg.eigvalsh(A)
    lam, U = deflation.smallest_eigenpairs(sp.csr_matrix(A), k)
    smp = deflation.DeflatedSampler(sp.csr_matrix(A), U)
    Ainv = np.linalg.inv(A)
    vals = []
    for x in _enumerate(n):
        y = smp.solver.solve(smp.project(x[:, None]))[:, 0]
        vals.append(mlmc.quad(x, y).real)
    vals = np.array(vals)
    assert abs(vals.mean() - (np.sum(1.0 / lam_all) - np.sum(1.0 / lam_all[:k]))) < 1e-12
    B = Ainv @ (np.eye(n) - U @ U.T)
    S = B + B.T
    off = S - np.diag(np.diag(S))
    assert abs(np.mean((vals - vals.mean()) ** 2) - 0.5 * np.sum(off ** 2)) < 1e-12
    # total: mean + direct term = tr(A^-1)
    assert abs(vals.mean() + smp.direct().real - np.trace(Ainv)) < 1e-12


def test_split_exact_for_any_orthonormal_u():
    # approximate eigenvectors keep the split exact: E[x^T A^-1 (I - U U^T) x]
    # + tr(U^T A^-1 U) = tr(A^-1) for a random orthonormal U, while the sum of
    # reciprocal Rayleigh quotients that stands in for sum 1/lambda_i does not
    rng = np.random.default_rng(4)
    n, k = 9, 4
    G = rng.standard_normal((n, n))
    A = G @ G.T + n * np.eye(n)
    U, _ = np.linalg.qr(rng.standard_normal((n, k)))
    smp = deflation.DeflatedSampler(sp.csr_matrix(A), U)
    Ainv = np.linalg.inv(A)
    m = np.mean([mlmc.quad(x, smp.solver.solve(smp.project(x[:, None]))[:, 0]).real
                 for x in _enumerate(n)])
    assert abs(m + smp.direct().real - np.trace(Ainv)) < 1e-12
    rq = np.array([U[:, i] @ A @ U[:, i] for i in range(k)])
    assert abs(m + np.sum(1.0 / rq) - np.trace(Ainv)) > 1e-3


def test_deflated_sample_is_plain_sample_minus_projected_part():
    # same probe stream as plain Hutchinson: s_defl = x^T A^-1 x - x^T A^-1 U U^T x
    A, _ = hierarchy.poisson_hierarchy(16, 2)
    lam, U = deflation.smallest_eigenpairs(A[0], 8)
    smp = deflation.DeflatedSampler(A[0], U)
    s = smp.sample(5, 0, 6)
    plain = smp.hutchinson(5, 0, 6)
    X = smp.probes(5, 0, 6)
    Ainv = np.linalg.inv(A[0].toarray())
    corr = np.array([X[:, j] @ Ainv @ U @ (U.T @ X[:, j]) for j in range(6)])
    assert np.allclose(s.real, plain.real - corr, rtol=0, atol=1e-10)


@pytest.fixture(scope="module")
def c0_deflated():
    A, _ = hierarchy.poisson_hierarchy(64, 2)
    lam, U = deflation.smallest_eigenpairs(A[0], 32)
    return A[0], lam, deflation.DeflatedSampler(A[0], U)


def test_c0_deflated_variance_matches_formula(c0_deflated):
    # V = 2 sum_{i != j} B_ij^2 (symmetric B = A^-1 (I - Pi), Rademacher probes),
    # below the plain Hutchinson variance of C0; the sample variance agrees
    A, lam, smp = c0_deflated
    Ainv = np.linalg.inv(A.toarray())
    B = Ainv - smp.U @ np.diag(1.0 / lam) @ smp.U.T
    off = B - np.diag(np.diag(B))
    V = 2.0 * np.sum(off ** 2)
    assert V < 0.5 * C0_PLAIN_VAR
    s = smp.sample(11, 0, 400)
    m, v = mlmc.mean_and_var(s)
    assert abs(v / V - 1.0) < 0.35
    assert abs(m.real - np.trace(B)) < 4.0 * math.sqrt(V / 400)


def test_c0_deflated_hutchinson_trace(c0_deflated):
    _, lam, smp = c0_deflated
    for seed in (1, 2):
        r = deflation.deflated_hutchinson_trace(smp, 1e-2, seed)
        assert r["rmsd"] <= 1e-2 * r["tau"] * (1 + 1e-12)
        assert abs(r["trace"].real - C0_EXACT) < 4.0 * r["rmsd"]
        assert abs(r["direct"].real - np.sum(1.0 / lam)) < 1e-9 * np.sum(1.0 / lam)
