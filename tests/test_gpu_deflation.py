"""GPU parity of deflated Hutchinson (Sec. 4.2 eqs. orth_proj / defl; the
comparison method of Sec. 5): the library's subspace-iteration eigenpairs
against the closed-form Poisson spectrum and the oracle's dense eigenvectors,
the direct term, every deflated sample against the oracle's exact sample for the
library's own deflation space, the estimator's sample counts, and the full-size
1024^2 operator on sampled outputs (exact sine-transform solves)."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import deflation, hierarchy, operators, philox
from tests.gpu_util import from_dev, require_gpu

pytestmark = pytest.mark.gpu


def _closed_form_eigs(N):
    s = 4.0 * np.sin(np.arange(1, N + 1) * np.pi / (2 * (N + 1))) ** 2
    return np.sort((s[:, None] + s[None, :]).ravel())


def _gap_k(lam, lo):
    # smallest k >= lo with a 2% gap after eigenvalue k (degenerate pairs of the
    # square grid are kept together)
    k = lo
    while lam[k] - lam[k - 1] < 0.02 * lam[k]:
        k += 1
    return k


@pytest.fixture(scope="module")
def poisson64():
    require_gpu()
    import paper_2108_11281_amd as m
    N = 64
    lam = _closed_form_eigs(N)
    k = _gap_k(lam, 20)
    est = m.TraceEstimator("poisson2d", N, 3, 3, precision="fp32_ir64", nb=32, solve_tol=1e-12)
    rep = est.deflation_setup(k, eig_tol=1e-5, max_iter=200, solve_tol=1e-10, seed=3)
    ev, U, direct = est.deflation_export(k)
    A, _ = hierarchy.poisson_hierarchy(N, 2)
    return dict(N=N, k=k, lam=lam, est=est, rep=rep, ev=ev, U=from_dev(U), direct=direct,
                A=A[0])


def test_eigenpairs_match_closed_form_and_oracle(poisson64):
    d = poisson64
    k, lam = d["k"], d["lam"]
    assert d["rep"]["max_residual"] <= 1e-5, d["rep"]
    # Ritz values: second order in the residual
    assert np.max(np.abs(d["ev"] - lam[:k]) / lam[:k]) <= 1e-8
    U = d["U"].T                      # n x k
    assert np.allclose(U.T @ U, np.eye(k), atol=1e-10)
    lo, Uo = deflation.smallest_eigenpairs(d["A"], k)
    # same invariant subspace: the projectors agree (first order in the residual)
    Pg, Po = U @ U.T, Uo @ Uo.T
    assert np.linalg.norm(Pg - Po, 2) <= 1e-3
    # direct term: tr(U^T A^-1 U) recomputed by the oracle for the library's U,
    # and sum 1/lambda_i of the closed form
    orc = deflation.DeflatedSampler(d["A"], U)
    assert abs(d["direct"] - orc.direct().real) <= 1e-10 * abs(d["direct"])
    assert abs(d["direct"] - np.sum(1.0 / lam[:k])) <= 1e-7 * abs(d["direct"])
    assert abs(d["rep"]["sum_inv_eig"] - np.sum(1.0 / lam[:k])) <= 1e-7 * abs(d["direct"])


def test_deflated_samples_match_oracle(poisson64):
    d = poisson64
    U = d["U"].T
    orc = deflation.DeflatedSampler(d["A"], U)
    s, err = d["est"].deflated_sample(7, 3, 40, with_error=True)
    ref = orc.sample(7, 3, 40)
    plain = orc.hutchinson(7, 3, 40)
    scale = np.maximum(np.abs(ref), np.abs(plain))
    assert np.all(np.abs(s - ref) <= 1e-8 * scale), np.max(np.abs(s - ref) / scale)
    assert np.all(err <= 1e-8)
    # the same probes as plain Hutchinson: the deflated sample is the plain one
    # minus the part the projector takes out
    Ainv = np.linalg.inv(d["A"].toarray())
    X = orc.probes(7, 3, 40)
    corr = np.array([X[:, j] @ Ainv @ U @ (U.T @ X[:, j]) for j in range(40)])
    assert np.all(np.abs(s.real - (plain.real - corr)) <= 1e-8 * scale)


def test_deflated_estimator_matches_oracle_counts(poisson64):
    d = poisson64
    U = d["U"].T
    orc = deflation.DeflatedSampler(d["A"], U)
    exact = operators.poisson2d_trace_inverse(d["N"])
    for seed in (1, 2):
        r = d["est"].deflated_hutchinson(1e-2, seed)
        ro = deflation.deflated_hutchinson_trace(orc, 1e-2, seed, nb=32)
        assert r["n_samples"][0] == ro["n_samples"], (r["n_samples"], ro["n_samples"])
        assert abs(r["trace"].real - ro["trace"].real) <= 1e-8 * abs(ro["trace"].real)
        assert abs(r["coarse"].real - d["direct"]) <= 1e-12 * abs(d["direct"])
        assert abs(r["trace"].real - exact) <= 4.0 * r["rmsd"]
        # deflation takes out variance: fewer samples than plain Hutchinson
        rp = d["est"].hutchinson(1e-2, seed)
        assert r["n_samples"][0] < rp["n_samples"][0]


def test_full_size_poisson1024_deflation_and_samples():
    # the 1024^2 headline operator: Ritz values against the closed form, the
    # direct term against sum 1/lambda_i, and sampled deflated samples against
    # exact sine-transform solves of x_perp with the library's own U
    require_gpu()
    import paper_2108_11281_amd as m
    N, k = 1024, 32
    lam = _closed_form_eigs(N)
    k = _gap_k(lam, k)
    est = m.TraceEstimator("poisson2d", N, 6, 6, precision="fp32_ir64", nb=128,
                           solve_tol=1e-10)
    rep = est.deflation_setup(k, eig_tol=1e-4, max_iter=200, solve_tol=1e-8, seed=5)
    assert rep["max_residual"] <= 1e-4, rep
    ev, Ud, direct = est.deflation_export(k)
    assert np.max(np.abs(ev - lam[:k]) / lam[:k]) <= 1e-6
    assert abs(direct - np.sum(1.0 / lam[:k])) <= 1e-6 * direct
    U = from_dev(Ud).T
    s, err = est.deflated_sample(9, 100, 4, with_error=True)
    assert np.all(err <= 1e-8)
    X = np.stack([philox.rademacher(N * N, 9, 100 + j, 1, stream=3) for j in range(4)],
                 axis=1)
    Xp = X - U @ (U.T @ X)
    Y = operators.poisson2d_solve_dst(N, Xp, 4.0, 1.0)
    ref = np.array([X[:, j] @ Y[:, j] for j in range(4)])
    plain = operators.poisson2d_solve_dst(N, X, 4.0, 1.0)
    scale = np.array([abs(X[:, j] @ plain[:, j]) for j in range(4)])
    assert np.all(np.abs(s.real - ref) <= 1e-8 * scale), np.abs(s.real - ref) / scale


def test_csr_graph_deflation_matches_oracle():
    # a matrix-given operator: the shifted Laplacian of a random geometric graph
    require_gpu()
    import paper_2108_11281_amd as m
    from workloads import graph_laplacian
    A = sp.csr_matrix(graph_laplacian(3000, degree=8.0, shift=1e-2, seed=4))
    k = 16
    est = m.TraceEstimator("csr", 0, 3, 3, matrix=A, precision="fp32_ir64", nb=16,
                           solve_tol=1e-12)
    rep = est.deflation_setup(k, eig_tol=1e-6, max_iter=300, solve_tol=1e-10, seed=2)
    assert rep["max_residual"] <= 1e-6, rep
    ev, Ud, direct = est.deflation_export(k)
    lo, Uo = deflation.smallest_eigenpairs(A, k)
    assert np.max(np.abs(ev - lo) / lo) <= 1e-9
    U = from_dev(Ud).T
    orc = deflation.DeflatedSampler(A, U)
    assert abs(direct - orc.direct().real) <= 1e-10 * abs(direct)
    s = est.deflated_sample(3, 0, 20)
    ref = orc.sample(3, 0, 20)
    plain = orc.hutchinson(3, 0, 20)
    scale = np.maximum(np.abs(ref), np.abs(plain))
    assert np.all(np.abs(s - ref) <= 1e-8 * scale)


def test_deflation_errors():
    require_gpu()
    import paper_2108_11281_amd as m
    from workloads import gauge_field
    est = m.TraceEstimator("poisson2d", 32, 2, 2, nb=8)
    with pytest.raises(m.MLMCError):      # no deflation space yet
        est.deflated_sample(1, 0, 2)
    with pytest.raises(m.MLMCError):      # n_defl out of range
        est.deflation_setup(0)
    w = m.TraceEstimator("wilson2d", 16, 2, 2, mass=0.1, field=gauge_field(16, seed=3),
                         block=4, n_vec=4, setup_sweeps=4, nb=8)
    with pytest.raises(m.MLMCError):      # non-Hermitian operator kind
        w.deflation_setup(4)
