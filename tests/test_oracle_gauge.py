"""Pins of the oracle's gauge Laplacian (Example 4.2) and its test-vector
aggregation hierarchy."""
import os

import numpy as np
import scipy.sparse as sp

from oracle import hierarchy, mlmc, operators
from workloads import gauge_field

HERE = os.path.dirname(os.path.abspath(__file__))


def test_nnz_and_sizes_match_table_2():
    for line in open(os.path.join(HERE, "golden", "gauge_laplace_nnz_table2.txt")):
        if line.startswith("#") or not line.strip():
            continue
        N, n, nnz = (int(v) for v in line.split())
        A = operators.gauge_laplacian(N, gauge_field(N, sigma=0.3, seed=1))
        assert A.shape == (n, n) and A.nnz == nnz


def test_hermitian_positive_definite_and_free_field():
    N = 12
    A = operators.gauge_laplacian(N, gauge_field(N, sigma=0.3, seed=2))
    assert abs(A - A.conj().T).max() == 0
    assert np.linalg.eigvalsh(A.toarray()).min() > 0
    # zero phases: the periodic Laplacian (+ m) with its closed-form spectrum
    F = operators.gauge_laplacian(N, np.zeros((2, N, N)), mass=0.25)
    tr = np.trace(np.linalg.inv(F.toarray())).real
    assert abs(tr - operators.gauge_laplacian_free_trace(N, 0.25)) <= 1e-12 * tr
    # a row by hand: site (x, y) = (2, 3) couples to its four neighbours
    th = gauge_field(N, sigma=0.3, seed=2)
    s = 3 * N + 2
    assert np.isclose(A[s, s], 4.0)
    assert np.isclose(A[s, 3 * N + 3], -np.exp(1j * th[0, 3, 2]))
    assert np.isclose(A[s, 3 * N + 1], -np.exp(-1j * th[0, 3, 1]))
    assert np.isclose(A[s, 4 * N + 2], -np.exp(1j * th[1, 3, 2]))
    assert np.isclose(A[s, 2 * N + 2], -np.exp(-1j * th[1, 2, 2]))


def test_gauge_covariance():
    # a random gauge transformation changes the links but not the spectrum or
    # the trace of the inverse
    N = 10
    th = gauge_field(N, sigma=0.3, seed=3)
    phi = np.random.default_rng(4).uniform(-np.pi, np.pi, N * N)
    A = operators.gauge_laplacian(N, th)
    B = operators.gauge_laplacian(N, operators.gauge_transform(N, th, phi))
    D = sp.diags(np.exp(1j * phi))
    assert abs(B - D @ A @ D.conj().T).max() <= 1e-14
    assert np.allclose(np.linalg.eigvalsh(A.toarray()), np.linalg.eigvalsh(B.toarray()),
                       atol=1e-12)
    ta = np.trace(np.linalg.inv(A.toarray()))
    tb = np.trace(np.linalg.inv(B.toarray()))
    assert abs(ta - tb) <= 1e-12 * abs(ta)


def test_hierarchy_is_orthonormal_and_telescopes():
    N, L = 16, 3
    th = gauge_field(N, sigma=0.3, seed=5)
    A, P = hierarchy.gauge_hierarchy(N, th, 0.0, L, block=2, n_vec=2, sweeps=6)
    assert [a.shape[0] for a in A] == [256, 8 * 8 * 2, 4 * 4 * 2]
    for l in range(L - 1):
        Pd = P[l].toarray()
        assert np.allclose(Pd.conj().T @ Pd, np.eye(Pd.shape[1]), atol=1e-13)
        Ad = A[l + 1].toarray()
        assert np.abs(Ad - Ad.conj().T).max() <= 1e-13 * np.abs(Ad).max()
        assert np.linalg.eigvalsh(Ad).min() > 0
    smp = mlmc.LevelSampler(A, P, complex_probe=True)
    t = [np.trace(np.linalg.inv(a.toarray())).real for a in A]
    total = sum(t[l] - t[l + 1] for l in range(L - 1)) + smp.coarse().real
    assert abs(total - t[0]) <= 1e-12 * t[0]
