"""Pins of the oracle's general decomposition (Sec. 4.1 with non-orthonormal
prolongations) on Example 4.1's hierarchy: 2D Laplacian, bilinear
interpolation, R = P^T, Galerkin coarse operators."""
import itertools
import os

import numpy as np
import scipy.sparse as sp

from oracle import hierarchy, mlmc, operators

HERE = os.path.dirname(os.path.abspath(__file__))


def test_nnz_matches_table_1():
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "laplace_bilinear_nnz_table1.txt"))
            if l.strip() and not l.startswith("#")]
    for N in (63, 127, 255):
        want = [(int(r[1]), int(r[2]), float(r[3])) for r in rows if int(r[0]) == N]
        A, _ = hierarchy.laplace_bilinear_hierarchy(N, len(want))
        for level, side, nnz in want:
            Al = A[level - 1]
            assert Al.shape[0] == side * side
            assert float("%.2e" % Al.nnz) == nnz, (N, level, Al.nnz, nnz)


def test_bilinear_weights_and_coarse_stencil():
    N = 15
    P = hierarchy.bilinear_interpolation(N)
    assert P.shape == (N * N, 7 * 7)
    # every fine point's weights sum to 1 away from the boundary; the weights
    # are 1 (coincident), 1/2 (on a grid line between two), 1/4 (cell centre)
    Pd = P.toarray()
    assert set(np.round(np.unique(Pd[Pd != 0]), 12)) == {0.25, 0.5, 1.0}
    iy, ix = np.divmod(np.arange(N * N), N)
    inner = (iy > 0) & (iy < N - 1) & (ix > 0) & (ix < N - 1)
    assert np.allclose(Pd[inner].sum(axis=1), 1.0)
    # not orthonormal: R P != I, so Remark 4.3 does not apply
    assert np.abs(Pd.T @ Pd - np.eye(49)).max() > 0.5
    # the Galerkin operator of the 5-point Laplacian is the 9-point stencil
    # c [-1 -2 -1; -2 12 -2; -1 -2 -1] at interior coarse points
    A, _ = hierarchy.laplace_bilinear_hierarchy(N, 2)
    Ac = A[1].toarray()
    c = 3 * 7 + 3                      # coarse point (3, 3)
    st = np.array([[Ac[c, c + dy * 7 + dx] for dx in (-1, 0, 1)] for dy in (-1, 0, 1)])
    assert np.allclose(st / st[1, 1], np.array([[-1, -2, -1], [-2, 12, -2], [-1, -2, -1]]) / 12)


def test_general_decomposition_telescopes_to_the_closed_form_trace():
    N, L = 31, 4
    A, P = hierarchy.laplace_bilinear_hierarchy(N, L)
    smp = mlmc.GeneralLevelSampler(A, P, complex_probe=False)
    Ph = [sp.identity(N * N, format="csr")]
    for l in range(L - 1):
        Ph.append(Ph[-1] @ P[l])
    # exact E[s_l] = tr(Phat_l A_l^-1 Rhat_l) - tr(Phat_{l+1} A_{l+1}^-1 Rhat_{l+1})
    t = [np.trace(Ph[l].toarray() @ np.linalg.inv(A[l].toarray()) @ Ph[l].toarray().T)
         for l in range(L)]
    assert abs(smp.coarse().real - t[-1]) <= 1e-10 * t[-1]
    total = sum(t[l] - t[l + 1] for l in range(L - 1)) + smp.coarse().real
    exact = operators.poisson2d_trace_inverse(N)
    assert abs(total - exact) <= 1e-10 * exact


def test_sample_mean_by_enumeration():
    # all 2^9 Rademacher probes of the 3 x 3 grid with its 1 x 1 coarse level:
    # the mean of x^T A^-1 x - x^T P A_c^-1 P^T x is tr(A^-1) - tr(P A_c^-1 P^T)
    A, P = hierarchy.laplace_bilinear_hierarchy(3, 2)
    smp = mlmc.GeneralLevelSampler(A, P, complex_probe=False)
    X = np.array(list(itertools.product((1.0, -1.0), repeat=9))).T
    a, b = smp.parts_for(1, X)
    Pd = P[0].toarray()
    exact = (np.trace(np.linalg.inv(A[0].toarray()))
             - np.trace(Pd @ np.linalg.inv(A[1].toarray()) @ Pd.T))
    assert abs((a - b).mean() - exact) <= 1e-13 * abs(exact)
    # the Philox samples follow the same formula
    s = smp.sample(1, 5, 0, 4)
    Xp = smp.probes(1, 5, 0, 4)
    a, b = smp.parts_for(1, Xp)
    assert np.allclose(s, a - b, rtol=0, atol=1e-14)


def test_orthonormal_hierarchy_gives_the_simplified_expectations():
    # with R P = I (2x2 aggregation) the general form's expected differences
    # are Remark 4.3's tr(A_l^-1) - tr(A_{l+1}^-1)
    N, L = 16, 3
    A, P = hierarchy.poisson_hierarchy(N, L)
    gen = mlmc.GeneralLevelSampler(A, P, complex_probe=False)
    assert abs(gen.coarse().real - np.trace(np.linalg.inv(A[-1].toarray()))) <= 1e-10 * abs(
        gen.coarse())
    X = np.array([mlmc.philox.rademacher(N * N, 3, k, 2) for k in range(4000)]).T
    a, b = gen.parts_for(2, X)
    want = np.trace(np.linalg.inv(A[1].toarray())) - np.trace(np.linalg.inv(A[2].toarray()))
    # a Monte-Carlo mean: within 5 standard errors
    d = a - b
    assert abs(d.mean() - want) <= 5 * d.std(ddof=1) / np.sqrt(len(d))
