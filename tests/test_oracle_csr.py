"""Pins of the oracle's hierarchy for operators given as sparse matrices:
greedy aggregation, first-fit colouring, the multicolour Gauss-Seidel sweep and
the Galerkin hierarchy with orthonormal piecewise-constant aggregation
(Sec. 4.1; Remark 4.3 for R P = I)."""
import itertools

import numpy as np
import scipy.sparse as sp

from oracle import hierarchy, operators
from oracle.mlmc import coarse_trace
from workloads import graph_laplacian


def _path(n, d=2.5):
    return sp.diags([-1.0, d, -1.0], [-1, 0, 1], shape=(n, n)).tocsr()


def _closed_nbhd(A, i):
    A = sp.csr_matrix(A)
    lo, hi = A.indptr[i], A.indptr[i + 1]
    return {i} | {int(j) for j, v in zip(A.indices[lo:hi], A.data[lo:hi]) if v != 0}


def test_aggregation_of_a_path_by_hand():
    # path 0-1-...-6: 0 founds {0,1}; 1 and 2 have an assigned neighbour; 3
    # founds {2,3,4}; 4, 5 blocked; 6 founds {5,6}; nothing is left for pass 2
    agg, seeds = hierarchy.greedy_aggregation(_path(7), return_seeds=True)
    assert agg.tolist() == [0, 0, 1, 1, 1, 2, 2]
    assert seeds.tolist() == [0, 3, 6]
    # path of 5: 0 founds {0,1}, 2 is blocked, 3 founds {2,3,4}
    assert hierarchy.greedy_aggregation(_path(5)).tolist() == [0, 0, 1, 1, 1]
    # pass 2 on a path of 4 with seeds 0 and 3 ({0,1}, {2,3}): no leftovers;
    # a star's centre takes everything
    star = sp.lil_matrix((5, 5))
    for i in range(5):
        star[i, i] = 4.0
    for j in range(1, 5):
        star[0, j] = star[j, 0] = -1.0
    assert hierarchy.greedy_aggregation(star.tocsr()).tolist() == [0, 0, 0, 0, 0]


def test_pass_two_joins_the_strongest_neighbour():
    # edges 0-1, 1-2, 2-4, 3-4: 0 founds {0,1}; 2 is blocked by 1; 3 founds
    # {3,4}; 2 is left over with neighbours 1 (weight 1) and 4 (weight 5): it
    # joins 4's aggregate
    A = sp.lil_matrix((5, 5))
    for i in range(5):
        A[i, i] = 10.0
    for i, j, w in [(0, 1, 1.0), (1, 2, 1.0), (2, 4, 5.0), (3, 4, 1.0)]:
        A[i, j] = A[j, i] = -w
    assert hierarchy.greedy_aggregation(A.tocsr()).tolist() == [0, 0, 1, 1, 1]
    A[2, 4] = A[4, 2] = -0.5    # now 1 is the stronger neighbour
    assert hierarchy.greedy_aggregation(A.tocsr()).tolist() == [0, 0, 0, 1, 1]


def test_aggregation_characterised_on_a_random_graph():
    A = graph_laplacian(400, degree=6.0, seed=3)
    n = A.shape[0]
    agg, seeds = hierarchy.greedy_aggregation(A, return_seeds=True)
    N = [_closed_nbhd(A, i) for i in range(n)]
    sset = set(seeds.tolist())
    # the seeds are the first-in-index-order maximal set of unknowns whose
    # closed neighbourhoods are pairwise disjoint
    for a, s in enumerate(seeds):
        assert all(not (N[s] & N[t]) for t in seeds[:a])
        assert all(agg[j] == a for j in N[s])
    for v in range(n):
        if v not in sset:
            assert any(N[v] & N[t] for t in seeds if t < v), v
    # every aggregate is connected, every unknown assigned, numbers 0..nc-1
    assert agg.min() == 0 and set(agg.tolist()) == set(range(len(seeds)))
    covered = set().union(*(N[s] for s in seeds))
    for v in range(n):
        if v not in covered:    # pass 2: joined through a covered neighbour
            assert any(agg[j] == agg[v] and j in covered for j in N[v] - {v}), v
    P = hierarchy.aggregate_prolongation(agg)
    assert np.allclose((P.T @ P).toarray(), np.eye(P.shape[1]), atol=1e-15)


def test_first_fit_colouring():
    for N in (4, 7, 8):
        A = operators.poisson2d(N)
        assert np.array_equal(hierarchy.first_fit_coloring(A), hierarchy.site_coloring(N))
    assert hierarchy.first_fit_coloring(_path(6)).tolist() == [0, 1, 0, 1, 0, 1]
    A = graph_laplacian(400, degree=8.0, seed=5)
    col = hierarchy.first_fit_coloring(A)
    C = sp.coo_matrix(A)
    off = C.row != C.col
    assert np.all(col[C.row[off]] != col[C.col[off]])        # proper
    for i in range(A.shape[0]):                              # first fit
        earlier = {int(col[j]) for j in _closed_nbhd(A, i) if j < i}
        assert set(range(col[i])) <= earlier, i


def test_multicolour_sweep_fixed_point_and_convergence():
    A = graph_laplacian(300, degree=8.0, shift=0.5, seed=2)
    col = hierarchy.first_fit_coloring(A)
    assert col.max() >= 3          # more than two classes
    rng = np.random.default_rng(0)
    b = rng.standard_normal(A.shape[0])
    xs = sp.linalg.spsolve(A.tocsc(), b)
    for rev in (False, True):
        x1 = hierarchy.multicolour_gs_sweeps(A, b, xs, col, 1, rev)
        assert np.max(np.abs(x1 - xs)) < 1e-12 * np.max(np.abs(xs))
    x = hierarchy.multicolour_gs_sweeps(A, b, np.zeros_like(b), col, 150)
    assert np.max(np.abs(x - xs)) < 1e-8 * np.max(np.abs(xs))
    # a diagonal operator: one colour, one sweep solves it
    D = sp.diags(np.arange(1.0, 6.0)).tocsr()
    c1 = hierarchy.first_fit_coloring(D)
    assert c1.tolist() == [0] * 5
    x = hierarchy.multicolour_gs_sweeps(D, np.ones(5), np.zeros(5), c1, 1)
    assert np.allclose(x, 1.0 / np.arange(1.0, 6.0), rtol=0, atol=1e-15)


def test_given_aggregates_reproduce_the_grid_hierarchies():
    N, L = 16, 3
    A, P = hierarchy.poisson_hierarchy(N, L)
    Ac, Pc = hierarchy.csr_hierarchy(A[0], L, aggs=[p.indices for p in P])
    for a, b in zip(A, Ac):
        assert abs(a - b).max() <= 1e-14
    for p, q in zip(P, Pc):
        assert abs(p - q).max() == 0
    from workloads import varcoef_faces
    k = varcoef_faces(8, seed=3)
    A, P = hierarchy.varcoef_hierarchy(8, k, 1e-3, 2)
    Ac, Pc = hierarchy.csr_hierarchy(A[0], 2, aggs=[P[0].indices])
    assert abs(A[1] - Ac[1]).max() <= 1e-14 * abs(A[1]).max()


def test_graph_hierarchy_galerkin_and_telescoping():
    A0 = graph_laplacian(500, degree=8.0, shift=1e-2, seed=4)
    A, P = hierarchy.csr_hierarchy(A0, 3)
    for l in range(2):
        assert A[l + 1].shape[0] < A[l].shape[0] / 3        # coarsens
        R = P[l].T
        assert np.allclose((R @ P[l]).toarray(), np.eye(P[l].shape[1]), atol=1e-15)
        Ad = A[l + 1].toarray()
        assert np.abs(Ad - Ad.T).max() <= 1e-14 * np.abs(Ad).max()
        assert np.linalg.eigvalsh(Ad).min() > 0
    # A_1 1 = shift 1 and P_1 sqrt(|J|) = 1, so A_2 sqrt(|J|) = shift sqrt(|J|)
    sq = np.sqrt(np.bincount(P[0].indices))
    assert np.allclose(A[1] @ sq, 1e-2 * sq, rtol=0, atol=1e-12)
    # E[s_l] = tr(A_l^-1) - tr(A_{l+1}^-1) (R P = I), so the level means and the
    # coarsest term sum to tr(A^-1)
    tr = [np.trace(np.linalg.inv(a.toarray())) for a in A]
    total = sum(tr[l] - np.trace(P[l] @ np.linalg.inv(A[l + 1].toarray()) @ P[l].T)
                for l in range(2)) + coarse_trace(A[2]).real
    assert abs(total - tr[0]) <= 1e-10 * tr[0]


def test_level_difference_mean_by_enumeration():
    # all 2^n Rademacher probes on a 12-unknown graph: the sample mean of
    # x^T A^-1 x - (R x)^T A_c^-1 (R x) is tr(A^-1) - tr(A_c^-1) exactly
    A0 = graph_laplacian(12, degree=3.0, shift=0.3, seed=6)
    A, P = hierarchy.csr_hierarchy(A0, 2)
    Ai, Aci = np.linalg.inv(A[0].toarray()), np.linalg.inv(A[1].toarray())
    R = P[0].T.toarray()
    X = np.array(list(itertools.product((1.0, -1.0), repeat=12))).T
    Xc = R @ X
    s = np.einsum("ik,ik->k", X, Ai @ X) - np.einsum("ik,ik->k", Xc, Aci @ Xc)
    assert abs(s.mean() - (np.trace(Ai) - np.trace(Aci))) <= 1e-12 * np.trace(Ai)
