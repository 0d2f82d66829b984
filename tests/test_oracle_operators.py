"""Pins for the oracle's operators and aggregation hierarchies."""
import itertools

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import hierarchy, operators
from workloads import gauge_field, varcoef_faces


@pytest.mark.parametrize("N", [5, 8, 16])
def test_poisson_closed_form_trace_matches_dense_inverse(N):
    A = operators.poisson2d(N).toarray()
    assert np.allclose(np.sort(np.linalg.eigvalsh(A)),
                       np.sort(operators.poisson2d_eigenvalues(N)), atol=1e-12)
    ref = np.trace(np.linalg.inv(A))
    assert abs(operators.poisson2d_trace_inverse(N) - ref) < 1e-12 * ref


def test_poisson_is_kron_form_of_example():
    # L^N = B kron I + I kron B, B = tridiag(-1, 2, -1) (Example 4.1)
    N = 7
    e = np.ones(N)
    B = np.diag(2 * e) - np.diag(e[:-1], 1) - np.diag(e[:-1], -1)
    L = np.kron(B, np.eye(N)) + np.kron(np.eye(N), B)
    assert np.array_equal(operators.poisson2d(N).toarray(), L)


@pytest.mark.parametrize("N,table", [(63, 1.96e4), (127, 8.01e4), (255, 3.24e5)])
def test_poisson_nnz_matches_table1(N, table):
    # Table 1 prints nnz to three digits; fine-level rows are the 5-point operator
    A = operators.poisson2d(N)
    assert A.nnz == operators.poisson2d_nnz(N)
    assert abs(A.nnz - table) <= 0.005 * table


def test_dst_solver_matches_dense():
    N = 12
    rng = np.random.default_rng(1)
    B = rng.standard_normal((N * N, 3))
    for diag, off in [(4.0, 1.0), (2.0, 0.5), (4.3, 1.0)]:
        A = operators.poisson2d(N, diag, off).toarray()
        ref = np.linalg.solve(A, B)
        assert np.allclose(operators.poisson2d_solve_dst(N, B, diag, off), ref,
                           rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("N", [4, 8, 64])
def test_aggregation_galerkin_is_half_poisson(N):
    # Remark 4.3 setting: orthonormal columns, R P = I; Galerkin of L^N is L^{N/2}/2
    P = hierarchy.aggregation_2d(N)
    assert (P.T @ P - sp.identity(P.shape[1])).count_nonzero() == 0
    Ac = hierarchy.galerkin(operators.poisson2d(N), P)
    assert abs(Ac - 0.5 * operators.poisson2d(N // 2)).max() == 0.0


def test_aggregation_3d_and_varcoef_galerkin_faces():
    # Coarse operator of 2x2x2 orthonormal aggregation is again 7-point, with face
    # coefficient (sum of the 4 fine faces between two aggregates)/8, shift kept.
    N = 4
    k = varcoef_faces(N, seed=3)
    A = operators.varcoef3d(N, k, 1e-3)
    P = hierarchy.aggregation_3d(N)
    assert np.allclose((P.T @ P).toarray(), np.eye(P.shape[1]), atol=1e-15)
    Ac = hierarchy.galerkin(A, P)
    Nc = N // 2
    kc = np.zeros((3, Nc, Nc, Nc + 1))
    for d, a, b, f in itertools.product(range(3), range(Nc), range(Nc), range(Nc + 1)):
        kc[d, a, b, f] = k[d, 2 * a:2 * a + 2, 2 * b:2 * b + 2, 2 * f].sum() / 8.0
    assert abs(Ac - operators.varcoef3d(Nc, kc, 1e-3)).max() < 1e-14


def test_varcoef_is_symmetric_positive_definite_and_row_sums():
    N = 4
    k = varcoef_faces(N, seed=5)
    A = operators.varcoef3d(N, k, 0.0).toarray()
    assert np.allclose(A, A.T)
    assert np.linalg.eigvalsh(A).min() > 0
    # an interior row sums to zero without the shift (pure diffusion)
    i = (1 * N + 1) * N + 1
    assert abs(A[i].sum()) < 1e-13


def _wilson_small(N=6, seed=2, m0=0.1):
    th = gauge_field(N, seed=seed)
    return operators.wilson2d(N, th, m0), th


def test_wilson_gamma5_hermiticity():
    # J S = S^* J (Example 4.3)
    D, _ = _wilson_small()
    J = operators.gamma5(36)
    assert abs(J @ D @ J - D.conj().T).max() < 1e-15


def test_wilson_block_form_is_gauge_laplacian():
    # eq. matrix_Schwinger: spin-ordered S = [[G, B], [-B^*, G]], G the gauge
    # Laplacian of Example 4.2; here D = S/2 with m0 = m/2.
    N, m0 = 5, 0.3
    D, th = _wilson_small(N, 4, m0)
    n = N * N
    perm = np.concatenate([2 * np.arange(n), 2 * np.arange(n) + 1])
    S = 2.0 * D.toarray()[np.ix_(perm, perm)]
    G = np.zeros((n, n), dtype=complex)
    for j in range(N):          # paper's row index i runs along x (Theta), j along y (Phi)
        for i in range(N):
            r = j * N + i
            G[r, r] += 4.0
            G[r, j * N + (i + 1) % N] -= np.exp(1j * th[0, j, i])
            G[r, ((j + 1) % N) * N + i] -= np.exp(1j * th[1, j, i])
            G[r, j * N + (i - 1) % N] -= np.exp(-1j * th[0, j, (i - 1) % N])
            G[r, ((j - 1) % N) * N + i] -= np.exp(-1j * th[1, (j - 1) % N, i])
    m = 2.0 * m0
    assert np.allclose(S[:n, :n], G + m * np.eye(n), atol=1e-14)
    assert np.allclose(S[n:, n:], G + m * np.eye(n), atol=1e-14)
    assert np.allclose(S[n:, :n], -S[:n, n:].conj().T, atol=1e-14)


def test_wilson_free_field_smallest_eigenvalue_is_m0():
    N, m0 = 8, 0.05
    D = operators.wilson2d(N, np.zeros((2, N, N)), m0).toarray()
    ev = np.linalg.eigvals(D)
    assert abs(np.abs(ev).min() - m0) < 1e-12


def test_wilson_trace_inverse_is_real():
    # eigenvalues in conjugate pairs => tr(D^-1) real
    D, _ = _wilson_small(6, 9, 0.2)
    t = np.trace(np.linalg.inv(D.toarray()))
    assert abs(t.imag) < 1e-12 * abs(t.real)


def test_wilson_testvector_aggregation_is_orthonormal_nearest_neighbour():
    N = 8
    th = gauge_field(N, seed=1)
    A, P = hierarchy.wilson_hierarchy(N, th, 0.1, levels=3, block=2, n_vec=4,
                                      sweeps=3, seed=1)
    for Pl in P:
        assert abs(Pl.conj().T @ Pl - sp.identity(Pl.shape[1])).max() < 1e-13
    # coarse operator couples each coarse site only to itself and its 4 neighbours
    Nc, dof = 4, 4
    Ac = A[1].toarray()
    for S in range(Nc * Nc):
        Y, X = divmod(S, Nc)
        allowed = {S, Y * Nc + (X + 1) % Nc, Y * Nc + (X - 1) % Nc,
                   ((Y + 1) % Nc) * Nc + X, ((Y - 1) % Nc) * Nc + X}
        for T in range(Nc * Nc):
            if T not in allowed:
                assert np.abs(Ac[S * dof:(S + 1) * dof, T * dof:(T + 1) * dof]).max() == 0
    # test vectors were smoothed: |A v|/|v| drops well below its value at the start
    _, V = hierarchy.testvector_aggregation(A[0], N, 2, 2, 4, 10, 1, 1)
    from oracle import philox
    for j in range(4):
        v0 = philox.z4(A[0].shape[0], 1, j, 1, stream=philox.STREAM_TESTVEC)
        r0 = np.linalg.norm(A[0] @ v0) / np.linalg.norm(v0)
        r = np.linalg.norm(A[0] @ V[:, j]) / np.linalg.norm(V[:, j])
        assert r < 0.6 * r0


def test_block_rbgs_sweep_fixed_point():
    # the exact solution is a fixed point of the block Gauss-Seidel sweep
    N = 6
    D, _ = _wilson_small(N, 3, 0.4)
    rng = np.random.default_rng(0)
    x = rng.standard_normal(D.shape[0]) + 1j * rng.standard_normal(D.shape[0])
    b = D @ x
    assert np.allclose(hierarchy.block_rbgs_sweep(D, x, N, 2, b), x, atol=1e-13)


def test_red_black_sweep_is_permuted_lexicographic_gauss_seidel():
    # with the unknowns ordered colour 0 first, a red-black sweep of a 5-point
    # (or 7-point) operator is the point Gauss-Seidel splitting
    # (D + L) x_new = b - U x of the permuted matrix
    import scipy.sparse.linalg as spla
    from oracle import operators
    rng = np.random.default_rng(3)
    cases = [(operators.poisson2d(7), hierarchy.site_coloring(7)),
             (operators.varcoef3d(4, np.exp(rng.standard_normal((3, 4, 4, 5))), 1e-3),
              hierarchy.site_coloring_3d(4))]
    for A, colour in cases:
        A = A.tocsr()
        n = A.shape[0]
        b, x = rng.standard_normal(n), rng.standard_normal(n)
        for reverse in (False, True):
            first = 1 if reverse else 0
            perm = np.concatenate([np.flatnonzero(colour == first),
                                   np.flatnonzero(colour != first)])
            Ap = A[perm][:, perm]
            rhs = b[perm] - sp.triu(Ap, 1) @ x[perm]
            xp = spla.spsolve_triangular(sp.tril(Ap).tocsr(), rhs, lower=True)
            ref = np.empty(n)
            ref[perm] = xp
            got = hierarchy.rbgs_sweeps(A, b, x, colour, 1, reverse=reverse)
            assert np.allclose(got, ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    # repeated sweeps converge to the solution of the SPD system
    A, colour = cases[0]
    b = rng.standard_normal(A.shape[0])
    x = hierarchy.rbgs_sweeps(A, b, np.zeros_like(b), colour, 200)
    assert np.linalg.norm(A @ x - b) <= 1e-10 * np.linalg.norm(b)


def test_spin_preserving_aggregation_keeps_the_spin_symmetry():
    """Example 4.3: J S = S^* J on the fine lattice; with the test vectors split
    by spin (2 n_vec coarse unknowns per aggregate) the coarse operators keep
    J_c A_c = A_c^* J_c, so their eigenvalues pair up as (lambda, conj(lambda))
    and tr(A_c^-1) is real; without the split they do not."""
    N, nv = 8, 2
    th = gauge_field(N, seed=4)
    A, P = hierarchy.wilson_hierarchy(N, th, 0.1, levels=3, block=2, n_vec=nv, sweeps=6,
                                      seed=1, spin_split=True)
    sides, dofs = [N, N // 2, N // 4], [2, 2 * nv, 2 * nv]
    for l in range(3):
        J = hierarchy.spin_sign(sides[l] ** 2, dofs[l])
        D = A[l]
        assert abs(J @ D @ J - D.conj().T).max() <= 1e-13 * abs(D).max(), l
        if l < 2:
            Jc = hierarchy.spin_sign(sides[l + 1] ** 2, dofs[l + 1])
            assert abs(J @ P[l] - P[l] @ Jc).max() == 0       # P maps spin to spin
            Pd = P[l].toarray()
            assert np.allclose(Pd.conj().T @ Pd, np.eye(Pd.shape[1]), atol=1e-13)
    tr = np.trace(np.linalg.inv(A[2].toarray()))
    assert abs(tr.imag) <= 1e-10 * abs(tr)
    ev = np.linalg.eigvals(A[1].toarray())
    gap = np.abs(ev.conj()[:, None] - ev[None, :]).min(axis=1)   # conj(lambda) is one too
    assert gap.max() <= 1e-9 * np.abs(ev).max()
    # the plain aggregation with the same number of coarse unknowns breaks it
    A2, _ = hierarchy.wilson_hierarchy(N, th, 0.1, levels=2, block=2, n_vec=2 * nv, sweeps=6,
                                       seed=1)
    J = hierarchy.spin_sign((N // 2) ** 2, 2 * nv)
    assert abs(J @ A2[1] @ J - A2[1].conj().T).max() > 1e-3 * abs(A2[1]).max()
