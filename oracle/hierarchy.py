"""Aggregation hierarchies {A_l, P_l, R_l} with orthonormal P and R = P^H.

Test infrastructure (see the package docstring).

Sec. 4.1 defines the hierarchy: coarse operators A_{l+1} = R_l A_l P_l
(Petrov-Galerkin), P_l = R_l^* for Hermitian A.  Remark 4.3 treats the case
R_l P_l = I of aggregation with orthonormal columns, which is what every
hierarchy here is:
* 2D: 2x2 blocks of grid points form an aggregate; P has entry 1/2 in each of
  the four rows of an aggregate (orthonormal piecewise constants).
* 3D: 2x2x2 blocks, entries 1/sqrt(8).
* General sparse operators: greedy aggregates of the matrix graph, entries
  1/sqrt(|J|) (see the section at the end of this file).
* Wilson: b x b blocks of lattice sites form an aggregate; P restricted to one
  aggregate is an orthonormal basis of the span of n_vec near-null test
  vectors restricted to that aggregate (Example 4.3, the aggregation sketch:
  components of approximate small eigenvectors assembled over aggregates and
  orthogonalised).
The Galerkin product is formed here as a plain sparse product R A P.
"""
import numpy as np
import scipy.sparse as sp

from . import philox


def aggregation_2d(N):
    """Orthonormal 2x2 aggregation P in R^{N^2 x (N/2)^2} (index iy*N + ix)."""
    assert N % 2 == 0
    Nc = N // 2
    iy, ix = np.divmod(np.arange(N * N), N)
    cols = (iy // 2) * Nc + (ix // 2)
    return sp.csr_matrix((np.full(N * N, 0.5), (np.arange(N * N), cols)),
                         shape=(N * N, Nc * Nc))


def aggregation_3d(N):
    """Orthonormal 2x2x2 aggregation P in R^{N^3 x (N/2)^3}."""
    assert N % 2 == 0
    Nc = N // 2
    i = np.arange(N ** 3)
    z, rem = np.divmod(i, N * N)
    y, x = np.divmod(rem, N)
    cols = ((z // 2) * Nc + (y // 2)) * Nc + (x // 2)
    return sp.csr_matrix((np.full(N ** 3, 1.0 / np.sqrt(8.0)), (i, cols)),
                         shape=(N ** 3, Nc ** 3))


def galerkin(A, P):
    """A_{l+1} = R_l A_l P_l with R_l = P_l^H (Sec. 4.1)."""
    return (P.conj().T @ A @ P).tocsr()


def poisson_hierarchy(N, levels, diag=4.0, off=1.0):
    """A_1..A_levels and P_1..P_{levels-1} for the 2D Poisson operator."""
    from .operators import poisson2d
    A = [poisson2d(N, diag, off)]
    P = []
    n = N
    for _ in range(levels - 1):
        P.append(aggregation_2d(n))
        A.append(galerkin(A[-1], P[-1]))
        n //= 2
    return A, P


def varcoef_hierarchy(N, k, shift, levels):
    """A_1..A_levels and P_1..P_{levels-1} for the 3D diffusion operator."""
    from .operators import varcoef3d
    A = [varcoef3d(N, k, shift)]
    P = []
    n = N
    for _ in range(levels - 1):
        P.append(aggregation_3d(n))
        A.append(galerkin(A[-1], P[-1]))
        n //= 2
    return A, P


# ---------------------------------------------------------------------------
# Wilson: test-vector aggregation
# ---------------------------------------------------------------------------

def site_coloring(N):
    """Red (0) / black (1) colour of each site of an N x N lattice: (x+y) mod 2."""
    y, x = np.divmod(np.arange(N * N), N)
    return (x + y) % 2


def site_coloring_3d(N):
    """Red (0) / black (1) colour of each cell of an N^3 grid: (x+y+z) mod 2,
    cell index (z*N + y)*N + x."""
    z, rest = np.divmod(np.arange(N ** 3), N * N)
    y, x = np.divmod(rest, N)
    return (x + y + z) % 2


def coloured_gs_sweep(A, v, colour, b, order=(0, 1)):
    """One block Gauss-Seidel sweep over the colour classes listed in `order`.

    For each class m in turn the unknowns of m are solved exactly with the
    others held: v_m <- A_mm^{-1} (b_m - A_{m,rest} v_rest).  With a red-black
    colouring of a nearest-neighbour operator (or any proper colouring of the
    matrix graph) A_mm is (block) diagonal.
    """
    A = A.tocsr()
    for c in order:
        m = colour == c
        Amm = A[m][:, m]
        rhs = b[m] - A[m][:, ~m] @ v[~m]
        v = v.copy()
        v[m] = sp.linalg.spsolve(Amm.tocsc(), rhs)
    return v


def rbgs_sweeps(A, b, x, colour, sweeps, reverse=False):
    """`sweeps` red-black sweeps from x; reverse: colour 1 first (the
    post-smoothing order that keeps a V-cycle symmetric)."""
    order = (1, 0) if reverse else (0, 1)
    for _ in range(sweeps):
        x = coloured_gs_sweep(A, x, colour, b, order)
    return x


def block_rbgs_sweep(A, v, N, dof, b=None):
    """One red-black block Gauss-Seidel sweep for A v = b (b = 0 by default).

    Sites of colour 0 are updated first, then colour 1; each site's dof x dof
    diagonal block is solved exactly: v_S <- A_SS^{-1} (b_S - A_{S,rest} v_rest).
    """
    n = A.shape[0]
    if b is None:
        b = np.zeros(n, dtype=A.dtype)
    return coloured_gs_sweep(A, v, np.repeat(site_coloring(N), dof), b)


def orthonormal_basis(V):
    """Q of V = Q R with R upper triangular and a real positive diagonal."""
    Q, R = np.linalg.qr(V)
    d = np.diag(R)
    phase = d / np.abs(d)
    return Q * np.conj(phase)[None, :]


def testvector_aggregation(A, N, dof, block, n_vec, sweeps, seed, level, spin_split=False):
    """Aggregation P for a lattice operator with `dof` unknowns per site.

    Test vectors: n_vec Z4 start vectors (stream 2, sample j, this level), then
    `sweeps` red-black block Gauss-Seidel sweeps on A v = 0.  Aggregates are
    block x block site squares; within each, the n_vec restricted vectors are
    orthonormalised (QR with positive diagonal).  Coarse site S = Y*Nc + X,
    coarse unknown S*nc + c.

    spin_split (the spin-structure-preserving aggregation of Example 4.3):
    within each aggregate the test vectors are restricted separately to the
    unknowns of each spin (a site's first dof/2 unknowns carry spin 0, the rest
    spin 1; on the fine lattice the two spin components) and each part is
    orthonormalised on its own, so each aggregate gets nc = 2 n_vec coarse
    unknowns, the first n_vec on spin 0 and the rest on spin 1, and P maps
    spin to spin.  Otherwise nc = n_vec.
    """
    n = A.shape[0]
    assert n == N * N * dof and N % block == 0
    V = np.empty((n, n_vec), dtype=np.complex128)
    for j in range(n_vec):
        v = philox.z4(n, seed, j, level, stream=philox.STREAM_TESTVEC)
        for _ in range(sweeps):
            v = block_rbgs_sweep(A, v, N, dof)
        V[:, j] = v
    Nc = N // block
    nc = 2 * n_vec if spin_split else n_vec
    half = dof // 2
    rows, cols, vals = [], [], []
    for Y in range(Nc):
        for X in range(Nc):
            S = Y * Nc + X
            parts = [[] for _ in range(2 if spin_split else 1)]
            for yy in range(block):
                for xx in range(block):
                    s = (Y * block + yy) * N + (X * block + xx)
                    for a in range(dof):
                        parts[a // half if spin_split else 0].append(s * dof + a)
            for p, idx in enumerate(parts):
                Q = orthonormal_basis(V[idx, :])
                for r, i in enumerate(idx):
                    for j in range(n_vec):
                        rows.append(i)
                        cols.append(S * nc + p * n_vec + j)
                        vals.append(Q[r, j])
    P = sp.csr_matrix((np.array(vals), (rows, cols)), shape=(n, Nc * Nc * nc))
    return P, V


def wilson_hierarchy(N, theta, m0, levels, block=4, n_vec=8, sweeps=20, seed=1,
                     spin_split=False):
    """A_1..A_levels, P_1..P_{levels-1} for the Wilson operator (Example 4.3);
    spin_split: spin-structure-preserving aggregation on every level."""
    from .operators import wilson2d
    A = [wilson2d(N, theta, m0)]
    P = []
    n_side, dof = N, 2
    for lvl in range(1, levels):
        Pl, _ = testvector_aggregation(A[-1], n_side, dof, block, n_vec, sweeps,
                                       seed, lvl, spin_split)
        P.append(Pl)
        A.append(galerkin(A[-1], Pl))
        n_side //= block
        dof = 2 * n_vec if spin_split else n_vec
    return A, P


def gauge_hierarchy(N, theta, mass, levels, block=4, n_vec=4, sweeps=20, seed=1):
    """A_1..A_levels, P_1..P_{levels-1} for the gauge Laplacian (Example 4.2):
    test-vector aggregation as for the Wilson operator, one unknown per fine
    site (the example's adaptive smoothed aggregation is not reproduced)."""
    from .operators import gauge_laplacian
    A = [gauge_laplacian(N, theta, mass)]
    P = []
    n_side, dof = N, 1
    for lvl in range(1, levels):
        Pl, _ = testvector_aggregation(A[-1], n_side, dof, block, n_vec, sweeps, seed, lvl)
        P.append(Pl)
        A.append(galerkin(A[-1], Pl))
        n_side //= block
        dof = n_vec
    return A, P


def spin_sign(n_sites, dof):
    """J on a lattice level: +1 on a site's first dof/2 unknowns (spin 0), -1 on
    the rest; on the fine lattice (dof 2) the gamma5 of Example 4.3."""
    return sp.diags(np.tile(np.repeat([1.0, -1.0], dof // 2), n_sites))


# ---------------------------------------------------------------------------
# General sparse operators: aggregation and colouring on the matrix graph
# ---------------------------------------------------------------------------
#
# Sec. 4.1 takes the hierarchy as given: aggregates of unknowns and, on each,
# the coarse basis.  For an operator given only as a sparse matrix (the
# gauge-Laplacian and graph examples of Sec. 5 leave this to an algebraic
# multigrid package), the aggregates here come from plain two-pass greedy
# aggregation on the graph of A (j is a neighbour of i when i != j and
# a_ij != 0), visiting unknowns in index order, and P holds the orthonormal
# piecewise constants 1/sqrt(|J|) of each aggregate J.  The smoother's colour
# classes come from first-fit greedy colouring of the same graph in index
# order.  Plain Python loops: for the small cases of the tests.

def matrix_graph(A):
    """Neighbour lists [(j, |a_ij|), ...] of every row, in column order."""
    A = sp.csr_matrix(A).sorted_indices()
    out = []
    for i in range(A.shape[0]):
        lo, hi = A.indptr[i], A.indptr[i + 1]
        out.append([(int(j), abs(v)) for j, v in zip(A.indices[lo:hi], A.data[lo:hi])
                    if j != i and v != 0])
    return out


def greedy_aggregation(A, return_seeds=False):
    """Aggregate number of every unknown (numbered in order of creation).

    Pass 1: an unknown whose neighbours are all still unassigned founds an
    aggregate with them.  Pass 2: every unknown left over joins the pass-1
    aggregate of its neighbour with the largest |a_ij| (the smallest j among
    equal ones); after pass 1 each such unknown has a neighbour in a pass-1
    aggregate, since otherwise it would have founded one.  return_seeds: also
    the founding unknown of every aggregate.
    """
    nbrs = matrix_graph(A)
    n = len(nbrs)
    agg = [-1] * n
    seeds = []
    for i in range(n):
        if agg[i] < 0 and all(agg[j] < 0 for j, _ in nbrs[i]):
            agg[i] = len(seeds)
            for j, _ in nbrs[i]:
                agg[j] = len(seeds)
            seeds.append(i)
    first = list(agg)
    for i in range(n):
        if agg[i] < 0:
            best = None
            for j, w in nbrs[i]:
                if first[j] >= 0 and (best is None or w > best[0]):
                    best = (w, j)
            agg[i] = first[best[1]]
    agg = np.array(agg, dtype=np.int64)
    return (agg, np.array(seeds, dtype=np.int64)) if return_seeds else agg


def aggregate_prolongation(agg):
    """P with entry 1/sqrt(|J|) in row i, column J = agg[i] (orthonormal columns)."""
    agg = np.asarray(agg)
    n, nc = len(agg), int(agg.max()) + 1
    size = np.bincount(agg, minlength=nc)
    assert np.all(size > 0), "aggregate numbers must be 0..nc-1 without gaps"
    return sp.csr_matrix((1.0 / np.sqrt(size[agg]), (np.arange(n), agg)), shape=(n, nc))


def first_fit_coloring(A):
    """Colour of every unknown: the smallest colour not taken by a neighbour
    with a smaller index (unknowns visited in index order)."""
    nbrs = matrix_graph(A)
    colour = [0] * len(nbrs)
    for i, nb in enumerate(nbrs):
        used = {colour[j] for j, _ in nb if j < i}
        c = 0
        while c in used:
            c += 1
        colour[i] = c
    return np.array(colour, dtype=np.int64)


def multicolour_gs_sweeps(A, b, x, colour, sweeps, reverse=False):
    """`sweeps` Gauss-Seidel sweeps over the colour classes 0, 1, ... (reverse:
    from the last class down, the post-smoothing order)."""
    C = int(np.max(colour)) + 1
    order = tuple(range(C - 1, -1, -1)) if reverse else tuple(range(C))
    for _ in range(sweeps):
        x = coloured_gs_sweep(A, x, colour, b, order)
    return x


def csr_hierarchy(A, levels, aggs=None):
    """A_1..A_levels, P_1..P_{levels-1} of a sparse operator: greedy aggregation
    on every level, or the given aggregate maps aggs[l] (level l+1 unknown ->
    aggregate), orthonormal piecewise-constant P, Galerkin coarse operators."""
    def canonical(M):     # storage order only: columns ascending, no zeros
        M = sp.csr_matrix(M, dtype=np.float64)
        M.sum_duplicates()
        M.eliminate_zeros()
        return M.sorted_indices()
    A = [canonical(A)]
    P = []
    for l in range(levels - 1):
        agg = greedy_aggregation(A[-1]) if aggs is None else np.asarray(aggs[l])
        P.append(aggregate_prolongation(agg))
        A.append(canonical(galerkin(A[-1], P[-1])))
    return A, P


# ---------------------------------------------------------------------------
# Example 4.1: bilinear interpolation (non-orthonormal P, R = P^T)
# ---------------------------------------------------------------------------

def linear_interpolation_1d(Nf):
    """p in R^{Nf x Nc}, Nc = floor(Nf/2): coarse point I sits at fine point
    2I+1; fine point 2I+1 takes it with weight 1, fine points 2I and 2I+2 with
    weight 1/2 (Dirichlet: the boundary values are zero)."""
    Nc = Nf // 2
    p = sp.lil_matrix((Nf, Nc))
    for I in range(Nc):
        p[2 * I + 1, I] = 1.0
        p[2 * I, I] = 0.5
        if 2 * I + 2 < Nf:
            p[2 * I + 2, I] = 0.5
    return p.tocsr()


def bilinear_interpolation(Nf):
    """Standard bilinear interpolation from the Nc x Nc to the Nf x Nf grid
    (Example 4.1), unknowns numbered iy*N + ix: the tensor product of the 1D
    linear interpolations, so fine points take weights 1, 1/2 and 1/4."""
    p = linear_interpolation_1d(Nf)
    return sp.kron(p, p).tocsr()


def laplace_bilinear_hierarchy(N, levels):
    """Example 4.1's hierarchy: A_1 the 5-point Laplacian (diagonal 4), P_l the
    bilinear interpolation, R_l = P_l^T, A_{l+1} = R_l A_l P_l; N_{l+1} = floor(N_l/2)."""
    from .operators import poisson2d
    A = [poisson2d(N)]
    P = []
    n = N
    for _ in range(levels - 1):
        P.append(bilinear_interpolation(n))
        Ac = galerkin(A[-1], P[-1])
        Ac.eliminate_zeros()
        A.append(Ac.sorted_indices())
        n //= 2
    return A, P
