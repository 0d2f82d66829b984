"""Seeded synthetic operator data and workload parameter sets.

Stand-ins for the paper's matrices (Sec. 5): the Laplace example is generated
exactly; the thermalized Schwinger configuration and the pyAMG gauge-Laplacian
generator are not available, so U(1) link phases are drawn i.i.d. Gaussian;
the 3D diffusion batch uses log-normal face coefficients.
"""
import json
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))


def gauge_field(N, sigma=0.5, seed=1):
    """Link phases theta[mu, y, x] ~ N(0, sigma^2) i.i.d. on an N x N lattice."""
    rng = np.random.default_rng(np.random.SeedSequence([0x6A09E667, 3, seed, N]))
    return rng.normal(0.0, sigma, size=(2, N, N))


def varcoef_faces(N, sigma=1.0, seed=1000):
    """Face coefficients k = exp(g), g ~ N(0, sigma^2), shape [3, N, N, N+1]."""
    rng = np.random.default_rng(np.random.SeedSequence([0x6A09E667, 4, seed, N]))
    return np.exp(rng.normal(0.0, sigma, size=(3, N, N, N + 1)))


def batch_problem_sizes(count=32, lo=32, hi=128, step=8, seed=7):
    """Grid sides drawn uniformly from the multiples of `step` in [lo, hi]."""
    rng = np.random.default_rng(np.random.SeedSequence([0x6A09E667, 6, seed]))
    choices = np.arange(lo, hi + 1, step)
    return [int(v) for v in rng.choice(choices, size=count)]


def varcoef_levels(N, max_coarse=512):
    """Hierarchy depth of a 3D diffusion problem: halve the side while it is even
    and the level still has more than max_coarse cells."""
    L, side = 1, N
    while side % 2 == 0 and side ** 3 > max_coarse:
        side //= 2
        L += 1
    return L


def nn_init_weights(seed=1):
    """Initial weights of the learned smoother (3 layers of 3x3 convolutions,
    8 -> 16 -> 16 -> 4 channels, flattened W1, W2, W3 with shape [Co, Ci, 3, 3]):
    He-scaled normal draws (fan-in 9 Ci), the last layer scaled by 0.1."""
    rng = np.random.default_rng(np.random.SeedSequence([0x6A09E667, 7, seed]))
    out = []
    for k, (co, ci) in enumerate(((16, 8), (16, 16), (4, 16))):
        std = np.sqrt(2.0 / (9 * ci)) * (0.1 if k == 2 else 1.0)
        out.append(rng.normal(0.0, std, size=(co, ci, 3, 3)).ravel())
    return np.concatenate(out)


def graph_laplacian(n, degree=8.0, shift=1e-2, seed=1):
    """Shifted Laplacian L + shift*I of a random geometric graph, as CSR.

    n points uniform in the unit square, an edge (weight 1) between every two
    points closer than r = sqrt(degree / (pi n)), so the mean degree is about
    `degree` away from the boundary.  The points are numbered cell by cell
    (cells of side r, row-major, points in a cell by x) so that neighbours have
    nearby indices.  Returns a scipy.sparse CSR matrix with sorted indices.
    """
    import scipy.sparse as sp
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(np.random.SeedSequence([0x6A09E667, 8, seed, n]))
    pts = rng.random((n, 2))
    r = float(np.sqrt(degree / (np.pi * n)))
    cells = np.floor(pts / r).astype(np.int64)
    order = np.lexsort((pts[:, 0], cells[:, 0], cells[:, 1]))
    pts = pts[order]
    pairs = cKDTree(pts).query_pairs(r, output_type="ndarray")
    i, j = pairs[:, 0], pairs[:, 1]
    W = sp.coo_matrix((np.ones(2 * len(i)), (np.concatenate([i, j]), np.concatenate([j, i]))),
                      shape=(n, n)).tocsr()
    deg = np.asarray(W.sum(axis=1)).ravel()
    A = (sp.diags(deg + shift) - W).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    return A


def laplace_matrix(N):
    """The 2D 5-point Laplacian of Example 4.1 (diagonal 4, neighbours -1,
    Dirichlet), N^2 x N^2, unknown iy*N + ix, as a scipy CSR matrix."""
    import scipy.sparse as sp
    e = np.ones(N)
    T = sp.diags([-e[:-1], 2 * e, -e[:-1]], [-1, 0, 1])
    I = sp.identity(N)
    A = (sp.kron(T, I) + sp.kron(I, T)).tocsr()
    A.sort_indices()
    return A


def bilinear_prolongations(N, levels):
    """The levels-1 interpolation matrices of Example 4.1's hierarchy: grid sides
    N_{l+1} = floor(N_l / 2), coarse point I at fine point 2I+1, fine points
    weighted 1, 1/2, 1/4 (tensor product of 1D linear interpolation, Dirichlet
    boundary), unknowns iy*N + ix; scipy CSR matrices N_l^2 x N_{l+1}^2."""
    import scipy.sparse as sp
    out, n = [], N
    for _ in range(levels - 1):
        nc = n // 2
        rows, cols, vals = [], [], []
        for I in range(nc):
            for f, w in ((2 * I, 0.5), (2 * I + 1, 1.0), (2 * I + 2, 0.5)):
                if f < n:
                    rows.append(f)
                    cols.append(I)
                    vals.append(w)
        p = sp.csr_matrix((vals, (rows, cols)), shape=(n, nc))
        out.append(sp.kron(p, p).tocsr())
        n = nc
    return out


def wilson_mass(N):
    """m0 for the Wilson workload at lattice side N (tuned on the CPU so that the
    smallest |eigenvalue| is about 1e-2), or None if not tuned yet."""
    path = os.path.join(_HERE, "wilson_mass.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        table = json.load(f)
    v = table.get(str(N))
    return None if v is None else float(v["m0"])


# Workload parameter sets.  Level counts are L_mlmc (levels of the trace
# decomposition) and L_solver (levels of the multigrid solver).
WORKLOADS = {
    "poisson64_fp64": dict(
        kind="poisson2d", N=64, levels_mlmc=3, levels_solver=3, nb=128,
        precision="fp64", eps=1e-2, solve_tol=1e-12, seeds=[1, 2, 3, 4, 5]),
    "poisson1024_fp32ir": dict(
        kind="poisson2d", N=1024, levels_mlmc=6, levels_solver=6, nb=128,
        precision="fp32_ir64", eps=1e-3, solve_tol=1e-10, seeds=[1, 2, 3, 4, 5]),
    "wilson256_c64ir": dict(
        kind="wilson2d", N=256, levels_mlmc=3, levels_solver=3, nb=128,
        precision="fp32_ir64", eps=1e-3, solve_tol=1e-10, block=4, n_vec=8,
        setup_sweeps=20, theta_sigma=0.5, gauge_seed=1),
    "varcoef3d_batch32": dict(
        kind="varcoef3d", count=32, lo=32, hi=128, nb=64, precision="fp32_ir64",
        shift=1e-3, coef_sigma=1.0, solve_tol=1e-10),
    "wilson512_learned": dict(
        kind="wilson2d", N=512, levels_mlmc=3, levels_solver=4, nb=128,
        precision="fp32_ir64", eps=1e-3, solve_tol=1e-10, block=4, n_vec=8,
        setup_sweeps=20, theta_sigma=0.5, gauge_seed=1, learned=True),
    "laplace1023_bilinear_fp32ir": dict(
        kind="csr", N=1023, levels_mlmc=7, levels_solver=8, nb=128, precision="fp32_ir64",
        eps=1e-3, solve_tol=1e-10),
    "gauge256_c64ir": dict(
        kind="gauge2d", N=256, levels_mlmc=4, levels_solver=4, nb=128, precision="fp32_ir64",
        eps=1e-3, solve_tol=1e-10, n_vec=4, setup_sweeps=20, theta_sigma=0.3, gauge_seed=1,
        mass=0.0),
    "graph1m_fp32ir": dict(
        kind="csr", n=1 << 20, degree=8.0, shift=1e-2, graph_seed=1, levels_mlmc=4,
        levels_solver=4, nb=128, precision="fp32_ir64", eps=1e-3, solve_tol=1e-10),
}


def workload(name):
    return dict(WORKLOADS[name])
