"""Sparse FP64 operators A = A_1, assembled entry by entry.

Test infrastructure (see the package docstring).

* 2D Poisson, Example 4.1: L^N = B kron I + I kron B with B = tridiag(-1, 2, -1),
  i.e. 4 on the diagonal and -1 for each of the (up to) four grid neighbours,
  Dirichlet boundary.  Grid index i = iy*N + ix.  Its eigenvalues are known in
  closed form (the example says so), which gives tr((L^N)^-1) exactly.
* Wilson-like 2-spin U(1) operator, after Example 4.3 (eq. schwinger_coupling,
  with the paper's sigma_1 and sigma_2), halved and with m0 = m/2:
      D = (m0+2) I - 1/2 sum_mu [ (I - sigma_mu) U_mu(x) delta_{x+mu}
                                 + (I + sigma_mu) conj(U_mu(x-mu)) delta_{x-mu} ]
  on an N x N periodic lattice.  Site s = y*N + x, unknown 2*s + spin.
  U_mu(x) = exp(i theta[mu, y, x]); mu = 0 is the x direction (the paper's
  Theta, paired with sigma_1), mu = 1 the y direction (Phi, sigma_2).
* Gauge Laplacian, Example 4.2: one unknown per site of an N x N periodic
  lattice, row s = (x, y):
      (4 + m) u_s - U_0(s) u_{s+x} - U_1(s) u_{s+y}
                  - conj(U_0(s-x)) u_{s-x} - conj(U_1(s-y)) u_{s-y},
  U_mu(s) = exp(i theta[mu, y, x]) (the example's Theta for mu = 0, Phi for
  mu = 1); Hermitian, positive definite for m > 0 or non-trivial phases.
* 3D 7-point variable-coefficient diffusion with Dirichlet faces:
      A = sum_interior faces k_f (e_i - e_j)(e_i - e_j)^T
        + sum_boundary faces k_f e_i e_i^T + shift * I,
  cell i = (z*N + y)*N + x; face coefficients k[d][a][b][f] for direction d
  (0 = x, 1 = y, 2 = z), the two transverse indices (a, b) and face f = 0..N
  along d, face f lying between cells f-1 and f (f = 0 and f = N are the
  boundary faces).
"""
import numpy as np
import scipy.sparse as sp

SIGMA1 = np.array([[0.0, 1.0], [1.0, 0.0]], dtype=np.complex128)
SIGMA2 = np.array([[0.0, 1.0j], [-1.0j, 0.0]], dtype=np.complex128)  # paper's sign


def poisson2d(N, diag=4.0, off=1.0):
    """A = diag*I - off*(grid neighbours) on an N x N Dirichlet grid (Example 4.1)."""
    rows, cols, vals = [], [], []
    for iy in range(N):
        for ix in range(N):
            i = iy * N + ix
            rows.append(i)
            cols.append(i)
            vals.append(diag)
            for dx, dy in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                jx, jy = ix + dx, iy + dy
                if 0 <= jx < N and 0 <= jy < N:
                    rows.append(i)
                    cols.append(jy * N + jx)
                    vals.append(-off)
    n = N * N
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


def poisson2d_eigenvalues(N):
    """Eigenvalues of L^N: 4 sin^2(j pi / (2(N+1))) + 4 sin^2(k pi / (2(N+1)))."""
    t = 4.0 * np.sin(np.arange(1, N + 1) * np.pi / (2.0 * (N + 1))) ** 2
    return (t[:, None] + t[None, :]).reshape(-1)


def poisson2d_trace_inverse(N):
    """T(N) = tr((L^N)^-1) as the sum of reciprocal eigenvalues (Example 4.1)."""
    return float(np.sum(1.0 / poisson2d_eigenvalues(N)))


def poisson2d_nnz(N):
    """Number of nonzeros of the 5-point L^N: 5N^2 - 4N."""
    return 5 * N * N - 4 * N


def wilson2d(N, theta, m0):
    """Wilson-like 2-spin operator on an N x N periodic lattice (see module doc).

    theta: float array [2, N, N] of link phases theta[mu, y, x].
    """
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.shape == (2, N, N)
    I2 = np.eye(2, dtype=np.complex128)
    fwd = [I2 - SIGMA1, I2 - SIGMA2]
    bwd = [I2 + SIGMA1, I2 + SIGMA2]
    rows, cols, vals = [], [], []

    def put(s_row, s_col, blk):
        for a in range(2):
            for b in range(2):
                if blk[a, b] != 0:
                    rows.append(2 * s_row + a)
                    cols.append(2 * s_col + b)
                    vals.append(blk[a, b])

    for y in range(N):
        for x in range(N):
            s = y * N + x
            put(s, s, (m0 + 2.0) * I2)
            for mu, (dx, dy) in enumerate(((1, 0), (0, 1))):
                # forward hop: couples x to x + mu with U_mu(x)
                xf, yf = (x + dx) % N, (y + dy) % N
                u = np.exp(1j * theta[mu, y, x])
                put(s, yf * N + xf, -0.5 * u * fwd[mu])
                # backward hop: couples x to x - mu with conj(U_mu(x - mu))
                xb, yb = (x - dx) % N, (y - dy) % N
                ub = np.exp(-1j * theta[mu, yb, xb])
                put(s, yb * N + xb, -0.5 * ub * bwd[mu])
    n = 2 * N * N
    return sp.csr_matrix((np.array(vals), (rows, cols)), shape=(n, n))


def gauge_laplacian(N, theta, mass=0.0):
    """Gauge Laplacian of Example 4.2 (see module doc); theta [2, N, N]."""
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.shape == (2, N, N)
    rows, cols, vals = [], [], []
    for y in range(N):
        for x in range(N):
            s = y * N + x
            rows.append(s)
            cols.append(s)
            vals.append(4.0 + mass)
            for mu, t in ((0, y * N + (x + 1) % N), (1, ((y + 1) % N) * N + x)):
                u = np.exp(1j * theta[mu, y, x])
                rows += [s, t]          # the forward hop and its Hermitian partner
                cols += [t, s]
                vals += [-u, -np.conj(u)]
    return sp.csr_matrix((np.array(vals), (rows, cols)), shape=(N * N, N * N))


def gauge_transform(N, theta, phi):
    """Link phases after the gauge transformation u_s -> exp(i phi_s) u_s:
    theta_mu(s) + phi(s) - phi(s + mu); the operator becomes D A D^* with
    D = diag(exp(i phi)), so its spectrum and tr(A^-1) are unchanged."""
    theta = np.array(theta, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64).reshape(N, N)
    theta[0] += phi - np.roll(phi, -1, axis=1)
    theta[1] += phi - np.roll(phi, -1, axis=0)
    return theta


def gauge_laplacian_free_trace(N, mass):
    """tr(A^-1) of the gauge Laplacian with all phases zero: the periodic
    Laplacian plus m, eigenvalues m + 4 - 2 cos(2 pi k/N) - 2 cos(2 pi l/N)."""
    c = 2.0 - 2.0 * np.cos(2.0 * np.pi * np.arange(N) / N)
    return float(np.sum(1.0 / (mass + c[:, None] + c[None, :])))


def gamma5(n_sites):
    """J = I kron diag(1, -1) with the spin index innermost (Example 4.3)."""
    return sp.diags(np.tile([1.0, -1.0], n_sites))


def varcoef3d(N, k, shift):
    """3D 7-point variable-coefficient operator (see module doc).

    k: float array [3, N, N, N+1]; k[0][z][y][f] are x-faces, k[1][z][x][f]
    y-faces, k[2][y][x][f] z-faces.
    """
    k = np.asarray(k, dtype=np.float64)
    assert k.shape == (3, N, N, N + 1)
    n = N ** 3
    diag = np.full(n, float(shift))
    rows, cols, vals = [], [], []

    def cell(x, y, z):
        return (z * N + y) * N + x

    for d in range(3):
        for a in range(N):
            for b in range(N):
                for f in range(N + 1):
                    kf = k[d, a, b, f]
                    # cells on either side of face f along direction d
                    if d == 0:
                        lo = cell(f - 1, b, a) if f >= 1 else None
                        hi = cell(f, b, a) if f < N else None
                    elif d == 1:
                        lo = cell(b, f - 1, a) if f >= 1 else None
                        hi = cell(b, f, a) if f < N else None
                    else:
                        lo = cell(b, a, f - 1) if f >= 1 else None
                        hi = cell(b, a, f) if f < N else None
                    if lo is not None:
                        diag[lo] += kf
                    if hi is not None:
                        diag[hi] += kf
                    if lo is not None and hi is not None:
                        rows += [lo, hi]
                        cols += [hi, lo]
                        vals += [-kf, -kf]
    A = sp.csr_matrix((vals, (rows, cols)), shape=(n, n)) + sp.diags(diag)
    return A.tocsr()


def poisson2d_solve_dst(N, B, diag=4.0, off=1.0):
    """Exact A^{-1} B for A = diag*I - off*neighbours (Dirichlet, N x N grid).

    The eigenvectors of L^N are products of discrete sines (Example 4.1: the
    eigenvalues are known explicitly), so the orthonormal type-I sine transform
    diagonalises A; eigenvalue (j, k) is
        diag - 2*off*cos(j pi/(N+1)) - 2*off*cos(k pi/(N+1)).
    B: [N*N] or [N*N, m]; returns the same shape.  FFT-based, O(n log n).
    """
    from scipy.fft import dstn
    B = np.asarray(B)
    vec = B.ndim == 1
    if vec:
        B = B[:, None]
    c = np.cos(np.arange(1, N + 1) * np.pi / (N + 1))
    lam = diag - 2.0 * off * (c[:, None] + c[None, :])
    out = np.empty(B.shape, dtype=np.result_type(B.dtype, np.float64))
    for j in range(B.shape[1]):
        G = B[:, j].reshape(N, N)
        H = dstn(G, type=1, norm="ortho")
        out[:, j] = dstn(H / lam, type=1, norm="ortho").reshape(-1)
    return out[:, 0] if vec else out
