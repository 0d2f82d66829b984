"""Exact level-difference samples, the direct coarsest trace and the MLMC driver.

Test infrastructure (see the package docstring).

Per-sample value (Remark 4.3 with the estimator of Sec. 4.1): for a level
l < L and a probe x in C^{n_l},
    s = x^H A_l^{-1} x - (R_l x)^H A_{l+1}^{-1} (R_l x),   R_l = P_l^H,
the same x entering both terms.  Its expectation is
tr(A_l^{-1}) - tr(P_l A_{l+1}^{-1} R_l), and these telescope with the
coarsest term tr(A_L^{-1}) (Remark 4.2, computed by inverting A_L) to
tr(A^{-1}) (eq. tr_ml_dec).  Solves here are exact: dense LU for n <= 4096,
otherwise a sparse LU followed by one FP64 refinement step.

Estimator (Sec. 2, the MLMC estimator with its 1/N_l factors -- the version
printed in Sec. 4.1 drops them, read as a typo) and its accuracy control
(Sec. 5): tau is the mean of five pilot plain Hutchinson estimates minus their
root mean square deviation; the level-difference RMSD targets satisfy
sum_l rho_l^2 = (eps*tau)^2, equal split rho_l = eps*tau/sqrt(L-1) by default,
given weights as in Example 4.3, or the optimal allocation of Sec. 2
(N_l proportional to sqrt(V_l/C_l), read with the multiplier
mu = eps^-2 sum_k sqrt(V_k C_k), which is what the cost formula printed next to
it requires); at least five estimates per level difference (Example 4.1).
"Root mean square deviation" of a mean of N samples is read as the standard
error sqrt(s^2/N) with the Bessel-corrected sample variance s^2.

Batch rule (a reading: the paper adds one estimate at a time): after the
initial min_samples per level, every round recomputes the targets and, for each
level whose RMSD exceeds its target, draws min(nb, ceil(V_l/rho_l^2) - N_l)
further samples (at least one).  The library's driver follows the same rule so
that both draw the same samples.
"""
import math

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import philox

DENSE_MAX = 4096

ALLOC_EQUAL = 0
ALLOC_WEIGHTS = 1
ALLOC_GILES = 2


class ExactSolver:
    """y = A^{-1} b exactly (up to FP64 rounding) for a fixed sparse A."""

    def __init__(self, A):
        self.A = sp.csr_matrix(A)
        self.n = A.shape[0]
        self.dtype = np.complex128 if np.iscomplexobj(A.data) else np.float64
        if self.n <= DENSE_MAX:
            self.lu = sla.lu_factor(self.A.toarray())
            self.splu = None
        else:
            self.lu = None
            self.splu = spla.splu(self.A.tocsc())

    def solve(self, B):
        B = np.asarray(B)
        if self.lu is not None:
            return sla.lu_solve(self.lu, B)
        Y = self.splu.solve(B)
        R = B - self.A @ Y                 # one step of FP64 refinement
        return Y + self.splu.solve(R)


def coarse_trace(A_L):
    """tr(A_L^{-1}) by explicit inversion of the coarsest operator (Remark 4.2)."""
    return complex(np.trace(np.linalg.inv(sp.csr_matrix(A_L).toarray())))


def quad(x, y):
    """x^H y summed in index order (FP64)."""
    return complex(np.vdot(x, y))


class LevelSampler:
    """Exact level-difference samples for a hierarchy (A_1..A_L, P_1..P_{L-1})."""

    def __init__(self, A, P, complex_probe, problem=0):
        self.A = A
        self.P = P
        self.L = len(A)
        self.complex_probe = complex_probe
        self.problem = problem
        self._solvers = {}

    def solver(self, level):
        if level not in self._solvers:
            self._solvers[level] = ExactSolver(self.A[level - 1])
        return self._solvers[level]

    def probes(self, level, seed, first, count, stream=philox.STREAM_PROBE):
        n = self.A[level - 1].shape[0]
        X = np.stack([philox.probe(n, seed, first + j, level, self.complex_probe,
                                   stream, self.problem)
                      for j in range(count)], axis=1)
        return X

    def sample(self, level, seed, first, count):
        """s_{l,k}, k = first..first+count-1 (Remark 4.3 form)."""
        assert 1 <= level < self.L
        X = self.probes(level, seed, first, count)
        Y = self.solver(level).solve(X)
        R = self.P[level - 1].conj().T
        Xc = R @ X
        Z = self.solver(level + 1).solve(Xc)
        return np.array([quad(X[:, j], Y[:, j]) - quad(Xc[:, j], Z[:, j])
                         for j in range(count)])

    def sample_parts(self, level, seed, first, count):
        """(x^H A_l^-1 x, (Rx)^H A_{l+1}^-1 (Rx)) separately."""
        X = self.probes(level, seed, first, count)
        Y = self.solver(level).solve(X)
        Xc = self.P[level - 1].conj().T @ X
        Z = self.solver(level + 1).solve(Xc)
        return (np.array([quad(X[:, j], Y[:, j]) for j in range(count)]),
                np.array([quad(Xc[:, j], Z[:, j]) for j in range(count)]))

    def hutchinson(self, seed, first, count, stream=philox.STREAM_HUTCH, level=1):
        """Plain Hutchinson samples x^H A_level^{-1} x (eq. plain_tr_estimate)."""
        X = self.probes(level, seed, first, count, stream)
        Y = self.solver(level).solve(X)
        return np.array([quad(X[:, j], Y[:, j]) for j in range(count)])

    def coarse(self):
        return coarse_trace(self.A[-1])

    def cost(self, level):
        """Cost model of one level-difference sample: n_l + n_{l+1} unknowns."""
        return float(self.A[level - 1].shape[0] + self.A[level].shape[0])


class GeneralLevelSampler(LevelSampler):
    """Exact level-difference samples of the general decomposition of Sec. 4.1
    for any P_l (R_l = P_l^H): with a probe x on the finest level,
        s = x^H Phat_l A_l^{-1} Rhat_l x - x^H Phat_{l+1} A_{l+1}^{-1} Rhat_{l+1} x,
    Rhat_l = R_{l-1} ... R_1, Phat_l = P_1 ... P_{l-1}; the coarsest term is
    tr(A_L^{-1} Rhat_L Phat_L) (Remark 4.2, trace of a product commutes).  Both
    quadratic forms are taken as written: the solution is prolongated back to
    the finest level and multiplied with x there."""

    def probes(self, level, seed, first, count, stream=philox.STREAM_PROBE):
        n = self.A[0].shape[0]
        return np.stack([philox.probe(n, seed, first + j, level, self.complex_probe,
                                      stream, self.problem)
                         for j in range(count)], axis=1)

    def restrict_to(self, level, X):
        for l in range(level - 1):
            X = self.P[l].conj().T @ X
        return X

    def prolong_from(self, level, Y):
        for l in range(level - 2, -1, -1):
            Y = self.P[l] @ Y
        return Y

    def parts_for(self, level, X):
        """(x^H Phat_l A_l^-1 Rhat_l x, x^H Phat_{l+1} A_{l+1}^-1 Rhat_{l+1} x) for
        the columns x of X."""
        parts = []
        for lv in (level, level + 1):
            Y = self.prolong_from(lv, self.solver(lv).solve(self.restrict_to(lv, X)))
            parts.append(np.array([quad(X[:, j], Y[:, j]) for j in range(X.shape[1])]))
        return parts[0], parts[1]

    def sample_parts(self, level, seed, first, count):
        return self.parts_for(level, self.probes(level, seed, first, count))

    def sample(self, level, seed, first, count):
        assert 1 <= level < self.L
        a, b = self.sample_parts(level, seed, first, count)
        return a - b

    def coarse(self):
        L = self.L
        Rh = sp.identity(self.A[0].shape[0], format="csr")
        Ph = Rh
        for l in range(L - 1):
            Rh = self.P[l].conj().T @ Rh
            Ph = Ph @ self.P[l]
        M = (Rh @ Ph).toarray()
        return complex(np.trace(np.linalg.inv(sp.csr_matrix(self.A[-1]).toarray()) @ M))


def mean_and_var(s):
    """Mean and Bessel-corrected variance E|s - mean|^2 (convention of Sec. 3)."""
    s = np.asarray(s, dtype=np.complex128)
    N = len(s)
    m = complex(np.sum(s)) / N
    if N < 2:
        return m, 0.0
    d = s - m
    return m, float(np.sum((d.real * d.real) + (d.imag * d.imag))) / (N - 1)


def pilot_tau(sampler, seed, npilot=5):
    """tau = |mean| - RMSD of five pilot Hutchinson estimates (Sec. 5)."""
    y = sampler.hutchinson(seed, 0, npilot, stream=philox.STREAM_PILOT)
    m, v = mean_and_var(y)
    tau = abs(m) - math.sqrt(v / npilot)
    if tau <= 0.0:
        tau = abs(m)
    return tau, y


def level_weights(alloc, L, var, cost, weights=None):
    """Fractions w_l (sum 1) of the variance budget (eps*tau)^2 per level."""
    nl = L - 1
    if alloc == ALLOC_EQUAL:
        return [1.0 / nl] * nl
    if alloc == ALLOC_WEIGHTS:
        w = list(weights)
        assert len(w) == nl
        t = sum(w)
        return [x / t for x in w]
    # Sec. 2: N_l = mu sqrt(V_l/C_l) gives rho_l^2 = V_l/N_l
    # = (eps tau)^2 sqrt(V_l C_l) / sum_k sqrt(V_k C_k)
    g = [math.sqrt(max(var[l], 0.0) * cost[l]) for l in range(nl)]
    t = sum(g)
    if t <= 0.0:
        return [1.0 / nl] * nl
    return [x / t for x in g]


def mlmc_trace(sampler, eps, seed, nb=128, min_samples=5, alloc=ALLOC_EQUAL,
               weights=None, tau=None, max_samples=1 << 22):
    """Multilevel Monte-Carlo estimate of tr(A^-1) (Sec. 4.1, control of Sec. 5).

    Returns a dict: trace, rmsd, tau, samples per level, level means/variances.
    """
    L = sampler.L
    nl = L - 1
    if tau is None:
        tau, _ = pilot_tau(sampler, seed)
    target2 = (eps * tau) ** 2
    cost = [sampler.cost(l + 1) for l in range(nl)]
    samples = [list(sampler.sample(l + 1, seed, 0, min_samples)) for l in range(nl)]
    rounds = 0
    while True:
        stats = [mean_and_var(s) for s in samples]
        var = [v for _, v in stats]
        w = level_weights(alloc, L, var, cost, weights)
        todo = []
        for l in range(nl):
            N = len(samples[l])
            rho2 = w[l] * target2
            if var[l] / N > rho2:
                if rho2 > 0.0:
                    need = math.ceil(var[l] / rho2) - N
                else:
                    need = nb
                add = max(1, min(nb, need, max_samples - N))
                if N >= max_samples:
                    raise RuntimeError("level %d exceeded max_samples" % (l + 1))
                todo.append((l, add))
        if not todo:
            break
        for l, add in todo:
            N = len(samples[l])
            samples[l] += list(sampler.sample(l + 1, seed, N, add))
        rounds += 1
    stats = [mean_and_var(s) for s in samples]
    coarse = sampler.coarse()
    trace = sum(m for m, _ in stats) + coarse
    rmsd = math.sqrt(sum(v / len(s) for (_, v), s in zip(stats, samples)))
    return dict(trace=trace, rmsd=rmsd, tau=tau, coarse=coarse,
                n_samples=[len(s) for s in samples],
                level_mean=[m for m, _ in stats], level_var=[v for _, v in stats],
                samples=samples, rounds=rounds)


def hutchinson_trace(sampler, eps, seed, nb=128, min_samples=5, tau=None,
                     max_samples=1 << 22):
    """Plain Hutchinson (eq. plain_tr_estimate) to RMSD <= eps*tau, same batch rule."""
    if tau is None:
        tau, _ = pilot_tau(sampler, seed)
    target2 = (eps * tau) ** 2
    s = list(sampler.hutchinson(seed, 0, min_samples))
    while True:
        m, v = mean_and_var(s)
        N = len(s)
        if v / N <= target2:
            break
        need = math.ceil(v / target2) - N if target2 > 0 else nb
        add = max(1, min(nb, need, max_samples - N))
        if N >= max_samples:
            raise RuntimeError("exceeded max_samples")
        s += list(sampler.hutchinson(seed, N, add))
    m, v = mean_and_var(s)
    return dict(trace=m, rmsd=math.sqrt(v / len(s)), tau=tau, n_samples=len(s))


class PoissonDSTSampler(LevelSampler):
    """Exact samples for the 2D Poisson hierarchy at sizes where sparse LU is slow.

    Uses A_l = 2^{1-l} (diag I - off neighbours) on the N_l = N/2^{l-1} grid --
    the Galerkin identity of 2x2 orthonormal aggregation (checked against the
    sparse Galerkin product in the tests) -- and the exact sine-transform solver.
    """

    def __init__(self, N, levels, diag=4.0, off=1.0):
        from .hierarchy import aggregation_2d
        self.N = N
        self.L = levels
        self.diag = diag
        self.off = off
        self.complex_probe = False
        self.problem = 0
        self.sides = [N >> l for l in range(levels)]
        self.P = [aggregation_2d(self.sides[l]) for l in range(levels - 1)]
        self.A = None

    def coeffs(self, level):
        s = 2.0 ** (1 - level)
        # diag' = diag - 2 off, off' = off/2 per level: exact scaling when diag = 4 off
        d, c = self.diag, self.off
        for _ in range(level - 1):
            d, c = d - 2.0 * c, 0.5 * c
        return d, c

    def size(self, level):
        return self.sides[level - 1] ** 2

    def probes(self, level, seed, first, count, stream=philox.STREAM_PROBE):
        n = self.size(level)
        return np.stack([philox.probe(n, seed, first + j, level, False, stream)
                         for j in range(count)], axis=1)

    def _solve(self, level, B):
        from .operators import poisson2d_solve_dst
        d, c = self.coeffs(level)
        return poisson2d_solve_dst(self.sides[level - 1], B, d, c)

    def sample(self, level, seed, first, count):
        X = self.probes(level, seed, first, count)
        Y = self._solve(level, X)
        Xc = self.P[level - 1].T @ X
        Z = self._solve(level + 1, Xc)
        return np.array([quad(X[:, j], Y[:, j]) - quad(Xc[:, j], Z[:, j])
                         for j in range(count)])

    def sample_parts(self, level, seed, first, count):
        X = self.probes(level, seed, first, count)
        Y = self._solve(level, X)
        Xc = self.P[level - 1].T @ X
        Z = self._solve(level + 1, Xc)
        return (np.array([quad(X[:, j], Y[:, j]) for j in range(count)]),
                np.array([quad(Xc[:, j], Z[:, j]) for j in range(count)]))

    def hutchinson(self, seed, first, count, stream=philox.STREAM_HUTCH, level=1):
        X = self.probes(level, seed, first, count, stream)
        Y = self._solve(level, X)
        return np.array([quad(X[:, j], Y[:, j]) for j in range(count)])

    def coarse(self):
        from .operators import poisson2d_eigenvalues
        d, c = self.coeffs(self.L)
        Nl = self.sides[-1]
        lam = poisson2d_eigenvalues(Nl)         # of 4I - neighbours
        # d I - c neighbours = c (4I - neighbours) + (d - 4c) I
        return complex(np.sum(1.0 / (c * lam + (d - 4.0 * c))))

    def cost(self, level):
        return float(self.size(level) + self.size(level + 1))
