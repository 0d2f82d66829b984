"""Deflated Hutchinson, the comparison method of Sec. 5 (test infrastructure only).

Sec. 4.2 (eqs. orth_proj and defl) splits A^{-1} with an orthogonal projector
Pi = U U^H onto k (smallest) eigenvectors or singular vectors of A:
    tr(A^{-1}) = tr(A^{-1} (I - Pi)) + tr(A^{-1} Pi),
estimates the first trace with Hutchinson's estimator and computes the second
directly.  Sec. 5 uses, for Hermitian A, the n_defl eigenvectors of the
smallest eigenvalues; then tr(A^{-1} Pi) = sum_i 1/lambda_i.

Readings taken here (the paper's text in Sec. 5 names the projector "I - U U^*"
and then estimates tr(A^{-1}(I - Pi)), which contradicts eq. orth_proj; eq.
orth_proj is taken, Pi = U U^H):
  * a sample is x^H A^{-1} (I - Pi) x = x^H A^{-1} x_perp with
    x_perp = x - U (U^H x) (the 2 n n_defl projection work Sec. 5 counts); its
    expectation is tr(A^{-1}(I - Pi)) for every orthonormal U (Theorem on
    Hutchinson's estimator), so approximate eigenvectors leave it unbiased;
  * the direct term is tr(A^{-1} Pi) = tr(U^H A^{-1} U) = sum_i u_i^H A^{-1} u_i
    (trace commutes, eq. trace_commute), which equals sum_i 1/lambda_i for exact
    eigenvectors and keeps the split exact for approximate ones;
  * probes are those of plain Hutchinson (RNG stream 3), so a deflated sample is
    the plain sample of the same index minus x^H A^{-1} Pi x;
  * accuracy control as for plain Hutchinson in Sec. 5: tau from five pilot
    plain Hutchinson estimates, samples until their RMSD is at most eps * tau.
"""
import math

import numpy as np
import scipy.sparse as sp

from . import mlmc, philox


def smallest_eigenpairs(A, k):
    """The k smallest eigenvalues (ascending) of a Hermitian A and orthonormal
    eigenvectors (columns), by a dense Hermitian eigen-decomposition."""
    import scipy.linalg as sla
    M = A.toarray() if sp.issparse(A) else np.asarray(A)
    lam, V = sla.eigh(M, subset_by_index=[0, k - 1])
    return lam.copy(), V.copy()


class DeflatedSampler:
    """Samples x^H A^{-1} (I - U U^H) x of a Hermitian A (exact solves)."""

    def __init__(self, A, U, complex_probe=False):
        self.A = sp.csr_matrix(A)
        self.U = np.asarray(U)
        self.n = self.A.shape[0]
        self.complex_probe = complex_probe
        self.solver = mlmc.ExactSolver(self.A)

    def probes(self, seed, first, count, stream=philox.STREAM_HUTCH):
        return np.stack([philox.probe(self.n, seed, first + j, 1, self.complex_probe, stream)
                         for j in range(count)], axis=1)

    def project(self, X):
        """(I - U U^H) X."""
        return X - self.U @ (self.U.conj().T @ X)

    def sample(self, seed, first, count):
        X = self.probes(seed, first, count)
        Y = self.solver.solve(self.project(X))
        return np.array([mlmc.quad(X[:, j], Y[:, j]) for j in range(count)])

    def hutchinson(self, seed, first, count, stream=philox.STREAM_HUTCH, level=1):
        """Plain Hutchinson samples x^H A^{-1} x (the pilot of Sec. 5)."""
        X = self.probes(seed, first, count, stream)
        Y = self.solver.solve(X)
        return np.array([mlmc.quad(X[:, j], Y[:, j]) for j in range(count)])

    def direct(self):
        """tr(A^{-1} Pi) = tr(U^H A^{-1} U)."""
        W = self.solver.solve(self.U)
        return complex(np.trace(self.U.conj().T @ W))


def deflated_hutchinson_trace(sampler, eps, seed, nb=128, min_samples=5, tau=None,
                              max_samples=1 << 22):
    """Deflated Hutchinson estimate of tr(A^{-1}) to RMSD <= eps * tau (Sec. 5),
    with the batch rule of plain Hutchinson; estimate = sample mean + direct term."""
    if tau is None:
        tau, _ = mlmc.pilot_tau(sampler, seed)
    target2 = (eps * tau) ** 2
    s = list(sampler.sample(seed, 0, min_samples))
    while True:
        m, v = mlmc.mean_and_var(s)
        N = len(s)
        if v / N <= target2:
            break
        need = math.ceil(v / target2) - N if target2 > 0 else nb
        add = max(1, min(nb, need, max_samples - N))
        if N >= max_samples:
            raise RuntimeError("exceeded max_samples")
        s += list(sampler.sample(seed, N, add))
    m, v = mlmc.mean_and_var(s)
    direct = sampler.direct()
    return dict(trace=m + direct, deflated_mean=m, direct=direct,
                rmsd=math.sqrt(v / len(s)), tau=tau, n_samples=len(s), var=v)
