"""The learned-smoother workload at its own size: the Wilson-like operator on the
512 x 512 lattice (n = 524,288 complex unknowns; 4 solver levels, 3 MLMC levels,
the mass tuned so that the smallest |eigenvalue| is 1e-2), with a network trained
on the method's own plain solves replacing two of the four finest-level sweeps.
A sparse direct factorisation of this operator does not fit a test, so the oracle
checks column by column: the Z4 probes bit for bit, every FP64 residual of the
returned level-1 solutions with its own operator, the exported coarse operator
against the Galerkin product of the oracle's operator with the exported
orthonormal prolongation, the level-2 residuals with it, and each sample's two
quadratic forms."""
import numpy as np
import pytest

from oracle import operators, philox
from tests.gpu_util import from_dev, require_gpu
from workloads import gauge_field, nn_init_weights, wilson_mass

pytestmark = pytest.mark.gpu

N, LS, L, SEED, COUNT = 512, 4, 3, 11, 12


@pytest.fixture(scope="module")
def setup():
    require_gpu()
    import paper_2108_11281_amd as m
    m0 = wilson_mass(N)
    th = gauge_field(N, sigma=0.5, seed=1)
    est = m.TraceEstimator("wilson2d", N, LS, L, mass=m0, field=th, block=4, n_vec=8,
                           setup_sweeps=20, setup_seed=1, precision="fp32_ir64", nb=32,
                           nu_pre=2, nu_post=2, solve_tol=1e-10, learned=1)
    rep = est.learned_train(nn_init_weights(1), n_batches=2, crops_per_column=4, steps=300,
                            batch=128, lr=2e-3, seed=5)
    A1 = operators.wilson2d(N, th, m0).tocsr()
    return est, A1, rep


def test_full_size_learned_samples(setup):
    est, A1, rep = setup
    assert np.isfinite(rep["loss_last"]) and rep["loss_last"] < rep["loss_first"], rep
    n1 = est.level_size(1)
    X = est.probes(1, SEED, 0, COUNT)
    x = from_dev(X, complex_=True)
    for k in range(COUNT):
        assert np.array_equal(x[k], philox.z4(n1, SEED, k, 1)), k
    apps0, fb0 = est.learned_stats()
    Y, rel = est.solve(1, X)
    apps1, fb1 = est.learned_stats()
    assert apps1 > apps0 and fb1 == fb0          # the network ran, no fallback
    assert np.all(rel <= 1e-10), np.max(rel)
    y = from_dev(Y, complex_=True)
    # the level-2 operator and the transfer, exported; A_2 = P^H A_1 P with the
    # oracle's A_1 (Sec. 4.1), P orthonormal (Remark 4.3)
    P = est.export_level(1, "P")
    A2 = est.export_level(2, "A")
    G = (P.conj().T @ A1 @ P).tocsr()
    D = (A2 - G).tocoo()
    assert (np.max(np.abs(D.data)) if D.nnz else 0.0) <= 1e-12 * abs(G).max()
    PP = (P.conj().T @ P).tocoo()
    off = PP.row != PP.col
    assert np.max(np.abs(PP.data[~off] - 1.0)) < 1e-12
    assert (np.max(np.abs(PP.data[off])) if off.any() else 0.0) < 1e-12
    xc = (P.conj().T @ x.T).T
    Xc = est.restrict(1, X)
    assert np.max(np.abs(from_dev(Xc, complex_=True) - xc)) <= 1e-12 * np.max(np.abs(xc))
    Z, relz = est.solve(2, Xc)
    assert np.all(relz <= 1e-10)
    z = from_dev(Z, complex_=True)
    s, err = est.sample_level(1, SEED, 0, COUNT, with_error=True)
    assert np.all(err <= 1e-8), np.max(err)
    for k in range(COUNT):
        r1 = np.linalg.norm(x[k] - A1 @ y[k]) / np.linalg.norm(x[k])
        r2 = np.linalg.norm(xc[k] - A2 @ z[k]) / np.linalg.norm(xc[k])
        assert r1 <= 2e-10 and r2 <= 1e-8, (k, r1, r2)
        a, b = np.vdot(x[k], y[k]), np.vdot(xc[k], z[k])
        assert abs(s[k] - (a - b)) <= 1e-8 * (abs(a) + abs(b)), k
