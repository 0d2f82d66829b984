"""The boundary's export of the hierarchy for every operator kind (A_l and P_l as
sparse matrices) against the oracle's own hierarchy, and the MLMC_ENOCONV
contract of mlmc_sample_level (partial results, level and sample named)."""
import ctypes

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import hierarchy
from tests.gpu_util import require_gpu
from workloads import gauge_field, varcoef_faces

pytestmark = pytest.mark.gpu


def _close(A, B, tol):
    D = (sp.csr_matrix(A) - sp.csr_matrix(B)).tocoo()
    scale = max(abs(sp.csr_matrix(B)).max(), 1e-300)
    return (np.max(np.abs(D.data)) if D.nnz else 0.0) <= tol * scale


def _canonical(M):
    # columns ascending within every row, no repeated or zero entries
    M = sp.csr_matrix(M)
    for i in range(M.shape[0]):
        c = M.indices[M.indptr[i]:M.indptr[i + 1]]
        assert np.all(np.diff(c) > 0), i
    assert np.all(M.data != 0)


def test_export_poisson_levels_and_prolongations():
    require_gpu()
    import paper_2108_11281_amd as m
    N, L = 64, 4
    est = m.TraceEstimator("poisson2d", N, L, L, nb=4)
    A, P = hierarchy.poisson_hierarchy(N, L)
    for l in range(1, L + 1):
        Al = est.export_level(l, "A")
        _canonical(Al)
        assert Al.shape == A[l - 1].shape and (Al != A[l - 1]).nnz == 0, l   # exact
        if l < L:
            Pl = est.export_level(l, "P")
            _canonical(Pl)
            assert (Pl != P[l - 1]).nnz == 0, l


def test_export_varcoef_levels_and_prolongations():
    require_gpu()
    import paper_2108_11281_amd as m
    N, L = 16, 3
    faces = varcoef_faces(N, seed=1000)
    est = m.TraceEstimator("varcoef3d", N, L, L, shift=1e-3, field=faces, nb=4)
    A, P = hierarchy.varcoef_hierarchy(N, faces, 1e-3, L)
    for l in range(1, L + 1):
        Al = est.export_level(l, "A")
        _canonical(Al)
        assert _close(Al, A[l - 1], 1e-14), l
        if l < L:
            assert _close(est.export_level(l, "P"), P[l - 1], 1e-15), l


def test_export_wilson_and_gauge_levels():
    require_gpu()
    import paper_2108_11281_amd as m
    N, L, m0 = 16, 3, 0.1
    th = gauge_field(N, seed=3)
    est = m.TraceEstimator("wilson2d", N, L, L, mass=m0, field=th, block=4, n_vec=4,
                           setup_sweeps=4, setup_seed=1, nb=4)
    A, P = hierarchy.wilson_hierarchy(N, th, m0, L, block=4, n_vec=4, sweeps=4, seed=1)
    A1 = est.export_level(1, "A")
    _canonical(A1)
    assert _close(A1, A[0], 1e-14)
    for l in (1, 2):
        Pl = est.export_level(l, "P")
        _canonical(Pl)
        # the library's test-vector bases agree with the oracle's to ~1e-12
        assert _close(Pl, P[l - 1], 1e-9), l
        # P^H P = I (orthonormal aggregation, Remark 4.3)
        G = (Pl.conj().T @ Pl).toarray()
        assert np.max(np.abs(G - np.eye(G.shape[0]))) < 1e-12
    # coarse operators: the exported A_{l+1} equals the Galerkin product of the
    # exported A_l and P_l
    for l in (1, 2):
        Al, Pl, Ac = est.export_level(l, "A"), est.export_level(l, "P"), est.export_level(l + 1, "A")
        assert _close(Ac, Pl.conj().T @ Al @ Pl, 1e-12), l
    g = m.TraceEstimator("gauge2d", N, 2, 2, mass=0.0, field=gauge_field(N, sigma=0.3, seed=2),
                         block=4, n_vec=4, setup_sweeps=4, setup_seed=1, nb=4)
    from oracle import operators
    Ag = g.export_level(1, "A")
    assert _close(Ag, operators.gauge_laplacian(N, gauge_field(N, sigma=0.3, seed=2), 0.0),
                  1e-14)


def test_export_csr_given_prolongation():
    require_gpu()
    import paper_2108_11281_amd as m
    from workloads import bilinear_prolongations, laplace_matrix
    N, Ls = 31, 3
    P = bilinear_prolongations(N, Ls)
    est = m.TraceEstimator("csr", 0, Ls, Ls, matrix=laplace_matrix(N), prolongations=P, nb=4)
    for l in (1, 2):
        assert _close(est.export_level(l, "P"), P[l - 1], 0.0), l
    assert _close(est.export_level(2, "A"), P[0].T @ laplace_matrix(N) @ P[0], 1e-14)


def test_export_rejects_bad_levels():
    require_gpu()
    import paper_2108_11281_amd as m
    est = m.TraceEstimator("poisson2d", 32, 3, 3, nb=4)
    with pytest.raises(m.MLMCError):
        est.export_level(3, "P")          # no prolongation on the coarsest level
    with pytest.raises(m.MLMCError):
        est.export_level(4, "A")


def test_enoconv_keeps_partial_results_and_names_the_sample():
    # an iteration budget far too small for solve_tol: every solve fails; the
    # call returns MLMC_ENOCONV, names the level and the first failed sample, and
    # the failed samples are NaN (no stale values)
    require_gpu()
    import paper_2108_11281_amd as m
    est = m.TraceEstimator("poisson2d", 64, 3, 3, nb=4, solve_tol=1e-14, max_iter=1,
                           max_refine=1)
    out = np.full((6, 2), 7.0)
    err = np.full(6, 7.0)
    rc = est._lib.mlmc_sample_level(est._ctx, 1, 3, 10, 6,
                                    out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    err.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    assert rc == m._capi.MLMC_ENOCONV
    msg = est._lib.mlmc_last_error(est._ctx).decode()
    assert "level 1" in msg and "sample 10" in msg and "column 0" in msg, msg
    assert np.all(np.isnan(out[:4])) and np.all(np.isnan(err[:4]))
    assert np.all(out[4:] == 7.0)          # the batch after the failing one is not run
    # a converging configuration on the same operator still works afterwards
    ok = m.TraceEstimator("poisson2d", 64, 3, 3, nb=4, solve_tol=1e-12)
    s = ok.sample_level(1, 3, 10, 6)
    assert np.all(np.isfinite(s))


def test_stream_copy_measurement_kernel():
    # the streaming copy that measures the sustained HBM rate: exact copy of a
    # multiple of 16 bytes (a ragged last group of four 16-byte words), and
    # misaligned or ragged sizes rejected
    torch = require_gpu()
    import ctypes
    import paper_2108_11281_amd as m
    a = torch.arange(1 << 18, dtype=torch.float32, device="cuda") * 0.5 + 1.0
    b = torch.zeros(a.numel() + 4, dtype=torch.float32, device="cuda")
    m.stream_copy(a[: (1 << 18) - 12], b[: (1 << 18) - 12])
    torch.cuda.synchronize()
    assert torch.equal(b[: (1 << 18) - 12], a[: (1 << 18) - 12])
    assert int(torch.count_nonzero(b[(1 << 18) - 12:])) == 0
    lib = m.lib()
    p = ctypes.c_void_p
    assert lib.mlmc_stream_copy(p(a.data_ptr() + 4), p(b.data_ptr()), 64, None) == -1
    assert lib.mlmc_stream_copy(p(a.data_ptr()), p(b.data_ptr()), 20, None) == -1
