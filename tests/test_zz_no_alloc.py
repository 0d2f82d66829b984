"""The allocation-free smoother entry point (mlmc_smooth_noalloc) against the
allocating one (mlmc_smooth) through the C ABI: same kernels, so the same bits,
on two calls in a row (the second on a smaller input), with no device
allocation by the library during the call, and a clear error beyond the fixed
workspace."""
import ctypes

import numpy as np
import pytest

from tests.gpu_util import from_dev, require_gpu, to_dev
from workloads import gauge_field

pytestmark = pytest.mark.gpu


def _call(est, fn, level, B, X, sweeps, flags, rc=None):
    rcode = fn(est._ctx, int(level), int(B.shape[0]), int(sweeps), int(flags),
               ctypes.c_void_p(B.data_ptr()), ctypes.c_void_p(X.data_ptr()),
               ctypes.c_void_p(rc.data_ptr()) if rc is not None else None)
    est._sync()
    return rcode


def _allocs():
    import torch
    return torch.cuda.memory_stats().get("allocation.all.allocated", 0)


def _compare(est, level, nrhs, sweeps, flags, restrict, seed, complex_=False):
    import torch
    lib = est._lib
    n = est.level_size(level)
    w = 2 * n if complex_ else n
    rng = np.random.default_rng(seed)
    B = to_dev(rng.standard_normal((nrhs, w)))
    X0 = to_dev(rng.standard_normal((nrhs, w)))
    nc = est.level_size(level + 1) * (2 if complex_ else 1)
    Xa, Xb = X0.clone(), X0.clone()
    rca = torch.zeros((nrhs, nc), dtype=torch.float64, device="cuda") if restrict else None
    rcb = torch.zeros((nrhs, nc), dtype=torch.float64, device="cuda") if restrict else None
    torch.cuda.synchronize()
    a0 = _allocs()
    assert _call(est, lib.mlmc_smooth, level, B, Xa, sweeps, flags, rca) == 0
    a1 = _allocs()
    assert _call(est, lib.mlmc_smooth_noalloc, level, B, Xb, sweeps, flags, rcb) == 0, \
        lib.mlmc_last_error(est._ctx)
    a2 = _allocs()
    # the library's device memory comes from torch's caching allocator: the
    # allocating entry point shows up in its count, the allocation-free one not
    assert a1 > a0 and a2 == a1, (a0, a1, a2)
    assert np.array_equal(from_dev(Xa), from_dev(Xb))
    if restrict:
        assert np.array_equal(from_dev(rca), from_dev(rcb))


@pytest.mark.parametrize("precision", ["fp32_ir64", "fp64"])
def test_noalloc_poisson_matches_allocating_entry_point(precision):
    require_gpu()
    import paper_2108_11281_amd as m
    est = m.TraceEstimator("poisson2d", 256, 4, 4, nb=16, precision=precision)
    # two calls in a row, the second on a smaller input (fewer columns, coarser
    # level): the workspace keeps the first call's contents
    _compare(est, 1, 12, 4, m._capi.SMOOTH_ZERO_START, True, 1)
    _compare(est, 2, 5, 3, 0, True, 2)
    _compare(est, 1, 3, 2, m._capi.SMOOTH_REVERSE, False, 3)


def test_noalloc_wilson_matches_allocating_entry_point():
    require_gpu()
    import paper_2108_11281_amd as m
    N = 32
    est = m.TraceEstimator("wilson2d", N, 3, 3, mass=0.1, field=gauge_field(N, seed=2), block=4,
                           n_vec=8, setup_sweeps=6, setup_seed=1, precision="fp32_ir64", nb=8)
    _compare(est, 1, 8, 4, m._capi.SMOOTH_ZERO_START, True, 4, complex_=True)
    _compare(est, 1, 2, 3, 0, False, 5, complex_=True)


def test_noalloc_rejects_inputs_beyond_its_workspace():
    require_gpu()
    import paper_2108_11281_amd as m
    import torch
    # 1024^2 FP32 working copies: 3 x 4 MiB per column, so 8 columns exceed 64 MiB
    est = m.TraceEstimator("poisson2d", 1024, 4, 4, nb=8, precision="fp32_ir64")
    n = est.level_size(1)
    B = torch.zeros((8, n), dtype=torch.float64, device="cuda")
    X = torch.zeros((8, n), dtype=torch.float64, device="cuda")
    rc = _call(est, est._lib.mlmc_smooth_noalloc, 1, B, X, 2, 0)
    assert rc == m._capi.MLMC_EINVAL
    assert b"workspace" in est._lib.mlmc_last_error(est._ctx)
    # a fitting size on the same context still works
    assert _call(est, est._lib.mlmc_smooth_noalloc, 1, B[:4], X[:4], 2, 0) == 0
