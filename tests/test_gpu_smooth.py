"""GPU parity of the smoother kernels (the V-cycle's red-black Gauss-Seidel
sweeps, called through mlmc_smooth) against the oracle's coloured sweep, and
the two-sweep fused pass of the 2D Poisson levels against two one-sweep passes,
bit for bit."""
import numpy as np
import pytest

from oracle import hierarchy
from tests.gpu_util import from_dev, require_gpu, to_dev
from workloads import gauge_field, varcoef_faces

pytestmark = pytest.mark.gpu

NRHS = 5
# FP32 sweeps against the FP64 oracle: inputs rounded to FP32 and a few
# roundings per update; the sweep is a contraction, so the error stays at a
# few FP32 ulps of the largest value
TOL = {"fp64": 1e-13, "fp32_ir64": 1e-5}


def _check(est, A, colour, level, precision, complex_=False, sweeps=(1, 2, 3), tol=None,
           zero_start=False):
    tol = TOL[precision] if tol is None else max(tol, TOL[precision])
    rng = np.random.default_rng(level)
    n = A.shape[0]
    B = rng.standard_normal((NRHS, n))
    X = rng.standard_normal((NRHS, n))
    if complex_:
        B = B + 1j * rng.standard_normal((NRHS, n))
        X = X + 1j * rng.standard_normal((NRHS, n))
    if zero_start:   # the V-cycle's pre-smoothing: forward sweeps from X = 0
        X = np.zeros_like(B)
    for sw in sweeps:
        for reverse in ((False,) if zero_start else (False, True)):
            if zero_start:
                got = from_dev(est.smooth(level, to_dev(B), None, sw, zero_start=True), complex_)
            else:
                got = from_dev(est.smooth(level, to_dev(B), to_dev(X), sw, reverse), complex_)
            for k in range(NRHS):
                ref = hierarchy.rbgs_sweeps(A, B[k], X[k], colour, sw, reverse)
                err = np.max(np.abs(got[k] - ref))
                assert err <= tol * np.max(np.abs(ref)), (level, sw, reverse, k, err)


def _poisson(N, L, precision):
    require_gpu()
    import paper_2108_11281_amd as m
    return m.TraceEstimator("poisson2d", N, L, L, nb=8, precision=precision)


# sides 200 -> 100 -> 50 -> 25: the register-march kernels on 200 and 100
# (ragged last wave of columns and last row segment), the LDS tile kernel on 50;
# 128 -> 64 -> 32: power-of-two edges, the march kernel's smallest side (64);
# 512 -> 256 and 392 -> 196: five and three waves of 120 columns per row (512,
# 256), the last one mostly outside the grid (392, 196)
@pytest.mark.parametrize("precision", ["fp32_ir64", "fp64"])
@pytest.mark.parametrize("N,L", [(200, 4), (128, 3), (512, 3), (392, 3)])
def test_poisson_sweeps_match_oracle(N, L, precision):
    est = _poisson(N, L, precision)
    A, _ = hierarchy.poisson_hierarchy(N, L)
    for level in range(1, L):
        side = N >> (level - 1)
        _check(est, A[level - 1], hierarchy.site_coloring(side), level, precision)


@pytest.mark.parametrize("precision", ["fp32_ir64", "fp64"])
@pytest.mark.parametrize("N", [200, 512])
def test_fused_two_sweep_pass_equals_two_passes_bitwise(precision, N):
    # 200, 100: two waves of 120 columns per row, the second ragged, and one;
    # 512, 256: five and three waves
    est = _poisson(N, 3, precision)
    rng = np.random.default_rng(7)
    for level in (1, 2):
        n = est.level_size(level)
        B = to_dev(rng.standard_normal((NRHS, n)))
        X = to_dev(rng.standard_normal((NRHS, n)))
        for reverse in (False, True):
            one = X
            for sw in range(1, 4):
                one = est.smooth(level, B, one, 1, reverse)
                fused = est.smooth(level, B, X, sw, reverse)
                assert np.array_equal(from_dev(fused), from_dev(one)), (level, sw, reverse)


@pytest.mark.parametrize("precision", ["fp32_ir64", "fp64"])
@pytest.mark.parametrize("N", [200, 384])
def test_pre_pass_restricted_residual(precision, N):
    # the V-cycle's last pre-smoothing pass writes R (b - A x) with the swept x;
    # two fused sweeps do it in one pass, one sweep with the stand-alone kernel
    # (384, 192: the restriction's 116-column waves, four and two per row)
    est = _poisson(N, 3, precision)
    A, P = hierarchy.poisson_hierarchy(N, 3)
    rng = np.random.default_rng(11)
    for level in (1, 2):
        n = est.level_size(level)
        Bh = rng.standard_normal((NRHS, n))
        B, X = to_dev(Bh), to_dev(rng.standard_normal((NRHS, n)))
        for sw in (1, 2, 3):
            xr, rc = est.smooth(level, B, X, sw, restrict=True)
            assert np.array_equal(from_dev(xr), from_dev(est.smooth(level, B, X, sw)))
            x, r = from_dev(xr), from_dev(rc)
            Al, Pl = A[level - 1], P[level - 1]
            for k in range(NRHS):
                ref = Pl.T @ (Bh[k] - Al @ x[k])
                bound = np.max(Pl.T @ (np.abs(Bh[k]) + abs(Al) @ np.abs(x[k])))
                assert np.max(np.abs(r[k] - ref)) <= TOL[precision] * bound, (level, sw, k)
        # the fused pass and the stand-alone kernel form the same values
        x1 = est.smooth(level, B, X, 1)
        xa, rca = est.smooth(level, B, x1, 1, restrict=True)
        xb, rcb = est.smooth(level, B, X, 2, restrict=True)
        assert np.array_equal(from_dev(xa), from_dev(xb))
        assert np.array_equal(from_dev(rca), from_dev(rcb)), level


@pytest.mark.parametrize("precision", ["fp32_ir64", "fp64"])
def test_wilson_and_block_sweeps_match_oracle(precision):
    require_gpu()
    import paper_2108_11281_amd as m
    N, L, m0 = 32, 3, 0.1
    th = gauge_field(N, seed=2)
    est = m.TraceEstimator("wilson2d", N, L, L, mass=m0, field=th, block=4, n_vec=8,
                           setup_sweeps=6, setup_seed=1, precision=precision, nb=8)
    A, _ = hierarchy.wilson_hierarchy(N, th, m0, L, block=4, n_vec=8, sweeps=6, seed=1)
    # level 1: 2 spins per site (1 sweep: the one-colour kernel pair; 2: two
    # fused two-colour passes, x -> scratch -> x; 3: one in-place sweep, then
    # two fused passes); level 2: 8 coarse unknowns per 4 x 4 aggregate
    _check(est, A[0], np.repeat(hierarchy.site_coloring(N), 2), 1, precision, True, (1, 2, 3))
    # (the oracle's own test-vector basis agrees with the library's to ~1e-12,
    # so the coarse operator, and the sweep through it, to about 1e-9)
    _check(est, A[1], np.repeat(hierarchy.site_coloring(N // 4), 8), 2, precision, True, (1, 2),
           tol=1e-9)


@pytest.mark.parametrize("precision", ["fp32_ir64", "fp64"])
def test_wilson_sweeps_tile16_match_oracle(precision):
    # side 16: the fused pass takes one 16 x 16 tile whose halo wraps onto the
    # tile itself
    require_gpu()
    import paper_2108_11281_amd as m
    N, L, m0 = 16, 2, 0.1
    th = gauge_field(N, seed=3)
    est = m.TraceEstimator("wilson2d", N, L, L, mass=m0, field=th, block=4, n_vec=4,
                           setup_sweeps=4, setup_seed=1, precision=precision, nb=8)
    A, _ = hierarchy.wilson_hierarchy(N, th, m0, L, block=4, n_vec=4, sweeps=4, seed=1)
    _check(est, A[0], np.repeat(hierarchy.site_coloring(N), 2), 1, precision, True, (1, 2, 3, 4))


# N = 20: the fused 3D sweep marches all planes (20, 10); N = 40: z segments of
# 16 planes (the last ragged) and 5 tiles of 8 rows on level 1
@pytest.mark.parametrize("precision", ["fp32_ir64", "fp64"])
@pytest.mark.parametrize("N", [20, 40])
def test_varcoef_sweeps_match_oracle(precision, N):
    require_gpu()
    import paper_2108_11281_amd as m
    L = 3
    faces = varcoef_faces(N, seed=1000)
    est = m.TraceEstimator("varcoef3d", N, L, L, shift=1e-3, field=faces, nb=8,
                           precision=precision)
    A, P = hierarchy.varcoef_hierarchy(N, faces, 1e-3, L)
    rng = np.random.default_rng(12)
    for level in (1, 2):
        _check(est, A[level - 1], hierarchy.site_coloring_3d(N >> (level - 1)), level, precision,
               sweeps=(1, 2))
        # the V-cycle's residual restriction R (b - A x) of the swept x
        n = est.level_size(level)
        Bh = rng.standard_normal((NRHS, n))
        xr, rc = est.smooth(level, to_dev(Bh), to_dev(rng.standard_normal((NRHS, n))), 2,
                            restrict=True)
        x, r = from_dev(xr), from_dev(rc)
        Al, Pl = A[level - 1], P[level - 1]
        for k in range(NRHS):
            ref = Pl.T @ (Bh[k] - Al @ x[k])
            bound = np.max(abs(Pl.T) @ (np.abs(Bh[k]) + abs(Al) @ np.abs(x[k])))
            assert np.max(np.abs(r[k] - ref)) <= TOL[precision] * bound, (level, k)


def test_smooth_rejects_bad_arguments():
    est = _poisson(64, 3, "fp32_ir64")
    import paper_2108_11281_amd as m
    import torch
    B = torch.zeros((2, est.level_size(3)), dtype=torch.float64, device="cuda")
    with pytest.raises(m.MLMCError):   # no smoother on the coarsest level
        est.smooth(3, B, B, 1)
    B = torch.zeros((2, est.level_size(1)), dtype=torch.float64, device="cuda")
    with pytest.raises(m.MLMCError):
        est.smooth(1, B, B, -1)
    with pytest.raises(m.MLMCError):   # the restricted residual follows a forward pass
        est.smooth(1, B, B, 2, reverse=True, restrict=True)


def test_varcoef_in_place_sweep_above_side_128():
    # sides above 128 keep the in-place pair of colour launches (the fused 3D
    # pass holds a row of at most 128 cells in one wave)
    require_gpu()
    import paper_2108_11281_amd as m
    from oracle import operators
    N = 136
    faces = varcoef_faces(N, seed=1000)
    est = m.TraceEstimator("varcoef3d", N, 4, 4, shift=1e-3, field=faces, nb=4,
                           precision="fp32_ir64")
    A = operators.varcoef3d(N, faces, 1e-3).tocsr()
    colour = hierarchy.site_coloring_3d(N)
    rng = np.random.default_rng(4)
    B = rng.standard_normal((2, A.shape[0]))
    X = rng.standard_normal((2, A.shape[0]))
    for reverse in (False, True):
        got = from_dev(est.smooth(1, to_dev(B), to_dev(X), 1, reverse))
        for k in range(2):
            ref = hierarchy.rbgs_sweeps(A, B[k], X[k], colour, 1, reverse)
            err = np.max(np.abs(got[k] - ref))
            assert err <= TOL["fp32_ir64"] * np.max(np.abs(ref)), (reverse, k, err)


# The zero-start kernel forms that every V-cycle pre-smoothing runs (the first
# pass reads no iterate): Poisson one- and two-sweep passes from zero (march and
# tile sides, both precisions), the Wilson fused two-colour pass from zero (32^2
# tiles and the 16^2 lattice whose halo wraps onto its one tile), the coarse
# block-stencil sweep, and the 3D fused sweep from zero.
@pytest.mark.parametrize("precision", ["fp32_ir64", "fp64"])
@pytest.mark.parametrize("N,L", [(200, 4), (128, 3)])
def test_poisson_zero_start_sweeps_match_oracle(N, L, precision):
    est = _poisson(N, L, precision)
    A, P = hierarchy.poisson_hierarchy(N, L)
    rng = np.random.default_rng(21)
    for level in range(1, L):
        side = N >> (level - 1)
        _check(est, A[level - 1], hierarchy.site_coloring(side), level, precision,
               sweeps=(1, 2, 3, 4), zero_start=True)
        # with the restricted residual of the pre-smoothing's last pass
        n = est.level_size(level)
        Bh = rng.standard_normal((NRHS, n))
        for sw in (1, 2, 3, 4):
            xr, rc = est.smooth(level, to_dev(Bh), None, sw, restrict=True, zero_start=True)
            x, r = from_dev(xr), from_dev(rc)
            Al, Pl = A[level - 1], P[level - 1]
            for k in range(NRHS):
                ref = hierarchy.rbgs_sweeps(Al, Bh[k], np.zeros(n),
                                            hierarchy.site_coloring(side), sw, False)
                assert np.max(np.abs(x[k] - ref)) <= TOL[precision] * np.max(np.abs(ref))
                rref = Pl.T @ (Bh[k] - Al @ x[k])
                bound = np.max(Pl.T @ (np.abs(Bh[k]) + abs(Al) @ np.abs(x[k])))
                assert np.max(np.abs(r[k] - rref)) <= TOL[precision] * bound, (level, sw, k)


@pytest.mark.parametrize("precision", ["fp32_ir64", "fp64"])
@pytest.mark.parametrize("N,nvec", [(16, 4), (32, 8)])
def test_wilson_zero_start_sweeps_match_oracle(N, nvec, precision):
    require_gpu()
    import paper_2108_11281_amd as m
    L, m0 = (2 if N == 16 else 3), 0.1
    th = gauge_field(N, seed=3 if N == 16 else 2)
    sweeps = 4 if N == 16 else 6
    est = m.TraceEstimator("wilson2d", N, L, L, mass=m0, field=th, block=4, n_vec=nvec,
                           setup_sweeps=sweeps, setup_seed=1, precision=precision, nb=8)
    A, _ = hierarchy.wilson_hierarchy(N, th, m0, L, block=4, n_vec=nvec, sweeps=sweeps, seed=1)
    _check(est, A[0], np.repeat(hierarchy.site_coloring(N), 2), 1, precision, True,
           (1, 2, 3, 4), zero_start=True)
    if L > 2:
        _check(est, A[1], np.repeat(hierarchy.site_coloring(N // 4), nvec), 2, precision, True,
               (1, 2), tol=1e-9, zero_start=True)


@pytest.mark.parametrize("precision", ["fp32_ir64", "fp64"])
def test_varcoef_zero_start_sweeps_match_oracle(precision):
    require_gpu()
    import paper_2108_11281_amd as m
    N, L = 40, 3
    faces = varcoef_faces(N, seed=1000)
    est = m.TraceEstimator("varcoef3d", N, L, L, shift=1e-3, field=faces, nb=8,
                           precision=precision)
    A, _ = hierarchy.varcoef_hierarchy(N, faces, 1e-3, L)
    for level in (1, 2):
        _check(est, A[level - 1], hierarchy.site_coloring_3d(N >> (level - 1)), level,
               precision, sweeps=(1, 2, 3), zero_start=True)


def test_zero_start_rejects_reverse():
    import paper_2108_11281_amd as m
    import torch
    est = _poisson(64, 3, "fp32_ir64")
    B = torch.zeros((2, est.level_size(1)), dtype=torch.float64, device="cuda")
    with pytest.raises(m.MLMCError):
        est.smooth(1, B, None, 2, reverse=True, zero_start=True)
