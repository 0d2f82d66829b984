"""Full-size 2D Poisson (1024^2, 6 levels, 128 RHS, FP32 + FP64 refinement):
sampled per-sample parity against the oracle's exact sine-transform solver."""
import numpy as np
import pytest

from oracle import mlmc, operators
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def full():
    require_gpu()
    import paper_2108_11281_amd as m
    est = m.TraceEstimator("poisson2d", 1024, 6, 6, precision="fp32_ir64", nb=128,
                           solve_tol=1e-10)
    yield est
    est.close()


def test_coarse_trace_closed_form(full):
    # A_6 = 2^-5 L^32 so tr(A_6^-1) = 32 T(32)
    ref = 32.0 * operators.poisson2d_trace_inverse(32)
    assert abs(full.coarse_trace().real - ref) <= 1e-11 * ref


@pytest.mark.parametrize("level", [1, 3, 5])
def test_sampled_parity_full_batch(full, level):
    # one full launch of 128 samples; the oracle checks 3 of them one by one
    s, err = full.sample_level(level, 2024, 0, 128, with_error=True)
    assert np.all(np.isfinite(s))
    assert np.all(err <= 1e-8)
    orc = mlmc.PoissonDSTSampler(1024, 6)
    for k in (0, 77, 127):
        ref = orc.sample(level, 2024, k, 1)[0]
        a, b = orc.sample_parts(level, 2024, k, 1)
        scale = abs(a[0]) + abs(b[0])
        assert abs(s[k] - ref) <= 1e-8 * scale, (k, s[k], ref)
