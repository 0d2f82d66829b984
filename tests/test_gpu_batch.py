"""The batch of uneven problems: several 3D diffusion problems of different
sizes sampled concurrently (one HIP stream and one host worker per problem slot)
give bit-identical samples to sampling each problem alone, and those samples
match the oracle."""
import numpy as np
import pytest

from oracle import hierarchy, mlmc
from tests.gpu_util import quad_scale, require_gpu
from workloads import varcoef_faces, varcoef_levels

pytestmark = pytest.mark.gpu

SHIFT = 1e-3


def _problems(sides, nb=16):
    torch = require_gpu()
    import paper_2108_11281_amd as m
    ests = []
    for p, N in enumerate(sides):
        L = varcoef_levels(N, max_coarse=64)
        ests.append(m.TraceEstimator("varcoef3d", N, L, L, shift=SHIFT,
                                     field=varcoef_faces(N, seed=1000 + p), nb=nb,
                                     precision="fp32_ir64", solve_tol=1e-12,
                                     stream=torch.cuda.Stream()))
    return ests


def test_concurrent_batch_equals_sequential_and_oracle():
    import paper_2108_11281_amd as m
    sides = [16, 24, 8, 16]
    ests = _problems(sides)
    seeds = [1000 + p for p in range(len(sides))]
    s_conc, sec = m.batch_sample(ests, 1, seeds, 3, 20, workers=3)
    assert np.all(sec > 0)
    for p, e in enumerate(ests):
        alone = e.sample_level(1, seeds[p], 3, 20)
        assert np.array_equal(s_conc[p], alone), p
    # against the oracle's exact level differences (two smallest problems)
    for p in (0, 2):
        N = sides[p]
        L = varcoef_levels(N, max_coarse=64)
        A, P = hierarchy.varcoef_hierarchy(N, varcoef_faces(N, seed=1000 + p), SHIFT, L)
        orc = mlmc.LevelSampler(A, P, complex_probe=False)
        ref = orc.sample(1, seeds[p], 3, 20)
        scale = quad_scale(orc.sample_parts(1, seeds[p], 3, 20))
        assert np.all(np.abs(s_conc[p] - ref) <= 1e-8 * scale)


def test_batch_rejects_bad_arguments():
    import paper_2108_11281_amd as m
    ests = _problems([8, 8])
    with pytest.raises(m.MLMCError):
        m.batch_sample([ests[0], ests[0]], 1, [1, 2], 0, 4)     # same context twice
    with pytest.raises(m.MLMCError):
        m.batch_sample(ests, 5, [1, 2], 0, 4)                   # level not sampleable
