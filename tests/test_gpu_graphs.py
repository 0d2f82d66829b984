"""HIP-graph replay of the refined CG's iteration pairs gives bitwise the same
solutions, samples and iteration counts as direct launches (several solves in a
row, so every graph is replayed many times with eager work in between)."""
import numpy as np
import pytest

from tests.gpu_util import from_dev, require_gpu
from workloads import varcoef_faces

pytestmark = pytest.mark.gpu


def _pair(kind, N, L, **kw):
    require_gpu()
    import paper_2108_11281_amd as m
    common = dict(precision="fp32_ir64", nb=16, solve_tol=1e-11, nu_pre=2, nu_post=2)
    if kind == "varcoef3d":
        common.update(shift=1e-3, field=varcoef_faces(N, seed=1000))
    common.update(kw)
    return (m.TraceEstimator(kind, N, L, L, graphs=0, **common),
            m.TraceEstimator(kind, N, L, L, graphs=1, **common))


@pytest.mark.parametrize("kind,N,L", [("poisson2d", 128, 4), ("varcoef3d", 16, 3)])
def test_graph_replay_is_bitwise_identical(kind, N, L):
    plain, graph = _pair(kind, N, L)
    for seed in (1, 2, 3):
        a = plain.sample_level(1, seed, 0, 21)
        ca = plain.counters()
        b = graph.sample_level(1, seed, 0, 21)
        cb = graph.counters()
        assert np.array_equal(a, b), seed
        assert ca[:3] == cb[:3], (ca, cb)
    B = plain.probes(1, 9, 0, 16)
    Ya, ra = plain.solve(1, B)
    Yb, rb = graph.solve(1, B)
    assert np.array_equal(from_dev(Ya), from_dev(Yb)) and np.array_equal(ra, rb)


def test_graphs_step_aside_while_timing():
    plain, graph = _pair("poisson2d", 128, 4)
    graph.set_timing(["rbgs_sweep"])
    a = plain.sample_level(1, 4, 0, 16)
    b = graph.sample_level(1, 4, 0, 16)
    assert np.array_equal(a, b)
    assert graph.kernel_stats("rbgs_sweep")[0] > 0
    graph.set_timing(False)
