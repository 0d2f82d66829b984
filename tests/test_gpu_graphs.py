"""HIP-graph replay of the refined CG's iteration pairs and of the FGMRES
iterations gives bitwise the same solutions, samples and iteration counts as
direct launches (several solves in a row, so every graph is replayed many times
with eager work in between)."""
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


def _lattice_pair(kind, precision, learned):
    require_gpu()
    import paper_2108_11281_amd as m
    from workloads import gauge_field
    N = 32
    if kind == "wilson2d":
        common = dict(mass=0.1, field=gauge_field(N, seed=1), n_vec=8, nu_pre=2, nu_post=2,
                      learned=1 if learned else 0)
    else:
        common = dict(mass=0.0, field=gauge_field(N, sigma=0.3, seed=1), n_vec=4, nu_pre=1,
                      nu_post=1)
    common.update(block=4, setup_sweeps=6, setup_seed=1, precision=precision, nb=16,
                  solve_tol=1e-11)
    return (m.TraceEstimator(kind, N, 3, 3, graphs=0, **common),
            m.TraceEstimator(kind, N, 3, 3, graphs=1, **common))


@pytest.mark.parametrize("kind,precision,learned", [
    ("wilson2d", "fp32_ir64", False), ("wilson2d", "fp64", False),
    ("wilson2d", "fp32_ir64", True), ("gauge2d", "fp32_ir64", False)])
def test_fgmres_graph_replay_is_bitwise_identical(kind, precision, learned):
    # every FGMRES iteration replayed from its graph (complex64 and complex128
    # bases, the learned smoother's V-cycle, the gauge Laplacian): the same
    # samples, solutions, iteration and V-cycle counts and network statistics
    plain, graph = _lattice_pair(kind, precision, learned)
    if learned:
        from workloads import nn_init_weights
        w = nn_init_weights(3) * 1.5
        plain.set_nn_weights(w)
        graph.set_nn_weights(w)
    for seed in (1, 2):
        a = plain.sample_level(1, seed, 0, 21)
        b = graph.sample_level(1, seed, 0, 21)
        assert np.array_equal(a, b), seed
        assert plain.counters()[:3] == graph.counters()[:3]
        if learned:
            assert plain.learned_stats() == graph.learned_stats()
    B = plain.probes(1, 9, 0, 16)
    Ya, ra = plain.solve(1, B)
    Yb, rb = graph.solve(1, B)
    assert np.array_equal(from_dev(Ya), from_dev(Yb)) and np.array_equal(ra, rb)
    plain.close()
    graph.close()
