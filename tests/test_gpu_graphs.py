"""Graph replay of steps against plain launches (both through the C ABI).

Two simulations of the same suspension: one on the null stream (every kernel launched one
by one), one on its own stream (runs of 2, 4, 6 or 10 steps replayed from one recorded HIP
graph, the rest launched one by one).  After
every run of steps, with eager work and synchronisation in between, the populations,
particle state and hydrodynamic sums must be bit-identical: the graph holds the same kernels
with the same arguments, the shear protocol comes from the device clock table, and every
reduction of the step is summed in a fixed order.
"""
import sys

import numpy as np
import pytest

import parity_util as PU

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1904_02929_amd import susp
    susp.lib()
    return torch


def _state(sim):
    R, U, W, Q = sim.get_particles()
    F, T, S, nl = sim.hydro()
    return [sim.get_populations(), R, U, W, Q, F, T, S, nl, sim.stress()[0]]


@pytest.mark.parametrize("kind", ["simple", "oscillatory"])
def test_graph_replay_is_bit_identical(torch_mod, kind):
    torch = torch_mod
    from paper_1904_02929_amd import susp
    box, pos, vel, om, rad, kw = PU.dense_workload((41, 48, 37), 0.40, 11, 1e-3)
    if kind == "oscillatory":
        kw = dict(shear_kind=2, g0_I=0.005, g0_F=0.002, period=30, ncyc_I=1, ncyc_F=2, theta=0.3)
    print("\n[graphs] %s shear, box %s, %d spheres" % (kind, box, len(rad)), flush=True)
    sys.stdout.flush()
    p_a = susp.make_params(box, radius=rad, pos=pos, vel=vel, omega=om, precision=susp.FP32, **kw)
    p_b = susp.make_params(box, radius=rad, pos=pos, vel=vel, omega=om, precision=susp.FP32, **kw)
    plain = susp.Simulation(p_a)  # null stream: kernels one by one
    side = torch.cuda.Stream()
    graph = susp.Simulation(p_b, stream=side)
    assert graph.stream.cuda_stream != 0
    for chunk, pairs in ((7, 1), (5, 1), (3, 0), (10, 5), (1, 5), (40, 5), (13, 2), (24, 3)):
        graph.use_graphs(pairs)
        plain.step(chunk)
        graph.step(chunk)
        torch.cuda.synchronize()
        a, b = _state(plain), _state(graph)
        for k, (x, y) in enumerate(zip(a, b)):
            assert np.array_equal(x, y), "chunk %d: field %d differs (rel %g)" % (chunk, k, PU.rel(y, x, 1e-300))
        assert plain.clock() == graph.clock()
    plain.close()
    graph.close()


def test_graph_replay_large_lattice(torch_mod):
    # a lattice of 2^22 nodes (several bricks along every axis, lists of many spheres):
    # plain launches and graph replays must still agree bit for bit
    torch = torch_mod
    from paper_1904_02929_amd import susp
    box, pos, vel, om, rad, kw = PU.dense_workload((256, 128, 128), 0.30, 21, 2e-4)
    print("\n[graphs] large lattice, box %s, %d spheres" % (box, len(rad)), flush=True)
    sys.stdout.flush()
    p_a = susp.make_params(box, radius=rad, pos=pos, vel=vel, omega=om, precision=susp.FP32, **kw)
    p_b = susp.make_params(box, radius=rad, pos=pos, vel=vel, omega=om, precision=susp.FP32, **kw)
    plain = susp.Simulation(p_a)
    side = torch.cuda.Stream()
    graph = susp.Simulation(p_b, stream=side)
    for chunk, pairs in ((3, 0), (10, 5), (7, 2)):
        graph.use_graphs(pairs)
        plain.step(chunk)
        graph.step(chunk)
        torch.cuda.synchronize()
        a, b = _state(plain), _state(graph)
        for k, (x, y) in enumerate(zip(a, b)):
            assert np.array_equal(x, y), "chunk %d: field %d differs" % (chunk, k)
    plain.close()
    graph.close()
