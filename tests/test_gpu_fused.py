"""The micro-physics fused with the persistent raytrace (one launch per half
of an A3 step, or per A2 step, for float storage and grids with one point
source) on the GPU.  Every tile integrates its own cells with the arithmetic
of the separate micro-physics kernels and then sweeps, so a fused step must
equal the separate kernels (tiles of 8) bit for bit: neutral fractions,
energies, columns, clocks, timesteps and work counters, in FP32 and both
mixed forms (their double re-solves done inside the fused launch), in A3 and
A2, for uneven batches advanced by replayed step graphs, and at the 256^3
size of the timed workload.  A batch holding a grid with several sources does
not fuse and still gives the same results."""
import numpy as np
import pytest

from paper_1201_5651_amd import binding, synth
from gpu_util import KB, to_np

pytestmark = pytest.mark.gpu

P = binding.PI_TILE_PERSISTENT


def _start(spec, seed, radius):
    nH = synth.lognormal_density(spec.shape, spec.nH_mean, 1.0, seed)
    x, T = synth.ionised_sphere(spec, radius)
    return nH, x, T


def _advance_grid(spec, precision, edge, steps, order, seed=11, radius=6.0):
    nH, x, T = _start(spec, seed, radius)
    g = binding.Grid(spec, precision=precision)
    g.raytrace_tile = edge
    g.load(nH, x, T0=50.0)
    if g.E is not None:
        import torch
        g.E.copy_(torch.as_tensor(1.5 * KB * nH * (2.0 - x) * T, dtype=g.dtype))
    g.raytrace()
    g.work_counters(reset=True)
    for _ in range(steps):
        (g.step_o2 if order == 2 else g.step_o1)(spec.t_end)
    out = (g.state(), to_np(g.x), None if g.E is None else to_np(g.E), to_np(g.tau),
           g.work_counters())
    g.close()
    return out


def _same(a, b):
    (sa, xa, Ea, ta, wa), (sb, xb, Eb, tb, wb) = a, b
    assert sa == sb
    assert np.array_equal(xa, xb)
    assert np.array_equal(ta, tb)
    if Ea is not None:
        assert np.array_equal(Ea, Eb)
    assert wa == wb
    print("# work counters", wa, flush=True)


@pytest.mark.parametrize("order", [2, 1])
@pytest.mark.parametrize("precision", ["fp32", "mixed", "mixed_front"])
def test_fused_step_equals_separate_kernels(precision, order):
    """A clumpy 40x36x44 grid with an off-centre source and a partly ionised
    start (a front to integrate, cells for the double re-solve), 6 steps."""
    spec = synth.cfg2(n=40).with_(n=(40, 36, 44), src=(13, 20, 30))
    print("# fused", precision, "order", order, flush=True)
    _same(_advance_grid(spec, precision, 8, 6, order), _advance_grid(spec, precision, P, 6, order))


def test_fused_step_resolves_in_double():
    """The mixed-front form re-solves front cells in double inside the fused
    launch: the counter of double re-solves is positive and equal to the
    separate kernels'."""
    spec = synth.cfg2(n=40).with_(n=(40, 36, 44), src=(13, 20, 30))
    a = _advance_grid(spec, "mixed_front", 8, 3, 2)
    b = _advance_grid(spec, "mixed_front", P, 3, 2)
    assert a[4]["resolved_fp64"] > 0
    _same(a, b)


@pytest.mark.parametrize("precision", ["fp32", "mixed"])
def test_fused_batch_graph_replays(precision):
    """Three uneven grids (one with a fixed temperature and a source on a
    corner), 8 replayed step graphs with host synchronisation between some."""
    a = synth.cfg2(n=20).with_(n=(20, 24, 18), src=(10, 12, 9))
    b = synth.cfg1(n=(16, 16, 16), dx=synth.cfg1().dx * 2).with_(src=(0, 0, 0))
    c = synth.cfg2(n=28).with_(n=(28, 12, 20), src=(5, 6, 15), Q=3e48)
    specs = [a, b, c]
    nHs = [synth.lognormal_density(s.shape, s.nH_mean, 1.0, 40 + i) if s.thermal == "evolve"
           else np.full(s.shape, s.nH_mean) for i, s in enumerate(specs)]
    out = {}
    for edge in (8, P):
        bt = binding.Batch(specs, precision=precision)
        bt.raytrace_tile = edge
        bt.load(nHs, T0s=[s.T0 for s in specs], t_end=[s.t_end for s in specs])
        bt.work_counters(reset=True)
        for k in range(8):
            bt.step_o2()
            if k % 3 == 2:
                bt.state()
        out[edge] = (bt.state(), [(to_np(G.x), to_np(G.tau)) for G in bt.grids],
                     bt.work_counters())
        bt.close()
    assert out[8][0] == out[P][0]
    assert out[8][2] == out[P][2]
    for (xa, ta), (xb, tb) in zip(out[8][1], out[P][1]):
        assert np.array_equal(xa, xb)
        assert np.array_equal(ta, tb)


def test_batch_with_several_sources_does_not_fuse():
    """A batch holding a grid with two sources runs the separate kernels with
    the persistent raytrace: same results as tiles of 8."""
    a = synth.cfg2(n=20).with_(n=(20, 24, 18), src=(10, 12, 9))
    b = a.with_(src=(3, 5, 6), more_sources=(((15, 20, 12), 2e48),))
    specs = [a, b]
    nHs = [synth.lognormal_density(s.shape, s.nH_mean, 1.0, 50 + i) for i, s in enumerate(specs)]
    out = {}
    for edge in (8, P):
        bt = binding.Batch(specs, precision="mixed")
        bt.raytrace_tile = edge
        bt.load(nHs, T0s=[s.T0 for s in specs], t_end=[s.t_end for s in specs])
        for _ in range(5):
            bt.step_o2()
        out[edge] = (bt.state(), [(to_np(G.x), to_np(G.tau)) for G in bt.grids])
        bt.close()
    assert out[8][0] == out[P][0]
    for (xa, ta), (xb, tb) in zip(out[8][1], out[P][1]):
        assert np.array_equal(xa, xb)
        assert np.array_equal(ta, tb)


def test_fused_step_full_size_mixed():
    """The timed workload's grid (256^3 lognormal medium, central 5e48 /s
    blackbody source, mixed precision) from the neutral start: 4 fused A3
    steps equal 4 steps of the separate kernels bit for bit."""
    spec = synth.cfg3(n=256)
    nH = synth.density(spec)
    out = {}
    for edge in (8, P):
        print("# 256^3 steps, raytrace", edge, flush=True)
        g = binding.Grid(spec, precision="mixed")
        g.raytrace_tile = edge
        g.load(nH, 1.0, T0=spec.T0)
        for _ in range(4):
            g.step_o2(spec.t_end)
        out[edge] = (g.state(), to_np(g.x), to_np(g.E), to_np(g.tau))
        g.close()
    assert out[8][0] == out[P][0]
    for a, b in zip(out[8][1:], out[P][1:]):
        assert np.array_equal(a, b)


CR_CASES = [  # (h, tau_buf, from, to, tau_out): predictor, corrector, corrector timing form, A2
    (0.5, binding.PI_BUF_N, binding.PI_BUF_N, binding.PI_BUF_HALF, binding.PI_BUF_HALF),
    (1.0, binding.PI_BUF_HALF, binding.PI_BUF_N, binding.PI_BUF_N, binding.PI_BUF_N),
    (1.0, binding.PI_BUF_HALF, binding.PI_BUF_N, binding.PI_BUF_HALF, binding.PI_BUF_N),
    (1.0, binding.PI_BUF_N, binding.PI_BUF_N, binding.PI_BUF_N, binding.PI_BUF_N),
]


@pytest.mark.parametrize("precision", ["fp32", "mixed", "mixed_front", "fp64"])
def test_chem_raytrace_equals_chem_step_then_raytrace(precision):
    """pi_chem_raytrace (fused where the grid allows it) against pi_chem_step
    followed by pi_raytrace on tiles of 8, for the buffer pairings of the
    step's predictor and corrector, the corrector's timing form and A2: every
    state, column and work counter equal bit for bit."""
    import torch
    spec = synth.cfg2(n=40).with_(n=(40, 36, 44), src=(13, 20, 30))
    nH, x, T = _start(spec, 5, 6.0)
    out = {}
    for edge, fused in ((8, False), (P, True)):
        g = binding.Grid(spec, precision=precision)
        g.raytrace_tile = edge
        g.load(nH, x, T0=50.0)
        g.E.copy_(torch.as_tensor(1.5 * KB * nH * (2.0 - x) * T, dtype=g.dtype))
        g.raytrace()
        g.timestep(spec.t_end)
        # the half-step buffers start as copies of state n
        for a, b in (("x_half", "x"), ("E_half", "E"), ("tau_half", "tau")):
            getattr(g, a).copy_(getattr(g, b))
        g.work_counters(reset=True)
        res = []
        for h, tb, fr, to, tout in CR_CASES:
            if fused:
                g.chem_raytrace(h, tb, fr, to, tout, use_device_dt=True)
            else:
                g.chem_step(h, tb, fr, to, use_device_dt=True)
                g.raytrace(to, tout)
            res.append([to_np(getattr(g, k)) for k in ("x", "E", "tau", "x_half", "E_half",
                                                        "tau_half")])
        out[fused] = (res, g.work_counters(), g.state())
        g.close()
    assert out[False][1] == out[True][1] and out[False][2] == out[True][2]
    for ra, rb in zip(out[False][0], out[True][0]):
        for a, b in zip(ra, rb):
            assert np.array_equal(a, b)
