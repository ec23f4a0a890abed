"""Degenerate and extreme inputs on the GPU: no source, a fully ionised start,
and the largest grid the serving workload admits (512^3)."""
import numpy as np
import pytest

import oracle
from paper_1201_5651_amd import binding, synth
from gpu_util import float_bar, pair, rel, rel_x, stored, to_np

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_no_source_no_recombination_leaves_the_state(oracle_lib, precision):
    """Q = 0 with the table spectrum, no recombination or collisions: nothing
    changes x; columns stay those of the start and the oracle agrees."""
    spec = synth.cfg2(n=12).with_(Q=0.0, alpha_B=0.0, collisional=False, precision=precision)
    nH = synth.lognormal_density(spec.shape, 10.0, 1.0, 3)
    x0 = np.random.default_rng(2).uniform(0.1, 1.0, spec.shape)
    g, pb, st = pair(spec, nH, x0=x0, T0=300.0, precision=precision)
    xs = to_np(g.x)
    for _ in range(3):
        g.step_o2(spec.t_rec)
        pb.step(st, spec.t_rec)
    assert np.array_equal(to_np(g.x), xs)
    assert np.all(np.isfinite(st["x"])) and np.max(rel_x(st["x"], x0)) == 0.0
    g.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_ionised_start(oracle_lib, precision):
    """A start with x = 1e-6 everywhere (ionised gas recombining and being
    re-ionised): steps agree with the oracle."""
    spec = synth.cfg2(n=12).with_(precision=precision)
    nH = synth.lognormal_density(spec.shape, 10.0, 1.0, 4)
    g, pb, st = pair(spec, nH, x0=np.full(spec.shape, 1e-6), T0=1e4, precision=precision)
    for _ in range(4):
        g.step_o2(spec.t_end)
        pb.step(st, spec.t_end)
    err = rel_x(to_np(g.x), st["x"])
    if precision == "fp64":
        assert np.max(err) < 1e-9
    else:
        float_bar(to_np(g.x), st["x"], 1e-4, "mixed ionised start x")
    g.close()


def test_512_cubed_raytrace_and_steps(oracle_lib):
    """The largest grid of the serving workload: 512^3 (134 M cells) of the
    clumpy medium in mixed precision.  The raytrace of a synthetic partly
    ionised state (an ionised sphere of 150 cells' radius) matches the
    oracle's on every cell, and a few A3 steps from it run with finite
    diagnostics."""
    import torch
    spec = synth.cfg3(n=512)
    nH = stored(synth.density(spec), "mixed")
    x, T = synth.ionised_sphere(spec, 150.0)
    x = stored(x, "mixed")
    g = binding.Grid(spec, precision="mixed")
    g.load(nH, x, T0=spec.T0)
    want = oracle.Problem.from_spec(spec).raytrace(nH, x)
    got = to_np(g.tau)
    assert np.all((got == 0) == (want == 0))
    m = want > 1e-3
    float_bar(got[m], want[m], 1e-4, "512^3 mixed columns")
    assert np.max(np.abs(got[~m] - want[~m])) < 1e-7
    del got, want
    g.E.copy_(torch.as_tensor(1.5 * 1.380649e-16 * nH * (2.0 - x) * T, dtype=g.dtype))
    for _ in range(3):
        g.step_o2(spec.t_end)
    d = g.diagnostics()
    assert d["nonfinite"] == 0 and d["n_ion"] > 0
    g.close()
