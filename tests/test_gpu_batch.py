"""Batched form on the GPU: many uneven grids advanced by one launch per kernel
(each step a replayed HIP graph).  A grid's results must not depend on the
batch around it: every grid of a batch is compared bit for bit with the same
grid advanced alone, and small batches are compared with the oracle."""
import numpy as np
import pytest

from paper_1201_5651_amd import binding, synth
from gpu_util import pair, rel, rel_x, to_np

pytestmark = pytest.mark.gpu


def _specs(precision):
    """Three uneven grids: different shapes, source vertices (one on a corner,
    one off-centre), spectra, thermal modes and luminosities."""
    a = synth.cfg2(n=20)
    a = synth.GridSpec(**{**a.__dict__, "name": "a", "n": (20, 24, 18), "src": (10, 12, 9),
                          "precision": precision})
    b = synth.cfg1(n=(16, 16, 16), dx=synth.cfg1().dx * 2)
    b = synth.GridSpec(**{**b.__dict__, "name": "b", "precision": precision})
    c = synth.cfg2(n=28)
    c = synth.GridSpec(**{**c.__dict__, "name": "c", "n": (28, 12, 20), "src": (5, 6, 15),
                          "Q": 3e48, "precision": precision})
    return [a, b, c]


def _densities(specs):
    out = []
    for i, s in enumerate(specs):
        if s.thermal == "evolve":
            out.append(synth.lognormal_density(s.shape, s.nH_mean, 1.0, 10 + i))
        else:
            out.append(np.full(s.shape, s.nH_mean))
    return out


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_matches_grids_advanced_alone_bitwise(precision):
    specs = _specs(precision)
    nHs = _densities(specs)
    t_end = [s.t_end for s in specs]
    steps = 6
    alone = []
    for s, nH in zip(specs, nHs):
        g = binding.Grid(s, precision=precision)
        g.load(nH, 1.0, T0=s.T0)
        for _ in range(steps):
            g.step_o2(s.t_end)
        t, n, _ = g.state()
        alone.append((t, n, to_np(g.x), None if g.E is None else to_np(g.E), to_np(g.tau)))
        g.close()
    b = binding.Batch(specs, precision=precision)
    b.load(nHs, T0s=[s.T0 for s in specs], t_end=t_end)
    for k in range(steps):
        b.step_o2()
        if k % 2 == 1:
            b.state()   # host synchronisation between graph replays
    t, n, _ = b.state()
    for i, (ta, na, xa, Ea, taua) in enumerate(alone):
        G = b.grids[i]
        assert n[i] == na == steps
        assert t[i] == ta
        assert np.array_equal(to_np(G.x), xa), i
        assert np.array_equal(to_np(G.tau), taua), i
        if Ea is not None:
            assert np.array_equal(to_np(G.E), Ea), i
    b.close()


def test_batch_grids_stop_at_their_own_t_end():
    specs = _specs("fp64")
    nHs = _densities(specs)
    # grid 0 stops after a short interval, the others go on
    t_end = [specs[0].t_rec * 1e-3, specs[1].t_end, specs[2].t_end]
    b = binding.Batch(specs)
    b.load(nHs, T0s=[s.T0 for s in specs], t_end=t_end)
    for _ in range(40):
        b.step_o2()
    t, n, _ = b.state()
    assert t[0] == t_end[0]
    x0 = to_np(b.grids[0].x)
    for _ in range(3):
        b.step_o2()
    t2, n2, _ = b.state()
    assert n2[0] == n[0] and t2[0] == t[0]
    assert np.array_equal(to_np(b.grids[0].x), x0)
    assert n2[1] == n[1] + 3 and n2[2] == n[2] + 3
    d = b.diagnostics()
    assert all(di["nonfinite"] == 0 for di in d)
    b.close()


def test_batch_parity_with_oracle(oracle_lib):
    """Two grids of one batch against the oracle run grid by grid (FP64)."""
    specs = _specs("fp64")[:2]
    nHs = _densities(specs)
    b = binding.Batch(specs)
    b.load(nHs, T0s=[s.T0 for s in specs], t_end=[s.t_end for s in specs])
    import oracle
    for _ in range(4):
        b.step_o2()
    for i, (s, nH) in enumerate(zip(specs, nHs)):
        pb = oracle.Problem.from_spec(s)
        st = pb.initial_state(np.asarray(nH, dtype=np.float64), T0=s.T0)
        for _ in range(4):
            pb.step(st, s.t_end)
        assert np.max(rel_x(to_np(b.grids[i].x), st["x"])) < 1e-9
        m = st["tau"] > 0
        assert np.max(rel(to_np(b.grids[i].tau)[m], st["tau"][m])) < 1e-9
        if st["E"] is not None:
            assert np.max(rel(to_np(b.grids[i].E), st["E"])) < 1e-9
    b.close()


def test_batch_of_generated_uneven_grids_runs_and_conserves():
    """A small generated batch (uneven n, lognormal and uniform media) runs a
    few steps with finite states and an ionised volume that grows."""
    specs = synth.batch_specs(count=6, seed=3, nmin=16, nmax=40, precision="mixed")
    nHs = [synth.density(s) for s in specs]
    b = binding.Batch(specs)
    b.load(nHs, T0s=[s.T0 for s in specs], t_end=[s.t_end for s in specs])
    d0 = b.diagnostics()
    for _ in range(8):
        b.step_o2()
    d1 = b.diagnostics()
    t, n, _ = b.state()
    assert all(k == 8 for k in n)
    for a, c in zip(d0, d1):
        assert c["nonfinite"] == 0
        assert c["v_ion"] > a["v_ion"]
    b.close()


def test_nan_in_one_grid_stays_in_that_grid():
    """A non-finite value planted in one grid's state is reported for that grid
    only; the other grids of the batch advance bit for bit as they do alone."""
    specs = _specs("fp64")
    nHs = _densities(specs)
    alone = {}
    for i in (0, 2):
        g = binding.Grid(specs[i])
        g.load(nHs[i], 1.0, T0=specs[i].T0)
        for _ in range(5):
            g.step_o2(specs[i].t_end)
        alone[i] = to_np(g.x)
        g.close()
    b = binding.Batch(specs)
    b.load(nHs, T0s=[s.T0 for s in specs], t_end=[s.t_end for s in specs])
    b.grids[1].x[3, 4, 5] = float("nan")
    for _ in range(5):
        b.step_o2()
    d = b.diagnostics(raise_on_nan=False)
    assert d[1]["nonfinite"] > 0
    assert d[0]["nonfinite"] == 0 and d[2]["nonfinite"] == 0
    for i in (0, 2):
        assert np.array_equal(to_np(b.grids[i].x), alone[i])
    with pytest.raises(binding.PiError) as e:
        b.diagnostics()
    assert e.value.status == binding.PI_ENAN
    b.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_checkpoint_and_resume_is_bitwise(precision):
    """The state is the caller's fields plus the clock: copying them into a new
    grid and setting its clock continues the run bit for bit."""
    spec = _specs(precision)[0]
    nH = _densities([spec])[0]
    g = binding.Grid(spec, precision=precision)
    g.load(nH, 1.0, T0=spec.T0)
    for _ in range(5):
        g.step_o2(spec.t_end)
    t, n, _ = g.state()
    saved = {k: getattr(g, k).clone() for k in ("nH", "x", "E", "tau")}
    for _ in range(4):
        g.step_o2(spec.t_end)
    want_x, want_E, want_t = to_np(g.x), to_np(g.E), g.state()[0]
    g.close()
    r = binding.Grid(spec, precision=precision)
    for k, v in saved.items():
        getattr(r, k).copy_(v)
    r.set_time(t, n)
    for _ in range(4):
        r.step_o2(spec.t_end)
    assert r.state()[0] == want_t
    assert np.array_equal(to_np(r.x), want_x)
    assert np.array_equal(to_np(r.E), want_E)
    r.close()
