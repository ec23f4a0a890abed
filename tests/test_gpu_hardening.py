"""Spectral-hardening set-up (Sect. 4): a 37 500 K blackbody source in a
uniform medium resolved at several cell optical depths, on the GPU against
the oracle, and the whole grid of runs of that section (every cell optical
depth with every density) advanced as one batch."""
import numpy as np
import pytest

from paper_1201_5651_amd import binding, synth
from gpu_util import float_bar, pair, rel, rel_x, to_np

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtau0", [30.0, 10.0])
def test_hardening_parity_fp64(oracle_lib, dtau0):
    """A3-dt02 steps from the neutral start agree with the oracle to 1e-9 in
    x, T and the diagnostics (front radius)."""
    spec = synth.hardening(dtau0, 100.0)
    g, pb, st = pair(spec, synth.density(spec), T0=spec.T0)
    for _ in range(12):
        g.step_o2(spec.t_end)
        pb.step(st, spec.t_end)
    assert np.max(rel_x(to_np(g.x), st["x"])) < 1e-9
    Tg = pb.temperature(st["nH"], to_np(g.x), to_np(g.E))
    Tw = pb.temperature(st["nH"], st["x"], st["E"])
    assert np.max(rel(Tg, Tw)) < 1e-9
    assert g.diagnostics()["r_ion"] == pytest.approx(pb.diagnostics(st)["r_ion"], rel=1e-9)
    g.close()


@pytest.mark.parametrize("dtau0", [30.0, 10.0])
def test_hardening_parity_mixed(oracle_lib, dtau0):
    spec = synth.hardening(dtau0, 100.0, precision="mixed")
    g, pb, st = pair(spec, synth.density(spec), T0=spec.T0, precision="mixed")
    for _ in range(12):
        g.step_o2(spec.t_end)
        pb.step(st, spec.t_end)
    Tg = pb.temperature(st["nH"], to_np(g.x), to_np(g.E))
    Tw = pb.temperature(st["nH"], st["x"], st["E"])
    float_bar(to_np(g.x), st["x"], 1e-4, "mixed hardening x dtau0 %g" % dtau0)
    float_bar(Tg, Tw, 1e-4, "mixed hardening T dtau0 %g" % dtau0)
    g.close()


def test_hardening_grid_as_one_batch():
    """The twelve runs of Sect. 4 (cell optical depth 1, 3, 10, 30 with n_H =
    10, 100, 1000; 27 M cells) advance together.  The three densities of one
    resolution are the same problem in units of R_S and t_rec, so after the
    same number of steps their clocks (in t_rec) and front radii (in R_S)
    agree to float rounding, and every front moves out."""
    specs = synth.hardening_specs("mixed")
    b = binding.Batch(specs)
    b.load([synth.density(s) for s in specs], T0s=[s.T0 for s in specs],
           t_end=[s.t_end for s in specs])
    d0 = b.diagnostics()
    for _ in range(10):
        b.step_o2()
    t, n, _ = b.state()
    d1 = b.diagnostics()
    assert all(k == 10 for k in n)
    by_res = {}
    for s, ti, a, c in zip(specs, t, d0, d1):
        assert c["nonfinite"] == 0
        assert c["r_ion"] > a["r_ion"]
        RS = 150.0 / (s.nH_mean * synth.SIGMA0)
        by_res.setdefault(round(s.dx * s.nH_mean * synth.SIGMA0, 6), []).append((ti / s.t_rec, c["r_ion"] / RS))
    assert len(by_res) == 4
    for runs in by_res.values():
        for tt, rr in runs[1:]:
            assert tt == pytest.approx(runs[0][0], rel=1e-4)
            assert rr == pytest.approx(runs[0][1], rel=1e-4)
    b.close()
