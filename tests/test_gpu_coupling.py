"""Time-centred density for the half-step raytrace (Sect. 2.2: the second
raytrace of A3 uses the half-step density, which a hydrodynamics code
supplies): GPU against the oracle, the identity case, and in a batch."""
import numpy as np
import pytest

from paper_1201_5651_amd import binding, synth
from gpu_util import float_bar, pair, rel, rel_x, stored, to_np

pytestmark = pytest.mark.gpu


def _case(precision):
    spec = synth.cfg2(n=20).with_(precision=precision)
    nH = synth.lognormal_density(spec.shape, 10.0, 1.0, 6)
    k, j, i = np.meshgrid(*(np.arange(m) for m in spec.shape), indexing="ij")
    nh2 = nH * (1.0 + 0.3 * np.sin(0.5 * i + 0.3 * j - 0.2 * k))
    return spec, nH, nh2


def _grid(spec, nH, nh2, precision):
    g = binding.Grid(spec, precision=precision, time_centred_density=nh2 is not None)
    g.load(nH, 1.0, T0=50.0)
    if nh2 is not None:
        g.nH_half.copy_(g.nH.new_tensor(nh2))
    return g


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_time_centred_density_parity(oracle_lib, precision):
    spec, nH, nh2 = _case(precision)
    g = _grid(spec, nH, nh2, precision)
    _, pb, st = pair(spec, nH, T0=50.0, precision=precision)
    nh2_stored = stored(nh2, precision)
    for _ in range(8):
        g.step_o2(spec.t_end)
        pb.step(st, spec.t_end, nH_half=nh2_stored)
    errx = rel_x(to_np(g.x), st["x"])
    Tg = pb.temperature(st["nH"], to_np(g.x), to_np(g.E))
    Tw = pb.temperature(st["nH"], st["x"], st["E"])
    if precision == "fp64":
        assert np.max(errx) < 1e-9 and np.max(rel(Tg, Tw)) < 1e-9
    else:
        float_bar(to_np(g.x), st["x"], 1e-4, precision + " time-centred density x")
        float_bar(Tg, Tw, 1e-4, precision + " time-centred density T")
    g.close()


def test_time_centred_density_equal_to_nH_is_the_plain_step():
    spec, nH, _ = _case("fp64")
    a = _grid(spec, nH, None, "fp64")
    b = _grid(spec, nH, np.asarray(nH), "fp64")
    for _ in range(5):
        a.step_o2(spec.t_end)
        b.step_o2(spec.t_end)
    assert np.array_equal(to_np(a.x), to_np(b.x))
    assert np.array_equal(to_np(a.tau), to_np(b.tau))
    a.close()
    b.close()


def test_time_centred_density_in_a_batch_bitwise():
    spec, nH, nh2 = _case("mixed")
    other = synth.cfg1(n=(16, 16, 16)).with_(precision="mixed")
    alone = []
    for s, d, h in ((spec, nH, nh2), (other, np.full(other.shape, 1.0), None)):
        g = _grid(s, d, h, "mixed")
        for _ in range(5):
            g.step_o2(s.t_end)
        alone.append(to_np(g.x))
        g.close()
    b = binding.Batch([spec, other], precision="mixed", time_centred_density=[True, False])
    b.load([nH, np.full(other.shape, 1.0)], T0s=[50.0, other.T0], t_end=[spec.t_end, other.t_end])
    b.grids[0].nH_half.copy_(b.grids[0].nH.new_tensor(nh2))
    for _ in range(5):
        b.step_o2()
    assert np.array_equal(to_np(b.grids[0].x), alone[0])
    assert np.array_equal(to_np(b.grids[1].x), alone[1])
    b.close()
