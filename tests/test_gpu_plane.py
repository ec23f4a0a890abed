"""Plane-parallel source (Sect. 3.1's slab test on a 3D grid) on the GPU:
row-scan raytrace, A3 steps and diagnostics against the oracle, photon
conservation, and plane-parallel grids batched with point-source grids."""
import numpy as np
import pytest

from paper_1201_5651_amd import binding, synth
from gpu_util import float_bar, pair, rel, rel_x, stored, to_np

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n", [(40, 12, 10), (150, 6, 5), (1, 3, 2), (64, 1, 1)])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_plane_raytrace_parity(oracle_lib, n, precision):
    """Columns from the lit face on a clumpy density and random x: FP64 within
    1e-12 of the oracle's row sums (summation order differs), float within
    1e-5; the first cell of every row sees no column."""
    spec = synth.plane(n=n, density="lognormal")
    rng = np.random.default_rng(7)
    nH = synth.density(spec)
    x = rng.uniform(0.0, 1.0, spec.shape)
    g, pb, _ = pair(spec, nH, x0=x, precision=precision)
    g.raytrace()
    got = to_np(g.tau)
    # the state as the grid stores it (float rounding in FP32)
    want = pb.raytrace(stored(nH, precision), stored(x, precision))
    assert np.all(got[..., 0] == 0)
    m = want > 0
    if m.any():
        assert np.max(rel(got[m], want[m])) < (1e-12 if precision == "fp64" else 1e-5)
    assert np.all(got[~m] == 0)
    g.close()


def test_plane_steps_parity_fp64(oracle_lib):
    spec = synth.plane(n=(80, 8, 6), density="lognormal")
    g, pb, st = pair(spec, synth.density(spec))
    for _ in range(10):
        g.step_o2(spec.t_end)
        pb.step(st, spec.t_end)
    assert g.state()[0] == pytest.approx(st["t"], rel=1e-14)
    assert np.max(rel_x(to_np(g.x), st["x"])) < 1e-9
    m = st["tau"] > 0
    assert np.max(rel(to_np(g.tau)[m], st["tau"][m])) < 1e-9
    dg, dw = g.diagnostics(), pb.diagnostics(st)
    assert dg["r_ion"] == pytest.approx(dw["r_ion"], rel=1e-9)
    assert dg["n_ion"] == pytest.approx(dw["n_ion"], rel=1e-9)
    g.close()


def test_plane_steps_parity_mixed(oracle_lib):
    spec = synth.plane(n=(80, 8, 6), density="lognormal", precision="mixed")
    g, pb, st = pair(spec, synth.density(spec), precision="mixed")
    for _ in range(10):
        g.step_o2(spec.t_end)
        pb.step(st, spec.t_end)
    float_bar(to_np(g.x), st["x"], 1e-4, "mixed plane-parallel x after 10 steps")
    g.close()


def test_plane_photon_count_on_gpu():
    """No recombinations: the ions per unit area follow F t (Sect. 3.1), to
    the 2% of A3-dt02 at each output time; every row of a uniform medium is
    the same."""
    spec = synth.plane(n=(100, 4, 4))
    g = binding.Grid(spec)
    g.load(synth.density(spec), 1.0)
    area = 4 * 4 * spec.dx ** 2
    for f in (0.1, 0.4, 0.8):
        g.run(f * spec.t_rec, check_every=8)
        d = g.diagnostics()
        assert d["n_ion"] / area / (spec.Q * d["t"]) == pytest.approx(1.0, abs=0.02)
        assert d["octants"] == 0
        x = to_np(g.x).reshape(-1, 100)
        assert np.all(x == x[0])
    g.close()


def test_plane_and_point_grids_in_one_batch_bitwise():
    """A plane-parallel grid and a point-source grid advanced as one batch
    give bit for bit what each gives alone."""
    specs = [synth.plane(n=(48, 10, 6), density="lognormal", precision="mixed"),
             synth.cfg2(n=20).with_(precision="mixed")]
    nHs = [synth.density(specs[0]), synth.lognormal_density(specs[1].shape, 10.0, 1.0, 4)]
    alone = []
    for s, nH in zip(specs, nHs):
        g = binding.Grid(s, precision="mixed")
        g.load(nH, 1.0, T0=s.T0)
        for _ in range(6):
            g.step_o2(s.t_end)
        alone.append((g.state()[0], to_np(g.x), to_np(g.tau)))
        g.close()
    b = binding.Batch(specs, precision="mixed")
    b.load(nHs, T0s=[s.T0 for s in specs], t_end=[s.t_end for s in specs])
    for _ in range(6):
        b.step_o2()
    t, _, _ = b.state()
    for i, (ta, xa, taua) in enumerate(alone):
        assert t[i] == ta
        assert np.array_equal(to_np(b.grids[i].x), xa)
        assert np.array_equal(to_np(b.grids[i].tau), taua)
    b.close()
