"""Algorithm 1 (Sect. 2.1, the implicit scheme with time-averaged attenuation)
on the GPU: one pass in raytrace order per step, against the oracle's pass."""
import math

import numpy as np
import pytest

from paper_1201_5651_amd import binding, synth
from gpu_util import float_bar, pair, rel, rel_x, to_np

pytestmark = pytest.mark.gpu

INF = math.inf
DT02_IMPLICIT = (0.1, INF, INF, INF)   # Table 1, dt02, implicit column


def _case(precision, n=16):
    spec = synth.cfg2(n=n).with_(precision=precision, K=DT02_IMPLICIT)
    nH = synth.lognormal_density(spec.shape, 10.0, 1.0, 8)
    return spec, nH


@pytest.mark.parametrize("n,src", [(16, None), ((20, 12, 14), (3, 9, 7))])
def test_a1_step_parity_fp64(oracle_lib, n, src):
    """Steps of A1 from the neutral start: x, T and the columns of the new
    state within 1e-9 of the oracle; the pass's time-averaged entering columns
    (tau_half) and optical depths per cell length (x_half) match the oracle's
    pass run on the same state with the same dt."""
    spec, _ = _case("fp64", 16)
    if isinstance(n, tuple):
        spec = spec.with_(n=n, src=src)
    nH = synth.lognormal_density(spec.shape, 10.0, 1.0, 8)
    g, pb, st = pair(spec, nH, T0=50.0)
    for k in range(4):
        before = {kk: (v.copy() if isinstance(v, np.ndarray) else v) for kk, v in st.items()}
        g.step_a1(spec.t_end)
        pb.step(st, spec.t_end, algo=1)
        _, _, dt = g.state()
        _, _, tavg, kbar = pb.a1_pass(before["nH"], before["x"], before["E"], dt)
        assert np.max(rel_x(to_np(g.x), st["x"])) < 1e-9, k
        Tg = pb.temperature(st["nH"], to_np(g.x), to_np(g.E))
        Tw = pb.temperature(st["nH"], st["x"], st["E"])
        assert np.max(rel(Tg, Tw)) < 1e-9
        m = st["tau"] > 0
        assert np.max(rel(to_np(g.tau)[m], st["tau"][m])) < 1e-9
        m = tavg > 1e-12
        assert np.max(rel(to_np(g.tau_half)[m], tavg[m])) < 1e-9
        kg = to_np(g.x_half) / (6.3e-18 * spec.dx)
        mk = kbar > 1e-12 * nH
        assert np.max(rel(kg[mk], kbar[mk])) < 1e-9
    g.close()


def test_a1_step_parity_mixed(oracle_lib):
    spec, nH = _case("mixed")
    g, pb, st = pair(spec, nH, T0=50.0, precision="mixed")
    for _ in range(4):
        g.step_a1(spec.t_end)
        pb.step(st, spec.t_end, algo=1)
    Tg = pb.temperature(st["nH"], to_np(g.x), to_np(g.E))
    Tw = pb.temperature(st["nH"], st["x"], st["E"])
    float_bar(to_np(g.x), st["x"], 1e-4, "mixed algorithm-1 x after 4 steps")
    float_bar(Tg, Tw, 1e-4, "mixed algorithm-1 T after 4 steps")
    g.close()


def test_a1_step_parity_mixed_front(oracle_lib):
    """PI_MIXED_FRONT: the pass integrates every ionisation-front cell (starting
    x in [1e-3, 0.5]) in double, out of line from the float integration: the
    double re-solve counter is positive once a front has formed, and x and T
    after 4 steps are within 1e-4 of the oracle on every cell."""
    spec, nH = _case("mixed_front")
    g, pb, st = pair(spec, nH, T0=50.0, precision="mixed_front")
    g.work_counters(reset=True)
    for _ in range(4):
        g.step_a1(spec.t_end)
        pb.step(st, spec.t_end, algo=1)
    assert g.work_counters()["resolved_fp64"] > 0
    Tg = pb.temperature(st["nH"], to_np(g.x), to_np(g.E))
    Tw = pb.temperature(st["nH"], st["x"], st["E"])
    float_bar(to_np(g.x), st["x"], 1e-4, "front-in-double algorithm-1 x after 4 steps")
    float_bar(Tg, Tw, 1e-4, "front-in-double algorithm-1 T after 4 steps")
    g.close()


def test_a1_stromgren_on_gpu(oracle_lib):
    """Config 1 with A1-dt02: 0.1 t_rec in one step, the front within 2% of
    R_S (1 - exp(-t/t_rec))^(1/3) up to 4 t_rec, and the oracle's state."""
    spec = synth.cfg1().with_(K=DT02_IMPLICIT)
    g, pb, st = pair(spec, np.full(spec.shape, 1.0))
    RS = synth.stromgren_radius(spec.Q, 1.0)
    g.step_a1(0.1 * spec.t_rec)
    assert g.state()[1] == 1
    pb.run(st, 0.1 * spec.t_rec, algo=1)
    for c in (0.3, 1.0, 4.0):
        while g.state()[0] < c * spec.t_rec:
            g.step_a1(c * spec.t_rec)
        pb.run(st, c * spec.t_rec, algo=1)
        d = g.diagnostics()
        Ra = RS * (1 - math.exp(-d["t"] / spec.t_rec)) ** (1 / 3)
        assert abs(d["r_ion"] / Ra - 1) < 0.02, c
        assert np.max(rel_x(to_np(g.x), st["x"])) < 1e-9
    g.close()


def test_a1_batch_matches_grids_alone():
    specs = [_case("mixed")[0], synth.cfg1(n=(12, 12, 12)).with_(precision="mixed", K=DT02_IMPLICIT)]
    nHs = [_case("mixed")[1], np.full(specs[1].shape, 1.0)]
    alone = []
    for s, nH in zip(specs, nHs):
        g = binding.Grid(s, precision="mixed")
        g.load(nH, 1.0, T0=s.T0)
        for _ in range(3):
            g.step_a1(s.t_end)
        alone.append((g.state()[0], to_np(g.x)))
        g.close()
    b = binding.Batch(specs, precision="mixed")
    b.load(nHs, T0s=[s.T0 for s in specs], t_end=[s.t_end for s in specs])
    for _ in range(3):
        b.step_a1()
    t, _, _ = b.state()
    for i, (ta, xa) in enumerate(alone):
        assert t[i] == ta
        assert np.array_equal(to_np(b.grids[i].x), xa)
    b.close()


def test_a1_rejects_plane_parallel_sources():
    spec = synth.plane(n=(16, 4, 4))
    g = binding.Grid(spec)
    g.load(synth.density(spec), 1.0)
    with pytest.raises(binding.PiError) as e:
        g.step_a1(spec.t_end)
    assert e.value.status == binding.PI_EINVAL
    g.close()
