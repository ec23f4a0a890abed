"""GPU <-> oracle parity of every operation of the hot path, through the C ABI.

FP64 bar: neutral fraction and temperature within 1e-9 relative (x with the
1e-12 floor of the paper's absolute tolerance on 1 - y), columns within 1e-12.
FP32 bar: 1e-4 relative.  All inputs are seeded and synthetic.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1201_5651_amd import binding, synth
from gpu_util import backward_ok, float_bar, pair, rel, rel_x, stored, to_np

pytestmark = pytest.mark.gpu

KB = 1.380649e-16

SHAPES = [
    ((8, 8, 8), (0, 0, 0)),
    ((16, 16, 16), (8, 8, 8)),
    ((17, 13, 11), (5, 9, 4)),
    ((24, 9, 20), (24, 0, 7)),
    ((12, 30, 7), (6, 15, 7)),
    ((1, 1, 1), (0, 1, 0)),
]


def _spec(n, src, **kw):
    base = dict(name="t", n=n, src=src, dx=3e17, Q=1e48, nH_mean=1.0)
    base.update(kw)
    return synth.GridSpec(**base)


@pytest.mark.parametrize("shape,src", SHAPES)
@pytest.mark.parametrize("weights", ["mellema", "geometric"])
def test_raytrace_parity_fp64(oracle_lib, shape, src, weights):
    rng = np.random.default_rng(hash((shape, src)) % 2**32)
    spec = _spec(shape, src, weights=weights)
    nH = rng.uniform(0.2, 5.0, spec.shape)
    x = rng.uniform(0.0, 1.0, spec.shape)
    x[rng.random(spec.shape) < 0.2] = 0.0
    g = binding.Grid(spec)
    g.load(nH, x)
    pb = oracle.Problem.from_spec(spec)
    want = pb.raytrace(np.ascontiguousarray(nH), np.ascontiguousarray(x))
    got = to_np(g.tau)
    assert np.all((got == 0) == (want == 0))
    m = want > 0
    if m.any():
        assert np.max(rel(got[m], want[m])) < 1e-12
    g.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_raytrace_tile_edges_give_identical_columns(precision):
    """Tiling changes the order of the sweep, not the arithmetic of any cell:
    4^3, 8^3 and 16^3 tiles, one launch per tile diagonal, and the persistent
    single-launch sweep give bitwise equal columns, and tuning settles on one
    of them."""
    spec = _spec((19, 22, 17), (7, 15, 9))
    rng = np.random.default_rng(21)
    g = binding.Grid(spec, precision=precision)
    assert g.raytrace_tile == 0
    g.load(rng.uniform(0.2, 5.0, spec.shape), rng.uniform(0.0, 1.0, spec.shape))
    P = binding.PI_TILE_PERSISTENT
    assert g.raytrace_tile in (4, 8, 16, P)
    cols = {}
    for edge in (4, 8, 16, P, P):
        g.raytrace_tile = edge
        g.tau.zero_()
        g.raytrace()
        cols[edge] = to_np(g.tau)
        assert g.state()[1] == 0   # (a synchronising read: no wait went over its limit)
    assert np.array_equal(cols[4], cols[8])
    assert np.array_equal(cols[4], cols[16])
    assert np.array_equal(cols[4], cols[P])
    with pytest.raises(binding.PiError):
        g.raytrace_tile = 5
    g.close()


@pytest.mark.parametrize("shape,src", SHAPES[:4])
def test_raytrace_parity_fp32(oracle_lib, shape, src):
    rng = np.random.default_rng(7)
    spec = _spec(shape, src)
    nH = rng.uniform(0.2, 5.0, spec.shape)
    x = rng.uniform(0.0, 1.0, spec.shape)
    g = binding.Grid(spec, precision="fp32")
    g.load(nH, x)
    pb = oracle.Problem.from_spec(spec)
    want = pb.raytrace(stored(nH, "fp64"), stored(x, "fp32"))
    got = to_np(g.tau)
    # every cell: the exact zero pattern (cells on the source's planes), and
    # the largest relative error over all the others, thin columns included
    zero = want == 0
    assert np.array_equal(got == 0, zero)
    float_bar(got[~zero], want[~zero], 1e-5, "fp32 raytrace %s" % (shape,), floor=1e-300)


def _chem_case(seed, thermal, spectrum, precision):
    rng = np.random.default_rng(seed)
    spec = _spec((20, 18, 16), (9, 9, 8), nH_mean=10.0, dx=4e17,
                 thermal=thermal, spectrum=spectrum, recomb="power" if thermal == "evolve" else "const",
                 collisional=thermal == "evolve", T0=50.0)
    cs = synth.random_cell_states(spec.ncells, seed=seed, thermal=thermal == "evolve")
    nH = cs["nH"].reshape(spec.shape)
    x = cs["x"].reshape(spec.shape)
    T = cs["T"].reshape(spec.shape)
    g = binding.Grid(spec, precision=precision)
    g.load(nH, x)
    pb = oracle.Problem.from_spec(spec)
    # the inputs as the grid holds them (rounded to float by numpy for the
    # float grids), given to both sides
    nHo, xo = stored(nH, precision), stored(x, precision)
    E = None
    if thermal == "evolve":
        E = stored(1.5 * KB * nHo * (2.0 - xo) * T, precision)
        g.E.copy_(__import__("torch").as_tensor(E, dtype=g.dtype))
    tau = stored(cs["tau"].reshape(spec.shape), precision)
    g.tau.copy_(__import__("torch").as_tensor(tau, dtype=g.dtype))
    return spec, g, pb, nHo, xo, E, tau


def _sensitivity(pb, nH, x, E, tau, h, xw):
    """Relative change of the oracle's result under 1e-12 relative changes of
    the entering columns and of the density: the conditioning of each cell's
    micro-integration."""
    xp, _ = pb.chem(nH, x, E, np.ascontiguousarray(tau * (1 + 1e-12)), h)
    xq, _ = pb.chem(np.ascontiguousarray(nH * (1 + 1e-12)), x, E, tau, h)
    return np.maximum(rel_x(xp, xw), rel_x(xq, xw))


@pytest.mark.parametrize("thermal,spectrum", [("fixed", "mono"), ("evolve", "mono"),
                                              ("evolve", "table"), ("fixed", "table")])
@pytest.mark.parametrize("h", [1e9, 3e10])
def test_chem_parity_fp64(oracle_lib, thermal, spectrum, h):
    """One micro-physics update of random physical cell states over a common
    interval.  Cells whose result the oracle itself moves by more than 1e-10
    under a 1e-12 change of the input columns are ill-conditioned (a
    temperature collapsing onto the floor, competing thermal equilibria over an
    interval far above the cell's own time-scales); there the GPU result must
    be the oracle's result for an input within a few rounding units of the
    given one, elsewhere the bar is 1e-9."""
    spec, g, pb, nH, x, E, tau = _chem_case(11, thermal, spectrum, "fp64")
    g.chem_step(h, binding.PI_BUF_N, binding.PI_BUF_N, binding.PI_BUF_HALF)
    xw, Ew = pb.chem(nH, x, E, tau, h)
    xg = to_np(g.x_half)
    sens = _sensitivity(pb, nH, x, E, tau, h, xw)
    well = sens <= 1e-10
    assert well.mean() > 0.95
    err = rel_x(xg, xw)
    assert np.max(err[well]) < 1e-9, np.max(err[well])
    assert np.all((xg >= 0) & (xg <= 1))
    Tg = None
    if E is not None:
        Tg = pb.temperature(nH, xg, to_np(g.E_half))
        Tw = pb.temperature(nH, xw, Ew)
        assert np.max(rel(Tg, Tw)[well]) < 1e-9
        assert np.all(np.isfinite(Tg)) and np.all(Tg >= 10.0 * (1 - 1e-12))
    # ill-conditioned cells: the oracle's own result at an input within a few
    # rounding units of the given one reproduces the GPU's
    ill = np.flatnonzero(~well.reshape(-1))
    bad = backward_ok(pb, spec, nH, x, E, tau, h, ill, xg, Tg, 1e-9,
                      (1e-13, -1e-13, 1e-12, -1e-12, 1e-11, -1e-11))
    print("fp64 chem: %d ill-conditioned cells, %d not reproduced" % (ill.size, len(bad)))
    assert not bad, bad[:10]


@pytest.mark.parametrize("thermal,spectrum", [("fixed", "mono"), ("evolve", "table")])
def test_chem_parity_fp32(oracle_lib, thermal, spectrum):
    spec, g, pb, nH, x, E, tau = _chem_case(12, thermal, spectrum, "fp32")
    h = 1e10
    g.chem_step(h, binding.PI_BUF_N, binding.PI_BUF_N, binding.PI_BUF_HALF)
    xw, Ew = pb.chem(nH, x, E, tau, h)
    # conditioning at the float rounding level: a cell is ill-conditioned when
    # a 1e-7 change of its inputs moves the oracle's result by more than 1e-5
    xp, _ = pb.chem(nH, x, E, np.ascontiguousarray(tau * (1 + 1e-7)), h)
    xq, _ = pb.chem(np.ascontiguousarray(nH * (1 + 1e-7)), x, E, tau, h)
    well = np.maximum(rel_x(xp, xw), rel_x(xq, xw)) <= 1e-5
    xg = to_np(g.x_half)
    float_bar(xg[well], xw[well], 1e-4, "fp32 chem x (well-conditioned)")
    Tg = None
    if E is not None:
        Tg = pb.temperature(nH, xg, to_np(g.E_half))
        Tw = pb.temperature(nH, xw, Ew)
        float_bar(Tg[well], Tw[well], 1e-4, "fp32 chem T (well-conditioned)")
    ill = np.flatnonzero(~well.reshape(-1))
    bad = backward_ok(pb, spec, nH, x, E, tau, h, ill, xg, Tg, 1e-4,
                      (1e-7, -1e-7, 3e-7, -3e-7, 1e-6, -1e-6))
    print("fp32 chem: %d ill-conditioned cells, %d not reproduced" % (ill.size, len(bad)))
    assert not bad, bad[:10]


@pytest.mark.parametrize("precision", ["mixed", "mixed_front"])
@pytest.mark.parametrize("thermal,spectrum", [("evolve", "mono"), ("evolve", "table")])
@pytest.mark.parametrize("h", [1e10, 3e10])
def test_chem_parity_mixed(oracle_lib, thermal, spectrum, h, precision):
    """PI_MIXED: float bulk, and a double re-solve of every cell whose substep
    control decided within 1e-3 of a threshold.  The largest float errors come
    from such decisions going the other way (a different, equally valid choice
    of substeps), not from conditioning; with the re-solve every
    well-conditioned cell is within 1e-4 of the oracle on the same inputs."""
    spec, g, pb, nH, x, E, tau = _chem_case(11, thermal, spectrum, precision)
    g.work_counters(reset=True)
    g.chem_step(h, binding.PI_BUF_N, binding.PI_BUF_N, binding.PI_BUF_HALF)
    w = g.work_counters(reset=True)
    xw, Ew = pb.chem(nH, x, E, tau, h)
    well = _sensitivity(pb, nH, x, E, tau, h, xw) <= 1e-10
    err = rel_x(to_np(g.x_half), xw)[well]
    Tg = pb.temperature(nH, to_np(g.x_half), to_np(g.E_half))
    Tw = pb.temperature(nH, xw, Ew)
    front = int(((x >= 1e-3) & (x <= 0.5)).sum()) if precision == "mixed_front" else 0
    print("%s: %d of %d cells re-solved in double (%d front cells); x err max %.3g, T err max %.3g"
          % (precision, w["resolved_fp64"], spec.ncells, front, err.max(), rel(Tg, Tw)[well].max()))
    # the cells whose float integration took a precision-sensitive decision,
    # and with mixed_front every front cell, are integrated in double
    assert front <= w["resolved_fp64"] < front + spec.ncells // 10
    assert err.max() < 1e-4
    assert rel(Tg, Tw)[well].max() < 1e-4
    ill = np.flatnonzero(~well.reshape(-1))
    bad = backward_ok(pb, spec, nH, x, E, tau, h, ill, to_np(g.x_half), Tg, 1e-4,
                      (1e-7, -1e-7, 3e-7, -3e-7, 1e-6, -1e-6))
    print("mixed chem: %d ill-conditioned cells, %d not reproduced" % (ill.size, len(bad)))
    assert not bad, bad[:10]
    # the input state is untouched (the re-solve reads it after the bulk pass)
    assert np.array_equal(to_np(g.x), x)


@pytest.mark.parametrize("thermal,spectrum", [("fixed", "mono"), ("evolve", "table")])
def test_timestep_parity(oracle_lib, thermal, spectrum):
    """eq. (4) reduced in FP64 on the device: the dt of one A2 step equals the
    oracle's minimum over cells."""
    spec, g, pb, nH, x, E, tau = _chem_case(13, thermal, spectrum, "fp64")
    want = pb.timestep(nH, x, E, tau)
    g.step_o1(1e30)
    _, n, got = g.state()
    assert n == 1
    assert got == pytest.approx(want, rel=1e-12)


def test_a3_step_parity_cfg1_first_steps(oracle_lib):
    spec = synth.cfg1()
    g, pb, st = pair(spec, np.full(spec.shape, 1.0))
    for _ in range(12):
        g.step_o2(spec.t_end)
        pb.step(st, spec.t_end)
    t, n, _ = g.state()
    assert n == 12
    assert t == pytest.approx(st["t"], rel=1e-12)
    assert np.max(rel_x(to_np(g.x), st["x"])) < 1e-9
    m = st["tau"] > 0
    assert np.max(rel(to_np(g.tau)[m], st["tau"][m])) < 1e-9


def test_a2_step_parity(oracle_lib):
    spec = synth.cfg1(n=(16, 16, 16), dx=synth.cfg1().dx * 2)
    g, pb, st = pair(spec, np.full(spec.shape, 1.0))
    for _ in range(6):
        g.step_o1(spec.t_end)
        pb.step(st, spec.t_end, algo=2)
    assert np.max(rel_x(to_np(g.x), st["x"])) < 1e-9


def test_cfg2_physics_steps_parity_fp64(oracle_lib):
    """Table spectrum, evolving temperature, collisions, all octants (24^3 slice
    of the 128^3 set-up at the same cell size)."""
    spec = synth.cfg2(n=24)
    rng = np.random.default_rng(5)
    nH = synth.lognormal_density(spec.shape, 10.0, 1.0, 3)
    g, pb, st = pair(spec, nH, T0=50.0)
    for _ in range(8):
        g.step_o2(spec.t_end)
        pb.step(st, spec.t_end)
    assert np.max(rel_x(to_np(g.x), st["x"])) < 1e-9
    Tg = pb.temperature(st["nH"], to_np(g.x), to_np(g.E))
    Tw = pb.temperature(st["nH"], st["x"], st["E"])
    assert np.max(rel(Tg, Tw)) < 1e-9


@pytest.mark.parametrize("precision", ["fp32", "mixed", "mixed_front"])
def test_cfg2_physics_steps_fp32(oracle_lib, precision):
    """Float and mixed A3 steps (the corrector updates the state in place)."""
    spec = synth.cfg2(n=24)
    nH = synth.lognormal_density(spec.shape, 10.0, 1.0, 3)
    g, pb, st = pair(spec, nH, T0=50.0, precision=precision)
    for _ in range(8):
        g.step_o2(spec.t_end)
        pb.step(st, spec.t_end)
    Tg = pb.temperature(st["nH"], to_np(g.x), to_np(g.E))
    Tw = pb.temperature(st["nH"], st["x"], st["E"])
    float_bar(to_np(g.x), st["x"], 1e-4, precision + " cfg2 24^3 x after 8 steps")
    float_bar(Tg, Tw, 1e-4, precision + " cfg2 24^3 T after 8 steps")


def test_cfg1_stromgren_on_gpu_and_parity(oracle_lib):
    """Config 1 to 4 t_rec on the GPU: the front follows
    R_S (1 - exp(-t/t_rec))^(1/3) within 2%, and at every output time the
    state matches the oracle's (run with the same output stops) to 1e-9."""
    spec = synth.cfg1()
    g, pb, st = pair(spec, np.full(spec.shape, 1.0))
    RS = synth.stromgren_radius(spec.Q, 1.0)
    for c in (0.01, 0.1, 1.0, 4.0):
        g.run(c * spec.t_rec, check_every=8)
        pb.run(st, c * spec.t_rec)
        d = g.diagnostics()
        Ra = RS * (1 - math.exp(-d["t"] / spec.t_rec)) ** (1 / 3)
        assert abs(d["r_ion"] / Ra - 1) < 0.02, (c, d["r_ion"] / Ra)
        t, n, _ = g.state()
        assert t == pytest.approx(st["t"], rel=1e-14)
        err = rel_x(to_np(g.x), st["x"])
        assert np.max(err) < 1e-9, (c, np.max(err))


def test_determinism_bitwise(oracle_lib):
    spec = synth.cfg2(n=20)
    nH = synth.lognormal_density(spec.shape, 10.0, 1.0, 9)
    outs = []
    for _ in range(2):
        g = binding.Grid(spec)
        g.load(nH, 1.0, T0=50.0)
        for _ in range(5):
            g.step_o2(spec.t_end)
        outs.append((to_np(g.x), to_np(g.E), to_np(g.tau), g.state()))
        g.close()
    for a, b in zip(outs[0][:3], outs[1][:3]):
        assert np.array_equal(a, b)
    assert outs[0][3] == outs[1][3]


def test_diagnostics_match_oracle(oracle_lib):
    spec = synth.cfg1()
    g, pb, st = pair(spec, np.full(spec.shape, 1.0))
    for _ in range(10):
        g.step_o2(spec.t_end)
        pb.step(st, spec.t_end)
    d = g.diagnostics()
    w = pb.diagnostics(st)
    for k in ("n_ion", "v_ion", "r_ion", "photo_rate", "recomb_rate"):
        assert d[k] == pytest.approx(w[k], rel=1e-9), k
    assert d["nonfinite"] == 0 and d["octants"] == 1
