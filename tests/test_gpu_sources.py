"""Several point sources on one grid: every source's columns, A3 steps and
diagnostics on the GPU against the oracle (each source traced on its own, the
rates of the sources added in every cell), such grids batched and served
beside one-source grids (bit for bit as alone), and the limit of the form
(algorithm 1 follows one source)."""
import numpy as np
import pytest

import oracle
from paper_1201_5651_amd import binding, synth
from gpu_util import float_bar, pair, rel, rel_x, stored, to_np

pytestmark = pytest.mark.gpu

# a grid spanning several tiles of every edge with ragged tails, sources in
# the interior, on an edge and at a corner of the box
SHAPE = (20, 18, 17)
SOURCES = [((15, 3, 12), 0.5), ((10, 18, 0), 0.25), ((0, 0, 17), 0.8)]


def _spec(nsrc, precision="fp64", shape=SHAPE):
    base = synth.cfg2(n=shape[0]).with_(n=shape, src=(5, 9, 4), precision=precision)
    more = tuple((v, f * base.Q) for v, f in SOURCES[: nsrc - 1])
    return base.with_(more_sources=more)


def _nH(spec, seed=3):
    return synth.lognormal_density(spec.shape, 10.0, 1.0, seed)


@pytest.mark.parametrize("nsrc", [2, 4])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_columns_of_every_source(oracle_lib, nsrc, precision):
    """Each source's columns are its own raytrace of the same state (FP64
    within 1e-12 of the oracle, float 1e-5), and every tile edge gives the
    same columns bit for bit."""
    spec = _spec(nsrc, precision)
    rng = np.random.default_rng(11)
    x = rng.uniform(0.0, 1.0, spec.shape)
    g, pb, _ = pair(spec, _nH(spec), x0=x, precision=precision)
    assert tuple(g.tau.shape) == (nsrc,) + spec.shape
    want = pb.raytrace(stored(_nH(spec), precision), stored(x, precision))
    got = to_np(g.tau)
    assert np.array_equal(got == 0, want == 0)
    m = want > 0
    assert np.max(rel(got[m], want[m])) < (1e-12 if precision == "fp64" else 1e-5)
    cols = {}
    P = binding.PI_TILE_PERSISTENT
    for edge in (4, 8, 16, P):
        g.raytrace_tile = edge
        g.tau.zero_()
        g.raytrace()
        cols[edge] = to_np(g.tau)
    assert np.array_equal(cols[4], cols[8]) and np.array_equal(cols[4], cols[16])
    assert np.array_equal(cols[4], cols[P])
    g.state()   # no persistent wait went over its limit
    g.close()


@pytest.mark.parametrize("nsrc", [2, 3, 4])
def test_a3_steps_parity_fp64(oracle_lib, nsrc):
    """A3 steps of a clumpy medium lit by several sources (table spectrum,
    evolving temperature): state, columns of every source, clock and FP64
    diagnostics within 1e-9 of the oracle."""
    spec = _spec(nsrc)
    g, pb, st = pair(spec, _nH(spec), T0=50.0)
    for _ in range(8):
        g.step_o2(spec.t_end)
        pb.step(st, spec.t_end)
    assert g.state()[0] == pytest.approx(st["t"], rel=1e-12)
    assert np.max(rel_x(to_np(g.x), st["x"])) < 1e-9
    Tg = pb.temperature(st["nH"], to_np(g.x), to_np(g.E))
    Tw = pb.temperature(st["nH"], st["x"], st["E"])
    assert np.max(rel(Tg, Tw)) < 1e-9
    m = st["tau"] > 0
    assert np.max(rel(to_np(g.tau)[m], st["tau"][m])) < 1e-9
    dg, dw = g.diagnostics(), pb.diagnostics(st)
    for k in ("n_ion", "v_ion", "r_ion", "photo_rate", "recomb_rate"):
        assert dg[k] == pytest.approx(dw[k], rel=1e-9), k
    # octants of every source: 8 around each interior vertex, 2 around the
    # vertex on an edge of the box, 1 around the corner vertex
    assert dg["octants"] == [8, 16, 18, 19][nsrc - 1]
    assert (1 - st["x"]).sum() > 10.0
    g.close()


@pytest.mark.parametrize("precision", ["fp32", "mixed"])
def test_a3_steps_parity_float(oracle_lib, precision):
    spec = _spec(4, precision)
    g, pb, st = pair(spec, _nH(spec), T0=50.0, precision=precision)
    for _ in range(8):
        g.step_o2(spec.t_end)
        pb.step(st, spec.t_end)
    Tg = pb.temperature(st["nH"], to_np(g.x), to_np(g.E))
    Tw = pb.temperature(st["nH"], st["x"], st["E"])
    float_bar(to_np(g.x), st["x"], 1e-4, precision + " four sources x after 8 steps")
    float_bar(Tg, Tw, 1e-4, precision + " four sources T after 8 steps")
    g.close()


def test_mirrored_sources_on_gpu_give_a_mirrored_state():
    """Two equal sources at mirror-image vertices of a mirror-symmetric
    medium: the GPU state stays symmetric to rounding (a beam weighted from
    the wrong vertex would break it)."""
    n = 16
    base = synth.cfg2(n=n)
    spec = base.with_(src=(3, 5, 6), Q=0.5 * base.Q, more_sources=(((n - 3, 5, 6), 0.5 * base.Q),))
    nH = _nH(spec, 5)
    nH = 0.5 * (nH + nH[:, :, ::-1])
    g = binding.Grid(spec)
    g.load(nH, 1.0, T0=50.0)
    for _ in range(6):
        g.step_o2(spec.t_end)
    x = to_np(g.x)
    assert np.max(rel_x(x, x[:, :, ::-1])) < 1e-12
    assert (1 - x).sum() > 1.0
    g.close()


def test_several_sources_limits():
    """Algorithm 1 follows one source's rays: a grid (or a batch holding a
    grid) with several sources is rejected with PI_EINVAL there and stays
    usable; a vertex outside the grid is rejected at creation."""
    spec = _spec(2, shape=(8, 8, 8)).with_(src=(4, 4, 4), more_sources=(((1, 2, 3), 1e47),))
    g = binding.Grid(spec)
    g.load(_nH(spec), 1.0, T0=50.0)
    with pytest.raises(binding.PiError) as e:
        g.step_a1(spec.t_end)
    assert e.value.status == binding.PI_EINVAL
    g.step_o2(spec.t_end)   # the grid is still usable
    g.close()
    b = binding.Batch([spec, spec.with_(more_sources=())])
    b.load([_nH(spec)] * 2, T0s=[50.0] * 2, t_end=[spec.t_end] * 2)
    with pytest.raises(binding.PiError) as e:
        b.step_a1()
    assert e.value.status == binding.PI_EINVAL
    b.close()
    with pytest.raises(binding.PiError) as e:
        binding.Grid(spec.with_(more_sources=(((9, 0, 0), 1e47),)))
    assert e.value.status == binding.PI_EINVAL


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_of_one_and_several_source_grids_bitwise(precision):
    """Grids with one source, with several, and a plane-parallel grid advanced
    as one batch (both kernel variants launched, each skipping the other's
    grids; one re-solve list) give bit for bit what each gives alone."""
    specs = [_spec(3, precision),
             synth.cfg2(n=14).with_(precision=precision),
             _spec(1, precision, shape=(11, 16, 9)).with_(
                 src=(3, 8, 4), more_sources=(((9, 2, 7), 4e47), ((0, 16, 0), 2e48),
                                              ((11, 5, 3), 1e47))),
             synth.plane(n=(40, 6, 5), density="lognormal", precision=precision)]
    nHs = [_nH(specs[0], 1), _nH(specs[1], 2), _nH(specs[2], 3), synth.density(specs[3])]
    alone = []
    for s, nH in zip(specs, nHs):
        g = binding.Grid(s, precision=precision)
        g.load(nH, 1.0, T0=s.T0)
        for _ in range(6):
            g.step_o2(s.t_end)
        alone.append((g.state(), to_np(g.x), None if g.E is None else to_np(g.E), to_np(g.tau),
                      g.diagnostics()))
        g.close()
    b = binding.Batch(specs, precision=precision)
    b.load(nHs, T0s=[s.T0 for s in specs], t_end=[s.t_end for s in specs])
    for _ in range(6):
        b.step_o2()
    t, n, _ = b.state()
    d = b.diagnostics()
    for i, (st, xa, Ea, taua, da) in enumerate(alone):
        assert (t[i], n[i]) == st[:2], i
        assert np.array_equal(to_np(b.grids[i].x), xa), i
        if Ea is not None:
            assert np.array_equal(to_np(b.grids[i].E), Ea), i
        assert np.array_equal(to_np(b.grids[i].tau), taua), i
        assert d[i]["octants"] == da["octants"], i
    assert [d[i]["octants"] for i in range(4)] == [18, 8, 8 + 8 + 1 + 4, 0]
    b.close()


def test_served_several_source_requests_match_alone():
    """Served requests with several sources (their columns take one array per
    source in the arena) next to one-source requests: each result is the grid
    advanced alone, bit for bit."""
    import time
    reqs = [(_spec(3, "mixed"), 1), (synth.cfg2(n=12).with_(precision="mixed"), 2),
            (_spec(1, "mixed", shape=(9, 10, 12)).with_(src=(4, 5, 6),
                                                         more_sources=(((1, 9, 2), 5e47),)), 3)]
    srv = binding.Server(precision="mixed", hbm_budget=64 << 20, max_active=4, steps_per_tick=2)
    tickets = []
    for s, seed in reqs:
        tickets.append(srv.submit(s, _nH(s, seed), T0=s.T0, t_end=2e-3 * s.t_rec))
    done, t0 = {}, time.time()
    while len(done) < len(tickets):
        assert time.time() - t0 < 120.0, "served requests did not finish"
        for tk in tickets:
            if tk not in done:
                st, info, x, T = srv.poll(tk)
                if st != binding.PI_PENDING:
                    done[tk] = (st, info, x)
        time.sleep(0.005)
    srv.close()
    for tk, (s, seed) in zip(tickets, reqs):
        st, info, x = done[tk]
        assert st == binding.PI_OK, info
        g = binding.Grid(s, precision="mixed")
        g.load(_nH(s, seed), 1.0, T0=s.T0)
        g.run(2e-3 * s.t_rec, check_every=8)
        t, n, _ = g.state()
        assert (info["t"], info["nsteps"]) == (t, n)
        assert np.array_equal(x, to_np(g.x))
        g.close()


def test_degenerate_sources_fp64(oracle_lib):
    """Degenerate cases: a further source of Q = 0 leaves the one-source
    result (the several-source kernels add exact zeros), and two sources of
    Q/2 at one vertex give the single source of Q to rounding."""
    base = synth.cfg2(n=12).with_(n=(12, 10, 9), src=(5, 4, 4))
    nH = _nH(base, 8)
    runs = {}
    for key, spec in (("one", base),
                      ("zero", base.with_(more_sources=(((2, 9, 1), 0.0),))),
                      ("split", base.with_(Q=0.5 * base.Q, more_sources=((base.src, 0.5 * base.Q),)))):
        g = binding.Grid(spec)
        g.load(nH, 1.0, T0=50.0)
        for _ in range(6):
            g.step_o2(spec.t_end)
        runs[key] = (to_np(g.x), to_np(g.E), g.state()[0], g.diagnostics())
        g.close()
    x1, E1, t1, d1 = runs["one"]
    for key in ("zero", "split"):
        x, E, t, d = runs[key]
        assert t == pytest.approx(t1, rel=1e-12), key
        assert np.max(rel_x(x, x1)) < 1e-10, key
        assert np.max(rel(E, E1)) < 1e-10, key
        assert d["photo_rate"] == pytest.approx(d1["photo_rate"], rel=1e-10), key
    assert runs["zero"][3]["octants"] == 8 + 8
    assert (1 - x1).sum() > 1.0


def test_four_sources_48cubed_mixed(oracle_lib):
    """A 48^3 clumpy grid (three 16^3 tiles a side) lit by four sources, one
    of them on an edge of the box, in mixed precision: six A3 steps against
    the oracle at the float bar, every source's columns included."""
    base = synth.cfg2(n=48).with_(src=(20, 30, 17), precision="mixed")
    spec = base.with_(more_sources=(((40, 8, 33), 0.7 * base.Q), ((5, 44, 44), 0.3 * base.Q),
                                    ((48, 24, 0), 1.5 * base.Q)))
    nH = synth.lognormal_density(spec.shape, 10.0, 1.0, 12)
    g, pb, st = pair(spec, nH, T0=50.0, precision="mixed")
    for _ in range(6):
        g.step_o2(spec.t_end)
        pb.step(st, spec.t_end)
    assert g.state()[0] == pytest.approx(st["t"], rel=1e-4)
    Tg = pb.temperature(st["nH"], to_np(g.x), to_np(g.E))
    Tw = pb.temperature(st["nH"], st["x"], st["E"])
    float_bar(to_np(g.x), st["x"], 1e-4, "mixed 48^3 four sources x")
    float_bar(Tg, Tw, 1e-4, "mixed 48^3 four sources T")
    # columns: relative where they are not tiny, absolute (in optical depth)
    # below 1e-3, where float rounding of the sum dominates
    tg, tw = to_np(g.tau), st["tau"]
    m = tw > 1e-3
    float_bar(tg[m], tw[m], 1e-4, "mixed 48^3 four sources columns")
    assert np.max(np.abs(tg[~m] - tw[~m])) < 1e-7
    assert g.diagnostics()["octants"] == 8 + 8 + 8 + 2
    assert (1 - st["x"]).sum() > 20.0
    g.close()
