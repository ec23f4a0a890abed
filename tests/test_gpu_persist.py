"""The persistent raytrace (PI_TILE_PERSISTENT: one launch, tiles claimed in
wavefront order, each waiting on its upstream tiles' done-flags) on the GPU:
its columns equal the staged sweep's bit for bit on ragged grids and sources
on faces and corners, in both precisions and on repeated calls (the flags
carry an epoch per call); a batch advanced by replayed step graphs with it
equals the same batch on staged tiles; a wait limit of zero, set from the
host, fails the waits, every workgroup still exits, the next synchronising
call reports PI_EDEVICE once, and the following raytrace is right again."""
import numpy as np
import pytest
import torch

from paper_1201_5651_amd import binding, synth
from gpu_util import to_np

pytestmark = pytest.mark.gpu

P = binding.PI_TILE_PERSISTENT

CASES = [((19, 22, 17), (7, 15, 9)), ((33, 16, 40), (0, 8, 39)), ((45, 70, 21), (44, 0, 10)),
         ((64, 64, 64), (32, 32, 32)), ((1, 1, 1), (0, 0, 0)), ((9, 1, 30), (9, 1, 0))]


def _grid(n, src, precision, seed):
    spec = synth.cfg2(n=20).with_(n=n, src=src)
    rng = np.random.default_rng(seed)
    g = binding.Grid(spec, precision=precision)
    g.raytrace_tile = 8
    g.load(rng.uniform(0.2, 5.0, spec.shape), rng.uniform(0.0, 1.0, spec.shape), T0=50.0)
    return g


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_persistent_columns_equal_staged_bitwise(precision, case):
    n, src = CASES[case]
    print("# persistent raytrace", precision, n, src, flush=True)
    g = _grid(n, src, precision, 100 + case)
    ref = to_np(g.tau)
    g.raytrace_tile = P
    assert g.raytrace_tile == P
    for _ in range(3):
        g.tau.zero_()
        g.raytrace()
        assert np.array_equal(to_np(g.tau), ref)
    g.state()   # no wait ran out
    g.close()


def test_wait_limit_zero_reports_edevice_once_then_recovers():
    g = _grid((64, 64, 64), (32, 32, 32), "fp32", 7)
    ref = to_np(g.tau)
    g.raytrace_tile = P
    g.set_raytrace_wait_limit(0.0)
    g.tau.zero_()
    g.raytrace()
    torch.cuda.synchronize()
    with pytest.raises(binding.PiError) as err:
        g.state()
    assert err.value.status == binding.PI_EDEVICE
    g.state()   # reported once
    g.set_raytrace_wait_limit(0.02)
    g.raytrace()
    assert np.array_equal(to_np(g.tau), ref)
    g.state()
    g.close()


def test_wait_limit_range():
    g = _grid((8, 8, 8), (4, 4, 4), "fp32", 3)
    for bad in (-1e-3, float("nan"), binding.PI_WAIT_LIMIT_MAX * 2):
        with pytest.raises(binding.PiError) as err:
            g.set_raytrace_wait_limit(bad)
        assert err.value.status == binding.PI_EINVAL
    g.set_raytrace_wait_limit(binding.PI_WAIT_LIMIT_MAX)
    g.close()


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_batch_graph_replays_with_persistent_raytrace(precision):
    """Three uneven grids, eight A3 steps replayed from the captured step graph
    with host synchronisation between some replays: the persistent raytrace
    gives the states and columns of tiles of 8, bit for bit."""
    a = synth.cfg2(n=20).with_(n=(20, 24, 18), src=(10, 12, 9))
    b = synth.cfg1(n=(16, 16, 16), dx=synth.cfg1().dx * 2)
    c = synth.cfg2(n=28).with_(n=(28, 12, 20), src=(5, 6, 15), Q=3e48)
    specs = [s.with_(precision=precision) for s in (a, b, c)]
    nHs = [synth.lognormal_density(s.shape, s.nH_mean, 1.0, 30 + i) if s.thermal == "evolve"
           else np.full(s.shape, s.nH_mean) for i, s in enumerate(specs)]
    out = {}
    for edge in (8, P):
        bt = binding.Batch(specs, precision=precision)
        bt.raytrace_tile = edge
        bt.load(nHs, T0s=[s.T0 for s in specs], t_end=[s.t_end for s in specs])
        for k in range(8):
            bt.step_o2()
            if k % 3 == 2:
                bt.state()
        t, n, _ = bt.state()
        out[edge] = (t, n, [(to_np(G.x), to_np(G.tau)) for G in bt.grids])
        bt.close()
    assert out[8][0] == out[P][0] and out[8][1] == out[P][1]
    for (xa, ta), (xb, tb) in zip(out[8][2], out[P][2]):
        assert np.array_equal(xa, xb)
        assert np.array_equal(ta, tb)
