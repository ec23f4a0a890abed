"""Checkpoints through the C ABI: pi_grid_save / pi_grid_load of a grid, and
pi_checkpoint / resumed submission of a served request.  A grid (or request)
continued from a checkpoint goes through the same arithmetic as the
uninterrupted one, so the continuation is compared bit for bit."""
import time

import numpy as np
import pytest

from paper_1201_5651_amd import binding, synth
from gpu_util import to_np

pytestmark = pytest.mark.gpu


def _grid(spec, precision, nH):
    g = binding.Grid(spec, precision=precision)
    g.load(nH, 1.0, T0=spec.T0)
    return g


@pytest.mark.parametrize("precision", ["fp64", "fp32", "mixed"])
def test_save_load_round_trip_continues_bit_for_bit(precision):
    """Run 6 steps, save, run 5 more; load the save into a second grid and run
    5 steps: the states, columns and clocks agree bit for bit.  The checkpoint
    holds the clock and the step count."""
    spec = synth.cfg2(n=20).with_(n=(20, 17, 23), src=(9, 8, 12))
    nH = synth.lognormal_density(spec.shape, 10.0, 1.0, 8)
    a = _grid(spec, precision, nH)
    for _ in range(6):
        a.step_o2(spec.t_end)
    ck = a.save()
    t6, n6, _ = a.state()
    for _ in range(5):
        a.step_o2(spec.t_end)
    b = binding.Grid(spec, precision=precision)
    b.restore(ck)
    assert b.state()[:2] == (t6, n6)
    for _ in range(5):
        b.step_o2(spec.t_end)
    assert a.state() == b.state()
    for k in ("x", "E", "tau", "nH"):
        assert np.array_equal(to_np(getattr(a, k)), to_np(getattr(b, k))), k
    a.close()
    b.close()


def test_checkpoint_sizes_and_layout_checks():
    spec = synth.cfg2(n=12)
    g = binding.Grid(spec, precision="fp32")
    g.load(np.full(spec.shape, 10.0), 1.0, T0=50.0)
    ck = g.save()
    ncell = spec.ncells
    # n_H, x, E and one column array of float, after the header
    assert (len(ck) - 4 * 4 * ncell) in range(64, 257)
    # a truncated checkpoint, or one of another layout, is refused
    with pytest.raises(binding.PiError):
        g.restore(ck[:-4])
    other = binding.Grid(spec.with_(n=(12, 12, 13)), precision="fp32")
    with pytest.raises(binding.PiError):
        other.restore(ck)
    other64 = binding.Grid(spec, precision="fp64")
    with pytest.raises(binding.PiError):
        other64.restore(ck)
    g.close()
    other.close()
    other64.close()


def _wait(srv, tk, timeout=120.0):
    t0 = time.time()
    while True:
        st, info, x, T = srv.poll(tk)
        if st != binding.PI_PENDING:
            return st, info, x, T
        assert time.time() - t0 < timeout, "served request did not finish"
        time.sleep(0.003)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_served_request_checkpoint_resumes_bit_for_bit(precision):
    """A running request is checkpointed; the checkpoint submitted to a second
    server continues to the same t_end and returns bit for bit the result of
    the uninterrupted request.  A grid loaded from the same checkpoint and
    stepped alone agrees too."""
    spec = synth.cfg2(n=18).with_(n=(18, 14, 16), src=(9, 7, 8), precision=precision)
    nH = synth.lognormal_density(spec.shape, 10.0, 1.0, 12)
    t_end = 0.01 * spec.t_rec
    srv = binding.Server(precision=precision, max_active=4, steps_per_tick=2)
    tk = srv.submit(spec, nH, T0=spec.T0, t_end=t_end)
    ck = None
    t0 = time.time()
    while ck is None:
        ck = srv.checkpoint(tk)
        assert time.time() - t0 < 60
    st, info, x_full, T_full = _wait(srv, tk)
    assert st == binding.PI_OK
    srv2 = binding.Server(precision=precision, max_active=4, steps_per_tick=3)
    tk2 = srv2.submit(spec, t_end=t_end, checkpoint=ck)
    st2, info2, x2, T2 = _wait(srv2, tk2)
    assert st2 == binding.PI_OK
    assert info2["nsteps"] == info["nsteps"] and info2["t"] == info["t"]
    assert np.array_equal(x2, x_full) and np.array_equal(T2, T_full)
    # the same checkpoint in a single grid
    g = binding.Grid(spec, precision=precision)
    g.restore(ck)
    g.run(t_end, check_every=4)
    assert np.array_equal(to_np(g.x), x_full)
    g.close()
    # a finished request cannot be checkpointed
    with pytest.raises(binding.PiError):
        srv.checkpoint(tk)
    srv.close()
    srv2.close()
