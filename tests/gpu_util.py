"""Helpers shared by the GPU parity tests (test code only)."""
import numpy as np

import oracle
from paper_1201_5651_amd import binding, synth


def rel_x(a, b):
    """relative error of neutral fractions: |a-b| / max(|b|, 1e-12)"""
    return np.abs(a - b) / np.maximum(np.abs(b), 1e-12)


def rel(a, b, floor=0.0):
    return np.abs(a - b) / np.maximum(np.abs(b), floor if floor > 0 else 1e-300)


def to_np(t):
    return t.detach().cpu().double().numpy()


def stored(a, precision):
    """An input as a grid of that precision holds it (float fields round it
    to float32), computed here with numpy so that the oracle's inputs never
    come from the device."""
    a = np.array(a, dtype=np.float64)   # always a copy: the oracle steps in place
    return a if precision == "fp64" else a.astype(np.float32).astype(np.float64)


def pair(spec, nH, x0=1.0, T0=None, precision=None):
    """A GPU grid and an oracle problem on the same inputs."""
    g = binding.Grid(spec, precision=precision)
    g.load(nH, x0, T0=T0)
    pb = oracle.Problem.from_spec(spec)
    st = pb.initial_state(np.asarray(nH, dtype=np.float64), x0=1.0 if not np.ndim(x0) else 1.0,
                          T0=T0 if T0 is not None else spec.T0)
    if np.ndim(x0):
        st["x"] = np.ascontiguousarray(np.asarray(x0, dtype=np.float64).reshape(pb.shape))
        if st["E"] is not None:
            st["E"] = pb.energy_from_temperature(st["nH"], st["x"], T0 if T0 is not None else spec.T0)
        st["tau"] = pb.raytrace(st["nH"], st["x"])
    return g, pb, st


def float_bar(got, want, bar, what, floor=1e-12):
    """Maximum relative error (|a-b| / max(|b|, floor)) over every cell, with
    the count of cells above the bar printed for the log."""
    err = np.abs(got - want) / np.maximum(np.abs(want), floor)
    print("%s: max rel err %.3g over %d cells (%d above %.0e)"
          % (what, err.max(), err.size, int((err > bar).sum()), bar))
    assert err.max() < bar, (what, float(err.max()))
    return err


def backward_ok(pb, spec, nH, x, E, tau, h, cells, x_got, T_got, bar, rel_steps):
    """For cells whose oracle result is ill-conditioned (it moves by far more
    than the bar under a change of the inputs at the rounding level), the GPU
    result must still be a result of the discrete method: the oracle's
    micro-integration of that cell, for an input within a few rounding units
    of the given one (relative changes rel_steps of the entering column and
    of the density), must reproduce it within the bar.  Returns the cells
    that no such input reproduces."""
    bad = []
    flat = lambda a: None if a is None else np.asarray(a).reshape(-1)
    nH, x, E, tau = flat(nH), flat(x), flat(E), flat(tau)
    x_got, T_got = flat(x_got), flat(T_got)
    for c in cells:
        geo, ell = pb.cell_env(int(c))
        E0 = 0.0 if E is None else E[c]
        ok = False
        for dn in (0.0,) + tuple(rel_steps):
            for dt in (0.0,) + tuple(rel_steps):
                n = nH[c] * (1 + dn)
                x1, E1 = pb.micro_cell(n, geo, ell, tau[c] * (1 + dt), x[c], E0, h)
                ex = abs(x_got[c] - x1) / max(abs(x1), 1e-12)
                eT = 0.0
                if E is not None:
                    T1 = max(2 * E1 / (3 * KB * nH[c] * (2 - x1)), 10.0)
                    eT = abs(T_got[c] - T1) / T1
                if ex < bar and eT < bar:
                    ok = True
                    break
            if ok:
                break
        if not ok:
            bad.append(int(c))
    return bad


KB = 1.380649e-16
