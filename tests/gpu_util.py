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
