"""FP64 CPU oracle of the A3 photoionisation source-term step (Mackey 2012).

TEST INFRASTRUCTURE ONLY.  The test-suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` are the only code allowed to import this
package.  The product (``paper_1201_5651_amd``) never imports it, and the two
share no code: this wrapper drives ``oracle.c`` through ctypes.

Every function here is a thin marshalling layer; the arithmetic lives in
``oracle.c`` and follows the paper section by section (see its header).
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# The same source built with OpenMP: the per-cell loops and the octants of the
# raytrace run on all host cores, with bitwise the same results.  Loaded
# instead of the plain build when ORACLE_OPENMP=1 is set before the first call
# (the multi-core leg of the CPU baseline).
_LIB_OMP = os.path.join(_HERE, "liboracle_omp.so")

KB = 1.380649e-16
EV = 1.602176634e-12
NTAB = 64
MAX_SRC = 4

GEOM_3D, GEOM_SPHERICAL_1D, GEOM_PLANAR_1D, GEOM_PLANE_3D = 0, 1, 2, 3
SPEC_MONO, SPEC_TABLE = 0, 1
T_FIXED, T_EVOLVE = 0, 1
ALPHA_CONST, ALPHA_POWER = 0, 1
W_GEOMETRIC, W_MELLEMA = 0, 1


def build(force: bool = False, openmp: bool = False) -> str:
    """Compile oracle.c into liboracle.so with plain gcc (no fast-math);
    openmp: the OpenMP build liboracle_omp.so."""
    out = _LIB_OMP if openmp else _LIB
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-std=c99", "-D_GNU_SOURCE", "-ffp-contract=off", "-fPIC"] + \
              (["-fopenmp"] if openmp else []) + ["-shared", "-o", out + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)
    return out


class Desc(C.Structure):
    _fields_ = [
        ("geometry", C.c_int32),
        ("n", C.c_int32 * 3),
        ("src", C.c_int32 * 3),
        ("dx", C.c_double),
        ("Q", C.c_double),
        ("sigma0", C.c_double),
        ("spectrum", C.c_int32),
        ("e_excess", C.c_double),
        ("table", C.POINTER(C.c_double)),
        ("thermal", C.c_int32),
        ("T_fixed", C.c_double),
        ("recomb", C.c_int32),
        ("alpha_B", C.c_double),
        ("collisional", C.c_int32),
        ("cooling", C.c_int32),
        ("weights", C.c_int32),
        ("source_cell_rule", C.c_int32),
        ("n_sub", C.c_int32),
        ("K", C.c_double * 4),
        ("nsrc", C.c_int32),
        ("src_more", (C.c_int32 * 3) * (MAX_SRC - 1)),
        ("Q_more", C.c_double * (MAX_SRC - 1)),
    ]


class Diag(C.Structure):
    _fields_ = [
        ("n_ion", C.c_double),
        ("v_ion", C.c_double),
        ("r_ion", C.c_double),
        ("photo_rate", C.c_double),
        ("recomb_rate", C.c_double),
        ("newton_fail", C.c_int64),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        omp = os.environ.get("ORACLE_OPENMP") == "1"
        target = _LIB_OMP if omp else _LIB
        path = target if os.path.exists(target) else build(openmp=omp)
        L = C.CDLL(path)
        dp = C.POINTER(C.c_double)
        pd = C.POINTER(Desc)
        L.orc_table_build.argtypes = [C.c_double, C.c_double, dp]
        L.orc_table_eval.argtypes = [dp, C.c_int, C.c_double, dp]
        L.orc_table_eval.restype = C.c_double
        for f in (L.orc_raytrace_sc, L.orc_raytrace_lc):
            f.argtypes = [pd, dp, dp, dp]
        L.orc_cell_env.argtypes = [pd, C.c_int64, dp, dp]
        L.orc_micro_cell.argtypes = [pd] + [C.c_double] * 7 + [dp, dp]
        L.orc_micro_cell_avg.argtypes = [pd] + [C.c_double] * 7 + [dp, dp, dp]
        L.orc_rhs_cell.argtypes = [pd] + [C.c_double] * 6 + [dp, dp]
        L.orc_cell_dt.argtypes = [pd] + [C.c_double] * 6
        L.orc_cell_dt.restype = C.c_double
        L.orc_timestep.argtypes = [pd, dp, dp, dp, dp, dp]
        L.orc_chem.argtypes = [pd, dp, dp, dp, dp, C.c_double, dp, dp]
        L.orc_step.argtypes = [pd, dp, dp, dp, dp, dp, C.c_double, C.c_int, dp]
        L.orc_step_tc.argtypes = [pd, dp, dp, dp, dp, dp, dp, C.c_double, C.c_int, dp]
        L.orc_a1_pass.argtypes = [pd, dp, dp, dp, C.c_double, dp, dp]
        L.orc_diagnostics.argtypes = [pd, dp, dp, dp, dp, C.POINTER(Diag)]
        L.orc_newton_failures.restype = C.c_int64
        L.orc_front_index_1d.argtypes = [C.c_int, dp]
        L.orc_mean_chord_source_cell.restype = C.c_double
        _lib = L
    return _lib


def _p(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def table_build(T_bb: float, Q: float) -> np.ndarray:
    """Blackbody rate table: rows tau, P, P1, H, H1 (shape (5, 64))."""
    out = np.zeros(5 * NTAB)
    rc = lib().orc_table_build(T_bb, Q, _p(out))
    if rc != 0:
        raise ValueError("orc_table_build failed")
    return out.reshape(5, NTAB)


def table_eval(table: np.ndarray, which: int, tau: float):
    d = C.c_double(0.0)
    v = lib().orc_table_eval(_p(np.ascontiguousarray(table).ravel()), which, tau, C.byref(d))
    return v, d.value


class Problem:
    """A grid description for the oracle plus the arrays it keeps alive."""

    def __init__(self, *, geometry=GEOM_3D, n=(8, 8, 8), src=(0, 0, 0), dx=1.0, Q=0.0,
                 sigma0=6.3e-18, spectrum=SPEC_MONO, e_excess=0.0, T_bb=1e5, thermal=T_FIXED,
                 T_fixed=1e4, recomb=ALPHA_CONST, alpha_B=2.59e-13, collisional=0,
                 cooling=1, weights=W_MELLEMA, source_cell_rule=1, n_sub=2,
                 K=(math.inf, math.inf, math.inf, 0.25), table=None, more_sources=()):
        d = Desc()
        d.geometry = geometry
        n3 = tuple(n) + (1,) * (3 - len(tuple(n)))
        s3 = tuple(src) + (0,) * (3 - len(tuple(src)))
        d.n[:] = n3
        d.src[:] = s3
        d.dx = dx
        d.Q = Q
        d.sigma0 = sigma0
        d.spectrum = spectrum
        d.e_excess = e_excess
        self.table = None
        if spectrum == SPEC_TABLE:
            self.table = np.ascontiguousarray(table if table is not None else table_build(T_bb, Q),
                                              dtype=np.float64).ravel()
            d.table = _p(self.table)
        d.thermal = thermal
        d.T_fixed = T_fixed
        d.recomb = recomb
        d.alpha_B = alpha_B
        d.collisional = collisional
        d.cooling = cooling
        d.weights = weights
        d.source_cell_rule = source_cell_rule
        d.n_sub = n_sub
        d.K[:] = K
        # further point sources: ((i, j, k), Q) each; columns then carry one
        # grid per source (tau_shape)
        more = list(more_sources)
        if len(more) > MAX_SRC - 1:
            raise ValueError(f"at most {MAX_SRC} sources")
        d.nsrc = 1 + len(more)
        for m, (v, q) in enumerate(more):
            d.src_more[m][:] = tuple(int(c) for c in v)
            d.Q_more[m] = float(q)
        self.desc = d
        self.shape = (n3[2], n3[1], n3[0]) if geometry in (GEOM_3D, GEOM_PLANE_3D) else (n3[0],)
        self.nsrc = d.nsrc
        self.tau_shape = (self.nsrc,) + self.shape if self.nsrc > 1 else self.shape

    @property
    def ncells(self):
        return int(np.prod(self.shape))

    def energy_from_temperature(self, nH, x, T):
        """Internal energy density of pure H with gamma = 5/3 (Sect. 2)."""
        return 1.5 * nH * (2.0 - x) * KB * T

    def temperature(self, nH, x, E):
        if self.desc.thermal == T_FIXED:
            return np.full_like(x, self.desc.T_fixed)
        return np.maximum(2.0 * E / (3.0 * KB * nH * (2.0 - x)), 10.0)

    def raytrace(self, nH, x, long_characteristics=False):
        tau = np.zeros(self.tau_shape)
        f = lib().orc_raytrace_lc if long_characteristics else lib().orc_raytrace_sc
        rc = f(C.byref(self.desc), _p(nH), _p(x), _p(tau))
        if rc != 0:
            raise RuntimeError("oracle raytrace failed")
        return tau

    def cell_env(self, cell):
        g, e = C.c_double(), C.c_double()
        lib().orc_cell_env(C.byref(self.desc), int(cell), C.byref(g), C.byref(e))
        return g.value, e.value

    def micro_cell(self, nH, geo, ell, tau_in, x0, E0, h):
        x1, E1 = C.c_double(), C.c_double()
        lib().orc_micro_cell(C.byref(self.desc), nH, geo, ell, tau_in, x0, E0, h,
                             C.byref(x1), C.byref(E1))
        return x1.value, E1.value

    def micro_cell_avg(self, nH, geo, ell, tau_in, x0, E0, h):
        """(x1, E1, tau_avg): the micro-integration and the cell's time-averaged
        optical depth -ln <exp(-n sigma0 ell x(t))> over h."""
        x1, E1, ta = C.c_double(), C.c_double(), C.c_double()
        lib().orc_micro_cell_avg(C.byref(self.desc), nH, geo, ell, tau_in, x0, E0, h,
                                 C.byref(x1), C.byref(E1), C.byref(ta))
        return x1.value, E1.value, ta.value

    def rhs_cell(self, nH, geo, ell, tau_in, x, E):
        fx, fE = C.c_double(), C.c_double()
        lib().orc_rhs_cell(C.byref(self.desc), nH, geo, ell, tau_in, x, E, C.byref(fx),
                           C.byref(fE))
        return fx.value, fE.value

    def cell_dt(self, nH, geo, ell, tau_in, x, E):
        return lib().orc_cell_dt(C.byref(self.desc), nH, geo, ell, tau_in, x, E)

    def timestep(self, nH, x, E, tau):
        dt = C.c_double()
        lib().orc_timestep(C.byref(self.desc), _p(nH), _p(x), _p(E), _p(tau), C.byref(dt))
        return dt.value

    def chem(self, nH, x0, E0, tau, h):
        x1 = np.empty_like(x0)
        E1 = None if E0 is None else np.empty_like(E0)
        lib().orc_chem(C.byref(self.desc), _p(nH), _p(x0), _p(E0), _p(tau), h, _p(x1), _p(E1))
        return x1, E1

    def step(self, state, t_end, algo=3, nH_half=None):
        """Advance ``state`` (dict nH, x, E or None, tau, t) by one step in place;
        ``nH_half``: time-centred density for the half-step raytrace."""
        t = C.c_double(state["t"])
        dt = C.c_double()
        nh = None if nH_half is None else np.ascontiguousarray(nH_half, dtype=np.float64)
        rc = lib().orc_step_tc(C.byref(self.desc), _p(state["nH"]), _p(nh), _p(state["x"]),
                               _p(state["E"]), _p(state["tau"]), C.byref(t), t_end, algo,
                               C.byref(dt))
        state["t"] = t.value
        return rc, dt.value

    def a1_pass(self, nH, x, E, dt):
        """Algorithm 1's combined pass over dt: returns (x, E, tau_avg, kbar)
        without touching the inputs."""
        x1 = np.ascontiguousarray(x, dtype=np.float64).copy()
        E1 = None if E is None else np.ascontiguousarray(E, dtype=np.float64).copy()
        ta = np.zeros_like(x1)
        kb = np.zeros_like(x1)
        rc = lib().orc_a1_pass(C.byref(self.desc), _p(np.ascontiguousarray(nH, dtype=np.float64)),
                               _p(x1), _p(E1), dt, _p(ta), _p(kb))
        if rc != 0:
            raise RuntimeError(f"orc_a1_pass failed ({rc})")
        return x1, E1, ta, kb

    def diagnostics(self, state):
        d = Diag()
        lib().orc_diagnostics(C.byref(self.desc), _p(state["nH"]), _p(state["x"]),
                              _p(state["E"]), _p(state["tau"]), C.byref(d))
        return {k: getattr(d, k) for k, _ in Diag._fields_}

    def initial_state(self, nH, x0=1.0, T0=None):
        nH = np.ascontiguousarray(np.broadcast_to(np.asarray(nH, dtype=np.float64), self.shape)).copy()
        x = np.full(self.shape, float(x0))
        E = None
        if self.desc.thermal == T_EVOLVE:
            E = self.energy_from_temperature(nH, x, 50.0 if T0 is None else T0)
        tau = self.raytrace(nH, x)
        return {"nH": nH, "x": x, "E": E, "tau": tau, "t": 0.0}

    def run(self, state, t_end, algo=3, max_steps=10**7, callback=None):
        steps = 0
        while state["t"] < t_end and steps < max_steps:
            rc, dt = self.step(state, t_end, algo)
            if rc != 0:
                break
            steps += 1
            if callback is not None:
                callback(state, steps, dt)
        return steps

    @classmethod
    def from_spec(cls, spec, **over):
        """Oracle problem for a ``synth.GridSpec`` (input description only)."""
        kw = dict(geometry=GEOM_PLANE_3D if getattr(spec, "source", "point") == "plane" else GEOM_3D,
                  n=tuple(spec.n), src=tuple(spec.src), dx=spec.dx, Q=spec.Q,
                  sigma0=6.3e-18, spectrum=SPEC_TABLE if spec.spectrum == "table" else SPEC_MONO,
                  e_excess=spec.e_excess, T_bb=spec.T_bb,
                  thermal=T_EVOLVE if spec.thermal == "evolve" else T_FIXED,
                  T_fixed=spec.T_fixed,
                  recomb=ALPHA_POWER if spec.recomb == "power" else ALPHA_CONST,
                  alpha_B=spec.alpha_B, collisional=int(spec.collisional),
                  cooling=int(spec.cooling),
                  weights=W_MELLEMA if spec.weights == "mellema" else W_GEOMETRIC,
                  source_cell_rule=int(spec.source_cell_rule), n_sub=spec.n_sub, K=tuple(spec.K),
                  more_sources=tuple(getattr(spec, "more_sources", ())))
        kw.update(over)
        return cls(**kw)


def newton_failures() -> int:
    return int(lib().orc_newton_failures())


def reset_newton_failures() -> None:
    lib().orc_reset_newton_failures()


def front_index_1d(x: np.ndarray) -> int:
    x = np.ascontiguousarray(x, dtype=np.float64)
    return int(lib().orc_front_index_1d(len(x), _p(x)))


def mean_chord_source_cell() -> float:
    return float(lib().orc_mean_chord_source_cell())
