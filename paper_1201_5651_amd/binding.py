"""Python binding of the C ABI in include/pi.h (ctypes).

Argument marshalling only: every step of the method runs in the HIP kernels of
libpi.so.  PyTorch provides the device memory (caller-owned field tensors) and
the stream handed to every call.  There is no CPU fallback: without a built
libpi.so, or without a GPU, the calls fail loudly.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpi.so")

PI_OK, PI_PENDING = 0, 1
PI_EINVAL, PI_ENOMEM, PI_EDEVICE, PI_EREJECTED, PI_ENAN, PI_ECANCELLED = -1, -2, -3, -4, -5, -6
PI_FP64, PI_FP32, PI_MIXED, PI_MIXED_FRONT = 0, 1, 2, 3
PRECISIONS = {"fp64": PI_FP64, "fp32": PI_FP32, "mixed": PI_MIXED, "mixed_front": PI_MIXED_FRONT}
PI_SPEC_MONO, PI_SPEC_TABLE = 0, 1
PI_T_FIXED, PI_T_EVOLVE = 0, 1
PI_ALPHA_CONST, PI_ALPHA_POWER = 0, 1
PI_W_GEOMETRIC, PI_W_MELLEMA = 0, 1
PI_SRC_POINT, PI_SRC_PLANE = 0, 1
PI_BUF_N, PI_BUF_HALF = 0, 1
PI_NDIAG = 8
PI_NWORK = 5
PI_NTAB = 64
PI_MAX_SRC = 4
PI_TILE_PERSISTENT = 0x108
PI_WAIT_LIMIT_MAX = 10.0

# every symbol include/pi.h declares
ABI_SYMBOLS = (
    "pi_grid_create", "pi_grid_destroy", "pi_raytrace", "pi_chem_step", "pi_timestep",
    "pi_step_o2", "pi_step_o1", "pi_init_energy", "pi_set_time", "pi_grid_state",
    "pi_diagnostics", "pi_work_counters", "pi_table_build", "pi_last_error", "pi_abi_version",
    "pi_batch_create", "pi_batch_destroy", "pi_batch_set_time", "pi_batch_init_energy",
    "pi_batch_raytrace", "pi_batch_step_o2", "pi_batch_state", "pi_batch_diagnostics",
    "pi_batch_work_counters",
    "pi_server_create", "pi_submit", "pi_poll", "pi_cancel", "pi_server_stats", "pi_server_destroy",
    "pi_set_raytrace_tile", "pi_get_raytrace_tile", "pi_batch_set_raytrace_tile",
    "pi_batch_get_raytrace_tile", "pi_set_raytrace_wait_limit", "pi_chem_raytrace",
    "pi_batch_set_raytrace_wait_limit",
    "pi_step_a1",
    "pi_batch_step_a1",
    "pi_grid_required_bytes", "pi_grid_save", "pi_grid_load", "pi_checkpoint",
    "pi_raytrace_static",
)


class PiError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"pi status {status}: {msg}")
        self.status = status


class GridDesc(C.Structure):
    _fields_ = [
        ("n", C.c_int32 * 3),
        ("src", C.c_int32 * 3),
        ("dx", C.c_double),
        ("Q", C.c_double),
        ("sigma0", C.c_double),
        ("spectrum", C.c_int32),
        ("e_excess", C.c_double),
        ("T_bb", C.c_double),
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
        ("precision", C.c_int32),
        ("source", C.c_int32),
        ("nsrc", C.c_int32),
        ("src_more", (C.c_int32 * 3) * (PI_MAX_SRC - 1)),
        ("Q_more", C.c_double * (PI_MAX_SRC - 1)),
    ]


class Fields(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("nH", "x", "E", "tau", "x_half", "E_half", "tau_half",
                                          "nH_half")]


class ServerDesc(C.Structure):
    _fields_ = [("hbm_budget", C.c_size_t), ("max_active", C.c_int32), ("precision", C.c_int32),
                ("steps_per_tick", C.c_int32)]


class Request(C.Structure):
    _fields_ = [("desc", GridDesc), ("nH", C.POINTER(C.c_double)), ("x0", C.POINTER(C.c_double)),
                ("T0", C.c_double), ("t_end", C.c_double), ("checkpoint", C.c_void_p),
                ("checkpoint_bytes", C.c_size_t)]


class Result(C.Structure):
    _fields_ = [("status", C.c_int32), ("t", C.c_double), ("nsteps", C.c_int64),
                ("latency_s", C.c_double), ("queue_s", C.c_double)]


_lib = None


def lib() -> C.CDLL:
    """Load libpi.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, d = C.c_void_p, C.c_int, C.c_int64, C.c_double
        dp = C.POINTER(C.c_double)
        L.pi_grid_create.argtypes = [C.POINTER(GridDesc), C.POINTER(Fields), C.POINTER(vp)]
        L.pi_grid_destroy.argtypes = [vp]
        L.pi_raytrace.argtypes = [vp, i32, i32, vp]
        L.pi_chem_step.argtypes = [vp, i32, d, i32, i32, i32, vp]
        L.pi_timestep.argtypes = [vp, d, vp]
        L.pi_step_o2.argtypes = [vp, d, vp]
        L.pi_step_o1.argtypes = [vp, d, vp]
        L.pi_step_a1.argtypes = [vp, d, vp]
        L.pi_init_energy.argtypes = [vp, d, i32, vp]
        L.pi_set_time.argtypes = [vp, d, i64, vp]
        L.pi_grid_state.argtypes = [vp, dp, C.POINTER(C.c_int64), dp, vp]
        L.pi_diagnostics.argtypes = [vp, dp, vp]
        L.pi_work_counters.argtypes = [vp, C.POINTER(C.c_int64), i32, vp]
        L.pi_table_build.argtypes = [d, d, dp]
        i64p = C.POINTER(C.c_int64)
        L.pi_batch_create.argtypes = [i32, C.POINTER(GridDesc), C.POINTER(Fields), C.POINTER(vp)]
        L.pi_batch_destroy.argtypes = [vp]
        L.pi_batch_set_time.argtypes = [vp, dp, i64p, dp, vp]
        L.pi_batch_init_energy.argtypes = [vp, dp, i32, vp]
        L.pi_batch_raytrace.argtypes = [vp, i32, i32, vp]
        L.pi_batch_step_o2.argtypes = [vp, vp]
        L.pi_batch_step_a1.argtypes = [vp, vp]
        L.pi_batch_state.argtypes = [vp, dp, i64p, dp, vp]
        L.pi_batch_diagnostics.argtypes = [vp, dp, vp]
        L.pi_batch_work_counters.argtypes = [vp, i64p, i32, vp]
        L.pi_server_create.argtypes = [C.POINTER(ServerDesc), C.POINTER(vp)]
        L.pi_submit.argtypes = [vp, C.POINTER(Request), C.POINTER(C.c_uint64)]
        L.pi_poll.argtypes = [vp, C.c_uint64, C.POINTER(Result), dp, dp]
        L.pi_cancel.argtypes = [vp, C.c_uint64]
        L.pi_server_stats.argtypes = [vp, dp]
        L.pi_server_destroy.argtypes = [vp]
        ip = C.POINTER(C.c_int)
        L.pi_set_raytrace_tile.argtypes = [vp, i32]
        L.pi_get_raytrace_tile.argtypes = [vp, ip]
        L.pi_batch_set_raytrace_tile.argtypes = [vp, i32]
        L.pi_batch_get_raytrace_tile.argtypes = [vp, ip]
        L.pi_set_raytrace_wait_limit.argtypes = [vp, C.c_double]
        L.pi_chem_raytrace.argtypes = [vp, i32, C.c_double, i32, i32, i32, i32, vp]
        L.pi_batch_set_raytrace_wait_limit.argtypes = [vp, C.c_double]
        szp = C.POINTER(C.c_size_t)
        L.pi_grid_required_bytes.argtypes = [C.POINTER(GridDesc), szp, szp]
        L.pi_grid_save.argtypes = [vp, vp, C.c_size_t, szp, vp]
        L.pi_grid_load.argtypes = [vp, vp, C.c_size_t, vp]
        L.pi_checkpoint.argtypes = [vp, C.c_uint64, vp, C.c_size_t, szp]
        L.pi_raytrace_static.argtypes = [C.POINTER(GridDesc), C.POINTER(Fields), i32, i32, vp]
        L.pi_last_error.restype = C.c_char_p
        L.pi_abi_version.restype = C.c_int
        for name in ABI_SYMBOLS:
            if name not in ("pi_last_error", "pi_abi_version"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def check(status: int) -> None:
    if status != PI_OK:
        raise PiError(status, lib().pi_last_error().decode())


def table_build(T_bb: float, Q: float):
    """pi_table_build: rows tau, P, -dP/dtau, H, -dH/dtau (host-only)."""
    import numpy as np
    out = np.zeros(5 * PI_NTAB)
    check(lib().pi_table_build(T_bb, Q, out.ctypes.data_as(C.POINTER(C.c_double))))
    return out.reshape(5, PI_NTAB)


def required_bytes(spec, precision: Optional[str] = None):
    """pi_grid_required_bytes: (caller-owned field bytes, library device bytes)."""
    d = desc_from_spec(spec, precision)
    fb, wb = C.c_size_t(), C.c_size_t()
    check(lib().pi_grid_required_bytes(C.byref(d), C.byref(fb), C.byref(wb)))
    return fb.value, wb.value


def desc_from_spec(spec, precision: Optional[str] = None, sigma0: float = 6.3e-18) -> GridDesc:
    """pi_grid_desc for a synth.GridSpec."""
    d = GridDesc()
    d.n[:] = tuple(int(v) for v in spec.n)
    d.src[:] = tuple(int(v) for v in spec.src)
    d.dx = spec.dx
    d.Q = spec.Q
    d.sigma0 = sigma0
    d.spectrum = PI_SPEC_TABLE if spec.spectrum == "table" else PI_SPEC_MONO
    d.e_excess = spec.e_excess
    d.T_bb = spec.T_bb
    d.thermal = PI_T_EVOLVE if spec.thermal == "evolve" else PI_T_FIXED
    d.T_fixed = spec.T_fixed
    d.recomb = PI_ALPHA_POWER if spec.recomb == "power" else PI_ALPHA_CONST
    d.alpha_B = spec.alpha_B
    d.collisional = int(spec.collisional)
    d.cooling = int(spec.cooling)
    d.weights = PI_W_MELLEMA if spec.weights == "mellema" else PI_W_GEOMETRIC
    d.source_cell_rule = int(spec.source_cell_rule)
    d.n_sub = int(spec.n_sub)
    d.K[:] = tuple(float(k) for k in spec.K)
    prec = precision or spec.precision
    d.precision = PRECISIONS[prec]
    d.source = PI_SRC_PLANE if getattr(spec, "source", "point") == "plane" else PI_SRC_POINT
    more = tuple(getattr(spec, "more_sources", ()))
    if len(more) > PI_MAX_SRC - 1:
        raise ValueError(f"at most {PI_MAX_SRC} sources")
    d.nsrc = 1 + len(more)
    for m, (v, q) in enumerate(more):
        d.src_more[m][:] = tuple(int(c) for c in v)
        d.Q_more[m] = float(q)
    return d


FIELD_NAMES = ("nH", "x", "E", "tau", "x_half", "E_half", "tau_half", "nH_half")


def raytrace_static(spec, fields, state=PI_BUF_N, tau_buf=PI_BUF_N, precision=None):
    """pi_raytrace_static on a GridFields (no grid object, nothing allocated
    by the library), on torch's current stream."""
    import torch
    d = desc_from_spec(spec, precision or fields.precision)
    f = fields.abi_fields()
    check(lib().pi_raytrace_static(C.byref(d), C.byref(f), state, tau_buf,
                                   C.c_void_p(torch.cuda.current_stream().cuda_stream)))


class GridFields:
    """Device field tensors of one grid (torch, caller-owned memory of the ABI)."""

    def __init__(self, spec, precision: str, device, time_centred_density: bool = False):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the photoionisation library needs a GPU (no CPU fallback)")
        self.spec = spec
        self.precision = precision
        self.dtype = torch.float64 if precision == "fp64" else torch.float32
        self.device = torch.device(device)
        z = lambda: torch.zeros(spec.shape, dtype=self.dtype, device=self.device)
        # columns: one grid of cells per source
        ns = 1 + len(tuple(getattr(spec, "more_sources", ())))
        tshape = (ns,) + tuple(spec.shape) if ns > 1 else spec.shape
        zt = lambda: torch.zeros(tshape, dtype=self.dtype, device=self.device)
        self.nH, self.x, self.tau = z(), z(), zt()
        self.x_half, self.tau_half = z(), zt()
        evolve = spec.thermal == "evolve"
        self.E = z() if evolve else None
        self.E_half = z() if evolve else None
        # time-centred density for the half-step raytrace (None: nH)
        self.nH_half = z() if time_centred_density else None

    def abi_fields(self) -> Fields:
        f = Fields()
        for k in FIELD_NAMES:
            t = getattr(self, k)
            setattr(f, k, t.data_ptr() if t is not None else None)
        return f

    def fill(self, nH, x=1.0):
        import torch
        self.nH.copy_(torch.as_tensor(nH, dtype=self.dtype).reshape(self.spec.shape))
        if isinstance(x, (int, float)):
            self.x.fill_(float(x))
        else:
            self.x.copy_(torch.as_tensor(x, dtype=self.dtype).reshape(self.spec.shape))


class Grid:
    """One photoionisation problem resident on the GPU.

    Owns its field tensors (torch, on ``device``) and the library handle.
    Methods map one-to-one onto the ABI calls, on torch's current stream.
    """

    def __init__(self, spec, device: str = "cuda:0", precision: Optional[str] = None,
                 time_centred_density: bool = False):
        self.spec = spec
        self.precision = precision or spec.precision
        self._fl = GridFields(spec, self.precision, device, time_centred_density)
        self.dtype, self.device = self._fl.dtype, self._fl.device
        for k in FIELD_NAMES:
            setattr(self, k, getattr(self._fl, k))
        f = self._fl.abi_fields()
        self._fields = f
        self._desc = desc_from_spec(spec, self.precision)
        h = C.c_void_p()
        check(lib().pi_grid_create(C.byref(self._desc), C.byref(f), C.byref(h)))
        self._h = h

    # -- stream
    @staticmethod
    def _stream():
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)

    # -- state
    def load(self, nH, x=1.0, T0: Optional[float] = None, t: float = 0.0, nsteps: int = 0):
        """Copy density and neutral fraction in, set E from T0 (T-evolving
        grids), raytrace the initial columns and set the clock."""
        self._fl.fill(nH, x)
        s = self._stream()
        if self.E is not None:
            check(lib().pi_init_energy(self._h, float(T0 if T0 is not None else self.spec.T0),
                                       PI_BUF_N, s))
        check(lib().pi_raytrace(self._h, PI_BUF_N, PI_BUF_N, s))
        check(lib().pi_set_time(self._h, float(t), int(nsteps), s))

    def raytrace(self, state=PI_BUF_N, tau_buf=PI_BUF_N):
        check(lib().pi_raytrace(self._h, state, tau_buf, self._stream()))

    def set_time(self, t: float, nsteps: int = 0):
        check(lib().pi_set_time(self._h, float(t), int(nsteps), self._stream()))

    def chem_step(self, h: float, tau_buf=PI_BUF_N, from_state=PI_BUF_N, to_state=PI_BUF_N,
                  use_device_dt: bool = False):
        check(lib().pi_chem_step(self._h, int(use_device_dt), float(h), tau_buf, from_state,
                                 to_state, self._stream()))

    def chem_raytrace(self, h: float, tau_buf=PI_BUF_N, from_state=PI_BUF_N, to_state=PI_BUF_N,
                      tau_out=PI_BUF_N, use_device_dt: bool = False):
        """pi_chem_raytrace: chem_step, then the raytrace of to_state into tau_out."""
        check(lib().pi_chem_raytrace(self._h, int(use_device_dt), float(h), tau_buf, from_state,
                                     to_state, tau_out, self._stream()))

    def timestep(self, t_end: float):
        check(lib().pi_timestep(self._h, float(t_end), self._stream()))

    def step_o2(self, t_end: float):
        check(lib().pi_step_o2(self._h, float(t_end), self._stream()))

    def step_o1(self, t_end: float):
        check(lib().pi_step_o1(self._h, float(t_end), self._stream()))

    def step_a1(self, t_end: float):
        """One step of algorithm 1 (the implicit scheme with time-averaged
        attenuation); afterwards x_half holds the time-averaged optical depth
        per cell length and tau_half the time-averaged entering columns."""
        check(lib().pi_step_a1(self._h, float(t_end), self._stream()))

    def state(self):
        t, dt = C.c_double(), C.c_double()
        n = C.c_int64()
        check(lib().pi_grid_state(self._h, C.byref(t), C.byref(n), C.byref(dt), self._stream()))
        return t.value, n.value, dt.value

    def diagnostics(self):
        out = (C.c_double * PI_NDIAG)()
        check(lib().pi_diagnostics(self._h, out, self._stream()))
        keys = ("n_ion", "v_ion", "r_ion", "photo_rate", "recomb_rate", "nonfinite", "octants", "t")
        return dict(zip(keys, list(out)))

    @property
    def raytrace_tile(self) -> int:
        v = C.c_int()
        check(lib().pi_get_raytrace_tile(self._h, C.byref(v)))
        return v.value

    @raytrace_tile.setter
    def raytrace_tile(self, edge: int):
        check(lib().pi_set_raytrace_tile(self._h, int(edge)))

    def set_raytrace_wait_limit(self, seconds: float):
        """pi_set_raytrace_wait_limit: longest wait of a persistent raytrace tile."""
        check(lib().pi_set_raytrace_wait_limit(self._h, float(seconds)))

    def work_counters(self, reset: bool = False):
        out = (C.c_int64 * PI_NWORK)()
        check(lib().pi_work_counters(self._h, out, int(reset), self._stream()))
        return {"accepted": out[0], "rejected": out[1], "fallbacks": out[2], "newton": out[3],
                "resolved_fp64": out[4]}

    def save(self) -> bytes:
        """pi_grid_save: the checkpoint of the grid's state and clock."""
        need = C.c_size_t()
        check(lib().pi_grid_save(self._h, None, 0, C.byref(need), self._stream()))
        buf = C.create_string_buffer(need.value)
        check(lib().pi_grid_save(self._h, buf, need.value, None, self._stream()))
        return buf.raw

    def restore(self, ckpt: bytes):
        """pi_grid_load: state, columns and clock from a checkpoint."""
        buf = C.create_string_buffer(bytes(ckpt), len(ckpt))
        check(lib().pi_grid_load(self._h, buf, len(ckpt), self._stream()))

    def run(self, t_end: float, order: int = 2, max_steps: int = 10**8, check_every: int = 64):
        """Step until t_end (order 2: algorithm 3; order 1: algorithm 2).
        Returns the number of steps taken; raises PiError if a burst of steps
        leaves the clock where it was before t_end."""
        t0, n0, _ = self.state()
        taken, t = 0, t0
        while taken < max_steps:
            burst = min(check_every, max_steps - taken)
            for _ in range(burst):
                (self.step_o2 if order == 2 else self.step_o1)(t_end)
            t_prev = t
            t, n, _ = self.state()
            if t >= t_end:
                taken = n - n0
                break
            if n - n0 == taken or t == t_prev:
                raise PiError(PI_EDEVICE, "no progress: the timestep of eq. (4) is zero")
            taken = n - n0
        return taken

    def close(self):
        if getattr(self, "_h", None):
            check(lib().pi_grid_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many grids advanced together (one launch per kernel for all of them,
    each step replayed from a captured HIP graph).  ``grids[i]`` holds the
    field tensors of grid i; every grid keeps its own clock and t_end."""

    def __init__(self, specs, device: str = "cuda:0", precision: Optional[str] = None,
                 time_centred_density=False):
        """``time_centred_density``: a bool for every grid, or one per grid,
        giving the grid an ``nH_half`` field for its half-step raytraces."""
        self.specs = list(specs)
        self.precision = precision or self.specs[0].precision
        tc = (list(time_centred_density) if isinstance(time_centred_density, (list, tuple))
              else [bool(time_centred_density)] * len(self.specs))
        self.grids = [GridFields(s, self.precision, device, c) for s, c in zip(self.specs, tc)]
        n = len(self.specs)
        self._descs = (GridDesc * n)(*[desc_from_spec(s, self.precision) for s in self.specs])
        self._fields = (Fields * n)(*[g.abi_fields() for g in self.grids])
        h = C.c_void_p()
        check(lib().pi_batch_create(n, self._descs, self._fields, C.byref(h)))
        self._h = h

    @property
    def n(self) -> int:
        return len(self.specs)

    _stream = staticmethod(Grid._stream)

    def _arr(self, vals, ctype=C.c_double):
        vals = list(vals)
        assert len(vals) == self.n
        return (ctype * self.n)(*vals)

    def load(self, nHs, x0s=None, T0s=None, t=0.0, t_end=None):
        """Density and neutral fraction of every grid, energies from T0,
        initial columns, clocks at t and the t_end of each grid."""
        for i, g in enumerate(self.grids):
            g.fill(nHs[i], 1.0 if x0s is None else x0s[i])
        s = self._stream()
        if any(sp.thermal == "evolve" for sp in self.specs):
            T0 = [float(T0s[i] if T0s is not None else sp.T0) for i, sp in enumerate(self.specs)]
            check(lib().pi_batch_init_energy(self._h, self._arr(T0), PI_BUF_N, s))
        check(lib().pi_batch_raytrace(self._h, PI_BUF_N, PI_BUF_N, s))
        t_end = [sp.t_end for sp in self.specs] if t_end is None else t_end
        self.set_time([t] * self.n if isinstance(t, (int, float)) else t, t_end)

    def set_time(self, t, t_end, nsteps=None):
        self._t_end = [float(v) for v in t_end]
        ns = None if nsteps is None else self._arr(nsteps, C.c_int64)
        check(lib().pi_batch_set_time(self._h, self._arr(t), ns, self._arr(t_end), self._stream()))

    def raytrace(self, state=PI_BUF_N, tau_buf=PI_BUF_N):
        check(lib().pi_batch_raytrace(self._h, state, tau_buf, self._stream()))

    def step_o2(self):
        check(lib().pi_batch_step_o2(self._h, self._stream()))

    def step_a1(self):
        check(lib().pi_batch_step_a1(self._h, self._stream()))

    @property
    def raytrace_tile(self) -> int:
        v = C.c_int()
        check(lib().pi_batch_get_raytrace_tile(self._h, C.byref(v)))
        return v.value

    @raytrace_tile.setter
    def raytrace_tile(self, edge: int):
        check(lib().pi_batch_set_raytrace_tile(self._h, int(edge)))

    def set_raytrace_wait_limit(self, seconds: float):
        """pi_batch_set_raytrace_wait_limit: longest wait of a persistent raytrace tile."""
        check(lib().pi_batch_set_raytrace_wait_limit(self._h, float(seconds)))

    def state(self):
        t, dt = (C.c_double * self.n)(), (C.c_double * self.n)()
        k = (C.c_int64 * self.n)()
        check(lib().pi_batch_state(self._h, t, k, dt, self._stream()))
        return list(t), list(k), list(dt)

    def diagnostics(self, raise_on_nan: bool = True):
        out = (C.c_double * (PI_NDIAG * self.n))()
        st = lib().pi_batch_diagnostics(self._h, out, self._stream())
        if st != PI_OK and (raise_on_nan or st != PI_ENAN):
            check(st)
        keys = ("n_ion", "v_ion", "r_ion", "photo_rate", "recomb_rate", "nonfinite", "octants", "t")
        return [dict(zip(keys, list(out)[i * PI_NDIAG:(i + 1) * PI_NDIAG])) for i in range(self.n)]

    def work_counters(self, reset: bool = False):
        out = (C.c_int64 * PI_NWORK)()
        check(lib().pi_batch_work_counters(self._h, out, int(reset), self._stream()))
        return {"accepted": out[0], "rejected": out[1], "fallbacks": out[2], "newton": out[3],
                "resolved_fp64": out[4]}

    def run(self, max_steps: int = 10**8, check_every: int = 32):
        """Step until every grid is at its t_end; returns the steps launched."""
        launched = 0
        while launched < max_steps:
            for _ in range(min(check_every, max_steps - launched)):
                self.step_o2()
                launched += 1
            t, _, _ = self.state()
            if all(ti >= te for ti, te in zip(t, self._t_end)):
                break
        return launched

    def close(self):
        if getattr(self, "_h", None):
            check(lib().pi_batch_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Served form: a worker thread in the library admits submitted grids into
    a device-memory arena and advances the running ones together.  Inputs and
    results are host arrays (copied by the library)."""

    def __init__(self, precision: str = "mixed", hbm_budget: int = 0, max_active: int = 64,
                 steps_per_tick: int = 4):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the photoionisation library needs a GPU (no CPU fallback)")
        torch.cuda.init()
        self.precision = precision
        d = ServerDesc(hbm_budget, max_active, PRECISIONS[precision],
                       steps_per_tick)
        h = C.c_void_p()
        check(lib().pi_server_create(C.byref(d), C.byref(h)))
        self._h = h
        self._specs = {}

    def submit(self, spec, nH=None, x0=None, T0: Optional[float] = None,
               t_end: Optional[float] = None, checkpoint: Optional[bytes] = None) -> int:
        """Queue a request; ``checkpoint`` (from Grid.save or Server.checkpoint)
        resumes a saved state instead of starting from nH, x0, T0."""
        import numpy as np
        dp = C.POINTER(C.c_double)
        nHp = x0p = None
        if checkpoint is None:
            nH = np.ascontiguousarray(nH, dtype=np.float64).reshape(-1)
            nHp = nH.ctypes.data_as(dp)
            x0a = None if x0 is None else np.ascontiguousarray(x0, dtype=np.float64).reshape(-1)
            x0p = None if x0a is None else x0a.ctypes.data_as(dp)
        ck = None if checkpoint is None else C.create_string_buffer(bytes(checkpoint), len(checkpoint))
        r = Request(desc_from_spec(spec, self.precision), nHp, x0p,
                    float(T0 if T0 is not None else spec.T0),
                    float(t_end if t_end is not None else spec.t_end),
                    C.cast(ck, C.c_void_p) if ck is not None else None,
                    0 if checkpoint is None else len(checkpoint))
        t = C.c_uint64()
        check(lib().pi_submit(self._h, C.byref(r), C.byref(t)))
        self._specs[t.value] = spec
        return t.value

    def checkpoint(self, ticket: int):
        """pi_checkpoint of a running request: bytes, or None while it is queued."""
        need = C.c_size_t()
        check(lib().pi_checkpoint(self._h, ticket, None, 0, C.byref(need)))
        buf = C.create_string_buffer(need.value)
        st = lib().pi_checkpoint(self._h, ticket, buf, need.value, None)
        if st == PI_PENDING:
            return None
        check(st)
        return buf.raw

    def poll(self, ticket: int):
        """(status, info, x, T): x and T are arrays of the grid's shape once
        status is PI_OK, else None."""
        import numpy as np
        spec = self._specs[ticket]
        res = Result()
        x = np.empty(spec.ncells)
        T = np.empty(spec.ncells)
        dp = C.POINTER(C.c_double)
        st = lib().pi_poll(self._h, ticket, C.byref(res), x.ctypes.data_as(dp), T.ctypes.data_as(dp))
        info = {"t": res.t, "nsteps": res.nsteps, "latency_s": res.latency_s, "queue_s": res.queue_s}
        if st == PI_PENDING:
            return st, info, None, None
        del self._specs[ticket]
        if st != PI_OK:
            info["error"] = lib().pi_last_error().decode()
            return st, info, None, None
        return st, info, x.reshape(spec.shape), T.reshape(spec.shape)

    def cancel(self, ticket: int):
        check(lib().pi_cancel(self._h, ticket))

    def stats(self):
        out = (C.c_double * 8)()
        check(lib().pi_server_stats(self._h, out))
        keys = ("completed", "cell_updates", "busy_s", "steps", "running", "queued", "arena_bytes",
                "rebuilds")
        return dict(zip(keys, list(out)))

    def close(self):
        if getattr(self, "_h", None):
            check(lib().pi_server_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
