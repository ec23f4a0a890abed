"""Seeded synthetic inputs shared by the tests, the bench and the smoke check.

This module only draws inputs and states problem set-ups (grid shape, source
vertex, cell size, luminosity, densities); it performs none of the method's
arithmetic, so the HIP path and the FP64 oracle can both be fed from it.

The workloads follow the set-ups of the paper (uniform static media around a
point source, Sect. 3.2; a blackbody source, Sect. 4) plus a clumpy medium: a
lognormal density built from a Gaussian random field with a Kolmogorov-like
power spectrum P(k) ~ k^-11/3.  No public data set is used or reproduced.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import Optional

import numpy as np

PC = 3.0857e18          # parsec [cm]
SIGMA0 = 6.3e-18        # threshold cross-section used by the paper [cm^2]
ALPHA_B_1E4 = 2.59e-13  # case-B recombination coefficient at 1e4 K [cm^3/s]
INF = math.inf

# Table 1 of the paper: (K1, K2, K3, K4) of the explicit algorithms, dt00..dt12.
EXPLICIT_CRITERIA = {
    "dt00": (INF, INF, INF, 1.0), "dt01": (INF, INF, INF, 0.5), "dt02": (INF, INF, INF, 0.25),
    "dt03": (INF, INF, INF, 0.125), "dt04": (INF, INF, INF, 0.0625),
    "dt05": (INF, 0.5, INF, 0.5), "dt06": (INF, 0.25, INF, 0.25), "dt07": (INF, 0.125, INF, 0.125),
    "dt08": (INF, 0.0625, INF, 0.0625),
    "dt09": (INF, 0.5, 0.5, INF), "dt10": (INF, 0.25, 0.25, INF), "dt11": (INF, 0.125, 0.125, INF),
    "dt12": (INF, 0.0625, 0.0625, INF),
}


def stromgren_radius(Q: float, nH: float, alpha: float = ALPHA_B_1E4) -> float:
    """Radius of the ionised sphere that balances Q against recombinations."""
    return (3.0 * Q / (4.0 * math.pi * alpha * nH * nH)) ** (1.0 / 3.0)


def recombination_time(nH: float, alpha: float = ALPHA_B_1E4) -> float:
    return 1.0 / (alpha * nH)


@dataclass
class GridSpec:
    """One photoionisation problem on a uniform Cartesian grid (CGS)."""
    name: str
    n: tuple                      # (nx, ny, nz)
    src: tuple                    # source vertex, 0..n[d] (point source)
    dx: float                     # cell size [cm]
    Q: float                      # ionising photons / s (point); photons / cm^2 / s (plane)
    nH_mean: float                # mean hydrogen density [cm^-3]
    density: str = "uniform"      # "uniform" | "lognormal"
    sigma_ln: float = 1.0
    seed: int = 0
    spectrum: str = "mono"        # "mono" | "table"
    T_bb: float = 1e5             # blackbody temperature of the table source [K]
    e_excess: float = 0.0         # mono: heating per photoionisation [erg]
    thermal: str = "fixed"        # "fixed" | "evolve"
    T_fixed: float = 1e4
    T0: float = 50.0              # initial temperature when thermal == "evolve"
    recomb: str = "const"         # "const" | "power"
    alpha_B: float = ALPHA_B_1E4
    collisional: bool = False
    cooling: bool = True
    weights: str = "mellema"      # "mellema" | "geometric"
    source_cell_rule: bool = True
    n_sub: int = 2
    K: tuple = EXPLICIT_CRITERIA["dt02"]
    t_end: float = 0.0            # [s]
    t_rec: float = 0.0            # reference recombination time [s]
    precision: str = "fp64"       # "fp64" | "fp32" | "mixed"
    source: str = "point"         # "point" (at vertex src) | "plane" (from x = -inf)
    more_sources: tuple = ()      # further point sources: ((i, j, k), Q) each

    @property
    def ncells(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])

    @property
    def shape(self) -> tuple:
        """Array shape (nz, ny, nx): x varies fastest in memory."""
        return (self.n[2], self.n[1], self.n[0])

    def with_(self, **kw) -> "GridSpec":
        return replace(self, **kw)


def lognormal_density(shape, mean: float, sigma_ln: float, seed: int,
                      spectral_index: float = -11.0 / 3.0) -> np.ndarray:
    """n = mean-normalised exp(sigma g - sigma^2/2), g a unit-variance Gaussian
    random field with power spectrum P(k) ~ k^spectral_index (k=0 removed),
    drawn from numpy's default_rng(seed).  Returns float64 in shape order."""
    rng = np.random.default_rng(seed)
    white = rng.standard_normal(shape)
    F = np.fft.rfftn(white)
    kz = np.fft.fftfreq(shape[0])[:, None, None]
    ky = np.fft.fftfreq(shape[1])[None, :, None]
    kx = np.fft.rfftfreq(shape[2])[None, None, :]
    k = np.sqrt(kx * kx + ky * ky + kz * kz)
    k[0, 0, 0] = 1.0
    filt = k ** (spectral_index / 2.0)
    filt[0, 0, 0] = 0.0
    g = np.fft.irfftn(F * filt, s=shape, axes=(0, 1, 2))
    g = (g - g.mean()) / g.std()
    n = np.exp(sigma_ln * g - 0.5 * sigma_ln * sigma_ln)
    return n * (mean / n.mean())


def density(spec: GridSpec) -> np.ndarray:
    if spec.density == "uniform":
        return np.full(spec.shape, float(spec.nH_mean))
    if spec.density == "lognormal":
        return lognormal_density(spec.shape, spec.nH_mean, spec.sigma_ln, spec.seed)
    raise ValueError(spec.density)


def cfg1(**kw) -> GridSpec:
    """32^3, n_H = 1, monochromatic 13.6 eV source of 1e48 /s on the corner
    vertex, T fixed at 1e4 K, collisions off, box 1.2 R_S, dt02, to 4 t_rec."""
    Q, nH = 1e48, 1.0
    RS = stromgren_radius(Q, nH)
    tr = recombination_time(nH)
    s = GridSpec(name="cfg1", n=(32, 32, 32), src=(0, 0, 0), dx=1.2 * RS / 32, Q=Q, nH_mean=nH,
                 t_end=4.0 * tr, t_rec=tr)
    return s.with_(**kw) if kw else s


def cfg2(n: int = 128, **kw) -> GridSpec:
    """128^3 uniform n_H = 10 around a centre vertex, 1e5 K blackbody source of
    1e48 /s with rates tabulated against optical depth (64 nodes), temperature
    evolved from 50 K with heating and cooling, box 2.4 R_S(1e4 K), to 1 t_rec."""
    Q, nH = 1e48, 10.0
    RS = stromgren_radius(Q, nH)
    tr = recombination_time(nH)
    dx = 2.4 * RS / 128
    s = GridSpec(name="cfg2", n=(n, n, n), src=(n // 2, n // 2, n // 2), dx=dx, Q=Q, nH_mean=nH,
                 spectrum="table", thermal="evolve", recomb="power", collisional=True,
                 t_end=1.0 * tr, t_rec=tr)
    return s.with_(**kw) if kw else s


def cfg3(n: int = 256, box_cells: int = 256, **kw) -> GridSpec:
    """256^3 clumpy medium: lognormal density (sigma_ln 1, spectrum k^-11/3,
    seed 1201), mean n_H = 5, central 1e5 K blackbody source of 5e48 /s, cfg2
    physics, box 2.4 R_S(mean), FP32 bulk with FP64 front cells.  The cell
    size is that of box_cells cells across 2.4 R_S: n < box_cells gives the
    central part of the same medium, box_cells = n the whole box coarser."""
    Q, nH = 5e48, 5.0
    RS = stromgren_radius(Q, nH)
    tr = recombination_time(nH)
    dx = 2.4 * RS / box_cells
    s = GridSpec(name="cfg3", n=(n, n, n), src=(n // 2, n // 2, n // 2), dx=dx, Q=Q, nH_mean=nH,
                 density="lognormal", sigma_ln=1.0, seed=1201, spectrum="table",
                 thermal="evolve", recomb="power", collisional=True, t_end=0.3 * tr,
                 t_rec=tr, precision="mixed")
    return s.with_(**kw) if kw else s


def plane(n=(100, 16, 16), density: str = "uniform", **kw) -> GridSpec:
    """Plane-parallel source at x = -infinity (Sect. 3.1's slab test on a 3D
    grid): monochromatic flux 1e9 photons/cm^2/s into n_H = 100 over 0.51 pc
    along x (cell optical depth ~10 at 100 cells), T fixed at 1e4 K, no
    recombinations or collisions, dt02; with a lognormal density (sigma_ln 1,
    seed 5) the rows differ and the front is corrugated.  The ions per unit
    area equal F t for a perfect integration; t_end is when they would fill
    the grid."""
    L, nH, F = 0.51 * PC, 100.0, 1e9
    dx = L / n[0]
    t_fill = L * nH / F
    s = GridSpec(name="plane", n=tuple(n), src=(0, 0, 0), dx=dx, Q=F, nH_mean=nH,
                 density=density, sigma_ln=1.0, seed=5, alpha_B=0.0, source="plane",
                 t_end=0.8 * t_fill, t_rec=t_fill)
    return s.with_(**kw) if kw else s


HARDENING_DTAU0 = (1.0, 3.0, 10.0, 30.0)
HARDENING_NH = (10.0, 100.0, 1000.0)


def hardening(dtau0: float, nH: float = 100.0, tau_S: float = 150.0, **kw) -> GridSpec:
    """Spectral-hardening set-up of Sect. 4: a 37 500 K blackbody source in a
    uniform medium, temperature evolved from 50 K with a temperature-dependent
    recombination rate, resolved with cell optical depth dtau0 = n_H sigma0 dx
    at threshold.

    The 3D grid is one octant around a corner source, of side 1.37 R_S (the
    paper's 1D grid spans 1.94 pc for R_S = 1.42 pc).  The optical depth of
    R_S at threshold, tau_S = n_H sigma0 R_S, is held at tau_S (the paper's 1D
    problem has ~2800, which no 3D grid resolves at dtau0 = 1), so the grid
    has about 1.37 tau_S / dtau0 cells a side.  Changing n_H at fixed tau_S
    and dtau0 scales R_S and t_rec both as 1/n_H (Q as 1/n_H), so the front
    expands at the same speed for every density, as the paper arranges."""
    RS = tau_S / (nH * SIGMA0)
    Q = 4.0 * math.pi / 3.0 * ALPHA_B_1E4 * nH * nH * RS ** 3
    tr = recombination_time(nH)
    dx = dtau0 / (nH * SIGMA0)
    n = int(math.ceil(1.37 * RS / dx))
    s = GridSpec(name=f"hard_dtau{dtau0:g}_n{nH:g}", n=(n, n, n), src=(0, 0, 0), dx=dx, Q=Q,
                 nH_mean=nH, spectrum="table", T_bb=37500.0, thermal="evolve", recomb="power",
                 collisional=True, t_end=2.0 * tr, t_rec=tr)
    return s.with_(**kw) if kw else s


def hardening_specs(precision: str = "mixed", dtau0s=HARDENING_DTAU0, nHs=HARDENING_NH) -> list:
    """The grid of Sect. 4: every cell optical depth with every density."""
    return [hardening(d, nH, precision=precision) for d in dtau0s for nH in nHs]


def batch_specs(count: int = 64, seed: int = 0, nmin: int = 32, nmax: int = 160,
                precision: str = "mixed") -> list:
    """Independent grids for the batched form: n ~ U{nmin..nmax}, uniform or
    lognormal density (p = 1/2) with mean log-uniform in [1, 100], Q
    log-uniform in [1e47, 1e50], centre-vertex source, box 2.4 R_S(Q, mean),
    cfg2 physics, each run to 1 t_rec."""
    out = []
    for i in range(count):
        rng = np.random.default_rng(seed * 100003 + i)
        n = int(rng.integers(nmin, nmax + 1))
        mean = float(10 ** rng.uniform(0.0, 2.0))
        Q = float(10 ** rng.uniform(47.0, 50.0))
        lognormal = bool(rng.random() < 0.5)
        RS = stromgren_radius(Q, mean)
        tr = recombination_time(mean)
        out.append(GridSpec(name=f"batch{i}", n=(n, n, n), src=(n // 2, n // 2, n // 2),
                            dx=2.4 * RS / n, Q=Q, nH_mean=mean,
                            density="lognormal" if lognormal else "uniform",
                            seed=int(rng.integers(0, 2**31 - 1)), spectrum="table",
                            thermal="evolve", recomb="power", collisional=True,
                            t_end=1.0 * tr, t_rec=tr, precision=precision))
    return out


def poisson_requests(count: int, rate: float = 20.0, seed: int = 5651, nmin: int = 48,
                     nmax: int = 256, n_outlier: int = 512, p_outlier: float = 0.01,
                     precision: str = "mixed") -> list:
    """Request stream for the served form: exponential inter-arrival times of
    mean 1/rate, n ~ U{nmin..nmax} (n_outlier with probability p_outlier),
    source vertex uniform in the central half of the box, densities and Q as in
    batch_specs, each run to 2 t_rec(mean).  Returns (arrival_time, GridSpec)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(count):
        t += float(rng.exponential(1.0 / rate))
        n = n_outlier if rng.random() < p_outlier else int(rng.integers(nmin, nmax + 1))
        mean = float(10 ** rng.uniform(0.0, 2.0))
        Q = float(10 ** rng.uniform(47.0, 50.0))
        lognormal = bool(rng.random() < 0.5)
        src = tuple(int(rng.integers(n // 4, 3 * n // 4 + 1)) for _ in range(3))
        RS = stromgren_radius(Q, mean)
        tr = recombination_time(mean)
        out.append((t, GridSpec(name=f"req{i}", n=(n, n, n), src=src, dx=2.4 * RS / n, Q=Q,
                                nH_mean=mean, density="lognormal" if lognormal else "uniform",
                                seed=int(rng.integers(0, 2**31 - 1)), spectrum="table",
                                thermal="evolve", recomb="power", collisional=True,
                                t_end=2.0 * tr, t_rec=tr, precision=precision)))
    return out


def ionised_sphere(spec: GridSpec, radius_cells: float, width_cells: float = 1.5,
                   x_in: float = 1e-4, T_in: float = 1e4):
    """A partly ionised start: neutral fraction x_in inside a sphere of the
    given radius (in cells) around the source vertex, 1 outside, joined by a
    tanh profile of the given width; temperature T_in inside, spec.T0
    outside, on the same profile.  Returns (x, T) in shape order.  Input
    generation only (a profile, not a solution of the method)."""
    k, j, i = np.meshgrid(*(np.arange(m) + 0.5 for m in spec.shape), indexing="ij")
    sx, sy, sz = spec.src
    r = np.sqrt((i - sx) ** 2 + (j - sy) ** 2 + (k - sz) ** 2)
    inside = 0.5 * (1.0 - np.tanh((r - radius_cells) / width_cells))
    x = x_in + (1.0 - x_in) * (1.0 - inside)
    T = spec.T0 + (T_in - spec.T0) * inside
    return x, T


def random_cell_states(count: int, seed: int, thermal: bool = True):
    """Random but physical per-cell states for micro-physics parity: density,
    neutral fraction (log-uniform down to 1e-7), temperature, entering optical
    depth and the chord/geometry of a cell 1-60 cells from the source.
    Returns a dict of float64 arrays (temperatures in K, not energies)."""
    rng = np.random.default_rng(seed)
    nH = 10 ** rng.uniform(-1.0, 3.0, count)
    x = 10 ** rng.uniform(-7.0, 0.0, count)
    x[rng.random(count) < 0.1] = 1.0
    T = 10 ** rng.uniform(1.5, 4.6, count) if thermal else np.full(count, 1e4)
    tau = np.where(rng.random(count) < 0.2, 0.0, 10 ** rng.uniform(-5.0, 3.0, count))
    return {"nH": nH, "x": x, "T": T, "tau": tau}
