"""Seeded synthetic initial fields (rho, ux, uy, T) for the runs.

This module holds inputs only, none of the scheme's arithmetic: it is shared by the library's
users, the tests and the oracle side, which each turn these FP64 host arrays into populations
with their own equilibrium.  Fields are row-major ``[Ny][Nx]`` float64 on the full grid (bulk
plus PML); node (x, y) sits at continuous coordinate (x, y).  Velocities and temperatures are
in thermal units (sound-speed unit c_s = 1), so a Mach number Ma gives |u0| = Ma.

Random numbers come from SplitMix64 (Steele, Lea and Flood, OOPSLA 2014), mapped to doubles in
[0, 1) from the top 53 bits.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, n: int) -> np.ndarray:
    """The first n outputs of SplitMix64 started from ``seed`` (uint64)."""
    with np.errstate(over="ignore"):
        k = np.arange(1, n + 1, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + k * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform(seed: int, n: int) -> np.ndarray:
    """n doubles in [0, 1) from SplitMix64."""
    return (splitmix64(seed, n) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


@dataclass
class Fields:
    rho: np.ndarray
    ux: np.ndarray
    uy: np.ndarray
    T: np.ndarray

    def as_tuple(self):
        return self.rho, self.ux, self.uy, self.T


def uniform_state(Nx, Ny, rho0=1.0, ux0=0.0, uy0=0.0, T0=1.0) -> Fields:
    shape = (Ny, Nx)
    return Fields(np.full(shape, float(rho0)), np.full(shape, float(ux0)),
                  np.full(shape, float(uy0)), np.full(shape, float(T0)))


def _grid(Nx, Ny):
    y, x = np.mgrid[0:Ny, 0:Nx].astype(np.float64)
    return x, y


def add_gaussian_pulse(F: Fields, xc, yc, amplitude, half_width) -> Fields:
    """Density-only pulse rho += A * 2^(-|x-xc|^2 / b^2), b the half-width at half maximum.
    Evaluated in a window of radius 8b + 2 around the centre: beyond it the term is below
    |A| 2^-64, which leaves any density near 1 unchanged in float64 (|A| <= 1e-2 here)."""
    Ny, Nx = F.rho.shape
    rw = 8.0 * half_width + 2.0
    x0, x1 = max(0, int(np.floor(xc - rw))), min(Nx, int(np.ceil(xc + rw)) + 1)
    y0, y1 = max(0, int(np.floor(yc - rw))), min(Ny, int(np.ceil(yc + rw)) + 1)
    if x0 >= x1 or y0 >= y1:
        return F
    y, x = np.mgrid[y0:y1, x0:x1].astype(np.float64)
    rho = F.rho.copy()
    rho[y0:y1, x0:x1] += amplitude * np.power(2.0, -((x - xc) ** 2 + (y - yc) ** 2) / half_width ** 2)
    F.rho = rho
    return F


def add_isentropic_vortex(F: Fields, xc, yc, strength, radius, rho0=1.0, T0=1.0) -> Fields:
    """Isentropic vortex of swirl peak ``strength`` (thermal units) at distance ``radius``:
    u_theta = eps (d/R) exp((1 - d^2/R^2)/2), T = T0 - (eps^2/4) exp(1 - d^2/R^2) (gamma = 2),
    rho scaled by T/T0 (isentropic for gamma = 2 gives rho ~ T)."""
    Ny, Nx = F.rho.shape
    x, y = _grid(Nx, Ny)
    dx, dy = x - xc, y - yc
    q = (dx * dx + dy * dy) / (radius * radius)
    amp = strength / radius * np.exp(0.5 * (1.0 - q))
    F.ux = F.ux - amp * dy
    F.uy = F.uy + amp * dx
    dT = -(strength ** 2 / 4.0) * np.exp(1.0 - q)
    F.T = F.T + dT
    F.rho = F.rho * (1.0 + dT / T0)
    return F


def add_noise(F: Fields, seed: int, amp_rho=1e-3, amp_u=1e-3, amp_T=1e-3) -> Fields:
    """Independent uniform node noise in [-amp, amp] on each field (parity inputs that make
    every node and every code path distinct)."""
    Ny, Nx = F.rho.shape
    n = Nx * Ny
    r = uniform(seed, 4 * n).reshape(4, Ny, Nx) * 2.0 - 1.0
    F.rho = F.rho + amp_rho * r[0]
    F.ux = F.ux + amp_u * r[1]
    F.uy = F.uy + amp_u * r[2]
    F.T = F.T + amp_T * r[3]
    return F


# ------------------------------------------------------------------------------------------
# Named workloads.  Each returns a dict with the run description and the initial fields.
# ------------------------------------------------------------------------------------------

@dataclass
class RunSpec:
    Lx: int
    Ly: int
    W: int
    sigma_max: float
    bc: str            # "zg" | "nrbc" | "periodic"
    tau: float = 0.8
    rho0: float = 1.0
    ux0: float = 0.0
    uy0: float = 0.0
    T0: float = 1.0
    steps: int = 0
    fields: Fields | None = field(default=None, repr=False)
    lattice: int = 37  # velocity stencil: 37 (D2Q37) or 17 (D2Q17)

    @property
    def Nx(self):
        return self.Lx + 2 * self.W

    @property
    def Ny(self):
        return self.Ly + 2 * self.W


def pulse_box(L=64, W=8, sigma_max=0.1, steps=200, bc="zg") -> RunSpec:
    """Plain method: L^2 bulk + W-cell PML each side, fluid at rest, Gaussian density pulse
    A = 1e-3, half-width 4 cells at the grid centre."""
    spec = RunSpec(L, L, W, sigma_max, bc, steps=steps)
    F = uniform_state(spec.Nx, spec.Ny)
    c = 0.5 * (spec.Nx - 1)
    spec.fields = add_gaussian_pulse(F, c, c, 1e-3, 4.0)
    return spec


def vortex_pulse(L=1024, W=32, sigma_max=0.1, mach=0.1, steps=10000, bc="nrbc", seed=2,
                 strength=0.05, radius=16.0) -> RunSpec:
    """L^2 bulk + W-cell PML, mean flow Mach ``mach`` in +x, isentropic vortex (strength 0.05,
    radius 16 cells) at the bulk centre plus a Gaussian pulse A = 1e-3, b = 4 whose centre is
    drawn uniformly in the central quarter of the bulk."""
    spec = RunSpec(L, L, W, sigma_max, bc, ux0=mach, steps=steps)
    F = uniform_state(spec.Nx, spec.Ny, 1.0, mach, 0.0, 1.0)
    c = 0.5 * (spec.Nx - 1)
    add_isentropic_vortex(F, c, c, strength, radius)
    u = uniform(seed, 2)
    px = W + L * (0.25 + 0.5 * u[0])
    py = W + L * (0.25 + 0.5 * u[1])
    spec.fields = add_gaussian_pulse(F, px, py, 1e-3, 4.0)
    return spec


def multi_pulse(L=4096, W=64, sigma_max=0.1, mach=0.05, steps=2000, bc="zg", seed=3,
                npulse=8) -> RunSpec:
    """L^2 bulk + W-cell PML, mean flow Mach ``mach``, ``npulse`` Gaussian pulses (b = 4) with
    amplitudes uniform in [1e-4, 1e-3] at seeded centres at least 16 cells inside the bulk."""
    spec = RunSpec(L, L, W, sigma_max, bc, ux0=mach, steps=steps)
    F = uniform_state(spec.Nx, spec.Ny, 1.0, mach, 0.0, 1.0)
    u = uniform(seed, 3 * npulse).reshape(npulse, 3)
    for k in range(npulse):
        px = W + 16 + (L - 32) * u[k, 0]
        py = W + 16 + (L - 32) * u[k, 1]
        amp = 1e-4 + 9e-4 * u[k, 2]
        add_gaussian_pulse(F, px, py, amp, 4.0)
    spec.fields = F
    return spec


def noisy_state(Nx, Ny, seed, rho0=1.0, ux0=0.0, uy0=0.0, T0=1.0, amp=1e-3) -> Fields:
    return add_noise(uniform_state(Nx, Ny, rho0, ux0, uy0, T0), seed, amp, amp, amp)


def batch_sweep(nruns=256, seed=4, steps=5000, sigma_max=0.1):
    """Uneven batch: bulk L in {128,256,512,1024}, PML W in {0,4,8,16,32}, boundary in {ZG, NRBC},
    initial data as ``vortex_pulse`` (Mach 0.1 mean flow, vortex + seeded pulse)."""
    specs = []
    for k in range(nruns):
        u = uniform(seed + k, 3)
        L = (128, 256, 512, 1024)[int(u[0] * 4)]
        W = (0, 4, 8, 16, 32)[int(u[1] * 5)]
        bc = ("zg", "nrbc")[int(u[2] * 2)]
        specs.append(vortex_pulse(L=L, W=W, sigma_max=sigma_max, mach=0.1, steps=steps, bc=bc,
                                  seed=seed + 1000 + k))
    return specs


def poisson_trace(n_jobs, rate=20.0, seed=5, L_min=128, L_max=2048, W_min=8, W_max=64,
                  steps_min=1000, steps_max=20000):
    """Serving trace: arrival times of a Poisson process (rate jobs/s), bulk side log-uniform in
    [L_min, L_max], PML W uniform in [W_min, W_max], steps uniform in [steps_min, steps_max],
    boundary uniform in {ZG, NRBC}.  Returns a list of (arrival_s, dict) without fields; fields
    are produced on admission by ``vortex_pulse`` with the job's seed."""
    u = uniform(seed, 5 * n_jobs).reshape(n_jobs, 5)
    t = np.cumsum(-np.log1p(-u[:, 0]) / rate)
    jobs = []
    for k in range(n_jobs):
        L = int(round(math.exp(math.log(L_min) + (math.log(L_max) - math.log(L_min)) * u[k, 1])))
        W = W_min + int(u[k, 2] * (W_max - W_min + 1))
        steps = steps_min + int(u[k, 3] * (steps_max - steps_min + 1))
        bc = ("zg", "nrbc")[int(u[k, 4] * 2)]
        jobs.append((float(t[k]), dict(L=L, W=W, steps=steps, bc=bc, seed=seed * 100000 + k)))
    return jobs
