"""Seeded synthetic workloads for the length-gauge hydrogen TDSE.

This module only describes inputs: grid shapes, pulse parameters in atomic
units, time steps and seeded random numbers.  It holds none of the method's
arithmetic and is the only code shared by the oracle side (tests, CPU
baseline) and the GPU side (tests, benchmark).

Unit conversions (laser intensity and wavelength to atomic units) use the
standard constants: the atomic unit of intensity 3.50944758e16 W/cm^2 and
hbar*c = 45.5633525 au*nm (omega = 45.5633525 / lambda[nm]).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import Optional

import numpy as np

AU_INTENSITY_W_CM2 = 3.50944758e16
AU_OMEGA_NM = 45.5633525
SINE_CARRIER_CEP = -math.pi / 2.0   # cos(w t - pi/2) = sin(w t)


def e0_from_intensity(intensity_w_cm2: float) -> float:
    return math.sqrt(intensity_w_cm2 / AU_INTENSITY_W_CM2)


def omega_from_wavelength(nm: float) -> float:
    return AU_OMEGA_NM / nm


@dataclass(frozen=True)
class PulseSpec:
    e0: float
    omega: float
    n_cycles: float
    cep: float = SINE_CARRIER_CEP
    t_on: float = 0.0

    @property
    def duration(self) -> float:
        return 2.0 * math.pi * self.n_cycles / self.omega


@dataclass(frozen=True)
class Workload:
    name: str
    n: int
    lmax: int
    dr: float
    stencil: int
    precision: str            # "fp64" or "fp32"
    method: str               # "taylor", "rk4", "lanczos"
    order: int                # Taylor order or Krylov dimension
    pulse: PulseSpec
    dt: float                 # step used (stable for explicit methods)
    dt_nominal: float         # step named in the workload description
    nsteps: int               # steps in the run or window
    obs_every: int
    r_ion: float
    z: float = 1.0
    t0: float = 0.0
    description: str = ""

    @property
    def unknowns(self) -> int:
        return (self.lmax + 1) * self.n

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)


def _cfg2_pulse() -> PulseSpec:
    return PulseSpec(e0_from_intensity(1e14), omega_from_wavelength(800.0), 4.0)


WORKLOADS = {
    # plain FP64, N=2000, dr=0.1, lmax=8, 3-point; E0 = 0.0534, w = 0.057, 2 cycles
    "hydrogen_n2000_l8_fp64": Workload(
        "hydrogen_n2000_l8_fp64", 2000, 8, 0.1, 3, "fp64", "rk4", 4,
        PulseSpec(0.0534, 0.057, 2.0), dt=5e-4, dt_nominal=0.05, nsteps=440_000,
        obs_every=100, r_ion=50.0,
        description="FP64 RK4/Taylor-4, 2-cycle sin^2 pulse, 1e14 W/cm^2, w=0.057"),
    # the same grid and pulse with the Taylor polynomial of order 4 (the same
    # stability region as RK4), one fused strip launch per step
    "hydrogen_n2000_l8_fp64_taylor4": Workload(
        "hydrogen_n2000_l8_fp64_taylor4", 2000, 8, 0.1, 3, "fp64", "taylor", 4,
        PulseSpec(0.0534, 0.057, 2.0), dt=5e-4, dt_nominal=0.05, nsteps=440_000,
        obs_every=100, r_ion=50.0,
        description="FP64 Taylor-4, 2-cycle sin^2 pulse, 1e14 W/cm^2, w=0.057"),
    # single large FP64 instance, Taylor order 8, 5-point
    "hydrogen_n20000_l64_fp64_taylor8": Workload(
        "hydrogen_n20000_l64_fp64_taylor8", 20000, 64, 0.05, 5, "fp64", "taylor", 8,
        _cfg2_pulse(), dt=3e-6, dt_nominal=0.01, nsteps=2000, obs_every=1, r_ion=50.0,
        description="FP64 Taylor-8, 4-cycle 800 nm 1e14 W/cm^2 sin^2 pulse"),
    # Lanczos m = 20 on the same grid, FP32 state with FP64 reductions
    "hydrogen_n20000_l64_fp32_lanczos20": Workload(
        "hydrogen_n20000_l64_fp32_lanczos20", 20000, 64, 0.05, 5, "fp32", "lanczos", 20,
        _cfg2_pulse(), dt=0.01, dt_nominal=0.01, nsteps=44_128, obs_every=1, r_ion=50.0,
        description="FP32-mixed Lanczos m=20, 4-cycle 800 nm 1e14 W/cm^2"),
    # long-wavelength stress test
    "hydrogen_n100000_l256_fp32_taylor8": Workload(
        "hydrogen_n100000_l256_fp32_taylor8", 100_000, 256, 0.05, 3, "fp32", "taylor", 8,
        PulseSpec(e0_from_intensity(2e14), omega_from_wavelength(1600.0), 3.0),
        dt=2e-7, dt_nominal=float("nan"), nsteps=200, obs_every=1, r_ion=50.0,
        description="FP32-mixed Taylor-8, 3-cycle 1600 nm 2e14 W/cm^2, 25.7M unknowns"),
}


# --------------------------------------------------------------------------
# batch of independent pulses on uneven grids
# --------------------------------------------------------------------------

BATCH_SEED = 13081856


@dataclass(frozen=True)
class BatchMember:
    n: int
    lmax: int
    intensity: float
    wavelength_nm: float
    n_cycles: int

    @property
    def pulse(self) -> PulseSpec:
        return PulseSpec(e0_from_intensity(self.intensity),
                         omega_from_wavelength(self.wavelength_nm), float(self.n_cycles))


def batch_members(count: int = 256, seed: int = BATCH_SEED):
    """Per member, drawn in this order from numpy's PCG64 default_rng(seed):
    log10 I ~ U[13, log10 5e14], lambda ~ U[400, 1600] nm, n_c ~ U{2..6},
    N ~ U{4000..16000}, lmax ~ U{16..64}."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        log_i = rng.uniform(13.0, math.log10(5e14))
        lam = rng.uniform(400.0, 1600.0)
        nc = int(rng.integers(2, 6, endpoint=True))
        n = int(rng.integers(4000, 16000, endpoint=True))
        lmax = int(rng.integers(16, 64, endpoint=True))
        out.append(BatchMember(n, lmax, 10.0 ** log_i, lam, nc))
    return out


BATCH_DR = 0.1
BATCH_STENCIL = 3
BATCH_ORDER = 8
BATCH_R_ION_FRACTION = 0.25      # r_b = 0.25 * R for each member
BATCH_DT_SAFETY = 0.8            # dt = 0.8 * y_8 / lambda_bound(member)


def random_state(seed: int, n: int, lmax: int, smooth: bool = False) -> np.ndarray:
    """Seeded complex128 test vector of shape [(lmax+1)*n] (unnormalised).
    smooth=True: per partial wave a random complex amplitude times
    sin^2(pi r/R) plus 0.1 times another random amplitude times sin(6 pi r/R)."""
    rng = np.random.default_rng(seed)
    if smooth:
        c = rng.standard_normal((lmax + 1, 4))
        a = (c[:, 0] + 1j * c[:, 1])[:, None]
        b = (c[:, 2] + 1j * c[:, 3])[:, None]
        r = np.arange(1, n + 1) / n
        v = a * (np.sin(np.pi * r) ** 2)[None, :] + 0.1 * b * np.sin(6 * np.pi * r)[None, :]
    else:
        v = rng.standard_normal((lmax + 1, n)) + 1j * rng.standard_normal((lmax + 1, n))
    return np.ascontiguousarray(v.reshape(-1))


def mixed_state(seed: int, n: int, lmax: int, dr: float) -> np.ndarray:
    """Seeded smooth complex128 state of shape [(lmax+1)*n] (unnormalised)
    that carries bound, excited and outgoing parts at once: hydrogen-like
    radial shapes r e^{-r} (l = 0), r^2 e^{-r/2} (l = 1) and r^3 e^{-r/3}
    (l = 2) with seeded complex amplitudes, plus 0.3 times a smooth seeded
    wave in every partial wave (random_state(seed, smooth=True), scaled to
    unit grid norm), whose sin^2 envelope over the box puts weight far out."""
    rng = np.random.default_rng(seed)
    c = rng.standard_normal((3, 2))
    amp = c[:, 0] + 1j * c[:, 1]
    r = (np.arange(n) + 1.0) * dr
    v = 0.3 * random_state(seed + 1, n, lmax, smooth=True)
    v /= math.sqrt(dr * float(np.vdot(v, v).real))
    shapes = (r * np.exp(-r), r ** 2 * np.exp(-r / 2.0), r ** 3 * np.exp(-r / 3.0))
    for l, (a, f) in enumerate(zip(amp, shapes)):
        if l <= lmax:
            v[l * n:(l + 1) * n] += a * f / math.sqrt(dr * float(np.dot(f, f)))
    return v


def outgoing_packet(seed: int, n: int, lmax: int, dr: float, r0: float = 20.0, sigma: float = 3.0,
                    k: float = 1.5) -> np.ndarray:
    """Seeded complex128 state of shape [(lmax+1)*n], normalised on the grid:
    a Gaussian packet exp(-(r - r0)^2 / (2 sigma^2)) moving outward with
    momentum k (au) in every partial wave, each wave with a seeded complex
    amplitude, plus the l = 0 bound-like shape r e^{-r} with weight 1/2, so
    the packet carries probability through a flux sphere beyond r0 into an
    absorber while part of the state stays near the origin."""
    rng = np.random.default_rng(seed)
    c = rng.standard_normal((lmax + 1, 2))
    r = (np.arange(n) + 1.0) * dr
    f = np.exp(-((r - r0) ** 2) / (2.0 * sigma ** 2)) * np.exp(1j * k * r)
    v = np.zeros((lmax + 1) * n, dtype=np.complex128)
    for l in range(lmax + 1):
        v[l * n:(l + 1) * n] = (c[l, 0] + 1j * c[l, 1]) * f
    v /= math.sqrt(dr * float(np.vdot(v, v).real))
    b = r * np.exp(-r)
    v[:n] += 0.5 * b / math.sqrt(dr * float(np.dot(b, b)))
    return v / math.sqrt(dr * float(np.vdot(v, v).real))
