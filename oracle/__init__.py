"""Plain FP64 CPU oracle for the finite-difference TDSE of arXiv:1308.1856.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package:
only ``tests/``, the smoke check and the benchmark's CPU-baseline leg do.  It
shares no code with the GPU library (``paper_1308_1856_amd``) and never imports
it.  The arithmetic lives in ``tdse_oracle.c`` (loops written out from the
paper's formulas, compiled with ``-ffp-contract=off``); this module marshals
numpy arrays into it and adds the bound eigenstates (``eigen.py``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tdse_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OBS_FIXED = 8
OBS_NAMES = ("t", "e_field", "norm", "p_g", "p_bound", "p_ion", "dipole", "accel")

TAYLOR, RK4, LANCZOS = 0, 1, 2
LENGTH, VELOCITY = 0, 1
SINE_SQR_E, SINE_SQR_A = 0, 1
RK_EULER, RK_CLASSIC4, RK_FEHLBERG45, RK_CASHKARP, RK_DORMANDPRINCE, RK_MERSON = range(6)
RK_MAX = 8


def build() -> str:
    """Compile the C oracle with gcc into oracle/liboracle.so."""
    cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-ffp-contract=off", "-fopenmp",
           "-Wall", "-Wextra", "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("lmax", ctypes.c_int32), ("stencil", ctypes.c_int32),
                ("gauge", ctypes.c_int32), ("dr", ctypes.c_double), ("z", ctypes.c_double),
                ("r_shift", ctypes.c_double)]


class _Pulse(ctypes.Structure):
    _fields_ = [("e0", ctypes.c_double), ("omega", ctypes.c_double), ("n_cycles", ctypes.c_double),
                ("cep", ctypes.c_double), ("t_on", ctypes.c_double), ("shape", ctypes.c_int32),
                ("pad_", ctypes.c_int32)]


@dataclass(frozen=True)
class Grid:
    n: int
    lmax: int
    dr: float
    stencil: int = 3
    z: float = 1.0
    r_shift: float = 0.0
    gauge: int = 0          # LENGTH or VELOCITY

    @property
    def size(self) -> int:
        return (self.lmax + 1) * self.n

    def c(self) -> _Grid:
        return _Grid(self.n, self.lmax, self.stencil, int(self.gauge), self.dr, self.z, self.r_shift)


@dataclass(frozen=True)
class Pulse:
    e0: float = 0.0
    omega: float = 1.0
    n_cycles: float = 1.0
    cep: float = 0.0
    t_on: float = 0.0
    shape: int = 0          # SINE_SQR_E or SINE_SQR_A

    def c(self) -> _Pulse:
        return _Pulse(self.e0, self.omega, self.n_cycles, self.cep, self.t_on, int(self.shape), 0)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        gp, pp = ctypes.POINTER(_Grid), ctypes.POINTER(_Pulse)
        L.orc_set_threads.argtypes, L.orc_set_threads.restype = [ctypes.c_int], None
        L.orc_max_threads.argtypes, L.orc_max_threads.restype = [], ctypes.c_int
        L.orc_radius.argtypes, L.orc_radius.restype = [gp, ctypes.c_int], ctypes.c_double
        L.orc_kappa.argtypes, L.orc_kappa.restype = [ctypes.c_int], ctypes.c_double
        L.orc_field.argtypes, L.orc_field.restype = [pp, ctypes.c_double], ctypes.c_double
        L.orc_apply_h.argtypes = [gp, ctypes.c_double, dp, dp]
        L.orc_vector_potential_step.argtypes = [pp, ctypes.c_double, ctypes.c_double]
        L.orc_vector_potential_step.restype = ctypes.c_double
        L.orc_vector_potential_at.argtypes = [pp, ctypes.c_double, ctypes.c_double]
        L.orc_vector_potential_at.restype = ctypes.c_double
        L.orc_radial_current_vel.argtypes = [gp, ctypes.c_int, ctypes.c_double, dp]
        L.orc_radial_current_vel.restype = ctypes.c_double
        L.orc_h_bound.argtypes, L.orc_h_bound.restype = [gp, ctypes.c_double], ctypes.c_double
        L.orc_taylor_step.argtypes = [gp, ctypes.c_double, ctypes.c_double, ctypes.c_int, dp]
        L.orc_rk4_step.argtypes = [gp, pp, ctypes.c_double, ctypes.c_double, dp]
        L.orc_lanczos_step.argtypes = [gp, ctypes.c_double, ctypes.c_double, ctypes.c_int, dp]
        L.orc_lanczos_step.restype = ctypes.c_int
        L.orc_jacobi_eig.argtypes = [ctypes.c_int, dp, dp]
        L.orc_rk_tableau.argtypes, L.orc_rk_tableau.restype = [ctypes.c_int, dp, dp, dp, dp], ctypes.c_int
        L.orc_rk_step.argtypes, L.orc_rk_step.restype = [gp, pp, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                                         dp], ctypes.c_double
        L.orc_propagate_rk.argtypes = [gp, pp, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int64,
                                       ctypes.c_int64, ctypes.c_double, dp, ctypes.c_int, ip, dp, dp, dp]
        L.orc_propagate_rk.restype = ctypes.c_double
        L.orc_mask.argtypes, L.orc_mask.restype = [ctypes.c_double, ctypes.c_double, ctypes.c_double], ctypes.c_double
        L.orc_apply_mask.argtypes = [gp, ctypes.c_double, ctypes.c_double, dp]
        L.orc_radial_current.argtypes, L.orc_radial_current.restype = [gp, ctypes.c_int, dp], ctypes.c_double
        L.orc_propagate_abs.argtypes = [gp, pp, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_int64, ctypes.c_int64, ctypes.c_double, dp, ctypes.c_int, ip, dp,
                                        ctypes.c_double, ctypes.c_double, ctypes.c_int, dp, dp, dp]
        L.orc_propagate_abs.restype = ctypes.c_int
        L.orc_imag_step.argtypes, L.orc_imag_step.restype = [gp, ctypes.c_double, ctypes.c_int, dp], ctypes.c_double
        L.orc_imag_propagate.argtypes = [gp, ctypes.c_double, ctypes.c_int, ctypes.c_int64, dp, dp]
        L.orc_initial_state.argtypes = [gp, dp, dp]
        L.orc_observables.argtypes = [gp, pp, ctypes.c_double, ctypes.c_double, dp, ctypes.c_int,
                                      ip, dp, dp, dp]
        L.orc_propagate.argtypes = [gp, pp, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_int64, ctypes.c_int64,
                                    ctypes.c_double, dp, ctypes.c_int, ip, dp, dp, dp]
        L.orc_propagate.restype = ctypes.c_int
        _lib = L
    return _lib


def set_threads(n: int) -> None:
    """OpenMP threads of the oracle's element-wise loops (results are
    bit-identical for every thread count)."""
    lib().orc_set_threads(int(n))


def max_threads() -> int:
    return int(lib().orc_max_threads())


def _dptr(a: np.ndarray):
    assert a.flags.c_contiguous and a.dtype in (np.float64, np.complex128)
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _iptr(a: np.ndarray):
    assert a.flags.c_contiguous and a.dtype == np.int32
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _state(g: Grid, psi) -> np.ndarray:
    psi = np.ascontiguousarray(psi, dtype=np.complex128).reshape(-1)
    if psi.size != g.size:
        raise ValueError(f"state has {psi.size} entries, grid needs {g.size}")
    return psi


def radius(g: Grid) -> np.ndarray:
    gc = g.c()
    return np.array([lib().orc_radius(ctypes.byref(gc), i) for i in range(g.n)])


def kappa(l: int) -> float:
    return lib().orc_kappa(int(l))


def field(p: Pulse, t: float) -> float:
    pc = p.c()
    return lib().orc_field(ctypes.byref(pc), float(t))


def vector_potential_step(p: Pulse, t: float, h: float) -> float:
    """-int_t^{t+h} E by 5-point Gauss-Legendre (the increment of A/c)."""
    pc = p.c()
    return lib().orc_vector_potential_step(ctypes.byref(pc), float(t), float(h))


def vector_potential_at(p: Pulse, t0: float, dt: float) -> float:
    """A/c at t0 from t_on by the same rule over ceil((t0 - t_on)/dt) equal pieces."""
    pc = p.c()
    return lib().orc_vector_potential_at(ctypes.byref(pc), float(t0), float(dt))


def h_bound(g: Grid, efield: float) -> float:
    """Gershgorin bound on the spectral radius of H(E) (H(A/c) in the velocity gauge)."""
    gc = g.c()
    return lib().orc_h_bound(ctypes.byref(gc), float(efield))


def apply_h(g: Grid, efield: float, psi) -> np.ndarray:
    psi = _state(g, psi)
    out = np.empty_like(psi)
    gc = g.c()
    lib().orc_apply_h(ctypes.byref(gc), float(efield), _dptr(psi), _dptr(out))
    return out


def taylor_step(g: Grid, efield: float, dt: float, order: int, psi) -> np.ndarray:
    psi = _state(g, psi).copy()
    gc = g.c()
    lib().orc_taylor_step(ctypes.byref(gc), float(efield), float(dt), int(order), _dptr(psi))
    return psi


def rk4_step(g: Grid, p: Pulse, t: float, dt: float, psi) -> np.ndarray:
    psi = _state(g, psi).copy()
    gc, pc = g.c(), p.c()
    lib().orc_rk4_step(ctypes.byref(gc), ctypes.byref(pc), float(t), float(dt), _dptr(psi))
    return psi


def lanczos_step(g: Grid, efield: float, dt: float, m: int, psi):
    """Returns (new state, Krylov dimension used)."""
    psi = _state(g, psi).copy()
    gc = g.c()
    used = lib().orc_lanczos_step(ctypes.byref(gc), float(efield), float(dt), int(m), _dptr(psi))
    return psi, used


def jacobi_eig(a: np.ndarray):
    """Eigenvalues (unsorted) and eigenvector columns of a dense symmetric matrix."""
    a = np.array(a, dtype=np.float64, order="C", copy=True)
    m = a.shape[0]
    v = np.empty((m, m))
    lib().orc_jacobi_eig(m, _dptr(a), _dptr(v))
    return np.diag(a).copy(), v


def initial_state(g: Grid):
    """(psi0, u0): the normalised 1s state in the l = 0 row, and that row."""
    psi = np.empty(g.size, dtype=np.complex128)
    u0 = np.empty(g.n)
    gc = g.c()
    lib().orc_initial_state(ctypes.byref(gc), _dptr(psi), _dptr(u0))
    return psi, u0


@dataclass
class ObsSetup:
    r_ion: float
    u0: np.ndarray
    phi: np.ndarray          # [n_states, n] bound eigenvectors
    state_l: np.ndarray      # [n_states] int32
    state_n: np.ndarray      # [n_states] principal quantum numbers

    @property
    def record(self) -> int:
        return OBS_FIXED + len(self.state_l)


def observables(g: Grid, p: Pulse, t: float, setup: ObsSetup, psi) -> np.ndarray:
    psi = _state(g, psi)
    out = np.empty(setup.record)
    gc, pc = g.c(), p.c()
    phi = np.ascontiguousarray(setup.phi, dtype=np.float64)
    sl = np.ascontiguousarray(setup.state_l, dtype=np.int32)
    lib().orc_observables(ctypes.byref(gc), ctypes.byref(pc), float(t), float(setup.r_ion),
                          _dptr(np.ascontiguousarray(setup.u0)), len(sl), _iptr(sl), _dptr(phi),
                          _dptr(psi), _dptr(out))
    return out


def propagate(g: Grid, p: Pulse, method: int, order_or_m: int, t0: float, dt: float,
              nsteps: int, obs_every: int, setup: ObsSetup, psi):
    """Runs nsteps steps; returns (state, observables [n_obs, record], min Krylov dim)."""
    psi = _state(g, psi).copy()
    n_obs = nsteps // obs_every if obs_every > 0 else 0
    obs = np.zeros((max(n_obs, 1), setup.record))
    gc, pc = g.c(), p.c()
    phi = np.ascontiguousarray(setup.phi, dtype=np.float64)
    sl = np.ascontiguousarray(setup.state_l, dtype=np.int32)
    used = lib().orc_propagate(ctypes.byref(gc), ctypes.byref(pc), int(method), int(order_or_m),
                               float(t0), float(dt), int(nsteps), int(obs_every),
                               float(setup.r_ion), _dptr(np.ascontiguousarray(setup.u0)), len(sl),
                               _iptr(sl), _dptr(phi), _dptr(psi), _dptr(obs))
    return psi, obs[:n_obs], used


def mask(r: float, r_b: float, p: float) -> float:
    """Absorbing mask M(r) (Sec. 2.1), the one-step factor of W."""
    return float(lib().orc_mask(float(r), float(r_b), float(p)))


def radial_current(g: Grid, j: int, psi) -> float:
    """J = sum_l Im[f_l^* df_l/dr] at grid point j (eq. flux, length gauge)."""
    psi = _state(g, psi)
    gc = g.c()
    return float(lib().orc_radial_current(ctypes.byref(gc), int(j), _dptr(psi)))


def radial_current_vel(g: Grid, j: int, a_tilde: float, psi) -> float:
    """The velocity-gauge current: radial_current plus 2 A~ sum_l kappa_{l+1} Re[f_l^* f_{l+1}]."""
    psi = _state(g, psi)
    gc = g.c()
    return float(lib().orc_radial_current_vel(ctypes.byref(gc), int(j), float(a_tilde), _dptr(psi)))


def propagate_abs(g: Grid, p: Pulse, method: int, order_or_m: int, t0: float, dt: float, nsteps: int,
                  obs_every: int, setup: "ObsSetup", psi, r_abs: float = 0.0, p_abs: float = 0.0,
                  flux_j: int = -1):
    """propagate with the absorbing mask after every step (r_abs > 0) and the
    time-integrated current at point flux_j (>= 0); returns (state, records,
    min Krylov dim, flux integral)."""
    psi = _state(g, psi).copy()
    n_obs = nsteps // obs_every if obs_every > 0 else 0
    obs = np.zeros((max(n_obs, 1), setup.record))
    flux = np.zeros(1)
    gc, pc = g.c(), p.c()
    phi = np.ascontiguousarray(setup.phi, dtype=np.float64)
    sl = np.ascontiguousarray(setup.state_l, dtype=np.int32)
    used = lib().orc_propagate_abs(ctypes.byref(gc), ctypes.byref(pc), int(method), int(order_or_m), float(t0),
                                   float(dt), int(nsteps), int(obs_every), float(setup.r_ion),
                                   _dptr(np.ascontiguousarray(setup.u0)), len(sl), _iptr(sl), _dptr(phi),
                                   float(r_abs), float(p_abs), int(flux_j), _dptr(psi), _dptr(obs), _dptr(flux))
    return psi, obs[:n_obs], used, float(flux[0])


def rk_tableau(method: int):
    """(c, a, b, bhat, stages) of an explicit Runge-Kutta method (appendix)."""
    c, b, bh = np.zeros(RK_MAX), np.zeros(RK_MAX), np.zeros(RK_MAX)
    a = np.zeros((RK_MAX, RK_MAX))
    s = lib().orc_rk_tableau(int(method), _dptr(c), _dptr(a), _dptr(b), _dptr(bh))
    return c[:s], a[:s, :s], b[:s], bh[:s], s


def rk_step(g: Grid, p: Pulse, method: int, t: float, dt: float, psi):
    """One step; returns (state, sigma_n)."""
    psi = _state(g, psi).copy()
    gc, pc = g.c(), p.c()
    sig = lib().orc_rk_step(ctypes.byref(gc), ctypes.byref(pc), int(method), float(t), float(dt), _dptr(psi))
    return psi, sig


def propagate_rk(g: Grid, p: Pulse, method: int, t0: float, dt: float, nsteps: int, obs_every: int,
                 setup: "ObsSetup", psi):
    """Runs nsteps steps; returns (state, observables [n_obs, record], sigma = sum of sigma_n)."""
    psi = _state(g, psi).copy()
    n_obs = nsteps // obs_every if obs_every > 0 else 0
    obs = np.zeros((max(n_obs, 1), setup.record))
    gc, pc = g.c(), p.c()
    phi = np.ascontiguousarray(setup.phi, dtype=np.float64)
    sl = np.ascontiguousarray(setup.state_l, dtype=np.int32)
    sigma = lib().orc_propagate_rk(ctypes.byref(gc), ctypes.byref(pc), int(method), float(t0), float(dt),
                                   int(nsteps), int(obs_every), float(setup.r_ion),
                                   _dptr(np.ascontiguousarray(setup.u0)), len(sl), _iptr(sl), _dptr(phi),
                                   _dptr(psi), _dptr(obs))
    return psi, obs[:n_obs], sigma


def imag_propagate(g: Grid, dtau: float, order: int, nsteps: int, psi):
    """Diffusion (imaginary-time) ground-state search (Sec. 4): normalises psi,
    runs nsteps field-free steps of the order-P Taylor polynomial of
    exp(-dtau H) with renormalisation; returns (state, energy per step)."""
    psi = _state(g, psi).copy()
    energy = np.zeros(max(int(nsteps), 1))
    gc = g.c()
    lib().orc_imag_propagate(ctypes.byref(gc), float(dtau), int(order), int(nsteps), _dptr(psi), _dptr(energy))
    return psi, energy[:nsteps]


from .eigen import bound_states, obs_setup  # noqa: E402  (needs Grid)

__all__ = ["Grid", "Pulse", "ObsSetup", "build", "lib", "radius", "kappa", "field", "h_bound", "apply_h",
           "taylor_step", "rk4_step", "lanczos_step", "jacobi_eig", "initial_state",
           "observables", "propagate", "imag_propagate", "mask", "radial_current", "propagate_abs", "rk_tableau", "rk_step", "propagate_rk", "bound_states", "obs_setup", "TAYLOR", "RK4", "LANCZOS",
           "OBS_FIXED", "OBS_NAMES"]
