"""Python binding of libtdse (MI355X finite-difference TDSE library).

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``libtdse.so`` (built by ``paper_1308_1856_amd/build.py``).
PyTorch provides device memory and the stream.  The functions mirror the C
ABI of ``include/tdse.h`` one to one; ``Propagator`` bundles a context with
its torch-owned buffers.  There is no CPU fallback: if the library is not
built, importing this package raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtdse.so")

TDSE_OK = 0
STATUS = {0: "TDSE_OK", -1: "TDSE_E_INVALID", -2: "TDSE_E_NOMEM", -3: "TDSE_E_HIP",
          -4: "TDSE_E_UNSTABLE", -5: "TDSE_E_BREAKDOWN", -6: "TDSE_E_NONFINITE", -7: "TDSE_E_WORKSPACE",
          -8: "TDSE_E_UNBOUND"}
FP64, FP32, FP48 = 0, 1, 2
METHOD_TAYLOR, METHOD_RK4, METHOD_LANCZOS, METHOD_TUNE, METHOD_RK_TABLEAU = 0, 1, 2, 3, 4
RK_EULER, RK_CLASSIC4, RK_FEHLBERG45, RK_CASHKARP, RK_DORMANDPRINCE, RK_MERSON = range(6)
GAUGE_LENGTH, GAUGE_VELOCITY = 0, 1
PULSE_SINE2_E, PULSE_SINE2_A = 0, 1
MAX_STATES = 15
OBS_FIELDS = ("t", "e_field", "norm", "p_g", "p_bound", "p_ion", "dipole", "accel")
OBS_DOUBLES = len(OBS_FIELDS) + MAX_STATES

EXPORTED = ("tdse_init_grid", "tdse_destroy", "tdse_last_error", "tdse_num_instances",
            "tdse_state_offset", "tdse_state_bytes", "tdse_workspace_bytes", "tdse_bind",
            "tdse_set_state", "tdse_get_state", "tdse_apply_H", "tdse_step_taylor",
            "tdse_step_rk4", "tdse_step_lanczos", "tdse_observables", "tdse_lambda_max_bound",
            "tdse_taylor_stability_limit", "tdse_timing_enable", "tdse_timing_read",
            "tdse_use_graphs", "tdse_set_obs_overlap", "tdse_set_obs_fusion", "tdse_obs_fusion", "tdse_set_rk4_fusion", "tdse_rk4_fusion", "tdse_autotune", "tdse_tile_rows", "tdse_sweep_variant",
            "tdse_autotune_taylor", "tdse_taylor_fusion", "tdse_taylor_fusion_kind",
            "tdse_set_taylor_fusion", "tdse_set_sweep_shape", "tdse_lanczos_dims",
            "tdse_observables_noalloc", "tdse_step_imag", "tdse_taylor_real_stability_limit",
            "tdse_step_rk", "tdse_rk_stability_limit", "tdse_set_absorber", "tdse_set_flux", "tdse_get_flux",
            "tdse_set_gauge", "tdse_gauge")


class TdseError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class GridDesc(ctypes.Structure):
    _fields_ = [("n_r", ctypes.c_int32), ("lmax", ctypes.c_int32), ("stencil", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("dr", ctypes.c_double), ("z_nuc", ctypes.c_double),
                ("r_ion", ctypes.c_double)]


class Pulse(ctypes.Structure):
    _fields_ = [("e0", ctypes.c_double), ("omega", ctypes.c_double), ("n_cycles", ctypes.c_double),
                ("cep", ctypes.c_double), ("t_on", ctypes.c_double), ("shape", ctypes.c_int32),
                ("pad_", ctypes.c_int32)]


class Obs(ctypes.Structure):
    _fields_ = [(f, ctypes.c_double) for f in OBS_FIELDS] + [("pop", ctypes.c_double * MAX_STATES)]


def _load():
    # torch ships its own HIP runtime with the same SONAME (libamdhip64.so.7).
    # Importing torch first makes libtdse bind to that already-loaded runtime,
    # so there is one HIP runtime in the process and torch's streams and
    # allocations are valid handles for the library.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                          "(hipcc --offload-arch=gfx950)")
    L = ctypes.CDLL(LIB_PATH)
    vp, dp, i32, i64 = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int32, ctypes.c_int64
    ctxp = ctypes.c_void_p
    sig = {
        "tdse_init_grid": ([ctypes.POINTER(GridDesc), i32, ctypes.POINTER(ctxp)], i32),
        "tdse_destroy": ([ctxp], None),
        "tdse_last_error": ([ctxp], ctypes.c_char_p),
        "tdse_num_instances": ([ctxp], i32),
        "tdse_state_offset": ([ctxp, i32], i64),
        "tdse_state_bytes": ([ctxp], ctypes.c_size_t),
        "tdse_workspace_bytes": ([ctxp, i32, i32], ctypes.c_size_t),
        "tdse_bind": ([ctxp, vp, vp, ctypes.c_size_t, vp], i32),
        "tdse_set_state": ([ctxp, i32, dp], i32),
        "tdse_get_state": ([ctxp, i32, dp], i32),
        "tdse_apply_H": ([ctxp, dp, vp, vp], i32),
        "tdse_step_taylor": ([ctxp, ctypes.POINTER(Pulse), dp, dp, i32, i32, i32, vp], i32),
        "tdse_step_rk4": ([ctxp, ctypes.POINTER(Pulse), dp, dp, i32, i32, vp], i32),
        "tdse_step_lanczos": ([ctxp, ctypes.POINTER(Pulse), dp, dp, i32, i32, i32, vp], i32),
        "tdse_observables": ([ctxp, ctypes.POINTER(Pulse), dp, ctypes.POINTER(Obs)], i32),
        "tdse_observables_noalloc": ([ctxp, ctypes.POINTER(Pulse), dp, ctypes.POINTER(Obs)], i32),
        "tdse_lambda_max_bound": ([ctxp, i32, ctypes.c_double], ctypes.c_double),
        "tdse_taylor_stability_limit": ([i32], ctypes.c_double),
        "tdse_taylor_real_stability_limit": ([i32], ctypes.c_double),
        "tdse_step_imag": ([ctxp, dp, i32, i32, vp], i32),
        "tdse_step_rk": ([ctxp, ctypes.POINTER(Pulse), dp, dp, i32, i32, i32, vp, vp], i32),
        "tdse_rk_stability_limit": ([i32], ctypes.c_double),
        "tdse_set_absorber": ([ctxp, dp, dp], i32),
        "tdse_set_gauge": ([ctxp, i32], i32),
        "tdse_gauge": ([ctxp], i32),
        "tdse_set_flux": ([ctxp, ctypes.POINTER(i32)], i32),
        "tdse_get_flux": ([ctxp, dp], i32),
        "tdse_timing_enable": ([ctxp, i32], i32),
        "tdse_timing_read": ([ctxp, ctypes.c_char_p, ctypes.POINTER(i64), dp], i32),
        "tdse_use_graphs": ([ctxp, i32], i32),
        "tdse_set_obs_overlap": ([ctxp, i32], i32),
        "tdse_set_obs_fusion": ([ctxp, i32], i32),
        "tdse_obs_fusion": ([ctxp], i32),
        "tdse_set_rk4_fusion": ([ctxp, i32], i32),
        "tdse_rk4_fusion": ([ctxp], i32),
        "tdse_autotune": ([ctxp, ctypes.POINTER(i32)], i32),
        "tdse_tile_rows": ([ctxp], i32),
        "tdse_sweep_variant": ([ctxp], i32),
        "tdse_autotune_taylor": ([ctxp, i32, ctypes.POINTER(i32), ctypes.POINTER(i32)], i32),
        "tdse_taylor_fusion": ([ctxp], i32),
        "tdse_taylor_fusion_kind": ([ctxp], i32),
        "tdse_set_taylor_fusion": ([ctxp, i32, i32, i32], i32),
        "tdse_set_sweep_shape": ([ctxp, i32, i32], i32),
        "tdse_lanczos_dims": ([ctxp, ctypes.POINTER(i32)], i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes, f.restype = args, res
    return L


lib = _load()


def _check(ctx, code: int):
    if code != TDSE_OK:
        msg = lib.tdse_last_error(ctx).decode() if ctx else ""
        raise TdseError(code, msg)


def _dvec(values, n: int):
    arr = (ctypes.c_double * n)(*[float(v) for v in values])
    return arr


def _pulses(pulses: Sequence) -> ctypes.Array:
    arr = (Pulse * len(pulses))()
    for k, p in enumerate(pulses):
        arr[k] = Pulse(float(p.e0), float(p.omega), float(p.n_cycles), float(p.cep), float(p.t_on),
                       int(getattr(p, "shape", 0)))
    return arr


# ------------------------------------------------------------------------
# thin wrappers with the C names
# ------------------------------------------------------------------------

def tdse_init_grid(grids: Sequence[GridDesc]) -> ctypes.c_void_p:
    arr = (GridDesc * len(grids))(*grids)
    ctx = ctypes.c_void_p()
    code = lib.tdse_init_grid(arr, len(grids), ctypes.byref(ctx))
    if code != TDSE_OK:
        raise TdseError(code, "tdse_init_grid rejected the grid description")
    return ctx


def tdse_destroy(ctx):
    lib.tdse_destroy(ctx)


def tdse_bind(ctx, d_state: int, d_work: int, work_bytes: int, stream: int):
    _check(ctx, lib.tdse_bind(ctx, d_state, d_work, work_bytes, stream))


def tdse_set_state(ctx, inst: int, host: Optional[np.ndarray]):
    if host is None:
        _check(ctx, lib.tdse_set_state(ctx, inst, None))
        return
    h = np.ascontiguousarray(host, dtype=np.complex128)
    _check(ctx, lib.tdse_set_state(ctx, inst, h.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))


def tdse_get_state(ctx, inst: int, count: int) -> np.ndarray:
    out = np.empty(count, dtype=np.complex128)
    _check(ctx, lib.tdse_get_state(ctx, inst, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return out


def tdse_apply_H(ctx, e_field: Sequence[float], d_in: int, d_out: int):
    n = lib.tdse_num_instances(ctx)
    _check(ctx, lib.tdse_apply_H(ctx, _dvec(e_field, n), d_in, d_out))


def tdse_step_taylor(ctx, pulses, t0, dt, order, nsteps, obs_every, d_obs):
    n = lib.tdse_num_instances(ctx)
    _check(ctx, lib.tdse_step_taylor(ctx, _pulses(pulses), _dvec(t0, n), _dvec(dt, n), order,
                                     nsteps, obs_every, d_obs))


def tdse_step_rk4(ctx, pulses, t0, dt, nsteps, obs_every, d_obs):
    n = lib.tdse_num_instances(ctx)
    _check(ctx, lib.tdse_step_rk4(ctx, _pulses(pulses), _dvec(t0, n), _dvec(dt, n), nsteps,
                                  obs_every, d_obs))


def tdse_step_lanczos(ctx, pulses, t0, dt, m, nsteps, obs_every, d_obs):
    n = lib.tdse_num_instances(ctx)
    _check(ctx, lib.tdse_step_lanczos(ctx, _pulses(pulses), _dvec(t0, n), _dvec(dt, n), m,
                                      nsteps, obs_every, d_obs))


def tdse_step_rk(ctx, pulses, t0, dt, method, nsteps, obs_every, d_obs, d_sigma=None):
    n = lib.tdse_num_instances(ctx)
    _check(ctx, lib.tdse_step_rk(ctx, _pulses(pulses), _dvec(t0, n), _dvec(dt, n), method, nsteps,
                                 obs_every, d_obs, d_sigma))


def tdse_rk_stability_limit(method: int) -> float:
    return lib.tdse_rk_stability_limit(int(method))


def tdse_step_imag(ctx, dtau, order, nsteps, d_energy):
    n = lib.tdse_num_instances(ctx)
    _check(ctx, lib.tdse_step_imag(ctx, _dvec(dtau, n), order, nsteps, d_energy))


def tdse_set_gauge(ctx, gauge: int):
    _check(ctx, lib.tdse_set_gauge(ctx, int(gauge)))


def tdse_set_absorber(ctx, r_abs, p_abs):
    n = lib.tdse_num_instances(ctx)
    _check(ctx, lib.tdse_set_absorber(ctx, _dvec(r_abs, n), _dvec(p_abs, n)))


def tdse_set_flux(ctx, i_flux):
    n = lib.tdse_num_instances(ctx)
    _check(ctx, lib.tdse_set_flux(ctx, (ctypes.c_int32 * n)(*[int(i) for i in i_flux])))


def tdse_get_flux(ctx) -> np.ndarray:
    n = lib.tdse_num_instances(ctx)
    out = (ctypes.c_double * n)()
    _check(ctx, lib.tdse_get_flux(ctx, out))
    return np.frombuffer(out, dtype=np.float64).copy()


def tdse_taylor_real_stability_limit(order: int) -> float:
    return lib.tdse_taylor_real_stability_limit(int(order))


def tdse_observables(ctx, pulses, t) -> np.ndarray:
    n = lib.tdse_num_instances(ctx)
    out = (Obs * n)()
    _check(ctx, lib.tdse_observables(ctx, _pulses(pulses), _dvec(t, n), out))
    return np.frombuffer(out, dtype=np.float64).reshape(n, OBS_DOUBLES).copy()


def tdse_observables_noalloc(ctx, pulses, t) -> np.ndarray:
    """tdse_observables with its scratch in the library's static device buffer."""
    n = lib.tdse_num_instances(ctx)
    out = (Obs * n)()
    _check(ctx, lib.tdse_observables_noalloc(ctx, _pulses(pulses), _dvec(t, n), out))
    return np.frombuffer(out, dtype=np.float64).reshape(n, OBS_DOUBLES).copy()


def tdse_lanczos_dims(ctx):
    """(Krylov dimension per instance, broke_down): the smallest dimension
    each instance used in the last Lanczos call; TDSE_E_BREAKDOWN is
    information, not an error, and comes back as broke_down = True."""
    n = lib.tdse_num_instances(ctx)
    out = (ctypes.c_int32 * n)()
    code = lib.tdse_lanczos_dims(ctx, out)
    if code not in (TDSE_OK, -5):
        _check(ctx, code)
    return list(out), code == -5


def tdse_lambda_max_bound(ctx, inst: int, e_max: float) -> float:
    return lib.tdse_lambda_max_bound(ctx, inst, float(e_max))


def tdse_taylor_stability_limit(order: int) -> float:
    return lib.tdse_taylor_stability_limit(int(order))


def tdse_timing_enable(ctx, enable: bool):
    _check(ctx, lib.tdse_timing_enable(ctx, 1 if enable else 0))


def tdse_autotune(ctx) -> int:
    rows = ctypes.c_int32()
    _check(ctx, lib.tdse_autotune(ctx, ctypes.byref(rows)))
    return rows.value


def tdse_autotune_taylor(ctx, order: int):
    k, rows = ctypes.c_int32(), ctypes.c_int32()
    _check(ctx, lib.tdse_autotune_taylor(ctx, int(order), ctypes.byref(k), ctypes.byref(rows)))
    return k.value, rows.value


def tdse_tile_rows(ctx) -> int:
    return lib.tdse_tile_rows(ctx)


def tdse_use_graphs(ctx, enable: bool):
    _check(ctx, lib.tdse_use_graphs(ctx, 1 if enable else 0))


def tdse_set_obs_overlap(ctx, enable: bool):
    _check(ctx, lib.tdse_set_obs_overlap(ctx, 1 if enable else 0))


def tdse_set_obs_fusion(ctx, enable: bool):
    _check(ctx, lib.tdse_set_obs_fusion(ctx, 1 if enable else 0))


def tdse_obs_fusion(ctx) -> bool:
    return bool(lib.tdse_obs_fusion(ctx))


def tdse_set_rk4_fusion(ctx, enable: bool):
    _check(ctx, lib.tdse_set_rk4_fusion(ctx, 1 if enable else 0))


def tdse_rk4_fusion(ctx) -> bool:
    return bool(lib.tdse_rk4_fusion(ctx))


def tdse_timing_read(ctx, kernel: str):
    n = ctypes.c_int64()
    ms = ctypes.c_double()
    _check(ctx, lib.tdse_timing_read(ctx, kernel.encode(), ctypes.byref(n), ctypes.byref(ms)))
    return n.value, ms.value


# ------------------------------------------------------------------------
# convenience: a context with torch-owned device buffers
# ------------------------------------------------------------------------

@dataclass(frozen=True)
class Grid:
    n: int
    lmax: int
    dr: float
    stencil: int = 3
    precision: int = FP64
    z: float = 1.0
    r_ion: float = 50.0

    def desc(self) -> GridDesc:
        return GridDesc(self.n, self.lmax, self.stencil, self.precision, self.dr, self.z, self.r_ion)


class Propagator:
    """One context (n_inst instances) plus its state and workspace on a GPU.

    `methods` lists (method, order_or_m) pairs the workspace must serve.  The
    library works on its own stream (default priority); every call first
    orders that stream after torch's current stream and afterwards orders
    torch's current stream after it, so torch code may use the buffers
    directly.  `graphs` turns on hipGraph replay of the step loop.
    """

    def __init__(self, grids: Sequence[Grid], methods=((METHOD_TAYLOR, 8),), device="cuda:0",
                 stream=None, graphs: bool = False):
        import torch
        self.torch = torch
        self.grids = list(grids)
        self.ctx = tdse_init_grid([g.desc() for g in self.grids])
        self.n_inst = len(self.grids)
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        sbytes = lib.tdse_state_bytes(self.ctx)
        wbytes = max(lib.tdse_workspace_bytes(self.ctx, m, o) for m, o in methods)
        # byte buffers (torch's caching allocator aligns to >= 512 B)
        self.state = torch.zeros(sbytes, dtype=torch.uint8, device=self.device)
        self.work = torch.zeros(wbytes, dtype=torch.uint8, device=self.device)
        self.work_bytes = wbytes
        torch.cuda.synchronize(self.device)
        tdse_bind(self.ctx, self.state.data_ptr(), self.work.data_ptr(), wbytes,
                  self.stream.cuda_stream)
        self.offsets = [lib.tdse_state_offset(self.ctx, k) for k in range(self.n_inst)]
        self.elem = {FP64: 16, FP32: 8, FP48: 12}[self.grids[0].precision]
        self.fusion_rows = 16   # rows of the fused tiles (the library's default until set or tuned)
        if graphs:
            tdse_use_graphs(self.ctx, True)

    def _enter(self):
        self.stream.wait_stream(self.torch.cuda.current_stream(self.device))

    def _leave(self):
        self.torch.cuda.current_stream(self.device).wait_stream(self.stream)

    def close(self):
        if self.ctx:
            self.torch.cuda.synchronize(self.device)
            tdse_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # state
    def set_state(self, inst: int, psi: Optional[np.ndarray] = None):
        self._enter()
        tdse_set_state(self.ctx, inst, psi)
        self._leave()

    def get_state(self, inst: int) -> np.ndarray:
        g = self.grids[inst]
        self._enter()
        return tdse_get_state(self.ctx, inst, (g.lmax + 1) * g.n)

    def new_vector(self):
        """A zeroed device vector shaped like the state (for apply_H)."""
        return self.torch.zeros_like(self.state)

    def obs_buffer(self, nsteps: int, obs_every: int):
        n_rec = nsteps // obs_every if obs_every > 0 else 0
        return self.torch.zeros((self.n_inst, max(n_rec, 1), OBS_DOUBLES), dtype=self.torch.float64,
                                device=self.device)

    def _per_inst(self, v):
        return [v] * self.n_inst if np.isscalar(v) else list(v)

    def apply_H(self, e_field, d_in, d_out):
        self._enter()
        tdse_apply_H(self.ctx, self._per_inst(e_field), d_in.data_ptr(), d_out.data_ptr())
        self._leave()

    def step_taylor(self, pulses, t0, dt, order, nsteps, obs_every=0, obs=None):
        ptr = obs.data_ptr() if obs is not None else None
        self._enter()
        tdse_step_taylor(self.ctx, self._pulse_list(pulses), self._per_inst(t0),
                         self._per_inst(dt), order, nsteps, obs_every, ptr)
        self._leave()

    def step_rk4(self, pulses, t0, dt, nsteps, obs_every=0, obs=None):
        ptr = obs.data_ptr() if obs is not None else None
        self._enter()
        tdse_step_rk4(self.ctx, self._pulse_list(pulses), self._per_inst(t0), self._per_inst(dt),
                      nsteps, obs_every, ptr)
        self._leave()

    def step_lanczos(self, pulses, t0, dt, m, nsteps, obs_every=0, obs=None):
        ptr = obs.data_ptr() if obs is not None else None
        self._enter()
        tdse_step_lanczos(self.ctx, self._pulse_list(pulses), self._per_inst(t0),
                          self._per_inst(dt), m, nsteps, obs_every, ptr)
        self._leave()

    def step_rk(self, pulses, t0, dt, method, nsteps, obs_every=0, obs=None, sigma=None):
        """Tableau Runge-Kutta steps; `sigma` a float64 device tensor of n_inst
        values the passive truncation estimate is added to (or None)."""
        ptr = obs.data_ptr() if obs is not None else None
        sptr = sigma.data_ptr() if sigma is not None else None
        self._enter()
        tdse_step_rk(self.ctx, self._pulse_list(pulses), self._per_inst(t0), self._per_inst(dt), method, nsteps,
                     obs_every, ptr, sptr)
        self._leave()

    def step_imag(self, dtau, order, nsteps, energy=None):
        """Diffusion (imaginary-time) steps; `energy` a float64 device tensor of
        n_inst * nsteps values (or None)."""
        ptr = energy.data_ptr() if energy is not None else None
        self._enter()
        tdse_step_imag(self.ctx, self._per_inst(dtau), order, nsteps, ptr)
        self._leave()

    def set_gauge(self, gauge: int):
        """GAUGE_LENGTH or GAUGE_VELOCITY for the following steps."""
        tdse_set_gauge(self.ctx, gauge)

    @property
    def gauge(self) -> int:
        return lib.tdse_gauge(self.ctx)

    def set_absorber(self, r_abs, p_abs):
        """Absorbing mask after every real-time step (r_abs <= 0: none)."""
        self._enter()
        tdse_set_absorber(self.ctx, self._per_inst(r_abs), self._per_inst(p_abs))
        self._leave()

    def set_flux(self, i_flux):
        """Flux points (radial index, -1: none); resets the accumulated yields."""
        self._enter()
        tdse_set_flux(self.ctx, self._per_inst(i_flux))
        self._leave()

    def flux_yield(self) -> np.ndarray:
        self._enter()
        out = tdse_get_flux(self.ctx)
        self._leave()
        return out

    def lanczos_dims(self):
        """(smallest Krylov dimension per instance in the last Lanczos call, broke_down)."""
        self._enter()
        return tdse_lanczos_dims(self.ctx)

    def observables(self, pulses, t) -> np.ndarray:
        self._enter()
        return tdse_observables(self.ctx, self._pulse_list(pulses), self._per_inst(t))

    def observables_noalloc(self, pulses, t) -> np.ndarray:
        self._enter()
        return tdse_observables_noalloc(self.ctx, self._pulse_list(pulses), self._per_inst(t))

    def use_graphs(self, enable: bool):
        tdse_use_graphs(self.ctx, enable)

    def set_obs_overlap(self, enable: bool):
        tdse_set_obs_overlap(self.ctx, enable)

    def set_obs_fusion(self, enable: bool):
        """Main observables summed in the Taylor step's last strip launch (on) or by their own pass."""
        tdse_set_obs_fusion(self.ctx, enable)

    @property
    def obs_fusion(self) -> bool:
        return tdse_obs_fusion(self.ctx)

    def set_rk4_fusion(self, enable: bool):
        tdse_set_rk4_fusion(self.ctx, enable)

    @property
    def rk4_fusion(self) -> bool:
        return tdse_rk4_fusion(self.ctx)

    def autotune(self) -> int:
        self._enter()
        rows = tdse_autotune(self.ctx)
        self._leave()
        return rows

    @property
    def tile_rows(self) -> int:
        return tdse_tile_rows(self.ctx)

    @property
    def sweep_variant(self) -> int:
        return lib.tdse_sweep_variant(self.ctx)

    def set_sweep_shape(self, rows: int, variant: int):
        _check(self.ctx, lib.tdse_set_sweep_shape(self.ctx, int(rows), int(variant)))

    def autotune_taylor(self, order: int):
        """(fused terms per launch or 0, rows per fused tile) chosen for `order`."""
        self._enter()
        out = tdse_autotune_taylor(self.ctx, order)
        self._leave()
        self.fusion_rows = out[1]
        return out

    @property
    def taylor_fusion(self) -> int:
        return lib.tdse_taylor_fusion(self.ctx)

    @property
    def taylor_fusion_kind(self) -> int:
        """Fused kernel in use: 0 LDS rings, 1 wave strips."""
        return lib.tdse_taylor_fusion_kind(self.ctx)

    def set_taylor_fusion(self, k: int, rows: int = 16, kind: int = 0):
        _check(self.ctx, lib.tdse_set_taylor_fusion(self.ctx, int(k), int(rows), int(kind)))
        self.fusion_rows = int(rows)

    def _pulse_list(self, pulses):
        if isinstance(pulses, (list, tuple)):
            return list(pulses)
        return [pulses] * self.n_inst

    def lambda_max_bound(self, inst: int, e_max: float) -> float:
        return tdse_lambda_max_bound(self.ctx, inst, e_max)

    def timing(self, enable: bool):
        tdse_timing_enable(self.ctx, enable)

    def timing_read(self, kernel: str):
        return tdse_timing_read(self.ctx, kernel)
