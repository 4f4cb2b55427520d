"""Reduced-precision storage against the FP64 GPU path on the workloads' own
shapes and windows (the FP64 path is pinned to the oracle by the parity
tests).  Targets: norm within 1e-6 of the FP64 run at every record; p_ion and
every bound population P_nl within 1e-5 relative wherever the FP64 value is
at least 1e-8 (below that, within 1e-13 absolute).

The 48-bit storage (TDSE_FP48) is held to these targets.  Plain FP32 storage
is run beside it and reported, not asserted: rounding the state to FP32 once
per step drifts coherently at the small explicit steps these grids need.

Windows start from a normalised mix of the 1s row and a smooth seeded wave in
every partial wave, so p_ion, the dipole and the excited populations are well
above zero from the first record.
"""
import math

import numpy as np
import pytest

import oracle
import workloads
from gpu_helpers import lib, say

pytestmark = pytest.mark.gpu

NORM_TOL, REL_TOL, FLOOR, ABS_BELOW = 1e-6, 1e-5, 1e-8, 1e-13


def target_errors(lo, hi):
    """Worst ratios to the targets of records `lo` against `hi` ([inst][rec][23])."""
    norm = np.max(np.abs(lo[..., 2] - hi[..., 2])) / NORM_TOL
    cols = [5] + list(range(8, 23))                 # p_ion, P_nl
    a, b = lo[..., cols], hi[..., cols]
    big = np.abs(b) >= FLOOR
    rel = np.where(big, np.abs(a - b) / np.where(big, np.abs(b), 1.0) / REL_TOL, np.abs(a - b) / ABS_BELOW)
    return float(norm), float(np.max(rel))


def mixed_state(n, lmax, dr, seed, z=1.0):
    g = oracle.Grid(n=n, lmax=lmax, dr=dr, stencil=3, z=z)
    u0, _ = oracle.initial_state(g)
    v = u0 + 0.4 * workloads.random_state(seed, n, lmax, smooth=True) / np.sqrt(n * dr)
    return v / np.sqrt(dr * np.vdot(v, v).real)


def run(grids, method, order, pulses, t0s, dts, steps, every, psis, fusion=None):
    t = lib()
    mcode = {"taylor": t.METHOD_TAYLOR, "lanczos": t.METHOD_LANCZOS}[method]
    prop = t.Propagator(grids, methods=((mcode, order),), graphs=True)
    if fusion:
        prop.set_taylor_fusion(*fusion)
    for k, psi in enumerate(psis):
        prop.set_state(k, psi)
    obs = prop.obs_buffer(steps, every)
    if method == "taylor":
        prop.step_taylor(pulses, t0s, dts, order, steps, every, obs)
    else:
        prop.step_lanczos(pulses, t0s, dts, order, steps, every, obs)
    o = obs.cpu().numpy()
    prop.close()
    return o


def compare(label, grids_of, *args):
    t = lib()
    res = {}
    for prec in (t.FP64, t.FP48, t.FP32):
        res[prec] = run(grids_of(prec), *args)
    e48 = target_errors(res[t.FP48], res[t.FP64])
    e32 = target_errors(res[t.FP32], res[t.FP64])
    o = res[t.FP64]
    say(f"{label}: FP48 norm {e48[0]:.2e}, p_ion/P_nl {e48[1]:.2e} of the targets; "
        f"FP32 norm {e32[0]:.2e}, p_ion/P_nl {e32[1]:.2e} (reported only); "
        f"FP64 p_ion {o[..., -1, 5].min():.2e}..{o[..., -1, 5].max():.2e}")
    assert e48[0] <= 1.0 and e48[1] <= 1.0
    return e48, e32


def test_batch_window_1000_steps_every_member():
    # the 256-member batch (uneven N, lmax, pulses; dr = 0.1, 3-point,
    # Taylor-8 at 0.8 of each member's stability limit), 1000 steps
    t = lib()
    members = workloads.batch_members()
    pulses = [t.Pulse(m.pulse.e0, m.pulse.omega, m.pulse.n_cycles, m.pulse.cep, m.pulse.t_on) for m in members]
    y = t.tdse_taylor_stability_limit(8)
    dts, psis, t0s = [], [], []
    for k, m in enumerate(members):
        g = oracle.Grid(n=m.n, lmax=m.lmax, dr=workloads.BATCH_DR, stencil=3)
        dts.append(workloads.BATCH_DT_SAFETY * y / oracle.h_bound(g, abs(m.pulse.e0)))
        psis.append(mixed_state(m.n, m.lmax, workloads.BATCH_DR, 1000 + k))
        t0s.append(0.5 * m.pulse.duration)          # mid-pulse: the field is on

    def grids_of(prec):
        return [t.Grid(m.n, m.lmax, workloads.BATCH_DR, 3, prec, 1.0,
                       workloads.BATCH_R_ION_FRACTION * m.n * workloads.BATCH_DR) for m in members]

    say("batch window: 256 members, 1000 Taylor-8 steps, FP64 / FP48 / FP32")
    compare("batch 1000 steps", grids_of, "taylor", 8, pulses, t0s, dts, 1000, 10, psis, (4, 32, 1))


def test_large_grid_window_200_steps():
    # N = 1e5, dr = 0.05, lmax = 256 (25.7M unknowns), 3-point, Taylor-8 at
    # dt = 2e-7, 1600 nm 2e14 W/cm^2 3-cycle pulse, 200 steps mid-pulse
    t = lib()
    wl = workloads.WORKLOADS["hydrogen_n100000_l256_fp32_taylor8"]
    p = t.Pulse(wl.pulse.e0, wl.pulse.omega, wl.pulse.n_cycles, wl.pulse.cep, wl.pulse.t_on)
    psi = mixed_state(wl.n, wl.lmax, wl.dr, 77)

    def grids_of(prec):
        return [t.Grid(wl.n, wl.lmax, wl.dr, wl.stencil, prec, 1.0, wl.r_ion)]

    say("large-grid window: 25.7M unknowns, 200 Taylor-8 steps, FP64 / FP48 / FP32")
    compare("25.7M grid 200 steps", grids_of, "taylor", 8, p, 0.5 * wl.pulse.duration, wl.dt, 200, 1, [psi],
            (4, 32, 1))


def test_lanczos_window_2000_steps():
    # N = 2e4, dr = 0.05, lmax = 64, 5-point, Lanczos m = 20 (4-cycle 800 nm
    # 1e14 W/cm^2 pulse), 2000 steps from mid-pulse at dt = 1e-4, where the
    # FP64 step reproduces itself to round-off (at dt = 0.01 a relative 1e-15
    # perturbation of the start grows to 1% of the state in 200 steps, in any
    # precision)
    t = lib()
    wl = workloads.WORKLOADS["hydrogen_n20000_l64_fp32_lanczos20"]
    p = t.Pulse(wl.pulse.e0, wl.pulse.omega, wl.pulse.n_cycles, wl.pulse.cep, wl.pulse.t_on)
    psi = mixed_state(wl.n, wl.lmax, wl.dr, 78)

    def grids_of(prec):
        return [t.Grid(wl.n, wl.lmax, wl.dr, wl.stencil, prec, 1.0, wl.r_ion)]

    say("Lanczos window: 1.3M unknowns, m = 20, 2000 steps of 1e-4 au, FP64 / FP48 / FP32")
    compare("Lanczos 2000 steps", grids_of, "lanczos", 20, p, 0.5 * wl.pulse.duration - 0.1, 1e-4, 2000, 20,
            [psi])
