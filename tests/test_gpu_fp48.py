"""48-bit storage (TDSE_FP48): every entry point against the FP64 oracle.

The 48-bit state keeps each FP64 component rounded to nearest at 36 mantissa
bits (relative 2^-37 = 7.3e-12 per stored element); arithmetic and reductions
are FP64.  A sweep's output is the FP64 result rounded once, so single
applications agree with the oracle to ~2^-37 of each element; a step of a
propagation rounds the state once per launch, so a window of s steps stays
within ~s * 2^-37 * (launches per step) of the oracle (tolerance 1e-9 for
the windows below, 40 steps, a few launches per step).

Sizes span several 256-point radial tiles with a ragged tail and several row
tiles; both stencils; single instances and an uneven batch.
"""
import numpy as np
import pytest

import oracle
import workloads
from gpu_helpers import (lib, obs_abs_tol, obs_columns, orc_grid, orc_pulse, read_vector, rel_err, say,
                         series_ratio, to_fp48)

pytestmark = pytest.mark.gpu

FP48 = 2
TOL48 = 1e-9


def make(grids, methods):
    t = lib()
    gs = [t.Grid(n, lm, dr, st, FP48, 1.0, rion) for (n, lm, dr, st, rion) in grids]
    return t.Propagator(gs, methods=methods)


def test_fp48_state_round_trip_is_the_rounding():
    # set_state stores each component rounded at 36 mantissa bits; get_state
    # returns exactly that value (planes h and l read back bit for bit)
    t = lib()
    n, lmax = 777, 5
    prop = make([(n, lmax, 0.1, 3, 20.0)], [(t.METHOD_TAYLOR, 2)])
    psi = workloads.random_state(21, n, lmax)
    psi[5] = 1e-300 + 0j          # tiny and subnormal-adjacent values survive
    psi[6] = -0.0 + 1e-310j
    prop.set_state(0, psi)
    got = prop.get_state(0)
    want = to_fp48(psi)
    say(f"fp48 round trip: max |got - want| = {np.max(np.abs(got - want)):.1e}")
    assert np.array_equal(got.view(np.uint64), want.view(np.uint64))
    assert np.array_equal(read_vector(prop, prop.state, 0).view(np.uint64), want.view(np.uint64))
    assert np.max(np.abs(want - psi) / np.maximum(np.abs(psi), 1e-300)) <= 2.0 ** -36
    prop.close()


@pytest.mark.parametrize("stencil", [3, 5])
@pytest.mark.parametrize("variant", [0, 4])
def test_fp48_apply_h(stencil, variant):
    t = lib()
    n, lmax, dr, e = 700, 9, 0.1, 0.071
    say(f"fp48 apply_H stencil={stencil} sweep variant={variant} N={n} lmax={lmax} seed=11")
    prop = make([(n, lmax, dr, stencil, 20.0)], [(t.METHOD_TAYLOR, 2)])
    prop.set_sweep_shape(4, variant)
    psi = to_fp48(workloads.random_state(11, n, lmax))
    prop.set_state(0, psi)
    out = prop.new_vector()
    prop.apply_H(e, prop.state, out)
    got = read_vector(prop, out, 0)
    ref = oracle.apply_h(orc_grid(prop.grids[0]), e, psi)
    # the FP64 result rounded once (2^-37 of the element) plus FP64 rounding
    # of the terms (1e-13 of the largest element covers the stencil's
    # cancellations)
    assert np.all(np.abs(got - ref) <= 2.0 ** -36 * np.abs(ref) + 1e-13 * np.max(np.abs(ref)))
    say(f"  rel err {rel_err(got, ref):.2e}")
    prop.close()


def test_fp48_rejects_shapes_without_a_48_bit_form():
    t = lib()
    prop = make([(300, 3, 0.1, 3, 10.0)], [(t.METHOD_TAYLOR, 8)])
    with pytest.raises(t.TdseError):
        prop.set_sweep_shape(4, 1)          # two radii per thread
    with pytest.raises(t.TdseError):
        prop.set_taylor_fusion(4, 16, 0)    # LDS-ring fused kernel
    prop.close()


def _run(method, order, grids, pulses, dts, steps, every, fusion=None, rk4_fused=True, obs_fusion=None,
         psis=None, t0=0.0):
    t = lib()
    mcode = {"taylor": t.METHOD_TAYLOR, "rk4": t.METHOD_RK4, "lanczos": t.METHOD_LANCZOS}[method]
    prop = make(grids, [(mcode, order)])
    if fusion is not None:
        prop.set_taylor_fusion(*fusion)
    if obs_fusion is not None:
        prop.set_obs_fusion(obs_fusion)
    prop.set_rk4_fusion(rk4_fused)
    for k in range(len(grids)):
        prop.set_state(k, None if psis is None else psis[k])
    obs = prop.obs_buffer(steps, every)
    if method == "taylor":
        prop.step_taylor(pulses, t0, dts, order, steps, every, obs)
    elif method == "rk4":
        prop.step_rk4(pulses, t0, dts, steps, every, obs)
    else:
        prop.step_lanczos(pulses, t0, dts, order, steps, every, obs)
    states = [prop.get_state(k) for k in range(len(grids))]
    o = obs.cpu().numpy()
    prop.close()
    return states, o


CASES = [
    ("taylor", 8, None, True, None),          # one launch per Horner term
    ("taylor", 8, (4, 16, 1), True, True),    # wave strips, observables in the launch
    ("taylor", 8, (3, 8, 1), True, False),    # 3 + 3 + 2 terms, observables by their pass
    ("taylor", 4, (4, 32, 1), True, True),
    ("taylor", 7, (7, 8, 1), True, True),     # one launch of 7 terms (a last launch of 7)
    ("taylor", 8, (5, 16, 1), True, True),    # 5 + 3 terms
    ("taylor", 8, (8, 16, 2), True, True),    # pair strips, observables in the launch
    ("taylor", 8, (3, 8, 2), True, False),    # pair strips, 3 + 3 + 2 terms
    ("taylor", 8, (8, 16, 3), True, True),    # pair strips, persistent launch
    ("rk4", 4, None, True, None),             # one strip launch per step
    ("rk4", 4, None, False, None),            # four stage launches
    ("lanczos", 12, None, True, None),
]


@pytest.mark.parametrize("stencil", [3, 5])
@pytest.mark.parametrize("method,order,fusion,rk4_fused,obs_fusion", CASES)
def test_fp48_steps_track_the_fp64_oracle(method, order, fusion, rk4_fused, obs_fusion, stencil):
    t = lib()
    grids = [(520, 7, 0.1, stencil, 12.0), (1300, 12, 0.1, stencil, 40.0), (257, 0, 0.1, stencil, 10.0)]
    pulses = [t.Pulse(0.06, 0.35, 2.0, 0.2, 0.0), t.Pulse(-0.04, 0.5, 3.0, 1.0, 0.0),
              t.Pulse(0.08, 0.2, 1.0, -0.5, 0.0)]
    steps, every = 40, 10
    say(f"fp48 {method}-{order} fusion={fusion} rk4_fused={rk4_fused} obs_fusion={obs_fusion} "
        f"stencil={stencil}: 3 uneven grids vs the oracle")
    # a state with p_ion, dipole and excited populations well above zero:
    # the normalised 1s row plus a smooth seeded wave in every partial wave
    psis = []
    for k, (n, lm, dr, st, rion) in enumerate(grids):
        g = oracle.Grid(n=n, lmax=lm, dr=dr, stencil=st)
        u0, _ = oracle.initial_state(g)
        v = u0 + 0.4 * workloads.random_state(40 + k, n, lm, smooth=True) / np.sqrt(n * dr)
        psis.append(to_fp48(v / np.sqrt(dr * np.vdot(v, v).real)))
    if method == "lanczos":
        dts = [1e-3, 1e-3, 1e-3]
    else:
        y = t.tdse_taylor_stability_limit(order)
        dts = []
        for (n, lm, dr, st, rion), p in zip(grids, pulses):
            gg = oracle.Grid(n=n, lmax=lm, dr=dr, stencil=st)
            dts.append(0.8 * y / oracle.h_bound(gg, abs(p.e0)))
    states, o = _run(method, order, grids, pulses, dts, steps, every, fusion, rk4_fused, obs_fusion, psis)
    ocode = {"taylor": oracle.TAYLOR, "rk4": oracle.RK4, "lanczos": oracle.LANCZOS}[method]
    for k, (n, lm, dr, st, rion) in enumerate(grids):
        g = oracle.Grid(n=n, lmax=lm, dr=dr, stencil=st)
        setup = oracle.obs_setup(g, r_ion=rion)
        ref, robs, _ = oracle.propagate(g, orc_pulse(pulses[k]), ocode, order, 0.0, dts[k], steps, every,
                                        setup, psis[k])
        err = rel_err(states[k], ref)
        gobs = o[k][:, :obs_columns(setup)]
        ratio = series_ratio(gobs, robs, TOL48, obs_abs_tol(g, setup, robs))
        say(f"  instance {k}: state {err:.2e}, observables worst ratio {ratio.max():.2e}, "
            f"p_ion {robs[-1, 5]:.3e}")
        assert err < TOL48
        assert np.all(ratio <= 1.0), ratio
        assert np.all(gobs[:, 0] == robs[:, 0]) and np.all(gobs[:, 1] == robs[:, 1])


def test_fp48_observables_entry_point():
    t = lib()
    n, lmax, dr = 900, 6, 0.1
    say("fp48 tdse_observables on a random state vs the oracle")
    prop = make([(n, lmax, dr, 5, 30.0)], [(t.METHOD_TAYLOR, 2)])
    psi = workloads.random_state(31, n, lmax)
    psi = to_fp48(psi / np.sqrt(dr * np.vdot(psi, psi).real))
    prop.set_state(0, psi)
    p = t.Pulse(0.05, 0.3, 2.0, 0.0, 0.0)
    got = prop.observables(p, 7.0)[0]
    g = orc_grid(prop.grids[0])
    setup = oracle.obs_setup(g, r_ion=30.0)
    ref = oracle.observables(g, orc_pulse(p), 7.0, setup, psi)
    prop.close()
    k = len(ref)
    # the oracle reads the same 48-bit values: FP64 summation order only
    ratio = series_ratio(got[None, :k], ref[None, :], 1e-12, obs_abs_tol(g, setup, ref[None, :]))
    say(f"  worst ratio to tolerance {ratio.max():.2e}")
    assert np.all(ratio <= 1.0), ratio
