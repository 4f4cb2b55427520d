"""GPU parity: every entry point of the C ABI against the FP64 oracle.

FP64 path: relative state error <= 1e-12 (||psi_gpu - psi_orc|| / ||psi_orc||)
and, per observable time series, max_t |x_gpu - x_orc| <= 1e-12 * max_t
|x_orc| + a, with a = 1e-13 for the fixed observables (sums of O(1) terms over
1e4-1e6 points carry ~sqrt(n)*eps ~ 1e-14 of round-off that depends on the
summation order, which differs between the two sides) and, for a population
P_nl, a = 2 delta + delta^2 with delta = 10 eps ||h_l|| / gap_nl: the two
sides compute the bound eigenvectors with different eigensolvers, and an
eigenvector is only defined to ~eps ||h_l|| / gap_nl.

Lanczos parity at 1e-12 needs a converged Krylov space (lambda_max dt of a
few units for m = 12-20); where it is far from converged (stiff grids, large
dt) the result amplifies round-off, and the tolerance is measured from the
oracle's own response to an eps-level perturbation of its input.

FP32 path (FP32 storage, FP64 arithmetic and reductions): every sweep rounds
its output to FP32 (relative 6e-8 per element), so single applications agree
to ~1e-7; propagation targets are populations and p_ion within 1e-5 relative
and norm drift below 1e-6.

Sizes span several 256-point radial tiles with a ragged tail and several
row tiles.
"""
import math

import numpy as np
import pytest

import oracle
import workloads
from gpu_helpers import (lib, obs_abs_tol, obs_columns, orc_grid, orc_pulse, read_vector, rel_err,
                         say, series_ratio, to_fp32)

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
FLOOR64 = 1e-13


def make(grids, methods, prec=0):
    t = lib()
    gs = [t.Grid(n, lm, dr, st, prec, 1.0, rion) for (n, lm, dr, st, rion) in grids]
    return t.Propagator(gs, methods=methods)


@pytest.mark.parametrize("stencil", [3, 5])
@pytest.mark.parametrize("prec", [0, 1])
def test_apply_h(stencil, prec):
    t = lib()
    n, lmax, dr, e = 700, 9, 0.1, 0.071
    say(f"apply_H stencil={stencil} prec={prec} N={n} lmax={lmax} seed=11")
    prop = make([(n, lmax, dr, stencil, 20.0)], [(t.METHOD_TAYLOR, 2)], prec)
    psi = workloads.random_state(11, n, lmax)
    if prec == 1:
        psi = to_fp32(psi)
    prop.set_state(0, psi)
    out = prop.new_vector()
    prop.apply_H(e, prop.state, out)
    got = read_vector(prop, out, 0)
    ref = oracle.apply_h(orc_grid(prop.grids[0]), e, psi)
    err = rel_err(got, ref)
    say(f"  rel err {err:.3e}")
    assert err < (2e-15 if prec == 0 else 1.2e-7)
    if prec == 0:
        # element by element, against the size of the terms that built each element
        assert np.max(np.abs(got - ref)) < 1e-13 * np.max(np.abs(ref))
    prop.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_apply_h_strip_sweep_bitwise(prec):
    # H psi on aligned wave strips of one level (sweep variants 4, 6) gives the
    # bits of the workgroup sweeps (variants 0 and 1), for both stencils, odd
    # N, a single row, N a whole number of tiles and one radius past it
    t = lib()
    say(f"apply_H on strips vs workgroup sweeps, prec {prec}")
    for n, lmax, stencil in ((701, 9, 3), (1999, 14, 5), (65, 0, 5), (130, 3, 3), (256, 2, 5), (257, 1, 3)):
        psi = workloads.random_state(5, n, lmax)
        if prec == 1:
            psi = to_fp32(psi)
        outs = []
        for rows, variant in ((4, 0), (8, 1), (4, 4), (1, 6), (16, 4)):
            prop = make([(n, lmax, 0.1, stencil, 20.0)], [(t.METHOD_TAYLOR, 2)], prec)
            prop.set_sweep_shape(rows, variant)
            prop.set_state(0, psi)
            out = prop.new_vector()
            prop.apply_H(0.043, prop.state, out)
            outs.append(read_vector(prop, out, 0))
            prop.close()
        for o in outs[1:]:
            assert np.array_equal(o, outs[0]), (n, lmax, stencil)


def _propagate_pair(method, order, n=520, lmax=7, dr=0.1, stencil=5, dt=4e-4, steps=40,
                    obs_every=10, prec=0, pulse=None, psi=None, t0=0.0, r_ion=12.0):
    t = lib()
    pulse = pulse or t.Pulse(0.06, 0.35, 2.0, 0.2, 0.0)
    grid = (n, lmax, dr, stencil, r_ion)
    mcode = {"taylor": t.METHOD_TAYLOR, "rk4": t.METHOD_RK4, "lanczos": t.METHOD_LANCZOS}[method]
    prop = make([grid], [(mcode, order)], prec)
    g = orc_grid(prop.grids[0])
    setup = oracle.obs_setup(g, r_ion=r_ion)
    if psi is None:
        psi, _ = oracle.initial_state(g)
    if prec == 1:
        psi = to_fp32(psi)
    prop.set_state(0, psi)
    obs = prop.obs_buffer(steps, obs_every)
    if method == "taylor":
        prop.step_taylor(pulse, t0, dt, order, steps, obs_every, obs)
    elif method == "rk4":
        prop.step_rk4(pulse, t0, dt, steps, obs_every, obs)
    else:
        prop.step_lanczos(pulse, t0, dt, order, steps, obs_every, obs)
    got = prop.get_state(0)
    gobs = obs.cpu().numpy()[0][:, :obs_columns(setup)]
    prop.close()
    ocode = {"taylor": oracle.TAYLOR, "rk4": oracle.RK4, "lanczos": oracle.LANCZOS}[method]
    ref, robs, _ = oracle.propagate(g, orc_pulse(pulse), ocode, order, t0, dt, steps, obs_every,
                                    setup, psi)
    _propagate_pair.last = (g, setup, psi, orc_pulse(pulse), ocode)
    return got, ref, gobs, robs


def _obs_ratio(gobs, robs):
    g, setup = _propagate_pair.last[:2]
    return series_ratio(gobs, robs, TOL64, obs_abs_tol(g, setup, robs))


@pytest.mark.parametrize("method,order,stencil", [("taylor", 8, 5), ("taylor", 4, 3), ("taylor", 1, 3),
                                                  ("taylor", 3, 5), ("rk4", 4, 3), ("rk4", 4, 5)])
def test_explicit_steps_fp64(method, order, stencil):
    say(f"{method}-{order} stencil={stencil} FP64 vs oracle")
    # below each order's imaginary-axis limit (lambda_max ~ 3.1e3 here); an
    # order-1 step has no stable interval, so it gets a vanishing dt
    dt = 4e-4 if order > 1 else 1e-10
    got, ref, gobs, robs = _propagate_pair(method, order, stencil=stencil, dt=dt)
    err = rel_err(got, ref)
    ratio = _obs_ratio(gobs, robs)
    say(f"  state {err:.2e}  observables worst ratio to tolerance {ratio.max():.2e}")
    assert err < TOL64
    assert np.all(ratio <= 1.0), ratio
    assert np.all(gobs[:, 0] == robs[:, 0])          # times identical
    assert np.all(gobs[:, 1] == robs[:, 1])          # fields identical (same libm on the host)


@pytest.mark.parametrize("stencil", [3, 5])
def test_rk4_one_launch_equals_stage_launches(stencil):
    # the four RK4 stages in one strip launch per step compute every element
    # from the same FP64 operands as the four stage launches: identical bits
    # (states and observable records), on a grid of odd N, a single row and an
    # uneven batch
    t = lib()
    say(f"RK4 in one launch vs four stage launches, stencil {stencil}")
    pulse = t.Pulse(0.06, 0.35, 2.0, 0.2, 0.0)
    cases = [[(523, 7, 0.1, stencil, 12.0)], [(65, 0, 0.1, stencil, 2.0)],
             [(1500, 12, 0.1, stencil, 50.0), (333, 3, 0.1, stencil, 10.0), (2047, 21, 0.1, stencil, 60.0)]]
    for grids in cases:
        res = []
        for fused in (False, True):
            prop = make(grids, [(t.METHOD_RK4, 4)], 0)
            prop.set_rk4_fusion(fused)
            assert prop.rk4_fusion == fused
            dts = [0.8 * t.tdse_taylor_stability_limit(4) / prop.lambda_max_bound(k, 0.06)
                   for k in range(len(grids))]
            for k in range(len(grids)):
                prop.set_state(k, None)
            obs = prop.obs_buffer(30, 3)
            prop.step_rk4(pulse, 0.5, dts, 30, 3, obs)
            res.append(([prop.get_state(k) for k in range(len(grids))], obs.cpu().numpy()))
            prop.close()
        for k in range(len(grids)):
            assert np.array_equal(res[0][0][k], res[1][0][k]), (grids, k)
        assert np.array_equal(res[0][1], res[1][1])


def test_rk4_one_launch_fp32_tracks_fp64_oracle():
    # FP32 storage: the one-launch step keeps the stage vectors in FP64, the
    # stage launches round them to FP32; both stay within a few FP32 roundings
    # per step of the FP64 oracle
    t = lib()
    say("RK4 FP32: one launch and stage launches vs the FP64 oracle")
    grid = (700, 9, 0.1, 5, 20.0)
    pulse = t.Pulse(0.06, 0.35, 2.0, 0.2, 0.0)
    g = None
    errs = []
    for fused in (True, False):
        prop = make([grid], [(t.METHOD_RK4, 4)], 1)
        prop.set_rk4_fusion(fused)
        g = orc_grid(prop.grids[0])
        psi, _ = oracle.initial_state(g)
        psi = to_fp32(psi)
        prop.set_state(0, psi)
        dt = 0.5 * t.tdse_taylor_stability_limit(4) / prop.lambda_max_bound(0, 0.06)
        prop.step_rk4(pulse, 0.0, dt, 40)
        got = prop.get_state(0)
        prop.close()
        setup = oracle.obs_setup(g, r_ion=20.0)
        ref, _, _ = oracle.propagate(g, orc_pulse(pulse), oracle.RK4, 4, 0.0, dt, 40, 0, setup, psi)
        errs.append(rel_err(got, ref))
    say(f"  one launch {errs[0]:.2e}, stage launches {errs[1]:.2e}")
    assert errs[0] < 4e-6 and errs[1] < 4e-6


@pytest.mark.parametrize("m,stencil,dt", [(12, 5, 1e-3), (20, 3, 2e-3), (1, 3, 1e-3)])
def test_lanczos_fp64(m, stencil, dt):
    say(f"lanczos m={m} stencil={stencil} dt={dt} FP64 vs oracle (converged Krylov space)")
    got, ref, gobs, robs = _propagate_pair("lanczos", m, stencil=stencil, dt=dt, steps=30)
    err = rel_err(got, ref)
    ratio = _obs_ratio(gobs, robs)
    say(f"  state {err:.2e}  observables worst ratio to tolerance {ratio.max():.2e}")
    assert err < TOL64
    assert np.all(ratio <= 1.0), ratio


@pytest.mark.parametrize("m,dt", [(12, 0.05), (20, 0.02)])
def test_lanczos_fp64_stiff(m, dt):
    # lambda_max dt ~ 60-150: the Krylov space is far from converged in the
    # upper spectrum and the result amplifies round-off.  Tolerance: 10x the
    # oracle's own spread under a relative 1e-15 perturbation of its input.
    say(f"lanczos m={m} dt={dt} FP64 vs oracle, unconverged regime")
    got, ref, _, _ = _propagate_pair("lanczos", m, stencil=5, dt=dt, steps=30)
    g, setup, psi, pulse, ocode = _propagate_pair.last
    rng = np.random.default_rng(99)
    pert = psi * (1 + 1e-15 * (rng.standard_normal(psi.size) + 1j * rng.standard_normal(psi.size)))
    ref2, _, _ = oracle.propagate(g, pulse, ocode, m, 0.0, dt, 30, 10, setup, pert)
    spread = rel_err(ref2, ref)
    err = rel_err(got, ref)
    say(f"  gpu vs oracle {err:.2e}; oracle vs perturbed oracle {spread:.2e}")
    assert err <= 10 * max(spread, 1e-15)
    assert abs(np.vdot(got, got).real / np.vdot(ref, ref).real - 1) < 1e-12   # unitary either way


def test_lanczos_breakdown_on_eigenstate():
    # a field-free eigenvector: the Krylov space is invariant after one vector
    t = lib()
    n, lmax, dr = 600, 3, 0.1
    g = oracle.Grid(n=n, lmax=lmax, dr=dr, stencil=3)
    e, phi, states = oracle.bound_states(g, 3)
    k = states.index((3, 2))
    psi = np.zeros(g.size, dtype=np.complex128)
    psi[2 * n:3 * n] = phi[k]
    say("lanczos breakdown on the 3d eigenvector")
    got, ref, _, _ = _propagate_pair("lanczos", 20, n=n, lmax=lmax, dr=dr, stencil=3, dt=0.5,
                                     steps=4, pulse=t.Pulse(0.0, 1.0, 1.0, 0.0, 0.0), psi=psi,
                                     obs_every=2)
    assert rel_err(got, np.exp(-1j * e[k] * 2.0) * psi) < 1e-12
    assert rel_err(got, ref) < 1e-12


def test_lanczos_dims_reports_breakdown_as_information():
    # an eigenvector breaks the Krylov process down after one vector in every
    # step: tdse_lanczos_dims gives TDSE_E_BREAKDOWN (information) with the
    # dimension used; a random state keeps the full dimension (TDSE_OK)
    t = lib()
    n, lmax, dr = 600, 3, 0.1
    g = oracle.Grid(n=n, lmax=lmax, dr=dr, stencil=3)
    e, phi, states = oracle.bound_states(g, 2)
    prop = make([(n, lmax, dr, 3, 20.0)], [(t.METHOD_LANCZOS, 12)])
    psi = np.zeros(g.size, dtype=np.complex128)
    psi[:n] = phi[states.index((1, 0))]
    prop.set_state(0, psi)
    prop.step_lanczos(t.Pulse(0.0, 1.0, 1.0, 0.0, 0.0), 0.0, 0.5, 12, 3)
    dims, broke = prop.lanczos_dims()
    say(f"lanczos dims on an eigenvector: {dims}, breakdown {broke}")
    assert broke and dims == [1]
    prop.set_state(0, workloads.random_state(3, n, lmax))
    prop.step_lanczos(t.Pulse(0.05, 0.3, 2.0, 0.0, 0.0), 0.0, 1e-3, 12, 2)
    dims, broke = prop.lanczos_dims()
    assert not broke and dims == [12]
    prop.close()


def test_fault_paths_nonfinite_and_workspace():
    # a NaN in the state makes tdse_observables return TDSE_E_NONFINITE; a
    # Lanczos call with a workspace sized for Taylor returns TDSE_E_WORKSPACE
    # and enqueues nothing (the state is unchanged)
    t = lib()
    n, lmax = 400, 4
    prop = make([(n, lmax, 0.1, 3, 20.0)], [(t.METHOD_TAYLOR, 8)])
    psi = workloads.random_state(8, n, lmax)
    psi[3 * n + 17] = np.nan
    prop.set_state(0, psi)
    with pytest.raises(t.TdseError) as e:
        prop.observables(t.Pulse(0.0, 1.0, 1.0, 0.0, 0.0), 0.0)
    assert e.value.code == -6
    prop.set_state(0, None)
    before = prop.get_state(0)
    with pytest.raises(t.TdseError) as e:
        prop.step_lanczos(t.Pulse(0.05, 0.3, 2.0, 0.0, 0.0), 0.0, 1e-3, 20, 4)
    assert e.value.code == -7
    assert np.array_equal(prop.get_state(0), before)
    prop.close()


def test_batch_matches_single_instances():
    t = lib()
    grids = [(300, 3, 0.1, 5, 8.0), (777, 10, 0.05, 5, 20.0), (257, 0, 0.2, 5, 10.0)]
    pulses = [t.Pulse(0.05, 0.3, 2.0, 0.0, 0.0), t.Pulse(-0.03, 0.5, 3.0, 1.0, 0.5),
              t.Pulse(0.08, 0.2, 1.0, -0.5, 0.0)]
    dts = [1e-3, 5e-5, 2e-3]            # each below its grid's order-7 stability limit
    t0s = [0.0, 0.3, 1.0]
    steps, every = 30, 10
    say("batched Taylor-7 over 3 uneven grids vs the oracle per grid")
    prop = make(grids, [(t.METHOD_TAYLOR, 7)])
    for k in range(3):
        prop.set_state(k, None)
    obs = prop.obs_buffer(steps, every)
    prop.step_taylor(pulses, t0s, dts, 7, steps, every, obs)
    gobs_all = obs.cpu().numpy()
    for k, (n, lm, dr, st, rion) in enumerate(grids):
        got = prop.get_state(k)
        g = oracle.Grid(n=n, lmax=lm, dr=dr, stencil=st)
        setup = oracle.obs_setup(g, r_ion=rion)
        psi0, _ = oracle.initial_state(g)
        ref, robs, _ = oracle.propagate(g, orc_pulse(pulses[k]), oracle.TAYLOR, 7, t0s[k], dts[k],
                                        steps, every, setup, psi0)
        err = rel_err(got, ref)
        ratio = series_ratio(gobs_all[k][:, :obs_columns(setup)], robs, TOL64, obs_abs_tol(g, setup, robs))
        say(f"  instance {k}: state {err:.2e} observables worst ratio {ratio.max():.2e}")
        assert err < TOL64 and np.all(ratio <= 1.0)
        assert np.all(gobs_all[k][:, obs_columns(setup):] == 0.0)   # unused population slots
    prop.close()


def test_observables_entry_point():
    t = lib()
    n, lmax, dr = 900, 6, 0.1
    say("tdse_observables on a random state vs the oracle")
    prop = make([(n, lmax, dr, 3, 30.0)], [(t.METHOD_TAYLOR, 2)])
    psi = workloads.random_state(5, n, lmax)
    psi /= np.sqrt(dr * np.vdot(psi, psi).real)
    prop.set_state(0, psi)
    p = t.Pulse(0.05, 0.057, 2.0, -math.pi / 2, 0.0)
    got = prop.observables(p, 37.25)[0]
    g = orc_grid(prop.grids[0])
    setup = oracle.obs_setup(g, r_ion=30.0)
    ref = oracle.observables(g, orc_pulse(p), 37.25, setup, psi)
    prop.close()
    k = len(ref)
    ratio = series_ratio(got[None, :k], ref[None, :], TOL64, obs_abs_tol(g, setup, ref[None, :]))
    say(f"  worst ratio to tolerance {ratio.max():.2e}")
    assert np.all(ratio <= 1.0), ratio


def test_unstable_dt_is_rejected_and_state_untouched():
    t = lib()
    prop = make([(400, 8, 0.1, 3, 20.0)], [(t.METHOD_TAYLOR, 4)])
    prop.set_state(0, None)
    before = prop.get_state(0)
    lam = prop.lambda_max_bound(0, 0.05)
    dt = 1.01 * t.tdse_taylor_stability_limit(4) / lam
    say(f"unstable dt {dt:.3e} (limit {t.tdse_taylor_stability_limit(4) / lam:.3e})")
    with pytest.raises(t.TdseError) as e:
        prop.step_taylor(t.Pulse(0.05, 0.3, 2.0, 0.0, 0.0), 0.0, dt, 4, 10)
    assert e.value.code == -4
    with pytest.raises(t.TdseError):
        prop.step_rk4(t.Pulse(0.05, 0.3, 2.0, 0.0, 0.0), 0.0, dt, 10)
    assert np.array_equal(prop.get_state(0), before)
    prop.close()


def test_fp32_taylor_tracks_fp64_oracle():
    # 5000 Taylor-8 steps with FP32 storage against the FP64 oracle.  Every
    # sweep rounds its output to FP32 (unit round-off u = 6e-8); the errors
    # random-walk, so the comparison is on a window of 5000 steps.
    t = lib()
    say("FP32-state Taylor-8, 5000 steps vs the FP64 oracle")
    pulse = t.Pulse(0.1, 0.5, 2.0, 0.0, 0.0)
    steps, every = 5000, 1000
    got, ref, gobs, robs = _propagate_pair("taylor", 8, n=600, lmax=8, dr=0.1, stencil=3,
                                           dt=8e-4, steps=steps, obs_every=every, prec=1,
                                           pulse=pulse, r_ion=5.0)
    pops_g, pops_r = gobs[:, 8:], robs[:, 8:]
    big = pops_r > 1e-3
    rel = np.abs(pops_g[big] - pops_r[big]) / pops_r[big]
    ion = np.abs(gobs[:, 5] - robs[:, 5]) / robs[:, 5]
    pb = np.abs(gobs[:, 4] - robs[:, 4]) / robs[:, 4]
    drift = np.max(np.abs(gobs[:, 2] - robs[:, 2]))
    say(f"  P_nl>1e-3 rel {rel.max():.2e}  p_bound rel {pb.max():.2e}  p_ion rel {ion.max():.2e} "
        f"(p_ion {robs[-1, 5]:.3e})  norm drift {drift:.2e}  |N-1| {np.max(np.abs(gobs[:, 2] - 1)):.2e}"
        f"  state {rel_err(got, ref):.2e}")
    assert robs[-1, 5] > 1e-3                                   # not a vacuous p_ion check
    assert ion.max() < 1e-5 and pb.max() < 1e-5 and drift < 1e-6
    assert rel.max() < 1e-4


def test_minimum_grid_and_single_partial_wave():
    # N = 8 (one partial tile), lmax = 0 (no coupling): all three methods
    for method, order in (("taylor", 4), ("rk4", 4), ("lanczos", 5)):
        say(f"{method} on N=8, lmax=0")
        got, ref, gobs, robs = _propagate_pair(method, order, n=8, lmax=0, dr=0.5, stencil=5,
                                               dt=2e-3, steps=10, obs_every=5)
        assert rel_err(got, ref) < TOL64
        assert np.all(_obs_ratio(gobs, robs) <= 1.0)


@pytest.mark.parametrize("method", ["taylor", "rk4", "lanczos"])
def test_graph_replay_matches_direct_launches(method):
    # 700 steps = chunks of 256, 256, 188 steps; observables every 64 steps,
    # so the first two chunks replay one graph.  The call is made twice and
    # each graph replay is compared bit for bit with direct launches.
    t = lib()
    grid = t.Grid(300, 5, 0.1, 5, t.FP64, 1.0, 10.0)
    mcode = {"taylor": t.METHOD_TAYLOR, "rk4": t.METHOD_RK4, "lanczos": t.METHOD_LANCZOS}[method]
    order = {"taylor": 8, "rk4": 4, "lanczos": 10}[method]
    pulse = t.Pulse(0.05, 0.4, 2.0, 0.0, 0.0)
    dt = 5e-4 if method != "lanczos" else 5e-3
    say(f"graph replay vs direct launches: {method}")
    results = []
    for graphs in (False, True):
        prop = t.Propagator([grid], methods=((mcode, order),), graphs=graphs)
        prop.set_state(0, None)
        states, records = [], []
        for call in range(2):
            obs = prop.obs_buffer(700, 64)
            t0 = call * 700 * dt
            if method == "taylor":
                prop.step_taylor(pulse, t0, dt, order, 700, 64, obs)
            elif method == "rk4":
                prop.step_rk4(pulse, t0, dt, 700, 64, obs)
            else:
                prop.step_lanczos(pulse, t0, dt, order, 700, 64, obs)
            states.append(prop.get_state(0))
            records.append(obs.cpu().numpy())
            _ = prop.observables(pulse, t0)        # eager work between replays
        prop.close()
        results.append((states, records))
    for call in range(2):
        assert np.array_equal(results[0][0][call], results[1][0][call])
        assert np.array_equal(results[0][1][call], results[1][1][call])


def test_autotune_keeps_results_bitwise(tmp_path, monkeypatch):
    t = lib()
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("TDSE_TUNE_CACHE", str(cache))
    grid = t.Grid(5000, 20, 0.1, 3, t.FP64, 1.0, 50.0)
    pulse = t.Pulse(0.05, 0.1, 2.0, 0.0, 0.0)
    say("autotune: Taylor-8 results before and after re-tiling")
    prop = t.Propagator([grid], methods=((t.METHOD_TAYLOR, 8),))
    dt = 0.8 * t.tdse_taylor_stability_limit(8) / prop.lambda_max_bound(0, 0.05)
    start_rows = prop.tile_rows
    out = []
    for tune in (False, True):
        prop.set_state(0, None)
        if tune:
            rows = prop.autotune()
            say(f"  rows {start_rows} -> {rows}")
            assert rows in (1, 2, 4, 8, 16, 32) and prop.tile_rows == rows
        prop.step_taylor(pulse, 10.0, dt, 8, 20)
        out.append(prop.get_state(0))
    prop.close()
    assert np.array_equal(out[0], out[1])
    assert cache.read_text().split()[-2] == str(rows)
    # a new context of the same shape class starts from the cached choice
    prop2 = t.Propagator([grid], methods=((t.METHOD_TAYLOR, 8),))
    assert prop2.tile_rows == rows
    prop2.close()


@pytest.mark.parametrize("stencil,k,rows,kind", [(5, 8, 4, 0), (5, 4, 16, 0), (3, 5, 3, 0), (3, 8, 32, 0),
                                                 (5, 8, 4, 1), (5, 4, 16, 1), (3, 5, 3, 1), (3, 8, 64, 1),
                                                 (3, 6, 1, 1), (5, 7, 9, 1),
                                                 (5, 8, 4, 2), (5, 4, 16, 2), (3, 5, 3, 2), (3, 8, 64, 2),
                                                 (3, 6, 1, 2), (5, 7, 9, 2), (3, 3, 2, 2), (5, 2, 5, 2),
                                                 (5, 8, 4, 3), (3, 5, 3, 3), (3, 8, 64, 3), (5, 7, 9, 3)])
def test_fused_taylor_bitwise_equal_to_per_term(stencil, k, rows, kind):
    # K Horner terms per launch (either fused kernel) compute every element
    # with the same FP64 expression as one launch per term: identical bits,
    # and the oracle's 1e-12
    t = lib()
    grid = t.Grid(700, 9, 0.1, stencil, t.FP64, 1.0, 12.0)
    pulse = t.Pulse(0.06, 0.35, 2.0, 0.2, 0.0)
    say(f"fused Taylor-8, K={k}, rows={rows}, stencil={stencil}, kind={kind} vs per-term and oracle")
    res = []
    for fuse in (0, k):
        prop = t.Propagator([grid], methods=((t.METHOD_TAYLOR, 8),))
        prop.set_taylor_fusion(fuse, rows, kind)
        prop.set_state(0, None)
        obs = prop.obs_buffer(31, 10)
        prop.step_taylor(pulse, 0.0, 4e-4, 8, 31, 10, obs)       # odd count: ends on the scratch side
        res.append((prop.get_state(0), obs.cpu().numpy()))
        prop.close()
    assert np.array_equal(res[0][0], res[1][0])
    # the strips sum the main observables in the step's last launch (another
    # order of the same FP64 sums); the LDS-ring kernel leaves them to the pass
    assert_records_match(res[1][1], res[0][1], main_bitwise=(kind == 0))
    g = orc_grid(grid)
    setup = oracle.obs_setup(g, r_ion=12.0)
    psi0, _ = oracle.initial_state(g)
    ref, robs, _ = oracle.propagate(g, orc_pulse(pulse), oracle.TAYLOR, 8, 0.0, 4e-4, 31, 10, setup, psi0)
    assert rel_err(res[1][0], ref) < TOL64


@pytest.mark.parametrize("kind", [0, 1, 2, 3])
def test_fused_taylor_fp32_and_graphs(kind):
    t = lib()
    grid = t.Grid(600, 8, 0.1, 3, t.FP32, 1.0, 5.0)
    pulse = t.Pulse(0.1, 0.5, 2.0, 0.0, 0.0)
    say(f"fused Taylor-8 (K=8, kind {kind}) with FP32 storage and graph replay")
    out = {}
    for fuse, graphs in ((0, False), (8, False), (8, True)):
        prop = t.Propagator([grid], methods=((t.METHOD_TAYLOR, 8),), graphs=graphs)
        prop.set_taylor_fusion(fuse, 16, kind)
        prop.set_state(0, None)
        states = []
        for call in range(2):
            obs = prop.obs_buffer(701, 64)
            prop.step_taylor(pulse, call * 701 * 8e-4, 8e-4, 8, 701, 64, obs)
            states.append((prop.get_state(0), obs.cpu().numpy()))
        prop.close()
        out[(fuse, graphs)] = states
    for call in range(2):
        # graphs replay the direct launches bit for bit
        assert np.array_equal(out[(8, False)][call][0], out[(8, True)][call][0])
        assert np.array_equal(out[(8, False)][call][1], out[(8, True)][call][1])
        # fused (FP64 intermediates) vs per-term (FP32 intermediates): rounding only
        d = rel_err(out[(8, False)][call][0], out[(0, False)][call][0])
        say(f"  call {call}: fused vs per-term FP32 state difference {d:.2e}")
        assert d < 1e-4


def test_autotune_taylor_choice_is_consistent():
    t = lib()
    grid = t.Grid(4000, 24, 0.1, 5, t.FP64, 1.0, 50.0)
    pulse = t.Pulse(0.05, 0.1, 2.0, 0.0, 0.0)
    prop = t.Propagator([grid], methods=((t.METHOD_TUNE, 0),))
    dt = 0.8 * t.tdse_taylor_stability_limit(8) / prop.lambda_max_bound(0, 0.05)
    prop.set_state(0, None)
    before = prop.get_state(0)
    k, rows = prop.autotune_taylor(8)
    say(f"autotune_taylor: K={k} rows={rows} kind={prop.taylor_fusion_kind}")
    assert np.array_equal(prop.get_state(0), before)           # state restored
    assert k == 0 or 2 <= k <= 8
    assert prop.taylor_fusion_kind in (0, 1, 2, 3)
    assert prop.obs_fusion in (True, False)     # the tuner's choice of the observables' summation
    obs_tuned = prop.obs_buffer(12, 1)
    prop.step_taylor(pulse, 5.0, dt, 8, 12, 1, obs_tuned)
    tuned = prop.get_state(0)
    prop.set_taylor_fusion(0, 16)
    prop.set_state(0, None)
    obs_plain = prop.obs_buffer(12, 1)
    prop.step_taylor(pulse, 5.0, dt, 8, 12, 1, obs_plain)
    assert np.array_equal(prop.get_state(0), tuned)
    assert_records_match(obs_tuned.cpu().numpy(), obs_plain.cpu().numpy(), main_bitwise=False)
    prop.close()


@pytest.mark.parametrize("kind", [0, 1, 2, 3])
def test_fused_taylor_batch_bitwise(kind):
    # uneven instances in one launch: each fused kernel matches the per-term
    # path bit for bit on every instance (FP64)
    t = lib()
    grids = [t.Grid(n, lmax, 0.1, 3, t.FP64, 1.0, 0.25 * n * 0.1)
             for n, lmax in ((1500, 12), (333, 3), (2047, 21))]
    pulses = [t.Pulse(0.05, 0.3, 2.0, 0.0, 0.0), t.Pulse(0.02, 0.1, 3.0, 0.5, 0.0),
              t.Pulse(0.08, 0.2, 2.0, -1.0, 0.0)]
    say(f"batch of 3, Taylor-8, fused kind {kind} (K=4, rows 8) vs per-term")
    res = []
    for fuse in (0, 4):
        prop = t.Propagator(grids, methods=((t.METHOD_TAYLOR, 8),))
        y = t.tdse_taylor_stability_limit(8)
        dts = [0.8 * y / prop.lambda_max_bound(k, abs(p.e0)) for k, p in enumerate(pulses)]
        prop.set_taylor_fusion(fuse, 8, kind)
        for k in range(3):
            prop.set_state(k, None)
        prop.step_taylor(pulses, [1.0] * 3, dts, 8, 17)
        res.append([prop.get_state(k) for k in range(3)])
        prop.close()
    for k in range(3):
        assert np.array_equal(res[0][k], res[1][k]), k


@pytest.mark.parametrize("graphs", [False, True])
def test_persistent_pair_strips_bitwise_vs_one_workgroup_per_tile(graphs):
    # The persistent launch (workgroups resident at once taking the tiles
    # from a work queue, most rows first) computes every tile as the launch
    # with one workgroup per tile does: on an uneven batch over several
    # chunks of steps, with the observables in the launch and graph replay,
    # states and records are identical bit for bit.  Two calls in a row check
    # that each launch leaves the queue reset for the next.
    t = lib()
    grids = [t.Grid(n, lmax, 0.1, 3, t.FP64, 1.0, 0.25 * n * 0.1)
             for n, lmax in ((1500, 12), (333, 3), (2047, 21), (900, 64), (4100, 1))]
    pulses = [t.Pulse(0.05, 0.3, 2.0, 0.0, 0.0), t.Pulse(0.02, 0.1, 3.0, 0.5, 0.0),
              t.Pulse(0.08, 0.2, 2.0, -1.0, 0.0), t.Pulse(0.03, 0.25, 2.0, 0.3, 0.0),
              t.Pulse(0.06, 0.15, 3.0, 0.0, 0.0)]
    nsteps, m = 300, len(grids)
    say(f"persistent pair strips (kind 3) vs one workgroup per tile (kind 2), graphs={graphs}")
    out = []
    for kind in (2, 3):
        prop = t.Propagator(grids, methods=((t.METHOD_TAYLOR, 8),), graphs=graphs)
        y = t.tdse_taylor_stability_limit(8)
        dts = [0.8 * y / prop.lambda_max_bound(k, abs(p.e0)) for k, p in enumerate(pulses)]
        prop.set_taylor_fusion(8, 16, kind)
        for k in range(m):
            prop.set_state(k, None)
        recs = []
        for call in range(2):
            obs = prop.obs_buffer(nsteps, 1)
            prop.step_taylor(pulses, [1.0 + call * nsteps * d for d in dts], dts, 8, nsteps, 1, obs)
            recs.append(obs.cpu().numpy())
        out.append(([prop.get_state(k) for k in range(m)], recs))
        prop.close()
    for k in range(m):
        assert np.array_equal(out[0][0][k], out[1][0][k]), k
    for a, b in zip(out[0][1], out[1][1]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("obs_every", [1, 2, 3])
def test_observables_beside_next_step_bitwise(obs_every):
    # The Taylor path computes the observables of step s on a second stream,
    # beside step s+1.  States and records must equal serial launches (overlap
    # off: every launch on one stream, in order), with direct launches, with
    # timing events on both streams and with graphs, over more than one chunk
    # of steps.
    t = lib()
    grid = t.Grid(4000, 16, 0.1, 5, t.FP64, 1.0, 100.0)
    pulse = t.Pulse(0.05, 0.2, 2.0, 0.0, 0.0)
    nsteps = 300
    say(f"observables every {obs_every} step(s) beside the next step vs serial launches")
    out = []
    for mode in ("serial", "direct", "timed", "graphs"):
        prop = t.Propagator([grid], methods=((t.METHOD_TAYLOR, 8),), graphs=(mode == "graphs"))
        prop.set_taylor_fusion(4, 8, 1)
        prop.set_obs_overlap(mode != "serial")
        if mode == "timed":
            prop.timing(True)
        dt = 0.8 * t.tdse_taylor_stability_limit(8) / prop.lambda_max_bound(0, 0.05)
        prop.set_state(0, None)
        obs = prop.obs_buffer(nsteps, obs_every)
        prop.step_taylor(pulse, 0.0, dt, 8, nsteps, obs_every, obs)
        out.append((prop.get_state(0), obs.cpu().numpy()))
        prop.close()
    for state, rec in out[1:]:
        assert np.array_equal(state, out[0][0])
        assert np.array_equal(rec, out[0][1])


MAIN_OBS = (2, 5, 6, 7)    # norm, p_ion, dipole, acceleration


def assert_records_match(a, b, main_bitwise):
    """Records [instance][record][column] of two runs of one propagation:
    bit for bit, except (main_bitwise False) the main observables, which may
    be summed in another order: 1e-13 of each instance's largest value, plus
    1e-12 absolute (the dipole and acceleration cancel between terms of
    order one, and r up to a few hundred au, so their rounding is absolute)."""
    a, b = np.asarray(a), np.asarray(b)
    assert a.shape == b.shape
    if main_bitwise:
        assert np.array_equal(a, b)
        return
    other = [c for c in range(a.shape[2]) if c not in MAIN_OBS]
    assert np.array_equal(a[:, :, other], b[:, :, other])
    for col in MAIN_OBS:
        scale = np.max(np.abs(b[:, :, col]), axis=1, keepdims=True)
        diff = np.abs(a[:, :, col] - b[:, :, col])
        assert np.all(diff <= 1e-13 * scale + 1e-12), (col, float(np.max(diff)), float(np.max(scale)))


@pytest.mark.parametrize("prec,stencil,kind", [(0, 5, 1), (1, 3, 1), (0, 5, 2), (1, 3, 2), (0, 3, 2),
                                               (0, 3, 3), (1, 5, 3)])
def test_observables_in_strip_launch_match_pass(prec, stencil, kind):
    # The main observables (norm, p_ion, dipole, acceleration) summed by the
    # step's last wave-strip launch agree with the observables pass to FP64
    # rounding (another order of the same sums); the populations, the states
    # and the other columns are unchanged bit for bit.  Batches with uneven
    # grids, ragged row blocks (17 rows in blocks of 8), several K, records
    # every step and every third step, with and without graphs.
    t = lib()
    # (the 65-radius single row and the two-row grid put the row past a
    # tile, which the launch computes for the last l-coupling, above lmax)
    grids = [t.Grid(2501, 16, 0.1, stencil, prec, 1.0, 60.0), t.Grid(1200, 5, 0.1, stencil, prec, 1.0, 30.0),
             t.Grid(777, 9, 0.1, stencil, prec, 1.0, 20.0), t.Grid(65, 0, 0.1, stencil, prec, 1.0, 3.0),
             t.Grid(300, 1, 0.1, stencil, prec, 1.0, 10.0)]
    pulses = [t.Pulse(0.06, 0.25, 2.0, 0.1, 0.0), t.Pulse(0.03, 0.4, 3.0, 0.0, 0.0), t.Pulse(0.08, 0.3, 2.0, 0.5, 0.0),
              t.Pulse(0.05, 0.5, 2.0, 0.0, 0.0), t.Pulse(0.07, 0.2, 2.0, 0.3, 0.0)]
    ng = len(grids)
    nsteps = 12
    say(f"observables in the strip launch vs their own pass, prec {prec}, stencil {stencil}")
    # (K = 7 and 5: Taylor-8's last launch has 1 and 3 terms)
    for K, rows, every, graphs in ((4, 8, 1, False), (3, 4, 3, True), (8, 16, 1, True), (2, 1, 2, False),
                                   (7, 8, 1, True), (5, 16, 3, False)):
        out = []
        for fused in (True, False):
            prop = t.Propagator(grids, methods=((t.METHOD_TAYLOR, 8),), graphs=graphs)
            prop.set_taylor_fusion(K, rows, kind)
            prop.set_obs_fusion(fused)
            assert prop.obs_fusion == fused
            dts = [0.5 * t.tdse_taylor_stability_limit(8) / prop.lambda_max_bound(k, 0.1) for k in range(ng)]
            for k in range(ng):
                prop.set_state(k, None)
            obs = prop.obs_buffer(nsteps, every)
            prop.step_taylor(pulses, [5.0, 3.0, 1.0, 2.0, 0.5], dts, 8, nsteps, every, obs)
            out.append(([prop.get_state(k) for k in range(ng)], obs.cpu().numpy()))
            prop.close()
        (sf, rf), (sp, rp) = out
        for a, b in zip(sf, sp):
            assert np.array_equal(a, b)
        assert_records_match(rf, rp, main_bitwise=False)


def test_explicit_sweep_shape_bitwise():
    # an explicit sweep shape (as the bench uses to reproduce a tuned one) gives the same bits
    t = lib()
    grid = t.Grid(3001, 11, 0.1, 5, t.FP64, 1.0, 50.0)
    pulse = t.Pulse(0.05, 0.2, 2.0, 0.3, 0.0)
    say("explicit sweep shapes: Taylor-8 bitwise across (rows, variant)")
    out = []
    for rows, variant in ((1, 0), (8, 1), (4, 2), (32, 3), (16, 4), (2, 6), (1, 4)):
        prop = t.Propagator([grid], methods=((t.METHOD_TAYLOR, 8),))
        prop.set_sweep_shape(rows, variant)
        assert (prop.tile_rows, prop.sweep_variant) == (rows, variant)
        dt = 0.8 * t.tdse_taylor_stability_limit(8) / prop.lambda_max_bound(0, 0.05)
        prop.set_state(0, None)
        prop.step_taylor(pulse, 0.0, dt, 8, 9)
        out.append(prop.get_state(0))
        prop.close()
    for o in out[1:]:
        assert np.array_equal(o, out[0])


@pytest.mark.parametrize("kind", [0, 1, 2, 3])
def test_fused_degenerate_shapes(kind):
    # the smallest grids (N = 8, a single row lmax = 0, strips wider than the
    # grid), order 1 and order 2, zero steps: fused == per-term bit for bit,
    # and zero steps leave the state alone
    t = lib()
    say(f"fused kind {kind}: degenerate shapes")
    for n, lmax, stencil in ((8, 0, 3), (8, 3, 5), (63, 0, 5), (65, 2, 3)):
        grid = t.Grid(n, lmax, 0.1, stencil, t.FP64, 1.0, 0.4)
        pulse = t.Pulse(0.05, 0.3, 2.0, 0.0, 0.0)
        for order in (1, 2, 5):
            res = []
            for fuse in (0, min(order, 4)):
                prop = t.Propagator([grid], methods=((t.METHOD_TAYLOR, order),))
                dt = 0.5 * t.tdse_taylor_stability_limit(order) / prop.lambda_max_bound(0, 0.05)
                prop.set_taylor_fusion(fuse, 3, kind)
                prop.set_state(0, None)
                before = prop.get_state(0)
                prop.step_taylor(pulse, 1.0, dt, order, 0)
                assert np.array_equal(prop.get_state(0), before)
                prop.step_taylor(pulse, 1.0, dt, order, 7)
                res.append(prop.get_state(0))
                prop.close()
            assert np.array_equal(res[0], res[1]), (n, lmax, stencil, order)
