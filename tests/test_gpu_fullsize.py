"""GPU parity at the full workload sizes, in the launch configuration the
benchmark uses.

- 1.3M unknowns (N = 20000, dr = 0.05, lmax = 64, 5-point), FP64, Taylor-8:
  three steps with observables, whole state and every record against the
  oracle (1e-12, the tolerances of test_gpu_parity).
- 25.7M unknowns (N = 100000, dr = 0.05, lmax = 256, 3-point), FP32 storage:
  one H application on an FP32-representable state against the oracle
  (element-wise round-off of one FP32 store), and two Taylor-8 steps against
  the FP64 oracle (two steps of FP32 rounding).
- the 256-member batch (104,476,250 unknowns, FP32 storage, per-member dt):
  one batched launch sequence, with four sampled members propagated by the
  oracle one by one.
Each runs with one launch per Horner term and with the execution shapes the
autotuners pick for the benchmark (wave-strip fused kernel, two-radii sweep).
"""
import math

import numpy as np
import pytest

import oracle
import workloads
from gpu_helpers import lib, obs_abs_tol, obs_columns, orc_grid, orc_pulse, read_vector, rel_err, say, series_ratio, to_fp32

pytestmark = pytest.mark.gpu


def shape(prop, sweep, fusion):
    if sweep is not None:
        prop.set_sweep_shape(*sweep)
    if fusion is not None:
        prop.set_taylor_fusion(*fusion)


@pytest.mark.parametrize("sweep,fusion", [(None, None), ((4, 1), (3, 8, 1)), ((2, 3), (4, 16, 0))])
def test_n20000_l64_fp64_taylor8_three_steps(sweep, fusion):
    t = lib()
    wl = workloads.WORKLOADS["hydrogen_n20000_l64_fp64_taylor8"]
    say(f"full size {wl.name}: 3 Taylor-8 steps vs oracle, sweep {sweep}, fusion {fusion}")
    g = t.Grid(wl.n, wl.lmax, wl.dr, wl.stencil, t.FP64, 1.0, wl.r_ion)
    prop = t.Propagator([g], methods=((t.METHOD_TAYLOR, 8),))
    shape(prop, sweep, fusion)
    prop.set_state(0, None)
    p = t.Pulse(wl.pulse.e0, wl.pulse.omega, wl.pulse.n_cycles, wl.pulse.cep, wl.pulse.t_on)
    t0 = 0.5 * wl.pulse.duration          # mid-pulse, strong field
    obs = prop.obs_buffer(3, 1)
    prop.step_taylor(p, t0, wl.dt, 8, 3, 1, obs)
    got = prop.get_state(0)
    gobs = obs.cpu().numpy()[0]
    prop.close()
    og = orc_grid(g)
    setup = oracle.obs_setup(og, r_ion=wl.r_ion)
    psi0, _ = oracle.initial_state(og)
    ref, robs, _ = oracle.propagate(og, orc_pulse(p), oracle.TAYLOR, 8, t0, wl.dt, 3, 1, setup, psi0)
    err = rel_err(got, ref)
    ratio = series_ratio(gobs[:, :obs_columns(setup)], robs, 1e-12, obs_abs_tol(og, setup, robs))
    say(f"  state {err:.2e}  observables worst ratio {ratio.max():.2e}")
    assert err < 1e-12 and np.all(ratio <= 1.0)


@pytest.mark.parametrize("sweep,fusion", [(None, None), ((8, 1), (4, 32, 1))])
def test_n100000_l256_fp32_apply_and_two_steps(sweep, fusion):
    t = lib()
    wl = workloads.WORKLOADS["hydrogen_n100000_l256_fp32_taylor8"]
    say(f"full size {wl.name}: apply_H and 2 Taylor-8 steps vs oracle, sweep {sweep}, fusion {fusion}")
    g = t.Grid(wl.n, wl.lmax, wl.dr, wl.stencil, t.FP32, 1.0, wl.r_ion)
    prop = t.Propagator([g], methods=((t.METHOD_TAYLOR, 8),))
    shape(prop, sweep, fusion)
    og = orc_grid(g)
    # a smooth FP32-representable state spread over every partial wave
    psi = to_fp32(workloads.random_state(3, wl.n, wl.lmax, smooth=True))
    prop.set_state(0, psi)
    out = prop.new_vector()
    e = 0.07
    prop.apply_H(e, prop.state, out)
    got = read_vector(prop, out, 0)
    ref = oracle.apply_h(og, e, psi)
    err = rel_err(got, ref)
    # one FP32 rounding of each output element
    elem = np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 1e-30 + 1e-7 * np.max(np.abs(ref))))
    say(f"  apply_H rel err {err:.2e}, worst element {elem:.2e}")
    assert err < 1.2e-7 and elem < 2e-7
    del out
    p = t.Pulse(wl.pulse.e0, wl.pulse.omega, wl.pulse.n_cycles, wl.pulse.cep, wl.pulse.t_on)
    t0 = 0.5 * wl.pulse.duration
    prop.set_state(0, None)
    prop.step_taylor(p, t0, wl.dt, 8, 2)
    got = prop.get_state(0)
    prop.close()
    psi0, _ = oracle.initial_state(og)
    ref, _, _ = oracle.propagate(og, orc_pulse(p), oracle.TAYLOR, 8, t0, wl.dt, 2, 0,
                                 oracle.ObsSetup(50.0, np.zeros(wl.n), np.zeros((0, wl.n)),
                                                 np.zeros(0, np.int32), np.zeros(0, np.int32)),
                                 to_fp32(psi0))
    err = rel_err(got, ref)
    say(f"  2 steps, FP32 storage vs FP64 oracle: {err:.2e}")
    assert err < 5e-7          # a few FP32 roundings of each element


@pytest.mark.parametrize("sweep,fusion", [(None, None), ((4, 3), (5, 64, 1))])
def test_batch_256_sampled_members(sweep, fusion):
    t = lib()
    members = workloads.batch_members()
    grids, pulses, dts = [], [], []
    for m in members:
        R = m.n * workloads.BATCH_DR
        grids.append(t.Grid(m.n, m.lmax, workloads.BATCH_DR, workloads.BATCH_STENCIL, t.FP32, 1.0,
                            workloads.BATCH_R_ION_FRACTION * R))
        pp = m.pulse
        pulses.append(t.Pulse(pp.e0, pp.omega, pp.n_cycles, pp.cep, pp.t_on))
    say(f"batch of {len(grids)} members, {sum((g.lmax + 1) * g.n for g in grids)} unknowns")
    prop = t.Propagator(grids, methods=((t.METHOD_TAYLOR, workloads.BATCH_ORDER),))
    shape(prop, sweep, fusion)
    y8 = t.tdse_taylor_stability_limit(workloads.BATCH_ORDER)
    for k, pp in enumerate(pulses):
        dts.append(workloads.BATCH_DT_SAFETY * y8 / prop.lambda_max_bound(k, abs(pp.e0)))
        prop.set_state(k, None)
    t0s = [0.5 * m.pulse.duration for m in members]
    steps, every = 3, 3
    obs = prop.obs_buffer(steps, every)
    prop.step_taylor(pulses, t0s, dts, workloads.BATCH_ORDER, steps, every, obs)
    gobs = obs.cpu().numpy()
    for k in (0, 17, 128, 255):
        m = members[k]
        got = prop.get_state(k)
        og = oracle.Grid(n=m.n, lmax=m.lmax, dr=workloads.BATCH_DR, stencil=workloads.BATCH_STENCIL)
        setup = oracle.obs_setup(og, r_ion=grids[k].r_ion)
        psi0, _ = oracle.initial_state(og)
        ref, robs, _ = oracle.propagate(og, orc_pulse(pulses[k]), oracle.TAYLOR, workloads.BATCH_ORDER,
                                        t0s[k], dts[k], steps, every, setup, to_fp32(psi0))
        err = rel_err(got, ref)
        norm_d = abs(gobs[k, -1, 2] - robs[-1, 2])
        pb = abs(gobs[k, -1, 4] - robs[-1, 4]) / robs[-1, 4]
        say(f"  member {k}: N={m.n} lmax={m.lmax} dt={dts[k]:.2e} state {err:.2e} "
            f"norm diff {norm_d:.2e} p_bound rel {pb:.2e}")
        assert err < 5e-7 and norm_d < 1e-6 and pb < 1e-5
    prop.close()


def test_n20000_l64_fp32_lanczos20_steps():
    # the Lanczos workload at full size: FP32 basis vectors and state, FP64
    # dots, re-orthogonalisation and exponential, against the FP64 oracle
    t = lib()
    wl = workloads.WORKLOADS["hydrogen_n20000_l64_fp32_lanczos20"]
    say(f"full size {wl.name}: 3 Lanczos-20 steps vs the FP64 oracle")
    g = t.Grid(wl.n, wl.lmax, wl.dr, wl.stencil, t.FP32, 1.0, wl.r_ion)
    prop = t.Propagator([g], methods=((t.METHOD_LANCZOS, wl.order),))
    prop.set_state(0, None)
    p = t.Pulse(wl.pulse.e0, wl.pulse.omega, wl.pulse.n_cycles, wl.pulse.cep, wl.pulse.t_on)
    t0 = 0.5 * wl.pulse.duration
    obs = prop.obs_buffer(3, 1)
    prop.step_lanczos(p, t0, wl.dt, wl.order, 3, 1, obs)
    got = prop.get_state(0)
    gobs = obs.cpu().numpy()[0]
    prop.close()
    og = orc_grid(g)
    setup = oracle.obs_setup(og, r_ion=wl.r_ion)
    psi0, _ = oracle.initial_state(og)
    ref, robs, _ = oracle.propagate(og, orc_pulse(p), oracle.LANCZOS, wl.order, t0, wl.dt, 3, 1, setup,
                                    to_fp32(psi0))
    err = rel_err(got, ref)
    norm_d = np.max(np.abs(gobs[:, 2] - robs[:, 2]))
    pb = np.max(np.abs(gobs[:, 4] - robs[:, 4]) / robs[:, 4])
    say(f"  state {err:.2e}  norm diff {norm_d:.2e}  p_bound rel {pb:.2e}")
    # FP32 storage of the state and of 20 basis vectors per step: a few FP32
    # roundings per element and step
    assert err < 2e-6 and norm_d < 1e-6 and pb < 1e-5
