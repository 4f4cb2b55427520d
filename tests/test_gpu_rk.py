"""GPU parity of the tableau Runge-Kutta propagator (appendix "Runge-Kutta",
eq. RKDeriv) against the FP64 oracle: Euler, classic RK4, Fehlberg 4(5),
Cash-Karp 5(4), Dormand-Prince 5(4), Merson 4(3).

FP64: state within 1e-12 relative, observable records within the parity
tolerance of the other methods, and the passive truncation estimate sigma =
sum_n sigma_n within 1e-10 relative plus the round-off of its cancellation:
sigma_n comes from the pair's difference dt sum (b_i - bhat_i) k_i, whose
terms cancel to O((lambda dt)^5), so each step's deviation carries an absolute
round-off of ~eps times the state's rms (and, with 48-bit storage, of 2^-35
lambda_max dt times the rms from the stored stage vectors).  The Fehlberg and
Cash-Karp pairs carry their fifth-order solution, whose stability polynomial
leaves the imaginary axis near 0: their steps are tiny and their sigma sits
near that floor.  48-bit storage: state within 1e-9, records within 1e-9
relative plus the 2^-36 rounding of the terms of each sum (norm-like sums
<= 1; the dipole's r weights up to r_max, the acceleration's 1/r^2 up to
1/dr^2), sigma within 1e-6.  Uneven batches, both stencils.
"""
import numpy as np
import pytest

import oracle
import workloads
from gpu_helpers import (lib, obs_abs_tol, obs_columns, orc_pulse, rel_err, say, series_ratio, to_fp48)

pytestmark = pytest.mark.gpu

NAMES = {0: "Euler", 1: "RK4", 2: "Fehlberg45", 3: "CashKarp", 4: "DormandPrince", 5: "Merson"}


@pytest.mark.parametrize("prec", [0, 2])
@pytest.mark.parametrize("stencil", [3, 5])
@pytest.mark.parametrize("method", [0, 1, 2, 3, 4, 5])
def test_rk_tableau_steps_match_the_oracle(method, stencil, prec):
    import torch
    t = lib()
    grids = [(520, 7, 0.1, stencil, 12.0), (1299, 11, 0.1, stencil, 40.0), (257, 0, 0.2, stencil, 10.0)]
    pulses = [t.Pulse(0.06, 0.35, 2.0, 0.2, 0.0), t.Pulse(-0.04, 0.5, 3.0, 1.0, 0.0),
              t.Pulse(0.08, 0.2, 1.0, -0.5, 0.0)]
    steps, every = 30, 10
    y = t.tdse_rk_stability_limit(method)
    say(f"rk {NAMES[method]} stencil={stencil} prec={prec}: 3 uneven grids, {steps} steps (limit y={y:.4f})")
    prop = t.Propagator([t.Grid(n, lm, dr, st, prec, 1.0, rion) for (n, lm, dr, st, rion) in grids],
                        methods=((t.METHOD_RK_TABLEAU, method),), graphs=True)
    psis, dts = [], []
    for k, (n, lm, dr, st, rion) in enumerate(grids):
        v = workloads.random_state(60 + k, n, lm)
        v = v / np.sqrt(dr * np.vdot(v, v).real)
        psis.append(to_fp48(v) if prec == 2 else v)
        prop.set_state(k, psis[k])
        lam = prop.lambda_max_bound(k, abs(pulses[k].e0))
        dts.append(0.8 * y / lam if method != 0 else 1e-10)
    obs = prop.obs_buffer(steps, every)
    sigma = torch.zeros(len(grids), dtype=torch.float64, device="cuda")
    prop.step_rk(pulses, 0.25, dts, method, steps, every, obs, sigma)
    states = [prop.get_state(k) for k in range(len(grids))]
    o = obs.cpu().numpy()
    sg = sigma.cpu().numpy()
    prop.close()
    tol = 1e-12 if prec == 0 else 1e-9
    stol = 1e-10 if prec == 0 else 1e-6
    for k, (n, lm, dr, st, rion) in enumerate(grids):
        g = oracle.Grid(n=n, lmax=lm, dr=dr, stencil=st)
        setup = oracle.obs_setup(g, r_ion=rion)
        ref, robs, rsig = oracle.propagate_rk(g, orc_pulse(pulses[k]), method, 0.25, dts[k], steps, every, setup,
                                              psis[k])
        err = rel_err(states[k], ref)
        atol = obs_abs_tol(g, setup, robs)
        if prec == 2:
            r_max = n * dr
            floor = np.full_like(atol, 2.0 ** -36)
            floor[6], floor[7] = 2.0 ** -36 * 2 * r_max, 2.0 ** -36 * 2 / dr ** 2
            atol = atol + floor
        ratio = series_ratio(o[k][:, :obs_columns(setup)], robs, tol, atol)
        rms = np.sqrt(np.mean(np.abs(psis[k]) ** 2))
        lam_dt = dts[k] * oracle.h_bound(g, abs(pulses[k].e0))
        sfloor = steps * rms * (4 * np.finfo(float).eps + (2.0 ** -35 * lam_dt if prec == 2 else 0.0))
        serr = abs(sg[k] - rsig) / (stol * rsig + sfloor)
        say(f"  instance {k}: state {err:.2e}, records worst ratio {ratio.max():.2e}, sigma {sg[k]:.3e} "
            f"(oracle {rsig:.3e}, ratio to tolerance {serr:.1e}), lambda dt {lam_dt:.2e}")
        assert err < tol
        assert np.all(ratio <= 1.0), ratio
        assert np.all(o[k][:, 0] == robs[:, 0]) and np.all(o[k][:, 1] == robs[:, 1])
        if method in (0, 1):
            assert sg[k] == 0.0 and rsig == 0.0
        else:
            assert serr <= 1.0


def test_rk_classic4_tableau_matches_the_rk4_launches():
    # the tableau form of RK4 and the dedicated RK4 kernels compute the same
    # step (to FP64 rounding: the stage combinations are summed differently)
    t = lib()
    grid = (700, 9, 0.1, 5, 20.0)
    p = t.Pulse(0.06, 0.35, 2.0, 0.2, 0.0)
    res = []
    for tableau in (True, False):
        prop = t.Propagator([t.Grid(*grid[:4], 0, 1.0, grid[4])],
                            methods=((t.METHOD_RK_TABLEAU, 1), (t.METHOD_RK4, 4)))
        prop.set_state(0, None)
        dt = 0.5 * t.tdse_taylor_stability_limit(4) / prop.lambda_max_bound(0, 0.06)
        if tableau:
            prop.step_rk(p, 0.0, dt, 1, 40)
        else:
            prop.step_rk4(p, 0.0, dt, 40)
        res.append(prop.get_state(0))
        prop.close()
    say(f"rk tableau RK4 vs RK4 kernels: {rel_err(res[0], res[1]):.2e}")
    assert rel_err(res[0], res[1]) < 1e-13


def test_rk_rejects_an_unstable_step():
    t = lib()
    prop = t.Propagator([t.Grid(300, 2, 0.1, 3, 0, 1.0, 10.0)], methods=((t.METHOD_RK_TABLEAU, 4),))
    prop.set_state(0, None)
    before = prop.get_state(0)
    lam = prop.lambda_max_bound(0, 0.05)
    with pytest.raises(t.TdseError) as err:
        prop.step_rk(t.Pulse(0.05, 0.3, 2.0, 0.0, 0.0), 0.0, 1.01 * t.tdse_rk_stability_limit(4) / lam, 4, 3)
    assert err.value.code == -4
    assert np.array_equal(prop.get_state(0), before)
    prop.close()
