"""GPU parity of the absorbing boundary (Sec. 2, "Absorbing potential": the
mask 1 - cos^p[(pi/2)(1 - r/r_b)] after every step) and the flux yield (Sec.
4, eq. yield in the length gauge: the trapezoid time integral of the radial
current at one radius) against the FP64 oracle.

A batch of four uneven grids starts from outgoing packets (an l-mixed Gaussian
moving out at k = 1.5 au plus a bound part), run long enough for the packets
to cross the flux sphere and reach the absorber: two instances absorb and
count the flux, one counts the flux without an absorber, one has neither
(the plain step).  Taylor-8 (wave strips; with the absorber on the
observables take their own pass), RK4 (fused strips) and Lanczos (m = 16,
converged: lambda_max dt <= 2), both stencils, FP64 and 48-bit storage.
Tolerances: state max(1e-12, steps eps) (FP64: an eps-sized rounding
difference per step, coherent at worst over the thousands of steps the
packets need; Lanczos: (m + lambda_max dt) eps per step, the rounding of the
m-vector recombination and the phase error of the two sides' different
exponentials of T) / 4 sqrt(steps) 2^-36 (48-bit: one rounding at 2^-37 of every stored
element per step, independent from step to step) relative; records as the other parity tests (48-bit: plus the 2^-36 rounding
of each summed term);
yield max(1e-11, the state tolerance) relative plus 1e-15 (FP64) / 1e-8 plus
1e-12 (48-bit): the current's difference quotient loses log10(1/(k dr)) < 1
digit.

Plus a property at a larger size (N = 2000, dr = 0.05, lmax = 32, a batch of
four, Taylor-8 in the tuned launch shape, 3-point stencil): the discrete
continuity equation of the 3-point Hamiltonian balances the flux yield
against the probability moved beyond the sphere and the probability the
mask removed, to the trapezoid rule's O(dt^2).
"""
import numpy as np
import pytest

import oracle
import workloads
from gpu_helpers import lib, obs_abs_tol, obs_columns, orc_pulse, rel_err, say, series_ratio, to_fp48

pytestmark = pytest.mark.gpu

# (n, lmax, dr, r_ion, r_abs, p_abs, i_flux)
# coarse grids (k dr <= 0.3 for the packet) keep the oracle's runs short
GRIDS = [(350, 3, 0.2, 12.0, 65.0, 200.0, 174), (451, 5, 0.16, 20.0, 70.0, 100.0, 174),
         (200, 0, 0.3, 10.0, 0.0, 0.0, -1), (320, 2, 0.2, 15.0, 0.0, 0.0, 149)]


@pytest.mark.parametrize("prec", [0, 2])
@pytest.mark.parametrize("stencil", [3, 5])
@pytest.mark.parametrize("method", ["taylor", "rk4", "lanczos"])
def test_absorber_and_flux_match_the_oracle(method, stencil, prec):
    import torch
    t = lib()
    mcode = {"taylor": (t.METHOD_TAYLOR, 8), "rk4": (t.METHOD_RK4, 4), "lanczos": (t.METHOD_LANCZOS, 16)}[method]
    pulses = [t.Pulse(0.03, 0.3, 2.0, 0.0, 0.0), t.Pulse(-0.02, 0.5, 3.0, 0.7, 0.0),
              t.Pulse(0.04, 0.2, 1.0, 0.0, 0.0), t.Pulse(0.025, 0.4, 2.0, -0.3, 0.0)]
    prop = t.Propagator([t.Grid(n, lm, dr, stencil, prec, 1.0, rion) for (n, lm, dr, rion, _, _, _) in GRIDS],
                        methods=(mcode,), graphs=True)
    if method == "taylor":
        prop.set_taylor_fusion(8, 16, 1)        # wave strips, one launch per step
    psis, dts = [], []
    for k, (n, lm, dr, *_rest) in enumerate(GRIDS):
        v = workloads.outgoing_packet(70 + k, n, lm, dr)
        psis.append(to_fp48(v) if prec == 2 else v)
        prop.set_state(k, psis[k])
        lam = prop.lambda_max_bound(k, abs(pulses[k].e0))
        if method == "taylor":
            dts.append(0.8 * t.tdse_taylor_stability_limit(8) / lam)
        elif method == "rk4":
            dts.append(0.8 * t.tdse_taylor_stability_limit(4) / lam)
        else:
            dts.append(2.0 / lam)
    # the packet (k = 1.5 au) from r0 = 20 au crosses the flux spheres at
    # 28-35 au within 10 au of time; the masks remove a part of more than
    # 1e-3 per step from ~50 au on, which its centre reaches at 20 au
    steps = int(np.ceil(28.0 / min(dts) / 100.0)) * 100
    every = steps // 10
    prop.set_absorber([g[4] for g in GRIDS], [g[5] for g in GRIDS])
    prop.set_flux([g[6] for g in GRIDS])
    say(f"absorber {method} stencil={stencil} prec={prec}: 4 uneven grids, {steps} steps, records every {every}")
    obs = prop.obs_buffer(steps, every)
    half = steps // 2
    # two calls: the yields carry over, the second call starts its
    # trapezoid from the current of the state it starts from
    for s0, cnt in ((0, half), (half, steps - half)):
        o_view = obs[:, s0 // every:(s0 + cnt) // every]
        buf = prop.obs_buffer(cnt, every)
        t0 = [s0 * dt for dt in dts]
        if method == "taylor":
            prop.step_taylor(pulses, t0, dts, 8, cnt, every, buf)
        elif method == "rk4":
            prop.step_rk4(pulses, t0, dts, cnt, every, buf)
        else:
            prop.step_lanczos(pulses, t0, dts, 16, cnt, every, buf)
        o_view.copy_(buf)
    y = prop.flux_yield()
    states = [prop.get_state(k) for k in range(len(GRIDS))]
    o = obs.cpu().numpy()
    prop.close()
    # FP64: the two sides round each step differently (another operation
    # order), a relative difference of order eps per step that can add up
    # coherently over the ~3e4 steps; 48-bit storage rounds every stored
    # element at 2^-37 relative once per step (and launch): independent
    # roundings add up as sqrt(steps)
    # Lanczos adds per step the rounding of its m-vector recombination and
    # the two sides' different exponentials of T (eps lambda_max dt, R8)
    eps = np.finfo(float).eps
    per_step = eps * (1.0 if method != "lanczos" else mcode[1] + 2.0)
    tol = max(1e-12, steps * per_step) if prec == 0 else 4.0 * np.sqrt(steps) * 2.0 ** -36
    ytol = (max(1e-11, tol), 1e-15) if prec == 0 else (1e-8, 1e-12)
    ocode = {"taylor": oracle.TAYLOR, "rk4": oracle.RK4, "lanczos": oracle.LANCZOS}[method]
    for k, (n, lm, dr, rion, r_abs, p_abs, j) in enumerate(GRIDS):
        g = oracle.Grid(n=n, lmax=lm, dr=dr, stencil=stencil)
        setup = oracle.obs_setup(g, r_ion=rion)
        ref_a, rob_a, _, f_a = oracle.propagate_abs(g, orc_pulse(pulses[k]), ocode, mcode[1], 0.0, dts[k], half,
                                                    every, setup, psis[k], r_abs=r_abs, p_abs=p_abs, flux_j=j)
        ref, rob_b, _, f_b = oracle.propagate_abs(g, orc_pulse(pulses[k]), ocode, mcode[1], half * dts[k], dts[k],
                                                  steps - half, every, setup, ref_a, r_abs=r_abs, p_abs=p_abs,
                                                  flux_j=j)
        robs = np.concatenate([rob_a, rob_b])
        yref = f_a + f_b
        err = rel_err(states[k], ref)
        # a record is a quadratic form f* A f: a state error d moves it by up
        # to 2 ||A|| ||f|| d, with ||A|| <= 1 for the norm-like sums and
        # populations, r_max for the dipole and 2/dr^2 for the acceleration
        # sum; d = the state tolerance (plus, 48-bit, the 2^-36 rounding of
        # each summed term)
        w = np.ones_like(obs_abs_tol(g, setup, robs))
        w[0] = w[1] = 0.0
        w[6], w[7] = n * dr, 2.0 / dr ** 2
        atol = obs_abs_tol(g, setup, robs) + 2.0 * tol * w
        if prec == 2:
            atol = atol + 2.0 ** -36 * np.maximum(w, 1.0) * 2.0
        ratio = series_ratio(o[k][:, :obs_columns(setup)], robs, tol, atol)
        norm_end = robs[-1, 2]
        say(f"  instance {k}: state {err:.2e}, records worst ratio {ratio.max():.2e}, yield {y[k]:.12f} "
            f"(oracle {yref:.12f}, diff {abs(y[k] - yref):.1e}), final norm {norm_end:.6f}")
        assert err < tol
        assert np.all(ratio <= 1.0), ratio
        assert abs(y[k] - yref) <= ytol[0] * abs(yref) + ytol[1]
        if j < 0:
            assert y[k] == 0.0
        else:
            assert yref > 0.05
        if r_abs > 0:
            assert norm_end < 0.9       # the absorber took a part of the packet


def test_flux_balance_at_a_larger_size():
    t = lib()
    n, lm, dr = 2000, 32, 0.05
    j, r_abs, p_abs = 799, 95.0, 200.0          # flux sphere at 40 au, absorbing from ~60 au
    nb = 4
    prop = t.Propagator([t.Grid(n, lm, dr, 3, t.FP64, 1.0, 30.0) for _ in range(nb)],
                        methods=((t.METHOD_TAYLOR, 8), (t.METHOD_TUNE, 0)), graphs=True)
    prop.autotune_taylor(8)
    psi0 = [workloads.outgoing_packet(90 + k, n, lm, dr) for k in range(nb)]
    for k in range(nb):
        prop.set_state(k, psi0[k])
    pulses = [t.Pulse(0.02 * (k + 1), 0.3, 2.0, 0.0, 0.0) for k in range(nb)]
    lam = max(prop.lambda_max_bound(k, 0.08) for k in range(nb))
    dt = 0.8 * t.tdse_taylor_stability_limit(8) / lam
    steps = int(round(45.0 / dt))
    prop.set_absorber(r_abs, p_abs)
    prop.set_flux(j)
    say(f"flux balance: batch {nb} x N={n}, lmax={lm}, Taylor-8 fusion {prop.taylor_fusion}, {steps} steps of {dt:.2e}")
    prop.step_taylor(pulses, 0.0, dt, 8, steps)
    y = prop.flux_yield()
    for k in range(nb):
        psi = prop.get_state(k)
        f, f0 = psi.reshape(lm + 1, n), psi0[k].reshape(lm + 1, n)
        outside = lambda a: dr * (np.sum(np.abs(a[:, j + 1:]) ** 2) + 0.5 * np.sum(np.abs(a[:, j]) ** 2))
        absorbed = 1.0 - dr * np.vdot(psi, psi).real
        moved = outside(f) - outside(f0)
        say(f"  instance {k}: yield {y[k]:.8f}, moved {moved:.8f}, absorbed {absorbed:.8f}, "
            f"balance {y[k] - moved - absorbed:.2e}")
        assert absorbed > 0.2
        assert abs(y[k] - (moved + absorbed)) < 1e-6


def test_absorber_and_flux_reject_bad_arguments():
    t = lib()
    prop = t.Propagator([t.Grid(300, 2, 0.1, 3, 0, 1.0, 10.0), t.Grid(200, 1, 0.1, 3, 0, 1.0, 10.0)])
    for r_abs, p_abs in (([50.0, 0.0], [0.0, 0.0]), ([float("nan"), 0.0], [1.0, 1.0]),
                         ([20.0, 10.0], [100.0, -1.0])):
        with pytest.raises(t.TdseError) as err:
            prop.set_absorber(r_abs, p_abs)
        assert err.value.code == -1
    for i_flux in ([300, -1], [-2, 0], [0, 200]):
        with pytest.raises(t.TdseError):
            prop.set_flux(i_flux)
    # r_abs <= 0 switches an instance off; the last index is allowed
    prop.set_absorber([0.0, -1.0], [0.0, 0.0])
    prop.set_flux([299, 199])
    assert np.array_equal(prop.flux_yield(), np.zeros(2))
    prop.close()
