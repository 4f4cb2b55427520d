"""Pins of the oracle's velocity gauge: the V form of the coupling (Sec. 2,
the radial TDSE in the two gauges, with the fourth-order first derivative of
the finite-difference formulation) and the vector potential (Sec. 3, eq.
VectorStep: A~ = A/c advanced by 5-point Gauss-Legendre; the SineA pulse of
eq. VecSinSinCosE).

- vector potential: the accumulated quadrature against the closed form of the
  SineA pulse, A~ = -E0 sin^2(W tau) sin(w tau + phi); the SineA field against
  -dA~/dt of that closed form; the sine-squared-E pulse against adaptive
  quadrature (scipy); per-step increments summing to the value at the end;
- coupling: applied to the partial waves of a Cartesian test function (a
  displaced Gaussian, projected on Y_l0 by Gauss-Legendre quadrature in
  cos(theta)), against the partial waves of -i A~ d/dz of the same function
  differentiated analytically; the error falls at the stencil's order.  This
  fixes the signs of the l/r terms: the printed ones (d/dr + l/r on f_{l-1})
  would give 2g + r g' for p_z on an s wave r g(r) instead of r g';
- H in the velocity gauge is Hermitian;
- gauge invariance: from 1s through a SineA pulse (A(T) = 0) the length and
  velocity gauges give the same populations after the pulse, and the same
  norm, dipole, p_ion and flux yield at every record (|psi|^2 and the current
  do not depend on the gauge), to the discretisation error.  The populations
  do not see the sign of A (parity); the dipole does.
"""
import math

import numpy as np
import pytest
from scipy.integrate import quad


def sine_a(orc, e0=0.07, omega=0.4, nc=3.0, cep=0.3, t_on=1.0):
    return orc.Pulse(e0, omega, nc, cep, t_on, orc.SINE_SQR_A)


def a_closed(p, t):
    T = 2 * math.pi * p.n_cycles / p.omega
    tau = t - p.t_on
    if tau <= 0 or tau >= T:
        return 0.0
    return -p.e0 * math.sin(math.pi * tau / T) ** 2 * math.sin(p.omega * tau + p.cep)


def test_vector_potential_of_sine_a_matches_its_closed_form(orc):
    p = sine_a(orc)
    T = 2 * math.pi * p.n_cycles / p.omega
    for t in np.linspace(0.0, p.t_on + T, 37):
        assert abs(orc.vector_potential_at(p, t, 0.05) - a_closed(p, t)) < 1e-13
    # past the end the piece holding t_on + T integrates across the kink of
    # E' there: a quadrature error of order dt^2 |E'| dt, still about 0
    for t in (p.t_on + T + 0.13, p.t_on + T + 3.0):
        assert abs(orc.vector_potential_at(p, t, 0.05)) < 1e-8
    # E = -dA~/dt: a fourth-order central difference of the closed form
    h = 1e-3
    for t in np.linspace(p.t_on + 0.3, p.t_on + T - 0.3, 23):
        d = (-a_closed(p, t + 2 * h) + 8 * a_closed(p, t + h) - 8 * a_closed(p, t - h) + a_closed(p, t - 2 * h))
        assert abs(orc.field(p, t) + d / (12 * h)) < 1e-11


def test_vector_potential_of_sine_squared_field_matches_adaptive_quadrature(orc):
    p = orc.Pulse(0.05, 0.45, 2.5, -0.7, 0.5)
    T = 2 * math.pi * p.n_cycles / p.omega
    for t in np.linspace(p.t_on + 0.1, p.t_on + T + 1.0, 17):
        ref = -quad(lambda x: orc.field(p, x), p.t_on, min(t, p.t_on + T), epsabs=1e-14, epsrel=1e-13,
                    limit=400)[0]
        assert abs(orc.vector_potential_at(p, t, 0.02) - ref) < 1e-12
    # the per-step increments add up to the value at the end of the steps
    dt, a = 0.05, 0.0
    for s in range(400):
        a += orc.vector_potential_step(p, p.t_on + s * dt, dt)
    assert abs(a - orc.vector_potential_at(p, p.t_on + 400 * dt, dt)) < 1e-15


def partial_waves(fun, r, lmax, nmu=96):
    """f_l(r) = r * int fun(r, mu) Y_l0 dOmega by Gauss-Legendre in mu."""
    mu, w = np.polynomial.legendre.leggauss(nmu)
    out = np.zeros((lmax + 1, r.size), dtype=complex)
    vals = fun(r[:, None], mu[None, :])
    for l in range(lmax + 1):
        ylm = math.sqrt((2 * l + 1) / (4 * math.pi)) * np.polynomial.legendre.Legendre.basis(l)(mu)
        out[l] = r * (2 * math.pi * ((vals * ylm[None, :]) @ w))
    return out


@pytest.mark.parametrize("stencil,order", [(3, 2), (5, 4)])
def test_coupling_is_a_times_p_z_on_partial_waves(orc, stencil, order):
    alpha, z0, a = 0.8, 2.5, 0.37
    psi = lambda r, mu: np.exp(-alpha * (r * r - 2 * r * z0 * mu + z0 * z0)) * (1 + 0.3j * r * mu)
    # d/dz at fixed x, y: z = r mu
    dpsi = lambda r, mu: psi(r, mu) * (-2 * alpha * (r * mu - z0)) + \
        np.exp(-alpha * (r * r - 2 * r * z0 * mu + z0 * z0)) * 0.3j
    errs = []
    lmax = 12
    for dr in (0.1, 0.05):
        n = int(round(14.0 / dr))
        g = orc.Grid(n=n, lmax=lmax, dr=dr, stencil=stencil, gauge=orc.VELOCITY)
        r = (np.arange(n) + 1) * dr
        f = partial_waves(psi, r, lmax)
        want = -1j * a * partial_waves(dpsi, r, lmax)
        got = (orc.apply_h(g, a, f.ravel()) - orc.apply_h(g, 0.0, f.ravel())).reshape(lmax + 1, n)
        # rows below lmax see both neighbours (the top row lacks l = lmax + 1);
        # the 5-point derivative at r_1 reaches r = -dr, where the zero of
        # the box's padding stands for the odd continuation -f(dr): an
        # O(f'(0)) error of that one point, left out here
        i0 = 0 if stencil == 3 else 1
        errs.append(np.max(np.abs(got[:lmax, i0:] - want[:lmax, i0:])) / np.max(np.abs(want[:lmax])))
    rate = math.log2(errs[0] / errs[1])
    assert errs[1] < (2e-3 if order == 2 else 2e-5), errs
    assert abs(rate - order) < 0.3, (errs, rate)


def test_velocity_gauge_h_is_hermitian(orc):
    rng = np.random.default_rng(3)
    for stencil in (3, 5):
        g = orc.Grid(n=150, lmax=6, dr=0.1, stencil=stencil, gauge=orc.VELOCITY)
        u = rng.standard_normal(g.size) + 1j * rng.standard_normal(g.size)
        v = rng.standard_normal(g.size) + 1j * rng.standard_normal(g.size)
        hu, hv = orc.apply_h(g, 0.8, u), orc.apply_h(g, 0.8, v)
        lhs, rhs = np.vdot(u, hv), np.conj(np.vdot(v, hu))
        scale = np.linalg.norm(u) * np.linalg.norm(v) * orc.h_bound(g, 0.8)
        assert abs(lhs - rhs) < 1e-14 * scale
        # the Gershgorin bound covers the spectrum: ||H v|| <= bound ||v||
        assert np.linalg.norm(hv) <= orc.h_bound(g, 0.8) * np.linalg.norm(v)


@pytest.mark.parametrize("stencil,tol_pop,tol_dip,tol_flux", [(3, 5e-6, 5e-5, 3e-3), (5, 2e-6, 1e-5, 1e-4)])
def test_gauges_agree_through_a_sine_a_pulse(orc, stencil, tol_pop, tol_dip, tol_flux):
    dr, n, lmax = 0.2, 300, 8
    res = {}
    for gauge in (orc.LENGTH, orc.VELOCITY):
        g = orc.Grid(n=n, lmax=lmax, dr=dr, stencil=stencil, gauge=gauge)
        setup = orc.obs_setup(g, r_ion=15.0)
        psi0, _ = orc.initial_state(g)
        p = orc.Pulse(0.1, 0.5, 2.0, 0.0, 0.0, orc.SINE_SQR_A)
        gl = orc.Grid(n=n, lmax=lmax, dr=dr, stencil=stencil)
        dt = 0.8 * 3.3961 / orc.h_bound(gl, 0.2)
        steps = int(math.ceil(2 * math.pi * 2.0 / 0.5 / dt / 20)) * 20
        _, obs, _, flux = orc.propagate_abs(g, p, orc.TAYLOR, 8, 0.0, dt, steps, steps // 20, setup, psi0,
                                            flux_j=int(round(20.0 / dr)) - 1)
        res[gauge] = obs, flux
    (oL, fL), (oV, fV) = res[orc.LENGTH], res[orc.VELOCITY]
    assert 0.05 < 1.0 - oL[-1, 3] < 0.9                          # the pulse moved the atom
    assert np.max(np.abs(oL[-1, 8:] - oV[-1, 8:])) < tol_pop     # populations after the pulse
    assert abs(oL[-1, 3] - oV[-1, 3]) < tol_pop                 # p_g
    for col in (2, 5, 6):                                       # norm, p_ion, dipole at every record
        assert np.max(np.abs(oL[:, col] - oV[:, col])) < tol_dip * max(1.0, np.max(np.abs(oL[:, col])))
    assert fL > 1e-5 and abs(fL - fV) < tol_flux * fL


def test_velocity_gauge_dipole_sees_the_sign_of_a(orc):
    # the populations are the same for A and -A (parity), the dipole is not:
    # the V run with the field reversed differs from the L run at O(1)
    dr, n = 0.2, 200
    out = []
    for gauge, sign in ((orc.LENGTH, 1.0), (orc.VELOCITY, -1.0)):
        g = orc.Grid(n=n, lmax=6, dr=dr, stencil=3, gauge=gauge)
        setup = orc.obs_setup(g, r_ion=15.0)
        psi0, _ = orc.initial_state(g)
        p = orc.Pulse(sign * 0.1, 0.5, 1.0, 0.0, 0.0, orc.SINE_SQR_A)
        dt = 0.8 * 3.3961 / orc.h_bound(orc.Grid(n=n, lmax=6, dr=dr, stencil=3), 0.2)
        steps = int(math.ceil(4 * math.pi / dt / 10)) * 10
        out.append(orc.propagate(g, p, orc.TAYLOR, 8, 0.0, dt, steps, steps // 10, setup, psi0)[1])
    assert np.max(np.abs(out[0][:, 6] - out[1][:, 6])) > 1e-2


def test_velocity_gauge_steps_agree_across_methods(orc):
    # RK4, its tableau form and Taylor-4 without field take the same step;
    # with the field, RK4 by the tableau equals the dedicated RK4 step
    g = orc.Grid(n=200, lmax=4, dr=0.1, stencil=5, gauge=orc.VELOCITY)
    p = orc.Pulse(0.3, 0.5, 2.0, 0.2, 0.0, orc.SINE_SQR_A)
    setup = orc.obs_setup(g, r_ion=10.0)
    rng = np.random.default_rng(8)
    psi0 = rng.standard_normal(g.size) + 1j * rng.standard_normal(g.size)
    a, _, _ = orc.propagate(g, p, orc.RK4, 4, 3.0, 1e-3, 30, 0, setup, psi0)
    b, _, _ = orc.propagate_rk(g, p, orc.RK_CLASSIC4, 3.0, 1e-3, 30, 0, setup, psi0)
    assert np.linalg.norm(a - b) / np.linalg.norm(a) < 1e-14
    # a single public RK4 step from t starts from A~(t) by the composite rule
    c = orc.rk4_step(g, p, 3.0, 1e-3, psi0) if hasattr(orc, "rk4_step") else None
    if c is not None:
        d, _, _ = orc.propagate(g, p, orc.RK4, 4, 3.0, 1e-3, 1, 0, setup, psi0)
        assert np.linalg.norm(c - d) / np.linalg.norm(d) < 1e-15
