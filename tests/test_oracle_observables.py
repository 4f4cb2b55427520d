"""Pins of the oracle's observables, field and inputs.

Checks against the analytic 1s density of Fig. "1sHydroRad", orthonormality
of the bound eigenvectors, the parity selection rule for <z> of an
eigenstate, Ehrenfest's theorem during a pulse, the spatial-yield identity
p_i + p_b = norm (eq. Norm), norm conservation, and textbook unit
conversions and pulse properties.
"""
import math

import numpy as np
import pytest
from scipy.integrate import quad

import workloads


def test_initial_state_is_analytic_1s(orc):
    # Fig. "1sHydroRad": radial density 4 r^2 exp(-2 r); the grid-normalised
    # state approaches it as dr -> 0.
    for dr, tol in ((0.1, 2e-3), (0.02, 1e-4)):
        g = orc.Grid(n=int(40 / dr), lmax=2, dr=dr)
        psi, u0 = orc.initial_state(g)
        r = orc.radius(g)
        dens = np.abs(psi[:g.n]) ** 2
        assert np.max(np.abs(dens - 4 * r ** 2 * np.exp(-2 * r))) < tol
        assert np.all(psi[g.n:] == 0)
        assert g.dr * np.sum(dens) == pytest.approx(1.0, abs=1e-14)


def test_populations_of_eigenstates(orc):
    g = orc.Grid(n=1500, lmax=4, dr=0.1, stencil=5)
    setup = orc.obs_setup(g, r_ion=50.0)
    assert len(setup.state_l) == 15
    assert list(setup.state_n[:5]) == [1, 2, 3, 4, 5] and list(setup.state_l[5:9]) == [1] * 4
    for k in range(15):
        psi = np.zeros(g.size, dtype=np.complex128)
        l = setup.state_l[k]
        psi[l * g.n:(l + 1) * g.n] = setup.phi[k] * np.exp(0.3j)
        obs = orc.observables(g, orc.Pulse(), 0.0, setup, psi)
        pops = obs[orc.OBS_FIXED:]
        assert pops[k] == pytest.approx(1.0, abs=1e-12)
        assert np.delete(pops, k).max() < 1e-20
        assert obs[4] == pytest.approx(1.0, abs=1e-12)
        assert abs(obs[6]) == 0.0                  # single partial wave: no dipole
    psi0, _ = orc.initial_state(g)
    obs = orc.observables(g, orc.Pulse(), 0.0, setup, psi0)
    assert obs[3] == pytest.approx(1.0, abs=1e-14)          # p_g of psi(0) itself
    assert obs[8] > 0.99 and obs[8] < 1.0                   # analytic vs grid 1s


def test_dipole_zero_for_field_free_eigenstate_of_coupled_grid(orc):
    # A field-free eigenstate has definite parity, so <z> = 0 even when it is
    # spread over several partial waves of equal parity.
    g = orc.Grid(n=800, lmax=4, dr=0.1)
    setup = orc.obs_setup(g, r_ion=30.0)
    psi = np.zeros(g.size, dtype=np.complex128)
    psi[0:g.n] = setup.phi[1]                  # 2s
    psi[2 * g.n:3 * g.n] = setup.phi[9]        # 3d, same parity
    obs = orc.observables(g, orc.Pulse(), 0.0, setup, psi)
    assert obs[6] == 0.0


def test_spatial_yield_identity_and_ehrenfest(orc):
    # During a pulse: p_i(r_b) + p_b(r_b) = norm with p_b the inner sum, the
    # norm is conserved to round-off, and the second time difference of <z>
    # tracks <z''> (Ehrenfest; grid and dt errors only).
    g = orc.Grid(n=400, lmax=6, dr=0.1)
    p = orc.Pulse(e0=0.1, omega=0.5, n_cycles=3.0, cep=0.0)
    setup = orc.obs_setup(g, r_ion=12.0)
    psi0, _ = orc.initial_state(g)
    dt = 1e-3                                   # stable: h_bound * dt ~ 2.3 < 3.39
    assert orc.h_bound(g, 0.1) * dt < 3.39
    psi, obs, _ = orc.propagate(g, p, orc.TAYLOR, 8, 0.0, dt, 4000, 1, setup, psi0)
    assert np.max(np.abs(obs[:, 2] - 1.0)) < 1e-11
    r = orc.radius(g)
    inner = g.dr * np.sum(np.abs(psi.reshape(g.lmax + 1, g.n)[:, r <= 12.0]) ** 2)
    assert obs[-1, 5] + inner == pytest.approx(obs[-1, 2], abs=1e-14)
    z = obs[:, 6]
    zdd = (z[2:] - 2 * z[1:-1] + z[:-2]) / dt ** 2
    acc = obs[1:-1, 7]
    assert np.max(np.abs(zdd - acc)) < 0.03 * np.max(np.abs(acc))
    assert np.max(np.abs(acc)) > 3e-3                         # the check is not vacuous


def test_field_shape(orc):
    p = orc.Pulse(e0=0.0534, omega=0.057, n_cycles=2.0, cep=workloads.SINE_CARRIER_CEP)
    T = 2 * math.pi * 2 / 0.057
    assert T == pytest.approx(220.4626, abs=1e-4)
    ts = np.linspace(-10, T + 10, 4001)
    e = np.array([orc.field(p, t) for t in ts])
    assert np.all(e[(ts < 0) | (ts > T)] == 0.0)
    assert np.max(np.abs(e)) <= 0.0534
    # Hann envelope: at the centre the field is E0 cos(w T/2 + phi)
    assert orc.field(p, T / 2) == pytest.approx(0.0534 * math.cos(0.057 * T / 2 + p.cep), rel=1e-14)
    # sine carrier, whole cycles: the pulse carries no net area, A(T) = 0
    area, _ = quad(lambda t: orc.field(p, t), 0, T, limit=400)
    assert abs(area) < 1e-10


def test_unit_conversions_textbook():
    assert workloads.e0_from_intensity(1e14) == pytest.approx(0.0533803, abs=2e-7)
    assert workloads.e0_from_intensity(2e14) == pytest.approx(0.0754911, abs=2e-7)
    assert workloads.omega_from_wavelength(800) == pytest.approx(0.0569542, abs=2e-7)
    assert workloads.omega_from_wavelength(1600) == pytest.approx(0.0284771, abs=2e-7)


def test_batch_recipe_is_deterministic():
    a = workloads.batch_members()
    b = workloads.batch_members()
    assert a == b and len(a) == 256
    assert all(4000 <= m.n <= 16000 and 16 <= m.lmax <= 64 and 2 <= m.n_cycles <= 6 for m in a)
    assert all(1e13 <= m.intensity <= 5e14 and 400 <= m.wavelength_nm <= 1600 for m in a)
    total = sum((m.lmax + 1) * m.n for m in a)
    assert total == 104_476_250


@pytest.mark.parametrize("theta", [0.3, 1.1])
def test_p_g_is_the_probability_of_the_initial_state(orc, theta):
    # eq. p_g read as a probability: for psi = e^{i a} cos(theta) u0 + sin(theta) v
    # with v orthogonal to u0 (built here by Gram-Schmidt in the grid inner
    # product dr * sum), p_g = cos^2(theta).  The amplitude |<u0|f_0>| would give
    # |cos(theta)| instead, and a missing dr or a missing square fails too.
    g = orc.Grid(n=700, lmax=3, dr=0.1, stencil=5)
    setup = orc.obs_setup(g, r_ion=30.0)
    _, u0 = orc.initial_state(g)
    r = orc.radius(g)
    w = (r ** 2 * np.exp(-0.5 * r) * (1.0 + 0.3j * np.sin(r))).astype(np.complex128)
    w -= g.dr * np.vdot(u0, w) * u0
    w /= math.sqrt(g.dr * np.vdot(w, w).real)
    assert abs(g.dr * np.vdot(u0, w)) < 1e-14
    psi = np.zeros(g.size, dtype=np.complex128)
    psi[:g.n] = np.exp(0.7j) * math.cos(theta) * u0 + math.sin(theta) * w
    # a component in another partial wave does not enter p_g
    psi[g.n:2 * g.n] = 0.2 * u0
    obs = orc.observables(g, orc.Pulse(), 0.0, setup, psi)
    assert obs[3] == pytest.approx(math.cos(theta) ** 2, abs=1e-13)
    assert abs(obs[3] - abs(math.cos(theta))) > 0.04     # the two readings differ here


def test_initial_state_for_nuclear_charge_two(orc):
    # Fig. "1sHydroRad" for a hydrogen-like ion of charge Z: the 1s radial
    # density is 4 Z^3 r^2 exp(-2 Z r); the grid state approaches it.
    z = 2.0
    for dr, tol in ((0.02, 2e-3), (0.005, 1.5e-4)):
        g = orc.Grid(n=int(20 / dr), lmax=1, dr=dr, z=z)
        psi, _ = orc.initial_state(g)
        r = orc.radius(g)
        dens = np.abs(psi[:g.n]) ** 2
        assert np.max(np.abs(dens - 4 * z ** 3 * r ** 2 * np.exp(-2 * z * r))) < tol
