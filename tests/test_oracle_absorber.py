"""Pins of the oracle's absorbing potential (Sec. 2.1) and flux yield (Sec. 4,
eq. flux and eq. yield in the length gauge).

The discrete radial current is pinned by the continuity equation of the
finite-difference Hamiltonian itself: with the 3-point stencil, the centred
current J_j = sum_l Im[f_l,j^* (f_l,j+1 - f_l,j-1) / (2 dr)] at point j is the
mean of the exact staggered fluxes through j -+ 1/2, so its time integral
equals the change of P_{>j} + (dr/2) sum_l |f_l,j|^2 (the field couples
partial waves at the same radius and moves no probability radially).  With
the absorbing mask, which is 1 to machine precision inside the flux radius,
the absorbed probability closes the balance:
int J dt = Delta(P_{>j} + dr/2 |f_j|^2) + (N(0) - N(T)).  The 5-point current
(4th-order point derivative) is not the stencil's conservative flux; it meets
the same balance to O(dr^4) for a smooth packet.  The mask itself is 1 at the
origin, 0 at r_b and decreasing in between.
"""
import math

import numpy as np
import pytest


def packet(orc, g, r0=20.0, sigma=3.0, k=1.5, lmax_fill=1):
    """An outgoing Gaussian packet (momentum k) in the lowest partial waves."""
    r = (np.arange(g.n) + 1) * g.dr
    f = np.exp(-((r - r0) ** 2) / (2 * sigma**2)) * np.exp(1j * k * r)
    psi = np.zeros(g.size, dtype=np.complex128)
    for l in range(min(lmax_fill, g.lmax) + 1):
        psi[l * g.n:(l + 1) * g.n] = f / (l + 1)
    return psi / math.sqrt(g.dr * np.vdot(psi, psi).real)


def outside(g, psi, j):
    """P_{>j} + (dr/2) sum_l |f_l,j|^2, by plain sums."""
    f = psi.reshape(g.lmax + 1, g.n)
    return g.dr * (np.sum(np.abs(f[:, j + 1:]) ** 2) + 0.5 * np.sum(np.abs(f[:, j]) ** 2))


def test_mask_shape(orc):
    rb, p = 100.0, 200.0
    rs = np.linspace(0.0, rb, 2001)
    m = np.array([orc.mask(r, rb, p) for r in rs])
    assert m[0] == 1.0 and m[-1] == 0.0 and orc.mask(rb + 1.0, rb, p) == 0.0
    assert np.all(np.diff(m) <= 0.0)
    assert orc.mask(0.4 * rb, rb, p) == 1.0        # no absorption inside the flux radius used below


def test_three_point_current_is_the_discrete_continuity_equation(orc):
    g = orc.Grid(n=800, lmax=2, dr=0.1, stencil=3)
    pulse = orc.Pulse(0.05, 0.5, 2.0, 0.3, 0.0)
    setup = orc.obs_setup(g, r_ion=30.0)
    psi0 = packet(orc, g)
    j = 349                                       # r = 35 au
    dt = 0.8 * 3.3961 / orc.h_bound(g, 0.05)
    n = int(round(12.0 / dt))                     # the packet crosses r_j (k = 1.5 au)
    psi, _, _, flux = orc.propagate_abs(g, pulse, orc.TAYLOR, 8, 0.0, dt, n, 0, setup, psi0, flux_j=j)
    moved = outside(g, psi, j) - outside(g, psi0, j)
    assert moved > 0.3
    # trapezoid rule in time: O(dt^2) with dt ~ 0.0055
    assert abs(flux - moved) < 2e-6 * moved


def test_absorbed_probability_closes_the_flux_balance(orc):
    g = orc.Grid(n=1000, lmax=1, dr=0.1, stencil=3)
    pulse = orc.Pulse(0.0, 1.0, 1.0, 0.0, 0.0)
    setup = orc.obs_setup(g, r_ion=30.0)
    psi0 = packet(orc, g)
    j, r_abs, p_abs = 399, 100.0, 200.0           # flux at 40 au, mask reaching 0 at the wall
    dt = 0.8 * 3.3961 / orc.h_bound(g, 0.0)
    n = int(round(60.0 / dt))
    psi, _, _, flux = orc.propagate_abs(g, pulse, orc.TAYLOR, 8, 0.0, dt, n, 0, setup, psi0, r_abs=r_abs,
                                        p_abs=p_abs, flux_j=j)
    absorbed = 1.0 - g.dr * np.vdot(psi, psi).real
    moved = outside(g, psi, j) - outside(g, psi0, j)
    assert absorbed > 0.5                         # most of the packet left through the absorber
    assert abs(flux - (moved + absorbed)) < 1e-5
    # without the mask the norm is kept (no absorption anywhere else)
    psi_free, _, _, _ = orc.propagate_abs(g, pulse, orc.TAYLOR, 8, 0.0, dt, 50, 0, setup, psi0)
    assert abs(g.dr * np.vdot(psi_free, psi_free).real - 1.0) < 1e-12


def test_five_point_current_meets_the_balance_at_fourth_order(orc):
    g = orc.Grid(n=800, lmax=1, dr=0.1, stencil=5)
    pulse = orc.Pulse(0.0, 1.0, 1.0, 0.0, 0.0)
    setup = orc.obs_setup(g, r_ion=30.0)
    psi0 = packet(orc, g)
    j = 349
    dt = 0.8 * 3.3961 / orc.h_bound(g, 0.0)
    n = int(round(12.0 / dt))
    psi, _, _, flux = orc.propagate_abs(g, pulse, orc.TAYLOR, 8, 0.0, dt, n, 0, setup, psi0, flux_j=j)
    moved = outside(g, psi, j) - outside(g, psi0, j)
    # (k dr)^4 ~ 5e-4 for k = 1.5, dr = 0.1: the point current differs from the
    # conservative flux at that order
    assert moved > 0.3 and abs(flux - moved) < 1e-3 * moved
