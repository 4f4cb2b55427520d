"""Pins of the oracle's Hamiltonian against what the paper and hydrogen fix.

Every check here compares the oracle with something other than itself: the
paper's printed ground-state energies, the hydrogen spectrum, Legendre
integrals for the angular coupling, the hydrogen polarisability and linear
Stark splitting, Hermiticity and the band structure of Fig. 1.
"""
import json
import math
import os

import numpy as np
import pytest
from numpy.polynomial import legendre as npleg
from scipy.sparse.linalg import eigsh

from _hmat import sparse_h

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def dense_h(orc, g, efield):
    """Brute force: the matrix of the oracle's apply_h, column by column."""
    size = g.size
    m = np.empty((size, size), dtype=np.complex128)
    e = np.zeros(size, dtype=np.complex128)
    for j in range(size):
        e[j] = 1.0
        m[:, j] = orc.apply_h(g, efield, e)
        e[j] = 0.0
    return m


def test_kappa_matches_legendre_integral(orc):
    # k_{l,l-1} = <Y_l0| cos theta |Y_{l-1,0}> by Gauss-Legendre quadrature of
    # normalised Legendre polynomials (independent of the closed form).
    x, w = npleg.leggauss(64)
    for l in range(1, 12):
        pl = npleg.legval(x, [0] * l + [1]) * math.sqrt((2 * l + 1) / 2)
        pm = npleg.legval(x, [0] * (l - 1) + [1]) * math.sqrt((2 * l - 1) / 2)
        assert orc.kappa(l) == pytest.approx(np.sum(w * pl * x * pm), rel=1e-13)
    assert orc.kappa(0) == 0.0
    assert orc.kappa(1) == pytest.approx(1 / math.sqrt(3), rel=4e-16)


@pytest.mark.parametrize("stencil", [3, 5])
def test_band_structure_fig1(orc, stencil):
    # Fig. 1 (length gauge): banded diagonal blocks, diagonal off-diagonal
    # blocks coupling l to l +- 1 only, nothing else.
    g = orc.Grid(n=12, lmax=3, dr=0.3, stencil=stencil)
    s = 1 if stencil == 3 else 2
    m = dense_h(orc, g, 0.07)
    n = g.n
    for l in range(g.lmax + 1):
        for lp in range(g.lmax + 1):
            blk = m[l * n:(l + 1) * n, lp * n:(lp + 1) * n]
            i, j = np.nonzero(blk)
            if l == lp:
                assert np.all(np.abs(i - j) <= s)
                assert np.count_nonzero(np.diag(blk, s)) == n - s   # full band
            elif abs(l - lp) == 1:
                assert np.all(i == j) and len(i) == n
            else:
                assert len(i) == 0
    m0 = dense_h(orc, g, 0.0)
    for l in range(g.lmax):
        assert not np.any(m0[l * n:(l + 1) * n, (l + 1) * n:(l + 2) * n])


@pytest.mark.parametrize("stencil", [3, 5])
def test_hermitian(orc, stencil):
    rng = np.random.default_rng(7)
    g = orc.Grid(n=200, lmax=6, dr=0.1, stencil=stencil)
    u = rng.standard_normal(g.size) + 1j * rng.standard_normal(g.size)
    v = rng.standard_normal(g.size) + 1j * rng.standard_normal(g.size)
    a = np.vdot(u, orc.apply_h(g, 0.3, v))
    b = np.vdot(orc.apply_h(g, 0.3, u), v)
    assert abs(a - b) <= 1e-12 * abs(a)


def test_paper_ground_energy_5point(orc):
    # Sec. 6.1: with 4th-order differences, box 800 au, dr = 0.2 the ground
    # state comes out near -0.47 au; shifting the grid by -0.02 au gives ~-0.5.
    with open(os.path.join(GOLDEN, "paper_ground_energy.json")) as f:
        golden = json.load(f)
    for case in golden["values"]:
        g = orc.Grid(n=4000, lmax=0, dr=0.2, stencil=5, r_shift=case["offset_au"])
        e, _, _ = orc.bound_states(g, 1)
        assert abs(e[0] - case["e_1s_au"]) < case["abs_tol"], (case, e[0])


def test_hydrogen_levels_3point_second_order(orc):
    # 3-point levels approach -1/(2 n^2) with an O(dr^2) error.
    errs = {}
    for dr in (0.1, 0.05):
        g = orc.Grid(n=int(round(300 / dr)), lmax=2, dr=dr, stencil=3)
        e, _, states = orc.bound_states(g, 5)
        errs[dr] = np.array([abs(ei + 0.5 / n ** 2) for ei, (n, l) in zip(e, states)])
        assert np.all(errs[dr] < 0.15 * dr ** 2), errs[dr]
    ratio = errs[0.1][0] / errs[0.05][0]
    assert 3.8 < ratio < 4.2


def test_hydrogen_levels_5point_l_ge_1(orc):
    # For l >= 1 the zero-padded 4th-order stencil is accurate to ~1e-6.
    g = orc.Grid(n=6000, lmax=2, dr=0.05, stencil=5)
    e, _, states = orc.bound_states(g, 5)
    for ei, (n, l) in zip(e, states):
        if l >= 1:
            assert abs(ei + 0.5 / n ** 2) < 2e-6, (n, l, ei)


@pytest.mark.parametrize("stencil", [3, 5])
def test_apply_h_eigen_residual(orc, stencil):
    # The C operator and the banded eigenvectors agree: H phi = E phi.
    g = orc.Grid(n=1500, lmax=3, dr=0.1, stencil=stencil)
    e, phi, states = orc.bound_states(g, 5)
    for ek, ph, (n, l) in zip(e, phi, states):
        psi = np.zeros(g.size, dtype=np.complex128)
        psi[l * g.n:(l + 1) * g.n] = ph
        res = orc.apply_h(g, 0.0, psi) - ek * psi
        assert np.linalg.norm(res) < 1e-10 * np.linalg.norm(psi)


def _ground_in_field(orc, g, field, sigma=-0.6, k=1):
    w, v = eigsh(sparse_h(orc, g, field).real.tocsc(), k=k, sigma=sigma, which="LM")
    order = np.argsort(w)
    return w[order], v[:, order]


def test_quadratic_stark_shift(orc):
    # Hydrogen 1s in a static field F: E(F) - E(0) = -(9/4) F^2 - (3555/64) F^4,
    # reached at O(dr^2) on the 3-point grid.
    F = 0.005
    expect = -2.25 * F ** 2 - 3555 / 64 * F ** 4
    rel = {}
    for dr in (0.05, 0.025):
        g = orc.Grid(n=int(round(50 / dr)), lmax=8, dr=dr, stencil=3)
        shift = _ground_in_field(orc, g, F)[0][0] - _ground_in_field(orc, g, 0.0)[0][0]
        rel[dr] = shift / expect - 1
    assert abs(rel[0.05]) < 3e-3
    assert 3.5 < rel[0.05] / rel[0.025] < 4.5


def test_linear_stark_n2(orc):
    # The n = 2 manifold (m = 0: 2s and 2p0) splits linearly, -1/8 +- 3F.
    F = 1e-3
    g = orc.Grid(n=1200, lmax=6, dr=0.05, stencil=3)
    w, _ = _ground_in_field(orc, g, F, sigma=-0.13, k=4)
    near = np.sort(w[np.abs(w + 0.125) < 0.01])
    assert len(near) == 2
    assert near[1] - near[0] == pytest.approx(6 * F, rel=0.01)


def test_stark_dipole_and_acceleration(orc):
    # Hellmann-Feynman: <z> = dE/dF = -(9/2) F - (3555/16) F^3 for the
    # field-dressed ground state; Ehrenfest: <z''> = 0 in a stationary state.
    F = 0.005
    g = orc.Grid(n=1000, lmax=8, dr=0.05, stencil=3)
    _, v = _ground_in_field(orc, g, F)
    psi = v[:, 0].astype(np.complex128) / math.sqrt(g.dr * np.dot(v[:, 0], v[:, 0]))
    setup = orc.obs_setup(g, r_ion=20.0)
    # Observables are taken with no pulse (E = 0), so the acceleration record
    # holds -<cos(theta)/r^2> alone, which must cancel the static force: +F.
    obs = orc.observables(g, orc.Pulse(), 0.0, setup, psi)
    assert obs[2] == pytest.approx(1.0, abs=1e-12)
    assert obs[6] == pytest.approx(-4.5 * F - 3555 / 16 * F ** 3, rel=3e-3)
    assert obs[7] == pytest.approx(F, rel=3e-3)


def test_hydrogen_like_levels_charge_two(orc):
    # He+ (Z = 2): 3-point levels approach -Z^2/(2 n^2).  In the scaled radius
    # Z r the grid spacing is Z dr, so the error is Z^2 times the hydrogen
    # error at spacing Z dr: below 0.15 Z^4 dr^2, with ratio 4 per halving.
    z = 2.0
    errs = {}
    for dr in (0.05, 0.025):
        g = orc.Grid(n=int(round(150 / dr)), lmax=2, dr=dr, stencil=3, z=z)
        e, _, states = orc.bound_states(g, 5)
        errs[dr] = np.array([abs(ei + z * z * 0.5 / n ** 2) for ei, (n, l) in zip(e, states)])
        assert np.all(errs[dr] < 0.15 * z ** 4 * dr ** 2), errs[dr]
    assert 3.8 < errs[0.05][0] / errs[0.025][0] < 4.2
    # the Z = 1 levels are not the answer (a dropped Z would land there)
    assert abs(e[0] + 0.5) > 1.0


def test_stark_dipole_and_acceleration_charge_two(orc):
    # He+ 1s in a static field F: polarisability 9/(2 Z^4), so Hellmann-Feynman
    # gives <z> = -(9/2) F / Z^4; a stationary state feels no net force, so the
    # acceleration record taken without a pulse, -2 Z sum kappa Re int f* f/r^2
    # (eq. DipoleAccel for charge Z), must equal +F.  A factor 2 in place of 2Z
    # would give F/2.
    z, F = 2.0, 0.02
    g = orc.Grid(n=1000, lmax=8, dr=0.025, stencil=3, z=z)
    _, v = _ground_in_field(orc, g, F, sigma=-2.2)
    psi = v[:, 0].astype(np.complex128) / math.sqrt(g.dr * np.dot(v[:, 0], v[:, 0]))
    setup = orc.obs_setup(g, r_ion=10.0)
    obs = orc.observables(g, orc.Pulse(), 0.0, setup, psi)
    assert obs[6] == pytest.approx(-4.5 * F / z ** 4, rel=3e-3)
    assert obs[7] == pytest.approx(F, rel=3e-3)
