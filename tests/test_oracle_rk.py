"""Pins of the oracle's explicit Runge-Kutta methods (appendix "Runge-Kutta",
eq. RKDeriv): Euler, classic RK4, Fehlberg 4(5), Cash-Karp 5(4),
Dormand-Prince 5(4), Merson 4(3).

The paper names the methods but prints no tableau; the tableaux are pinned
by Butcher's order conditions (every condition up to each weight row's
order, and the row-sum condition c_i = sum_j a_ij: a wrong digit anywhere
breaks one), the steps by the exact action of the stability polynomial on an
eigenvector, the measured convergence order with a time-dependent field,
and the identity of the tableau form of RK4 with the oracle's own RK4 and
with Taylor-4 without field.  The embedded deviation sigma_n is pinned by its
closed form on an eigenvector.
"""
import math

import numpy as np
import pytest
from scipy.sparse.linalg import eigsh

from _hmat import sparse_h

# (method, order of b, order of bhat or None)
METHODS = [(0, 1, None), (1, 4, None), (2, 5, 4), (3, 5, 4), (4, 5, 4), (5, 4, 3)]


def order_conditions(b, a, c, p):
    """Residuals of Butcher's order conditions up to order p (rooted trees up
    to five nodes)."""
    one = np.ones_like(c)
    A = a
    res = [b @ one - 1.0]
    if p >= 2:
        res += [b @ c - 1 / 2]
    if p >= 3:
        res += [b @ c**2 - 1 / 3, b @ A @ c - 1 / 6]
    if p >= 4:
        res += [b @ c**3 - 1 / 4, b @ (c * (A @ c)) - 1 / 8, b @ A @ c**2 - 1 / 12, b @ A @ A @ c - 1 / 24]
    if p >= 5:
        res += [b @ c**4 - 1 / 5, b @ (c**2 * (A @ c)) - 1 / 10, b @ (c * (A @ c**2)) - 1 / 15,
                b @ (c * (A @ A @ c)) - 1 / 30, b @ (A @ c) ** 2 - 1 / 20, b @ A @ c**3 - 1 / 20,
                b @ A @ (c * (A @ c)) - 1 / 40, b @ A @ A @ c**2 - 1 / 60, b @ A @ A @ A @ c - 1 / 120]
    return np.abs(np.array(res))


@pytest.mark.parametrize("method,p,phat", METHODS)
def test_tableaux_satisfy_their_order_conditions(orc, method, p, phat):
    c, a, b, bh, s = orc.rk_tableau(method)
    assert s == len(c) and np.all(np.triu(a) == 0.0)          # explicit
    assert np.max(np.abs(a.sum(axis=1) - c)) < 1e-15           # row sums
    assert np.max(order_conditions(b, a, c, p)) < 1e-14
    if phat is not None:
        assert np.max(order_conditions(bh, a, c, phat)) < 1e-14
        # and the embedded row is of lower order than b: it fails order p
        assert np.max(order_conditions(bh, a, c, p)) > 1e-6


def stability_poly(b, a, z):
    """R(z) = 1 + sum_k (b^T A^(k-1) 1) z^k, the step's factor on dy/dt = lambda y."""
    v = np.ones(len(b))
    r, zk = 1.0 + 0j, 1.0 + 0j
    for _ in range(len(b)):
        zk *= z
        r += (b @ v) * zk
        v = a @ v
    return r


@pytest.mark.parametrize("method,p,phat", METHODS)
def test_step_on_an_eigenvector_is_the_stability_polynomial(orc, method, p, phat):
    # field free: the step multiplies an eigenvector of energy E by R(-i E dt);
    # the deviation of the pair is (R_b - R_bhat)(-i E dt) times the vector.
    # A coarse grid (lambda_max ~ 8 au) allows a long step, |E dt| up to 1.5,
    # where the pair's deviation, O((E dt)^5), stands far above round-off
    g = orc.Grid(n=60, lmax=0, dr=0.5, stencil=3)
    vals, vecs = np.linalg.eigh(sparse_h(orc, g, 0.0).toarray().real)
    c, a, b, bh, s = orc.rk_tableau(method)
    p0 = orc.Pulse(0.0, 1.0, 1.0, 0.0, 0.0)
    dt = 0.3
    for j in (0, 30, 50):            # E dt from -0.14 to about 1.5
        phi = vecs[:, j] / math.sqrt(g.dr) + 0j
        got, sig = orc.rk_step(g, p0, method, 0.3, dt, phi)
        z = -1j * vals[j] * dt
        want = stability_poly(b, a, z) * phi
        assert np.max(np.abs(got - want)) < 1e-13 * np.max(np.abs(phi))
        rms = math.sqrt(np.sum(np.abs(phi) ** 2) / phi.size)
        dev = abs(stability_poly(b, a, z) - stability_poly(bh, a, z)) * rms if phat else 0.0
        assert abs(sig - dev) <= 1e-9 * dev + 1e-15 * rms
        if phat:
            assert dev > 1e-10 * rms


@pytest.mark.parametrize("method,p,phat", METHODS)
def test_global_order_with_a_time_dependent_field(orc, method, p, phat):
    # self-convergence with a time-dependent field (a non-autonomous problem):
    # the differences between runs at dt, dt/2 and dt/4 fall by 2^p, on a
    # coarse grid (lambda_max dt <= 0.5) in the asymptotic regime
    g = orc.Grid(n=60, lmax=1, dr=0.5, stencil=3)
    pulse = orc.Pulse(0.1, 1.0, 1.0, 0.4, 0.0)
    setup = orc.obs_setup(g, r_ion=10.0)
    psi0, _ = orc.initial_state(g)
    T, dt0 = 1.2, 0.05
    s = [orc.propagate_rk(g, pulse, method, 0.0, dt, int(round(T / dt)), 0, setup, psi0)[0]
         for dt in (dt0, dt0 / 2, dt0 / 4)]
    rate = math.log2(np.linalg.norm(s[0] - s[1]) / np.linalg.norm(s[1] - s[2]))
    assert abs(rate - p) < 0.15, rate


def test_tableau_rk4_agrees_with_the_rk4_step_and_taylor4(orc):
    g = orc.Grid(n=300, lmax=4, dr=0.1, stencil=5)
    pulse = orc.Pulse(0.05, 0.3, 2.0, 0.0, 0.0)
    setup = orc.obs_setup(g, r_ion=10.0)
    rng = np.random.default_rng(5)
    psi0 = rng.standard_normal(g.size) + 1j * rng.standard_normal(g.size)
    dt = 1e-3
    a, _, _ = orc.propagate(g, pulse, orc.RK4, 4, 0.2, dt, 20, 0, setup, psi0)
    b, _, sig = orc.propagate_rk(g, pulse, orc.RK_CLASSIC4, 0.2, dt, 20, 0, setup, psi0)
    assert np.linalg.norm(a - b) / np.linalg.norm(a) < 1e-14 and sig == 0.0
    off = orc.Pulse(0.0, 1.0, 1.0, 0.0, 0.0)
    c, _, _ = orc.propagate(g, off, orc.TAYLOR, 4, 0.0, dt, 20, 0, setup, psi0)
    d, _, _ = orc.propagate_rk(g, off, orc.RK_CLASSIC4, 0.0, dt, 20, 0, setup, psi0)
    assert np.linalg.norm(c - d) / np.linalg.norm(c) < 1e-14
