"""Pins of the oracle's time steps (Taylor, RK4, Lanczos) and eigensolver.

Each check ties the oracle to mathematics it must reproduce: the exact action
of a polynomial step on an eigenvector, a dense matrix exponential (scipy
expm) on tiny grids, convergence orders, the identity of RK4 and Taylor-4 for
an autonomous linear system, the invariance of the norm under Lanczos, the
parity symmetry E -> -E, and LAPACK's symmetric eigensolver.
"""
import math

import numpy as np
import pytest
from scipy.linalg import expm

from _hmat import sparse_h


def smooth_state(g, seed=1):
    rng = np.random.default_rng(seed)
    r = (np.arange(g.n) + 1) * g.dr
    rows = []
    for l in range(g.lmax + 1):
        a, b = rng.standard_normal(2) + 1j * rng.standard_normal(2)
        rows.append((a * r ** (l + 1) * np.exp(-r / (1.5 + l)) + 0.2 * b * r * np.exp(-0.3 * r))
                    * np.exp(1j * rng.uniform(0, 2 * np.pi)))
    psi = np.concatenate(rows)
    return psi / np.sqrt(g.dr * np.vdot(psi, psi).real)


def taylor_poly(x, order):
    return sum(x ** k / math.factorial(k) for k in range(order + 1))


@pytest.mark.parametrize("stencil,order", [(3, 4), (5, 8), (3, 8)])
def test_taylor_on_eigenstate_is_the_polynomial(orc, stencil, order):
    # For H phi = E phi a degree-P step multiplies phi by sum_k (-i E dt)^k/k!.
    g = orc.Grid(n=600, lmax=2, dr=0.1, stencil=stencil)
    e, phi, states = orc.bound_states(g, 3)
    k = states.index((2, 1))
    psi = np.zeros(g.size, dtype=np.complex128)
    psi[g.n:2 * g.n] = phi[k]
    dt, steps = 0.004, 200          # below the explicit stability limit (~5e-3 here)
    out = psi
    for _ in range(steps):
        out = orc.taylor_step(g, 0.0, dt, order, out)
    expect = taylor_poly(-1j * e[k] * dt, order) ** steps * psi
    assert np.linalg.norm(out - expect) < 1e-12 * np.linalg.norm(psi)


@pytest.mark.parametrize("order", [2, 3, 4])
def test_taylor_local_error_order(orc, order):
    # One step against the dense exponential: error ~ dt^(P+1).
    g = orc.Grid(n=40, lmax=3, dr=0.2, stencil=5)
    h = sparse_h(orc, g, 0.05).toarray()
    psi = smooth_state(g)
    errs = []
    for dt in (4e-3, 2e-3):
        exact = expm(-1j * dt * h) @ psi
        errs.append(np.linalg.norm(orc.taylor_step(g, 0.05, dt, order, psi) - exact))
    assert errs[0] / errs[1] == pytest.approx(2 ** (order + 1), rel=0.15)


def test_rk4_equals_taylor4_without_field(orc):
    g = orc.Grid(n=300, lmax=4, dr=0.1, stencil=3)
    psi = smooth_state(g, 3)
    a = orc.rk4_step(g, orc.Pulse(), 0.0, 1e-3, psi)
    b = orc.taylor_step(g, 0.0, 1e-3, 4, psi)
    assert np.linalg.norm(a - b) < 1e-14 * np.linalg.norm(b)


def _run(orc, g, p, method, order, dt, t_end, psi):
    steps = int(round(t_end / dt))
    setup = orc.obs_setup(g, r_ion=5.0, n_max=2)
    out, _, _ = orc.propagate(g, p, method, order, 0.0, dt, steps, 0, setup, psi)
    return out


def test_global_orders_with_time_dependent_field(orc):
    # RK4 is 4th order; a step with H frozen at the midpoint (Taylor, Lanczos)
    # is 2nd order in the time dependence (and would be 1st order if H were
    # frozen at the start of the step).
    g = orc.Grid(n=60, lmax=4, dr=0.25, stencil=3)
    p = orc.Pulse(e0=0.4, omega=3.0, n_cycles=2.0, cep=0.3)
    psi = smooth_state(g, 5)
    t_end = 0.8
    ref = _run(orc, g, p, orc.RK4, 4, 2.5e-5, t_end, psi)
    e_rk = [np.linalg.norm(_run(orc, g, p, orc.RK4, 4, dt, t_end, psi) - ref) for dt in (4e-4, 2e-4)]
    e_ty = [np.linalg.norm(_run(orc, g, p, orc.TAYLOR, 8, dt, t_end, psi) - ref) for dt in (4e-4, 2e-4)]
    assert e_rk[0] / e_rk[1] == pytest.approx(16, rel=0.2)
    assert e_ty[0] / e_ty[1] == pytest.approx(4, rel=0.1)


def test_lanczos_full_dimension_is_exact(orc):
    g = orc.Grid(n=16, lmax=2, dr=0.3, stencil=5)
    h = sparse_h(orc, g, 0.08).toarray()
    psi = smooth_state(g, 7)
    for dt in (0.01, 0.2):
        exact = expm(-1j * dt * h) @ psi
        out, used = orc.lanczos_step(g, 0.08, dt, g.size, psi)
        assert np.linalg.norm(out - exact) < 1e-12 * np.linalg.norm(psi), (dt, used)


def test_lanczos_eigenstate_breakdown_gives_exact_phase(orc):
    g = orc.Grid(n=800, lmax=3, dr=0.1, stencil=3)
    e, phi, states = orc.bound_states(g, 3)
    k = states.index((3, 2))
    psi = np.zeros(g.size, dtype=np.complex128)
    psi[2 * g.n:3 * g.n] = phi[k]
    out, used = orc.lanczos_step(g, 0.0, 0.7, 20, psi)
    assert used == 1
    assert np.linalg.norm(out - np.exp(-1j * e[k] * 0.7) * psi) < 1e-13 * np.linalg.norm(psi)


def test_lanczos_matches_taylor_and_keeps_norm(orc):
    # Both approximate exp(-i H dt) psi with the same frozen H.
    g = orc.Grid(n=400, lmax=6, dr=0.1, stencil=5)
    psi = smooth_state(g, 11)
    dt = 2e-4
    a, used = orc.lanczos_step(g, 0.05, dt, 20, psi)
    b = orc.taylor_step(g, 0.05, dt, 8, psi)
    assert used == 20
    assert np.linalg.norm(a - b) < 1e-11 * np.linalg.norm(b)
    big, _ = orc.lanczos_step(g, 0.05, 0.05, 20, psi)       # far beyond explicit stability
    assert np.vdot(big, big).real == pytest.approx(np.vdot(psi, psi).real, rel=1e-13)


def test_parity_symmetry_is_exact(orc):
    # E0 -> -E0 maps f_l to (-1)^l f_l; with sign flips exact in IEEE
    # arithmetic the two runs agree bit for bit.
    g = orc.Grid(n=200, lmax=5, dr=0.1, stencil=5)
    psi0, _ = orc.initial_state(g)
    p = orc.Pulse(e0=0.06, omega=0.3, n_cycles=2.0, cep=0.1)
    q = orc.Pulse(e0=-0.06, omega=0.3, n_cycles=2.0, cep=0.1)
    setup = orc.obs_setup(g, r_ion=10.0, n_max=3)
    for method, order in ((orc.TAYLOR, 4), (orc.RK4, 4), (orc.LANCZOS, 10)):
        a, oa, _ = orc.propagate(g, p, method, order, 0.0, 5e-3, 60, 20, setup, psi0)
        b, ob, _ = orc.propagate(g, q, method, order, 0.0, 5e-3, 60, 20, setup, psi0)
        sign = np.repeat((-1.0) ** np.arange(g.lmax + 1), g.n)
        if method == orc.LANCZOS:
            assert np.abs(b - sign * a).max() < 1e-14
        else:
            assert np.array_equal(b, sign * a)
        assert np.allclose(ob[:, 6], -oa[:, 6], rtol=1e-13, atol=0)       # dipole flips
        assert np.allclose(ob[:, 8:], oa[:, 8:], rtol=1e-12, atol=1e-300)  # populations equal


def test_jacobi_matches_lapack(orc):
    rng = np.random.default_rng(3)
    a = rng.standard_normal((20, 20))
    a = a + a.T
    w, v = orc.jacobi_eig(a)
    assert np.allclose(np.sort(w), np.linalg.eigvalsh(a), rtol=0, atol=1e-12)
    assert np.allclose(v @ np.diag(w) @ v.T, a, atol=1e-12)
    assert np.allclose(v.T @ v, np.eye(20), atol=1e-13)
    # graded tridiagonal, like a Lanczos matrix of a stiff operator
    d = np.geomspace(0.5, 8e5, 20) * np.where(np.arange(20) % 2, 1, -1)
    e = np.geomspace(0.1, 3e5, 19)
    t = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
    w, v = orc.jacobi_eig(t)
    ref = np.linalg.eigvalsh(t)
    assert np.allclose(np.sort(w), ref, rtol=1e-13, atol=1e-9)


def test_thread_count_does_not_change_results(orc):
    # the element-wise loops may run on several threads; every element is
    # computed by one thread with the same operations and every sum runs on
    # one thread in index order, so the results are bit-identical
    g = orc.Grid(n=900, lmax=9, dr=0.1, stencil=5)
    p = orc.Pulse(0.06, 0.3, 2.0, 0.1, 0.0)
    setup = orc.obs_setup(g, r_ion=20.0)
    psi0 = smooth_state(g, 17)
    out = []
    for th in (1, 4):
        orc.set_threads(th)
        runs = [orc.propagate(g, p, code, order, 0.3, dt, 6, 2, setup, psi0)
                for code, order, dt in ((orc.TAYLOR, 8, 2e-4), (orc.RK4, 4, 2e-4), (orc.LANCZOS, 10, 0.01))]
        out.append(runs)
    orc.set_threads(1)
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
