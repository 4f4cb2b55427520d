"""Pins of the oracle's diffusion (imaginary-time) ground-state search, Sec. 4
"Ground state calculation" (eq. e_g).

Checks against what is fixed independently of the iteration: the paper's
printed energies of its diffusion runs (about -0.47 au without, about -0.5 au
with the -0.02 au grid offset; 4th-order differences, dr = 0.2, box 800 au),
the lowest eigenpair of the same Hamiltonian from a library eigensolver, the
closed form of one step on an exact eigenvector, the closed-form decay of an
excited admixture, the angular-momentum selection the paper describes, and
the hydrogen level -1/(2n^2) at O(dr^2).
"""
import json
import math
import os

import numpy as np
import pytest
from scipy.sparse.linalg import eigsh

from _hmat import sparse_h

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def taylor_poly(x, order):
    """sum_{k<=P} (-x)^k / k!, the step polynomial of exp(-x)."""
    return sum((-x) ** k / math.factorial(k) for k in range(order + 1))


def lowest(orc, g, l, k=2):
    """Lowest k eigenpairs of the field-free block h_l, grid-normalised."""
    h = sparse_h(orc, g, 0.0).real.tocsr()
    blk = h[l * g.n:(l + 1) * g.n, l * g.n:(l + 1) * g.n]
    vals, vecs = eigsh(blk, k=k, sigma=-1.0, which="LM")
    order = np.argsort(vals)
    vecs = vecs[:, order] / math.sqrt(g.dr)
    return vals[order], vecs


def test_paper_diffusion_energies(orc):
    # Example 1, the diffusion runs: ~ -0.47 au without and ~ -0.5 au with an
    # offset of -0.02 au (4th-order FD, dr = 0.2, box 800 au, first point at dr)
    ref = json.load(open(os.path.join(GOLDEN, "paper_ground_energy.json")))
    for v in ref["values"]:
        g = orc.Grid(n=4000, lmax=0, dr=0.2, stencil=5, r_shift=v["offset_au"])
        psi0, _ = orc.initial_state(g)
        _, e = orc.imag_propagate(g, 0.02, 8, 2500, psi0)
        assert abs(e[-1] - v["e_1s_au"]) <= v["abs_tol"], (v, e[-1])
        assert abs(e[-1] - e[-2]) < 1e-12          # converged


def test_converges_to_the_lowest_eigenpair(orc):
    # the energy estimate and the state reach the lowest eigenpair of the same
    # discrete Hamiltonian as found by ARPACK (shift-invert)
    g = orc.Grid(n=600, lmax=0, dr=0.1, stencil=3)
    vals, vecs = lowest(orc, g, 0)
    rng = np.random.default_rng(3)
    psi0 = rng.standard_normal(g.n) * np.exp(-0.05 * np.arange(g.n)) + 0j
    dtau = 0.8 * 2.0 / orc.h_bound(g, 0.0)
    psi, e = orc.imag_propagate(g, dtau, 8, 20000, psi0)
    assert abs(e[-1] - vals[0]) < 1e-11 * abs(vals[0])
    overlap = abs(g.dr * np.vdot(vecs[:, 0], psi)) ** 2
    assert overlap > 1 - 1e-12
    assert abs(g.dr * np.vdot(psi, psi).real - 1) < 1e-13     # renormalised


@pytest.mark.parametrize("order", [4, 8])
def test_one_step_on_an_eigenvector_is_the_polynomial(orc, order):
    # on an exact eigenvector with eigenvalue E the step multiplies by p(dtau E)
    # (p the truncated exp(-x)), so E_est = -ln(p^2) / (2 dtau)
    g = orc.Grid(n=500, lmax=0, dr=0.1, stencil=5)
    vals, vecs = lowest(orc, g, 0, k=3)
    dtau = 0.05
    for j in range(3):
        psi, e = orc.imag_propagate(g, dtau, order, 1, vecs[:, j] + 0j)
        want = -math.log(taylor_poly(dtau * vals[j], order) ** 2) / (2 * dtau)
        assert abs(e[0] - want) < 1e-11
        assert abs(g.dr * np.vdot(vecs[:, j], psi)) ** 2 > 1 - 1e-12


def test_excited_admixture_decays_by_the_polynomial_ratio(orc):
    # psi = phi_0 + a phi_1: after n steps the coefficient ratio is
    # a (p(dtau E_1) / p(dtau E_0))^n
    g = orc.Grid(n=500, lmax=0, dr=0.1, stencil=3)
    vals, vecs = lowest(orc, g, 0, k=2)
    a, dtau, n, order = 0.3, 0.01, 200, 6
    psi, _ = orc.imag_propagate(g, dtau, order, n, vecs[:, 0] + a * vecs[:, 1] + 0j)
    c0 = g.dr * np.vdot(vecs[:, 0], psi)
    c1 = g.dr * np.vdot(vecs[:, 1], psi)
    ratio = (taylor_poly(dtau * vals[1], order) / taylor_poly(dtau * vals[0], order)) ** n
    assert abs((c1 / c0).real - a * ratio) < 1e-10 and abs((c1 / c0).imag) < 1e-14


def test_symmetry_selects_the_lowest_state_of_each_l(orc):
    # no field, no coupling between partial waves: a start in l = 1 only
    # settles into the lowest l = 1 state (2p), and l = 0 stays exactly zero
    g = orc.Grid(n=800, lmax=1, dr=0.1, stencil=3)
    vals, _ = lowest(orc, g, 1)
    r = (np.arange(g.n) + 1) * g.dr
    psi0 = np.zeros(g.size, dtype=np.complex128)
    psi0[g.n:] = r * np.exp(-0.3 * r)
    psi, e = orc.imag_propagate(g, 0.8 * 2.0 / orc.h_bound(g, 0.0), 8, 30000, psi0)
    assert np.all(psi[:g.n] == 0)
    assert abs(e[-1] - vals[0]) < 1e-10
    assert abs(e[-1] + 0.125) < 2e-3                  # 2p: -1/8 au at O(dr^2)


def test_hydrogen_level_converges_at_second_order(orc):
    # 3-point differences: E_1s -> -1/2 at O(dr^2): error ratio 4 on halving dr
    errs = []
    for dr in (0.1, 0.05):
        g = orc.Grid(n=int(60 / dr), lmax=0, dr=dr, stencil=3)
        psi0, _ = orc.initial_state(g)
        _, e = orc.imag_propagate(g, 0.8 * 2.0 / orc.h_bound(g, 0.0), 8, 4000, psi0)
        errs.append(e[-1] + 0.5)
    assert abs(errs[0] / errs[1] - 4.0) < 0.05
