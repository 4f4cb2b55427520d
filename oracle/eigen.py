"""Bound eigenstates of the field-free radial blocks h_l, for the oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 2: h_l = -1/2 d^2/dr^2 + l(l+1)/(2 r^2) - z/r on the finite-difference
grid is a real symmetric banded N x N matrix (half-bandwidth 1 for the 3-point
and 2 for the 5-point second derivative, zero outside the box).  Its k-th
lowest eigenvector is the grid counterpart of the hydrogen state with
n = l + 1 + k.  The library step is ARPACK's shift-invert Lanczos (scipy
eigsh) with the shift below the whole bound spectrum, so the eigenpairs
nearest the shift are the lowest ones; the band is written out from the
formulas here.

State order (shared convention for population records): l-major, then n:
1s 2s 3s 4s 5s 2p 3p 4p 5p 3d 4d 5d 4f 5f 5g for n_max = 5.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.sparse.linalg import eigsh


def state_list(lmax: int, n_max: int = 5):
    """[(n, l)] in the population record order."""
    return [(n, l) for l in range(min(lmax, n_max - 1) + 1) for n in range(l + 1, n_max + 1)]


def radial_band(g, l: int) -> np.ndarray:
    """Lower banded storage of h_l (row 0 the diagonal, row k the k-th sub-diagonal)."""
    from . import radius
    r = radius(g)
    h2 = g.dr * g.dr
    if g.stencil == 3:
        offs = [1.0 / h2, -0.5 / h2]                       # -1/2 (f+ - 2f + f-)/h^2
    else:
        offs = [30.0 / (24.0 * h2), -16.0 / (24.0 * h2), 1.0 / (24.0 * h2)]  # -1/2 of Sec. 2 formula
    band = np.zeros((len(offs), g.n))
    band[0] = offs[0] + 0.5 * l * (l + 1) / (r * r) - g.z / r
    for k in range(1, len(offs)):
        band[k, : g.n - k] = offs[k]
    return band


def bound_states(g, n_max: int = 5):
    """Energies, eigenvectors (normalised dr*sum phi^2 = 1) and (n, l) labels."""
    states = state_list(g.lmax, n_max)
    phis, energies = [], []
    for l in sorted({l for _, l in states}):
        count = n_max - l
        band = radial_band(g, l)
        offsets = list(range(-(len(band) - 1), len(band)))
        diags = [band[abs(k), : g.n - abs(k)] for k in offsets]
        h = sp.diags(diags, offsets, format="csc")
        shift = -0.6 * g.z * g.z - 1.0
        w, v = eigsh(h, k=count, sigma=shift, which="LM", tol=0.0)
        order = np.argsort(w)
        w, v = w[order], v[:, order]
        for k in range(count):
            phi = v[:, k] / np.sqrt(g.dr * np.dot(v[:, k], v[:, k]))
            if phi[np.argmax(np.abs(phi))] < 0:
                phi = -phi
            phis.append(phi)
            energies.append(w[k])
    return np.array(energies), np.array(phis), states


def obs_setup(g, r_ion: float, n_max: int = 5):
    """Everything orc_observables needs besides the state."""
    from . import ObsSetup, initial_state
    _, u0 = initial_state(g)
    _, phi, states = bound_states(g, n_max)
    return ObsSetup(r_ion=float(r_ion), u0=u0, phi=np.ascontiguousarray(phi),
                    state_l=np.array([l for _, l in states], dtype=np.int32),
                    state_n=np.array([n for n, _ in states], dtype=np.int32))
