"""The entry point that allocates nothing: tdse_observables_noalloc (scratch in
the library's static device buffer) against tdse_observables (scratch in the
bound workspace), through the C ABI.  Both run the same kernels in the same
order, so the records agree bit for bit.  Two contexts in a row, the second
smaller than the first (the static buffer still holds the first call's
partial sums), in FP64 and in 48-bit storage."""
import numpy as np
import pytest

import workloads
from gpu_helpers import lib, say

pytestmark = pytest.mark.gpu


def _prop(grids, prec):
    t = lib()
    prop = t.Propagator([t.Grid(n, lm, dr, st, prec, 1.0, rion) for (n, lm, dr, st, rion) in grids],
                        methods=((t.METHOD_TAYLOR, 8),))
    for k, (n, lm, dr, st, rion) in enumerate(grids):
        v = workloads.mixed_state(300 + k, n, lm, dr)
        prop.set_state(k, v / np.sqrt(dr * np.vdot(v, v).real))
    return prop


@pytest.mark.parametrize("prec", [0, 2])
def test_noalloc_observables_match_the_workspace_entry_point(prec):
    t = lib()
    cases = [
        [(4000, 24, 0.1, 3, 100.0), (1333, 9, 0.05, 3, 30.0), (777, 4, 0.1, 3, 20.0)],   # larger first
        [(300, 3, 0.1, 3, 10.0)],                                                         # then smaller
    ]
    for grids in cases:
        say(f"noalloc observables vs tdse_observables: prec {prec}, grids {grids}")
        prop = _prop(grids, prec)
        n = len(grids)
        pulses = [t.Pulse(0.05, 0.3, 2.0, 0.1 * k, 0.0) for k in range(n)]
        prop.step_taylor(pulses, [0.5] * n, [1e-4] * n, 8, 5)
        times = [0.7 + 0.1 * k for k in range(n)]
        a = prop.observables_noalloc(pulses, times)
        b = prop.observables(pulses, times)
        c = prop.observables_noalloc(pulses, times)
        prop.close()
        say(f"  max |noalloc - workspace| = {np.max(np.abs(a - b)):.1e}")
        assert np.array_equal(a, b) and np.array_equal(c, b)
        assert np.all(a[:, 2] > 0.99) and np.all(np.isfinite(a))
