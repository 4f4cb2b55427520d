"""Host-side checks of the C-ABI library (no GPU needed).

The library loads, exports every function include/tdse.h declares, validates
descriptors, sizes its buffers, and its stability bookkeeping agrees with
independent computations (the oracle's Gershgorin bound, the exact
imaginary-axis limit 2*sqrt(2) of the degree-4 Taylor polynomial, the true
spectral radius from a sparse eigensolver).
"""
import ctypes
import math
import os
import re

import numpy as np
import pytest
from scipy.sparse.linalg import eigsh

from _hmat import sparse_h

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def tdse():
    import paper_1308_1856_amd as t
    return t


def header_functions():
    txt = open(os.path.join(ROOT, "include", "tdse.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(tdse_[a-zA-Z0-9_]+)\s*\(", txt)))


def test_exports_every_declared_symbol(tdse):
    names = header_functions()
    assert len(names) >= 19
    lib = ctypes.CDLL(tdse.LIB_PATH)
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(tdse.EXPORTED) == names


def test_single_hip_runtime(tdse):
    # libtdse must share torch's HIP runtime: exactly one libamdhip64 mapped
    maps = open("/proc/self/maps").read().splitlines()
    hip = {l.split()[-1] for l in maps if "libamdhip64" in l}
    assert len(hip) == 1, hip


def test_stability_limits(tdse):
    assert tdse.tdse_taylor_stability_limit(4) == pytest.approx(2 * math.sqrt(2), abs=1e-9)
    assert tdse.tdse_taylor_stability_limit(3) == pytest.approx(math.sqrt(3), abs=1e-9)
    y8 = tdse.tdse_taylor_stability_limit(8)
    p8 = lambda y: abs(sum((1j * y) ** k / math.factorial(k) for k in range(9)))
    assert p8(y8) <= 1 + 1e-12 and p8(y8 + 1e-6) > 1 + 1e-12
    assert tdse.tdse_taylor_stability_limit(2) < 2e-3       # P = 2 has no stable interval
    assert tdse.tdse_taylor_stability_limit(0) == 0.0


def test_real_axis_stability_limits(tdse):
    # the diffusion step's polynomial sum (-x)^k/k!: |p| <= 1 on [0, 2] for
    # P = 1, 2 (|1 - x| and 1 - x + x^2/2 reach 1 at x = 2), the classical
    # 2.785 of RK4 for P = 4, and at each limit the next x leaves the interval
    p = lambda x, P: abs(sum((-x) ** k / math.factorial(k) for k in range(P + 1)))
    assert tdse.tdse_taylor_real_stability_limit(1) == pytest.approx(2.0, abs=1e-9)
    assert tdse.tdse_taylor_real_stability_limit(2) == pytest.approx(2.0, abs=1e-9)
    assert tdse.tdse_taylor_real_stability_limit(4) == pytest.approx(2.785293563, abs=1e-6)
    for P in (3, 6, 8, 12):
        x = tdse.tdse_taylor_real_stability_limit(P)
        assert p(x, P) <= 1 + 2e-12 and p(x + 1e-6, P) > 1 + 1e-12
        assert all(p(y, P) <= 1 + 2e-12 for y in np.linspace(0, x, 2001))


def test_rk_stability_limits_from_the_oracle_tableaux(tdse, orc):
    # the library's limit for each tableau equals the one found from the
    # oracle's copy of the tableau: |R(iy)| <= 1 with R(z) = 1 + sum_k
    # (b^T A^(k-1) 1) z^k; RK4 gives the Taylor-4 value 2 sqrt(2)
    assert tdse.tdse_rk_stability_limit(1) == pytest.approx(2 * math.sqrt(2), abs=1e-9)
    assert tdse.tdse_rk_stability_limit(0) < 2e-6                     # Euler: none
    assert tdse.tdse_rk_stability_limit(6) == 0.0                     # unknown method
    for m in range(6):
        c, a, b, bh, s = orc.rk_tableau(m)
        gam = [1.0]
        v = np.ones(s)
        for _ in range(s):
            gam.append(float(b @ v))
            v = a @ v
        R = lambda y: abs(sum(gk * (1j * y) ** k for k, gk in enumerate(gam)))
        y = tdse.tdse_rk_stability_limit(m)
        assert R(y) <= 1 + 2e-12 and R(y + 1e-6) > 1 + 1e-12
        assert all(R(x) <= 1 + 2e-12 for x in np.linspace(0, y, 1001))


@pytest.mark.parametrize("stencil,lmax,dr", [(3, 8, 0.1), (5, 12, 0.05)])
def test_lambda_bound_against_oracle_and_spectrum(tdse, orc, stencil, lmax, dr):
    g = tdse.Grid(600, lmax, dr, stencil)
    ctx = tdse.tdse_init_grid([g.desc()])
    try:
        b = tdse.tdse_lambda_max_bound(ctx, 0, 0.05)
        og = orc.Grid(n=600, lmax=lmax, dr=dr, stencil=stencil)
        assert b == pytest.approx(orc.h_bound(og, 0.05), rel=1e-14)
        lam = eigsh(sparse_h(orc, og, 0.05).real, k=1, which="LA", return_eigenvectors=False)[0]
        assert lam <= b <= 1.05 * lam
    finally:
        tdse.tdse_destroy(ctx)


def test_rejects_bad_descriptors(tdse):
    bad = [tdse.GridDesc(4, 2, 3, 0, 0.1, 1.0, 10.0),        # n < 8
           tdse.GridDesc(100, 2, 4, 0, 0.1, 1.0, 10.0),      # stencil
           tdse.GridDesc(100, -1, 3, 0, 0.1, 1.0, 10.0),     # lmax
           tdse.GridDesc(100, 2, 3, 3, 0.1, 1.0, 10.0),      # precision
           tdse.GridDesc(100, 2, 3, 0, 0.0, 1.0, 10.0),      # dr
           tdse.GridDesc(100, 2, 3, 0, 0.1, 0.0, 10.0)]      # z
    for d in bad:
        with pytest.raises(tdse.TdseError) as e:
            tdse.tdse_init_grid([d])
        assert e.value.code == -1
    mixed = [tdse.Grid(100, 2, 0.1, 3).desc(), tdse.Grid(100, 2, 0.1, 5).desc()]
    with pytest.raises(tdse.TdseError):
        tdse.tdse_init_grid(mixed)


def test_sizes_and_offsets(tdse):
    grids = [tdse.Grid(1000, 4, 0.1), tdse.Grid(777, 9, 0.1), tdse.Grid(4096, 0, 0.1)]
    ctx = tdse.tdse_init_grid([g.desc() for g in grids])
    try:
        offs = [tdse.lib.tdse_state_offset(ctx, k) for k in range(3)]
        assert offs[0] == 0
        assert all(o % 64 == 0 for o in offs)
        assert offs[1] >= 5 * 1000 and offs[2] >= offs[1] + 10 * 777
        sb = tdse.lib.tdse_state_bytes(ctx)
        assert sb >= (offs[2] + 4096) * 16 and sb % 256 == 0
        wt = tdse.lib.tdse_workspace_bytes(ctx, tdse.METHOD_TAYLOR, 8)
        wr = tdse.lib.tdse_workspace_bytes(ctx, tdse.METHOD_RK4, 4)
        wl = tdse.lib.tdse_workspace_bytes(ctx, tdse.METHOD_LANCZOS, 20)
        assert wr - wt == sb and wl - wt == 18 * sb
        assert tdse.lib.tdse_state_offset(ctx, 3) == -1
    finally:
        tdse.tdse_destroy(ctx)


def test_fp48_state_is_two_planes(tdse):
    # 48-bit storage: plane h (8 B per element) and plane l (4 B per element)
    # of P elements each, P the element count rounded up to 64: 12 P bytes,
    # plane l starting 256-byte aligned
    grids = [tdse.Grid(1000, 4, 0.1, 3, tdse.FP48), tdse.Grid(777, 9, 0.1, 3, tdse.FP48)]
    ctx = tdse.tdse_init_grid([g.desc() for g in grids])
    try:
        offs = [tdse.lib.tdse_state_offset(ctx, k) for k in range(2)]
        total = offs[1] + 10 * 777
        plane = (total + 63) // 64 * 64
        assert tdse.lib.tdse_state_bytes(ctx) == 12 * plane
        assert (8 * plane) % 256 == 0
    finally:
        tdse.tdse_destroy(ctx)


def test_noalloc_observables_refuse_grids_beyond_the_static_scratch(tdse):
    # 20000 small grids need ~10 MB of scratch (step scalars, partial sums,
    # records), more than the static 8 MiB: refused before any device work
    # (the context is not even bound)
    ctx = tdse.tdse_init_grid([tdse.Grid(8, 0, 0.5).desc()] * 20000)
    try:
        pulses = [tdse.Pulse(0.0, 1.0, 1.0, 0.0, 0.0)] * 20000
        with pytest.raises(tdse.TdseError) as e:
            tdse.tdse_observables_noalloc(ctx, pulses, [0.0] * 20000)
        assert e.value.code == -7
        assert "scratch" in tdse.lib.tdse_last_error(ctx).decode()
    finally:
        tdse.tdse_destroy(ctx)
    # a small context passes the size check and stops at the missing binding
    ctx = tdse.tdse_init_grid([tdse.Grid(300, 3, 0.1).desc()])
    try:
        with pytest.raises(tdse.TdseError) as e:
            tdse.tdse_observables_noalloc(ctx, [tdse.Pulse(0.0, 1.0, 1.0, 0.0, 0.0)], [0.0])
        assert e.value.code == -8
    finally:
        tdse.tdse_destroy(ctx)


def test_calls_before_bind_fail_cleanly(tdse):
    ctx = tdse.tdse_init_grid([tdse.Grid(100, 2, 0.1).desc()])
    try:
        with pytest.raises(tdse.TdseError) as e:
            tdse.tdse_step_taylor(ctx, [tdse.Pulse(0, 1, 1, 0, 0)], [0.0], [1e-3], 4, 1, 0, None)
        assert e.value.code == -8
        assert "bound" in tdse.lib.tdse_last_error(ctx).decode()
    finally:
        tdse.tdse_destroy(ctx)


def test_bind_rejects_small_workspace_before_touching_the_device(tdse):
    # a workspace below the fixed tables is refused (TDSE_E_WORKSPACE) before
    # any HIP call; the pointers are never dereferenced
    ctx = tdse.tdse_init_grid([tdse.Grid(300, 3, 0.1).desc()])
    try:
        need = tdse.lib.tdse_workspace_bytes(ctx, tdse.METHOD_TAYLOR, 8)
        sb = tdse.lib.tdse_state_bytes(ctx)
        code = tdse.lib.tdse_bind(ctx, 1 << 20, 1 << 21, need - 3 * sb, None)
        assert code == -7
        assert "workspace" in tdse.lib.tdse_last_error(ctx).decode()
        # misaligned device pointers are refused as invalid
        assert tdse.lib.tdse_bind(ctx, (1 << 20) + 16, 1 << 21, need, None) == -1
    finally:
        tdse.tdse_destroy(ctx)


def test_lanczos_dims_needs_a_bound_context(tdse):
    ctx = tdse.tdse_init_grid([tdse.Grid(100, 2, 0.1).desc()])
    try:
        with pytest.raises(tdse.TdseError) as e:
            tdse.tdse_lanczos_dims(ctx)
        assert e.value.code == -8
    finally:
        tdse.tdse_destroy(ctx)


def test_pulse_marshalling_keeps_the_shape(tdse):
    arr = tdse._pulses([tdse.Pulse(0.1, 0.5, 2.0, 0.3, 1.0, tdse.PULSE_SINE2_A), tdse.Pulse(0.2, 0.4, 3.0, 0.0, 0.0)])
    assert arr[0].shape == tdse.PULSE_SINE2_A and arr[1].shape == tdse.PULSE_SINE2_E
    assert (arr[0].e0, arr[0].omega, arr[0].n_cycles, arr[0].cep, arr[0].t_on) == (0.1, 0.5, 2.0, 0.3, 1.0)


@pytest.mark.parametrize("stencil,lmax", [(3, 4), (5, 6)])
def test_velocity_gauge_lambda_bound(tdse, orc, stencil, lmax):
    # tdse_lambda_max_bound in the velocity gauge takes a bound on |A/c| and
    # agrees with the oracle's Gershgorin bound; it covers the spectrum of H
    g = tdse.Grid(300, lmax, 0.1, stencil)
    ctx = tdse.tdse_init_grid([g.desc()])
    try:
        with pytest.raises(tdse.TdseError):
            tdse.tdse_set_gauge(ctx, 2)
        tdse.tdse_set_gauge(ctx, tdse.GAUGE_VELOCITY)
        assert tdse.lib.tdse_gauge(ctx) == tdse.GAUGE_VELOCITY
        b = tdse.tdse_lambda_max_bound(ctx, 0, 0.7)
        og = orc.Grid(n=300, lmax=lmax, dr=0.1, stencil=stencil, gauge=orc.VELOCITY)
        assert b == pytest.approx(orc.h_bound(og, 0.7), rel=1e-14)
        lam = eigsh(sparse_h(orc, og, 0.7), k=1, which="LM", return_eigenvectors=False)[0]
        assert abs(lam) <= b
        tdse.tdse_set_gauge(ctx, tdse.GAUGE_LENGTH)
        og = orc.Grid(n=300, lmax=lmax, dr=0.1, stencil=stencil)
        assert tdse.tdse_lambda_max_bound(ctx, 0, 0.7) == pytest.approx(orc.h_bound(og, 0.7), rel=1e-14)
    finally:
        tdse.tdse_destroy(ctx)


def test_absorber_and_flux_need_a_bound_context(tdse):
    ctx = tdse.tdse_init_grid([tdse.Grid(100, 2, 0.1).desc()])
    try:
        for call in (lambda: tdse.tdse_set_absorber(ctx, [50.0], [100.0]), lambda: tdse.tdse_set_flux(ctx, [10]),
                     lambda: tdse.tdse_get_flux(ctx)):
            with pytest.raises(tdse.TdseError) as e:
                call()
            assert e.value.code == -8
    finally:
        tdse.tdse_destroy(ctx)


@pytest.mark.parametrize("stencil", [3, 5])
def test_every_fused_shape_fits_its_workspace_region(tdse, stencil):
    # every fused kernel, term count and strip height builds a tile table
    # that fits the region the context reserved for it (the narrowest tiles
    # of any kind, one row each); checked on the host before any upload
    grids = [tdse.Grid(n, lmax, 0.1, stencil).desc() for n, lmax in ((5001, 7), (130, 0), (777, 33))]
    ctx = tdse.tdse_init_grid(grids)
    try:
        for kind in (0, 1, 2, 3):
            for k in range(1, 9):
                for rows in (1, 3, 16, 64):
                    assert tdse.lib.tdse_set_taylor_fusion(ctx, k, rows, kind) == 0, (kind, k, rows)
    finally:
        tdse.tdse_destroy(ctx)
