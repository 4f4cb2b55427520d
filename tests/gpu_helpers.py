"""Shared helpers of the GPU parity tests: run the library and the oracle on
the same seeded inputs and compare."""
from __future__ import annotations

import sys

import numpy as np

import oracle
import workloads

OBS_N = oracle.OBS_FIXED


def say(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def lib():
    import paper_1308_1856_amd as t
    return t


def read_vector(prop, buf, inst: int) -> np.ndarray:
    """complex128 copy of instance `inst` of a state-shaped device byte buffer."""
    import torch
    g = prop.grids[inst]
    cnt = (g.lmax + 1) * g.n
    if prop.elem == 12:
        # 48-bit storage: plane h (upper words of re, im), then plane l (the
        # next 16 bits of re in the low half, of im in the high half)
        words = buf.view(torch.int32).cpu().numpy().view(np.uint32)
        plane = (words.size * 4) // 12
        off = prop.offsets[inst]
        h = words[2 * off:2 * (off + cnt)].astype(np.uint64)
        lo = words[2 * plane + off:2 * plane + off + cnt].astype(np.uint64)
        re = (h[0::2] << np.uint64(32)) | ((lo & np.uint64(0xFFFF)) << np.uint64(16))
        im = (h[1::2] << np.uint64(32)) | (lo & np.uint64(0xFFFF0000))
        return re.view(np.float64) + 1j * im.view(np.float64)
    dt = torch.float64 if prop.elem == 16 else torch.float32
    flat = buf.view(dt)
    off = prop.offsets[inst] * 2
    vals = flat[off:off + 2 * cnt].cpu().numpy().astype(np.float64)
    return vals[0::2] + 1j * vals[1::2]


def orc_grid(g) -> oracle.Grid:
    return oracle.Grid(n=g.n, lmax=g.lmax, dr=g.dr, stencil=g.stencil, z=g.z)


def orc_pulse(p) -> oracle.Pulse:
    return oracle.Pulse(p.e0, p.omega, p.n_cycles, p.cep, p.t_on)


def to_fp32(v: np.ndarray) -> np.ndarray:
    return v.astype(np.complex64).astype(np.complex128)


def to_fp48(v: np.ndarray) -> np.ndarray:
    """The value 48-bit storage keeps: each FP64 component rounded to nearest
    (ties away from zero) at 36 mantissa bits."""
    def r(x):
        b = np.ascontiguousarray(x, dtype=np.float64).view(np.uint64) + np.uint64(0x8000)
        return (b & ~np.uint64(0xFFFF)).view(np.float64)
    return r(v.real) + 1j * r(v.imag)


def rel_err(a: np.ndarray, b: np.ndarray) -> float:
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def series_err(gpu: np.ndarray, ref: np.ndarray, floor: float) -> np.ndarray:
    """Per column: max_t |gpu - ref| / max(max_t |ref|, floor)."""
    scale = np.maximum(np.max(np.abs(ref), axis=0), floor)
    return np.max(np.abs(gpu - ref), axis=0) / scale


def obs_columns(setup) -> int:
    return OBS_N + len(setup.state_l)


EPS = np.finfo(np.float64).eps


def obs_abs_tol(g: oracle.Grid, setup, ref: np.ndarray, floor: float = 1e-13,
                c: float = 10.0) -> np.ndarray:
    """Absolute tolerance per observable column for the reference series `ref`.

    Fixed columns get `floor` (summation-order round-off).  A population
    P = |<phi_nl|f_l>|^2 also inherits the difference between two
    independently computed eigenvectors, |d phi| <= delta = c eps ||h_l|| /
    gap_nl (eigenvector conditioning), so |dP| <= 2 sqrt(P_max) delta +
    delta^2 (||f_l|| <= 1); p_bound sums these."""
    e6, _, states6 = oracle.bound_states(g, 6)
    energy = {st: e for st, e in zip(states6, e6)}
    tol = [floor] * oracle.OBS_FIXED
    pb = 0.0
    for k, (n, l) in enumerate(zip(setup.state_n, setup.state_l)):
        hl = oracle.h_bound(oracle.Grid(n=g.n, lmax=int(l), dr=g.dr, stencil=g.stencil, z=g.z), 0.0)
        nb = [energy[(j, l)] for j in (n - 1, n + 1) if (j, l) in energy]
        gap = min(abs(energy[(n, l)] - x) for x in nb)
        delta = c * EPS * hl / gap
        pmax = float(np.max(np.abs(ref[..., oracle.OBS_FIXED + k])))
        t = 2 * np.sqrt(pmax) * delta + delta * delta + floor
        tol.append(t)
        pb += t
    tol[4] = pb + floor
    return np.array(tol)


def series_ratio(gpu: np.ndarray, ref: np.ndarray, rel: float, abs_tol) -> np.ndarray:
    """Per column: max_t |gpu - ref| / (rel * max_t |ref| + abs_tol); <= 1 passes."""
    return np.max(np.abs(gpu - ref), axis=0) / (rel * np.max(np.abs(ref), axis=0) + abs_tol)
