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


def rel_err(a: np.ndarray, b: np.ndarray) -> float:
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def series_err(gpu: np.ndarray, ref: np.ndarray, floor: float) -> np.ndarray:
    """Per column: max_t |gpu - ref| / max(max_t |ref|, floor)."""
    scale = np.maximum(np.max(np.abs(ref), axis=0), floor)
    return np.max(np.abs(gpu - ref), axis=0) / scale


def obs_columns(setup) -> int:
    return OBS_N + len(setup.state_l)
