"""Writes the long-window golden trajectories of the FP64 oracle.

Calls only the oracle (and the seeded input recipes of `workloads`); nothing
here comes from the GPU library.  Run from the repository root:

    python tests/golden/make_golden.py [name ...]

Each trajectory is one .npz file (float64 arrays, no pickles) plus an entry in
golden_trajectories.json with the recipe:
  rk4_n2000_l8_full, taylor4_n2000_l8_full
      N = 2000, dr = 0.1, lmax = 8, 3-point; E0 = 0.0534, w = 0.057, 2-cycle
      sine-squared pulse with a sine carrier; dt = 5e-4 (stable), 440,000
      steps to t = 220 from the normalised 1s state; records every 1000 steps;
      the final state in full.
  taylor8_n20000_l64_window
      N = 20000, dr = 0.05, lmax = 64, 5-point; 800 nm, 1e14 W/cm^2, 4-cycle
      pulse; Taylor-8 at dt = 3e-6, 2000 steps from mid-pulse, starting from
      workloads.mixed_state(5) normalised (bound, excited and outgoing parts);
      records every 10 steps; every 101st element of the final state and its
      projections <v_k|psi> on three seeded vectors v_k =
      workloads.random_state(900 + k).
  lanczos20_n20000_l64_window
      the same grid and pulse; Lanczos m = 20 at dt = 1e-4 (lambda_max dt =
      83), 200 steps from mid-pulse, same start; records every 10 steps; final
      state sampled as above.  The oracle also runs from the start perturbed
      by a seeded relative 1e-15 (state_sample_perturbed, records_perturbed):
      at this step the two runs agree to round-off (the Krylov step is
      reproducible), while at the workload's dt = 0.01 (lambda_max dt = 8e3)
      the same perturbation grows to a 1% difference of the state within 200
      steps, where no two implementations can agree closer than that.
"""
from __future__ import annotations

import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402

SAMPLE_STRIDE = 101
N_PROJ = 3


def cfg1(method_name):
    wl = workloads.WORKLOADS["hydrogen_n2000_l8_fp64"]
    return dict(n=wl.n, lmax=wl.lmax, dr=wl.dr, stencil=wl.stencil, e0=wl.pulse.e0, omega=wl.pulse.omega,
                n_cycles=wl.pulse.n_cycles, cep=wl.pulse.cep, t_on=0.0, method=method_name,
                order=4, dt=wl.dt, steps=440_000, obs_every=1000, t0=0.0, r_ion=wl.r_ion, start="1s",
                state="full")


def cfg2(method_name, order, dt, steps, perturbed=False):
    wl = workloads.WORKLOADS["hydrogen_n20000_l64_fp64_taylor8"]
    return dict(n=wl.n, lmax=wl.lmax, dr=wl.dr, stencil=wl.stencil, e0=wl.pulse.e0, omega=wl.pulse.omega,
                n_cycles=wl.pulse.n_cycles, cep=wl.pulse.cep, t_on=0.0, method=method_name, order=order,
                dt=dt, steps=steps, obs_every=10, t0=0.5 * wl.pulse.duration, r_ion=wl.r_ion,
                start="mixed_state(5)", state="sampled", perturbed=perturbed)


TRAJ = {
    "rk4_n2000_l8_full": cfg1("rk4"),
    "taylor4_n2000_l8_full": cfg1("taylor"),
    "taylor8_n20000_l64_window": cfg2("taylor", 8, 3e-6, 2000),
    "lanczos20_n20000_l64_window": cfg2("lanczos", 20, 1e-4, 200, perturbed=True),
}


def start_state(c, g):
    if c["start"] == "1s":
        psi, _ = oracle.initial_state(g)
        return psi
    v = workloads.mixed_state(5, c["n"], c["lmax"], c["dr"])
    return v / math.sqrt(c["dr"] * float(np.vdot(v, v).real))


def projection_vectors(c):
    return [workloads.random_state(900 + k, c["n"], c["lmax"]) for k in range(N_PROJ)]


def make(name):
    c = TRAJ[name]
    g = oracle.Grid(n=c["n"], lmax=c["lmax"], dr=c["dr"], stencil=c["stencil"])
    p = oracle.Pulse(c["e0"], c["omega"], c["n_cycles"], c["cep"], c["t_on"])
    setup = oracle.obs_setup(g, r_ion=c["r_ion"])
    psi0 = start_state(c, g)
    code = {"rk4": oracle.RK4, "taylor": oracle.TAYLOR, "lanczos": oracle.LANCZOS}[c["method"]]
    oracle.set_threads(oracle.max_threads())
    t0 = time.perf_counter()
    psi, obs, used = oracle.propagate(g, p, code, c["order"], c["t0"], c["dt"], c["steps"], c["obs_every"],
                                      setup, psi0)
    wall = time.perf_counter() - t0
    arrays = {"records": obs}
    if c["state"] == "full":
        arrays["state"] = psi
    else:
        arrays["state_sample"] = psi[::SAMPLE_STRIDE]
        arrays["projections"] = np.array([np.vdot(v, psi) for v in projection_vectors(c)])
    if c.get("perturbed"):
        rng = np.random.default_rng(4242)
        pert = psi0 * (1 + 1e-15 * (rng.standard_normal(psi0.size) + 1j * rng.standard_normal(psi0.size)))
        psi_p, obs_p, _ = oracle.propagate(g, p, code, c["order"], c["t0"], c["dt"], c["steps"], c["obs_every"],
                                           setup, pert)
        arrays["state_sample_perturbed"] = psi_p[::SAMPLE_STRIDE]
        arrays["records_perturbed"] = obs_p
    np.savez(os.path.join(HERE, name + ".npz"), **arrays)
    entry = dict(c, file=name + ".npz", sample_stride=SAMPLE_STRIDE, n_projections=N_PROJ,
                 oracle_seconds=round(wall, 1), oracle_threads=oracle.max_threads(),
                 record_columns=list(oracle.OBS_NAMES) + [f"P_{n}{'spdfg'[l]}" for n, l in
                                                          zip(setup.state_n, setup.state_l)],
                 krylov_min=int(used))
    print(f"{name}: {c['steps']} steps in {wall:.1f} s", flush=True)
    return entry


def main(names):
    meta_path = os.path.join(HERE, "golden_trajectories.json")
    meta = json.load(open(meta_path)) if os.path.exists(meta_path) else {}
    for name in names or list(TRAJ):
        meta[name] = make(name)
        with open(meta_path, "w") as f:
            json.dump(meta, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:])
