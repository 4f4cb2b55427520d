#!/usr/bin/env python3
"""Throughput of the TDSE hot path on one MI355X.

One step = one Taylor-8 time step of the FP64 single-instance workload
(N = 20000, dr = 0.05, lmax = 64, 5-point stencil): the field at the step
midpoint, eight fused Horner sweeps of H(t).psi and the FP64 observables
(norm, p_g, the 15 populations n <= 5, p_ion, dipole, dipole acceleration)
after every step.  `value` is H.psi applications per second (8 per step).

Also reported on the same line:
  roofline      the Horner-term kernel: algorithmic bytes per launch (read
                w, read psi, write w: 3 x 16 B per unknown) over its mean
                duration from HIP events on the library's stream, against
                the 8 TB/s HBM peak;
  fp32_mixed    the same workload with FP32 storage and FP64 arithmetic and
                reductions: steps/s, speedup over FP64, and its error against
                the FP64 GPU run;
  cpu_baseline  the FP64 C oracle on the host for a bounded sample of the
                same workload (whole steps), one core.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402

METRIC = "H·ψ applies/s & HBM GB/s fraction; steps/s FP32-mixed vs FP64 at stated error"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", default="hydrogen_n20000_l64_fp64_taylor8",
                    choices=sorted(workloads.WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_prop(tdse, wl, precision, method_code):
    g = tdse.Grid(wl.n, wl.lmax, wl.dr, wl.stencil, precision, wl.z, wl.r_ion)
    prop = tdse.Propagator([g], methods=((method_code, wl.order),))
    prop.set_state(0, None)
    return prop


def run_steps(prop, tdse, wl, t0, nsteps, obs):
    p = tdse.Pulse(wl.pulse.e0, wl.pulse.omega, wl.pulse.n_cycles, wl.pulse.cep, wl.pulse.t_on)
    if wl.method == "taylor":
        prop.step_taylor(p, t0, wl.dt, wl.order, nsteps, wl.obs_every, obs)
    elif wl.method == "rk4":
        prop.step_rk4(p, t0, wl.dt, nsteps, wl.obs_every, obs)
    else:
        prop.step_lanczos(p, t0, wl.dt, wl.order, nsteps, wl.obs_every, obs)


def timed(prop, tdse, wl, torch, steps, warmup, kernel):
    obs_w = prop.obs_buffer(max(warmup, 1), wl.obs_every)
    obs = prop.obs_buffer(steps, wl.obs_every)
    run_steps(prop, tdse, wl, wl.t0, warmup, obs_w)
    torch.cuda.synchronize()
    t_start = wl.t0 + warmup * wl.dt
    t0 = time.perf_counter()
    run_steps(prop, tdse, wl, t_start, steps, obs)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # second pass of the same length with HIP events around each launch of the
    # dominant kernel (kept out of the wall-clock pass above)
    prop.timing(True)
    run_steps(prop, tdse, wl, t_start + steps * wl.dt, steps, obs)
    launches, kms = prop.timing_read(kernel)
    prop.timing(False)
    torch.cuda.synchronize()
    return wall, launches, kms, obs


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 "
                                   "(the multi-GPU sharding is described, not built)"}))
        sys.exit(2)
    import torch
    import paper_1308_1856_amd as tdse

    wl = workloads.WORKLOADS[args.workload]
    prec = tdse.FP64 if wl.precision == "fp64" else tdse.FP32
    mcode = {"taylor": tdse.METHOD_TAYLOR, "rk4": tdse.METHOD_RK4,
             "lanczos": tdse.METHOD_LANCZOS}[wl.method]
    kernel = {"taylor": "taylor_term", "rk4": "rk4_stage", "lanczos": "lanczos_sweep_a"}[wl.method]
    applies_per_step = {"taylor": wl.order, "rk4": 4, "lanczos": wl.order}[wl.method]
    U = wl.unknowns
    elem = 16 if prec == tdse.FP64 else 8
    bytes_per_unknown = {"taylor": 3 * elem, "rk4": 4 * elem}.get(wl.method)

    log(f"bench: workload {wl.name} U={U} method={wl.method}-{wl.order} dt={wl.dt} "
        f"steps={args.steps} warmup={args.warmup}")
    prop = make_prop(tdse, wl, prec, mcode)
    wall, launches, kms, obs = timed(prop, tdse, wl, torch, args.steps, args.warmup, kernel)
    psi_main = prop.get_state(0)
    steps_per_s = args.steps / wall
    value = applies_per_step * steps_per_s
    avg_ms = kms / max(launches, 1)
    log(f"bench: {steps_per_s:.1f} steps/s, {value:.1f} applies/s, {kernel} mean {avg_ms * 1e3:.2f} us "
        f"over {launches} launches")
    achieved = None
    if bytes_per_unknown:
        achieved = bytes_per_unknown * U / (avg_ms * 1e-3) / 1e9
    obs_last = obs.cpu().numpy()[0, -1]
    prop.close()
    del prop
    torch.cuda.empty_cache()

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "H·ψ applies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == tdse.FP64 else "f32-storage/f64-arith",
        "data": "synthetic",
        "config": {"workload": wl.name, "n_r": wl.n, "lmax": wl.lmax, "dr": wl.dr,
                   "stencil": wl.stencil, "method": wl.method, "order": wl.order,
                   "dt": wl.dt, "dt_nominal": wl.dt_nominal, "unknowns": U,
                   "obs_every": wl.obs_every, "parallelism": "single GPU"},
        "steps_per_s": steps_per_s,
        "roofline": {
            "bound": "hbm",
            "kernel": kernel,
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
            "traffic": None,
            "algorithmic_bytes_per_launch": (bytes_per_unknown * U) if bytes_per_unknown else None,
            "mean_launch_us": avg_ms * 1e3,
            "launches_timed": launches,
        },
        "final_observables": {"norm": float(obs_last[2]), "p_ion": float(obs_last[5]),
                              "p_bound": float(obs_last[4])},
    }

    if not args.no_fp32 and prec == tdse.FP64:
        wl32 = wl.with_(precision="fp32")
        prop = make_prop(tdse, wl32, tdse.FP32, mcode)
        wall32, l32, k32, obs32 = timed(prop, tdse, wl32, torch, args.steps, args.warmup, kernel)
        psi32 = prop.get_state(0)
        o32 = obs32.cpu().numpy()[0, -1]
        prop.close()
        del prop
        torch.cuda.empty_cache()
        sps32 = args.steps / wall32
        rel_state = float(np.linalg.norm(psi32 - psi_main) / np.linalg.norm(psi_main))
        out["fp32_mixed"] = {
            "steps_per_s": sps32,
            "applies_per_s": applies_per_step * sps32,
            "speedup_vs_fp64": sps32 / steps_per_s,
            "kernel_mean_us": 1e3 * k32 / max(l32, 1),
            "kernel_gbs": (3 * 8 * U / (k32 / max(l32, 1) * 1e-3) / 1e9) if wl.method == "taylor" else None,
            "rel_state_error_vs_fp64": rel_state,
            "norm_drift_vs_fp64": float(abs(o32[2] - obs_last[2])),
            "p_bound_rel_error_vs_fp64": float(abs(o32[4] - obs_last[4]) / abs(obs_last[4])),
            "steps_compared": 2 * args.steps + args.warmup,
        }
        log(f"bench: fp32 {sps32:.1f} steps/s ({sps32 / steps_per_s:.2f}x), state diff {rel_state:.2e}")

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds, applies_per_step)

    print(json.dumps(out), flush=True)


def cpu_baseline(wl, seconds, applies_per_step):
    import oracle
    g = oracle.Grid(n=wl.n, lmax=wl.lmax, dr=wl.dr, stencil=wl.stencil, z=wl.z)
    p = oracle.Pulse(wl.pulse.e0, wl.pulse.omega, wl.pulse.n_cycles, wl.pulse.cep, wl.pulse.t_on)
    setup = oracle.obs_setup(g, r_ion=wl.r_ion)
    psi, _ = oracle.initial_state(g)
    code = {"taylor": oracle.TAYLOR, "rk4": oracle.RK4, "lanczos": oracle.LANCZOS}[wl.method]
    t0 = time.perf_counter()
    psi, _, _ = oracle.propagate(g, p, code, wl.order, wl.t0, wl.dt, 1, 1, setup, psi)
    one = time.perf_counter() - t0
    n = max(1, int(seconds / max(one, 1e-6)))
    t0 = time.perf_counter()
    oracle.propagate(g, p, code, wl.order, wl.t0 + wl.dt, wl.dt, n, 1, setup, psi)
    el = time.perf_counter() - t0
    log(f"bench: cpu oracle {n} steps in {el:.1f} s")
    return {"value": applies_per_step * n / el, "unit": "H·ψ applies/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{n} whole {wl.method}-{wl.order} steps (with per-step observables) of the "
                      f"same workload, FP64 C oracle, 1 thread, {el:.1f} s",
            "steps_per_s": n / el}


if __name__ == "__main__":
    main()
