#!/usr/bin/env python3
"""Throughput of the TDSE hot path on one MI355X.

One step = one Taylor-8 time step of the FP64 single-instance workload
(N = 20000, dr = 0.05, lmax = 64, 5-point stencil): the field at the step
midpoint, eight Horner terms of H(t).psi and the FP64 observables (norm,
p_g, the 15 populations n <= 5, p_ion, dipole, dipole acceleration) after
every step.  `value` is H.psi applications per second (8 per step).  The
execution shape (sweep tiles; one launch per Horner term or K terms per
fused launch, and which fused kernel) is chosen by the library's autotuners
before the timed region (--autotune 2, the default).

Also reported on the same line:
  roofline      the dominant kernel of the step (the Horner-term sweep, or
                the fused K-term kernel): algorithmic bytes per launch (read
                the input vector, read psi, write the output: 3 x c B per
                unknown, c = 16 B FP64 / 8 B FP32) over its mean duration
                from HIP events on the library's stream, against the 8 TB/s
                HBM peak; `traffic` comes from the committed rocprofv3
                counter summary for the same kernel and shape (null if there
                is none, or if the kernel source changed since);
  hpsi_sweep    the plain H.psi apply (tdse_apply_H: read psi, write H psi,
                2c B per unknown) on the same grid, same report;
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
BATCH_NAME = "batch256_fp32_taylor8"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", default="hydrogen_n20000_l64_fp64_taylor8",
                    choices=sorted(workloads.WORKLOADS) + [BATCH_NAME])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--graphs", type=int, default=1, help="replay step chunks as HIP graphs")
    ap.add_argument("--rk4-stages", action="store_true",
                    help="RK4 in four stage launches per step (default: one launch per step)")
    ap.add_argument("--autotune", type=int, default=2,
                    help="0: fixed shapes; 1: autotune the sweep tiles; 2: also choose the Taylor fusion")
    ap.add_argument("--sweep", default=None, metavar="ROWS,VARIANT",
                    help="fixed sweep tile shape instead of the sweep autotuner (profiling runs)")
    ap.add_argument("--fusion", default=None, metavar="K,ROWS,KIND[,OBS]",
                    help="fixed Taylor fusion instead of the Taylor autotuner (profiling runs); OBS 1: the "
                         "main observables summed in the step's last strip launch, 0: by their own pass")
    return ap.parse_args()


def apply_shape(prop, args, autotune, order):
    """Execution shape: explicit (--sweep / --fusion) or from the autotuners."""
    if args.sweep:
        rows, variant = (int(x) for x in args.sweep.split(","))
        prop.set_sweep_shape(rows, variant)
    elif autotune:
        prop.autotune()
    if args.fusion:
        vals = [int(x) for x in args.fusion.split(",")]
        prop.set_taylor_fusion(*vals[:3])
        if len(vals) > 3:
            prop.set_obs_fusion(bool(vals[3]))
    elif autotune > 1 and order:
        prop.autotune_taylor(order)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_prop(tdse, wl, precision, method_code, graphs=True, autotune=True):
    g = tdse.Grid(wl.n, wl.lmax, wl.dr, wl.stencil, precision, wl.z, wl.r_ion)
    methods = ((method_code, wl.order), (tdse.METHOD_TAYLOR, 2), (tdse.METHOD_TUNE, 0))
    prop = tdse.Propagator([g], methods=methods, graphs=bool(graphs))
    apply_shape(prop, ARGS, autotune, wl.order if wl.method == "taylor" else 0)
    if wl.method == "rk4" and ARGS is not None and ARGS.rk4_stages:
        prop.set_rk4_fusion(False)
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


def timed(prop, tdse, wl, torch, steps, warmup, kernel, graphs):
    obs_w = prop.obs_buffer(max(warmup, 1), wl.obs_every)
    obs = prop.obs_buffer(steps, wl.obs_every)
    t = wl.t0
    run_steps(prop, tdse, wl, t, warmup, obs_w)
    t += warmup * wl.dt
    if graphs:
        # capture and instantiate the chunk graphs of a K-step call outside the
        # timed region (replays of the same pattern reuse them)
        run_steps(prop, tdse, wl, t, steps, obs)
        t += steps * wl.dt
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run_steps(prop, tdse, wl, t, steps, obs)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    t += steps * wl.dt
    # second pass of the same length with HIP events around each launch of the
    # dominant kernel (direct launches; kept out of the wall-clock pass above)
    prop.timing(True)
    run_steps(prop, tdse, wl, t, steps, obs)
    launches, kms = prop.timing_read(kernel)
    prop.timing(False)
    torch.cuda.synchronize()
    return wall, launches, kms, obs


def source_digest(name):
    """sha256 over a kernel source and the device headers it includes."""
    import hashlib
    h = hashlib.sha256()
    for part in (name, "device_common.hpp", "tdse_internal.hpp"):
        with open(os.path.join(ROOT, "paper_1308_1856_amd", "csrc", part), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def shape_of(prop, kernel):
    if kernel == "taylor_fused":
        return {"fuse_k": prop.taylor_fusion, "rows": getattr(prop, "fusion_rows", None),
                "kind": prop.taylor_fusion_kind, "obs_fusion": int(prop.obs_fusion)}
    return {"tile_rows": prop.tile_rows, "sweep_variant": prop.sweep_variant}


def profile_entry(workload, kernel, precision, shape):
    """The committed counter summary of this kernel and shape, or None (also
    when the kernel source changed since the counters were taken)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        table = json.load(f)
    for e in table.get("entries", []):
        if (e["workload"], e["kernel"], e["precision"]) != (workload, kernel, precision):
            continue
        if any(e["shape"].get(k) != v for k, v in shape.items() if k in e["shape"]):
            continue
        if e.get("source_sha256") != source_digest(e["source"]):
            return None
        return e
    return None


def traffic_for(workload, kernel, precision, shape):
    """HBM bytes per launch from the committed counter summary, or None."""
    e = profile_entry(workload, kernel, precision, shape)
    return e["hbm_bytes_per_launch"] if e else None


def valu_busy_for(workload, kernel, precision, shape):
    """VALU busy percentage (rocprofv3 VALUBusy) from the committed summary, or None."""
    e = profile_entry(workload, kernel, precision, shape)
    return e.get("valu_busy_pct") if e else None


def hpsi_sweep(prop, tdse, torch, U, elem, reps=40):
    """Mean duration of the plain H.psi apply on the bound grid (HIP events)."""
    out = prop.new_vector()
    e = 0.01
    for _ in range(3):
        prop.apply_H(e, prop.state, out)
    torch.cuda.synchronize()
    prop.timing(True)
    for _ in range(reps):
        prop.apply_H(e, prop.state, out)
    launches, kms = prop.timing_read("apply_h")
    prop.timing(False)
    torch.cuda.synchronize()
    us = 1e3 * kms / max(launches, 1)
    bytes_ = 2 * elem * U
    gbs = bytes_ / (us * 1e-6) / 1e9
    return {"bound": "hbm", "kernel": "apply_h", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": gbs / HBM_PEAK_GBS, "algorithmic_bytes_per_launch": bytes_, "mean_launch_us": us,
            "launches_timed": launches, "applies_per_s": 1e6 / us,
            "shape": {"tile_rows": prop.tile_rows, "sweep_variant": prop.sweep_variant}}


def taylor_bytes_per_launch(elem, U, launches, steps):
    """Algorithmic bytes per Horner launch, averaged over a step's L launches.

    Each launch reads its input vector and psi and writes its output (3 c U);
    the first launch of a step reads psi as its input, so it reads it once
    (2 c U): (3 L - 1) c U per step.
    """
    L = max(launches, 1) / max(steps, 1)
    return (3.0 * L - 1.0) / L * elem * U


def dominant_kernel(prop, method):
    """Timing family of the launch that carries a step's sweeps."""
    if method == "taylor":
        return "taylor_fused" if prop.taylor_fusion > 0 else "taylor_term"
    if method == "rk4":
        return "rk4_fused" if prop.rk4_fusion else "rk4_stage"
    return {"lanczos": "lanczos_sweep_a"}[method]


def batch_setup(tdse, precision):
    members = workloads.batch_members()
    grids, pulses = [], []
    for m in members:
        R = m.n * workloads.BATCH_DR
        grids.append(tdse.Grid(m.n, m.lmax, workloads.BATCH_DR, workloads.BATCH_STENCIL, precision,
                               1.0, workloads.BATCH_R_ION_FRACTION * R))
        pp = m.pulse
        pulses.append(tdse.Pulse(pp.e0, pp.omega, pp.n_cycles, pp.cep, pp.t_on))
    return members, grids, pulses


def run_batch_prec(tdse, torch, precision, args, autotune=None):
    members, grids, pulses = batch_setup(tdse, precision)
    order = workloads.BATCH_ORDER
    autotune = args.autotune if autotune is None else autotune
    prop = tdse.Propagator(grids, methods=((tdse.METHOD_TAYLOR, order),
                                           (tdse.METHOD_TUNE, 0)), graphs=bool(args.graphs))
    if autotune <= 1:
        # the plain path: one launch per term, whatever --fusion says
        saved, args.fusion = args.fusion, None
        apply_shape(prop, args, autotune, order)
        args.fusion = saved
    else:
        apply_shape(prop, args, autotune, order)
    kernel = dominant_kernel(prop, "taylor")
    y = tdse.tdse_taylor_stability_limit(order)
    dts = [workloads.BATCH_DT_SAFETY * y / prop.lambda_max_bound(k, abs(p.e0)) for k, p in enumerate(pulses)]
    for k in range(len(grids)):
        prop.set_state(k, None)
    t = [0.0] * len(grids)

    def run(n, obs):
        nonlocal t
        prop.step_taylor(pulses, t, dts, order, n, 1, obs)
        t = [tk + n * d for tk, d in zip(t, dts)]

    obs_w = prop.obs_buffer(max(args.warmup, 1), 1)
    obs = prop.obs_buffer(args.steps, 1)
    run(args.warmup, obs_w)
    if args.graphs:
        run(args.steps, obs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run(args.steps, obs)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prop.timing(True)
    run(args.steps, obs)
    launches, kms = prop.timing_read(kernel)
    prop.timing(False)
    rows = (prop.tile_rows, prop.sweep_variant, prop.taylor_fusion)
    o = obs.cpu().numpy()[:, -1, :]
    U = sum((g.lmax + 1) * g.n for g in grids)
    elem = 16 if precision == tdse.FP64 else 8
    prec_name = "fp64" if precision == tdse.FP64 else "fp32"
    shape = shape_of(prop, kernel)
    traffic = traffic_for(BATCH_NAME, kernel, prec_name, shape)
    valu = valu_busy_for(BATCH_NAME, kernel, prec_name, shape)
    sweep = hpsi_sweep(prop, tdse, torch, U, elem)
    sweep["traffic"] = traffic_for(BATCH_NAME, "apply_h", prec_name, sweep["shape"])
    sweep["valu_busy_pct"] = valu_busy_for(BATCH_NAME, "apply_h", prec_name, sweep["shape"])
    prop.close()
    del prop
    torch.cuda.empty_cache()
    return dict(wall=wall, launches=launches, kms=kms, rows=rows, obs=o, U=U, dts=dts, n=len(grids),
                kernel=kernel, shape=shape, traffic=traffic, valu=valu, sweep=sweep)


def run_batch(args, tdse, torch):
    log(f"bench: batch of 256 members, FP32 storage, Taylor-8, steps={args.steps} warmup={args.warmup}")
    r32 = run_batch_prec(tdse, torch, tdse.FP32, args)
    log(f"bench: batch FP32 {args.steps / r32['wall']:.1f} steps/s")
    r64 = run_batch_prec(tdse, torch, tdse.FP64, args)
    log(f"bench: batch FP64 {args.steps / r64['wall']:.1f} steps/s")
    # the plain FP64 path: one launch per Horner term (sweep tiles tuned, no fusion)
    r64p = run_batch_prec(tdse, torch, tdse.FP64, args, autotune=min(args.autotune, 1))
    log(f"bench: batch FP64 one launch per term {args.steps / r64p['wall']:.1f} steps/s")
    sps = args.steps / r32["wall"]
    U = r32["U"]
    avg_ms = r32["kms"] / max(r32["launches"], 1)
    bpl32 = taylor_bytes_per_launch(8, U, r32["launches"], args.steps)
    achieved = bpl32 / (avg_ms * 1e-3) / 1e9
    avg64 = r64["kms"] / max(r64["launches"], 1)
    bpl64 = taylor_bytes_per_launch(16, U, r64["launches"], args.steps)
    drift = float(np.max(np.abs(r32["obs"][:, 2] - r64["obs"][:, 2])))
    pb = float(np.max(np.abs(r32["obs"][:, 4] - r64["obs"][:, 4]) / np.abs(r64["obs"][:, 4])))
    out = {
        "metric": METRIC, "value": workloads.BATCH_ORDER * r32["n"] * sps, "unit": "H·ψ applies/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * r32["wall"] / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32-storage/f64-arith", "data": "synthetic",
        "config": {"workload": BATCH_NAME, "members": r32["n"], "unknowns": U,
                   "seed": workloads.BATCH_SEED, "dr": workloads.BATCH_DR, "stencil": workloads.BATCH_STENCIL,
                   "method": "taylor", "order": workloads.BATCH_ORDER, "obs_every": 1,
                   "dt_range": [min(r32["dts"]), max(r32["dts"])], "parallelism": "single GPU",
                   "tile_rows_variant_fusion": r32["rows"], "kernel_shape": r32["shape"],
                   "graphs": bool(args.graphs)},
        "steps_per_s": sps,
        "roofline": {"bound": "hbm", "kernel": r32["kernel"], "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": r32["traffic"],
                     "valu_busy_pct": r32["valu"],
                     "algorithmic_bytes_per_launch": bpl32, "mean_launch_us": avg_ms * 1e3,
                     "launches_timed": r32["launches"]},
        "hpsi_sweep": r32["sweep"],
        "fp64_batched": {"steps_per_s": args.steps / r64["wall"],
                         "fp32_speedup_vs_fp64": sps / (args.steps / r64["wall"]),
                         "kernel": r64["kernel"], "kernel_mean_us": avg64 * 1e3,
                         "kernel_gbs": bpl64 / (avg64 * 1e-3) / 1e9,
                         "max_norm_diff_fp32_vs_fp64": drift,
                         "max_p_bound_rel_diff_fp32_vs_fp64": pb,
                         "steps_compared": (3 if args.graphs else 2) * args.steps + args.warmup,
                         "hpsi_sweep": r64["sweep"]},
        "fp64_one_launch_per_term": {"steps_per_s": args.steps / r64p["wall"],
                                     "fp32_speedup_vs_it": sps / (args.steps / r64p["wall"]),
                                     "kernel": r64p["kernel"],
                                     "kernel_mean_us": 1e3 * r64p["kms"] / max(r64p["launches"], 1)},
    }
    if not args.no_cpu_baseline:
        members = workloads.batch_members()
        import oracle
        m = members[0]
        wl = workloads.Workload("batch_member0", m.n, m.lmax, workloads.BATCH_DR, workloads.BATCH_STENCIL,
                                "fp64", "taylor", workloads.BATCH_ORDER, m.pulse, dt=r32["dts"][0],
                                dt_nominal=float("nan"), nsteps=0, obs_every=1,
                                r_ion=workloads.BATCH_R_ION_FRACTION * m.n * workloads.BATCH_DR)
        cb = cpu_baseline(wl, args.cpu_seconds, workloads.BATCH_ORDER)
        cb["sample"] = "member 0 of the batch (N=%d, lmax=%d): %s" % (m.n, m.lmax, cb["sample"])
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


ARGS = None


def main():
    global ARGS
    args = parse()
    ARGS = args
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; --gpus must be 1 "
                                   "(the multi-GPU sharding is described, not implemented)"}))
        sys.exit(2)
    import torch
    import paper_1308_1856_amd as tdse
    if args.workload == BATCH_NAME:
        return run_batch(args, tdse, torch)

    wl = workloads.WORKLOADS[args.workload]
    prec = tdse.FP64 if wl.precision == "fp64" else tdse.FP32
    mcode = {"taylor": tdse.METHOD_TAYLOR, "rk4": tdse.METHOD_RK4,
             "lanczos": tdse.METHOD_LANCZOS}[wl.method]
    applies_per_step = {"taylor": wl.order, "rk4": 4, "lanczos": wl.order}[wl.method]
    U = wl.unknowns
    elem = 16 if prec == tdse.FP64 else 8
    bytes_per_unknown = {"taylor": 3 * elem, "rk4": 4 * elem}.get(wl.method)

    log(f"bench: workload {wl.name} U={U} method={wl.method}-{wl.order} dt={wl.dt} "
        f"steps={args.steps} warmup={args.warmup}")
    prop = make_prop(tdse, wl, prec, mcode, args.graphs, args.autotune)
    tile_rows = prop.tile_rows
    variant = prop.sweep_variant
    fusion = prop.taylor_fusion
    kernel = dominant_kernel(prop, wl.method)
    wall, launches, kms, obs = timed(prop, tdse, wl, torch, args.steps, args.warmup, kernel, args.graphs)
    psi_main = prop.get_state(0)
    steps_per_s = args.steps / wall
    value = applies_per_step * steps_per_s
    avg_ms = kms / max(launches, 1)
    log(f"bench: {steps_per_s:.1f} steps/s, {value:.1f} applies/s, {kernel} mean {avg_ms * 1e3:.2f} us "
        f"over {launches} launches")
    bytes_per_launch = None
    if wl.method == "taylor":
        bytes_per_launch = taylor_bytes_per_launch(elem, U, launches, args.steps)
    elif wl.method == "lanczos":
        # sweep A of iteration j reads q_0..q_j and writes w: (j + 2) c U,
        # averaged over j = 0 .. m-1
        bytes_per_launch = (wl.order + 3) / 2.0 * elem * U
    elif kernel == "rk4_fused":
        # one launch per step: read psi, write the new psi
        bytes_per_launch = 2.0 * elem * U
    elif bytes_per_unknown:
        bytes_per_launch = bytes_per_unknown * U
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9 if bytes_per_launch else None
    obs_last = obs.cpu().numpy()[0, -1]
    shape = shape_of(prop, kernel)
    prec_name = "fp64" if prec == tdse.FP64 else "fp32"
    traffic = traffic_for(wl.name, kernel, prec_name, shape)
    valu = valu_busy_for(wl.name, kernel, prec_name, shape)
    sweep = hpsi_sweep(prop, tdse, torch, U, elem)
    sweep["traffic"] = traffic_for(wl.name, "apply_h", prec_name, sweep["shape"])
    sweep["valu_busy_pct"] = valu_busy_for(wl.name, "apply_h", prec_name, sweep["shape"])
    log(f"bench: H.psi apply {sweep['mean_launch_us']:.2f} us = {sweep['achieved']:.0f} GB/s "
        f"(frac {sweep['frac']:.3f})")
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
                   "obs_every": wl.obs_every, "parallelism": "single GPU",
                   "tile_rows": tile_rows, "sweep_variant": variant, "taylor_fusion": fusion,
                   "kernel_shape": shape, "graphs": bool(args.graphs)},
        "steps_per_s": steps_per_s,
        "roofline": {
            "bound": "hbm",
            "kernel": kernel,
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
            "traffic": traffic,
            "valu_busy_pct": valu,
            "algorithmic_bytes_per_launch": bytes_per_launch,
            "mean_launch_us": avg_ms * 1e3,
            "launches_timed": launches,
        },
        "hpsi_sweep": sweep,
        "final_observables": {"norm": float(obs_last[2]), "p_ion": float(obs_last[5]),
                              "p_bound": float(obs_last[4])},
    }

    if not args.no_fp32 and prec == tdse.FP64:
        wl32 = wl.with_(precision="fp32")
        prop = make_prop(tdse, wl32, tdse.FP32, mcode, args.graphs, args.autotune)
        kernel32 = dominant_kernel(prop, wl.method)
        wall32, l32, k32, obs32 = timed(prop, tdse, wl32, torch, args.steps, args.warmup, kernel32, args.graphs)
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
            "kernel": kernel32,
            "kernel_mean_us": 1e3 * k32 / max(l32, 1),
            "kernel_gbs": (taylor_bytes_per_launch(8, U, l32, args.steps) / (k32 / max(l32, 1) * 1e-3) / 1e9)
                          if wl.method == "taylor" else None,
            "rel_state_error_vs_fp64": rel_state,
            "norm_drift_vs_fp64": float(abs(o32[2] - obs_last[2])),
            "p_bound_rel_error_vs_fp64": float(abs(o32[4] - obs_last[4]) / abs(obs_last[4])),
            "steps_compared": (3 if args.graphs else 2) * args.steps + args.warmup,
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
