#!/usr/bin/env python3
"""Throughput of the TDSE hot path on one MI355X.

One step (default workload) = one Taylor-8 time step of the 256-member batch:
256 hydrogen grids of uneven size (N in 4000..16000, lmax in 16..64, dr =
0.1, 3-point stencil; 104,476,250 complex unknowns in all, seed 13081856),
each with its own laser pulse (intensity, wavelength, cycles) and its own
stable dt, advanced together: the fields at the step midpoints, eight Horner
terms of H(t).psi per member and the FP64 observables of every member (norm,
p_g, the 15 populations n <= 5, p_ion, dipole, dipole acceleration) after
every step.  `value` is member H.psi applications per second (8 x 256 per
step) with FP64 state storage; the execution shape (sweep tiles; one launch
per Horner term or K terms per fused launch, and the fused kernel) is chosen
by the library's autotuners before the timed region (--autotune 2).

Also reported on the same line:
  roofline      the dominant kernel of the step (the fused K-term strip
                launch): algorithmic bytes per launch ((3L - 1) c U per step of
                L launches, c = 16 B FP64) over its mean duration from HIP
                events on the stream of each launch, against the 8 TB/s HBM
                peak; `traffic` from the committed rocprofv3 counter summary of
                the same kernel and shape (null if there is none, or if the
                kernel source changed since);
  hpsi_sweep    the plain H.psi apply (read psi, write H psi: 2c B per unknown)
                on the batch, same report, at the fastest of the tuned sweep
                shape and a few strip shapes (APPLY_SHAPES);
  precisions    48-bit and FP32 storage (FP64 arithmetic and reductions): steps
                per second, speedup over FP64, and a 1000-step window of every
                member from mid-pulse (a mixed bound / excited / outgoing start)
                against the FP64 run, with pass/fail against the targets (norm
                within 1e-6, p_ion and every P_nl >= 1e-8 within 1e-5 relative);
  fp64_one_launch_per_term
                the plain FP64 GPU path (one launch per Horner term);
  fp64_vs_oracle
                member 0 of the FP64 batch against the FP64 C oracle over the
                steps of the CPU sample (same start, same dt);
  cpu_baseline  the FP64 C oracle on the host cores for a bounded sample of
                member 0 (whole steps), at 1 thread and at all threads, scaled
                to member applies by unknowns, with the CPU model.

--workload selects a single-instance workload instead (see workloads.WORKLOADS).
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
BATCH_NAME = "batch256_taylor8"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default 200 batch, 2000 single)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed steps (default 20 batch, 200 single)")
    ap.add_argument("--window", type=int, default=1000, help="steps of the precision comparison window")
    ap.add_argument("--precisions", default="fp48,fp32", help="storage precisions timed beside FP64")
    ap.add_argument("--workload", default=BATCH_NAME,
                    choices=sorted(workloads.WORKLOADS) + [BATCH_NAME])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true", help="time FP64 only (no other storage precisions)")
    ap.add_argument("--no-plain", action="store_true",
                    help="skip the plain FP64 path (one launch per Horner term) of the batch")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--graphs", type=int, default=1, help="replay step chunks as HIP graphs")
    ap.add_argument("--rk4-stages", action="store_true",
                    help="RK4 in four stage launches per step (default: one launch per step)")
    ap.add_argument("--autotune", type=int, default=2,
                    help="0: fixed shapes; 1: autotune the sweep tiles; 2: also choose the Taylor fusion")
    ap.add_argument("--no-apply-search", action="store_true",
                    help="time the plain H.psi apply on the sweep shape in use only")
    ap.add_argument("--sweep", default=None, metavar="ROWS,VARIANT",
                    help="fixed sweep tile shape instead of the sweep autotuner (profiling runs)")
    ap.add_argument("--fusion", default=None, metavar="K,ROWS,KIND[,OBS]",
                    help="fixed Taylor fusion instead of the Taylor autotuner (profiling runs); OBS 1: the "
                         "main observables summed in the step's last strip launch, 0: by their own pass")
    args = ap.parse_args()
    batch = args.workload == BATCH_NAME
    if args.steps is None:
        args.steps = 200 if batch else 2000
    if args.warmup is None:
        args.warmup = 20 if batch else 200
    return args


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
    for part in (name, "device_common.hpp", "strip_common.hpp", "pstrip_body.hpp", "tdse_internal.hpp"):
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


# tile shapes (rows, sweep variant) the plain apply is also timed on: the
# sweep autotuner times Horner-term sweeps (which also read psi), whose best
# shape need not be the apply's
APPLY_SHAPES = ((2, 6), (4, 6), (4, 4), (8, 6))


def hpsi_sweep(prop, tdse, torch, U, elem, reps=40):
    """Mean duration of the plain H.psi apply on the bound grid (HIP events),
    at the fastest of the tuned sweep shape and APPLY_SHAPES (only the tuned
    one with --no-apply-search); the tuned shape is restored afterwards."""
    out = prop.new_vector()
    e = 0.01
    tuned = (prop.tile_rows, prop.sweep_variant)
    search = ARGS is None or not getattr(ARGS, "no_apply_search", False)
    best = None
    for shape in [tuned] + ([s for s in APPLY_SHAPES if s != tuned] if search else []):
        prop.set_sweep_shape(*shape)
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
        if best is None or us < best[0]:
            best = (us, launches, shape)
    prop.set_sweep_shape(*tuned)
    us, launches, shape = best
    bytes_ = 2 * elem * U
    gbs = bytes_ / (us * 1e-6) / 1e9
    return {"bound": "hbm", "kernel": "apply_h", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": gbs / HBM_PEAK_GBS, "algorithmic_bytes_per_launch": bytes_, "mean_launch_us": us,
            "launches_timed": launches, "applies_per_s": 1e6 / us,
            "shape": {"tile_rows": shape[0], "sweep_variant": shape[1]}}


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


PREC_NAMES = {0: "fp64", 1: "fp32", 2: "fp48"}
ELEM_BYTES = {0: 16, 1: 8, 2: 12}
NORM_TOL, REL_TOL, POP_FLOOR, ABS_BELOW = 1e-6, 1e-5, 1e-8, 1e-13


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


def mixed_states(members):
    """Normalised window starts: bound, excited and outgoing parts at once."""
    out = []
    for k, m in enumerate(members):
        v = workloads.mixed_state(2000 + k, m.n, m.lmax, workloads.BATCH_DR)
        out.append(v / math.sqrt(workloads.BATCH_DR * float(np.vdot(v, v).real)))
    return out


def target_check(lo, hi):
    """Records lo against hi ([member][record][23]): worst norm difference, worst
    relative p_ion / P_nl difference where the reference is >= 1e-8 (below it
    the absolute difference, held to 1e-13), and pass/fail per target."""
    dn = float(np.max(np.abs(lo[..., 2] - hi[..., 2])))
    cols = [5] + list(range(8, 23))
    a, b = lo[..., cols], hi[..., cols]
    big = np.abs(b) >= POP_FLOOR
    rel = float(np.max(np.where(big, np.abs(a - b) / np.where(big, np.abs(b), 1.0), 0.0)))
    small = float(np.max(np.where(big, 0.0, np.abs(a - b))))
    pion = lo[..., 5], hi[..., 5]
    return {"max_norm_diff": dn, "norm_pass": dn <= NORM_TOL,
            "max_rel_diff_pion_pops": rel, "max_abs_diff_below_1e-8": small,
            "pion_pops_pass": rel <= REL_TOL and small <= ABS_BELOW,
            "max_rel_diff_pion": float(np.max(np.abs(pion[0] - pion[1]) / np.maximum(np.abs(pion[1]), 1e-300))),
            "p_ion_range": [float(np.min(pion[1])), float(np.max(pion[1]))]}


def run_batch_prec(tdse, torch, precision, args, autotune=None, window=None, check_steps=0):
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

    def run(n, obs, every=1):
        nonlocal t
        prop.step_taylor(pulses, t, dts, order, n, every, obs)
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
    U = sum((g.lmax + 1) * g.n for g in grids)
    elem = ELEM_BYTES[precision]
    prec_name = PREC_NAMES[precision]
    shape = shape_of(prop, kernel)
    traffic = traffic_for(BATCH_NAME, kernel, prec_name, shape)
    valu = valu_busy_for(BATCH_NAME, kernel, prec_name, shape)
    sweep = hpsi_sweep(prop, tdse, torch, U, elem)
    sweep["traffic"] = traffic_for(BATCH_NAME, "apply_h", prec_name, sweep["shape"])
    sweep["valu_busy_pct"] = valu_busy_for(BATCH_NAME, "apply_h", prec_name, sweep["shape"])
    res = dict(wall=wall, launches=launches, kms=kms, U=U, dts=dts, n=len(grids), kernel=kernel, shape=shape,
               traffic=traffic, valu=valu, sweep=sweep, elem=elem)
    if window:
        # the precision window: every member from a mixed state, mid-pulse
        starts, wsteps = window
        for k in range(len(grids)):
            prop.set_state(k, starts[k])
        t = [0.5 * m.pulse.duration for m in members]
        wobs = prop.obs_buffer(wsteps, 10)
        run(wsteps, wobs, 10)
        res["window_records"] = wobs.cpu().numpy()
    if check_steps:
        # member 0 (all members run) from the 1s state at t = 0, as the CPU sample
        for k in range(len(grids)):
            prop.set_state(k, None)
        t = [0.0] * len(grids)
        cobs = prop.obs_buffer(check_steps, 1)
        run(check_steps, cobs, 1)
        res["check_state0"] = prop.get_state(0)
        res["check_records0"] = cobs.cpu().numpy()[0]
    prop.close()
    del prop
    torch.cuda.empty_cache()
    return res


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def run_batch(args, tdse, torch):
    prec_codes = {"fp48": tdse.FP48, "fp32": tdse.FP32}
    extra = [p for p in args.precisions.split(",") if p] if not args.no_fp32 else []
    log(f"bench: batch of 256 members, Taylor-8, FP64 + {extra}, steps={args.steps} warmup={args.warmup}")
    members = workloads.batch_members()
    m0 = members[0]
    cb = None
    if not args.no_cpu_baseline:
        wl0 = workloads.Workload("batch_member0", m0.n, m0.lmax, workloads.BATCH_DR, workloads.BATCH_STENCIL,
                                 "fp64", "taylor", workloads.BATCH_ORDER, m0.pulse, dt=float("nan"),
                                 dt_nominal=float("nan"), nsteps=0, obs_every=1,
                                 r_ion=workloads.BATCH_R_ION_FRACTION * m0.n * workloads.BATCH_DR)
        cb = cpu_baseline_batch(tdse, wl0, args.cpu_seconds)
    starts = mixed_states(members) if args.window > 0 else None
    window = (starts, args.window) if starts is not None else None
    r64 = run_batch_prec(tdse, torch, tdse.FP64, args, window=window,
                         check_steps=cb["check_steps"] if cb else 0)
    sps = args.steps / r64["wall"]
    log(f"bench: batch FP64 {sps:.1f} steps/s, {r64['kernel']} mean {1e3 * r64['kms'] / max(r64['launches'], 1):.1f} us")
    others = {}
    for name in extra:
        r = run_batch_prec(tdse, torch, prec_codes[name], args, window=window)
        others[name] = r
        log(f"bench: batch {name.upper()} {args.steps / r['wall']:.1f} steps/s")
    # the plain FP64 path: one launch per Horner term (sweep tiles tuned, no fusion)
    r64p = None
    if not args.no_plain:
        r64p = run_batch_prec(tdse, torch, tdse.FP64, args, autotune=min(args.autotune, 1))
        log(f"bench: batch FP64 one launch per term {args.steps / r64p['wall']:.1f} steps/s")
    U = r64["U"]
    avg_ms = r64["kms"] / max(r64["launches"], 1)
    bpl = taylor_bytes_per_launch(16, U, r64["launches"], args.steps)
    achieved = bpl / (avg_ms * 1e-3) / 1e9
    out = {
        "metric": METRIC, "value": workloads.BATCH_ORDER * r64["n"] * sps, "unit": "H·ψ applies/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * r64["wall"] / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": BATCH_NAME, "members": r64["n"], "unknowns": U,
                   "seed": workloads.BATCH_SEED, "dr": workloads.BATCH_DR, "stencil": workloads.BATCH_STENCIL,
                   "method": "taylor", "order": workloads.BATCH_ORDER, "obs_every": 1,
                   "dt_range": [min(r64["dts"]), max(r64["dts"])], "parallelism": "single GPU",
                   "kernel_shape": r64["shape"], "graphs": bool(args.graphs)},
        "steps_per_s": sps,
        "unknown_applies_per_s": workloads.BATCH_ORDER * U * sps,
        "roofline": {"bound": "hbm", "kernel": r64["kernel"], "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": r64["traffic"],
                     "valu_busy_pct": r64["valu"],
                     "algorithmic_bytes_per_launch": bpl, "mean_launch_us": avg_ms * 1e3,
                     "launches_timed": r64["launches"]},
        "hpsi_sweep": r64["sweep"],
        "precisions": {},
        "fp64_one_launch_per_term": None if r64p is None else {
            "steps_per_s": args.steps / r64p["wall"], "fused_speedup_vs_it": sps / (args.steps / r64p["wall"]),
            "kernel": r64p["kernel"], "kernel_mean_us": 1e3 * r64p["kms"] / max(r64p["launches"], 1)},
    }
    for name, r in others.items():
        s_r = args.steps / r["wall"]
        a_ms = r["kms"] / max(r["launches"], 1)
        b = taylor_bytes_per_launch(r["elem"], U, r["launches"], args.steps)
        entry = {"steps_per_s": s_r, "applies_per_s": workloads.BATCH_ORDER * r["n"] * s_r,
                 "speedup_vs_fp64": s_r / sps,
                 "speedup_vs_fp64_one_launch_per_term": (s_r / (args.steps / r64p["wall"])) if r64p else None,
                 "kernel": r["kernel"], "kernel_shape": r["shape"], "kernel_mean_us": a_ms * 1e3,
                 "kernel_gbs": b / (a_ms * 1e-3) / 1e9, "kernel_frac": b / (a_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                 "bytes_per_unknown": r["elem"], "hpsi_sweep_gbs": r["sweep"]["achieved"]}
        if window:
            chk = target_check(r["window_records"], r64["window_records"])
            chk["window"] = (f"{args.window} steps of every member from t = T/2, start: normalised "
                             f"workloads.mixed_state(2000 + k); records every 10 steps")
            entry["vs_fp64"] = chk
        out["precisions"][name] = entry
        log(f"bench: {name}: {entry.get('vs_fp64')}")
    if cb:
        ref_state, ref_rec = cb.pop("ref_state"), cb.pop("ref_records")
        g_state, g_rec = r64["check_state0"], r64["check_records0"]
        k = ref_rec.shape[1]
        out["fp64_vs_oracle"] = {
            "member": 0, "steps": cb["check_steps"],
            "rel_state_error": float(np.linalg.norm(g_state - ref_state) / np.linalg.norm(ref_state)),
            "max_record_diff": float(np.max(np.abs(g_rec[:, :k] - ref_rec)))}
        cb.pop("check_steps")
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


def cpu_baseline_batch(tdse, wl, seconds):
    """The oracle on member 0 of the batch, from its 1s state at t = 0 with the
    member's dt: timed at 1 thread and at all threads of the host (the results
    are bit-identical), scaled to member applies of the batch's mean size."""
    import oracle
    members = workloads.batch_members()
    U_mean = sum((m.lmax + 1) * m.n for m in members) / len(members)
    g = oracle.Grid(n=wl.n, lmax=wl.lmax, dr=wl.dr, stencil=wl.stencil, z=wl.z)
    p = oracle.Pulse(wl.pulse.e0, wl.pulse.omega, wl.pulse.n_cycles, wl.pulse.cep, wl.pulse.t_on)
    setup = oracle.obs_setup(g, r_ion=wl.r_ion)
    psi0, _ = oracle.initial_state(g)
    dt = workloads.BATCH_DT_SAFETY * tdse.tdse_taylor_stability_limit(wl.order) / oracle.h_bound(g, abs(wl.pulse.e0))
    U0 = (wl.lmax + 1) * wl.n
    res = {}
    nthreads = oracle.max_threads()
    for th in (1, nthreads):
        oracle.set_threads(th)
        t0 = time.perf_counter()
        oracle.propagate(g, p, oracle.TAYLOR, wl.order, 0.0, dt, 2, 1, setup, psi0)
        one = (time.perf_counter() - t0) / 2
        n = max(4, int(0.5 * seconds / max(one, 1e-6)))
        t0 = time.perf_counter()
        psi, obs, _ = oracle.propagate(g, p, oracle.TAYLOR, wl.order, 0.0, dt, n, 1, setup, psi0)
        el = time.perf_counter() - t0
        res[th] = dict(steps=n, seconds=el, steps_per_s=n / el, state=psi, records=obs)
        log(f"bench: cpu oracle member 0, {th} thread(s): {n} steps in {el:.1f} s")
    oracle.set_threads(nthreads)
    top = res[nthreads]
    scale = wl.order * U0 / U_mean
    return {"value": scale * top["steps_per_s"], "unit": "H·ψ applies/s", "cores": nthreads, "kind": "oracle",
            "sample": (f"{top['steps']} whole Taylor-8 steps (with per-step observables) of batch member 0 "
                       f"(N={wl.n}, lmax={wl.lmax}, {U0} unknowns) from its 1s state, FP64 C oracle, "
                       f"{nthreads} threads, {top['seconds']:.1f} s; member applies scaled to the batch mean "
                       f"of {U_mean:.0f} unknowns"),
            "cpu_model": cpu_model(), "threads": nthreads,
            "unknown_applies_per_s": wl.order * U0 * top["steps_per_s"],
            "one_thread": {"value": scale * res[1]["steps_per_s"], "steps": res[1]["steps"],
                           "seconds": res[1]["seconds"], "unknown_applies_per_s": wl.order * U0 * res[1]["steps_per_s"]},
            "check_steps": top["steps"], "ref_state": top["state"], "ref_records": top["records"]}


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
    prec = {"fp64": tdse.FP64, "fp32": tdse.FP32, "fp48": tdse.FP48}[wl.precision]
    mcode = {"taylor": tdse.METHOD_TAYLOR, "rk4": tdse.METHOD_RK4,
             "lanczos": tdse.METHOD_LANCZOS}[wl.method]
    applies_per_step = {"taylor": wl.order, "rk4": 4, "lanczos": wl.order}[wl.method]
    U = wl.unknowns
    elem = {tdse.FP64: 16, tdse.FP32: 8, tdse.FP48: 12}[prec]
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
    prec_name = PREC_NAMES[prec]
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
        "dtype": {0: "f64", 1: "f32-storage/f64-arith", 2: "f48-storage/f64-arith"}[prec],
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

    extra = [p for p in args.precisions.split(",") if p] if not args.no_fp32 and prec == tdse.FP64 else []
    out["precisions"] = {}
    for name in extra:
        code = {"fp48": tdse.FP48, "fp32": tdse.FP32}[name]
        wlx = wl.with_(precision=name)
        prop = make_prop(tdse, wlx, code, mcode, args.graphs, args.autotune)
        kx = dominant_kernel(prop, wl.method)
        wallx, lx, kmx, obsx = timed(prop, tdse, wlx, torch, args.steps, args.warmup, kx, args.graphs)
        psix = prop.get_state(0)
        ox = obsx.cpu().numpy()[0, -1]
        prop.close()
        del prop
        torch.cuda.empty_cache()
        spsx = args.steps / wallx
        rel_state = float(np.linalg.norm(psix - psi_main) / np.linalg.norm(psi_main))
        ex = ELEM_BYTES[code]
        out["precisions"][name] = {
            "steps_per_s": spsx,
            "applies_per_s": applies_per_step * spsx,
            "speedup_vs_fp64": spsx / steps_per_s,
            "kernel": kx,
            "kernel_mean_us": 1e3 * kmx / max(lx, 1),
            "kernel_gbs": (taylor_bytes_per_launch(ex, U, lx, args.steps) / (kmx / max(lx, 1) * 1e-3) / 1e9)
                          if wl.method == "taylor" else None,
            "rel_state_error_vs_fp64": rel_state,
            "norm_diff_vs_fp64": float(abs(ox[2] - obs_last[2])),
            "p_bound_rel_diff_vs_fp64": float(abs(ox[4] - obs_last[4]) / abs(obs_last[4])),
            "steps_compared": (3 if args.graphs else 2) * args.steps + args.warmup,
        }
        log(f"bench: {name} {spsx:.1f} steps/s ({spsx / steps_per_s:.2f}x), state diff {rel_state:.2e}")

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds, applies_per_step)

    print(json.dumps(out), flush=True)


def cpu_baseline(wl, seconds, applies_per_step):
    """The oracle on the same workload (whole steps from the same start), at
    1 thread and at all threads of the host (bit-identical results)."""
    import oracle
    g = oracle.Grid(n=wl.n, lmax=wl.lmax, dr=wl.dr, stencil=wl.stencil, z=wl.z)
    p = oracle.Pulse(wl.pulse.e0, wl.pulse.omega, wl.pulse.n_cycles, wl.pulse.cep, wl.pulse.t_on)
    setup = oracle.obs_setup(g, r_ion=wl.r_ion)
    psi, _ = oracle.initial_state(g)
    code = {"taylor": oracle.TAYLOR, "rk4": oracle.RK4, "lanczos": oracle.LANCZOS}[wl.method]
    nthreads = oracle.max_threads()
    res = {}
    for th in (1, nthreads):
        oracle.set_threads(th)
        t0 = time.perf_counter()
        oracle.propagate(g, p, code, wl.order, wl.t0, wl.dt, 1, 1, setup, psi)
        one = time.perf_counter() - t0
        n = max(1, int(0.5 * seconds / max(one, 1e-6)))
        t0 = time.perf_counter()
        oracle.propagate(g, p, code, wl.order, wl.t0, wl.dt, n, 1, setup, psi)
        el = time.perf_counter() - t0
        res[th] = (n, el)
        log(f"bench: cpu oracle {th} thread(s): {n} steps in {el:.1f} s")
    oracle.set_threads(nthreads)
    n, el = res[nthreads]
    n1, el1 = res[1]
    return {"value": applies_per_step * n / el, "unit": "H·ψ applies/s", "cores": nthreads,
            "kind": "oracle",
            "sample": f"{n} whole {wl.method}-{wl.order} steps (with per-step observables) of the "
                      f"same workload, FP64 C oracle, {nthreads} threads, {el:.1f} s",
            "cpu_model": cpu_model(), "steps_per_s": n / el,
            "one_thread": {"value": applies_per_step * n1 / el1, "steps": n1, "seconds": el1}}


if __name__ == "__main__":
    main()
