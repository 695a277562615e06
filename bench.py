#!/usr/bin/env python3
"""Throughput of the ERPP particle/fluid coupling step on one MI355X.

Default workload: the shear-flow-shaped box (256 x 128 x 128 nodes,
4pi x 2pi x 2pi, 4e5 particles, 70% in 2000 Gaussian blobs, mean shear S = 1
plus a k^-5/3 fluctuation, three Stokes-time populations, sigma = 1.5 dx, M = 8,
dt = 2e-4), run in the FP32 tiled path (FP64 particle integration) as a
captured HIP graph per step.  Inputs are seeded synthetic arrays already
resident in HBM when the timed region starts.

Prints ONE JSON line: particle-steps/s over the timed steps, the roofline of the
dominant kernel (HIP-event durations of each stage, measured in this run), the
plain FP64 GPU path on the same inputs, the accuracy against the FP64 oracle on a
particle sample and a node window, and the oracle itself timed on the host.
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-steps/s and %HBM peak, FP32 batched vs FP64 plain, at ≤1e-5 rel L2"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
LDS_PEAK_TOPS = 256 * 32 * 2.4e9 / 1e12     # 256 CUs x 32 banks x 2.4 GHz (dword ops)
STAGES_FAST = ["bin_count", "scan", "eval", "scatter", "update"]
# kernels of each stage (rocprofv3 names without template arguments)
STAGE_KERNELS = {"bin_count": ["k_bin_count"], "scan": ["k_scan_reduce", "k_scan_down"],
                 "eval": ["k_eval"], "scatter": ["k_block_sums", "k_pencil_scale", "k_scatter"],
                 "update": ["k_gather_sorted", "k_update"]}
WORKLOADS = {"c1": 1, "c2": 2, "c3": 3, "c3cube": 33, "c4": 4, "c5": 5}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=16)
    ap.add_argument("--workload", default="c3", choices=sorted(WORKLOADS))
    ap.add_argument("--tile", default=None,
                    help="scatter shape THREADS,T1,T2 (skips the autotuner)")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--stage-steps", type=int, default=10)
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the particle-force variants (integrators, Faxen, added mass)")
    ap.add_argument("--no-target", action="store_true",
                    help="skip the 256^3 target of the shear workload (c3cube)")
    ap.add_argument("--no-coupled", action="store_true",
                    help="skip the two-way coupled run (coupling step + fluid step)")
    ap.add_argument("--rows-per-item", type=int, default=0, metavar="R",
                    help="stencil rows per work item of the scatter (2..4; default: the "
                         "autotuner's choice, or 3 with --tile / --no-tune)")
    ap.add_argument("--no-stream-copy", action="store_true",
                    help="skip the device-copy bandwidth measurement")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="also run one plain device copy of MIB MiB (the reference kernel "
                         "for scaling HBM counter readings)")
    return ap.parse_args()


def byte_model(boxes, M):
    """Algorithmic bytes per step and per kernel launch (FP32 path)."""
    np_tot = sum(b.np_ for b in boxes)
    ng_tot = sum(int(np.prod(b.n)) for b in boxes)
    touched = sum(min(int(np.prod(b.n)), 8 * b.np_) for b in boxes)
    nbins = None
    step = 224 * np_tot + 12 * ng_tot + 12 * touched
    per_kernel = {
        # delayed position read, rank write, histogram atomic
        "bin_count": 32 * np_tot,
        # delayed position + drag, rank, bin start read; 32-byte record written
        "eval": (24 + 12 + 4 + 4 + 32) * np_tot,
        # records read once, forcing written once (12 B per node)
        "scatter": 32 * np_tot + 12 * ng_tot,
        # x, v, tau, level n-1-M (x, D) read; x, v, ring slot written; carrier
        "update": (24 + 24 + 4 + 36 + 24 + 24 + 36) * np_tot + 12 * touched,
    }
    return step, per_kernel, nbins


def scatter_flops(boxes, stencil_nodes):
    # 7 flops per stencil node: w = gx * gyz (1), three multiply-adds (6)
    return sum(7.0 * stencil_nodes(b) * b.np_ for b in boxes)


def stencil_nodes_of(box):
    s = box.spec.sigma_dx * box.spec.cutoff
    # mean lattice count of the ball of radius s (in grid units)
    return 4.0 / 3.0 * math.pi * s ** 3


def kernel_source_hash():
    """Hash of the fast path's kernel sources with // comments, indentation and
    blank lines dropped: a change of code, not of its comments or layout,
    invalidates the recorded counter summary."""
    h = hashlib.sha256()
    for name in ("fast.hip", "erpp_device.hpp", "erpp_internal.hpp"):
        with open(os.path.join(ROOT, "paper_1405_6969_amd", "csrc", name)) as fh:
            for line in fh:
                code = line.split("//", 1)[0].strip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def traffic_from_profiles(stage, workload):
    """HBM bytes per launch of a stage's kernels (stage None: of the whole step)
    from a committed rocprofv3 counter summary (profiles/traffic*.json) taken on
    the current kernel source and on this workload; else None."""
    data = None
    sha = kernel_source_hash()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "traffic*.json"))):
        try:
            d = json.load(open(path))
        except Exception:
            continue
        if d.get("kernel_sha") == sha and d.get("workload") == workload:
            data = d
            break
    if data is None:
        return None
    total, found = 0.0, False
    for name, ent in data.get("kernels", {}).items():
        if stage is None or name.split("<")[0] in STAGE_KERNELS[stage]:
            total += ent.get("bytes_per_launch", 0.0)
            found = True
    return round(total) if found else None


def measure_fast(boxes, w, K, W, args, erpp, torch, tile=None, stage_steps=10):
    """The FP32 path on one workload: M + 1 eager steps fill the delay ring (every
    later step deposits a live forcing), the autotuner picks the pencil (or the
    given tile is set), W warm-up steps (graph capture and replays), then K
    timed graph replays bracketed by HIP events on the plan's stream.  Then the
    per-stage durations of stage_steps more steps (HIP events around each
    stage).  Returns the measurements, the plan and its device boxes."""
    M, dt = w.M, w.dt
    dbs = upload_boxes(boxes, M, erpp.F32_FAST, erpp)
    plan = erpp.Plan(dbs, M, dt, precision=erpp.F32_FAST)
    prefill = M + 1
    plan.run(0, prefill, graph=False)
    torch.cuda.synchronize()
    if tile is not None:
        plan.set_tile(tuple(tile))
    elif args.tile:
        plan.set_tile(tuple(int(a) for a in args.tile.split(",")))
    elif not args.no_tune:
        plan.tune(None)
    if getattr(args, "rows_per_item", 0):
        plan.set_rows_per_item(args.rows_per_item)
    tile = plan.get_tile()
    steps_done = prefill
    plan.run(steps_done, W, graph=True)          # capture, then W replays (untimed)
    steps_done += W
    torch.cuda.synchronize()
    log(f"[bench] {w.name}: {prefill} ring-filling steps, {W} warm-up steps, tile {tile}")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    plan.run(steps_done, K, graph=True)
    e1.record()
    torch.cuda.synchronize()
    steps_done += K
    ms_step = e0.elapsed_time(e1) / K
    np_tot = sum(b.np_ for b in boxes)
    value = np_tot / (ms_step * 1e-3)
    log(f"[bench] {w.name}: timed {K} steps: {ms_step * 1e3:.1f} us/step, "
        f"{value:.3e} particle-steps/s")
    stage_ms = plan.stage_times(steps_done, stage_steps)
    steps_done += stage_steps
    torch.cuda.synchronize()
    log(f"[bench] {w.name}: stage us: " +
        ", ".join(f"{n}={t * 1e3:.1f}" for n, t in zip(STAGES_FAST, stage_ms)))
    step_bytes, kbytes, _ = byte_model(boxes, M)
    dom = int(np.argmax(stage_ms))
    dom_name = STAGES_FAST[dom]
    dom_bytes = kbytes.get(dom_name, 0)
    achieved = dom_bytes / (stage_ms[dom] * 1e-3) / 1e9
    roof = {"kernel": "+".join(STAGE_KERNELS[dom_name]), "bound": "hbm",
            "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic_from_profiles(dom_name, w.name),
            "algorithmic_bytes_per_launch": dom_bytes,
            "avg_launch_us": round(stage_ms[dom] * 1e3, 2)}
    if dom_name == "scatter":
        fl = scatter_flops(boxes, stencil_nodes_of)
        lds_ops = 3.0 * sum(stencil_nodes_of(b) * b.np_ for b in boxes)
        roof["secondary"] = {
            "fp32_tflops": round(fl / (stage_ms[dom] * 1e-3) / 1e12, 2),
            "fp32_peak_tflops": FP32_PEAK_TFLOPS,
            "lds_atomic_tops": round(lds_ops / (stage_ms[dom] * 1e-3) / 1e12, 3),
            "lds_peak_tops": round(LDS_PEAK_TOPS, 2)}
    step_gbs = step_bytes / (ms_step * 1e-3) / 1e9
    # the same step's HBM bytes as the counters measured them (FETCH_SIZE +
    # WRITE_SIZE of every kernel, profiles/traffic.json), when they apply
    counted = traffic_from_profiles(None, w.name)
    counted_frac = (round(counted / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
                    if counted else None)
    res = {"value": value, "ms_per_step": ms_step, "tile": list(tile),
           "rows_per_item": plan.get_rows_per_item(), "prefill": prefill,
           "warmup": W, "steps": K, "steps_done": steps_done,
           "hbm_frac_step": round(step_gbs / HBM_PEAK_GBS, 4),
           "hbm_frac_step_counted": counted_frac,
           "algorithmic_bytes_per_step": step_bytes,
           "stage_us": {n: round(t * 1e3, 2) for n, t in zip(STAGES_FAST, stage_ms)},
           "roofline": roof}
    return res, plan, dbs


def measure_plain(boxes, w, ms_fast, erpp, torch, nrep=10):
    """The plain FP64 path on the same inputs: M + 1 eager steps, one graph
    capture and replay (untimed), then nrep timed replays."""
    M, dt = w.M, w.dt
    np_tot = sum(b.np_ for b in boxes)
    pdb = upload_boxes(boxes, M, erpp.F64_PLAIN, erpp)
    pplan = erpp.Plan(pdb, M, dt, precision=erpp.F64_PLAIN)
    pplan.run(0, M + 1, graph=False)
    pplan.run(M + 1, 1, graph=True)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    pplan.run(M + 2, nrep, graph=True)
    b.record()
    torch.cuda.synchronize()
    pms = a.elapsed_time(b) / nrep
    pplan.close()
    del pdb
    torch.cuda.empty_cache()
    log(f"[bench] {w.name}: FP64 plain {pms * 1e3:.1f} us/step (x{pms / ms_fast:.1f})")
    return {"ms_per_step": round(pms, 4), "value": round(np_tot / (pms * 1e-3), 1),
            "steps": nrep, "speedup_fp32_vs_fp64_plain": round(pms / ms_fast, 2)}


def upload_boxes(boxes, M, prec, erpp):
    out = []
    for b in boxes:
        u = b.u.astype(np.float32) if prec == erpp.F32_FAST else b.u
        s = b.spec
        out.append(erpp.device_box(b.n, b.L, b.x, b.v, b.tau, u, M, b.m_p, s.rho_f, s.nu,
                                   b.sigma, s.cutoff, s.shear, precision=prec))
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); multi-GPU "
              f"sharding is described in DESIGN.md and not built.", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads
    import paper_1405_6969_amd as erpp

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    t0 = time.time()
    w = workloads.config(WORKLOADS[args.workload])
    boxes = workloads.make_boxes(w)
    log(f"[bench] workload {w.name}: {len(boxes)} box(es), "
        f"{sum(b.np_ for b in boxes)} particles, inputs in {time.time() - t0:.1f}s")
    M, dt = w.M, w.dt
    W, K = max(args.warmup, 1), args.steps
    np_tot = sum(b.np_ for b in boxes)

    # ------------------------------------------------------- FP32 tiled path
    res, plan, dbs = measure_fast(boxes, w, K, W, args, erpp, torch,
                                  stage_steps=args.stage_steps)
    ms_step, value, tile = res["ms_per_step"], res["value"], res["tile"]

    # ------------------------------------------------------- FP64 plain path
    plain = None
    if not args.no_plain:
        plain = measure_plain(boxes, w, ms_step, erpp, torch)

    # ------------------------------------------------------- accuracy vs oracle
    accuracy = None
    if not args.no_check and len(boxes) == 1:
        accuracy = check_accuracy(boxes[0], dbs[0], w, res["steps_done"])
        log(f"[bench] accuracy {accuracy}")
    plan.close()
    del dbs
    torch.cuda.empty_cache()

    # ------------------------------------------- the 256^3 target of the same mix
    target = None
    if args.workload == "c3" and not args.no_target:
        wt = workloads.config(WORKLOADS["c3cube"])
        tboxes = workloads.make_boxes(wt)
        Kt = min(K, 100)
        tres, tplan, tdbs = measure_fast(tboxes, wt, Kt, W, args, erpp, torch,
                                         stage_steps=args.stage_steps)
        tacc = None
        if not args.no_check:
            tacc = check_accuracy(tboxes[0], tdbs[0], wt, tres["steps_done"])
            log(f"[bench] {wt.name}: accuracy {tacc}")
        tplan.close()
        del tdbs
        torch.cuda.empty_cache()
        tplain = None if args.no_plain else measure_plain(tboxes, wt, tres["ms_per_step"],
                                                          erpp, torch)
        target = {"workload": wt.name, "grid": list(tboxes[0].n),
                  "particles": sum(b.np_ for b in tboxes),
                  "value": round(tres["value"], 1), "unit": "particle-steps/s",
                  "ms_per_step": round(tres["ms_per_step"], 6), "steps": Kt,
                  "warmup": W, "prefill_steps": tres["prefill"], "tile": tres["tile"],
                  "rows_per_item": tres["rows_per_item"],
                  "hbm_frac_step": tres["hbm_frac_step"],
                  "hbm_frac_step_counted": tres["hbm_frac_step_counted"],
                  "algorithmic_bytes_per_step": tres["algorithmic_bytes_per_step"],
                  "stage_us": tres["stage_us"], "roofline": tres["roofline"],
                  "fp64_plain": tplain, "accuracy": tacc}
        del tboxes

    # ------------------------------------------------------- oracle on the host
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(boxes[0], w)
        log(f"[bench] oracle {cpu}")

    coupled = None
    if not args.no_coupled and len(boxes) == 1:
        coupled = bench_coupled(boxes[0], w, tile, min(K, 100), erpp, torch)
        log(f"[bench] coupled {coupled}")
    variants = None
    if not args.no_variants and len(boxes) == 1:
        torch.cuda.empty_cache()
        variants = bench_variants(boxes[0], w, tile, min(K, 100), erpp, torch)
        log(f"[bench] variants {variants}")
    copy_bw = None if args.no_stream_copy else stream_copy(torch)
    if copy_bw:
        log(f"[bench] stream copy {copy_bw}")
    if args.copy_calibration > 0:
        nel = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(nel, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copy calibration: {args.copy_calibration} MiB read + written")
        del src, dst
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "particle-steps/s", "n_gpus": 1,
        "steps": K, "warmup": W, "ms_per_step": round(ms_step, 6), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded; no dataset)",
        "config": {"workload": w.name, "boxes": len(boxes),
                   "grid": list(boxes[0].n) if len(boxes) == 1 else "ensemble",
                   "particles": np_tot, "M": M, "dt": dt, "sigma_dx": boxes[0].spec.sigma_dx,
                   "tile": list(tile), "rows_per_item": res["rows_per_item"], "graph": True,
                   "integration": "f64",
                   "prefill_steps": res["prefill"]},
        "hbm_frac_step": res["hbm_frac_step"],
        "hbm_frac_step_counted": res["hbm_frac_step_counted"],
        "algorithmic_bytes_per_step": res["algorithmic_bytes_per_step"],
        "stage_us": res["stage_us"],
        "roofline": res["roofline"],
        "fp64_plain": plain,
        "accuracy": accuracy,
        "target": target,
        "cpu_baseline": cpu,
        "coupled": coupled,
        "variants": variants,
        "stream_copy": copy_bw,
    }
    print(json.dumps(out), flush=True)


def stream_copy(torch, mib=512, reps=20):
    """Achievable HBM rate beside the published 8 TB/s: a plain device-to-device copy of
    `mib` MiB (read + written), timed with events on torch's current stream, where the
    copy runs."""
    nel = mib * (1 << 20) // 4
    src = torch.ones(nel, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    b.synchronize()
    ms = a.elapsed_time(b) / reps
    del src, dst
    torch.cuda.empty_cache()
    nbytes = 2 * nel * 4
    return {"mib": mib, "bytes_per_copy": nbytes, "us": round(ms * 1e3, 2),
            "gbs": round(nbytes / (ms * 1e-3) / 1e9, 1),
            "frac_of_peak": round(nbytes / (ms * 1e-3) / 8e12, 4)}


def bench_coupled(box, w, tile, K, erpp, torch):
    """Two-way coupling on the same grid and particles without the mean shear
    (the fluid step is for periodic boxes at rest): each step is the coupling
    step followed by the App. E fluid step (hipFFT), replayed as one graph.
    Also times the fluid step alone; its algorithmic traffic is u and f read
    and u written, 36 B per node in FP32."""
    M, dt, s = w.M, w.dt, box.spec
    v = box.v.copy()
    if s.shear != 0.0:
        v[0] -= s.shear * (box.x[1] - 0.5 * box.L[1])
    db = erpp.device_box(box.n, box.L, box.x, v, box.tau, box.u.astype(np.float32), M, box.m_p,
                         s.rho_f, s.nu, box.sigma, s.cutoff, 0.0, precision=erpp.F32_FAST)
    plan = erpp.Plan([db], M, dt, precision=erpp.F32_FAST)
    plan.set_tile(tile)
    fl = erpp.Fluid(box.n, box.L, s.nu, dt, precision=erpp.F32_FAST)
    warm = M + 4
    plan.run_coupled([fl], 0, warm, graph=True)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    plan.run_coupled([fl], warm, K, graph=True)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / K
    # the fluid step alone, on a copy of the field with the last forcing
    u2 = db.u.clone()
    nf = 20
    a.record()
    for _ in range(nf):
        fl.step(u2, db.f)
    b.record()
    torch.cuda.synchronize()
    fms = a.elapsed_time(b) / nf
    nodes = int(np.prod(box.n))
    fbytes = 36 * nodes
    plan.close()
    fl.close()
    del db, u2
    torch.cuda.empty_cache()
    return {"workload": f"{w.name} without mean shear", "steps": K,
            "ms_per_step": round(ms, 4), "value": round(box.np_ / (ms * 1e-3), 1),
            "unit": "particle-steps/s",
            "fluid_step": {"us": round(fms * 1e3, 1), "grid": list(box.n),
                           "algorithmic_bytes": fbytes,
                           "achieved_gbs": round(fbytes / (fms * 1e-3) / 1e9, 1)}}


def bench_variants(box, w, tile, K, erpp, torch):
    """The particle-force options on the same particles and carrier without the
    mean shear (Heun and the added mass are defined for boxes at rest): the
    coupling step per graph replay and the update stage alone (HIP events), for
    explicit Euler, the exponential integrator, Heun with the self term removed
    at each stage, the Faxen term (a_p = 0.6 dx), the added mass on top of it
    (a = 0.6 dx), the Basset term on top of the Faxen term, and all three
    (the full force).  Units: ms per step, us for the update stage."""
    M, dt, s = w.M, w.dt, box.spec
    v = box.v.copy()
    if s.shear != 0.0:
        v[0] -= s.shear * (box.x[1] - 0.5 * box.L[1])
    a_p = 0.6 * box.dx[0]
    cases = [("euler", None, 0.0, 0.0, 0.0), ("exponential", erpp.EXPONENTIAL, 0.0, 0.0, 0.0),
             ("heun", erpp.HEUN, 0.0, 0.0, 0.0), ("faxen", None, a_p, 0.0, 0.0),
             ("added_mass", None, a_p, a_p, 0.0), ("basset", None, a_p, 0.0, a_p),
             ("full_force", None, a_p, a_p, a_p)]
    out = {"workload": f"{w.name} without mean shear", "steps": K, "a_p": round(a_p, 6)}
    for name, integ, fax, am, bs in cases:
        db = erpp.device_box(box.n, box.L, box.x, v, box.tau, box.u.astype(np.float32), M,
                             box.m_p, s.rho_f, s.nu, box.sigma, s.cutoff, 0.0,
                             precision=erpp.F32_FAST)
        plan = erpp.Plan([db], M, dt, precision=erpp.F32_FAST)
        plan.set_tile(tile)
        if integ is not None:
            plan.set_integrator(integ)
        if fax > 0.0:
            plan.set_faxen(0, fax)
        if am > 0.0:
            plan.set_added_mass(0, am)
        if bs > 0.0:
            plan.set_basset(0, bs)
        warm = M + 4
        plan.run(0, warm, graph=True)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        plan.run(warm, K, graph=True)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / K
        st = plan.stage_times(warm + K, 10)
        out[name] = {"ms_per_step": round(ms, 4), "update_us": round(st[4] * 1e3, 1)}
        plan.close()
        del db
    torch.cuda.empty_cache()
    return out


def check_accuracy(box, db, w, steps_done):
    """Oracle on (a) 4000 random particles for v and (b) the particles that can
    reach a 32^3 node window for f; particles are independent under a frozen
    carrier, so both subsets are exact."""
    import torch
    import oracle

    M, dt = w.M, w.dt
    rng = np.random.default_rng(20250101)
    P = oracle.params_for_box(box, M, dt, 1)
    u = box.u.astype(np.float32).astype(np.float64)
    sample = rng.choice(box.np_, size=min(4000, box.np_), replace=False)
    run = oracle.Run(P, u, box.x[:, sample], box.v[:, sample], box.tau[sample])
    for _ in range(steps_done):
        run.step(want_f=False)
    v_gpu = db.v.cpu().numpy()[:, sample]
    ev = float(np.linalg.norm(v_gpu - run.v) / np.linalg.norm(run.v))
    # window: 32^3 nodes at a seeded offset; particles within 3 sigma + drift
    wn = tuple(min(32, n) for n in box.n)
    lo = tuple(int(rng.integers(0, n)) for n in box.n)
    vmax = float(np.max(np.abs(box.v))) + float(np.max(np.abs(box.u))) \
        + abs(box.spec.shear) * box.L[1]
    margin = box.spec.cutoff * box.sigma + 2.0 * vmax * steps_done * dt + 2 * box.dx[0]
    keep = np.ones(box.np_, bool)
    for d in range(3):
        c = (lo[d] + 0.5 * (wn[d] - 1)) * box.dx[d]
        dd = box.x[d] - c
        dd -= box.L[d] * np.round(dd / box.L[d])
        half = 0.5 * (wn[d] - 1) * box.dx[d] + margin
        keep &= np.abs(dd) <= half
    idx = np.nonzero(keep)[0]
    run2 = oracle.Run(P, u, box.x[:, idx], box.v[:, idx], box.tau[idx])
    for n in range(steps_done - 1):
        run2.step(want_f=False)
    fo, _ = run2.step(want_f=True, lo=lo, wn=wn)
    fg = db.f.double().cpu().numpy()
    iz = (np.arange(wn[2]) + lo[2]) % box.n[2]
    iy = (np.arange(wn[1]) + lo[1]) % box.n[1]
    ix = (np.arange(wn[0]) + lo[0]) % box.n[0]
    fw = fg[:, iz][:, :, iy][:, :, :, ix]
    nrm = np.linalg.norm(fo)
    ef = float(np.linalg.norm(fw - fo) / nrm) if nrm > 0 else None
    return {"rel_l2_v_sample": ev, "v_sample": int(sample.size), "rel_l2_f_window": ef,
            "f_window": {"lo": list(lo), "n": list(wn), "particles": int(idx.size)},
            "steps": steps_done}


def host_cpu():
    """CPU model, logical CPUs of the machine and CPUs this process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return model, os.cpu_count(), usable


def cpu_baseline(box, w, steps1=2, steps_all=6, max_threads=16):
    """The oracle as it stands, timed on the host: full steps with the delayed
    forcing live, after the M steps that fill its history.

    One thread: oracle.Run.step on the whole box.  All usable cores (at most
    max_threads, the host share of one GPU): the same step split into pieces the
    oracle computes independently -- the particle update of disjoint particle
    subsets (one oracle.Run per subset; particles do not interact under the
    frozen carrier) and the forcing of disjoint z-slab windows of the grid
    (oracle.deposit of the whole delayed level on each window) -- run by Python
    threads, which execute the oracle's C calls concurrently (ctypes releases
    the interpreter lock).  The pieces together equal the one-thread step."""
    import threading
    import oracle
    M, dt = w.M, w.dt
    P = oracle.params_for_box(box, M, dt, 1)
    u = box.u.astype(np.float32).astype(np.float64)
    model, ncpu, usable = host_cpu()
    nth = max(1, min(usable or 1, max_threads, int(os.environ.get("OMP_NUM_THREADS", "64"))))

    # one thread
    run = oracle.Run(P, u, box.x, box.v, box.tau)
    for _ in range(M):
        run.step(want_f=False)
    t = time.perf_counter()
    for _ in range(steps1):
        run.step(want_f=True)
    t1 = time.perf_counter() - t
    del run

    # all usable cores
    parts = np.array_split(np.arange(box.np_), nth)
    runs = [oracle.Run(P, u, box.x[:, idx], box.v[:, idx], box.tau[idx]) for idx in parts]
    nz = box.n[2]
    zcut = np.linspace(0, nz, nth + 1).astype(int)
    wins = [((0, 0, int(zcut[k])), (box.n[0], box.n[1], int(zcut[k + 1] - zcut[k])))
            for k in range(nth) if zcut[k + 1] > zcut[k]]

    def parallel(fn, items):
        th = [threading.Thread(target=fn, args=(it,)) for it in items]
        for x in th:
            x.start()
        for x in th:
            x.join()

    def advance(r):
        r.step(want_f=False)

    for _ in range(M):
        parallel(advance, runs)
    t = time.perf_counter()
    for _ in range(steps_all):
        n = runs[0].n
        slot = (n - M) % (M + 1)
        X = np.concatenate([r.ring_x[slot] for r in runs], axis=1)
        D = np.concatenate([r.ring_d[slot] for r in runs], axis=1)

        def deposit(win):
            oracle.deposit(P, X, D, lo=win[0], wn=win[1])

        parallel(deposit, wins)
        parallel(advance, runs)
    tall = time.perf_counter() - t
    return {"value": round(steps_all * box.np_ / tall, 1), "unit": "particle-steps/s",
            "cores": nth, "kind": "oracle", "seconds": round(tall, 2),
            "one_thread": {"value": round(steps1 * box.np_ / t1, 1), "seconds": round(t1, 2),
                           "steps": steps1},
            "cpu_model": model, "os_cpu_count": ncpu, "usable_cpus": usable,
            "sample": f"{steps_all} full steps (steps {M}..{M + steps_all - 1}, forcing live) "
                      f"of {w.name}: {box.np_} particles, {int(np.prod(box.n))} nodes; "
                      f"{nth} threads: particle updates over {nth} particle subsets, forcing "
                      f"over {len(wins)} z-slab windows (the one-thread figure: {steps1} steps "
                      f"of the unsplit oracle step)"}


if __name__ == "__main__":
    main()
