#!/usr/bin/env python3
"""Throughput of the Vlasov translation step on one MI355X.

Workload (default): the HBM-filling partition.  128 x 128 x 64 periodic
spatial cells of the blob mixture: cold solar-wind Maxwellians (about 80
velocity blocks each) beside hot bi-Maxwellian-plus-beam cells (about 4,400
blocks each) in a seeded blob pattern, hot fraction 0.0993 for a mean of about
500 blocks per cell; 100^3 velocity cells in 4^3 blocks; f stored in BF16,
reconstructed in FP32, with the Courant number, flux integral, update,
rounding carry, mass ledger and moments in FP64.  A step is the whole path:
coalesced ghost update, x, y and z shears (block growth, work list, PPM
remap), end-of-step pruning and the FP64 velocity moments.

Prints one JSON line.  `value` is useful phase-space cell updates per second
(3 x local phase-space cells per step, inputs resident in HBM), `roofline`
describes the shear kernel (the dominant one), `cpu_baseline` the FP64 CPU
oracle on a sub-box of the same workload.  The same line carries
`fp32_reference` (the mixture at half the z extent in FP32) and
`fp32_vs_fp64` (the uneven mixture, 40 % hot, at 96 x 96 x 12 in FP32 and in
plain FP64, and the FP32 step's speedup).

--workload maxwellian selects the smooth sparse-Maxwellian partition
(64 x 64 x 32, one Maxwellian per cell) instead.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "phase-space cell updates/s per x/y/z translation step (FP32 vs FP64) + HBM GB/s"
STORAGES = {"f64": 0, "f32": 1, "bf16": 2}
BYTES = {"f64": 8, "f32": 4, "bf16": 2}
HOT_500 = 0.0993   # hot fraction of the blob mixture for a mean of ~500 blocks per cell


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("k_sweep.hip", "vl_storage.h", "vl_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_2504_21450_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def variant_key(v):
    """'a,b,c': the shear variants of the first, second and third shear."""
    return ",".join(str(int(x)) for x in (v if isinstance(v, (tuple, list)) else (v, v, v)))


def parse_variant(s):
    v = [int(x) for x in s.split(",")]
    if len(v) == 1:
        return v[0]
    if len(v) != 3:
        raise argparse.ArgumentTypeError("one variant or three (first,second,third shear)")
    return tuple(v)


def measured_traffic(storage, variant, workload):
    """HBM bytes per shear launch from the committed rocprofv3 counter runs of
    the same command, if they were taken on the current kernel source: the
    counters give, for each variant profiled, the bytes of the first, second
    and third shear launch of a step; a step that runs variants (a, b, c)
    moves the mean of a's first, b's second and c's third.  None if the
    counters are stale or a variant was not profiled."""
    path = os.path.join(ROOT, "profiles", "shear_traffic_%s.json" % storage)
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("kernel_source_hash") != kernel_source_hash() or d.get("workload") != workload:
        return None
    by = d.get("hbm_bytes_per_launch_by_shear", {})
    vs = [int(x) for x in variant_key(variant).split(",")]
    if not all(str(v) in by for v in vs):
        return None
    return sum(by[str(v)][s] for s, v in enumerate(vs)) / 3.0


def representative_subbox(w, size, stride=4):
    """Origin of a size-box of the workload whose hot-cell fraction is nearest
    the whole box's (the smooth workload: its centre)."""
    import numpy as np

    hot = (w.fields or {}).get("hot")
    if hot is None:
        return tuple((w.n[d] - size[d]) // 2 for d in range(3))
    h = hot.reshape(w.n[2], w.n[1], w.n[0]).astype(np.float64)
    target = h.mean()
    best, best_lo = None, (0, 0, 0)
    for z in range(0, w.n[2], stride):
        for y in range(0, w.n[1], stride):
            for x in range(0, w.n[0], stride):
                sub = np.take(np.take(np.take(h, np.arange(z, z + size[2]) % w.n[2], 0),
                                      np.arange(y, y + size[1]) % w.n[1], 1),
                              np.arange(x, x + size[0]) % w.n[0], 2)
                d = abs(sub.mean() - target)
                if best is None or d < best:
                    best, best_lo = d, (x, y, z)
    return best_lo


def host_cpu():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return model, avail


def cpu_baseline(w, sample, min_seconds=10.0, max_steps=20):
    """Time the FP64 oracle on a sub-box of the workload (explicit ghost
    domain from the full box for the first step, then periodic)."""
    import numpy as np

    import oracle
    from paper_2504_21450_amd import workloads as W

    size = tuple(int(v) for v in sample.split("x"))
    lo = representative_subbox(w, size)
    cells = W.subbox_cells(w.n, lo, size, 3)
    model, avail = host_cpu()
    threads = int(os.environ.get("OMP_NUM_THREADS", avail))
    if w.f is not None:
        off, ids, f = W.take_cells(w.offsets, w.ids, w.f, cells)
    else:  # device-sampled workload: the host sampler gives the oracle its input
        off, ids, f = W.sample_cells(W.table_model(w.fields["params"]), w.nblk, w.vmin, w.dv,
                                     w.sparse_min, w.vbuffer, w.seed, cells,
                                     threads=min(16, threads), batch=4)
    o = oracle.OraclePartition(size, w.nblk, w.dx, w.vmin, w.dv, w.order, w.sparse_min, w.vbuffer)
    o.load_padded(off, ids, f)
    oracle.lib().vlo_mark_ghosts_valid(o._h)
    local_ps = 0
    P = tuple(s + 6 for s in size)
    for z in range(3, 3 + size[2]):
        for y in range(3, 3 + size[1]):
            for x in range(3, 3 + size[0]):
                q = x + P[0] * (y + P[1] * z)
                local_ps += int(off[q + 1] - off[q]) * 64
    blocks0 = local_ps // 64
    t_steps, nsteps, useful = 0.0, 0, 0
    while nsteps < max_steps and (t_steps < min_seconds or nsteps == 0):
        if nsteps > 0:
            o.fill_ghosts()
        t0 = time.perf_counter()
        s = o.step(w.dt)
        t_steps += time.perf_counter() - t0
        useful += 3 * local_ps
        local_ps = s["blocks"] * 64
        nsteps += 1
    return {"value": useful / t_steps, "unit": "phase-space cell updates/s", "cores": threads,
            "kind": "oracle",
            "sample": "%s sub-box at %s of %s (%.0f blocks per cell), %d FP64 steps (first with the "
                      "real ghost domain), %.1f s" % (sample, "x".join(map(str, lo)), w.name,
                                                      blocks0 / np.prod(size), nsteps, t_steps),
            "cpu": model, "host_threads_available": avail}


def make_partition(kind, n, hot, storage, slack, order, gt_level):
    """The workload and its partition on cuda:0 (mixtures sampled on the device)."""
    from paper_2504_21450_amd import binding as B
    from paper_2504_21450_amd import workloads as W

    if kind == "mixture":
        from paper_2504_21450_amd import devsample
        w = W.blob_mixture(n=n, hot_fraction=hot, sample=False, storage=STORAGES[storage])
        w.order = order
        p = devsample.sample_partition(w, slack=slack, gt_level=gt_level)
    else:
        w = W.maxwellian_sparse(n=n, threads=min(16, os.cpu_count() or 1))
        w.storage = STORAGES[storage]
        w.order = order
        p = B.Partition.from_workload(w, slack=slack, gt_level=gt_level)
    return w, p


def run(p, w, storage, mode, steps, warmup, tune_steps, variant=None, graph_steps=0):
    """Autotune (real steps), warm up, then time `steps` whole steps (ghost
    update, three shears, pruning, moments) with per-kernel HIP events."""
    import ctypes as C

    import numpy as np
    import torch

    from paper_2504_21450_amd import binding as B

    dn = torch.empty(p.ncell, dtype=torch.float64, device="cuda:0")
    dV = torch.empty(p.ncell * 3, dtype=torch.float64, device="cuda:0")
    dP = torch.empty(p.ncell * 6, dtype=torch.float64, device="cuda:0")

    def moments():
        rc = p.lib.vl_moments(p.h, C.c_void_p(dn.data_ptr()), C.c_void_p(dV.data_ptr()),
                              C.c_void_p(dP.data_ptr()), None)
        if rc:
            raise B.VlasovError("vl_moments", rc)

    def step():
        if mode == B.VL_COALESCED:
            p.fill_ghosts()
        rc = p.lib.vl_translate_step(p.h, float(w.dt), mode, None)
        if rc:
            raise B.VlasovError("vl_translate_step", rc)
        moments()

    tune = None
    if tune_steps > 0:
        best, ms = p.autotune(w.dt, mode, steps_per_variant=tune_steps)
        tune = {"variant": best, "shear_ms_per_step": ms, "steps": tune_steps * len(ms)}
        log("autotune: variants %s, shear ms/step per variant %s"
            % (variant_key(best), ["%.2f" % v for v in ms]))
    chosen = tune["variant"] if tune else p.variants()[0]
    if variant is not None:
        p.set_variant(variant)
        chosen = variant
        if tune:
            tune["overridden_by"] = variant
    for _ in range(warmup):
        step()
    p.sync()
    blocks0 = p.local_blocks()
    c0 = p.counters()
    p.profile_start(64 * (steps + 1))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t1
    prof = p.profile_stop()
    p.sync()
    c1 = p.counters()
    blocks1 = p.local_blocks()
    bs = BYTES[storage]
    local_ps = 0.5 * (blocks0 + blocks1) * 64
    computed = c1["cum_upd"] - c0["cum_upd"]
    read = c1["cum_read"] - c0["cum_read"]
    shear_ms, shear_n = prof["shear"]
    out = {
        "elapsed": elapsed, "steps": steps, "ms_per_step": 1e3 * elapsed / steps,
        "value": 3 * local_ps * steps / elapsed, "computed_updates_per_s": computed / elapsed,
        "blocks": int(blocks1), "variant": chosen, "autotune": tune,
        "shear_bytes_per_launch": (read + computed) * bs / max(shear_n, 1),
        "shear_avg_launch_s": shear_ms / max(shear_n, 1) / 1e3, "shear_launches": shear_n,
        "kernel_ms_per_step": {k: v[0] / steps for k, v in prof.items()},
        "per_shear": [{"axis": "xyz"[w.order[s]],
                       "ms": prof["shear%d" % (s + 1)][0] / max(prof["shear%d" % (s + 1)][1], 1),
                       "algorithmic_gb": (c1["upd%d" % s] + c1["read%d" % s]) * bs / 1e9,
                       "items": c1["items%d" % s]} for s in range(3)],
    }
    for s in out["per_shear"]:
        s["gbs"] = s["algorithmic_gb"] / (s["ms"] / 1e3) if s["ms"] > 0 else None
    out["shear_gbs"] = out["shear_bytes_per_launch"] / out["shear_avg_launch_s"] / 1e9 if shear_n else None
    if graph_steps > 0:
        # the same steps replayed from HIP graphs (ghost update, shears and
        # pruning recorded once per list region; moments launched as before)
        for _ in range(2):
            p.graph_step(w.dt, mode)
            moments()
        p.sync()
        b0 = p.local_blocks()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        for _ in range(graph_steps):
            p.graph_step(w.dt, mode)
            moments()
        torch.cuda.synchronize()
        ge = time.perf_counter() - t2
        p.sync()
        b1 = p.local_blocks()
        out["graph"] = {"steps": graph_steps, "ms_per_step": 1e3 * ge / graph_steps,
                        "value": 3 * 0.5 * (b0 + b1) * 64 * graph_steps / ge}
        log("graph replay: %.2f ms/step" % (1e3 * ge / graph_steps))
    # one more step (untimed) with the FP64 mass statistics: the mass held in
    # f and the mass in f plus the rounding ledger, each against the mass
    # before the step less what the pruning removed
    if mode == B.VL_COALESCED:
        p.fill_ghosts()
    st = p.step(w.dt, mode, stats=True)
    m0 = st["mass_before"]
    out["mass_one_step"] = {
        "stored_only_rel": (st["mass_after"] + st["pruned_mass"] - m0) / m0,
        "stored_plus_ledger_rel": (st["mass_after"] + st["pruned_mass"] + st["ledger_mass"] - m0) / m0,
        "pruned_rel": st["pruned_mass"] / m0}
    return out


def accel_run(kind, n, hot, storage, steps, slack=3.0):
    """Acceleration steps (the Lorentz-force half of the split step) on a
    partition of their own, in seeded per-cell fields: time per step, and the
    remap kernel's algorithmic bytes (each of the three remaps reads and
    writes every block once: 6 x 64 values per block) per launch over its
    HIP-event time.  The blocks that the three remaps create stay until the
    step's pruning, so the pool needs room for about half as many again as
    the hot cells hold (slack 3)."""
    import torch

    from paper_2504_21450_amd import workloads as W

    t0 = time.time()
    w, p = make_partition(kind, n, hot, storage, slack, (0, 1, 2), 3)
    log("acceleration workload %s %s: %d blocks, workspace %.1f GB (%.0f s)" % (
        "x".join(map(str, n)), storage, w.nblocks, p.ws_bytes / 1e9, time.time() - t0))
    EB, dt = W.lorentz_fields(p.ncell)
    fields = torch.tensor(EB.reshape(-1), dtype=torch.float64, device="cuda:0")
    qm = 9.58e7
    p.accelerate(dt, qm, fields)  # warm-up
    p.sync()
    b0 = p.local_blocks()
    p.profile_start(16 * steps + 16)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        p.accelerate(dt, qm, fields)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = p.profile_stop()
    b1 = p.local_blocks()
    ms, nl = prof["accel"]
    bytes_per_launch = 6 * 64 * BYTES[storage] * 0.5 * (b0 + b1)
    gbs = bytes_per_launch / (ms / max(nl, 1) / 1e3) / 1e9 if nl else None
    del fields
    p.close()
    del p
    torch.cuda.empty_cache()
    return {"workload": w.name, "storage": storage, "initial_blocks": int(w.nblocks),
            "fields": "seeded per-cell E, B (|B| 5-15 nT, random direction; E x B drift ~1e5 m/s; "
                      "parallel E up to 2 velocity cells per step); gyration 0.15-0.45 rad per step",
            "steps": steps, "ms_per_step": 1e3 * el / steps,
            "kernel_ms_per_step": {"accel": ms / steps, "prune": prof["prune"][0] / steps},
            "local_blocks": int(b1), "algorithmic_bytes_per_launch": bytes_per_launch,
            "avg_launch_ms": ms / max(nl, 1), "gbs": gbs, "frac_of_hbm_peak": (gbs or 0.0) / HBM_PEAK_GBS,
            "block_updates_per_s": 3 * 0.5 * (b0 + b1) * 64 * steps / el}


def side_run(kind, n, hot, storage, steps, tune_steps, slack=None):
    """A shorter measurement of another workload or storage (for the extras).
    Pool slack: 1.8, or 1.4 in FP64 (the 96x96x12 mixture at 40 % hot holds
    2e8 blocks; its ~18 steps grow the hot regions by ~1.27x, and FP64 at 1.8
    would need 309 GiB)."""
    if slack is None:
        slack = 1.4 if storage == "f64" else 1.8
    import torch

    from paper_2504_21450_amd import binding as B

    t0 = time.time()
    w, p = make_partition(kind, n, hot, storage, slack, (0, 1, 2), 3)
    log("%s %s %s: %d blocks, workspace %.1f GB (%.0f s)" % (kind, "x".join(map(str, n)), storage,
                                                             w.nblocks, p.ws_bytes / 1e9, time.time() - t0))
    r = run(p, w, storage, B.VL_COALESCED, steps, 2, tune_steps)
    p.close()
    del p
    torch.cuda.empty_cache()
    return {"workload": w.name, "storage": storage, "ms_per_step": r["ms_per_step"], "value": r["value"],
            "shear_gbs": r["shear_gbs"], "shear_frac_of_peak": (r["shear_gbs"] or 0.0) / HBM_PEAK_GBS,
            "kernel_ms_per_step": r["kernel_ms_per_step"], "variant": variant_key(r["variant"]),
            "local_blocks": r["blocks"], "steps": steps}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="mixture", choices=["mixture", "maxwellian"])
    ap.add_argument("--storage", default=None, choices=sorted(STORAGES),
                    help="storage of f (default bf16 for the mixture, f64 for the Maxwellian case)")
    ap.add_argument("--nx", default=None, help="local spatial box (default 128x128x64 for the mixture, "
                                               "64x64x32 for the Maxwellian case)")
    ap.add_argument("--hot", type=float, default=HOT_500, help="hot-cell fraction of the mixture")
    ap.add_argument("--mode", default="coalesced", choices=["coalesced", "per_sweep"])
    ap.add_argument("--order", default="xyz", choices=["xyz", "zxy", "yzx"],
                    help="shear order (the paper's is zxy)")
    ap.add_argument("--gt-level", type=int, default=3, choices=[1, 2, 3],
                    help="Ghost Translation level of the coalesced mode (3 = exact)")
    ap.add_argument("--slack", type=float, default=None,
                    help="block and list capacity over the initial block count (default 2.0: the "
                         "mixture's hot regions grow by ~7.5 %% in the first step and ~1 %% per step "
                         "after, and every step of a default run fits, 50 as well)")
    ap.add_argument("--tune-steps", type=int, default=1,
                    help="real steps per shear variant for the autotuner, on the measured partition "
                         "before warmup (0 to skip)")
    ap.add_argument("--variant", type=parse_variant, default=None,
                    help="shear variant for the timed steps, one for all shears or 'a,b,c' for the "
                         "first, second and third (the autotuner's steps still run unless "
                         "--tune-steps 0, so the state evolves as in a default run)")
    ap.add_argument("--graph-steps", type=int, default=None,
                    help="steps replayed from recorded HIP graphs after the timed region "
                         "(default: min(--steps, 10); 0 to skip)")
    ap.add_argument("--accel-steps", type=int, default=3,
                    help="acceleration steps timed after the translation steps (0 to skip)")
    ap.add_argument("--extra-steps", type=int, default=5,
                    help="timed steps of the FP32 reference and of the FP32-vs-FP64 comparison "
                         "(0 skips both)")
    ap.add_argument("--cpu-sample", default="24x24x12", help="oracle sub-box")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="after the timed steps, run 1 GiB device-to-device copies (a reference "
                         "kernel for HBM counter calibration under rocprofv3)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build runs on one GPU only (the multi-GPU halo exchange is a "
              "design, not an implementation); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2504_21450_amd import binding as B

    mixture = args.workload == "mixture"
    storage = args.storage or ("bf16" if mixture else "f64")
    n = tuple(int(v) for v in (args.nx or ("128x128x64" if mixture else "64x64x32")).split("x"))
    slack = args.slack if args.slack is not None else 2.0
    order = tuple("xyz".index(a) for a in args.order)
    mode = B.VL_COALESCED if args.mode == "coalesced" else B.VL_PER_SWEEP
    gsteps = min(args.steps, 10) if args.graph_steps is None else args.graph_steps

    t0 = time.time()
    log("generating workload %s (%s) ..." % ("x".join(map(str, n)), storage))
    w, p = make_partition(args.workload, n, args.hot, storage, slack, order, args.gt_level)
    log("generated %d blocks (%.3e phase-space cells) in %.1f s; workspace %.1f GB"
        % (w.nblocks, w.nblocks * 64.0, time.time() - t0, p.ws_bytes / 1e9))
    r = run(p, w, storage, mode, args.steps, args.warmup, args.tune_steps, args.variant, gsteps)
    log("timed %d steps in %.3f s; kernel ms per step %s" % (
        args.steps, r["elapsed"], {k: round(v, 2) for k, v in r["kernel_ms_per_step"].items()}))
    if args.calibrate_copy:
        src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda:0").fill_(1)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    blocks_per_cell = np.diff(w.offsets)
    p.close()
    del p
    torch.cuda.empty_cache()

    variant = r["variant"]
    achieved = r["shear_gbs"]
    traffic = (measured_traffic(storage, variant, w.name)
               if args.gt_level == 3 and args.order == "xyz" and args.mode == "coalesced" else None)
    what = ("HBM-filling blob mixture, BF16 storage with FP32 reconstruction and FP64 flux, update, "
            "ledger and moments" if mixture and storage == "bf16" else
            "blob mixture" if mixture else "smooth sparse Maxwellians")
    out = {
        "metric": METRIC,
        "value": r["value"],
        "unit": "phase-space cell updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": storage,
        "data": "synthetic",
        "config": {"workload": "%s: %s, coalesced-ghost sparse translation (%s mode%s%s)"
                               % (w.name, what, args.mode,
                                  "" if args.gt_level == 3 else ", GT%d" % args.gt_level,
                                  "" if args.order == "xyz" else ", %s order" % args.order),
                   "cells": list(n), "velocity_cells": [4 * b for b in w.nblk], "storage": storage,
                   "hot_fraction": args.hot if mixture else None,
                   "initial_blocks": int(w.nblocks), "local_blocks": r["blocks"],
                   "local_ps_cells": int(r["blocks"] * 64),
                   "blocks_per_cell": {"min": int(blocks_per_cell.min()),
                                       "median": float(np.median(blocks_per_cell)),
                                       "max": int(blocks_per_cell.max()),
                                       "mean": float(blocks_per_cell.mean())},
                   "steps_before_timing": (r["autotune"]["steps"] if r["autotune"] else 0) + args.warmup,
                   "dt_over_dx_max_courant": w.max_courant()},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_sweep (PPM shear), %s storage, variants %s" % (storage, variant_key(variant)),
                     "algorithmic_bytes_per_launch": r["shear_bytes_per_launch"],
                     "avg_launch_ms": 1e3 * r["shear_avg_launch_s"], "launches": r["shear_launches"]},
        "computed_updates_per_s": r["computed_updates_per_s"],
        "kernel_ms_per_step": r["kernel_ms_per_step"],
        "autotune": r["autotune"],
        "per_shear": r["per_shear"],
    }
    if "graph" in r:
        out["graph"] = r["graph"]
    out["mass_one_step"] = r["mass_one_step"]
    if args.accel_steps > 0:
        acc_n = (n[0], n[1], max(1, n[2] // 2)) if mixture else n
        acc = accel_run(args.workload, acc_n, args.hot, storage, args.accel_steps)
        log("acceleration: %.2f ms/step, remap kernel %.2f ms (%.0f GB/s)" % (
            acc["ms_per_step"], acc["avg_launch_ms"], acc["gbs"] or 0.0))
        out["acceleration"] = acc
    if mixture and args.extra_steps > 0:
        ref_n = (n[0], n[1], max(1, n[2] // 2))
        log("FP32 reference at %s ..." % "x".join(map(str, ref_n)))
        out["fp32_reference"] = side_run("mixture", ref_n, args.hot, "f32", args.extra_steps, 1)
        cmp_n = (96, 96, 12)
        log("FP32 vs plain FP64 on the uneven mixture at %s ..." % "x".join(map(str, cmp_n)))
        f64 = side_run("mixture", cmp_n, 0.4, "f64", args.extra_steps, 1)
        f32 = side_run("mixture", cmp_n, 0.4, "f32", args.extra_steps, 1)
        out["fp32_vs_fp64"] = {"workload": f32["workload"], "fp64": f64, "fp32": f32,
                               "speedup_fp32_over_fp64": f64["ms_per_step"] / f32["ms_per_step"]}
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a %s sub-box ..." % args.cpu_sample)
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_sample)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
