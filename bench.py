#!/usr/bin/env python3
"""Throughput of the Vlasov translation step on one MI355X.

Workload (default): the sparse FP64 partition of 64 x 64 x 32 periodic
spatial cells with a coalesced ghost domain, 100^3 velocity cells in 4^3
blocks, one Maxwellian per cell (seeded smooth fields), blocks kept where
max f >= 1e-15 s^3 m^-6 plus the 6 face-neighbour blocks.  A step is the whole
path: coalesced ghost update, x, y and z shears (block growth, work list, PPM
remap) and end-of-step pruning, plus the FP64 velocity moments.

Prints one JSON line.  `value` is useful phase-space cell updates per second
(3 x local phase-space cells per step, inputs resident in HBM), `roofline`
describes the shear kernel (the dominant one) against the 8 TB/s HBM peak,
and `cpu_baseline` the FP64 CPU oracle on a sub-box of the same workload.

--workload mixture selects the uneven batched-cell workload instead: cold
solar-wind cells (~80 blocks) beside hot mixture cells (~4,300 blocks) in a
blob pattern (--hot sets the hot fraction), sampled on the device.
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


def cpu_baseline(w, sample, min_seconds=10.0, max_steps=40):
    """Time the FP64 oracle on a sub-box of the workload (explicit ghost
    domain from the full box for the first step, then periodic)."""
    import numpy as np

    import oracle
    from paper_2504_21450_amd import workloads as W

    size = tuple(int(v) for v in sample.split("x"))
    lo = tuple((w.n[d] - size[d]) // 2 for d in range(3))
    cells = W.subbox_cells(w.n, lo, size, 3)
    if w.f is not None:
        off, ids, f = W.take_cells(w.offsets, w.ids, w.f, cells)
    else:  # device-sampled workload: the host sampler gives the oracle its input
        off, ids, f = W.sample_cells(W.table_model(w.fields["params"]), w.nblk, w.vmin, w.dv,
                                     w.sparse_min, w.vbuffer, w.seed, cells,
                                     threads=min(16, os.cpu_count() or 1), batch=4)
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
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": useful / t_steps, "unit": "phase-space cell updates/s", "cores": cores,
            "kind": "oracle",
            "sample": "%s sub-box of %s, %d FP64 steps (first with the real ghost domain), %.1f s"
                      % (sample, w.name, nsteps, t_steps)}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--storage", default="f64", choices=sorted(STORAGES))
    ap.add_argument("--mode", default="coalesced", choices=["coalesced", "per_sweep"])
    ap.add_argument("--order", default="xyz", choices=["xyz", "zxy", "yzx"],
                    help="shear order (the paper's is zxy)")
    ap.add_argument("--gt-level", type=int, default=3, choices=[1, 2, 3],
                    help="Ghost Translation level of the coalesced mode (3 = exact)")
    ap.add_argument("--workload", default="maxwellian", choices=["maxwellian", "mixture"])
    ap.add_argument("--hot", type=float, default=0.4, help="hot-cell fraction of the mixture")
    ap.add_argument("--nx", default="64x64x32", help="local spatial box")
    ap.add_argument("--cpu-sample", default=None, help="oracle sub-box (default 24x24x12; "
                                                         "8x8x4 for the mixture)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--slack", type=float, default=None,
                    help="block and list capacity over the initial block count (default 2.0; 1.25 "
                         "for the mixture; the smooth case spreads by ~0.7 %% of blocks per step)")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="skip the shear-kernel autotuner (it runs real steps before warmup)")
    ap.add_argument("--variant", type=parse_variant, default=None,
                    help="shear variant for the timed steps, one for all shears or 'a,b,c' for the "
                         "first, second and third (the autotuner's steps still run unless "
                         "--no-autotune, so the state evolves as in a default run)")
    ap.add_argument("--graph-steps", type=int, default=None,
                    help="steps replayed from recorded HIP graphs after the timed region "
                         "(default: --steps; 0 to skip)")
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
    from paper_2504_21450_amd import workloads as W

    n = tuple(int(v) for v in args.nx.split("x"))
    mixture = args.workload == "mixture"
    slack = args.slack if args.slack is not None else (1.25 if mixture else 2.0)
    cpu_sample = args.cpu_sample or ("8x8x4" if mixture else "24x24x12")
    t0 = time.time()
    log("generating workload %s ..." % (n,))
    tune = None
    if mixture:
        from paper_2504_21450_amd import devsample
        if args.autotune:
            # tune on a smaller partition of the same mixture, so that the
            # measured partition starts its timed steps near its initial state;
            # it keeps the z extent (the z pencils' length decides the last
            # shear's variant) and at most 32 cells along x and y
            proxy_n = (min(n[0], 32), min(n[1], 32), n[2])
            wp = W.blob_mixture(n=proxy_n, hot_fraction=args.hot, sample=False,
                                storage=STORAGES[args.storage])
            pp = devsample.sample_partition(wp, slack=4.0)
            best, ms = pp.autotune(wp.dt, B.VL_COALESCED if args.mode == "coalesced" else B.VL_PER_SWEEP,
                                   steps_per_variant=2)
            tune = {"variant": best, "shear_ms_per_step": ms, "proxy": "x".join(map(str, proxy_n))}
            log("autotune on %s: variants %s, shear ms/step per variant %s"
                % (tune["proxy"], variant_key(best), ["%.2f" % v for v in ms]))
            pp.close()
            del pp
            torch.cuda.empty_cache()
        w = W.blob_mixture(n=n, hot_fraction=args.hot, sample=False, storage=STORAGES[args.storage])
        w.order = tuple("xyz".index(a) for a in args.order)
        p = devsample.sample_partition(w, slack=slack, gt_level=args.gt_level)
        if tune is not None:
            p.set_variant(tune["variant"])
    else:
        w = W.maxwellian_sparse(n=n, threads=min(16, os.cpu_count() or 1))
        w.storage = STORAGES[args.storage]
        w.order = tuple("xyz".index(a) for a in args.order)
        p = B.Partition.from_workload(w, slack=slack, gt_level=args.gt_level)
    log("generated %d blocks (%.3e phase-space cells) in %.1f s"
        % (w.nblocks, w.nblocks * 64.0, time.time() - t0))
    mode = B.VL_COALESCED if args.mode == "coalesced" else B.VL_PER_SWEEP

    log("partition initialised: workspace %.1f GB" % (p.ws_bytes / 1e9))
    dn = torch.empty(p.ncell, dtype=torch.float64, device="cuda:0")
    dV = torch.empty(p.ncell * 3, dtype=torch.float64, device="cuda:0")
    dP = torch.empty(p.ncell * 6, dtype=torch.float64, device="cuda:0")
    import ctypes as C

    def step():
        if mode == B.VL_COALESCED:
            p.fill_ghosts()
        rc = p.lib.vl_translate_step(p.h, float(w.dt), mode, None)
        if rc:
            raise B.VlasovError("vl_translate_step", rc)
        rc = p.lib.vl_moments(p.h, C.c_void_p(dn.data_ptr()), C.c_void_p(dV.data_ptr()),
                              C.c_void_p(dP.data_ptr()), None)
        if rc:
            raise B.VlasovError("vl_moments", rc)

    if args.autotune and not mixture:
        best, ms = p.autotune(w.dt, mode, steps_per_variant=2)
        tune = {"variant": best, "shear_ms_per_step": ms}
        log("autotune: variants %s, shear ms/step per variant %s" % (variant_key(best), ["%.2f" % v for v in ms]))
    variant = tune["variant"] if tune else 0
    if args.variant is not None:
        p.set_variant(args.variant)
        variant = args.variant
        if tune:
            tune["overridden_by"] = args.variant
    for _ in range(args.warmup):
        step()
    p.sync()
    log("warmup done")
    blocks0 = p.local_blocks()
    c0 = p.counters()
    p.profile_start(64 * (args.steps + 1))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t1
    prof = p.profile_stop()
    p.sync()
    c1 = p.counters()
    blocks1 = p.local_blocks()
    log("timed %d steps in %.3f s" % (args.steps, elapsed))

    bs = BYTES[args.storage]
    local_ps = 0.5 * (blocks0 + blocks1) * 64
    useful = 3 * local_ps * args.steps
    computed = c1["cum_upd"] - c0["cum_upd"]
    read = c1["cum_read"] - c0["cum_read"]
    shear_ms, shear_n = prof["shear"]
    shear_bytes = (read + computed) * bs      # algorithmic payload bytes of the shears
    per_launch = shear_bytes / max(shear_n, 1)
    avg_launch_s = shear_ms / max(shear_n, 1) / 1e3
    achieved = per_launch / avg_launch_s / 1e9
    traffic = (measured_traffic(args.storage, variant, w.name)
               if args.gt_level == 3 and args.order == "xyz" and args.mode == "coalesced" else None)

    out = {
        "metric": METRIC,
        "value": useful / elapsed,
        "unit": "phase-space cell updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.storage,
        "data": "synthetic",
        "config": {"workload": "%s coalesced-ghost sparse translation (%s storage, %s mode%s%s)"
                               % (w.name, args.storage, args.mode,
                                  "" if args.gt_level == 3 else ", GT%d" % args.gt_level,
                                  "" if args.order == "xyz" else ", %s order" % args.order),
                   "cells": list(n), "velocity_cells": [4 * b for b in w.nblk],
                   "local_blocks": int(blocks1), "local_ps_cells": int(blocks1 * 64),
                   "blocks_per_cell": [int(v) for v in np.percentile(np.diff(w.offsets), [0, 50, 100])],
                   "dt_over_dx_max_courant": w.max_courant()},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_sweep (PPM shear), variants %s" % variant_key(variant),
                     "algorithmic_bytes_per_launch": per_launch,
                     "avg_launch_ms": 1e3 * avg_launch_s, "launches": shear_n},
        "computed_updates_per_s": computed / elapsed,
        "kernel_ms_per_step": {k: v[0] / args.steps for k, v in prof.items()},
        "autotune": tune,
        "per_shear": [{"axis": "xyz"[w.order[s]],
                       "ms": prof["shear%d" % (s + 1)][0] / max(prof["shear%d" % (s + 1)][1], 1),
                       "algorithmic_gb": (c1["upd%d" % s] + c1["read%d" % s]) * bs / 1e9,
                       "items": c1["items%d" % s]} for s in range(3)],
    }
    for s in out["per_shear"]:
        s["gbs"] = s["algorithmic_gb"] / (s["ms"] / 1e3) if s["ms"] > 0 else None
    gsteps = args.steps if args.graph_steps is None else args.graph_steps
    if gsteps > 0:
        # the same steps replayed from HIP graphs (ghost update, shears and
        # pruning recorded once per list region; moments launched as before)
        def moments():
            rc = p.lib.vl_moments(p.h, C.c_void_p(dn.data_ptr()), C.c_void_p(dV.data_ptr()),
                                  C.c_void_p(dP.data_ptr()), None)
            if rc:
                raise B.VlasovError("vl_moments", rc)
        for _ in range(2):
            p.graph_step(w.dt, mode)
            moments()
        p.sync()
        b0 = p.local_blocks()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        for _ in range(gsteps):
            p.graph_step(w.dt, mode)
            moments()
        torch.cuda.synchronize()
        ge = time.perf_counter() - t2
        p.sync()
        b1 = p.local_blocks()
        out["graph"] = {"steps": gsteps, "ms_per_step": 1e3 * ge / gsteps,
                        "value": 3 * 0.5 * (b0 + b1) * 64 * gsteps / ge}
        log("graph replay: %.2f ms/step" % (1e3 * ge / gsteps))
    if args.calibrate_copy:
        src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda:0").fill_(1)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a %s sub-box ..." % cpu_sample)
        out["cpu_baseline"] = cpu_baseline(w, cpu_sample)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
