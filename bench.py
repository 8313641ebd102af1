#!/usr/bin/env python3
"""Benchmark: candidate formulae evaluated per second on one MI355X.

A step is one pass of the whole hot path over one batch of synthetic input: the
learning jobs of the long-trace workload (5 propositions, 4096 + 4096 traces of
length 64..512, Bernoulli(0.3) letters, planted formula of size 11, unit costs,
cost bound 13, multi-word 64-bit rows), seeds 0..3, each solved from a
device-resident specification, the four in flight together on the 4 lanes of a
batch executor (own stream, equal workspace slice, hash table each).  The metric is
the number of canonical candidates evaluated, over the timed wall time.

The same line carries the scale workload (3 propositions, 1024 + 1024 traces of
length 16..32, bound 11, 32-bit rows; 8 jobs, 4 in flight) as a secondary object.

Prints ONE JSON line: the metric and its config, per-kernel GPU time (HIP events on
the library's streams), the roofline of the level pipeline and the CPU oracle timed
on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import gc
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0            # MI355X HBM3E, 8 TB/s
LONG_JOB_GIB = 46                # workspace a long job needs (its largest: ~41 GiB), with a margin
KERNEL_SRC = os.path.join(ROOT, "paper_2402_12373_amd", "csrc", "ltl_kernels.hip")
TRAFFIC_FILES = [os.path.join(ROOT, "profiles", f) for f in ("traffic_long.json", "traffic_scale.json")]


def measured_traffic(kind: str, workload_key: str):
    """Calibrated HBM bytes per launch of a kernel kind, from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary -- only for the workload the counters were taken on,
    and only if the kernel source is unchanged since."""
    import hashlib
    try:
        src = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    except OSError:
        return None
    for path in TRAFFIC_FILES:
        try:
            rec = json.load(open(path))
        except (OSError, ValueError):
            continue
        if rec.get("kernel_source_sha256") != src or rec.get("workload_key") != workload_key:
            continue
        k = rec.get("per_launch_bytes", {}).get(kind)
        return None if k is None else float(k)
    return None
# level-pipeline kernels (evaluation, write pass, verification, compaction, probe, fallback)
LEVEL_KERNELS = ("k_level", "k_probe", "k_materialize", "k_mark_members", "k_compact_small", "k_mark", "k_scan_",
                 "k_scatter", "k_or_bits", "k_fallback")


def summarize_counters(fetch_dir: str, write_dir: str, workload_key: str, out_path: str) -> None:
    """Writes the calibrated HBM bytes per level-kernel dispatch from two rocprofv3 --pmc runs
    of this bench (FETCH_SIZE, then WRITE_SIZE, --output-format csv) that each ran with
    --copy-calibration-mib 1024: the largest copy dispatch of each run (1 GiB read and
    written) gives the factor that turns the counter's KiB into bytes."""
    import csv
    import glob
    import hashlib

    def per_dispatch(d, counter):
        v = {}
        files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
        if not files:
            raise SystemExit(f"no counter_collection.csv under {d}")
        for f in files:
            with open(f) as fh:
                for r in csv.DictReader(fh):
                    if r["Counter_Name"] == counter:
                        e = v.setdefault((f, r["Dispatch_Id"]), [r["Kernel_Name"], 0.0])
                        e[1] += float(r["Counter_Value"])
        return list(v.values())

    def is_level(name):
        base = name.split("(")[0].split("<")[0].replace("void ", "").replace("ltl::", "").strip()
        return base.startswith(LEVEL_KERNELS)

    F, W = per_dispatch(fetch_dir, "FETCH_SIZE"), per_dispatch(write_dir, "WRITE_SIZE")
    gib_kib = float(1 << 20)
    scale = []
    for D in (F, W):
        copies = [val for name, val in D if "copyBuffer" in name]
        if not copies:
            raise SystemExit("no copy dispatch to calibrate with (run with --copy-calibration-mib 1024)")
        scale.append(gib_kib / max(copies))
    fetch = [val * scale[0] * 1024 for name, val in F if is_level(name)]
    write = [val * scale[1] * 1024 for name, val in W if is_level(name)]
    if not fetch or len(fetch) != len(write):
        raise SystemExit(f"level dispatches differ between the runs: {len(fetch)} vs {len(write)}")
    per = (sum(fetch) + sum(write)) / len(fetch)
    rec = {"kernel_source_sha256": hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest(),
           "per_launch_bytes": {"level": per}, "dispatches": {"level": len(fetch)},
           "read_bytes_per_launch": sum(fetch) / len(fetch), "write_bytes_per_launch": sum(write) / len(write),
           "calibration": {"fetch_factor": round(scale[0], 4), "write_factor": round(scale[1], 4)},
           "note": "calibrated FETCH_SIZE + WRITE_SIZE per dispatch of the level kernels, one bench step + warm-up",
           "workload_key": workload_key}
    with open(out_path, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps({"per_launch_MB": round(per / 1e6, 3), "dispatches": len(fetch),
                      "fetch_factor": rec["calibration"]["fetch_factor"],
                      "write_factor": rec["calibration"]["write_factor"], "out": out_path}))


VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12   # 32-bit integer lane-ops/s: 256 CUs x 64 lanes x 2.4 GHz = 39.3 T


def workload_key(args) -> str:
    """Names a fixed workload with its seeds and bound (the key of a committed counter summary)."""
    from ltl_inputs import synth
    if not args.seeds:
        args.seeds = "0-3" if args.workload == "long" else "0-7"
    bound = args.bound or (16 if args.workload == "hamming" else synth.PRESETS[args.workload]["bound"])
    return (f"{args.workload} seeds {args.seeds} bound {bound}" + (" ruc" if args.ruc else "")
            + (" fkp" if args.ruc and args.fkp else "")
            + (" ucarry" if args.ucarry else "") + (" udoubling" if args.udoubling else ""))


def parse_seeds(s: str):
    out = []
    for part in s.split(","):
        if "-" in part:
            a, b = part.split("-")
            out += list(range(int(a), int(b) + 1))
        elif part:
            out.append(int(part))
    return out


# Algorithmic work per candidate, per 32-bit half-word of its matrix, in basic 32-bit
# integer operations:
#   connective: NOT 2, AND/OR 1, X 1, F 2 (x | -x), G 5, ATOM 0,
#               U by doubling (App. B, k steps) 5k-2, U by the carry adder 5
#   fingerprint 6 (premix: two shift-xor pairs and the row key added between them;
#               one 32x32->64 multiply-add)
#   separation 2 (xor with the expected bit, or into the violation word)
OP_OPS = {"atom": 0, "not": 2, "and": 1, "or": 1, "x": 1, "f": 2, "g": 5}
FP_SEP_OPS = 6 + 2


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    # the first three or four steps of a process run slow (9-12 ms against about 5 on the
    # scale workload), so the untimed warm-up covers them
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="long", choices=["tiny", "scale", "long", "batched", "hamming", "served"])
    ap.add_argument("--no-secondary", action="store_true",
                    help="long workload: skip the secondary scale-workload object")
    ap.add_argument("--rate", type=float, default=10.0, help="served workload: Poisson arrival rate (jobs/s)")
    ap.add_argument("--ham-length", type=int, default=4, help="hamming workload: length of the positive trace")
    ap.add_argument("--ham-delta", type=int, default=2, help="hamming workload: bit distance of the negatives")
    ap.add_argument("--jobs", type=int, default=256, help="batched workload: number of jobs")
    ap.add_argument("--lanes", type=int, default=0,
                    help="jobs in flight (lanes of a batch executor: own stream, equal workspace slice, hash "
                         "table); default 4 (a long job needs ~41 GiB, a slice of the default workspace 50); "
                         "1 = one job after another on one stream")
    ap.add_argument("--seeds", default="", help="job seeds, e.g. 0-7 (default: 0-3 for long, else 0-7)")
    ap.add_argument("--bound", type=int, default=0, help="cost bound (default: the workload's)")
    ap.add_argument("--workspace-gb", type=float, default=0.0)
    ap.add_argument("--ucarry", action="store_true", help="U by the carry adder at every level (LTL_CTX_U_CARRY)")
    ap.add_argument("--udoubling", action="store_true",
                    help="U by the doubling of App. B at every level (LTL_CTX_U_DOUBLING); default: the carry "
                         "adder")
    ap.add_argument("--lds-tiles", action="store_true",
                    help="binary tiles of whole-row levels stage 8 x 8 groups of child words in LDS instead of "
                         "reading 4 x 4 tiles into registers (LTL_CTX_LDS_TILES)")
    ap.add_argument("--split-tiles", type=int, default=0,
                    help="levels of fewer tiles run the row-split kernels (ltl_ctx_opts.split_tiles; "
                         "0 = the library default, 1 = whole-row kernels at every level)")
    ap.add_argument("--ruc", action="store_true",
                    help="relaxed uniqueness check (LTL_CTX_RUC, Sec. 5): a candidate is cached iff its 126-bit key "
                         "is new, no matrix compare")
    ap.add_argument("--fkp", action="store_true", help="with --ruc: first-k-percent keys (LTL_CTX_RUC_FKP, Sec. 7)")
    ap.add_argument("--big-alone", action="store_true",
                    help="batch lanes take turns for whole-row levels (LTL_BATCH_BIG_ALONE)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="batched: skip the autotuner (ltl_autotune on the largest of the first 16 jobs chooses "
                         "the binary tile shape and the whole-row level size for the plain and batched runs)")
    ap.add_argument("--one-stream", action="store_true",
                    help="lanes > 1: each lane runs every kernel on its own stream, the U class of a "
                         "whole-row level included (LTL_CTX_ONE_STREAM)")
    ap.add_argument("--slices", action="store_true",
                    help="batched/served: equal workspace slices per lane instead of one shared budget "
                         "with regions sized per job (LTL_BATCH_SHARED_BUDGET)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-timing", action="store_true",
                    help="no per-kernel HIP events (no kernel times, no roofline)")
    ap.add_argument("--cpu-levels", type=int, default=0,
                    help="levels per job in the CPU-baseline sample (default: 4 for the long workload, 15 for hamming, "
                         "6 for batched, else 8)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="before the run, copy this many MiB device-to-device (a kernel of known traffic for "
                         "scaling rocprofv3 FETCH_SIZE / WRITE_SIZE)")
    ap.add_argument("--summarize-counters", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "OUT_JSON"),
                    help="no run: write the calibrated bytes per level dispatch from two rocprofv3 --pmc runs "
                         "(FETCH_SIZE, WRITE_SIZE) of this bench with the same workload options")
    args = ap.parse_args()

    if args.summarize_counters:
        fd, wd, out = args.summarize_counters
        return summarize_counters(fd, wd, workload_key(args), out)

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build measures one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    if args.workload == "batched":
        return bench_batched(args)
    if args.workload == "served":
        return bench_served(args)
    out = bench_fixed(args)
    if args.workload == "long" and not args.no_secondary:
        import copy
        import torch
        torch.cuda.empty_cache()
        sa = copy.copy(args)
        sa.workload, sa.seeds, sa.lanes, sa.bound, sa.no_cpu_baseline = "scale", "", 0, 0, True
        sa.copy_calibration_mib = 0
        sec = bench_fixed(sa)
        keep = ("value", "unit", "ms_per_step", "steps", "warmup", "config", "roofline", "sequential", "minimal_costs",
                "statuses", "jobs_per_s", "candidates_per_kernel_s", "hbm_model")
        out["secondary"] = {"scale": {k: sec[k] for k in keep if k in sec}}
    print(json.dumps(out), flush=True)


def bench_fixed(args):
    """One fixed workload (tiny, scale, long, hamming): returns the JSON object."""
    import numpy as np
    import torch
    from paper_2402_12373_amd import ltl
    from ltl_inputs import synth

    if not args.seeds:
        args.seeds = "0-3" if args.workload == "long" else "0-7"
    seeds = parse_seeds(args.seeds)
    ops = None                       # every connective, negation anywhere
    if args.workload == "hamming":
        # Hamming(B, l, delta) with the U-free NNF operator set of the experiments (Sec. 7)
        cfg = dict(num_props=2, bound=16, word_bits=32 if args.ham_length <= 32 else 64)
        ops = (0xFF & ~(1 << ltl.U)) | ltl.OPS_NNF
        insts = [synth.hamming_instance(s, args.ham_length, args.ham_delta) for s in seeds]
        workload_desc = (f"hamming: Hamming(B, {args.ham_length}, {args.ham_delta}) over 2 props, 1+"
                         f"{insts[0].num_traces - 1} traces, U-free NNF operator set")
    else:
        cfg = dict(synth.PRESETS[args.workload])
        insts = [synth.preset_instance(args.workload, s)[0] for s in seeds]
        workload_desc = (f"{args.workload}: {cfg['num_props']} props, {cfg['k']}+{cfg['k']} traces, "
                         f"len {cfg['lo']}..{cfg['hi']}, p={cfg['p']}, planted size {cfg['size']}")
    if args.bound:
        cfg["bound"] = args.bound
    dev = [ltl.spec_to_device(i) for i in insts]            # inputs resident in HBM

    if args.copy_calibration_mib:
        n = args.copy_calibration_mib << 20
        src = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(1)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    copy_gbps = copy_ceiling(torch)

    free, total = torch.cuda.mem_get_info()
    ws_bytes = int(args.workspace_gb * 2 ** 30) if args.workspace_gb else int(min(free * 0.85, 200 * 2 ** 30))
    slots = 26 if args.workload != "tiny" else 20
    ucarry = (ltl.CTX_U_CARRY if args.ucarry else 0) | (ltl.CTX_U_DOUBLING if args.udoubling else 0) | \
        (ltl.CTX_RUC if args.ruc else 0) | (ltl.CTX_RUC_FKP if args.ruc and args.fkp else 0) | \
        (ltl.CTX_LDS_TILES if args.lds_tiles else 0)
    # timed steps: one event pair per level (level GPU time, for the roofline); the one-stream
    # pass: events around every kernel group (time per kernel kind)
    timed_flags = (0 if args.no_timing else ltl.CTX_TIMING_LEVEL) | ucarry
    full_flags = (0 if args.no_timing else ltl.CTX_TIMING) | ucarry
    lanes = args.lanes or 4
    if args.workload == "long" and not args.lanes:
        lanes = min(lanes, max(1, ws_bytes // (LONG_JOB_GIB << 30)))    # every lane must hold a whole job
    lanes = max(1, min(lanes, len(dev)))
    # lanes > 1: the batch executor takes the workspace in equal slices; the one-stream
    # comparison run afterwards gets a workspace of one lane's size, so both see the same
    # capacity per job
    ctx_bytes = ws_bytes if lanes == 1 else (ws_bytes // lanes) & ~255

    def one_stream_context():
        return ltl.Context(workspace_bytes=ctx_bytes, hash_slots_log2=slots,
                           flags=full_flags if lanes > 1 else timed_flags, split_tiles=args.split_tiles)

    ctx = None if lanes > 1 else one_stream_context()
    if lanes > 1:
        ex = ltl.Batch(lanes=lanes, workspace_bytes=ctx_bytes * lanes, hash_slots_log2=slots,
                       flags=timed_flags | (ltl.BATCH_BIG_ALONE if args.big_alone else 0)
                       | (ltl.CTX_ONE_STREAM if args.one_stream else 0))

        def step():
            res, dur, done = ex.run(dev, [cfg["bound"]] * len(dev), ops=ops)
            step.last = [(round(d - u, 3), round(d, 3)) for u, d in zip(dur, done)]
            return res, dur
    else:
        def step():
            res, dur = [], []
            for d in dev:
                a = time.perf_counter()
                res.append(ctx.learn(d, cfg["bound"], ops=ops))
                dur.append((time.perf_counter() - a) * 1e3)
            return res, dur

    for _ in range(args.warmup):
        step()
    results, job_ms, step_ms, step_jobs = [], [], [], []
    gc.collect()
    gc.disable()             # no collector pauses inside the timed steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        res, dur = step()
        step_ms.append(round((time.perf_counter() - ts) * 1e3, 3))
        step_jobs.append(getattr(step, "last", None))
        results += res
        job_ms += dur
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    gc.enable()
    wall = t1 - t0
    if lanes > 1:          # the batch's workspace goes back before the one-stream context takes its own
        ex.close()
        del ex
        torch.cuda.empty_cache()
        ctx = one_stream_context()

    cands = sum(r.candidates for r in results)
    value = cands / wall
    tb = [int(i.total_positions) for i in insts]
    tb_mean = sum(tb) / len(tb)

    # algorithmic work of the evaluation / verify kernels
    job = ctx.job(dev[0], 1)
    info = job.info()
    job.close()
    geom = dict(R=int(info.rows), halves=int(info.rows) * (int(info.word_bits) // 32), k=int(info.doubling_steps),
                cm_bytes=int(info.cm_bytes))
    # the U method the library used: the carry adder unless the doubling is forced
    u_carry = args.ucarry or not args.udoubling
    # lanes > 1: the levels of different jobs overlap on the device, so their summed event
    # time counts overlapping intervals more than once; the wall time of the timed steps is
    # the basis then (a lower bound of the fraction)
    roof, kern_ms, eval_tops, verify_gbs = roofline(ltl, results, geom, u_carry,
                                                    wall_ms=wall * 1e3 if lanes > 1 else None)
    t = measured_traffic(roof["kind"], workload_key(args))
    roof["traffic"] = None if t is None else round(t / 1e6, 3)
    roof["traffic_unit"] = "MB per launch (rocprofv3 FETCH_SIZE x2.0 + WRITE_SIZE x1.0)"

    # the same jobs one after another on one stream (context for the concurrent figure)
    seq = None
    if lanes > 1:
        gc.disable()
        torch.cuda.synchronize()
        a = time.perf_counter()
        sres = [ctx.learn(d, cfg["bound"], ops=ops) for d in dev]
        torch.cuda.synchronize()
        sw = time.perf_counter() - a
        gc.enable()
        same = all((x.status, x.cost, x.level_new, x.solution_index) == (y.status, y.cost, y.level_new, y.solution_index)
                   for x, y in zip(sres, results[:len(dev)]))
        sroof, skern, _, _ = roofline(ltl, sres, geom, u_carry)
        seq = {"candidates_per_s": round(sum(r.candidates for r in sres) / sw, 1), "ms_per_step": round(sw * 1e3, 3),
               "roofline_frac": sroof["frac"], "avg_launch_ms": sroof["avg_launch_ms"],
               "kernel_ms_per_step": {k: round(v, 3) for k, v in skern.items()},
               "valu_view": sroof.get("valu_view"), "verify_view": sroof.get("verify_view"),
               "identical_results": same}
    one_stream = sres if lanes > 1 else results[:len(dev)]
    # candidates over summed level-kernel time (one stream: no overlap between jobs)
    kms = sum(sum(r.level_ms) for r in one_stream)
    cand_kernel = sum(r.candidates for r in one_stream) / (kms * 1e-3) if kms else None
    # algorithmic HBM bytes (one matrix per candidate, children once per tile) over level-kernel time
    alg = sum(sum(r.level_bytes) for r in one_stream)
    hbm = {"bytes_per_step": alg, "GBps": round(alg / (kms * 1e-3) / 1e9, 1) if kms else None}
    if kms:
        hbm["frac_of_8TBps"] = round(alg / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
        hbm["copy_ceiling_GBps"] = round(copy_gbps, 1)
        hbm["frac_of_copy_ceiling"] = round(alg / (kms * 1e-3) / 1e9 / copy_gbps, 4)
    # per level of the largest job (one stream)
    big = max(range(len(one_stream)), key=lambda i: one_stream[i].candidates)
    rb = one_stream[big]
    per_level = [{"cost": c, "candidates": rb.level_candidates[c], "new": rb.level_new[c],
                  "kernel_ms": round(rb.level_ms[c], 4),
                  "candidates_per_kernel_s": round(rb.level_candidates[c] / (rb.level_ms[c] * 1e-3), 1)
                  if rb.level_ms[c] else None,
                  "alg_GBps": round(rb.level_bytes[c] / (rb.level_ms[c] * 1e-3) / 1e9, 1) if rb.level_ms[c] else None}
                 for c in range(1, rb.levels_done + 1)]
    # host-resident specifications: every job uploads its traces (PCIe included)
    torch.cuda.synchronize()
    a = time.perf_counter()
    hres = [ctx.learn(i, cfg["bound"], ops=ops) for i in insts]
    torch.cuda.synchronize()
    hw = time.perf_counter() - a

    out = {
        "metric": "candidate formulae evaluated/s",
        "value": round(value, 1),
        "unit": "candidates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "step_ms": step_ms,
        "slowest_step_jobs_start_end_ms": step_jobs[max(range(len(step_ms)), key=lambda i: step_ms[i])],
        "dtype": "u32" if cfg["word_bits"] == 32 else "u64",
        "data": "synthetic",
        "config": {"workload": f"{workload_desc}, cost bound {cfg['bound']}, seeds {args.seeds}",
                   "jobs_per_step": len(dev), "lanes": lanes, "hash_slots_log2": slots,
                   "u_operator": ("carry adder" if u_carry else "doubling (App. B)")
                   + ("" if args.ucarry or args.udoubling else " (the library default)"),
                   "dedup": ("relaxed (126-bit FKP keys, Sec. 7)" if args.fkp else "relaxed (126-bit keyed sums)")
                   if args.ruc else "exact (fingerprint + full compare)",
                   "binary_tiles": "LDS-staged 8 x 8 groups" if args.lds_tiles else "register 4 x 4"},
        "trace_bits_per_s": round(value * tb_mean, 1),
        "jobs_per_s": round(len(results) / wall, 3),
        "job_ms_p50": round(statistics.median(job_ms), 3),
        "job_ms_p99": round(float(np.percentile(job_ms, 99)), 3),
        "minimal_costs": [r.cost if r.status == 0 else None for r in results[:len(dev)]],
        "statuses": [r.status for r in results[:len(dev)]],
        "candidates_per_step": cands // args.steps,
        "level_gpu_ms_per_step": round(sum(sum(r.level_ms) for r in results) / args.steps, 3),
        "roofline": roof,
    }
    if seq is not None:
        out["sequential"] = seq
    out["candidates_per_kernel_s"] = round(cand_kernel, 1) if cand_kernel else None
    out["hbm_model"] = hbm
    out["per_level"] = {"job": f"seed {seeds[big]}", "levels": per_level}
    out["host_spec_candidates_per_s"] = round(sum(r.candidates for r in hres) / hw, 1)

    if not args.no_cpu_baseline:
        levels = args.cpu_levels or {"long": 4, "batched": 6, "hamming": 15}.get(args.workload, 8)
        out["cpu_baseline"] = cpu_baseline(insts, levels, ops)
    failed = [s for s, r in zip(seeds, results[:len(dev)]) if r.status < 0]
    if failed:
        print(f"warning: jobs of seeds {failed} ended in an error (statuses {out['statuses']}); "
              "fewer lanes or a larger workspace give each job more memory", file=sys.stderr, flush=True)
    ctx.close()
    return out


def bench_batched(args):
    """Batched learning: many uneven jobs, `lanes` in flight (ltl_learn_batch), against the
    plain path (the same jobs one at a time, same per-job workspace)."""
    import numpy as np
    import torch
    from paper_2402_12373_amd import ltl
    from ltl_inputs import synth
    jobs = synth.batched_jobs(0, args.jobs)
    insts = [j[0] for j in jobs]
    bounds = [j[1] for j in jobs]
    dev = [ltl.spec_to_device(i) for i in insts]
    free, _ = torch.cuda.mem_get_info()
    ws_bytes = int(args.workspace_gb * 2 ** 30) if args.workspace_gb else int(min(free * 0.85, 200 * 2 ** 30))
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    lanes = args.lanes or 4
    slice_bytes = (ws_bytes // lanes) & ~255
    slots = 0          # hash table sized by the library from each slice (2^26 slots from 1.6 GB)
    # autotuner: tile shape and level schedule, tuned on the slowest of the first 32 jobs
    # (an untimed pass with the defaults picks it: the configurations differ only on the
    # large levels of the large jobs)
    tune_flags, tune_split, tuning = 0, 0, None
    if not args.no_autotune:
        tctx = ltl.Context(workspace=ws)
        tctx.learn(dev[0], bounds[0])          # the first call of a process runs slow
        took = []
        for i in range(min(32, len(insts))):
            torch.cuda.synchronize()
            a = time.perf_counter()
            tctx.learn(dev[i], bounds[i])
            took.append(time.perf_counter() - a)
        probe = max(range(len(took)), key=lambda i: took[i])
        (tune_flags, tune_split), rows = tctx.autotune(dev[probe], bounds[probe])
        tctx.close()
        tuning = {"job": probe, "job_ms_default": round(took[probe] * 1e3, 3),
                  "chosen": {"flags": tune_flags, "split_tiles": tune_split},
                  "tried_ms": [{"flags": f, "split_tiles": t, "ms": round(ms, 3)} for f, t, ms in rows]}
    # plain path: one job per call, one at a time, in a workspace of one lane's size (slices)
    # or the whole workspace (shared budget: a job's region grows up to it)
    ctx = ltl.Context(workspace=ws[:slice_bytes], hash_slots_log2=slots, flags=tune_flags,
                      split_tiles=tune_split) if args.slices else \
        ltl.Context(workspace=ws, flags=tune_flags, split_tiles=tune_split)
    for d, b in zip(dev[:lanes], bounds[:lanes]):           # warm-up
        ctx.learn(d, b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain, plain_ms = [], []
    for d, b in zip(dev, bounds):
        a = time.perf_counter()
        plain.append(ctx.learn(d, b))
        plain_ms.append((time.perf_counter() - a) * 1e3)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    ctx.close()
    print(f"plain path: {len(plain)} jobs in {t_plain:.2f} s", file=sys.stderr, flush=True)
    # batched: a batch executor (lanes created once, outside the timed region)
    big = (ltl.BATCH_BIG_ALONE if args.big_alone else 0) | (ltl.CTX_ONE_STREAM if args.one_stream else 0)
    if args.slices:
        ex = ltl.Batch(lanes=lanes, workspace=ws[:slice_bytes * lanes], hash_slots_log2=slots,
                       flags=big | tune_flags, split_tiles=tune_split)
    else:      # one budget: regions sized by each job's estimated footprint
        ex = ltl.Batch(lanes=lanes, workspace=ws, flags=big | tune_flags | ltl.BATCH_SHARED_BUDGET,
                       split_tiles=tune_split)
    ex.run(dev[:lanes], bounds[:lanes])                     # warm-up: one job per lane
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res, dur, done = ex.run(dev, bounds)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    mem = None
    if not args.slices:
        st = ex.stats()
        mem = {"budget_gb": round(st.budget_bytes / 2 ** 30, 2), "peak_gb": round(st.peak_bytes / 2 ** 30, 2),
               "admissions": int(st.admissions), "reruns": int(st.reruns), "max_in_flight": int(st.max_in_flight)}
    ex.close()
    same = sum(1 for g, p in zip(res, plain) if (g.status, g.cost, g.level_new, g.level_candidates,
                                                 g.solution_index, g.solution) ==
               (p.status, p.cost, p.level_new, p.level_candidates, p.solution_index, p.solution))
    cands = sum(r.candidates for r in res)
    statuses = {}
    for r in res:
        statuses[str(r.status)] = statuses.get(str(r.status), 0) + 1
    out = {
        "metric": "learn jobs/s",
        "value": round(len(res) / t_batch, 3),
        "unit": "jobs/s",
        "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": round(t_batch * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": f"batched: {len(res)} jobs, props U{{2..5}}, traces/class log-U[16,2048], "
                               f"len U[8,128], planted size U[5,10], bound size+2; lanes {lanes}",
                   "lanes": lanes, "slice_gb": round(slice_bytes / 2 ** 30, 2)},
        "job_latency_ms_p50": round(float(np.percentile(done, 50)), 3),
        "job_latency_ms_p99": round(float(np.percentile(done, 99)), 3),
        "job_duration_ms_p50": round(float(np.percentile(dur, 50)), 3),
        "job_duration_ms_p99": round(float(np.percentile(dur, 99)), 3),
        "candidates_per_s": round(cands / t_batch, 1),
        "plain": {"jobs_per_s": round(len(res) / t_plain, 3), "wall_s": round(t_plain, 3),
                  "job_latency_ms_p50": round(float(np.percentile(np.cumsum(plain_ms), 50)), 3),
                  "job_latency_ms_p99": round(float(np.percentile(np.cumsum(plain_ms), 99)), 3),
                  "job_duration_ms_p50": round(float(np.percentile(plain_ms, 50)), 3),
                  "job_duration_ms_p99": round(float(np.percentile(plain_ms, 99)), 3)},
        "speedup_vs_plain": round(t_plain / t_batch, 3),
        "memory": mem,
        "autotune": tuning,
        "admission": "equal slices" if args.slices else "shared budget, regions by estimated footprint",
        "identical_to_plain": f"{same}/{len(res)}",
        "statuses": statuses,
    }
    print(json.dumps(out), flush=True)


def bench_served(args):
    """Serving: jobs of the batched mix arrive as a Poisson process (`--rate` jobs/s, seed 1)
    and free lanes take them in arrival order (ltl_batch_serve).  Reports completed jobs/s over
    the whole run and the latency from arrival to completion."""
    import numpy as np
    import torch
    from paper_2402_12373_amd import ltl
    from ltl_inputs import synth
    n = args.jobs
    jobs = synth.batched_jobs(0, n)
    insts = [j[0] for j in jobs]
    bounds = [j[1] for j in jobs]
    dev = [ltl.spec_to_device(i) for i in insts]
    arrival = synth.poisson_arrivals(1, n, args.rate)
    free, _ = torch.cuda.mem_get_info()
    ws_bytes = int(args.workspace_gb * 2 ** 30) if args.workspace_gb else int(min(free * 0.85, 200 * 2 ** 30))
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    lanes = args.lanes or 4
    slice_bytes = (ws_bytes // lanes) & ~255
    big = (ltl.BATCH_BIG_ALONE if args.big_alone else 0) | (ltl.CTX_ONE_STREAM if args.one_stream else 0)
    if args.slices:
        ex = ltl.Batch(lanes=lanes, workspace=ws[:slice_bytes * lanes], flags=big)
    else:      # one budget: regions sized by each job's estimated footprint
        ex = ltl.Batch(lanes=lanes, workspace=ws, flags=big | ltl.BATCH_SHARED_BUDGET)
    ex.run(dev[:lanes], bounds[:lanes])                     # warm-up: one job per lane
    torch.cuda.synchronize()
    print(f"serving {n} jobs arriving at {args.rate} jobs/s over {arrival[-1] / 1e3:.1f} s", file=sys.stderr,
          flush=True)
    t0 = time.perf_counter()
    res, dur, done = ex.serve(dev, bounds, arrival)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    mem = None
    if not args.slices:
        st = ex.stats()
        mem = {"budget_gb": round(st.budget_bytes / 2 ** 30, 2), "peak_gb": round(st.peak_bytes / 2 ** 30, 2),
               "admissions": int(st.admissions), "reruns": int(st.reruns), "max_in_flight": int(st.max_in_flight)}
    ex.close()
    lat = [d - a for d, a in zip(done, arrival)]
    statuses = {}
    for r in res:
        statuses[str(r.status)] = statuses.get(str(r.status), 0) + 1
    out = {
        "metric": "served learn jobs/s",
        "value": round(n / wall, 3),
        "unit": "jobs/s",
        "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": round(wall * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": f"served: {n} jobs of the batched mix, Poisson arrivals at {args.rate} jobs/s "
                               f"(seed 1), lanes {lanes}", "lanes": lanes,
                   "admission": "equal slices" if args.slices else "shared budget, regions by estimated footprint",
                   "slice_gb": round(slice_bytes / 2 ** 30, 2) if args.slices else None,
                   "arrival_span_s": round(arrival[-1] / 1e3, 3)},
        "memory": mem,
        "latency_ms_p50": round(float(np.percentile(lat, 50)), 3),
        "latency_ms_p99": round(float(np.percentile(lat, 99)), 3),
        "job_duration_ms_p50": round(float(np.percentile(dur, 50)), 3),
        "job_duration_ms_p99": round(float(np.percentile(dur, 99)), 3),
        "candidates_per_s": round(sum(r.candidates for r in res) / wall, 1),
        "statuses": statuses,
    }
    print(json.dumps(out), flush=True)


def roofline(ltl, results, geom, ucarry, wall_ms=None):
    """Roofline of the level kernels over `results` (HIP-event times summed per kind).

    The unit is the level pipeline (evaluation, write pass, verification, compaction):
    its algorithmic bytes (ltl_level_stats.alg_bytes: one matrix per candidate, written
    if new or compared if not, plus each child matrix once per tile) over its summed
    GPU time, against HBM.  Whole-row levels write in a pass of their own and row-split
    levels in the evaluation, so bytes are not split between kinds.  The evaluation's
    integer work is priced against VALU beside it.

    Time basis: the summed level spans (one event pair per level, first to last kernel)
    when the jobs ran one after another, so no two counted intervals overlap; the wall
    time `wall_ms` of the timed steps when jobs ran concurrently."""
    kinds = ("eval", "verify", "materialize", "compact", "fallback")
    kern_ms = {k: sum(r.kernel_ms[k] for r in results) for k in ltl.KERNEL_KINDS}
    kern_n = {k: sum(r.kernel_launches[k] for r in results) for k in ltl.KERNEL_KINDS}
    halves, k, cm_bytes = geom["halves"], geom["k"], geom["cm_bytes"]
    ops_total = 0.0
    bytes_level = 0.0
    bytes_verify = 0.0
    for r in results:
        E = r.level_new
        for c in range(1, r.levels_done + 1):
            C = r.level_candidates[c]
            if C == 0:
                continue
            if c == 1:
                ops_total += C * halves * (OP_OPS["atom"] + FP_SEP_OPS)
            else:
                x = c - 1
                un = E[x] if x >= 1 else 0
                u_pairs = sum(E[a] * E[x - a] for a in range(1, x))
                ao = 0
                for a in range(1, x // 2 + 1):
                    b = x - a
                    ao += E[a] * E[b] if a < b else E[a] * (E[a] - 1) // 2
                uop = 5 if ucarry else 5 * k - 2
                per_level_ops = un * (OP_OPS["f"] + OP_OPS["g"] + OP_OPS["x"] + OP_OPS["not"] + 4 * FP_SEP_OPS) \
                    + u_pairs * (uop + FP_SEP_OPS) + ao * (OP_OPS["and"] + OP_OPS["or"] + 2 * FP_SEP_OPS)
                ops_total += per_level_ops * halves
            bytes_level += r.level_bytes[c]
            bytes_verify += (C - r.level_new[c]) * cm_bytes
    level_ms = sum(sum(r.level_ms) for r in results)      # GPU time of the levels (either timing mode)
    summed_level_ms = level_ms
    if wall_ms is not None:
        level_ms = wall_ms
    launches = sum(kern_n[q] for q in kinds)
    eval_ms, verify_ms = kern_ms["eval"], kern_ms["verify"]
    eval_tops = ops_total / (eval_ms * 1e-3) / 1e12 if eval_ms else 0.0
    verify_gbs = bytes_verify / (verify_ms * 1e-3) / 1e9 if verify_ms else 0.0
    level_gbs = bytes_level / (level_ms * 1e-3) / 1e9 if level_ms else 0.0
    roof = {"bound": "hbm", "kernel": "level kernels (k_level, k_level_wg, k_level_all, write pass, compaction)",
            "achieved": round(level_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(level_gbs / HBM_PEAK_GBS, 4), "algorithmic_bytes": bytes_level,
            "kind": "level", "avg_launch_ms": round(level_ms / max(1, launches), 4), "launches": launches,
            "algorithmic_MB_per_launch": round(bytes_level / max(1, launches) / 1e6, 3),
            "time_basis": "summed level spans (jobs one after another)" if wall_ms is None
            else "wall time of the timed steps (jobs overlap)",
            "time_ms": round(level_ms, 3), "summed_level_ms": round(summed_level_ms, 3)}
    if eval_ms:        # per-kind times (LTL_CTX_TIMING)
        roof["valu_view"] = {"kernel": "evaluation", "achieved_Tops": round(eval_tops, 3),
                             "peak_Tops": round(VALU_PEAK_TOPS, 2), "frac": round(eval_tops / VALU_PEAK_TOPS, 4)}
        roof["verify_view"] = {"achieved_GBps": round(verify_gbs, 1), "frac": round(verify_gbs / HBM_PEAK_GBS, 4)}
    return roof, kern_ms, eval_tops, verify_gbs


def copy_ceiling(torch, mib: int = 1024) -> float:
    """Device-to-device copy rate (bytes read + written per second, GB/s): the measured
    ceiling of a kernel that only streams HBM."""
    n = mib << 20
    src = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(1)
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 5
    del src, dst
    return 2.0 * n / (ms * 1e-3) / 1e9


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


CPU_SAMPLE_S = 20.0   # oracle jobs are added to the sample until this much time has gone by


def oracle_rate(insts, levels, threads, ops=None):
    """Candidates and seconds of the oracle over levels 1..`levels` of the jobs in order, the
    first job always and further ones while the elapsed time is below CPU_SAMPLE_S."""
    from oracle import oracle as O
    t0 = time.perf_counter()
    cands = jobs = 0
    for inst in insts:
        r = O.learn(inst, levels, op_mask=O.ALL_OPS if ops is None else ops, mode=O.MODE_EXPAND, threads=threads)
        cands += sum(r.level_candidates[:r.levels_done + 1])
        jobs += 1
        dt = time.perf_counter() - t0
        print(f"cpu oracle ({threads} threads, levels 1..{levels}): job {jobs} done, {dt:.1f} s",
              file=sys.stderr, flush=True)
        if dt > CPU_SAMPLE_S:
            break
    return cands, time.perf_counter() - t0, jobs


def cpu_baseline(insts, levels, ops=None):
    """The CPU oracle, unchanged, on a bounded sample: the first `levels` cost levels of the
    jobs (as many as fit in about CPU_SAMPLE_S) on up to 16 host threads, and a smaller sample
    on one thread."""
    threads = min(16, os.cpu_count() or 1)
    cands, dt, jobs = oracle_rate(insts, levels, threads, ops)
    l1 = max(1, levels - 2)
    c1, d1, jobs1 = oracle_rate(insts, l1, 1, ops)
    return {"value": round(cands / dt, 1), "unit": "candidates/s", "cores": threads, "kind": "oracle",
            "sample": f"levels 1..{levels} of {jobs} of the {len(insts)} jobs ({cands} candidates, {dt:.1f} s)",
            "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "single_thread": {"value": round(c1 / d1, 1), "unit": "candidates/s",
                              "sample": f"levels 1..{l1} of {jobs1} of the jobs ({c1} candidates, {d1:.1f} s)"}}


if __name__ == "__main__":
    main()
