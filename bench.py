#!/usr/bin/env python3
"""Throughput of the DysonNet local estimator on one MI355X: E_loc samples per second with
log-ratios by ABACUS, next to full re-evaluation on the same GPU.

A step is one pass of the whole hot path over one batch of synthetic samples already
resident in HBM: connected elements of H, log psi, every log-ratio, E_loc. Parameter-only
work (S4 taps and tables) happens once per parameter update and is reported separately.
The default workload is the long-range Ising chain with N=256, four blocks, d=64, state 32,
2048 samples, FP32 (alpha=2, h=0.5). One JSON line is printed.

With --workload ragged32 it measures the ragged batch instead: 32 instances of different
chain lengths, depths and batch sizes (one model each) submitted together as one recorded
HIP graph; a step is one pass over all 37011 samples. --workload ragged64_small does the same
for 64 small instances (N <= 128, one or two blocks, d of 16 or 32, at most 256 samples each),
where the host work of per-instance calls matters.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import dataclasses
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp32": 157.3, "fp64": 78.6, "bf16": 2500.0}  # dense MFMA TFLOP/s of one MI355X
HBM_PEAK = 8000.0                      # GB/s


def mfma_peak(kind: str, prec: str, products: str, d: int):
    """(peak TFLOP/s, basis) for the algorithmic (float) flops of a kernel class. With
    three-term splits every float product costs six bf16 products, so the float-equivalent
    peak is the bf16 dense peak / 6; BF16-mixed models split into hi + lo terms (three bf16
    products per product: the bf16 dense peak / 3)."""
    split = products == "split3" and prec != "fp64"
    two = prec == "bf16"
    if kind == "conv" and split:
        return ((PEAK["bf16"] / 3, "bf16 dense peak / 3 (hi + lo split products)") if two else
                (PEAK["bf16"] / 6, "bf16 dense peak / 6 (three-term split products)"))
    if kind == "mix_deep" and two and d > 16:
        return PEAK["bf16"] / 3, "bf16 dense peak / 3 (hi + lo split products)"
    if kind == "mix_deep" and split and d > 16:
        return PEAK["bf16"] / 6, "bf16 dense peak / 6 (three-term split products)"
    return PEAK[prec if prec != "bf16" else "fp32"], ("fp64" if prec == "fp64" else "fp32") + " dense peak"


def products_label(prec: str, products: str, d: int) -> str:
    """What the matrix cores compute in this run: the product mode selects the Toeplitz
    products; channel mixing follows it for float models with d > 16, is on bf16-rounded
    operands for BF16-mixed ones (d > 16), and on the float matrix cores otherwise."""
    if prec == "fp64":
        return "f64 matrix cores"
    split = "three-term bf16 splits (six partial products, f32 accumulate: f32 error bound)"
    hilo = "hi + lo bf16 splits (three partial products, f32 accumulate: 16-bit operands)"
    toeplitz = (hilo if prec == "bf16" else split) if products == "split3" else "f32 matrix cores"
    if prec == "bf16" and d > 16:
        mix = hilo
    elif products == "split3" and d > 16:
        mix = split
    else:
        mix = "f32 matrix cores"
    return f"Toeplitz products: {toeplitz}; channel mixing: {mix}"


def source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2603_11189_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_class(name: str) -> str:
    """Map a demangled kernel name to the library's profile class."""
    if "mix_kernel" in name:
        mode = name.split("mix_kernel<")[1].split(",")[2].strip()
        return {"0": "mix_fwd", "1": "mix_tau", "2": "mix_deep"}[mode]
    for key, cls in (("conv_kernel", "conv"), ("conv_split_kernel", "conv"), ("phi_kernel", "phi"), ("slice_mma_kernel", "slice"),
                     ("deep_kernel", "mix_deep"), ("last_finish_kernel", "tail"), ("shallow_kernel", "tail"),
                     ("inject_w1_kernel", "conv"), ("inject_add_kernel", "mix_deep"),
                     ("lam_fwd_kernel", "link"), ("lam_gemm_kernel", "link"), ("lam_inv_kernel", "link"),
                     ("lam_param_kernel", "prep"), ("s4_taps_kernel", "s4gen"), ("prep_kernel", "prep"),
                     ("connected_kernel", "gen"), ("eloc_kernel", "eloc")):
        if key in name:
            return cls
    return "other"


def _db(d: str):
    """The rocprofv3 database (rocpd, SQLite) in directory d, or None."""
    import glob
    import sqlite3
    dbs = sorted(glob.glob(os.path.join(d, "*.db")))
    return sqlite3.connect(dbs[0]) if dbs else None


def _kernel_stats(d: str):
    """Per-kernel calls and durations of a rocprofv3 run: the CSV summary or the database."""
    import csv
    con = _db(d)
    if con is None:
        return list(csv.DictReader(open(os.path.join(d, "kt_kernel_stats.csv"))))
    out = []
    for name, n, tot in con.execute("select name, count(*), sum(duration) from kernels group by name"):
        out.append({"Name": name, "Calls": n, "TotalDurationNs": tot, "AverageNs": tot / n})
    return out


def _pmc_rows(d: str):
    """(kernel name, counter, value) per dispatch of a rocprofv3 --pmc run."""
    import csv
    con = _db(d)
    if con is None:
        return list(csv.DictReader(open(os.path.join(d, "pmc_counter_collection.csv"))))
    return [{"Kernel_Name": k, "Counter_Name": c, "Counter_Value": v}
            for k, c, v in con.execute("select kernel_name, counter_name, value from counters_collection")]


def summarize(args) -> None:
    """Turn raw rocprofv3 output directories into the short summaries kept in profiles/."""
    import collections
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    wl = args.workload
    if args.stats_dir:
        rows = _kernel_stats(args.stats_dir)
        total = sum(float(r["TotalDurationNs"]) for r in rows)
        out = [f"# Kernel time, {wl}, {args.stats_path} path\n",
               f"Command: `{args.stats_cmd}`\n",
               f"Source hash of csrc/: `{source_hash()}`\n",
               "| kernel | class | calls | total ms | avg us | share |", "|---|---|---|---|---|---|"]
        for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"]))[:14]:
            out.append(f"| `{r['Name'][:80]}` | {kernel_class(r['Name'])} | {r['Calls']} | "
                       f"{float(r['TotalDurationNs']) / 1e6:.2f} | {float(r['AverageNs']) / 1e3:.1f} | "
                       f"{100 * float(r['TotalDurationNs']) / total:.1f}% |")
        cls = collections.defaultdict(lambda: [0.0, 0])
        for r in rows:
            c = cls[kernel_class(r["Name"])]
            c[0] += float(r["TotalDurationNs"])
            c[1] += int(r["Calls"])
        out += ["", "Per class (the grouping `bench.py` uses for its roofline):", "",
                "| class | calls | avg us per launch |", "|---|---|---|"]
        for k, (ns, n) in sorted(cls.items(), key=lambda kv: -kv[1][0]):
            out.append(f"| {k} | {n} | {ns / n / 1e3:.1f} |")
        sfx = "" if args.stats_path == "ABACUS" else "_" + args.stats_path.lower().replace(" ", "_")
        with open(os.path.join(ROOT, "profiles", f"kernel_stats_{wl}{sfx}.md"), "w") as f:
            f.write("\n".join(out) + "\n")
    if args.util_dirs:
        # matrix-core and vector-ALU busy percentages (rocprofv3's derived MfmaUtil and VALUBusy)
        # per kernel class, averaged over the class's dispatches
        per = collections.defaultdict(lambda: collections.defaultdict(list))
        for d in args.util_dirs.split(","):
            for r in _pmc_rows(d):
                per[kernel_class(r["Kernel_Name"])][r["Counter_Name"]].append(float(r["Counter_Value"]))
        res = {"source_hash": source_hash(), "command": args.util_cmd, wl: {}}
        md = [f"# Matrix-core and vector-ALU busy, {wl}, ABACUS path\n", f"Command: `{args.util_cmd}`\n",
              f"Source hash of csrc/: `{source_hash()}`\n",
              "MfmaUtil = 100 * sum SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE * SIMDs); "
              "VALUBusy = 100 * sum SQ_ACTIVE_INST_VALU / CUs / GRBM_GUI_ACTIVE (rocprofv3's definitions).\n",
              "| class | dispatches | MfmaUtil % | VALUBusy % |", "|---|---|---|---|"]
        for k, v in sorted(per.items()):
            if "MfmaUtil" in v and "VALUBusy" in v:
                mu = sum(v["MfmaUtil"]) / len(v["MfmaUtil"])
                vb = sum(v["VALUBusy"]) / len(v["VALUBusy"])
                res[wl][k] = {"mfma_util_pct": mu, "valu_busy_pct": vb, "dispatches": len(v["MfmaUtil"])}
                md.append(f"| {k} | {len(v['MfmaUtil'])} | {mu:.1f} | {vb:.1f} |")
        path = os.path.join(ROOT, "profiles", "counters.json")
        old = json.load(open(path)) if os.path.exists(path) else {}
        if old.get("source_hash") == res["source_hash"]:
            old.update(res)
            res = old
        with open(path, "w") as f:
            json.dump(res, f, indent=1)
        with open(os.path.join(ROOT, "profiles", f"util_{wl}.md"), "w") as f:
            f.write("\n".join(md) + "\n")
    if args.pmc_dirs:
        per = {}
        for d in args.pmc_dirs.split(","):
            rows = _pmc_rows(d)
            for r in rows:
                per.setdefault(r["Counter_Name"], []).append(r)
        calib = {}
        for ctr, rows in per.items():
            big = max((r for r in rows if "copyBuffer" in r["Kernel_Name"]), key=lambda r: float(r["Counter_Value"]))
            calib[ctr] = (256 << 20) / (float(big["Counter_Value"]) * 1024)
        agg = collections.defaultdict(lambda: collections.defaultdict(list))
        for ctr, rows in per.items():
            for r in rows:
                agg[kernel_class(r["Kernel_Name"])][ctr].append(float(r["Counter_Value"]) * 1024 * calib[ctr])
        res = {"source_hash": source_hash(), "command": args.pmc_cmd,
               "calibration": {k: f"x{v:.3f} (256 MiB device copy)" for k, v in calib.items()}, wl: {}}
        md = [f"# HBM traffic per launch, {wl}, ABACUS path\n", f"Command (one run per counter): `{args.pmc_cmd}`\n",
              "Scale factors from a 256 MiB device copy in the same process: " +
              ", ".join(f"{k} x{v:.3f}" for k, v in calib.items()) + "\n",
              "| class | launches | fetch MB/launch | write MB/launch | total MB/launch |", "|---|---|---|---|---|"]
        for k, v in agg.items():
            if "FETCH_SIZE" in v and "WRITE_SIZE" in v:
                fe = sum(v["FETCH_SIZE"]) / len(v["FETCH_SIZE"])
                wr = sum(v["WRITE_SIZE"]) / len(v["WRITE_SIZE"])
                res[wl][k] = {"fetch_bytes_per_launch": fe, "write_bytes_per_launch": wr, "bytes_per_launch": fe + wr,
                              "launches": len(v["FETCH_SIZE"])}
                md.append(f"| {k} | {len(v['FETCH_SIZE'])} | {fe / 1e6:.1f} | {wr / 1e6:.1f} | {(fe + wr) / 1e6:.1f} |")
        path = os.path.join(ROOT, "profiles", "traffic.json")
        old = json.load(open(path)) if os.path.exists(path) else {}
        if old.get("source_hash") == res["source_hash"]:  # other workloads of the same sources
            old.update(res)
            res = old
        with open(path, "w") as f:
            json.dump(res, f, indent=1)
        with open(os.path.join(ROOT, "profiles", f"traffic_{wl}.md"), "w") as f:
            f.write("\n".join(md) + "\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="tfim_n256_l4_d64")
    ap.add_argument("--scale", default="baseline", choices=["baseline", "stress"])
    ap.add_argument("--prec", default="", choices=["", "fp64", "fp32", "bf16"],
                    help="arithmetic mode (default: the workload's own)")
    ap.add_argument("--paths", default="abacus,full")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--no-grad", action="store_true", help="skip the per-sample log-derivative leg")
    ap.add_argument("--no-tune", action="store_true", help="no autotuner in the sweep and the ragged batch")
    ap.add_argument("--tune", action="store_true",
                    help="autotune the launch shapes of the measured model first (default: the library's "
                         "default shapes, so that repeated runs and their profiles use the same launches)")
    ap.add_argument("--shapes", default="", help="CONV_NT,FLIP_MIB: set launch shapes instead of tuning")
    ap.add_argument("--flip-mib", type=int, default=16384,
                    help="without --shapes or --tune: HBM budget of the per-flip fields of one chunk (MiB)")
    ap.add_argument("--products", default="split3", choices=["split3", "fp32"],
                    help="float matrix-core products: three-term bf16 splits (default) or float32 matrix cores")
    ap.add_argument("--sampler", action="store_true",
                    help="screened typewriter sampler: Metropolis proposals per second on the workload")
    ap.add_argument("--eps-adaptive", action="store_true",
                    help="with --sampler: the tolerance buffer eps(n) instead of a fixed eps")
    ap.add_argument("--sr", action="store_true",
                    help="stochastic-reconfiguration update from the workload's per-sample log-derivatives")
    ap.add_argument("--sweep", action="store_true",
                    help="ABACUS vs full re-evaluation for N in 64..512 at L = 2 and 4 (one JSON line each)")
    ap.add_argument("--inject", action="store_true",
                    help="the workload's network with phi injected into the h stream (Fig. 1c block)")
    ap.add_argument("--paper-shapes", action="store_true",
                    help="with --sweep: the paper's matched runtime shapes instead (L=2, d=2, s=12, periodic, "
                         "Kac-normalised Ising J=-5, alpha=6, 1024 samples; N up to the library's 512)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run one plain device copy of 256 MiB (reference for HBM counters)")
    ap.add_argument("--summarize", action="store_true", help="write profiles/ summaries from raw rocprofv3 CSVs")
    ap.add_argument("--stats-dir", default="")
    ap.add_argument("--stats-cmd", default="")
    ap.add_argument("--stats-path", default="ABACUS", help="the estimator path the stats run timed")
    ap.add_argument("--pmc-dirs", default="")
    ap.add_argument("--pmc-cmd", default="")
    ap.add_argument("--util-dirs", default="", help="rocprofv3 --pmc MfmaUtil VALUBusy output directories")
    ap.add_argument("--util-cmd", default="")
    args = ap.parse_args()
    if args.summarize:
        summarize(args)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (the estimator would shard "
              "by sample). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import dn_inputs as di
    from paper_2603_11189_amd import _lib as L

    if args.workload in ("ragged32", "ragged64_small"):
        bench_ragged(args)
        return
    if args.sweep:
        bench_sweep(args)
        return
    if args.sampler:
        bench_sampler(args)
        return
    if args.sr:
        bench_sr(args)
        return
    w = di.WORKLOADS[args.workload]
    shape, ham = w.model, w.ham
    if args.inject:  # same parameter layout, phi added to each mixer input
        shape = dataclasses.replace(shape, inject_phi=1)
    Np = (shape.N + 63) // 64 * 64  # the library's padded chain length
    prec = args.prec or w.prec
    B = w.B
    M_max = shape.N if ham.kind == "lrtfim" else 2 * shape.N
    theta = torch.tensor(w.params(args.scale))
    spins_np = w.spin_batch()
    dev = torch.device("cuda")
    torch.cuda.init()
    L.lib()
    model = L.Model(shape, prec)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    model.set_params(theta)
    torch.cuda.synchronize()
    set_params_ms = (time.perf_counter() - t0) * 1e3
    spins = torch.tensor(spins_np, device=dev)
    bufs = {p: (torch.empty(B, dtype=torch.float64, device=dev),
                torch.empty((B, M_max), dtype=torch.float64, device=dev),
                torch.empty(B, dtype=torch.float64, device=dev)) for p in ("abacus", "full")}
    if args.copy_calib:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)  # 256 MiB
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    model.set_product_mode(args.products)
    tuned = None
    if args.shapes:
        nt, mib = (int(x) for x in args.shapes.split(","))
        model.set_launch_shapes(nt, mib << 20)
        tuned = {"conv_tiles_per_wave": nt, "flip_chunk_MiB": mib, "set_by": "--shapes"}
    elif args.tune and not args.no_tune:
        t0 = time.perf_counter()
        nt, bud = model.autotune(ham)
        tuned = {"conv_tiles_per_wave": nt, "flip_chunk_MiB": bud >> 20,
                 "tuning_s": round(time.perf_counter() - t0, 3)}
        log(f"[bench] autotuned launch shapes: {tuned}")
    else:
        # one model holds the GPU: its flip fields may take a larger share of HBM than the
        # library's default (sized for many models side by side)
        model.set_launch_shapes(0, args.flip_mib << 20)
        tuned = {"flip_chunk_MiB": args.flip_mib, "set_by": "--flip-mib"}
    results = {}
    for path in args.paths.split(","):
        log(f"[bench] {args.workload} path={path} warmup={args.warmup}")
        for _ in range(args.warmup):
            model.eloc(ham, spins, M_max, path=path, out=bufs[path])
        torch.cuda.synchronize()
        if not args.no_profile:
            model.profile_enable(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            model.eloc(ham, spins, M_max, path=path, out=bufs[path])
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        prof = model.profile_read() if not args.no_profile else {}
        model.profile_enable(False)
        results[path] = {"sec": el, "prof": prof}
        log(f"[bench] {path}: {el / args.steps * 1e3:.2f} ms/step, {B * args.steps / el:.1f} samples/s")

    grad = None
    if not args.no_grad and shape.bc == "open":
        # per-sample log-derivatives of the same batch (the consumer of E_loc in a VMC step)
        log(f"[bench] {args.workload} per-sample gradients")
        for _ in range(max(1, args.warmup)):
            model.grad_logpsi(spins)
        torch.cuda.synchronize()
        g_steps = max(1, min(args.steps, 5))
        t0 = time.perf_counter()
        for _ in range(g_steps):
            _, g, _ = model.grad_logpsi(spins)
            del g
        torch.cuda.synchronize()
        gsec = (time.perf_counter() - t0) / g_steps
        grad = {"ms_per_step": gsec * 1e3, "samples_per_s": B / gsec, "steps": g_steps,
                "params_per_sample": L.param_count(shape), "dtype": "f32" if prec == "fp32" else "f64"}
        log(f"[bench] gradients: {gsec * 1e3:.2f} ms/step")

    main_path = "abacus" if "abacus" in results else list(results)[0]
    el = results[main_path]["sec"]
    value = B * args.steps / el
    out = {
        "metric": "E_loc samples/sec, ABACUS vs full re-eval, N=256, at stated rel err vs FP64",
        "value": value,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp64": "f64", "bf16": "bf16-mixed (hi + lo bf16 operands, f32 accumulate)"}[prec],
        "data": "synthetic",
        "config": {"workload": args.workload + ("_inject_phi" if args.inject else ""), "N": shape.N, "L": shape.L,
                   "d": shape.d, "s": shape.s,
                   "B": B, "hamiltonian": f"{ham.kind} {ham.bc} J={ham.J} alpha={ham.alpha} h={ham.h}"
                   if ham.kind == "lrtfim" else f"j1j2 {ham.bc} J1={ham.J1} J2={ham.J2}",
                   "params": f"N(0,0.1^2) seed {w.param_seed}" if args.scale == "baseline" else "stress draw",
                   "path": main_path},
        "set_params_ms": set_params_ms,
        "launch_shapes": tuned or {"conv_tiles_per_wave": 4 if Np >= 256 else Np // 64, "flip_chunk_MiB": 3072,
                                   "set_by": "library defaults"},
        "products": products_label(prec, args.products, shape.d),
    }
    if grad:
        out["grad_logpsi"] = grad
        out["eloc_plus_grad_samples_per_s"] = B / (el / args.steps + grad["ms_per_step"] * 1e-3)
    if "full" in results and main_path != "full":
        fv = B * args.steps / results["full"]["sec"]
        out["full_reeval"] = {"value": fv, "ms_per_step": results["full"]["sec"] / args.steps * 1e3}
        out["speedup_vs_full"] = value / fv

    # roofline of the dominant kernel of the timed path, from the library's event profile
    prof = results[main_path]["prof"]
    if prof:
        per = {}
        for kind, (ms, n, fl, by) in prof.items():
            if n:
                per[kind] = {"ms_per_step": ms / args.steps, "launches_per_step": n / args.steps,
                             "tflops": fl / (ms * 1e-3) / 1e12 if ms > 0 else None,
                             "gbps": by / (ms * 1e-3) / 1e9 if ms > 0 else None}
        out["per_kernel"] = per
        dom = max(prof, key=lambda k: prof[k][0])
        ms, n, fl, by = prof[dom]
        achieved = fl / (ms * 1e-3) / 1e12
        peak, basis = mfma_peak(dom, prec, args.products, shape.d)
        traffic = None
        tpath = os.path.join(ROOT, "profiles", "traffic.json")
        if os.path.exists(tpath):
            with open(tpath) as f:
                tj = json.load(f)
            ent = tj.get(args.workload, {}).get(dom)
            if ent and tj.get("source_hash") == source_hash():
                traffic = ent["bytes_per_launch"]
        # the binding unit from the committed counters of the same sources (matrix-core busy,
        # vector-ALU busy, HBM bandwidth of the measured traffic), when they are there
        bound, util = "mfma", None
        cpath = os.path.join(ROOT, "profiles", "counters.json")
        if os.path.exists(cpath):
            with open(cpath) as f:
                cj = json.load(f)
            ent = cj.get(args.workload, {}).get(dom)
            if ent and cj.get("source_hash") == source_hash():
                hbm_pct = 100.0 * traffic / (ms / n * 1e-3) / (HBM_PEAK * 1e9) if traffic else 0.0
                util = {"mfma_util_pct": ent["mfma_util_pct"], "valu_busy_pct": ent["valu_busy_pct"],
                        "hbm_pct": hbm_pct, "source": "profiles/counters.json"}
                score = {"mfma": ent["mfma_util_pct"], "alu": ent["valu_busy_pct"], "hbm": hbm_pct}
                bound = max(score, key=score.get)
        out["roofline"] = {"bound": bound, "kernel": dom, "achieved": achieved, "peak": peak,
                           "unit": "TFLOP/s", "frac": achieved / peak, "traffic": traffic,
                           "peak_basis": basis, "avg_launch_ms": ms / n,
                           "algorithmic_flops_per_launch": fl / n, "algorithmic_bytes_per_launch": by / n,
                           "counters": util}

    # error of both GPU paths against the float64 oracle at the stress draw (every block
    # carries order-one signal there; at the baseline draw the network is nearly linear)
    if not args.no_cpu_baseline:
        out["err_stress_draw"] = stress_errors(args, w, shape, ham, prec, M_max, list(results))

    # CPU baseline (the oracle, untuned) on a bounded sample, and the error of both GPU paths
    if not args.no_cpu_baseline:
        import oracle as O
        from oracle.model import ModelDesc
        desc = ModelDesc.of(shape)
        gpu = {p: tuple(t.cpu() for t in bufs[p]) for p in results}
        budget = args.cpu_seconds
        t0 = time.perf_counter()
        done, errs = [], {p: {"eloc": 0.0, "lr": 0.0, "logpsi": 0.0} for p in results}
        ref_mag = {"eloc": 0.0, "lr": 0.0, "logpsi": 0.0}
        stride = max(1, B // 64)
        while time.perf_counter() - t0 < budget and len(done) * stride < B:
            b = len(done) * stride
            ref = O.eloc_plain(desc, ham, theta, spins_np[b:b + 1], M_max)
            done.append(b)
            for key, idx in (("logpsi", 0), ("lr", 1), ("eloc", 2)):
                r = {"logpsi": ref["logpsi"], "lr": ref["logratio"], "eloc": ref["eloc"]}[key]
                ref_mag[key] = max(ref_mag[key], r.abs().max().item())
                for p in results:
                    g = gpu[p][idx][b:b + 1]
                    errs[p][key] = max(errs[p][key], (g - r).abs().max().item())
        cpu_sec = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": len(done) / cpu_sec, "unit": "samples/s",
                               "cores": torch.get_num_threads(), "kind": "oracle",
                               "sample": f"{len(done)} of the {B} samples (every {stride}th), "
                                         f"float64 oracle, log-ratios by full re-evaluation, {cpu_sec:.1f} s"}
        # the same oracle on one thread (a bounded prefix of the same samples)
        nthr = torch.get_num_threads()
        torch.set_num_threads(1)
        t0, n1 = time.perf_counter(), 0
        while time.perf_counter() - t0 < args.cpu_seconds / 2 and n1 * stride < B:
            O.eloc_plain(desc, ham, theta, spins_np[n1 * stride:n1 * stride + 1], M_max)
            n1 += 1
        sec1 = time.perf_counter() - t0
        torch.set_num_threads(nthr)
        out["cpu_baseline"]["single_thread"] = {"value": n1 / sec1, "unit": "samples/s", "cores": 1,
                                                "sample": f"{n1} samples, {sec1:.1f} s"}
        out["err_vs_fp64_oracle"] = {
            p: {k: (errs[p][k] / ref_mag[k] if ref_mag[k] > 0 else 0.0) for k in errs[p]} for p in results}
        out["err_vs_fp64_oracle"]["measure"] = "max|x - x*| / max|x*| over the CPU sample (baseline draw)"
    print(json.dumps(out), flush=True)


def stress_errors(args, w, shape, ham, prec, M_max, paths, B_s: int = 8) -> dict:
    """Errors of both GPU paths against the float64 oracle on B_s samples of the workload at the
    stress draw: eps_lr = max|lr - lr*| / max|lr*|, eps_logpsi likewise, eps_E = max|E - E*| /
    max|E*|, and eps_E,net = max|E - E*| / max|E* - E*_(psi=1)| (relative to the network-dependent
    part of E_loc; E*_(psi=1) = hdiag + sum_m helem_m)."""
    import torch

    import oracle as O
    from oracle.model import ModelDesc
    from paper_2603_11189_amd import _lib as L

    theta = torch.tensor(w.params("stress"))
    sp = w.spin_batch(B_s)
    m = L.Model(shape, prec)
    m.set_params(theta)
    m.set_product_mode(args.products)
    ref = O.eloc_plain(ModelDesc.of(shape), ham, theta, sp, M_max)
    net = (ref["eloc"] - ref["hdiag"] - ref["helem"].sum(-1)).abs().max().item()
    spd = torch.tensor(sp, device="cuda")
    res = {"samples": B_s, "draw": "stress (order-one signal in every block)"}
    for p in paths:
        lp, lr, el = (t.cpu() for t in m.eloc(ham, spd, M_max, path=p))
        d_el = (el - ref["eloc"]).abs().max().item()
        res[p] = {"lr": (lr - ref["logratio"]).abs().max().item() / ref["logratio"].abs().max().item(),
                  "logpsi": (lp - ref["logpsi"]).abs().max().item() / ref["logpsi"].abs().max().item(),
                  "eloc": d_el / ref["eloc"].abs().max().item(), "eloc_net": d_el / net}
    m.close()
    return res


def _profiled(model, fn, steps):
    """Per-class (ms, launches, flops, bytes) of `steps` calls of fn, from the library's events."""
    import torch
    model.profile_enable(True)
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    prof = model.profile_read()
    model.profile_enable(False)
    return prof


def bench_sampler(args) -> None:
    """Screened typewriter sampler (dn_screened_sweep) on the workload's model at the stress draw
    (order-one signal in every block, so that proposals are rejected and the screen refreshes):
    B chains, blocks of 8 sites, one proposal per visited block, eps = 0.01; a step is one sweep
    (both parities). With --eps-adaptive the tolerance is the buffer eps(n) (16 entries, default
    0.2, gamma 1.5), calibrated during the warmup sweeps (the burn-in) and kept updating while
    timed."""
    import numpy as np
    import torch

    import dn_inputs as di
    from paper_2603_11189_amd import _lib as L

    w = di.WORKLOADS[args.workload]
    shape = w.model
    if args.inject:  # same parameter layout, phi added to each mixer input
        shape = dataclasses.replace(shape, inject_phi=1)
    prec = args.prec or w.prec
    spacing, eps = 8, 0.01
    dev = torch.device("cuda")
    torch.cuda.init()
    L.lib()
    m = L.Model(shape, prec)
    m.set_params(torch.tensor(w.params("stress")))
    spins = torch.tensor(w.spin_batch(), device=dev)
    B, N = spins.shape
    nblk = (N + spacing - 1) // spacing
    K = [((nblk - par) + 1) // 2 for par in (0, 1)]
    rng = np.random.Generator(np.random.PCG64(w.spin_seed + 77))
    draws = [[(torch.tensor(rng.random((B, K[par])), device=dev), torch.tensor(rng.random((B, K[par])), device=dev))
              for par in (0, 1)] for _ in range(4)]
    acc_n, ref_n = [0], [0]
    ebuf = torch.full((16,), 0.2, dtype=torch.float64, device=dev)
    eset = torch.zeros(16, dtype=torch.int32, device=dev)

    def sweep(i):
        for par in (0, 1):
            r, u = draws[i % 4][par]
            if args.eps_adaptive:
                a, rf = m.screened_sweep_adaptive(spins, spacing, par, r, u, ebuf, eset, 1.5)
            else:
                a, rf = m.screened_sweep(spins, spacing, par, r, u, eps)
            acc_n[0] += a
            ref_n[0] += rf

    for i in range(args.warmup):
        sweep(i)
    torch.cuda.synchronize()
    acc_n[0], ref_n[0] = 0, 0
    t0 = time.perf_counter()
    for i in range(args.steps):
        sweep(i)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / args.steps
    props = B * (K[0] + K[1])
    acc_tot = int(acc_n[0].sum().item()) if torch.is_tensor(acc_n[0]) else 0
    ref_tot = int(ref_n[0].sum().item()) if torch.is_tensor(ref_n[0]) else 0
    prof = _profiled(m, lambda: sweep(0), 1)
    dom = max(prof, key=lambda k: prof[k][0])
    ms, n, fl, by = prof[dom]
    peak, basis = mfma_peak(dom, prec, "split3", shape.d)
    out = {
        "metric": "Metropolis proposals/sec, screened typewriter sampler (ISA ratios by ABACUS)",
        "value": props / sec, "unit": "proposals/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": sec * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16": "bf16-mixed"}[prec], "data": "synthetic",
        "config": {"workload": args.workload + ("_inject_phi" if args.inject else "") + "_sampler", "N": N,
                   "L": shape.L, "d": shape.d, "chains": B,
                   "spacing": spacing, "eps": "adaptive eps(n), default 0.2, gamma 1.5" if args.eps_adaptive else eps,
                   "params": "stress draw", "step": "one sweep (both parities)"},
        "acceptance": acc_tot / (props * args.steps), "refreshes_per_proposal": ref_tot / (props * args.steps),
        "roofline": {"kernel": dom, "achieved": fl / (ms * 1e-3) / 1e12, "peak": peak, "unit": "TFLOP/s",
                     "frac": fl / (ms * 1e-3) / 1e12 / peak, "peak_basis": basis, "avg_launch_ms": ms / n},
        "per_kernel": {k: {"ms_per_step": v[0], "launches_per_step": v[1]} for k, v in prof.items() if v[1]},
    }
    print(json.dumps(out), flush=True)


def bench_sr(args) -> None:
    """One stochastic-reconfiguration update (dn_sr_update) from the workload's per-sample
    log-derivatives O [B x P] and local energies: conjugate gradients on (S + shift I) x = F, two
    passes over O per iteration; the roofline is HBM (O read twice per iteration)."""
    import torch

    import dn_inputs as di
    from paper_2603_11189_amd import _lib as L

    w = di.WORKLOADS[args.workload]
    shape, ham = w.model, w.ham
    prec = args.prec or w.prec
    dev = torch.device("cuda")
    torch.cuda.init()
    L.lib()
    m = L.Model(shape, prec)
    m.set_params(torch.tensor(w.params(args.scale)))
    spins = torch.tensor(w.spin_batch(), device=dev)
    M_max = shape.N if ham.kind == "lrtfim" else 2 * shape.N
    _, g, _ = m.grad_logpsi(spins)
    _, _, el = m.eloc(ham, spins, M_max, path="abacus")
    B, P = g.shape
    iters = 50
    for _ in range(args.warmup):
        m.sr_update(g, el, max_iter=iters, tol=0.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, _, it = m.sr_update(g, el, max_iter=iters, tol=0.0)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / args.steps
    passes = 2 * it + 2  # F and Obar, then a row and a column pass per iteration
    gbs = passes * g.numel() * g.element_size() / sec / 1e9
    out = {
        "metric": "SR updates/sec (conjugate gradients, fixed iteration count)",
        "value": 1.0 / sec, "unit": "updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": sec * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16": "f32"}[prec], "data": "synthetic",
        "config": {"workload": args.workload + "_sr", "samples": B, "params": P, "cg_iterations": it,
                   "O_bytes": g.numel() * g.element_size()},
        "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK, "unit": "GB/s", "frac": gbs / HBM_PEAK,
                     "traffic": None, "basis": f"{passes} passes over O per update"},
    }
    print(json.dumps(out), flush=True)


def bench_sweep(args) -> None:
    """Speedup of ABACUS over full re-evaluation on the same GPU across chain lengths: the
    long-range Ising chain (alpha=2, h=0.5), d=64, state 32, float32, B samples per N; or,
    with --paper-shapes, the paper's matched runtime shapes (L=2, d=2, state 12, token size 2,
    periodic, N = 100 .. 1000 spins). --inject: the same networks with phi injected."""
    import torch

    import dn_inputs as di
    from paper_2603_11189_amd import _lib as L

    dev = torch.device("cuda")
    torch.cuda.init()
    L.lib()
    if args.paper_shapes:
        B = 1024
        ham = di.HamSpec("lrtfim", "periodic", J=-5.0, alpha=6.0, h=1.0, paper_form=1)
        grid = [(di.ModelShape(N // 2, 2, 2, 12, act="silu", bc="periodic", token=2), 2)
                for N in (100, 250, 500, 1000)]
    else:
        B = 512
        ham = di.HamSpec("lrtfim", "open", J=1.0, alpha=2.0, h=0.5)
        grid = [(di.ModelShape(N, depth, 64, 32, act="silu", bc="open"), depth)
                for depth in (2, 4) for N in (64, 128, 256, 512)]
    if args.inject:  # the same networks with phi injected into the h stream
        grid = [(dataclasses.replace(shape, inject_phi=1), depth) for shape, depth in grid]
    for shape, depth in grid:
        N = shape.n_spins  # spins: one connected element per spin
        m = L.Model(shape, "fp32")
        m.set_params(torch.tensor(di.draw_params(shape, 1005, "baseline")))
        spins = torch.tensor(di.uniform_spins(B, N, 2005), device=dev)
        if not args.no_tune:
            m.autotune(ham)
        rate = {}
        for path in ("abacus", "full"):
            out = (torch.empty(B, dtype=torch.float64, device=dev),
                   torch.empty((B, N), dtype=torch.float64, device=dev),
                   torch.empty(B, dtype=torch.float64, device=dev))
            m.eloc(ham, spins, N, path=path, out=out)
            torch.cuda.synchronize()
            steps = 2
            t0 = time.perf_counter()
            for _ in range(steps):
                m.eloc(ham, spins, N, path=path, out=out)
            torch.cuda.synchronize()
            rate[path] = B * steps / (time.perf_counter() - t0)
        m.close()
        line = {"metric": "E_loc samples/sec, ABACUS vs full re-eval (sweep)", "N": N, "L": depth,
                "token": shape.token, "d": shape.d, "s": shape.s, "bc": shape.bc, "B": B, "dtype": "f32",
                "inject_phi": shape.inject_phi,
                "abacus": rate["abacus"],
                "full": rate["full"], "speedup": rate["abacus"] / rate["full"],
                "us_per_element": {p: 1e6 / (rate[p] * N) for p in rate}, "unit": "samples/s",
                "data": "synthetic"}
        log(f"[sweep] N={N} L={depth}: abacus {rate['abacus']:.0f}/s full {rate['full']:.0f}/s "
            f"x{line['speedup']:.2f}")
        print(json.dumps(line), flush=True)


def bench_ragged(args) -> None:
    """The ragged batch: 32 instances in one recorded graph, against per-instance calls."""
    import torch

    import dn_inputs as di
    from paper_2603_11189_amd import _lib as L

    small = args.workload == "ragged64_small"
    ws = di.ragged_small_instances() if small else di.ragged_instances()
    tag = args.workload
    dev = torch.device("cuda")
    torch.cuda.init()
    L.lib()
    models, thetas, spins, lps, els = [], [], [], [], []
    for w in ws:
        th = torch.tensor(w.params(args.scale))
        m = L.Model(w.model, "fp32")
        m.set_params(th)
        models.append(m)
        thetas.append(th)
        spins.append(torch.tensor(w.spin_batch(), device=dev))
        lps.append(torch.empty(w.B, dtype=torch.float64, device=dev))
        els.append(torch.empty(w.B, dtype=torch.float64, device=dev))
    hams = [w.ham for w in ws]
    Btot = sum(w.B for w in ws)

    def timed(fn, steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    graph = lambda: L.ragged_eloc(models, hams, spins, lps, els, n_streams=4, mode="graph")
    log(f"[bench] {tag}: {len(ws)} instances, {Btot} samples; recording + warmup {args.warmup}")
    for _ in range(max(1, args.warmup)):
        graph()
    sec = timed(graph, args.steps)
    log(f"[bench] {tag} graph: {sec * 1e3:.1f} ms/step, {Btot / sec:.1f} samples/s")
    eager = lambda: L.ragged_eloc(models, hams, spins, lps, els, n_streams=4, mode="eager")
    eager()
    sec_eager = timed(eager, max(1, args.steps // 2))
    log(f"[bench] {tag} eager 4 streams: {sec_eager * 1e3:.1f} ms/step")
    bufs = [(lps[i], torch.empty((w.B, w.model.N), dtype=torch.float64, device=dev), els[i])
            for i, w in enumerate(ws)]

    def per_instance():
        for i, w in enumerate(ws):
            models[i].eloc(w.ham, spins[i], w.model.N, path="abacus", out=bufs[i])

    per_instance()
    sec_seq = timed(per_instance, max(1, args.steps // 2))
    log(f"[bench] {tag} per-instance calls: {sec_seq * 1e3:.1f} ms/step")
    out = {
        "metric": f"E_loc samples/sec, ragged batch of {len(ws)} instances, ABACUS",
        "value": Btot / sec, "unit": "samples/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": sec * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": ({"workload": tag, "instances": len(ws), "N": "U{16..128}", "L": "U{1,2}",
                    "B": "U{32..256}", "samples": Btot, "d": "{16,32}", "s": "d/2",
                    "hamiltonian": "lrtfim open J=1 alpha=3 h=1", "submission": "one HIP graph, 4 streams"}
                   if small else
                   {"workload": tag, "instances": len(ws), "N": "U{32..512}", "L": "U{2,3,4}",
                    "B": "U{256..2048}", "samples": Btot, "d": 64, "s": 32,
                    "hamiltonian": "lrtfim open J=1 alpha=3 h=1", "submission": "one HIP graph, 4 streams"}),
        "eager_4_streams": {"ms_per_step": sec_eager * 1e3, "value": Btot / sec_eager},
        "per_instance_calls": {"ms_per_step": sec_seq * 1e3, "value": Btot / sec_seq},
    }
    if not args.no_profile:
        # kernel classes from one eager pass on one stream, bracketed by events per launch
        for m in models:
            m.profile_enable(True)
        L.ragged_eloc(models, hams, spins, lps, els, n_streams=1, mode="eager")
        torch.cuda.synchronize()
        tot = {}
        for m in models:
            for k, (ms, n, fl, by) in m.profile_read().items():
                t = tot.setdefault(k, [0.0, 0, 0.0, 0.0])
                t[0] += ms; t[1] += n; t[2] += fl; t[3] += by
            m.profile_enable(False)
        dom = max(tot, key=lambda k: tot[k][0])
        ms, n, fl, by = tot[dom]
        achieved = fl / (ms * 1e-3) / 1e12
        peak, basis = mfma_peak(dom, "fp32", "split3", max(w.model.d for w in ws))
        out["roofline"] = {"bound": "mfma", "kernel": dom, "achieved": achieved, "peak": peak,
                           "unit": "TFLOP/s", "frac": achieved / peak, "traffic": None, "peak_basis": basis,
                           "avg_launch_ms": ms / n, "algorithmic_flops_per_launch": fl / n,
                           "measured_on": "one eager pass on one stream (graph replays record no events)"}
        out["per_kernel"] = {k: {"ms_per_step": v[0], "launches_per_step": v[1],
                                 "tflops": v[2] / (v[0] * 1e-3) / 1e12 if v[0] > 0 else None}
                             for k, v in tot.items() if v[1]}
    if not args.no_cpu_baseline:
        import oracle as O
        from oracle.model import ModelDesc
        t0 = time.perf_counter()
        done, err, mag = 0, 0.0, 0.0
        gpu = [e.cpu() for e in els]
        i = 0
        while time.perf_counter() - t0 < args.cpu_seconds and i < len(ws):
            w = ws[i]
            sp = spins[i][:1].cpu().numpy()
            ref = O.eloc_plain(ModelDesc.of(w.model), w.ham, thetas[i], sp, w.model.N)
            err = max(err, abs(gpu[i][0].item() - ref["eloc"][0].item()))
            mag = max(mag, abs(ref["eloc"][0].item()))
            done += 1
            i += 1
        cpu_sec = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": done / cpu_sec, "unit": "samples/s", "cores": torch.get_num_threads(),
                               "kind": "oracle", "sample": f"sample 0 of instances 0..{done - 1}, float64 oracle, "
                                                           f"log-ratios by full re-evaluation, {cpu_sec:.1f} s"}
        out["err_vs_fp64_oracle"] = {"eloc": err / mag if mag else 0.0,
                                     "measure": "max|E - E*| / max|E*| over the CPU sample"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
