"""Benchmark: time-to-solution and Arnoldi GB/s of CB-GMRES on one MI355X.

Workload: the 3D 7-point upwind convection-diffusion system on a 128^3 grid
(n = 2,097,152, nnz = 14,581,760, nonsymmetric, global Peclet 10 per axis),
b ~ U[-1, 1] (seed 0), x0 = 0, restart m = 100, tol 1e-10 on the true
relative residual.  One step = one complete solve with the basis stored in
fp16 (the headline compressed format); solves with fp64 / fp32 / int16
storage run after the timed region for the compressed-vs-fp64 comparison.

Prints one JSON line.  `value` is the fp16-basis time to solution (seconds,
lower is better).  `roofline` covers the multi-dot kernel h = V^T w (the
dominant kernel, which also forms the newest row of the basis's Gram matrix
for step 8's re-dot): algorithmic bytes per launch (j * n * 2 + 8 n + n * 2
for j stored vectors: the basis, w, and the newest vector's tile) over its
duration in the timed solves, from HIP events the solver records at each
multi-dot launch's own start and end (only those launches are event-timed
in the timed region).  One more solve after the timed region times every
basis-streaming kernel (`orth_kernels_gbps`; `fused_update_redot` with
`--explicit-redot`).
`roofline.copy_gbps` is a 1 GiB device-to-device copy timed the same way
(`frac_of_copy` reads the multi-dot against it).  `--trace-summary` turns a
rocprofv3 kernel trace of these runs into per-j multi-dot rates.
`cpu_baseline` is the CPU oracle timed on five restart cycles (500 Arnoldi
steps) of the same solve on the host cores, scaled to the GPU's iteration
count.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "time-to-solution + Arnoldi GB/s at rel. residual 1e-10, CB vs fp64-basis"
HBM_PEAK_GBPS = 8000.0
KERNEL_SOURCES = ["paper_2009_12101_amd/csrc/cbg_kernels.hip",
                  "paper_2009_12101_amd/csrc/cbg_device.hpp"]
COPY_CALIB_BYTES = 256 * 2 ** 20


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_file(fmt: str, grid: int) -> str:
    return os.path.join(ROOT, "profiles", f"traffic_k_multidot_{fmt}_convdiff7_{grid}.json")


def pmc_summary(fetch_csv: str, write_csv: str, fmt: str, grid: int) -> dict:
    """HBM bytes per launch of the multi-dot kernel from two rocprofv3 --pmc
    runs (FETCH_SIZE, WRITE_SIZE; KiB per dispatch), each scaled by what the
    same counter reads for the plain 256 MiB elementwise pass (torch.neg)
    that `bench.py --calib-copy` runs first."""
    import csv
    fmt_id = {"fp64": 0, "fp32": 1, "fp16": 2, "bf16": 3, "e4m3": 4, "int32": 5, "int16": 6,
              "fp16s": 7}[fmt]
    kname = f"k_multidot<{fmt_id}, true>"

    def read(path, counter):
        rows = list(csv.DictReader(open(path)))
        by_kernel = {}
        for r in rows:
            if r.get("Counter_Name") != counter:
                continue
            by_kernel.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        copy = [v for k, vals in by_kernel.items() if "neg_kernel" in k for v in vals]
        md = [v for k, vals in by_kernel.items() if kname in k for v in vals]
        if not copy or not md:
            raise SystemExit(f"{path}: no copy-kernel or {kname} rows for {counter}")
        copy_kib = max(copy)                 # the 256 MiB calibration copy
        return sum(md) / len(md), copy_kib, len(md)

    f_kib, f_copy, nf = read(fetch_csv, "FETCH_SIZE")
    w_kib, w_copy, nw = read(write_csv, "WRITE_SIZE")
    f_scale = COPY_CALIB_BYTES / (f_copy * 1024.0)
    w_scale = COPY_CALIB_BYTES / (w_copy * 1024.0)
    out = {"kernel": kname, "format": fmt, "grid": grid,
           "fetch_bytes_per_launch": f_kib * 1024.0 * f_scale,
           "write_bytes_per_launch": w_kib * 1024.0 * w_scale,
           "fetch_scale": f_scale, "write_scale": w_scale, "launches": [nf, nw],
           "kernel_source_sha256": kernel_source_hash()}
    out["traffic_bytes_per_launch"] = out["fetch_bytes_per_launch"] + out["write_bytes_per_launch"]
    return out


def trace_summary(trace_csv: str, fmt: str, grid: int, restart: int = 100) -> dict:
    """Per-j durations of the basis-streaming kernels and the step SpMV from
    a rocprofv3 --kernel-trace CSV of bench runs.  The solver launches each
    of them once per Arnoldi step, j = 1..restart in every cycle (launches
    after a cycle ended return at once), so dispatch k of a kernel in launch
    order belongs to step j = k mod restart + 1.  Per kernel and j: the
    median duration over all cycles and the algorithmic GB/s; per kernel the
    j-weighted rate over all j and over j >= 20.  Algorithmic bytes: the
    multi-dot with the Gram row j n b_s + 8 n + n b_s; the one update of
    steps 5-10 j n b_s + 16 n; the step SpMV 12 nnz +
    4 (n+1) + 16 n + n b_s (the 7-point system: nnz = 7 N^3 - 6 N^2)."""
    import csv
    import statistics
    fmt_id = {"fp64": 0, "fp32": 1, "fp16": 2, "bf16": 3, "e4m3": 4, "int32": 5, "int16": 6,
              "fp16s": 7}[fmt]
    bs = {"fp64": 8, "fp32": 4, "fp16": 2, "bf16": 2, "e4m3": 1, "int32": 4, "int16": 2,
          "fp16s": 2}[fmt]
    n = grid ** 3
    nnz = 7 * grid ** 3 - 6 * grid ** 2
    kernels = {
        f"k_multidot<{fmt_id}, true>": lambda j: j * n * bs + 8.0 * n + n * bs,
        f"k_update<{fmt_id}, 6>": lambda j: j * n * bs + 16.0 * n,
        "k_spmv<256, 2048, 8>": lambda j: 12.0 * nnz + 4.0 * (n + 1) + 16.0 * n + n * bs,
    }
    rows = list(csv.DictReader(open(trace_csv)))
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    out = {"format": fmt, "grid": grid, "kernels": {}}
    for key, model in kernels.items():
        sel = [r for r in rows if key in r["Kernel_Name"]]
        if not sel or len(sel) % restart:
            raise SystemExit(f"{trace_csv}: {len(sel)} dispatches of {key}, not a multiple of "
                             f"{restart}")
        per_j = {}
        for k, r in enumerate(sel):
            per_j.setdefault(k % restart + 1, []).append(
                (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9)
        table = [{"j": j, "median_us": statistics.median(v) * 1e6,
                  "gbps": model(j) / statistics.median(v) / 1e9, "samples": len(v)}
                 for j, v in sorted(per_j.items())]

        def weighted(tab):
            return sum(model(t["j"]) for t in tab) / sum(t["median_us"] * 1e-6 for t in tab) / 1e9
        out["kernels"][key.rstrip(",")] = {
            "dispatches": len(sel), "j_weighted_gbps": weighted(table),
            "j_weighted_gbps_j_ge_20": weighted([t for t in table if t["j"] >= 20]),
            "per_j": table}
    md = out["kernels"][f"k_multidot<{fmt_id}, true>"]
    # the multi-dot's figures at the top level (the roofline kernel)
    out.update({"kernel": f"k_multidot<{fmt_id}, true>", "dispatches": md["dispatches"],
                "j_weighted_gbps_j_ge_20": md["j_weighted_gbps_j_ge_20"], "per_j": md["per_j"]})
    return out


def copy_rate_gbps(torch, dev, nbytes: int = 2 ** 30) -> float:
    """Device-to-device copy of nbytes (reads and writes nbytes), best of 5,
    timed with events on torch's current stream: the practical streaming
    rate the roofline fraction can also be read against."""
    src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = None
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del src, dst
    return 2.0 * nbytes / (best * 1e-3) / 1e9


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--grid", type=int, default=128)
    ap.add_argument("--format", default="fp16")
    ap.add_argument("--compare", default="fp64,fp32,int16")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--explicit-redot", action="store_true",
                    help="ablation: step 8's re-dot as an explicit multi-dot of the updated w "
                         "(fused with the update where the register tile allows)")
    ap.add_argument("--no-fuse", action="store_true",
                    help="with --explicit-redot: update and re-dot as two basis passes")
    ap.add_argument("--cpu-cycles", type=int, default=5,
                    help="restart cycles of the CPU oracle sample (about 2.5 s each on 16 cores)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run a plain 256 MiB device copy first (counter calibration)")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the multi-dot traffic record from two counter runs and exit")
    ap.add_argument("--trace-summary", metavar="KERNEL_TRACE_CSV",
                    help="print per-j rates of the step kernels from a kernel trace and exit")
    args = ap.parse_args()
    if args.trace_summary:
        print(json.dumps(trace_summary(args.trace_summary, args.format, args.grid)))
        return 0
    if args.pmc_summary:
        rec = pmc_summary(args.pmc_summary[0], args.pmc_summary[1], args.format, args.grid)
        with open(traffic_file(args.format, args.grid), "w") as f:
            json.dump(rec, f, indent=1)
        print(json.dumps(rec))
        return 0
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; "
                          "--gpus > 1 is not supported (single-GPU build)"}))
        return 2

    import numpy as np
    import torch

    import paper_2009_12101_amd as cbg
    from paper_2009_12101_amd import problems as P

    dev = torch.device("cuda:0")
    if args.calib_copy:
        # a plain elementwise pass of known size (reads and writes 256 MiB):
        # the counter runs scale FETCH_SIZE / WRITE_SIZE by what it reads
        src = torch.ones(COPY_CALIB_BYTES // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst
    m, tol, maxiter = 100, 1e-10, 20000
    t0 = time.time()
    A = P.convdiff7(args.grid)
    b = P.rhs_uniform(A.n, 0)
    log(f"generated {A.name}: n={A.n} nnz={A.nnz} in {time.time() - t0:.1f}s")
    Ad = cbg.DeviceCSR.from_host(A, dev)
    bd = torch.from_numpy(b).to(dev)
    ws = torch.empty(cbg.workspace_bytes(A.n, m, "fp64"), dtype=torch.uint8, device=dev)

    def one(fmt, profile):
        return cbg.solve(Ad, bd, restart=m, fmt=fmt, tol=tol, maxiter=maxiter, profile=profile,
                         workspace=ws, fuse=not args.no_fuse,
                         variant=("explicit_redot",) if args.explicit_redot else ())

    # the timed solves event-time the multi-dot launches only (the roofline
    # kernel); timing every basis kernel costs about 8% of a step
    for _ in range(args.warmup):
        one(args.format, "dot")
    torch.cuda.synchronize()
    log("warmup done")

    results = []
    torch.cuda.synchronize()
    start = time.perf_counter()
    for _ in range(args.steps):
        results.append(one(args.format, "dot"))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - start
    r0 = results[-1]
    ms_per_step = elapsed / args.steps * 1e3
    value = elapsed / args.steps
    dot_ms = sum(r.prof_dot_ms for r in results)
    dot_bytes = sum(r.prof_dot_bytes for r in results)
    dot_launch = sum(r.prof_dot_launches for r in results)
    # every basis-streaming kernel timed, in one extra solve after the timed
    # region
    full = one(args.format, True)
    torch.cuda.synchronize()
    fz_ms, fz_bytes, fz_launch = full.prof_fused_ms, full.prof_fused_bytes, full.prof_fused_launches
    orth_ms, orth_bytes = full.prof_orth_ms, full.prof_orth_bytes
    achieved = dot_bytes / (dot_ms * 1e-3) / 1e9 if dot_ms > 0 else 0.0
    x = r0.x.cpu().numpy()
    res_check = float(np.linalg.norm(b - A.to_scipy() @ x) / np.linalg.norm(b))
    log(f"{args.format}: {ms_per_step:.1f} ms/solve it={r0.iterations} cycles={r0.restarts} "
        f"res={res_check:.2e} multidot {achieved:.0f} GB/s")

    formats = {args.format: dict(seconds=value, iterations=r0.iterations, restarts=r0.restarts,
                                 reorths=r0.reorths, true_rel_res=res_check,
                                 arnoldi_gbps=r0.model_bytes / r0.seconds / 1e9)}
    for fmt in [f for f in args.compare.split(",") if f and f != args.format]:
        one(fmt, False)
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = one(fmt, False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        xr = r.x.cpu().numpy()
        formats[fmt] = dict(seconds=dt, iterations=r.iterations, restarts=r.restarts,
                            reorths=r.reorths,
                            true_rel_res=float(np.linalg.norm(b - A.to_scipy() @ xr)
                                               / np.linalg.norm(b)),
                            arnoldi_gbps=r.model_bytes / r.seconds / 1e9)
        log(f"{fmt}: {dt * 1e3:.1f} ms it={r.iterations}")

    copy_gbps = copy_rate_gbps(torch, dev)
    log(f"device copy: {copy_gbps:.0f} GB/s")

    cpu = None
    if not args.no_cpu:
        import oracle
        cyc = args.cpu_cycles
        t = time.perf_counter()
        o = oracle.gmres(A, b, restart=m, fmt=args.format, tol=tol, maxiter=cyc * m)
        dt = time.perf_counter() - t
        per_step = dt / max(o["iterations"], 1)
        cpu = {"value": per_step * r0.iterations, "unit": "s", "cores": oracle.get_threads(),
               "kind": "oracle",
               "sample": f"{o['iterations']} Arnoldi steps ({cyc} restart cycles) of the same "
                         f"{args.format}-basis solve on the host cores in {dt:.1f} s, scaled to "
                         f"the GPU's {r0.iterations} steps"}
        log(f"cpu oracle: {dt:.1f}s for {o['iterations']} steps")

    traffic = None
    tf = traffic_file(args.format, args.grid)
    if os.path.exists(tf):
        rec = json.load(open(tf))
        if rec.get("kernel_source_sha256") == kernel_source_hash():
            traffic = rec["traffic_bytes_per_launch"]

    line = {
        "metric": METRIC, "value": value, "unit": "s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"3D 7-point upwind convection-diffusion {args.grid}^3 "
                               f"(n={A.n}, nnz={A.nnz}), b~U[-1,1] seed 0, x0=0, "
                               f"restart {m}, tol {tol}",
                   "basis_format": args.format, "arithmetic": "fp64",
                   "parallelism": "single GPU"},
        "iterations": r0.iterations, "restarts": r0.restarts, "reorths": r0.reorths,
        "true_rel_res": res_check,
        "arnoldi_gbps": r0.model_bytes / r0.seconds / 1e9,
        "orth_kernels_gbps": orth_bytes / (orth_ms * 1e-3) / 1e9 if orth_ms > 0 else None,
        "fused_update_redot": None if fz_launch == 0 else {
            "gbps": fz_bytes / (fz_ms * 1e-3) / 1e9, "launches": fz_launch,
            "avg_launch_us": fz_ms * 1e3 / fz_launch},
        "formats": formats,
        "speedup_vs_fp64_basis": (formats["fp64"]["seconds"] / value) if "fp64" in formats
        else None,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic,
                     "kernel": f"k_multidot<{args.format}> (with the Gram row)",
                     "launches": dot_launch,
                     "copy_gbps": copy_gbps, "frac_of_copy": achieved / copy_gbps,
                     "avg_launch_us": dot_ms * 1e3 / max(dot_launch, 1),
                     "algorithmic_bytes_per_launch": dot_bytes / max(dot_launch, 1)},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
