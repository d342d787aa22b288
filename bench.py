"""Benchmark: time to solution and Arnoldi GB/s of CB-GMRES on one MI355X.

Configurations (`--config`, default D5; every input seeded and synthetic):

* D1  2D 5-point Poisson 64x64 (n = 4,096), b = A 1, restart 100, fp32 basis.
* D2  3D 7-point upwind convection-diffusion 128^3 (n = 2,097,152, nnz =
      14,581,760), b ~ U[-1, 1] seed 0, restart 100, fp16 basis.
* D3  3D 27-point lognormal diffusion 128^3 (n = 2,097,152, nnz =
      55,742,968), b ~ U[-1, 1] seed 0, restart 100, bf16 basis.
* D4  the learned preconditioner, trained on 256 instances of the 27-point
      generator at 64^3 (seeds 1..256), on the held-out 128^3 system (seed
      0), fp16 basis, restart 100.
* D5  27-point lognormal diffusion 160^3 (n = 4,096,000, nnz = 109,215,352),
      restart 200: the learned preconditioner (stored form, its build
      included) with an fp16 basis, against plain fp64-basis GMRES (M = I)
      and against Jacobi with the same basis.  The largest configuration
      that fits one GPU; the headline.

x0 = 0 and tol = 1e-10 on the true relative residual throughout.  One step
is one complete solve (for the learned configurations: building the stored
preconditioner from the matrix, then the solve).  Inputs are resident in HBM
before the timed region; the network is trained on the GPU before it (the
training time is reported), unless `--weights` loads trained parameters.
The comparison solves run after the timed region.

Prints one JSON line.  `value` is the headline solve's time to solution
(seconds, lower is better).  `roofline` covers the dominant kernel of the
configuration, HIP events recorded at each launch's own start and end in
the timed solves, on every 8th Arnoldi step's launch (an event pair delays
the launch it brackets by a few microseconds; `--events all` times every
launch): the multi-dot h = V^T w with the Gram row on D1/D2 (bytes
j n b_s + 8 n + n b_s per launch), the step SpMV with A on D3-D5, which
reads the sliced-ELL copy of A (12 e + 8 (n/64 + 1) + 16 n: values and
columns of the e stored entries, slice offsets, the gathered input and the
output; 12 nnz + 4 (n+1) + 16 n on the CSR arrays).  `cpu_baseline` times the CPU oracle (Fig. 1 as written, on
the host cores) on the same system: the whole solve where it fits the
sample budget, else a stated number of steps scaled to the GPU's count.
`--trace-summary` and `--pmc-summary` turn rocprofv3 outputs of these runs
into per-j rates and counter traffic.
"""
from __future__ import annotations

import argparse
import dataclasses
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
FMT_ID = {"fp64": 0, "fp32": 1, "fp16": 2, "bf16": 3, "e4m3": 4, "int32": 5, "int16": 6,
          "fp16s": 7}
FMT_BYTES = {"fp64": 8, "fp32": 4, "fp16": 2, "bf16": 2, "e4m3": 1, "int32": 4, "int16": 2,
             "fp16s": 2}


@dataclasses.dataclass
class Config:
    key: str
    system: str            # "poisson2d", "convdiff7" or "lognormal27"
    grid: int
    desc: str
    restart: int
    fmt: str
    precond: str           # "none" or "learned"
    compare: list          # (format, preconditioner) pairs timed after the headline
    kernel: str            # "multidot" or "spmv": the roofline kernel


CONFIGS = {
    "D1": Config("D1", "poisson2d", 64,
                 "2D 5-point Poisson 64x64 (n=4096, nnz=20224), b = A 1, x0=0, restart 100, "
                 "tol 1e-10", 100, "fp32", "none", [("fp64", "none")], "multidot"),
    "D2": Config("D2", "convdiff7", 128,
                 "3D 7-point upwind convection-diffusion 128^3 (n=2097152, nnz=14581760), "
                 "b~U[-1,1] seed 0, x0=0, restart 100, tol 1e-10", 100, "fp16", "none",
                 [("fp64", "none"), ("fp32", "none"), ("int16", "none")], "multidot"),
    "D3": Config("D3", "lognormal27", 128,
                 "3D 27-point lognormal diffusion 128^3 (n=2097152, nnz=55742968), sigma 1, "
                 "shift 1e-2, b~U[-1,1] seed 0, x0=0, restart 100, tol 1e-10", 100, "bf16",
                 "none", [("fp64", "none"), ("e4m3", "none"), ("fp16", "none")], "spmv"),
    "D4": Config("D4", "lognormal27", 128,
                 "learned preconditioner (trained on 256 27-point lognormal instances at 64^3) "
                 "on the held-out 27-point lognormal 128^3 system (n=2097152, nnz=55742968), "
                 "b~U[-1,1] seed 0, x0=0, restart 100, tol 1e-10", 100, "fp16", "learned",
                 [("fp16", "jacobi"), ("fp16", "none"), ("fp64", "none")], "spmv"),
    "D5": Config("D5", "lognormal27", 160,
                 "3D 27-point lognormal diffusion 160^3 (n=4096000, nnz=109215352), sigma 1, "
                 "shift 1e-2, b~U[-1,1] seed 0, x0=0, restart 200, tol 1e-10; learned "
                 "preconditioner (stored form, build included) vs plain fp64-basis GMRES",
                 200, "fp16", "learned",
                 [("fp64", "none"), ("fp16", "jacobi"), ("int16", "jacobi"),
                  ("int16", "learned"), ("fp16", "none")], "spmv"),
}


# Arnoldi steps of the CPU oracle's sample per configuration: the whole
# solve where it takes under about 40 s on a 16-thread host share (D2 19 s,
# D5 38 s measured), else a stated number of steps scaled to the GPU's count
CPU_STEPS = {"D1": 100000, "D2": 100000, "D3": 1000, "D4": 100000, "D5": 100000}


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_file(cfg: Config) -> str:
    return os.path.join(ROOT, "profiles", f"traffic_{cfg.kernel}_{cfg.fmt}_{cfg.system}_"
                                          f"{cfg.grid}.json")


def kernel_pattern(cfg: Config) -> str:
    """Substring of the roofline kernel's name in rocprofv3 outputs."""
    if cfg.kernel == "multidot":
        return f"k_multidot<{FMT_ID[cfg.fmt]}, true>"
    return "k_spmv_sell<0, true"    # the step SpMV on the sliced-ELL copy (27-point rows)


def pmc_summary(fetch_csv: str, write_csv: str, cfg: Config) -> dict:
    """HBM bytes per launch of the roofline kernel from two rocprofv3 --pmc
    runs (FETCH_SIZE, WRITE_SIZE; KiB per dispatch), each scaled by what the
    same counter reads for the plain 256 MiB elementwise pass (torch.neg)
    that `bench.py --calib-copy` runs first.  For the SpMV only the
    dispatches of the most frequent launch shape count (the steps')."""
    import csv
    pat = kernel_pattern(cfg)

    def read(path, counter):
        rows = [r for r in csv.DictReader(open(path)) if r.get("Counter_Name") == counter]
        by_kernel = {}
        for r in rows:
            by_kernel.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        copy = [v for k, vals in by_kernel.items() if "neg_kernel" in k for v in vals]
        cands = {k: v for k, v in by_kernel.items() if pat in k}
        if not copy or not cands:
            raise SystemExit(f"{path}: no copy-kernel or {pat} rows for {counter}")
        name, vals = max(cands.items(), key=lambda kv: len(kv[1]))
        return sum(vals) / len(vals), max(copy), len(vals), name

    f_kib, f_copy, nf, name = read(fetch_csv, "FETCH_SIZE")
    w_kib, w_copy, nw, _ = read(write_csv, "WRITE_SIZE")
    f_scale = COPY_CALIB_BYTES / (f_copy * 1024.0)
    w_scale = COPY_CALIB_BYTES / (w_copy * 1024.0)
    out = {"kernel": name, "config": cfg.key, "format": cfg.fmt,
           "fetch_bytes_per_launch": f_kib * 1024.0 * f_scale,
           "write_bytes_per_launch": w_kib * 1024.0 * w_scale,
           "fetch_scale": f_scale, "write_scale": w_scale, "launches": [nf, nw],
           "statistic": "mean over launches (as the algorithmic bytes per launch)",
           "kernel_source_sha256": kernel_source_hash()}
    out["traffic_bytes_per_launch"] = out["fetch_bytes_per_launch"] + out["write_bytes_per_launch"]
    return out


def trace_summary(trace_csv: str, cfg: Config) -> dict:
    """Per-j durations of the step kernels from a rocprofv3 --kernel-trace CSV
    of bench runs of a configuration.  A cycle starts with the residual SpMV
    (mode 2); inside it the solver launches each step kernel once per
    Arnoldi step, j = 1, 2, ..., and after the cycle has ended up to two
    chunks of launches that return at once.  The steps that did work are the
    leading step-SpMV dispatches of the cycle longer than 10 us (an SpMV that
    moves the matrix takes far longer, one that returns at once a few us),
    and dispatch k of each step kernel in the cycle belongs to step j = k + 1.
    Per kernel and j: the median duration over the cycles and the
    algorithmic GB/s; per kernel the j-weighted rate over all j and over
    j >= 20."""
    import csv
    import statistics
    import numpy as np
    from paper_2009_12101_amd import problems as P
    A = build_system(cfg, P)[0]
    n, nnz, bs = A.n, A.nnz, FMT_BYTES[cfg.fmt]
    fid = FMT_ID[cfg.fmt]
    rows = list(csv.DictReader(open(trace_csv)))
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    dur = lambda r: (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9

    def spmv_mode(name):
        targs = name.split("<", 1)[1].split(">", 1)[0].split(",")
        return int(targs[0] if "k_spmv_sell" in name else targs[-1])

    spmv = {}
    for r in rows:
        if "k_spmv" in r["Kernel_Name"]:
            spmv[r["Kernel_Name"]] = spmv.get(r["Kernel_Name"], 0) + 1
    step_spmv = max(spmv, key=spmv.get)
    mode = spmv_mode(step_spmv)
    gather = (mode & 8) != 0                     # an Arnoldi-step mode: stores v_j too
    if "k_spmv_sell" in step_spmv:
        lens = np.zeros(-(-n // 64) * 64, dtype=np.int64)
        lens[:n] = np.diff(A.row_ptr)
        entries = 64 * int(lens.reshape(-1, 64).max(axis=1).sum())
        targs = step_spmv.split("<", 1)[1].split(">", 1)[0].split(",")
        per_entry = 9.0 if targs[2].strip() == "true" else 12.0    # diagonal indices or int32
        sp_bytes = per_entry * entries + 8.0 * (len(lens) // 64 + 1) + 16.0 * n
    else:
        sp_bytes = 12.0 * nnz + 4.0 * (n + 1) + 16.0 * n
    sp_bytes += n * bs if gather else 0.0
    kernels = {
        step_spmv: lambda j: sp_bytes,
        f"k_multidot<{fid}, true>": lambda j: j * n * bs + 8.0 * n + n * bs,
        f"k_update<{fid}, 6>": lambda j: j * n * bs + 16.0 * n,
        # the stored form of the learned preconditioner with steps 13-14:
        # 27 codes of 2 bytes, w, dinv and z of 8 bytes, the stored entry
        f"k_stencil<{fid}, 0": lambda j: 54.0 * n + 24.0 * n + n * bs,
    }
    # cycles: from one residual SpMV to the next
    cycles, cur = [], None
    for r in rows:
        name = r["Kernel_Name"]
        if "k_spmv" in name and spmv_mode(name) == 2:
            cur = []
            cycles.append(cur)
        elif cur is not None:
            cur.append(r)
    out = {"config": cfg.key, "format": cfg.fmt, "cycles": len(cycles), "kernels": {}}
    for key, model in kernels.items():
        per_j = {}
        count = 0
        for cyc in cycles:
            nwork = 0
            for r in cyc:
                if r["Kernel_Name"] == step_spmv:
                    if dur(r) <= 10e-6:
                        break
                    nwork += 1
            sel = [r for r in cyc if key in r["Kernel_Name"]][:nwork]
            count += len(sel)
            for k, r in enumerate(sel):
                per_j.setdefault(k + 1, []).append(dur(r))
        if not per_j:
            continue
        table = [{"j": j, "median_us": statistics.median(v) * 1e6,
                  "gbps": model(j) / statistics.median(v) / 1e9, "samples": len(v)}
                 for j, v in sorted(per_j.items())]

        def weighted(tab):
            return (sum(model(t["j"]) for t in tab) /
                    sum(t["median_us"] * 1e-6 for t in tab) / 1e9) if tab else None
        out["kernels"][key] = {"dispatches_that_worked": count, "bytes_j1": model(1),
                               "j_weighted_gbps": weighted(table),
                               "j_weighted_gbps_j_ge_20": weighted([t for t in table
                                                                    if t["j"] >= 20]),
                               "per_j": table}
    return out


def build_system(cfg: Config, P):
    if cfg.system == "poisson2d":
        A = P.poisson2d(cfg.grid)
        return A, P.rhs_row_sums(A)
    A = P.convdiff7(cfg.grid) if cfg.system == "convdiff7" else P.lognormal27(cfg.grid, 0)
    return A, P.rhs_uniform(A.n, 0)


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


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="D5", choices=sorted(CONFIGS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-steps", type=int, default=None,
                    help="Arnoldi steps of the CPU oracle sample (a whole solve if it needs "
                         "no more; default sized for 10-30 s of host work per configuration)")
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="host threads of the CPU oracle (0: all the process may use)")
    ap.add_argument("--weights", default=None,
                    help="trained parameters (.npz of LearnedSPAI.save); trained here if absent")
    ap.add_argument("--train-count", type=int, default=256)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--workers", type=int, default=16,
                    help="host processes generating the training matrices")
    ap.add_argument("--explicit-redot", action="store_true",
                    help="ablation: steps 5-10 in Fig. 1's explicit form")
    ap.add_argument("--csr", action="store_true",
                    help="ablation: the SpMV on A's CSR arrays (no sliced-ELL copy)")
    ap.add_argument("--no-compare", action="store_true",
                    help="time the headline solves only (no all-kernel solve, no comparison "
                         "solves): the command a kernel-trace profile of the roofline kernel "
                         "runs, so every dispatch of it belongs to the timed solves")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run a plain 256 MiB device copy first (counter calibration)")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the roofline kernel's traffic record from two counter runs")
    ap.add_argument("--events", choices=["sampled", "all"], default="sampled",
                    help="roofline kernel's launches timed with HIP events in the timed solves: "
                         "every 8th Arnoldi step's (default) or all")
    ap.add_argument("--trace-summary", metavar="KERNEL_TRACE_CSV",
                    help="print per-j rates of the step kernels from a kernel trace and exit")
    args = ap.parse_args()
    cfg = CONFIGS[args.config]
    if args.trace_summary:
        print(json.dumps(trace_summary(args.trace_summary, cfg)))
        return 0
    if args.pmc_summary:
        rec = pmc_summary(args.pmc_summary[0], args.pmc_summary[1], cfg)
        with open(traffic_file(cfg), "w") as f:
            json.dump(rec, f, indent=1)
        print(json.dumps(rec))
        return 0
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; "
                          "--gpus > 1 is not supported (single-GPU build)"}))
        return 2

    learned = cfg.precond == "learned" or any(pc == "learned" for _, pc in cfg.compare)
    pool = None
    if learned and not args.weights and args.workers > 1:
        # training matrices are generated in processes forked before anything
        # touches the GPU
        import multiprocessing
        pool = multiprocessing.get_context("fork").Pool(args.workers)

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

    training = None
    model = None
    if learned:
        from paper_2009_12101_amd.spai import LearnedSPAI, make_instances
        model = LearnedSPAI(dev, seed=0)
        if args.weights:
            model.load(args.weights)
            training = {"weights": os.path.basename(args.weights)}
        else:
            t0 = time.time()
            data = make_instances(range(1, 1 + args.train_count), 64, dev, pool, log)
            if pool is not None:
                pool.close()
                pool.join()
            t_data = time.time() - t0
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            hist = model.train(data, args.epochs, 8, 1e-3)
            torch.cuda.synchronize()
            t_train = time.perf_counter() - t0
            del data
            torch.cuda.empty_cache()
            training = {"instances": args.train_count, "grid": 64, "epochs": args.epochs,
                        "batch": 8, "lr": 1e-3, "data_seconds": t_data,
                        "train_seconds": t_train, "loss_first_epoch": hist[0],
                        "loss_last_epoch": hist[-1]}
            log(f"trained on {args.train_count} instances: data {t_data:.1f}s, "
                f"training {t_train:.1f}s, loss {hist[0]:.4f} -> {hist[-1]:.4f}")

    t0 = time.time()
    A, b = build_system(cfg, P)
    log(f"generated {cfg.system} {cfg.grid}: n={A.n} nnz={A.nnz} in {time.time() - t0:.1f}s")
    Ad = cbg.DeviceCSR.from_host(A, dev, sell=False if args.csr else "auto")
    bd = torch.from_numpy(b).to(dev)
    m, tol, maxiter = cfg.restart, 1e-10, 20000
    pcs = {("stencil" if pc == "learned" else pc) for _, pc in cfg.compare + [(cfg.fmt,
                                                                               cfg.precond)]}
    need = max(cbg.workspace_bytes(A.n, m, f, pc) for f in ("fp64", cfg.fmt) for pc in pcs)
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    codes = sws = None
    if learned:
        codes = torch.empty(27 * cbg.basis_ld(A.n), dtype=torch.int16, device=dev)
        sws = torch.empty(cbg.spai_workspace_bytes(A.n, A.nnz, 0), dtype=torch.uint8,
                          device=dev)
    variant = ("explicit_redot",) if args.explicit_redot else ()

    def one(fmt, pc, profile):
        """One step: (for the learned preconditioner) its build from A, then
        the solve."""
        if pc == "learned":
            model.build_stencil(Ad, A.grid, ws=sws, out=codes)
            return cbg.solve(Ad, bd, restart=m, fmt=fmt, tol=tol, maxiter=maxiter,
                             precond="stencil", p_stencil=codes, grid=A.grid, fallback=True,
                             profile=profile, workspace=ws, hist=False, variant=variant)
        return cbg.solve(Ad, bd, restart=m, fmt=fmt, tol=tol, maxiter=maxiter, precond=pc,
                         profile=profile, workspace=ws, hist=False, variant=variant)

    prof_kind = ("dot" if cfg.kernel == "multidot" else "spmv") + \
        ("/sampled" if args.events == "sampled" else "")
    for _ in range(args.warmup):
        one(cfg.fmt, cfg.precond, prof_kind)
    torch.cuda.synchronize()
    log("warmup done")

    results = []
    torch.cuda.synchronize()
    start = time.perf_counter()
    for _ in range(args.steps):
        results.append(one(cfg.fmt, cfg.precond, prof_kind))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - start
    r0 = results[-1]
    value = elapsed / args.steps
    if cfg.kernel == "multidot":
        k_ms = sum(r.prof_dot_ms for r in results)
        k_bytes = sum(r.prof_dot_bytes for r in results)
        k_launch = sum(r.prof_dot_launches for r in results)
        k_name = f"k_multidot<{cfg.fmt}> (with the Gram row)"
    else:
        k_ms = sum(r.prof_spmv_ms for r in results)
        k_bytes = sum(r.prof_spmv_bytes for r in results)
        k_launch = sum(r.prof_spmv_launches for r in results)
        k_name = ("k_spmv_sell (the Arnoldi step's SpMV with A, sliced-ELL copy)"
                  if Ad.sell_col is not None else "k_spmv (the Arnoldi step's SpMV with A)")
    achieved = k_bytes / (k_ms * 1e-3) / 1e9 if k_ms > 0 else 0.0
    # the SpMV's rate restated on the bytes a CSR kernel would move for the
    # same product (12 nnz + 4 (n+1) + 16 n): what a CSR SpMV would need to
    # sustain to match this time; context beside `achieved`, not a roofline
    csr_equiv = None
    if cfg.kernel == "spmv" and Ad.sell_val is not None and achieved > 0:
        nsl = (A.n + 63) // 64
        per = 9.0 if Ad.sell_dix is not None else 12.0
        sell_bytes = per * Ad.sell_entries + 8.0 * (nsl + 1) + 16.0 * A.n
        csr_bytes = 12.0 * A.nnz + 4.0 * (A.n + 1) + 16.0 * A.n
        csr_equiv = achieved * csr_bytes / sell_bytes
    x = r0.x.cpu().numpy()
    S = A.to_scipy()
    res_check = float(np.linalg.norm(b - S @ x) / np.linalg.norm(b))
    log(f"{cfg.key} {cfg.fmt}+{cfg.precond}: {value * 1e3:.1f} ms/solve it={r0.iterations} "
        f"cycles={r0.restarts} res={res_check:.2e} {cfg.kernel} {achieved:.0f} GB/s")
    # every basis-streaming kernel and the step SpMV timed, in one extra solve
    full = None
    if not args.no_compare:
        full = one(cfg.fmt, cfg.precond, "all")
        torch.cuda.synchronize()

    def row(r, seconds):
        xr = r.x.cpu().numpy()
        return dict(seconds=seconds, iterations=r.iterations, restarts=r.restarts,
                    reorths=r.reorths, explicit_steps=r.explicit_steps, fell_back=r.fell_back,
                    true_rel_res=float(np.linalg.norm(b - S @ xr) / np.linalg.norm(b)),
                    arnoldi_gbps=r.model_bytes / r.seconds / 1e9)

    label = lambda f, pc: f"{f}+{pc}"
    runs = {label(cfg.fmt, cfg.precond): row(r0, value)}
    for fmt, pc in ([] if args.no_compare else cfg.compare):
        one(fmt, pc, False)
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = one(fmt, pc, False)
        torch.cuda.synchronize()
        runs[label(fmt, pc)] = row(r, time.perf_counter() - t)
        log(f"{label(fmt, pc)}: {runs[label(fmt, pc)]['seconds'] * 1e3:.1f} ms "
            f"it={r.iterations}")

    copy_gbps = copy_rate_gbps(torch, dev)
    log(f"device copy: {copy_gbps:.0f} GB/s")

    cpu = None
    if not args.no_cpu:
        import oracle
        if args.cpu_threads > 0:
            oracle.set_threads(args.cpu_threads)
        cpu_steps = args.cpu_steps if args.cpu_steps is not None else CPU_STEPS[cfg.key]
        steps = max(1, min(cpu_steps, r0.iterations + m))
        t = time.perf_counter()
        kw = {}
        sample = ""
        if cfg.precond == "learned":
            # the oracle's own build of the stored form from the same
            # trained weights: features, forward pass, float16 codes
            from oracle import spai as OS
            w = model.weights.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
            wf = w.view(np.float32).astype(np.float64)
            prm = model.params.cpu().numpy().astype(np.float64)
            nf, nh, no = OS.NFEAT, OS.NHID, OS.NOUT
            W1 = wf[:nf * nh].reshape(nf, nh)
            W2 = wf[nf * nh:nf * nh + nh * nh].reshape(nh, nh)
            W3 = wf[nf * nh + nh * nh:].reshape(nh, no)
            o = nf * nh
            b1, b2 = prm[o:o + nh], prm[o + nh + nh * nh:o + 2 * nh + nh * nh]
            b3 = prm[-no:]
            F = OS.features(A, A.grid)
            _, _, O = OS.forward(F, W1, b1, W2, b2, W3, b3)
            kw = dict(precond="stencil", grid=A.grid, fallback=True,
                      p_stencil=OS.stencil_codes(A, A.grid, O.astype(np.float32)))
            sample = "the oracle's build of the stored form from the trained weights, then "
        o = oracle.gmres(A, b, restart=m, fmt=cfg.fmt, tol=tol, maxiter=steps, **kw)
        dt = time.perf_counter() - t
        whole = o["status"] == 0
        scaled = dt if whole else dt / max(o["iterations"], 1) * r0.iterations
        cpu = {"value": scaled, "unit": "s", "cores": oracle.get_threads(),
               "cpu_model": cpu_model(), "kind": "oracle",
               "sample": (sample + f"the whole {cfg.fmt}-basis solve ({o['iterations']} "
                          f"Arnoldi steps, {o['restarts']} cycles) on the host cores in "
                          f"{dt:.1f} s" if whole else
                          sample + f"{o['iterations']} Arnoldi steps ({o['restarts']} cycles of "
                          f"restart {m}) of the same {cfg.fmt}-basis solve on the host cores in "
                          f"{dt:.1f} s, scaled to the GPU's {r0.iterations} steps")}
        log(f"cpu oracle: {dt:.1f}s for {o['iterations']} steps (status {o['status']})")

    traffic = None
    tf = traffic_file(cfg)
    if os.path.exists(tf):
        rec = json.load(open(tf))
        if rec.get("kernel_source_sha256") == kernel_source_hash():
            traffic = rec["traffic_bytes_per_launch"]

    head = runs[label(cfg.fmt, cfg.precond)]
    fp64 = runs.get(label("fp64", "none"))
    line = {
        "metric": METRIC, "value": value, "unit": "s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": value * 1e3, "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{cfg.key}: {cfg.desc}", "basis_format": cfg.fmt,
                   "preconditioner": ("learned, stored form (float16 corrections on the "
                                      "27-point slots), build included" if cfg.precond ==
                                      "learned" else cfg.precond),
                   "matrix_storage": ("sliced ELL (SELL-64) beside CSR"
                                      if Ad.sell_col is not None else "CSR"),
                   "arithmetic": "fp64", "parallelism": "single GPU"},
        "iterations": r0.iterations, "restarts": r0.restarts, "reorths": r0.reorths,
        "true_rel_res": res_check,
        "arnoldi_gbps": head["arnoldi_gbps"],
        "runs": runs,
        "speedup_vs_plain_fp64": fp64["seconds"] / value if fp64 else None,
        "speedup_vs_jacobi_same_basis": (runs[label(cfg.fmt, "jacobi")]["seconds"] / value
                                         if label(cfg.fmt, "jacobi") in runs else None),
        "training": training,
        "kernels_one_solve": None if full is None else {
            "orth_gbps": (full.prof_orth_bytes / (full.prof_orth_ms * 1e-3) / 1e9
                          if full.prof_orth_ms > 0 else None),
            "multidot_gbps": (full.prof_dot_bytes / (full.prof_dot_ms * 1e-3) / 1e9
                              if full.prof_dot_ms > 0 else None),
            "multidot_ms": full.prof_dot_ms,
            "spmv_gbps": (full.prof_spmv_bytes / (full.prof_spmv_ms * 1e-3) / 1e9
                          if full.prof_spmv_ms > 0 else None),
            "spmv_ms": full.prof_spmv_ms, "orth_ms": full.prof_orth_ms},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic,
                     "kernel": k_name, "launches": k_launch,
                     "timed_launches": ("every 8th Arnoldi step's launch in the timed solves"
                                        if args.events == "sampled" else
                                        "every launch in the timed solves"),
                     "copy_gbps": copy_gbps, "frac_of_copy": achieved / copy_gbps,
                     "avg_launch_us": k_ms * 1e3 / max(k_launch, 1),
                     "algorithmic_bytes_per_launch": k_bytes / max(k_launch, 1),
                     "csr_equivalent_gbps": csr_equiv},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
