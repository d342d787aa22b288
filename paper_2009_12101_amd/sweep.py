"""Restart-length sweep: speedup of a compressed basis over the fp64 basis.

The paper's restart study (Section 6, the restart-parameter figure) runs a
fixed number of restart cycles for each m with the numerics ignored, so that
every format does the same number of Arnoldi steps and the ratio of times
is the ratio of per-step costs.  This tool does the same on one GPU: for
each m it runs `cycles` full cycles (tolerance 0, maxiter = cycles * m) per
storage format and reports

* seconds, per-step microseconds and Arnoldi GB/s (the solver's algorithmic
  bytes over the measured time),
* the measured speedup over fp64 storage,
* the speedup the paper's memops model predicts (Section 4, Eq. 2-3 with
  Amdahl's law: per cycle the basis traffic of the default step, two reads
  of the j stored vectors per step, plus the SpMV's n_z(1+f) + (n+1)f
  values, at fp64 over the same at the format's width; vectors ignored),
* the speedup the solver's full byte model predicts (fp64 bytes / format
  bytes, vector traffic included), which the measured speedup approaches
  when every kernel runs at the same bandwidth, and
* the asymptote 8 / b_s (2 for 32-bit, 4 for 16-bit, 8 for 8-bit storage)
  that both models approach as m grows and the basis dominates.

    python -m paper_2009_12101_amd.sweep --system convdiff7_128 \\
        --restarts 10,20,50,100,150,200,300
"""
from __future__ import annotations

import argparse
import json
import sys
import time

from . import _binding as B
from . import problems as P


def system(name: str):
    kind, size = name.rsplit("_", 1)
    N = int(size)
    if kind == "convdiff7":
        A = P.convdiff7(N)
    elif kind == "lognormal27":
        A = P.lognormal27(N, 0)
    elif kind == "poisson2d":
        A = P.poisson2d(N)
    else:
        raise SystemExit(f"unknown system {name}")
    return A, P.rhs_uniform(A.n, 0)


def eq3_cycle_bytes(A, m: int, bs: int) -> float:
    """Bytes of one cycle of m steps by the paper's memops model (Eq. 2):
    step j reads the j stored vectors twice (the multi-dot and the one
    update of the default step) plus the SpMV's values, column indices and
    row pointers (n_z (1 + f) + (n + 1) f values of 8 bytes, f = 1/2)."""
    n, nnz = A.n, A.nnz
    basis = sum(2.0 * j * n * bs for j in range(1, m + 1))
    return basis + m * (12.0 * nnz + 4.0 * (n + 1))


def sweep(A, b, restarts, formats, cycles=10, device="cuda", log=None):
    import torch
    Ad = B.DeviceCSR.from_host(A, device)
    bd = torch.from_numpy(b).to(device)
    rows = []
    for m in restarts:
        ws = torch.empty(B.workspace_bytes(A.n, m, "fp64"), dtype=torch.uint8, device=device)
        per = {}
        for fmt in formats:
            kw = dict(restart=m, fmt=fmt, tol=0.0, maxiter=cycles * m, workspace=ws, hist=False)
            B.solve(Ad, bd, **dict(kw, maxiter=m))            # warm-up: one cycle
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = B.solve(Ad, bd, **kw)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            per[fmt] = dict(seconds=dt, steps=r.iterations, us_per_step=dt / r.iterations * 1e6,
                            model_bytes=r.model_bytes, gbps=r.model_bytes / dt / 1e9,
                            eq3_bytes=eq3_cycle_bytes(A, m, B.FORMAT_BYTES[fmt]),
                            asymptote=8.0 / B.FORMAT_BYTES[fmt])
        base = per.get("fp64")
        for fmt, v in per.items():
            if base is not None:
                v["speedup"] = base["seconds"] / v["seconds"]
                v["model_speedup"] = base["model_bytes"] / v["model_bytes"]
                v["eq3_speedup"] = base["eq3_bytes"] / v["eq3_bytes"]
        rows.append(dict(restart=m, formats=per))
        if log:
            log(f"m={m}: " + "  ".join(
                f"{f} {v['us_per_step']:.1f}us x{v.get('speedup', 1.0):.2f} "
                f"(eq3 x{v.get('eq3_speedup', 1.0):.2f}, bytes x{v.get('model_speedup', 1.0):.2f})"
                for f, v in per.items()))
    return rows


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--system", default="convdiff7_128")
    ap.add_argument("--restarts", default="10,20,50,100,150,200,300")
    ap.add_argument("--formats", default="fp64,fp32,fp16,bf16,e4m3,int32,int16,fp16s")
    ap.add_argument("--cycles", type=int, default=10)
    ap.add_argument("--json", default=None)
    a = ap.parse_args(argv)
    import torch
    A, b = system(a.system)
    rows = sweep(A, b, [int(m) for m in a.restarts.split(",")], a.formats.split(","),
                 a.cycles, torch.device("cuda:0"),
                 log=lambda s: print(s, file=sys.stderr, flush=True))
    out = dict(system=A.name, n=A.n, nnz=A.nnz, cycles=a.cycles, rows=rows)
    line = json.dumps(out)
    if a.json:
        with open(a.json, "w") as f:
            f.write(line + "\n")
    print(line, flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
