"""Numerical ablations of the Arnoldi step on one GPU.

The compressed bases cost extra iterations against the FP64 basis (the
paper's Table 2 reports this overhead per matrix and format).  This tool
solves one system to tolerance for each storage format and each variant of
the step, and reports iterations, time and the overhead against the FP64
basis with the unablated step, and the relative difference of each solution
from that fp64-basis solution (``x_err``; two solves that both meet the
tolerance can differ by up to 2 tol ||b|| / sigma_min(A)):

* ``default``: Fig. 1 as the solver runs it (SpMV on the FP64 v, CGS with
  the step-7 test, eta = 1/sqrt(2); the re-dot and the norm of step 6 from
  the Gram row the multi-dot forms, steps 5-10 in one update);
* ``twopass``: the Gram-form re-dot with the update, the norm and the second
  update as separate passes;
* ``spmv_vhat``: step 3 multiplies by the stored vector read back;
* ``cgs2``: a second CGS pass on every step;
* ``cgs1``: never a second pass (eta -> 0);
* ``mgs`` / ``mgs1``: modified Gram-Schmidt with the step-7 test / with one
  pass only (one launch per stored vector: slow by design);
* ``explicit``: step 8's re-dot as a second multi-dot of the updated w, the
  form Fig. 1 writes (fused with the update where the tile allows);
* formats include ``fp16s``, float16 with a per-vector power-of-two scale.

    python -m paper_2009_12101_amd.ablate --system convdiff7_128 \\
        --formats fp64,fp32,fp16,fp16s,bf16,int16 --json out.json
"""
from __future__ import annotations

import argparse
import json
import sys
import time

from . import _binding as B
from .sweep import system

VARIANTS = {
    "default": dict(),
    "spmv_vhat": dict(variant=("spmv_vhat",)),
    "cgs2": dict(variant=("always_reorth",)),
    "cgs1": dict(eta=1e-300),
    "mgs": dict(variant=("mgs",)),
    "mgs1": dict(variant=("mgs",), eta=1e-300),
    "twopass": dict(variant=("gram",)),
    "explicit": dict(variant=("explicit_redot",)),
}


def ablate(A, b, formats, variants, restart=100, tol=1e-10, maxiter=20000, precond="none",
           repeats=2, device="cuda", log=None):
    import torch
    Ad = B.DeviceCSR.from_host(A, device)
    bd = torch.from_numpy(b).to(device)
    ws = torch.empty(B.workspace_bytes(A.n, restart, "fp64", precond), dtype=torch.uint8,
                     device=device)
    rows = []
    x_ref = None
    for fmt in formats:
        for vname in variants:
            kw = dict(restart=restart, fmt=fmt, tol=tol, maxiter=maxiter, precond=precond,
                      workspace=ws, hist=False, **VARIANTS[vname])
            B.solve(Ad, bd, **dict(kw, maxiter=min(maxiter, restart)))     # warm-up
            best, r = None, None
            for _ in range(repeats):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                r = B.solve(Ad, bd, **kw)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                best = dt if best is None else min(best, dt)
            tr = r.true_rel_res          # the solver's closing ||b - A x|| / ||b||
            if fmt == "fp64" and vname == "default":
                x_ref = r.x.clone()
            x_err = None if x_ref is None else \
                float(torch.linalg.norm(r.x - x_ref) / torch.linalg.norm(x_ref))
            row = dict(format=fmt, variant=vname, status=r.status, iterations=r.iterations,
                       reorths=r.reorths, restarts=r.restarts, seconds=best,
                       true_rel_res=tr, x_err=x_err)
            rows.append(row)
            if log:
                log(f"{fmt:6s} {vname:10s} it={r.iterations:6d} reorth={r.reorths:6d} "
                    f"{best * 1e3:8.1f} ms res={tr:.2e} x_err={x_err} status={r.status}")
    base = {r["variant"]: r for r in rows if r["format"] == "fp64"}
    ref = base.get("default")
    for r in rows:
        if ref is not None and ref["iterations"] > 0:
            r["overhead"] = r["iterations"] / ref["iterations"]
            r["speedup"] = ref["seconds"] / r["seconds"]
    return rows


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--system", default="convdiff7_128")
    ap.add_argument("--formats", default="fp64,fp32,fp16,fp16s,bf16,int16")
    ap.add_argument("--variants", default=",".join(VARIANTS))
    ap.add_argument("--etas", default="",
                    help="extra variants: step-7 thresholds to sweep, e.g. 0.5,0.2,0.1")
    ap.add_argument("--restart", type=int, default=100)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--maxiter", type=int, default=20000)
    ap.add_argument("--precond", default="none")
    ap.add_argument("--repeats", type=int, default=2)
    ap.add_argument("--json", default=None)
    a = ap.parse_args(argv)
    import torch
    A, b = system(a.system)
    names = [v for v in a.variants.split(",") if v]
    for e in [x for x in a.etas.split(",") if x]:
        VARIANTS[f"eta={e}"] = dict(eta=float(e))
        names.append(f"eta={e}")
    rows = ablate(A, b, a.formats.split(","), names, a.restart, a.tol,
                  a.maxiter, a.precond, a.repeats, torch.device("cuda:0"),
                  log=lambda s: print(s, file=sys.stderr, flush=True))
    out = dict(system=A.name, n=A.n, nnz=A.nnz, restart=a.restart, tol=a.tol,
               precond=a.precond, rows=rows)
    line = json.dumps(out)
    if a.json:
        with open(a.json, "w") as f:
            f.write(line + "\n")
    print(line, flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
