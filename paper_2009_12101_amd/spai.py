"""Learned sparse-approximate-inverse preconditioner: training and inference.

An extension of the paper, which preconditions with scalar Jacobi (Section
6).  A per-row network (64 -> 64 -> 64 -> 32, ReLU, bf16 weights, fp32
biases, matrix-core products) maps features of row i of A to the values of
a right preconditioner P on A's pattern; the untrained network (last layer
zero) is exactly fp32 Jacobi.  Training minimises the mean of
||A P v - v||_2^2 over unit Arnoldi vectors v that plain GMRES produces on
the training matrices.

This module only orchestrates: every arithmetic step (features, forward and
backward passes, sparse products, Adam, the Arnoldi cycles that supply the
vectors) runs in libcbgmres.so.  Problem generation is CPU work on seeded
synthetic inputs.

Command line (one GPU):

    python -m paper_2009_12101_amd.spai --train-count 256 --train-grid 64 \\
        --epochs 30 --test-grid 128 --out weights.npz
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import sys
import time

import numpy as np

from . import _binding as B
from . import problems as P

VECTORS_PER_INSTANCE = 32      # v_1, v_4, ..., v_94 of one fp64 cycle of m = 100
VECTOR_STRIDE = 3
CYCLE = 100


def _torch():
    import torch
    return torch


@dataclasses.dataclass
class Instance:
    """One training matrix resident on the device."""
    A: "B.DeviceCSR"
    grid: tuple
    t_val: object          # values of A^T on A's pattern
    feat: object           # (n, 64) bf16 features
    V: object              # (n, K) fp16 Arnoldi vectors


class LearnedSPAI:
    """Parameters (fp32 masters + bf16 copy) and Adam state on the device."""

    def __init__(self, device, seed: int = 0):
        torch = _torch()
        self.device = device
        self.params = torch.from_numpy(init_params(seed)).to(device)
        self.weights = torch.empty(B.SPAI_NWEIGHT, dtype=torch.int16, device=device)
        B.spai_round_weights(self.params, self.weights)
        self.m1 = torch.zeros(B.SPAI_NPARAM, dtype=torch.float32, device=device)
        self.m2 = torch.zeros_like(self.m1)
        self.t = 0
        self.loss = torch.zeros(1, dtype=torch.float64, device=device)
        self.grad = torch.zeros(B.SPAI_NPARAM, dtype=torch.float64, device=device)

    # ------------------------------------------------------------ training
    def step(self, batch, lr: float = 1e-3, ws=None) -> float:
        """One Adam step on the mean loss over every vector of the batch."""
        K = sum(inst.V.shape[1] for inst in batch)
        for i, inst in enumerate(batch):
            B.spai_loss_grad(inst.A, inst.t_val, inst.grid, inst.feat, self.weights,
                             self.params, inst.V, 1.0 / K, self.loss, self.grad,
                             accumulate=i > 0, ws=ws)
        self.t += 1
        B.adam_step(self.params, self.m1, self.m2, self.weights, self.grad, self.t, lr=lr)
        return self.loss

    def train(self, data, epochs: int, batch: int = 8, lr: float = 1e-3, seed: int = 0,
              log=None):
        """Epochs over `data` in shuffled batches; returns the mean batch loss
        of each epoch."""
        torch = _torch()
        n_max = max(inst.A.n for inst in data)
        nnz_max = max(inst.A.nnz for inst in data)
        k_max = max(inst.V.shape[1] for inst in data)
        ws = torch.empty(B.spai_workspace_bytes(n_max, nnz_max, k_max), dtype=torch.uint8,
                         device=self.device)
        rng = np.random.default_rng(seed)
        history = []
        for ep in range(epochs):
            order = rng.permutation(len(data))
            losses = torch.zeros(0, dtype=torch.float64, device=self.device)
            parts = []
            for s in range(0, len(order), batch):
                self.step([data[i] for i in order[s:s + batch]], lr=lr, ws=ws)
                parts.append(self.loss.clone())
            losses = torch.cat(parts)
            mean = float(losses.mean().item())
            history.append(mean)
            if log:
                log(f"epoch {ep + 1}/{epochs}: mean batch loss {mean:.6e}")
        return history

    # ----------------------------------------------------------- inference
    def build(self, A: "B.DeviceCSR", grid, ws=None):
        """P values (nnz fp32) for CBG_PC_SPARSE."""
        return B.learned_build(A, grid, self.weights, self.params, ws=ws)

    def build_stencil(self, A: "B.DeviceCSR", grid, ws=None, out=None):
        """The stored form for CBG_PC_STENCIL: float16 corrections on the
        27-point slots (27 * basis_ld(n) codes, slot-major)."""
        return B.learned_build_stencil(A, grid, self.weights, self.params, p_stencil=out, ws=ws)

    # ----------------------------------------------------------- storage
    def save(self, path: str):
        np.savez(path, params=self.params.cpu().numpy(), m1=self.m1.cpu().numpy(),
                 m2=self.m2.cpu().numpy(), t=np.array([self.t]))

    def load(self, path: str):
        torch = _torch()
        with np.load(path, allow_pickle=False) as z:
            self.params.copy_(torch.from_numpy(z["params"].astype(np.float32)))
            self.m1.copy_(torch.from_numpy(z["m1"].astype(np.float32)))
            self.m2.copy_(torch.from_numpy(z["m2"].astype(np.float32)))
            self.t = int(z["t"][0])
        B.spai_round_weights(self.params, self.weights)
        return self


def init_params(seed: int) -> np.ndarray:
    """He-normal W1 (64x64) and W2 (64x64) from the seeded counter-based
    normal stream, stored fp32; W3, b1, b2, b3 zero (so P starts as Jacobi)."""
    nf, nh, no = B.SPAI_NFEAT, B.SPAI_NHID, B.SPAI_NOUT
    z = P.normal(seed, P.STREAM_WEIGHTS, nf * nh + nh * nh)
    w1 = (z[:nf * nh] * np.sqrt(2.0 / nf)).astype(np.float32)
    w2 = (z[nf * nh:] * np.sqrt(2.0 / nh)).astype(np.float32)
    out = np.zeros(B.SPAI_NPARAM, dtype=np.float32)
    out[:nf * nh] = w1
    o2 = nf * nh + nh
    out[o2:o2 + nh * nh] = w2
    return out


def _generate(args):
    N, seed = args
    A = P.lognormal27(N, seed)
    return A, P.rhs_uniform(A.n, seed)


def make_instances(seeds, N: int, device, pool=None, log=None):
    """Training matrices (27-point lognormal diffusion on N^3, one per seed):
    generated on the host (in `pool`, a multiprocessing pool forked before
    the GPU was touched, or serially), then on the device one fp64-basis
    GMRES cycle (m = 100, M = I, b ~ U[-1, 1] of the same seed) whose basis
    vectors v_1, v_4, ..., v_94 are kept as fp16."""
    torch = _torch()
    out = []
    ws = None
    t0 = time.time()
    jobs = [(N, int(s)) for s in seeds]
    gen = pool.imap(_generate, jobs) if pool is not None else map(_generate, jobs)
    for A, b in gen:
        Ad = B.DeviceCSR.from_host(A, device)
        need = B.workspace_bytes(A.n, CYCLE, "fp64")
        if ws is None or ws.numel() < need:
            ws = torch.empty(need, dtype=torch.uint8, device=device)
        r = B.solve(Ad, torch.from_numpy(b).to(device), restart=CYCLE, fmt="fp64",
                    tol=0.0, maxiter=CYCLE, workspace=ws, hist=False)
        if r.iterations != CYCLE:
            raise RuntimeError(f"{A.name}: the cycle ended after {r.iterations} steps")
        off, _ = B.workspace_basis(A.n, CYCLE, "fp64")
        ld = B.basis_ld(A.n)
        Vws = ws[off:off + CYCLE * ld * 8].view(torch.float64)
        V = B.spai_pack(Vws, ld, A.n, VECTORS_PER_INSTANCE, 0, VECTOR_STRIDE)
        sws = torch.empty(B.spai_workspace_bytes(A.n, A.nnz, 0), dtype=torch.uint8,
                          device=device)
        out.append(Instance(Ad, A.grid, B.csr_transpose_values(Ad, ws=sws),
                            B.spai_features(Ad, A.grid, ws=sws), V))
        if log and len(out) % 32 == 0:
            log(f"{len(out)}/{len(jobs)} training instances ({time.time() - t0:.1f}s)")
    torch.cuda.synchronize()
    return out


def compare(model: LearnedSPAI, A, b, fmt="fp16", restart=100, tol=1e-10, maxiter=20000,
            repeats=1, device="cuda", plain_fp64=False):
    """Time to solution of CB-GMRES with M = I, Jacobi, block-Jacobi (4 x 4
    blocks, adaptive or fp64 storage), the learned P in its stored form
    ("learned": float16 corrections on the 27-point slots, applied in the
    normalising pass) and as fp32 values on A's pattern ("learned_csr", one
    more CSR pass per step), each build (features to stored values)
    included in the time, all with the `fmt` basis; with plain_fp64 also
    plain GMRES (fp64 basis, M = I).  Block-Jacobi's set-up (inverting the
    blocks) is part of its solve."""
    torch = _torch()
    Ad = B.DeviceCSR.from_host(A, device)
    bd = torch.from_numpy(b).to(device)
    need = max(B.workspace_bytes(A.n, restart, fmt, "sparse"),
               B.workspace_bytes(A.n, restart, fmt, "stencil"),
               B.workspace_bytes(A.n, restart, fmt, "block_jacobi"),
               B.workspace_bytes(A.n, restart, "fp64", "none") if plain_fp64 else 0)
    ws = torch.empty(need, dtype=torch.uint8, device=device)
    sws = torch.empty(B.spai_workspace_bytes(A.n, A.nnz, 0), dtype=torch.uint8, device=device)
    rows = {}
    kinds = ["none", "jacobi", "block_jacobi", "block_jacobi_fp64", "learned", "learned_csr"] + \
        (["plain_fp64"] if plain_fp64 else [])
    codes = torch.empty(27 * B.basis_ld(A.n), dtype=torch.int16, device=device)
    for kind in kinds:
        best = None
        for _ in range(repeats + 1):            # the first run warms up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if kind == "learned":
                model.build_stencil(Ad, A.grid, ws=sws, out=codes)
                r = B.solve(Ad, bd, restart=restart, fmt=fmt, tol=tol, maxiter=maxiter,
                            precond="stencil", p_stencil=codes, grid=A.grid, fallback=True,
                            workspace=ws, hist=False)
            elif kind == "learned_csr":
                pv = model.build(Ad, A.grid, ws=sws)
                r = B.solve(Ad, bd, restart=restart, fmt=fmt, tol=tol, maxiter=maxiter,
                            precond="sparse", p_val=pv, fallback=True, workspace=ws,
                            hist=False)
            elif kind.startswith("block_jacobi"):
                # 4 x 4 blocks; stored at the adaptive precision, or all fp64
                r = B.solve(Ad, bd, restart=restart, fmt=fmt, tol=tol, maxiter=maxiter,
                            precond="block_jacobi", pc_block=4,
                            pc_prec=64 if kind.endswith("fp64") else 16, workspace=ws,
                            hist=False)
            elif kind == "plain_fp64":
                r = B.solve(Ad, bd, restart=restart, fmt="fp64", tol=tol, maxiter=maxiter,
                            precond="none", workspace=ws, hist=False)
            else:
                r = B.solve(Ad, bd, restart=restart, fmt=fmt, tol=tol, maxiter=maxiter,
                            precond=kind, workspace=ws, hist=False)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        rows[kind] = dict(seconds=best, iterations=r.iterations, restarts=r.restarts,
                          status=r.status, true_rel_res=r.true_rel_res,
                          fell_back=r.fell_back)
    return rows


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--train-count", type=int, default=256)
    ap.add_argument("--train-grid", type=int, default=64)
    ap.add_argument("--first-seed", type=int, default=1)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--init-seed", type=int, default=0)
    ap.add_argument("--test-grid", type=int, default=128)
    ap.add_argument("--test-system", default="lognormal27", choices=["lognormal27", "convdiff7"],
                    help="held-out system family (the network is trained on lognormal27)")
    ap.add_argument("--test-seed", type=int, default=0)
    ap.add_argument("--format", default="fp16",
                    help="basis storage of the test solves (comma list allowed)")
    ap.add_argument("--restart", type=int, default=100)
    ap.add_argument("--plain-fp64", action="store_true",
                    help="also time plain GMRES (fp64 basis, M = I) on the test system")
    ap.add_argument("--repeats", type=int, default=1)
    ap.add_argument("--workers", type=int, default=8,
                    help="host processes generating the training matrices")
    ap.add_argument("--out", default=None, help="save the trained parameters (.npz)")
    ap.add_argument("--load", default=None, help="skip training; load parameters (.npz)")
    ap.add_argument("--json", default=None, help="write the report here")
    a = ap.parse_args(argv)
    # the generator processes are forked before anything touches the GPU
    pool = None
    if not a.load and a.workers > 1:
        import multiprocessing
        pool = multiprocessing.get_context("fork").Pool(a.workers)
    torch = _torch()
    dev = torch.device("cuda:0")

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    model = LearnedSPAI(dev, a.init_seed)
    report = dict(train_count=a.train_count, train_grid=a.train_grid, epochs=a.epochs,
                  batch=a.batch, lr=a.lr)
    if a.load:
        model.load(a.load)
    else:
        t0 = time.time()
        data = make_instances(range(a.first_seed, a.first_seed + a.train_count), a.train_grid,
                              dev, pool, log)
        if pool is not None:
            pool.close()
            pool.join()
        report["data_seconds"] = time.time() - t0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        report["loss_history"] = model.train(data, a.epochs, a.batch, a.lr, log=log)
        torch.cuda.synchronize()
        report["train_seconds"] = time.perf_counter() - t0
        del data
        if a.out:
            model.save(a.out)
    if a.test_grid > 0:
        A = (P.lognormal27(a.test_grid, a.test_seed) if a.test_system == "lognormal27"
             else P.convdiff7(a.test_grid))
        b = P.rhs_uniform(A.n, a.test_seed)
        report["test"] = []
        for i, fmt in enumerate(a.format.split(",")):
            rows = compare(model, A, b, fmt=fmt, restart=a.restart, repeats=a.repeats,
                           device=dev, plain_fp64=a.plain_fp64 and i == 0)
            report["test"].append(dict(system=A.name, n=A.n, nnz=A.nnz, format=fmt,
                                       restart=a.restart, **rows))
            for k, v in rows.items():
                log(f"{fmt} {k:10s}: {v['seconds'] * 1e3:9.1f} ms  it={v['iterations']}  "
                    f"res={v['true_rel_res']:.2e}  status={v['status']}")
    line = json.dumps(report)
    if a.json:
        with open(a.json, "w") as f:
            f.write(line + "\n")
    print(line, flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
