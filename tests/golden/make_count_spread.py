"""Writes count_spread.json: iteration counts of the oracle's Fig. 1 form and
of its one-pass arrangement of steps 5-10 (Gram-form re-dot, one update; the
arrangement the library's default uses on normal steps) over 21 rounding-level
perturbations of b, for the systems and formats of
tests/test_gpu_solve.py::test_solve_parity_compressed.  Two correct
implementations of one iteration differ by rounding only, as these two do;
the record shows how far their count statistics drift apart (means, medians,
and the rank test the GPU test applies).  Only the oracle runs here.

    python tests/golden/make_count_spread.py      # about 2 min on 8 cores
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as orc                                   # noqa: E402
from paper_2009_12101_amd import problems as P         # noqa: E402

FORMATS = ["fp32", "fp16", "bf16", "e4m3", "int32", "int16", "fp16s"]
PROBLEMS = [("poisson2d_64", 100), ("convdiff7_20", 30), ("lognormal27_12", 40)]
NPERT = 21


def perturbed(b, seed):
    return b * (1.0 + 1e-15 * np.random.default_rng(1000 + seed).standard_normal(b.size))


def main():
    from scipy.stats import mannwhitneyu
    out = {"npert": NPERT, "perturbation": "b (1 + 1e-15 z), z ~ N(0,1), numpy seed 1000 + s",
           "cases": {}}
    for name, m in PROBLEMS:
        A, b, _ = P.workload(name)
        for fmt in FORMATS:
            f1, op = [], []
            for s in range(NPERT):
                bp = perturbed(b, s)
                kw = dict(restart=m, fmt=fmt, tol=1e-10, maxiter=20000)
                f1.append(int(orc.gmres(A, bp, **kw)["iterations"]))
                op.append(int(orc.gmres(A, bp, variant=("gram", "onepass"), **kw)["iterations"]))
            rec = {"fig1": f1, "onepass": op,
                   "mean_rel_diff": abs(np.mean(f1) - np.mean(op)) / np.mean(f1),
                   "median_rel_diff": abs(np.median(f1) - np.median(op)) / np.median(f1),
                   "mannwhitney_p": (float(mannwhitneyu(f1, op).pvalue)
                                     if len(set(f1 + op)) > 1 else 1.0)}
            out["cases"][f"{name}_{fmt}"] = rec
            print(f"{name} {fmt}: mean diff {rec['mean_rel_diff']:.3f}, median diff "
                  f"{rec['median_rel_diff']:.3f}, p {rec['mannwhitney_p']:.3g}", flush=True)
    with open(os.path.join(HERE, "count_spread.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
