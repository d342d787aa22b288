"""Host-side pieces of the learned preconditioner (no GPU): the parameter
layout the binding uses matches the C header, and the training module's seeded
initialisation matches the oracle's (the same counter-based normal stream,
W3 and the biases zero, so the untrained P is Jacobi)."""
import os
import re

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_defines():
    text = open(os.path.join(ROOT, "include", "cbgmres.h")).read()
    return {k: int(v) for k, v in re.findall(r"#define (CBG_SPAI_\w+) (\d+)", text)}


def test_layout_constants_match_header():
    from paper_2009_12101_amd import _binding as B
    d = header_defines()
    assert d["CBG_SPAI_NFEAT"] == B.SPAI_NFEAT == 64
    assert d["CBG_SPAI_NHID"] == B.SPAI_NHID == 64
    assert d["CBG_SPAI_NOUT"] == B.SPAI_NOUT == 32
    nf, nh, no = 64, 64, 32
    assert d["CBG_SPAI_NPARAM"] == B.SPAI_NPARAM == nf * nh + nh + nh * nh + nh + nh * no + no
    assert d["CBG_SPAI_NWEIGHT"] == B.SPAI_NWEIGHT == nf * nh + nh * nh + nh * no
    assert d["CBG_SPAI_MAX_K"] == B.SPAI_MAX_K


def test_init_params_match_oracle():
    from oracle import spai as S
    from paper_2009_12101_amd.spai import init_params
    for seed in (0, 3):
        got = init_params(seed).astype(np.float64)
        o = S.init_params(seed)
        ref = np.concatenate([o["W1"].ravel(), o["b1"], o["W2"].ravel(), o["b2"],
                              o["W3"].ravel(), o["b3"]])
        assert np.array_equal(got, ref)
        assert np.all(got[-(64 * 32 + 32):] == 0.0)      # W3, b3: P starts as Jacobi
