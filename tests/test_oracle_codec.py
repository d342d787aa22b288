"""Pins of the oracle's storage codec (the accessor of Section 5.2).

Each float format is checked against something other than the oracle's own
rounding routine: exhaustive code-point round trips, brute-force nearest
neighbour over every representable value, numpy's single-rounding float16
cast, torch's float32->bfloat16/float8_e4m3fn casts on float32-exact inputs,
and hand-derived code points (tests/golden/codec_points.txt). The integer
formats are checked against the closed-form properties of the per-vector
scale sigma = max|v| / max_int.
"""
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "codec_points.txt")


def _hexfloat(s):
    s = s.strip()
    return float.fromhex(s) if ("0x" in s or "0X" in s) else float(s)


def _golden_rows():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            if not line.strip() or line.startswith("#"):
                continue
            fmt, vin, codes, scale = [c.strip() for c in line.split("|")]
            v = [_hexfloat(t) for t in vin.split(",")]
            if fmt.startswith("int"):
                c = [int(t) for t in codes.split(",")]
            else:
                c = [int(t, 16) for t in codes.split(",")]
            rows.append((fmt, v, c, _hexfloat(scale)))
    return rows


@pytest.mark.parametrize("row", _golden_rows(), ids=lambda r: f"{r[0]}:{r[1]}")
def test_golden_points(orc, row):
    fmt, v, codes, scale = row
    q, sc = orc.encode(fmt, np.array(v))
    assert [int(x) for x in q] == codes
    if fmt in ("e4m3", "int16", "int32"):
        assert sc == scale


# ---------------------------------------------------------------- fp16 ----

def _f16_finite_codes():
    c = np.arange(65536, dtype=np.uint32).astype(np.uint16)
    vals = c.view(np.float16).astype(np.float64)
    keep = np.isfinite(vals)
    return c[keep], vals[keep]


def test_fp16_roundtrip_exhaustive(orc):
    codes, vals = _f16_finite_codes()
    q, _ = orc.encode("fp16", vals)
    assert np.array_equal(q, codes)
    assert np.array_equal(orc.decode("fp16", q).view(np.uint64), vals.view(np.uint64))


def test_fp16_midpoints_round_to_even(orc):
    codes, vals = _f16_finite_codes()
    pos = vals[(vals >= 0)]
    pos = np.unique(pos)
    lo, hi = pos[:-1], pos[1:]
    mid = (lo + hi) / 2                      # exact in binary64
    q, _ = orc.encode("fp16", mid)
    qlo = lo.astype(np.float16).view(np.uint16)
    qhi = hi.astype(np.float16).view(np.uint16)
    expect = np.where(qlo % 2 == 0, qlo, qhi)
    assert np.array_equal(q, expect)
    up, _ = orc.encode("fp16", np.nextafter(mid, np.inf))
    dn, _ = orc.encode("fp16", np.nextafter(mid, -np.inf))
    assert np.array_equal(up, qhi) and np.array_equal(dn, qlo)


def test_fp16_matches_numpy_single_rounding(orc):
    rng = np.random.default_rng(1)
    # entries of unit vectors, down into the subnormal range
    v = rng.uniform(-1, 1, 200000) * 10.0 ** rng.uniform(-9, 0, 200000)
    q, _ = orc.encode("fp16", v)
    assert np.array_equal(q, v.astype(np.float16).view(np.uint16))


def test_fp16_double_rounding_trap(orc):
    # rounding through float32 first would give 1.0; one rounding gives 1+2^-10
    x = 1.0 + 2.0 ** -11 + 2.0 ** -40
    q, _ = orc.encode("fp16", np.array([x]))
    assert int(q[0]) == 0x3C01


# ---------------------------------------------------------------- bf16 ----

def _bf16_table():
    c = np.arange(65536, dtype=np.uint32)
    with np.errstate(invalid="ignore"):
        vals = (c << 16).view(np.float32).astype(np.float64)
    return c.astype(np.uint16), vals


def _nearest_even(x, codes, vals):
    """Brute-force nearest representable value (ties to the even code)."""
    keep = np.isfinite(vals) & (vals >= 0) & ~((vals == 0) & (codes != 0))
    c, v = codes[keep], vals[keep]
    order = np.argsort(v)
    c, v = c[order], v[order]
    a = np.abs(x)
    k = np.searchsorted(v, a)
    k = np.clip(k, 1, len(v) - 1)
    lo, hi = v[k - 1], v[k]
    dlo, dhi = a - lo, hi - a
    pick_hi = (dhi < dlo) | ((dhi == dlo) & (c[k] % 2 == 0))
    out = np.where(pick_hi, c[k], c[k - 1]).astype(np.uint32)
    sign_bit = np.uint32(1 << (8 * 2 - 1)) if codes.max() > 255 else np.uint32(0x80)
    out = np.where(np.signbit(x), out | sign_bit, out)
    return out


def test_bf16_brute_force_nearest(orc):
    codes, vals = _bf16_table()
    rng = np.random.default_rng(2)
    v = rng.uniform(-1, 1, 100000) * 10.0 ** rng.uniform(-40, 0, 100000)
    q, _ = orc.encode("bf16", v)
    assert np.array_equal(q.astype(np.uint32), _nearest_even(v, codes, vals))


def test_bf16_midpoints_and_torch(orc):
    import torch
    codes, vals = _bf16_table()
    fin = np.isfinite(vals) & (vals >= 0) & (vals <= 1.0)
    pos = np.unique(vals[fin])
    lo, hi = pos[:-1], pos[1:]
    mid = (lo + hi) / 2
    q, _ = orc.encode("bf16", mid)
    assert np.array_equal(q.astype(np.uint32), _nearest_even(mid, codes, vals))
    # torch's float32 -> bfloat16 cast is one rounding on float32-exact inputs
    rng = np.random.default_rng(3)
    x = (rng.uniform(-1, 1, 50000) * 10.0 ** rng.uniform(-30, 0, 50000)).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    q, _ = orc.encode("bf16", x.astype(np.float64))
    assert np.array_equal(q, ref)


# ---------------------------------------------------------------- e4m3 ----

def _e4m3_torch_table():
    import torch
    c = torch.arange(256, dtype=torch.uint8)
    return np.arange(256, dtype=np.uint32), c.view(torch.float8_e4m3fn).float().numpy().astype(np.float64)


def test_e4m3_decode_table_matches_torch(orc):
    codes, tvals = _e4m3_torch_table()
    mine = orc.decode("e4m3", codes.astype(np.uint8), 1.0)
    both_nan = np.isnan(mine) & np.isnan(tvals)
    assert np.array_equal(np.isnan(mine), np.isnan(tvals))
    assert np.array_equal(mine[~both_nan], tvals[~both_nan])
    assert mine[0x7E] == 448.0 and mine[0x01] == 2.0 ** -9 and mine[0x38] == 1.0
    # a stored vector's value is its scale times the code's value (Section 4)
    for k in (-13, 5):
        scaled = orc.decode("e4m3", codes.astype(np.uint8), 2.0 ** k)
        assert np.array_equal(scaled[~both_nan], tvals[~both_nan] * 2.0 ** k)


def test_e4m3_scale_and_brute_force(orc):
    codes, tvals = _e4m3_torch_table()
    rng = np.random.default_rng(4)
    for trial in range(50):
        n = int(rng.integers(1, 3000))
        v = rng.standard_normal(n) * 10.0 ** rng.uniform(-3, 0, n)
        v /= np.linalg.norm(v)
        q, sc = orc.encode("e4m3", v)
        # scale is a power of two with max|v| / scale in (224, 448]
        assert np.frexp(sc)[0] == 0.5
        top = np.abs(v).max() / sc
        assert 224.0 < top <= 448.0
        ref = _nearest_even(v / sc, codes, tvals)
        assert np.array_equal(q.astype(np.uint32), ref)


def test_e4m3_scale_when_the_top_entry_is_exactly_448(orc):
    # max|v| * 2^-k must lie in (224, 448]: at exactly 448 the scale stays
    for top, k in ((1.75, -8), (448.0 * 2.0 ** 5, 5)):
        v = np.array([top, 0.5 * top, -0.25 * top, 0.0])
        q, sc = orc.encode("e4m3", v)
        assert sc == 2.0 ** k
        assert list(q) == [0x7E, 0x76, 0xEE, 0x00]      # 448, 224, -112, 0


def test_e4m3_matches_torch_on_f32_exact(orc):
    import torch
    rng = np.random.default_rng(5)
    x = (rng.uniform(-1, 1, 20000) * 10.0 ** rng.uniform(-4, 0, 20000)).astype(np.float32)
    x[0] = 1.0
    q, sc = orc.encode("e4m3", x.astype(np.float64))
    scaled = (x.astype(np.float64) / sc).astype(np.float32)   # exact: power-of-two scale
    ref = torch.from_numpy(scaled).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    assert np.array_equal(q, ref)


# -------------------------------------------------------------- int16/32 --

@pytest.mark.parametrize("fmt,M", [("int16", 32767), ("int32", 2147483647)])
def test_fixed_point_closed_form(orc, fmt, M):
    rng = np.random.default_rng(6)
    for trial in range(20):
        n = int(rng.integers(1, 5000))
        v = rng.standard_normal(n)
        v /= np.linalg.norm(v)
        q, sigma = orc.encode(fmt, v)
        vinf = np.abs(v).max()
        assert sigma == vinf / M
        k = np.argmax(np.abs(v))
        assert abs(int(q[k])) == M and np.sign(q[k]) == np.sign(v[k])
        assert np.all(np.abs(q.astype(np.int64)) <= M)
        # |q_i - v_i/sigma| <= 1/2 up to the rounding of the division
        err = np.abs(q.astype(np.float64) - v / sigma)
        assert err.max() <= 0.5 + M * 2.0 ** -52
        dec = orc.decode(fmt, q, sigma)
        assert np.array_equal(dec, sigma * q.astype(np.float64))
        assert np.abs(dec - v).max() <= sigma * (0.5 + M * 2.0 ** -51)


def test_zero_vector_and_empty(orc):
    for fmt in ("fp64", "fp32", "fp16", "bf16", "e4m3", "int32", "int16"):
        q, sc = orc.encode(fmt, np.zeros(5))
        assert np.all(orc.decode(fmt, q, sc) == 0.0)
        q, sc = orc.encode(fmt, np.zeros(0))
        assert q.shape == (0,)


def test_fp32_is_a_plain_cast(orc):
    rng = np.random.default_rng(7)
    v = rng.standard_normal(100000) * 10.0 ** rng.uniform(-40, 0, 100000)
    q, _ = orc.encode("fp32", v)
    assert np.array_equal(q.view(np.uint32), v.astype(np.float32).view(np.uint32))
