"""Pins: checks that tie the CPU oracle to what the paper and plain mathematics
fix, without re-deriving the oracle's own arithmetic.

Every check takes an ``oracle.Oracle`` (the real one, or a copy compiled with a
planted mistake) and raises AssertionError on failure.  The kinds of pins:

* exact rationals (``fractions.Fraction``): the change ratio of eq. (1), bin
  membership of Sec. IV-B-1, bin centres, and the element-wise error bound
  (Sec. III, VI), each within the rounding the binary64 evaluation allows;
* closed forms on constructed inputs whose ratios sit exactly on bin centres,
  so the selected bins, the indices and the escapes are known by construction;
* brute force on tiny inputs: top-k by rank counting, the index-table bit
  string built character by character, block offsets by direct counting;
* library/textbook special cases: min/max of the valid ratios;
* the paper's printed numbers: Fig. 2's block layout and the CMIP
  compression-ratio example of Sec. V-B (fixtures under ``tests/golden``);
* the dynamic-programming optimum of Sec. V-D as an upper bound on coverage.
"""
from __future__ import annotations

import bisect
import math
import os
from fractions import Fraction

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read_golden(name: str) -> dict:
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = (s.strip() for s in line.split("=", 1))
            out[k] = float(v) if any(c in v for c in ".e") else int(v)
    return out


# ----------------------------------------------------------------- inputs

def mixture_case(n: int, seed: int, dtype=np.float64, E=1e-3):
    """Lognormal previous values with 0.1 % zeros; ratio mixture
    70 % N(0, 2E), 25 % N(10E, 5E), 5 % U[-0.5, 0.5]."""
    rng = np.random.default_rng(seed)
    prev = rng.lognormal(0.0, 1.0, n)
    prev[rng.choice(n, max(1, n // 1000), replace=False)] = 0.0
    u = rng.random(n)
    r = np.where(u < 0.7, rng.normal(0, 2 * E, n),
                 np.where(u < 0.95, rng.normal(10 * E, 5 * E, n), rng.uniform(-0.5, 0.5, n)))
    if dtype == np.float32:
        p32 = prev.astype(np.float32)
        return p32, (p32.astype(np.float64) * (1 + r)).astype(np.float32)
    return prev, prev * (1 + r)


def adversarial_case(dtype=np.float64):
    """Signed zeros, infinities, NaNs with payloads, subnormals, huge values,
    equal values, negative values, and ratios just inside/outside the cap."""
    tiny = np.finfo(dtype).smallest_subnormal
    big = np.finfo(dtype).max
    nan_payload = (np.array([0x7FF8DEADBEEF0001], np.uint64).view(np.float64)[0]
                   if dtype == np.float64 else
                   np.array([0x7FC0BEEF], np.uint32).view(np.float32)[0])
    prev = np.array([0.0, -0.0, 1.0, np.inf, 1.0, -np.inf, 1.0, tiny, 2.0, big, -3.0,
                     1.0, 1.0, 5.0, -5.0, 7.0, 1.0, 1.0, np.nan, 1.0], dtype)
    curr = np.array([1.0, 2.0, np.inf, 1.0, -np.inf, 2.0, nan_payload, 1.0, 2.0, big, -3.0,
                     -0.0, 0.0, 5.0 * 1.0005, -5.0 * 1.0005, 7.0, tiny, -tiny, 1.0,
                     nan_payload], dtype)
    return prev, curr


def cap_case(E: float):
    """Ratios just above and just below the validity cap |d| <= E * 2^50."""
    cap = math.ldexp(E, 50)
    prev = np.array([1.0, 1.0, 1.0, 1.0, 1.0, 1.0])
    curr = np.array([1.0 + 4 * cap, 1.0 + cap / 4, 1.0 - cap / 4, 1.0 - 4 * cap, 1.0, 1.0])
    return prev, curr, np.array([False, True, True, False, True, True])


def centred_case(counts: dict, dtype=np.float64, E_exp: int = -10, seed: int = 0):
    """Points whose ratios are exactly (2m+1)E for bin m (E a power of two, the
    grid anchored at 0 by a ratio-0 point that belongs to bin 0).  Every
    product and quotient involved is exact, so a point is compressible exactly
    when its bin is selected."""
    E = 2.0 ** E_exp
    rng = np.random.default_rng(seed)
    bins = []
    for m, c in sorted(counts.items()):
        bins += [m] * c
    bins = np.array(bins, np.int64)
    d = (2 * bins + 1).astype(np.float64) * E
    # the anchor: one point of bin 0 has ratio exactly 0
    first0 = int(np.flatnonzero(bins == 0)[0])
    d[first0] = 0.0
    order = rng.permutation(bins.size)
    bins, d = bins[order], d[order]
    p = (2.0 ** rng.integers(-3, 4, bins.size)) * np.where(rng.random(bins.size) < 0.3, -1, 1)
    q = p * (1.0 + d)
    return p.astype(dtype), q.astype(dtype), bins, E


# ------------------------------------------------------------- small helpers

def bits(a: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(a)
    return a.view(np.uint32 if a.dtype == np.float32 else np.uint64)


def F(x) -> Fraction:
    return Fraction(float(x))


def type_ulp(x: float, dtype) -> float:
    if dtype == np.float32:
        return float(np.spacing(np.float32(abs(x))))
    return math.ulp(abs(x))


# ------------------------------------------------------------------- pins

def pin_ratio_exact(o):
    """eq. (1): the ratio equals (q - p)/p to within two binary64 roundings."""
    for dt in (np.float64, np.float32):
        p, q = mixture_case(3000, 5, dt)
        d, v = o.ratio(p, q, 1e-3)
        for j in np.flatnonzero(v)[:800]:
            ex = (F(q[j]) - F(p[j])) / F(p[j])
            err = abs(F(d[j]) - ex)
            assert err <= 2 * Fraction(math.ulp(float(ex))) + Fraction(1, 2 ** 1074), \
                f"ratio mismatch at {j}: {d[j]} vs {float(ex)}"


def pin_validity(o):
    """Invalid points: zero or non-finite previous value, non-finite new value
    or ratio, |ratio| beyond E*2^50."""
    for dt in (np.float64, np.float32):
        p, q = adversarial_case(dt)
        _, v = o.ratio(p, q, 1e-3)
        with np.errstate(all="ignore"):
            pp, qq = p.astype(np.float64), q.astype(np.float64)
            r = (qq - pp) / pp
            exp = (pp != 0) & np.isfinite(pp) & np.isfinite(qq) & np.isfinite(r) & \
                (np.abs(r) <= math.ldexp(1e-3, 50))
        assert np.array_equal(v, exp), (v, exp)
    p, q, exp = cap_case(1e-3)
    _, v = o.ratio(p, q, 1e-3)
    assert np.array_equal(v, exp), (v, exp)


def pin_range_minmax(o):
    """Sec. IV-A: lo/hi are the minimum and maximum of the valid ratios."""
    for seed in range(3):
        p, q = mixture_case(2000, 100 + seed)
        d, v = o.ratio(p, q, 1e-3)
        nv, lo, hi = o.range(d, v)
        assert nv == int(v.sum())
        assert lo == d[v].min() and hi == d[v].max()
    d = np.array([3.0, -0.0, 0.0, 5.0, -1.0])
    nv, lo, hi = o.range(d, np.array([0, 1, 1, 0, 0], bool))
    assert nv == 2 and lo == 0.0 and math.copysign(1, lo) < 0 and math.copysign(1, hi) > 0


def pin_bins_exact(o):
    """Sec. IV-B-1: bins of width 2E anchored at lo; the binary64 bin id is the
    exact floor((d - lo)/(2E)) except within rounding of a bin edge."""
    for E in (1e-3, 1e-4, 0.05):
        p, q = mixture_case(3000, 7, E=E)
        d, v = o.ratio(p, q, E)
        _, lo, hi = o.range(d, v)
        m = o.bin_ids(d, v, lo, E)
        for j in np.flatnonzero(v)[:1500]:
            t = (F(d[j]) - F(lo)) / (2 * F(E))
            fl = math.floor(t)
            near = min(t - fl, fl + 1 - t) < Fraction(1, 10 ** 9) * (1 + t)
            assert m[j] == fl or (near and abs(m[j] - fl) <= 1), (j, m[j], float(t))
        assert np.all(m[~v] == -1)


def pin_histogram(o):
    """Counts sum to the number of valid points and equal a direct count of
    the exact bins (points near a bin edge excluded from the comparison)."""
    E = 1e-3
    p, q = mixture_case(4000, 9)
    d, v = o.ratio(p, q, E)
    _, lo, _ = o.range(d, v)
    m = o.bin_ids(d, v, lo, E)
    ids, cnt = o.histogram(m, v)
    assert int(cnt.sum()) == int(v.sum())
    assert np.all(np.diff(ids) > 0) and np.all(cnt > 0)
    exact = {}
    for j in np.flatnonzero(v):
        t = (F(d[j]) - F(lo)) / (2 * F(E))
        b = math.floor(t)
        exact[b] = exact.get(b, 0) + 1
    got = dict(zip(ids.tolist(), cnt.tolist()))
    diff = sum(abs(exact.get(b, 0) - got.get(b, 0)) for b in set(exact) | set(got))
    assert diff <= 2, diff  # at most an edge point moving between neighbours


def _brute_topk(ids, counts, k):
    """b is selected iff fewer than k nonzero bins precede it, where a bin
    precedes another when its count is larger, or equal with a lower id."""
    sel = []
    for i in range(len(ids)):
        ahead = 0
        for j in range(len(ids)):
            if counts[j] > counts[i] or (counts[j] == counts[i] and ids[j] < ids[i]):
                ahead += 1
        if ahead < k:
            sel.append(ids[i])
    return sorted(sel)


def pin_topk_brute(o):
    """Sec. IV-B-1: the k bins with most points, ties to the lower id."""
    rng = np.random.default_rng(3)
    for trial in range(40):
        nb = int(rng.integers(1, 60))
        ids = np.sort(rng.choice(10 ** 6, nb, replace=False)).astype(np.int64)
        counts = rng.integers(1, 6, nb).astype(np.uint32)  # many ties
        k = int(rng.integers(1, 40))
        sel, tau = o.topk(ids, counts, k)
        exp = _brute_topk(ids.tolist(), counts.tolist(), k)
        assert sel.tolist() == exp, (trial, sel, exp)
        if nb > k:
            assert tau == min(int(counts[ids.tolist().index(s)]) for s in exp)
        else:
            assert tau == 0


def pin_centred_literal(o):
    """Constructed bin-centred data: counts {0:4, 1:7, 2:5, 3:5, 4:5, 6:1},
    B = 2 (k = 3).  Top-3 = bin 1 (7 points) and, of the three bins tied at 5,
    the two lowest: bins 2 and 3.  Indices follow bin order: 1->0, 2->1, 3->2.
    M = floor(13E/2E) + 1 = 7.  Every point of a selected bin is reconstructed
    exactly; every other point escapes."""
    for dt in (np.float64, np.float32):
        p, q, b, E = centred_case({0: 4, 1: 7, 2: 5, 3: 5, 4: 5, 6: 1}, dt)
        res = o.compress(p, q, E, 2)
        h = res.info
        assert h["M"] == 7 and h["lo"] == 0.0 and h["k_used"] == 3 and h["n_nonzero"] == 6
        assert res.sel_ids.tolist() == [1, 2, 3]
        assert h["tau"] == 5
        want = np.where(b == 1, 0, np.where(b == 2, 1, np.where(b == 3, 2, 3)))
        assert np.array_equal(res.index, want), (res.index, want)
        ok = want != 3
        assert np.array_equal(bits(res.recon[ok]), bits(q[ok]))  # exact reconstruction
        assert np.array_equal(bits(res.incomp), bits(q[~ok]))
        cen = res.centers.astype(np.float64)
        assert cen.tolist() == [3 * E, 5 * E, 7 * E, 0.0]


def pin_centred_small_k(o):
    """B = 1 picks the single fullest bin (tie -> lower id); with fewer
    nonzero bins than k every nonzero bin is selected."""
    p, q, b, E = centred_case({0: 3, 2: 3, 4: 2})
    res = o.compress(p, q, E, 1)
    assert res.sel_ids.tolist() == [0] and res.info["k_used"] == 1
    assert np.array_equal(res.index, np.where(b == 0, 0, 1))
    p, q, b, E = centred_case({0: 1, 3: 2, 9: 1})
    res = o.compress(p, q, E, 4)
    assert res.sel_ids.tolist() == [0, 3, 9] and res.info["k_used"] == 3 and res.info["tau"] == 0
    assert np.array_equal(res.index, np.where(b == 0, 0, np.where(b == 3, 1, 2)))
    assert res.info["n_inc"] == 0


def pin_all_equal(o):
    """All ratios equal: one bin, M = 1, lo = hi = that ratio."""
    p = np.array([1.0, 2.0, 4.0, -8.0, 0.5] * 20)
    q = p * 1.25
    res = o.compress(p, q, 1e-3, 8)
    h = res.info
    assert h["M"] == 1 and h["n_nonzero"] == 1 and h["k_used"] == 1
    assert h["lo"] == 0.25 and h["hi"] == 0.25 and res.sel_ids.tolist() == [0]


def pin_error_bound_exact(o):
    """Sec. III/VI: every indexed point is reconstructed within E|prev|
    (exact rationals; slack for the binary64 comparison) and its ratio lies
    within E of its bin centre (plus the centre's rounding); centres equal
    lo + (2m+1)E rounded to the snapshot type."""
    cases = [(np.float64, 1e-3, 8), (np.float32, 1e-3, 8), (np.float32, 2.0 ** -23, 8),
             (np.float64, 1e-12, 6)]
    for dt, E, B in cases:
        p, q = mixture_case(3000, 21, dt, E=max(E, 1e-6) if dt == np.float32 else E)
        if dt == np.float32 and E < 1e-6:  # ratios comparable to float32 rounding
            rng = np.random.default_rng(22)
            p = rng.lognormal(0, 1, 3000).astype(np.float32)
            q = (p.astype(np.float64) * (1 + rng.normal(0, 3e-6, 3000))).astype(np.float32)
        res = o.compress(p, q, E, B)
        d, v = o.ratio(p, q, E)
        lo = res.info["lo"]
        for i, m in enumerate(res.sel_ids.tolist()):
            c = F(res.centers[i])
            ex = F(lo) + (2 * m + 1) * F(E)
            # two binary64 roundings (product, sum) plus the rounding to the type
            tol = Fraction(math.ulp(max(abs(lo), (2 * m + 1) * E))) + \
                Fraction(type_ulp(float(ex), dt))
            assert abs(c - ex) <= tol, (i, m)
        idx = res.index.astype(np.int64)
        comp = np.flatnonzero(idx != (1 << B) - 1)
        assert comp.size > 0
        slack = 1 + Fraction(1, 2 ** 50)
        for j in comp:
            r, pj, qj = F(res.recon[j]), F(p[j]), F(q[j])
            assert abs(r - qj) <= F(E) * abs(pj) * slack, (dt, E, j)
            c = F(res.centers[idx[j]])
            tol = F(E) * (1 + Fraction(1, 2 ** 40)) + 4 * Fraction(type_ulp(float(c), dt))
            assert abs(F(d[j]) - c) <= tol, (dt, E, j)


def pin_escapes_bitexact(o):
    """Sec. III-C: incompressible values are stored as they are, in element
    order (signed zeros and NaN payloads preserved); invalid points escape."""
    for dt in (np.float64, np.float32):
        p, q = adversarial_case(dt)
        res = o.compress(p, q, 1e-3, 4)
        esc = res.index == (1 << 4) - 1
        _, v = o.ratio(p, q, 1e-3)
        assert np.all(esc[~v])
        assert np.array_equal(bits(res.incomp), bits(q[esc]))
        assert np.array_equal(bits(res.recon[esc]), bits(q[esc]))


def pin_packing_bitstring(o):
    """Sec. IV-C: the index table is the concatenation of the B low bits of each
    index, least significant bit first, cut into 32-bit little-endian words."""
    for B in (1, 3, 8, 10, 13, 16):
        p, q = mixture_case(777, 40 + B)
        res = o.compress(p, q, 1e-3, B)
        s = "".join(format(int(i), f"0{B}b")[::-1] for i in res.index)
        s += "0" * (-len(s) % 32)
        words = [int(s[w:w + 32][::-1], 2) for w in range(0, len(s), 32)]
        assert res.packed.tolist() == words, B


def pin_block_offsets(o):
    """Sec. IV-C: block p starts at element p * floor(8 * bytes / B) and stores
    the number of incompressible points before it."""
    p, q = mixture_case(5000, 55)
    for B, bb in ((8, 64), (5, 100), (13, 333)):
        res = o.compress(p, q, 1e-3, B, block_bytes=bb)
        epb = (8 * bb) // B
        assert res.info["elems_per_block"] == epb
        assert res.info["n_blocks"] == -(-5000 // epb) == res.block_inc_off.size
        esc = res.index == (1 << B) - 1
        for blk in range(res.block_inc_off.size):
            assert res.block_inc_off[blk] == int(esc[: blk * epb].sum())


def pin_fig2_layout(o):
    """Fig. 2: UU of ASR, n = 3,758,400 points, B = 13, 1 MB blocks ->
    8192 centres, 645,277 indices per block, 6 blocks."""
    g = read_golden("fig2_asr_uu_header.txt")
    n = g["total_data_num"]
    p = np.ones(n, np.float32)
    res = o.compress(p, p, 1e-3, g["index_bits"], block_bytes=g["block_bytes"], recon=False)
    assert res.centers.size == g["bin_centers_number"]
    assert res.info["elems_per_block"] == g["elements_per_block"]
    assert res.info["n_blocks"] == g["block_table_dim"]


def pin_cmip_cr(o):
    """Sec. V-B: with 12-bit indices, 2 % incompressible float32 points and a
    2.2x lossless index-table stage the compression ratio is about 5.2; the
    size accounting (2^B centres + n B bits + alpha n L, eq. (6)) must match the
    returned arrays and reproduce the example."""
    g = read_golden("cmip_cr_example.txt")
    n = 500_000
    B = g["index_bits"]
    rng = np.random.default_rng(0)
    E = 2.0 ** -10
    # every valid ratio is exactly +E/2 except one anchor at -E/2, so the single
    # bin's centre is +E/2 and every valid point is reconstructed within E
    p = (2.0 ** rng.integers(-3, 4, n)).astype(np.float32)
    q = p * np.float32(1 + 2.0 ** -11)
    q[0] = p[0] * np.float32(1 - 2.0 ** -11)
    nz = int(round(g["incompressible_fraction"] * n))
    p[1 + rng.choice(n - 1, nz, replace=False)] = 0.0  # invalid -> incompressible
    res = o.compress(p, q, E, B, recon=False)
    h = res.info
    assert h["n_inc"] == nz
    L = g["value_bits"] // 8
    assert h["compressed_bytes"] == res.centers.size * L + res.packed.size * 4 + res.incomp.size * L
    assert res.packed.size == -(-n * B // 32)
    cr_idx = (n * L) / (res.packed.size * 4 / g["index_table_lossless_ratio"] + res.incomp.size * L)
    assert round(cr_idx, int(g["reported_digits"])) in (5.2, 5.3), cr_idx
    assert abs(cr_idx - g["reported_cr"]) < 0.1


def pin_roundtrip(o):
    """Sec. III-E and V-C: decompression reproduces the compressor's
    reconstruction bit for bit, and a partial decompression of [s, s+len)
    equals that slice, for ranges inside one block, across blocks, and empty."""
    rng = np.random.default_rng(77)
    for dt, B, bb in ((np.float64, 8, 256), (np.float32, 10, 1000), (np.float64, 3, 0)):
        p, q = mixture_case(6000, 78, dt)
        res = o.compress(p, q, 1e-3, B, block_bytes=bb)
        out, fl = o.decompress(res, p)
        assert fl == 0
        assert np.array_equal(bits(out), bits(res.recon))
        for _ in range(12):
            s = int(rng.integers(0, 6000))
            ln = int(rng.integers(0, 6000 - s + 1))
            part, fl = o.decompress_range(res, p, s, ln)
            assert fl == 0 and np.array_equal(bits(part), bits(out[s:s + ln]))
        part, fl = o.decompress_range(res, p, 6000, 0)
        assert part.size == 0


def pin_decode_flags(o):
    """A corrupt index table is reported, not silently decoded: an index in
    [k_used, ESC) sets the bad-index flag; too many escapes set the overrun
    flag."""
    p, q, b, E = centred_case({0: 1, 3: 2, 9: 1})
    res = o.compress(p, q, E, 4)
    res.packed[0] = (res.packed[0] & ~np.uint32(0xF)) | np.uint32(7)  # index 7 >= k_used = 3
    _, fl = o.decompress(res, p)
    assert fl & 1
    p2, q2 = adversarial_case()
    res2 = o.compress(p2, q2, 1e-3, 4)
    res2.packed[:] = np.uint32(0xFFFFFFFF)  # every index = ESC
    res2.info["n_inc"] = 1
    res2._info.n_inc = 1
    _, fl = o.decompress(res2, p2)
    assert fl & 2


def pin_empty_and_tiny(o):
    """n = 0 and n = 1, and an input with no valid point."""
    e = np.zeros(0)
    res = o.compress(e, e, 1e-3, 8)
    assert res.info["n"] == 0 and res.info["n_blocks"] == 0 and res.packed.size == 0
    res = o.compress(np.array([2.0]), np.array([2.0]), 1e-3, 8)
    assert res.info["k_used"] == 1 and res.sel_ids.tolist() == [0] and res.info["n_blocks"] == 1
    p = np.zeros(10)
    res = o.compress(p, p + 1, 1e-3, 8)
    assert res.info["n_inc"] == 10 and res.info["M"] == 0 and res.info["k_used"] == 0
    assert res.centers.tolist() == [0.0] * 256


def _dp_opt(vals, W, k):
    """Sec. V-D (text form): OPT(i, j) = max(OPT(i+1, j), OPT(i+c(i), j-1) + c(i)),
    c(i) = number of sorted values in [v_i, v_i + W]; OPT(N+1, .) = OPT(., 0) = 0."""
    v = sorted(vals)
    N = len(v)
    c = [bisect.bisect_right(v, v[i] + W) - i for i in range(N)]
    opt = [[0] * (k + 1) for _ in range(N + 2)]
    for i in range(N - 1, -1, -1):
        for j in range(1, k + 1):
            opt[i][j] = max(opt[i + 1][j], opt[i + c[i]][j - 1] + c[i])
    return opt[0][k]


def pin_dp_bound(o):
    """Sec. V-D: no choice of k bins of width 2E covers more ratios than the
    dynamic-programming optimum; on bin-aligned clusters top-k attains it."""
    for seed, B in ((1, 3), (2, 4), (3, 2)):
        p, q = mixture_case(1200, 300 + seed)
        res = o.compress(p, q, 1e-3, B)
        d, v = o.ratio(p, q, 1e-3)
        lo = res.info["lo"]
        m = o.bin_ids(d, v, lo, 1e-3)
        covered = int(np.isin(m[v], res.sel_ids).sum())
        opt = _dp_opt(d[v].tolist(), 2e-3 * (1 + 1e-9), (1 << B) - 1)
        assert covered <= opt, (covered, opt)
    p, q, b, E = centred_case({0: 6, 2: 9, 5: 4, 8: 7, 9: 2})
    res = o.compress(p, q, E, 2)
    d, v = o.ratio(p, q, E)
    opt = _dp_opt(d.tolist(), 2 * E * (1 - 1e-9), 3)
    assert opt == 22 and int((res.index != 3).sum()) == 22


def pin_choose_B_centred(o):
    """Sec. IV-B-2, eqs. (5)-(6), on bin-centred data with counts
    {0:4000, 1:7000, 2:5000, 3:5000, 4:5000, 6:1000} (n = 27,000, float64):
    the 2^B - 1 fullest bins hold 7000 (B = 1), 17,000 (B = 2) and all points
    (B >= 3), so in bits 8 file_size(B) = 64 * 2^B + 27,000 B + 64 (27,000 - held):
    1,307,128, 694,256, 81,512, 109,024, ... and B = 3 is chosen.  Every point
    of a selected bin is compressible here, so the estimated incompressible
    count of every B equals the n_inc of the compression with that B."""
    counts = {0: 4000, 1: 7000, 2: 5000, 3: 5000, 4: 5000, 6: 1000}
    p, q, _, E = centred_case(counts)
    n = p.size
    B, bits = o.choose_B(p, q, E, 1, 16)
    assert B == 3
    assert bits[1:5] == [1307128, 694256, 81512, 109024]
    for b in range(1, 17):
        held = min(sum(sorted(counts.values(), reverse=True)[: (1 << b) - 1]), n)
        assert bits[b] == 64 * (1 << b) + n * b + 64 * (n - held), b
    for b in (1, 2, 3, 5):
        est_inc = (bits[b] - 64 * (1 << b) - n * b) // 64
        assert est_inc == o.compress(p, q, E, b).info["n_inc"], b
    # a narrower range: the smallest estimate within it
    B2, bits2 = o.choose_B(p, q, E, 4, 6)
    assert B2 == 4 and bits2[4] == 109024 and bits2[3] == 0 and bits2[7] == 0


def pin_choose_B_invalid(o):
    """No valid point: alpha = 1 for every B, so the size 2^B L + n B / 8 + n L
    grows with B and the lower end of the range is chosen; float32 L = 4."""
    p = np.zeros(1000, np.float32)
    q = np.linspace(-1, 1, 1000).astype(np.float32)
    B, bits = o.choose_B(p, q, 1e-3, 5, 9)
    assert B == 5
    assert bits[5:10] == [8 * (1 << b) * 4 + 1000 * b + 32 * 1000 for b in range(5, 10)]


def pin_choose_B_ties_lowest(o):
    """Equal estimates choose the smaller B.  Float64 counts {0:124, 1:2, 2:2}
    (n = 128): B = 1 holds 124 points, 64 * 2 + 128 + 64 * 4 = 512 bits; B = 2
    holds all, 64 * 4 + 256 = 512 bits; B = 3 needs 64 * 8 + 384 = 896.  B = 1
    is chosen."""
    p, q, _, E = centred_case({0: 124, 1: 2, 2: 2})
    B, bits = o.choose_B(p, q, E, 1, 3)
    assert (B, bits[1], bits[2], bits[3]) == (1, 512, 512, 896)


def _ew_grid(shift: int, E: float, seed: int):
    """Ratios (j - shift) / 8 for j = 0..7, each four times, on previous
    values +-2^s: every ratio, product and centre below is exact."""
    rng = np.random.default_rng(seed)
    j = np.repeat(np.arange(8), 4)
    rng.shuffle(j)
    p = (2.0 ** rng.integers(-3, 4, j.size)) * np.where(rng.random(j.size) < 0.3, -1, 1)
    q = p * (1.0 + (j - shift) / 8.0)
    return p, q, j


def pin_ew_grid(o):
    """Sec. III-B / IV-B-3, equal-width binning: ratios (j - s)/8, j = 0..7,
    B = 3.  The k = 7 chunks of [lo, hi] = [-s/8, (7-s)/8] are 1/8 wide, ratio
    j falls in chunk j (the largest, on hi, in the last chunk 6), and each
    centre is the chunk midpoint lo + (i + 1/2)/8.  Every point is then 1/16
    of |p| from its centre: all compress at E = 1/16 and none at a hair less."""
    for shift in (0, 3):
        p, q, j = _ew_grid(shift, 1.0 / 16, 11 + shift)
        res = o.compress(p, q, 1.0 / 16, 3, binning="equal_width")
        h = res.info
        assert h["lo"] == -shift / 8 and h["hi"] == (7 - shift) / 8
        assert h["k_used"] == 7 and h["M"] == 7 and h["n_inc"] == 0
        assert res.index.tolist() == np.minimum(j, 6).tolist()
        want = [(-shift + i + 0.5) / 8 for i in range(7)] + [0.0]
        assert res.centers.tolist() == want
        res = o.compress(p, q, 1.0 / 16 - 2.0 ** -30, 3, binning="equal_width")
        assert res.info["n_inc"] == p.size and res.index.tolist() == [7] * p.size


def pin_ew_degenerate(o):
    """Equal-width binning with every valid ratio equal: the range has width
    0, every valid point takes chunk 0 and every centre is that ratio; points
    with a zero previous value escape.  With no valid point nothing is
    selected."""
    p = np.array([1.0, 2.0, 0.0, -8.0, 0.5] * 10)
    q = p * 1.25 + np.where(p == 0, 3.0, 0.0)
    res = o.compress(p, q, 1e-3, 4, binning="equal_width")
    zero = p == 0
    assert res.index.tolist() == np.where(zero, 15, 0).tolist()
    assert res.centers.tolist() == [0.25] * 15 + [0.0]
    assert res.info["n_inc"] == zero.sum() and res.info["lo"] == res.info["hi"] == 0.25
    res = o.compress(np.zeros(6), np.ones(6), 1e-3, 4, binning="equal_width")
    assert res.info["k_used"] == 0 and res.info["n_inc"] == 6 and res.centers.tolist() == [0.0] * 16


def pin_ew_membership(o):
    """Equal-width binning on a mixture, checked point by point with exact
    rationals: a valid point's chunk i holds its ratio, lo + i w <= d <=
    lo + (i+1) w with w = (hi - lo)/k (to the rounding of one division), a
    compressed point is within E |p| of its reconstruction, and decompression
    returns the reconstruction."""
    E = 1e-3
    for dt, B in ((np.float64, 4), (np.float32, 6)):
        p, q = mixture_case(700, 31, dt)
        res = o.compress(p, q, E, B, binning="equal_width")
        h = res.info
        k = (1 << B) - 1
        lo, hi = F(h["lo"]), F(h["hi"])
        w = (hi - lo) / k
        slack = (hi - lo) * Fraction(1, 2 ** 50)
        esc = k
        for jj in range(p.size):
            pj, qj = float(p[jj]), float(q[jj])
            code = int(res.index[jj])
            if code == esc:
                continue
            d = F(np.float64((qj - pj) / pj))
            assert lo + code * w - slack <= d <= lo + (code + 1) * w + slack
            assert abs(F(res.recon[jj]) - F(qj)) <= F(E) * abs(F(pj)) * (1 + Fraction(1, 2 ** 40))
        out, fl = o.decompress(res, p)
        assert fl == 0 and np.array_equal(bits(out), bits(res.recon))


def _za_case(counts: dict, E_exp: int = -10, seed: int = 0):
    """Ratios exactly 2mE for bin m (E a power of two) on previous values
    +-2^s: with the anchor at -E, bin m = floor((2mE + E) / 2E) = m and its
    centre -E + (2m + 1)E = 2mE, all exact."""
    E = 2.0 ** E_exp
    rng = np.random.default_rng(seed)
    bins = np.array([m for m, c in sorted(counts.items()) for _ in range(c)], np.int64)
    rng.shuffle(bins)
    p = (2.0 ** rng.integers(-3, 4, bins.size)) * np.where(rng.random(bins.size) < 0.3, -1, 1)
    q = p * (1.0 + 2.0 * bins * E)
    return p, q, bins, E


def pin_za_centred(o):
    """Zero-anchored bins: ratios 2mE fall in bin m, negative bins included;
    the 2^B - 1 fullest win, their centres are 2mE, their points reconstruct
    exactly, the others escape.  Header: lo = -E, hi = 0, M = 0."""
    p, q, bins, E = _za_case({-3: 5, -1: 30, 0: 50, 1: 30, 4: 2})
    res = o.compress(p, q, E, 2, binning="zero_anchored")
    h = res.info
    assert res.sel_ids.tolist() == [-1, 0, 1]
    assert h["lo"] == -E and h["hi"] == 0.0 and h["M"] == 0
    assert h["n_nonzero"] == 5 and h["tau"] == 30 and h["k_used"] == 3 and h["n_inc"] == 7
    assert res.centers.tolist() == [-2 * E, 0.0, 2 * E, 0.0]
    want = np.select([bins == -1, bins == 0, bins == 1], [0, 1, 2], 3)
    assert res.index.tolist() == want.tolist()
    kept = want != 3
    assert np.array_equal(bits(res.recon[kept]), bits(q[kept]))


def pin_za_signed_ties(o):
    """Equal counts in bins -2 and 2: the single bin of B = 1 is the lower
    id, -2 (a tie order on unsigned ids would take 2)."""
    p, q, _, E = _za_case({-2: 10, 2: 10, 5: 3}, seed=3)
    res = o.compress(p, q, E, 1, binning="zero_anchored")
    assert res.sel_ids.tolist() == [-2] and res.info["tau"] == 10


def pin_za_edges(o):
    """Bin edges at odd multiples of E: ratio -E opens bin 0, E - 2^-52
    stays in bin 0, E opens bin 1, -E - 2^-52 lies in bin -1."""
    E = 2.0 ** -10
    p = np.ones(4)
    q = 1.0 + np.array([-E, E - 2.0 ** -52, E, -E - 2.0 ** -52])
    res = o.compress(p, q, E, 8, binning="zero_anchored")
    assert res.sel_ids.tolist() == [-1, 0, 1]
    assert res.index.tolist() == [1, 1, 2, 0]


def pin_za_reduces_to_topk(o):
    """When the smallest valid ratio is exactly -E, the paper's anchor (the
    minimum) is -E too: every output equals the top-k compression's except
    the header's hi and M."""
    E = 2.0 ** -10
    rng = np.random.default_rng(8)
    n = 5000
    r = np.round(rng.normal(0, 4 * E, n) * 2 ** 20) / 2 ** 20
    r = np.maximum(r, -E)
    r[17] = -E
    p = (2.0 ** rng.integers(-3, 4, n)) * np.where(rng.random(n) < 0.3, -1, 1)
    q = p * (1.0 + r)
    a = o.compress(p, q, E, 4, binning="zero_anchored")
    b = o.compress(p, q, E, 4)
    assert b.info["lo"] == -E
    for f in ("n_inc", "n_nonzero", "k_used", "tau", "lo"):
        assert a.info[f] == b.info[f], f
    assert np.array_equal(a.packed, b.packed) and np.array_equal(a.sel_ids, b.sel_ids)
    assert np.array_equal(bits(a.centers), bits(b.centers))
    assert np.array_equal(bits(a.recon), bits(b.recon))
    out, fl = o.decompress(a, p)
    assert fl == 0 and np.array_equal(bits(out), bits(a.recon))


def _pack_codes(codes, B):
    """Pack B-bit codes LSB-first into 32-bit words, character by character."""
    bitstr = "".join(format(int(c), f"0{B}b")[::-1] for c in codes)
    return _words_of(bitstr)


def _words_of(bitstr):
    bitstr = bitstr + "0" * (-len(bitstr) % 32)
    return np.array([int(bitstr[i:i + 32][::-1], 2) for i in range(0, len(bitstr), 32)], np.uint32)


def _eg_len(v, k):
    """Exponential-Golomb codeword length of order k: 2 * bits(v + 2^k) - 1 - k."""
    return 2 * (v + (1 << k)).bit_length() - 1 - k


def _group_table(offsets):
    """The 16-bit group offsets of a sub-block as its first four words."""
    return [offsets[i] | (offsets[i + 1] << 16) for i in range(0, 8, 2)]


def pin_lossless_literal(o):
    """Lossless index stage on hand-worked tables.  Codes [0, 0, 1, 2, 0]
    (B = 2): ranks 0, 1, 2, order 0 (9 bits; order 1 12, order 2 15); the
    sub-block opens with its eight group offsets (group 0 at bit 128, the
    empty groups 1..7 where the codewords end, 137), then the codewords
    1 1 010 011 1 = 459, padded to 160 bits.  Codes 5x5, 2x4, 7x3, 0x2, 1x1
    (B = 3): ranks 5->0, 2->1, 7->2, 0->3, 1->4 and the unused codes after
    them in code order; order 0 (41 bits against 42, 47, 60); codewords 1,
    010, 011, 00100, 00110 (the bits of x after its leading one least
    significant first)."""
    e = o.lossless_encode(_pack_codes([0, 0, 1, 2, 0], 2), 5, 2)
    assert e["code_of_rank"].tolist() == [0, 1, 2, 3] and e["k"] == 0
    assert e["bits_k"] == [9, 12, 15] and e["sub_off"].tolist() == [0, 160]
    assert e["stream"].tolist() == [128 | 137 << 16] + [137 | 137 << 16] * 3 + [459]
    codes = [5] * 5 + [2] * 4 + [7] * 3 + [0] * 2 + [1]
    e = o.lossless_encode(_pack_codes(codes, 3), len(codes), 3)
    assert e["code_of_rank"].tolist() == [5, 2, 7, 0, 1, 3, 4, 6]
    assert e["k"] == 0 and e["bits_k"] == [41, 42, 47, 60]
    want = _words_of("1" * 5 + "010" * 4 + "011" * 3 + "00100" * 2 + "00110")
    assert e["stream"].tolist() == _group_table([128] + [169] * 7) + want.tolist()
    assert e["sub_off"].tolist() == [0, 192]
    assert np.array_equal(o.lossless_decode(e), _pack_codes(codes, 3))
    # equal totals: two codes, five each, cost 5 * 1 + 5 * 3 = 20 bits at
    # order 0 and 5 * 2 + 5 * 2 = 20 at order 1; the smaller order is taken
    e = o.lossless_encode(_pack_codes([0, 1] * 5, 1), 10, 1)
    assert e["bits_k"] == [20, 20] and e["k"] == 0


def pin_lossless_structure(o):
    """On random tables crossing sub-block boundaries (B = 1, 5, 8, 13, 16):
    ranks order the codes by count (ties by code), every order's total is
    the sum of textbook exponential-Golomb lengths, the chosen order has
    the fewest bits (the smaller on ties), each sub-block is its bits
    rounded up to a word, the total is at least the table's entropy, and
    decoding returns the table."""
    rng = np.random.default_rng(61)
    S = 1024
    for B, n in ((1, 3 * S + 17), (5, 2 * S), (8, 5 * S + 1), (13, S + 3), (16, 2 * S + 99)):
        K = 1 << B
        w = rng.pareto(1.2, K) + 1e-3
        codes = rng.choice(K, n, p=w / w.sum())
        e = o.lossless_encode(_pack_codes(codes, B), n, B)
        cnt = np.bincount(codes, minlength=K)
        order = sorted(range(K), key=lambda c: (-cnt[c], c))
        assert e["code_of_rank"].tolist() == order
        rank = np.empty(K, np.int64)
        rank[order] = np.arange(K)
        tot = [sum(int(cnt[c]) * _eg_len(int(rank[c]), k) for c in range(K) if cnt[c])
               for k in range(B + 1)]
        assert e["bits_k"] == tot
        k = e["k"]
        assert tot[k] == min(tot) and all(t > tot[k] for t in tot[:k])
        lens = np.array([_eg_len(int(r), k) for r in rank[codes]])
        sub = [128 + int(lens[i:i + S].sum()) for i in range(0, n, S)]
        off = np.concatenate([[0], np.cumsum([(b + 31) // 32 * 32 for b in sub])])
        assert e["sub_off"].tolist() == off.tolist()
        # each sub-block's group table: 128 plus the bits of the groups before
        words = e["stream"]
        for si in range(len(sub)):
            w0 = int(off[si]) // 32
            got = [(int(words[w0 + i // 2]) >> (16 * (i % 2))) & 0xFFFF for i in range(8)]
            gl = [int(lens[si * S + g * 128: min(si * S + (g + 1) * 128, n)].sum())
                  if si * S + g * 128 < n else 0 for g in range(8)]
            assert got == [128 + sum(gl[:g]) for g in range(8)], (B, si)
        pr = cnt[cnt > 0] / n
        assert tot[k] >= -(cnt[cnt > 0] * np.log2(pr)).sum() - 1e-6
        assert np.array_equal(o.lossless_decode(e), _pack_codes(codes, B))


def pin_lossless_single_symbol_and_corrupt(o):
    """One symbol only: rank 0, order 0, one bit per code (groups of 128
    bits after the group table); an empty table; a stream of zeros and a
    stream whose group offset is moved by one bit are refused."""
    n = 1024 + 5
    e = o.lossless_encode(_pack_codes([3] * n, 4), n, 4)
    assert e["k"] == 0 and e["code_of_rank"][0] == 3
    assert e["sub_off"].tolist() == [0, 1152, 1312]
    assert e["stream"][:4].tolist() == _group_table([128 + 128 * g for g in range(8)])
    assert e["stream"][4:36].tolist() == [0xFFFFFFFF] * 32
    assert e["stream"][36:41].tolist() == _group_table([128] + [133] * 7) + [0x1F]
    e0 = o.lossless_encode(np.zeros(0, np.uint32), 0, 6)
    assert e0["sub_off"].tolist() == [0] and e0["stream"].size == 0
    bad = dict(e)
    bad["stream"] = np.zeros_like(e["stream"])
    try:
        o.lossless_decode(bad)
    except ValueError:
        pass
    else:
        raise AssertionError("a stream of zeros decoded")
    bad = dict(e)
    bad["stream"] = e["stream"].copy()
    bad["stream"][1] += 1  # group 2 starts one bit late: group 2 runs short
    try:
        o.lossless_decode(bad)
    except ValueError:
        pass
    else:
        raise AssertionError("a moved group offset decoded")
    bad = dict(e)
    bad["stream"] = e["stream"].copy()
    # sub-block 1: the empty groups 1..7 start one bit late, so group 0 ends
    # one bit before its successor (every codeword still in bounds)
    bad["stream"][36] += 1 << 16
    bad["stream"][37:40] += 1 + (1 << 16)
    try:
        o.lossless_decode(bad)
    except ValueError:
        pass
    else:
        raise AssertionError("a group ending before its successor decoded")


ALL_PINS = [
    pin_ratio_exact, pin_validity, pin_range_minmax, pin_bins_exact, pin_histogram,
    pin_topk_brute, pin_centred_literal, pin_centred_small_k, pin_all_equal,
    pin_error_bound_exact, pin_escapes_bitexact, pin_packing_bitstring, pin_block_offsets,
    pin_fig2_layout, pin_cmip_cr, pin_roundtrip, pin_decode_flags, pin_empty_and_tiny,
    pin_dp_bound, pin_choose_B_centred, pin_choose_B_invalid, pin_choose_B_ties_lowest,
    pin_ew_grid, pin_ew_degenerate, pin_ew_membership,
    pin_za_centred, pin_za_signed_ties, pin_za_edges, pin_za_reduces_to_topk,
    pin_lossless_literal, pin_lossless_structure, pin_lossless_single_symbol_and_corrupt,
]
