"""HIP library vs the CPU oracle, element by element (bit-exact), through the
C ABI.  Sizes span several tiles and ragged tails; edge cases cover empty and
one-element inputs, every index width, invalid points, the tail (out-of-
window) path of the histogram and the capacity flag."""
import math

import numpy as np
import pytest
import torch

import oracle
from gpu_util import bits, compare_compress, compare_decompress, gpu_compress, to_np
from paper_1703_02438_amd import inputs
from pins import adversarial_case, centred_case, mixture_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nk():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1703_02438_amd.numarck as nk
    return nk


def _ranges(n, rng, k=6, epb=None):
    out = [(0, n), (0, 0), (n, 0)]
    for _ in range(k):
        s = int(rng.integers(0, n + 1))
        out.append((s, int(rng.integers(0, n - s + 1))))
    if epb and epb >= 5 and n > epb + 10:
        out.append((epb - 5, 10))  # crosses a block boundary
    return out


def test_mixture_64cubed_fp64(nk):
    """64^3 float64, lognormal prev with 0.1 % zeros, 3-component ratio
    mixture, E = 1e-3, B = 8."""
    prev, curr = inputs.mixture_pair(64 ** 3, seed=1704)
    prev, curr = prev.numpy(), curr.numpy()
    c, o, p = compare_compress(nk, prev, curr, 1e-3, 8, label="mixture 64^3")
    compare_decompress(nk, c, o, p, prev, _ranges(prev.size, np.random.default_rng(1)))


def test_mixture_64cubed_fp32(nk):
    prev, curr = inputs.mixture_pair(64 ** 3, seed=1704, dtype=torch.float32)
    prev, curr = prev.numpy(), curr.numpy()
    c, o, p = compare_compress(nk, prev, curr, 1e-3, 8, label="mixture 64^3 f32")
    compare_decompress(nk, c, o, p, prev, _ranges(prev.size, np.random.default_rng(2)))


@pytest.mark.parametrize("n", [0, 1, 2, 3, 5, 31, 33, 4095, 4096, 4097, 12289, 100003])
@pytest.mark.parametrize("dt", [np.float64, np.float32])
def test_ragged_sizes(nk, n, dt):
    prev, curr = mixture_case(max(n, 1), 1000 + n, dt)
    prev, curr = prev[:n], curr[:n]
    B = 3 if n < 100 else 10
    c, o, p = compare_compress(nk, prev, curr, 1e-3, B, label="ragged")
    compare_decompress(nk, c, o, p, prev, _ranges(n, np.random.default_rng(n)))


@pytest.mark.parametrize("B", [1, 2, 3, 5, 8, 10, 12, 13, 15, 16])
def test_index_widths(nk, B):
    prev, curr = mixture_case(50021, 77 + B, np.float64, E=1e-4)
    c, o, p = compare_compress(nk, prev, curr, 1e-4, B, label="bits")
    compare_decompress(nk, c, o, p, prev, _ranges(prev.size, np.random.default_rng(B)))


@pytest.mark.parametrize("dt", [np.float64, np.float32])
def test_adversarial_values(nk, dt):
    """Signed zeros, infinities, NaN payloads, subnormals, huge values, tiled
    and shuffled among ordinary points."""
    ap, aq = adversarial_case(dt)
    mp, mq = mixture_case(30000, 5, dt)
    rng = np.random.default_rng(9)
    prev = np.concatenate([mp, np.tile(ap, 200)])
    curr = np.concatenate([mq, np.tile(aq, 200)])
    perm = rng.permutation(prev.size)
    prev, curr = prev[perm], curr[perm]
    c, o, p = compare_compress(nk, prev, curr, 1e-3, 6, label="adversarial")
    compare_decompress(nk, c, o, p, prev, _ranges(prev.size, rng))


@pytest.mark.parametrize("dt", [np.float64, np.float32])
def test_centred_ties(nk, dt):
    """Bin-centred data with ties across the top-k cut (known answer)."""
    counts = {0: 4, 1: 7, 2: 5, 3: 5, 4: 5, 6: 1}
    counts = {m: c * 1000 for m, c in counts.items()}
    prev, curr, b, E = centred_case(counts, dt)
    c, o, p = compare_compress(nk, prev, curr, E, 2, label="centred")
    assert to_np(c.bin_ids)[:3].tolist() == [1, 2, 3]
    compare_decompress(nk, c, o, p, prev)


@pytest.mark.parametrize("base,step", [(300_000, 7), (70, 1), (5_000, 3)])
def test_select_ties_at_large_counts(nk, base, step):
    """Top-k with ties across the cut at counts of every size: 40 bins whose
    counts take five values base + step j, eight bins each, and k = 15
    (B = 4), so tau is the second-largest value and 7 of its 8 bins are
    taken.  The counts' log-scale key leaves 0, 6 or 12 low bits to resolve
    (base 70, 5000, 300000), the last in two passes of 11 and 1 bits."""
    E = 2.0 ** -10
    counts = np.array([base + step * (m % 5) for m in range(40)])
    rng = np.random.default_rng(base)
    b = np.repeat(np.arange(40), counts)
    d = (2 * b + 1).astype(np.float64) * E
    d[0] = 0.0  # the anchor: a ratio-0 point of bin 0
    order = rng.permutation(b.size)
    d = d[order]
    p = (2.0 ** rng.integers(-3, 4, b.size)) * np.where(rng.random(b.size) < 0.3, -1, 1)
    prev, curr = p.astype(np.float32), (p * (1.0 + d)).astype(np.float32)
    c, o, _ = compare_compress(nk, prev, curr, E, 4, label=f"ties at {base}")
    h = c.header()
    assert h.tau == base + 3 * step and h.k_used == 15
    # the 8 bins of the largest count, then the first 7 of the next in id order
    top = sorted([m for m in range(40) if m % 5 == 4] + [m for m in range(40) if m % 5 == 3][:7])
    assert to_np(c.bin_ids)[:15].tolist() == top


def test_all_invalid(nk):
    prev = np.zeros(9000)
    curr = np.linspace(-1, 1, 9000)
    c, o, p = compare_compress(nk, prev, curr, 1e-3, 8, label="invalid")
    assert c.header().n_inc == 9000 and c.header().k_used == 0
    compare_decompress(nk, c, o, p, prev)


def test_all_equal(nk):
    prev = np.tile(np.array([1.0, 2.0, 4.0, -8.0, 0.5]), 3000)
    c, o, p = compare_compress(nk, prev, prev * 1.25, 1e-3, 8, label="equal")
    assert c.header().M == 1


@pytest.mark.parametrize("bb", [1, 2, 64, 1000, 65536])
def test_small_blocks(nk, bb):
    prev, curr = mixture_case(20011, 31, np.float32)
    B = 8
    c, o, p = compare_compress(nk, prev, curr, 1e-3, B, block_bytes=bb, label="blocks")
    epb = 8 * bb // B
    compare_decompress(nk, c, o, p, prev, _ranges(prev.size, np.random.default_rng(bb), 8, epb))


def tail_case(n=200_000, seed=3, dt=np.float64):
    """Ratios spread over [-0.5, 0.5] with E = 1e-5 (M = 50,000 bins > window):
    clusters at +0.4 and -0.45 lie outside the on-chip window around 0, so
    selected bins come from the tail below and above the window."""
    rng = np.random.default_rng(seed)
    prev = rng.lognormal(0, 1, n)
    u = rng.random(n)
    r = np.where(u < 0.3, rng.normal(0, 1e-5, n),
                 np.where(u < 0.5, rng.normal(0.4, 3e-5, n),
                          np.where(u < 0.7, rng.normal(-0.45, 3e-5, n), rng.uniform(-0.5, 0.5, n))))
    curr = prev * (1 + r)
    return prev.astype(dt), curr.astype(dt)


@pytest.mark.parametrize("B", [8, 12, 16])
def test_tail_bins_selected(nk, B):
    prev, curr = tail_case()
    c, o, p = compare_compress(nk, prev, curr, 1e-5, B, label="tail")
    h = c.header()
    assert h.M > 16384 and h.tail_count > 0
    ids = to_np(c.bin_ids)[: h.k_used]
    wb = h.window_base
    assert (ids < wb).any() and (ids >= wb + 16384).any()  # selected on both sides
    compare_decompress(nk, c, o, p, prev, _ranges(prev.size, np.random.default_rng(B)))


def test_tail_capacity(nk):
    """A workspace with a small tail capacity: exact while the tail fits, the
    overflow flag when it does not."""
    prev, curr = tail_case(60_000, 4)
    big = gpu_compress(nk, prev, curr, 1e-5, 8)[0]
    T = big.header().tail_count
    assert T > 1000
    ws = torch.empty(nk.numarck_workspace_bytes_tail(prev.size, nk.F64, T), dtype=torch.uint8,
                     device="cuda")
    c, _, _ = gpu_compress(nk, prev, curr, 1e-5, 8, ws=ws)
    assert c.header().flags == 0
    assert np.array_equal(to_np(c.packed), to_np(big.packed))
    ws = torch.empty(nk.numarck_workspace_bytes_tail(prev.size, nk.F64, T // 2), dtype=torch.uint8,
                     device="cuda")
    c, _, _ = gpu_compress(nk, prev, curr, 1e-5, 8, ws=ws)
    assert c.header().flags & nk.FLAG_TAIL_OVERFLOW


def test_flash_like_small(nk):
    """32^3 FLASH-like pair: smooth ratios plus Cauchy shocks -> a huge bin
    range with a sparse tail."""
    s = inputs.FlashSeries(edge=32, seed=11)
    prev = s.x.clone().numpy()
    curr = s.step().numpy()
    c, o, p = compare_compress(nk, prev, curr, 1e-3, 8, label="flash")
    assert c.header().M > 16384
    compare_decompress(nk, c, o, p, prev, _ranges(prev.size, np.random.default_rng(5)))


@pytest.mark.parametrize("spill", [False, True])
def test_climate_like_small(nk, spill):
    kw = dict(outlier_lo=-0.9, outlier_hi=1.5) if spill else {}
    s = inputs.ClimateSeries(nlat=180, nlon=360, seed=12, **kw)
    prev = s.x.clone().numpy()
    curr = s.step().numpy()
    c, o, p = compare_compress(nk, prev, curr, 1e-4, 10, label="climate")
    compare_decompress(nk, c, o, p, prev, _ranges(prev.size, np.random.default_rng(6)))


def test_deterministic(nk):
    prev, curr = tail_case(120_000, 8)
    a = gpu_compress(nk, prev, curr, 1e-5, 12)[0]
    b = gpu_compress(nk, prev, curr, 1e-5, 12)[0]
    ninc = a.header().n_inc
    assert ninc == b.header().n_inc
    assert torch.equal(a.incomp[:ninc].view(torch.uint8), b.incomp[:ninc].view(torch.uint8))
    for f in ("packed", "centers", "block_inc_off", "recon", "bin_ids", "hdr"):
        assert torch.equal(getattr(a, f).view(torch.uint8), getattr(b, f).view(torch.uint8)), f


def test_decode_flags(nk):
    prev, curr, b, E = centred_case({0: 1, 3: 2, 9: 1})
    c, p, q = gpu_compress(nk, prev, curr, E, 4)
    c.packed[0] = (c.packed[0] & ~0xF) | 7  # index 7 >= k_used = 3
    _, fl = nk.decompress(c, p)
    assert int(fl.item()) & nk.FLAG_BAD_INDEX
    c2, p2, _ = gpu_compress(nk, prev, curr, E, 4)
    c2.packed.fill_(-1)  # every index is the escape code
    _, fl = nk.decompress(c2, p2)
    assert int(fl.item()) & nk.FLAG_INC_OVERRUN


def _range_at(nk, c, p, s, ln, packed=None):
    """numarck_decompress_range through the C ABI, optionally with the index
    stream read from another buffer."""
    import ctypes
    h = c.header()
    out = torch.empty(max(ln, 1), dtype=c.dtype, device="cuda")
    fl = torch.zeros(1, dtype=torch.int32, device="cuda")
    ws = torch.empty(nk.numarck_decompress_workspace_bytes(ln), dtype=torch.uint8, device="cuda")
    pk = c.packed.data_ptr() if packed is None else packed
    nk._check(nk.numarck_decompress_range(
        ctypes.byref(h), p.data_ptr(), pk, c.centers.data_ptr(), c.incomp.data_ptr(),
        c.block_inc_off.data_ptr(), s, ln, out.data_ptr(), fl.data_ptr(), ws.data_ptr(),
        ws.numel(), torch.cuda.current_stream().cuda_stream), "numarck_decompress_range")
    return out[:ln], fl


@pytest.mark.parametrize("B", [4, 5, 8, 16])
def test_range_deep_in_block(nk, B):
    """Ranges that start far into a large compression block (the escapes
    before them are counted from the index stream in many pieces), ranges
    across block boundaries, and the same ranges with the index stream at a
    4-, 8- and 12-byte offset from a 16-byte boundary."""
    n = 3_000_017
    prev, curr = mixture_case(n, 500 + B, np.float32)
    c, o, p = compare_compress(nk, prev, curr, 1e-3, B, check_hist=False, label="deep")
    epb = c.header().elems_per_block
    assert epb >= 1 << 19
    rng = np.random.default_rng(B)
    want = [(epb - 1, 2), (epb + epb // 2 + 3, 70_001), (n - 1, 1), (n - 9000, 9000),
            (2 * epb - 8191, 8193), (n // 2 + 77, 100_000)]
    want += [(int(s), int(rng.integers(0, 200_001))) for s in rng.integers(0, n, 6)]
    ranges = [(min(s, n - 1), min(ln, n - min(s, n - 1))) for s, ln in want]
    orc = oracle.get()
    nw = c.header().packed_bytes // 4
    shifted = {}
    for off in (1, 2, 3):
        buf = torch.zeros(nw + 4, dtype=torch.int32, device="cuda")
        buf[off:off + nw] = c.packed[:nw]
        shifted[off] = buf
    for s, ln in ranges:
        r, rfl = orc.decompress_range(o, prev, s, ln)
        g, gfl = _range_at(nk, c, p, s, ln)
        assert int(gfl.item()) == rfl == 0
        assert np.array_equal(bits(to_np(g)), bits(r)), f"range {s},{ln}"
        for off, buf in shifted.items():
            g, gfl = _range_at(nk, c, p, s, ln, packed=buf.data_ptr() + 4 * off)
            assert int(gfl.item()) == 0
            assert np.array_equal(bits(to_np(g)), bits(r)), f"range {s},{ln} offset {4 * off}"


@pytest.mark.parametrize("E", [1e-310, 5e-324, 2.0 ** -1022])
def test_subnormal_error_bound(nk, E):
    """An error bound whose bin width 2E is subnormal (1/(2E) overflows):
    only ratios of exactly 0 are valid, and their bins come from the exact
    division; every other point escapes."""
    rng = np.random.default_rng(77)
    n = 70_001
    prev = rng.lognormal(0.0, 1.0, n)
    curr = np.where(rng.random(n) < 0.6, prev, prev * (1 + rng.normal(0, 1e-3, n)))
    c, o, p = compare_compress(nk, prev, curr, E, 8, label="subnormal E")
    assert c.header().M == 1
    compare_decompress(nk, c, o, p, prev, _ranges(n, rng))


def _certificate_case(n, dt, E, seed, anchor):
    """Points that sit on or next to what decides a point's bin and validity
    without the division: ratios on bin edges (lo + 2kE, or odd multiples of
    E for zero-anchored bins) and one or two ulps either side, ratios at the
    validity cap and next to it, subnormal and huge previous values, zeros
    and non-finite values, spread through the array so that every wave mixes
    them with ordinary points."""
    rng = np.random.default_rng(seed)
    p = rng.lognormal(0.0, 1.0, n) * rng.choice([-1.0, 1.0], n)
    k = rng.integers(-300, 300, n).astype(np.float64)
    base = -0.5 if anchor == "lo" else -E
    d = base + 2.0 * E * k
    d[0] = -0.5 if anchor == "lo" else d[0]  # the minimum ratio: lo = -0.5
    if anchor == "lo":
        d = np.maximum(d, -0.5)
    q = p * (1.0 + d)
    # one or two ulps either side of the edge
    nudge = rng.integers(-2, 3, n)
    q = q + nudge * np.spacing(q)
    cap = math.ldexp(E, 50)
    m = n // 50
    idx = rng.choice(np.arange(1, n), 6 * m, replace=False)
    a, b, c, e, f, g = np.split(idx, 6)
    p[a] = 1.0
    q[a] = 1.0 + cap * (1.0 + rng.integers(-4, 5, m) * 2.0 ** -52)  # at the cap
    p[b] = rng.choice([5e-324, 1e-310, -2.2e-308, 1e-320], m)  # subnormal prev
    q[b] = p[b] * rng.choice([1.0, 2.0, 0.5, -1.0], m)
    p[c] = rng.choice([1.7e308, -1.0e308, 8.9e307], m)  # reciprocal near underflow
    q[c] = p[c] * (1.0 + rng.normal(0, 2 * E, m))
    p[e] = rng.choice([0.0, -0.0, np.inf, -np.inf, np.nan], m)
    q[f] = rng.choice([np.inf, -np.inf, np.nan], m)
    q[g] = p[g] * 0.75  # ratio -0.25
    with np.errstate(all="ignore"):
        return p.astype(dt), q.astype(dt)


@pytest.mark.parametrize("dt", [np.float64, np.float32])
@pytest.mark.parametrize("E,B", [(2.0 ** -10, 8), (1e-3, 10), (3e-5, 12)])
def test_fast_bin_certificate_cases(nk, dt, E, B):
    """The bin passes take the change ratio through a reciprocal with an error
    certificate; where the certificate is unsure they recompute the exact
    division.  Inputs crowded with the cases at its edges match the oracle
    bit for bit, paper-anchored and zero-anchored."""
    prev, curr = _certificate_case(100_003, dt, E, int(E * 1e9) + B, "lo")
    c, o, p = compare_compress(nk, prev, curr, E, B, label="certificate")
    compare_decompress(nk, c, o, p, prev, _ranges(prev.size, np.random.default_rng(B)))
    prev, curr = _certificate_case(100_003, dt, E, int(E * 1e9) + B + 1, "zero")
    o = oracle.get().compress(prev, curr, E, B, binning="zero_anchored")
    P = torch.from_numpy(prev).to("cuda:0")
    Q = torch.from_numpy(curr).to("cuda:0")
    cz = nk.compress_zero_anchored(P, Q, E, B, recon=True, bin_ids=True)
    hz = cz.header()
    assert hz.n_inc == o.info["n_inc"] and hz.k_used == o.info["k_used"]
    assert np.array_equal(to_np(cz.packed[: o.info["packed_words"]]).view(np.uint32), o.packed)
    assert np.array_equal(bits(to_np(cz.incomp[: hz.n_inc])), bits(o.incomp))
    assert np.array_equal(bits(to_np(cz.recon[: hz.n])), bits(o.recon))
