"""Zero-anchored bins (numarck_compress_zero_anchored: fine bins of width 2E
anchored at -E, two passes over the snapshots) through the C ABI against the
CPU oracle, bit for bit in every output, the nonzero histogram included, and
decompression of the result."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import assert_matches_oracle, assert_same_compression, compare_decompress, to_np
from paper_1703_02438_amd import inputs
from pins import adversarial_case, mixture_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nk():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1703_02438_amd.numarck as nk
    return nk


def za_compare(nk, prev, curr, E, B, block_bytes=0, label="", ranges=None):
    orc = oracle.get()
    o = orc.compress(prev, curr, E, B, block_bytes=block_bytes, binning="zero_anchored")
    dev = torch.device("cuda:0")
    p = torch.from_numpy(np.ascontiguousarray(prev)).to(dev)
    q = torch.from_numpy(np.ascontiguousarray(curr)).to(dev)
    c = nk.compress_zero_anchored(p, q, E, B, block_bytes, recon=True, bin_ids=True)
    torch.cuda.synchronize()
    assert_matches_oracle(nk, c, o, prev, curr, E, B, block_bytes, check_hist=True,
                          label=f"za {label}")
    # without the reconstruction: the precoded encoder
    c2 = nk.compress_zero_anchored(p, q, E, B, block_bytes, bin_ids=True)
    assert_matches_oracle(nk, c2, o, prev, curr, E, B, block_bytes, check_hist=False,
                          label=f"za precoded {label}")
    if ranges is not None:
        compare_decompress(nk, c, o, p, prev, ranges, label=f"za {label}")
    return c, o


def _signed_case(counts, E=2.0 ** -10, seed=0):
    rng = np.random.default_rng(seed)
    bins = np.array([m for m, c in sorted(counts.items()) for _ in range(c)], np.int64)
    rng.shuffle(bins)
    p = (2.0 ** rng.integers(-3, 4, bins.size)) * np.where(rng.random(bins.size) < 0.3, -1, 1)
    return p, p * (1.0 + 2.0 * bins * E), E


def _far_case(n=200_000, seed=3):
    """Clusters at +0.4 and -0.45 with E = 1e-5: bins about +-20000, outside
    the window of 2^14 bins around ratio 0 (the exact tail path)."""
    rng = np.random.default_rng(seed)
    prev = rng.lognormal(0, 1, n)
    u = rng.random(n)
    r = np.where(u < 0.3, rng.normal(0, 1e-5, n),
                 np.where(u < 0.5, rng.normal(0.4, 3e-5, n),
                          np.where(u < 0.7, rng.normal(-0.45, 3e-5, n), rng.uniform(-0.5, 0.5, n))))
    return prev, prev * (1 + r)


def test_za_mixture_f64(nk):
    prev, curr = mixture_case(262_144, 1901)
    n = prev.size
    za_compare(nk, prev, curr, 1e-3, 8, label="mixture f64",
               ranges=[(0, n), (0, 0), (n // 3, 1000), (n - 17, 17)])


def test_za_mixture_f32_ragged(nk):
    prev, curr = mixture_case(100_003, 1902, np.float32, E=1e-4)
    za_compare(nk, prev, curr, 1e-4, 6, label="mixture f32", ranges=[(0, prev.size), (5, 50_000)])


@pytest.mark.parametrize("B", [1, 2, 3, 5, 8, 10, 12, 13, 15, 16])
def test_za_index_widths(nk, B):
    prev, curr = mixture_case(70_001, 1903 + B)
    za_compare(nk, prev, curr, 1e-3, B, label=f"B={B}")


@pytest.mark.parametrize("B", [8, 13, 16])
def test_za_far_tail(nk, B):
    prev, curr = _far_case()
    za_compare(nk, prev, curr, 1e-5, B, label=f"far tail B={B}", ranges=[(0, prev.size)])


def test_za_signed_ties(nk):
    """Equal counts in negative and positive bins: the lower (negative) ids
    win the tie."""
    p, q, E = _signed_case({-7: 300, -2: 500, 2: 500, 3: 500, 9: 40})
    c, o = za_compare(nk, p, q, E, 2, label="signed ties")
    assert o.sel_ids.tolist() == [-2, 2, 3]
    c, o = za_compare(nk, p, q, E, 1, label="signed ties B=1")
    assert o.sel_ids.tolist() == [-2]


@pytest.mark.parametrize("n", [0, 1, 2, 63, 4097])
def test_za_small_and_empty(nk, n):
    prev, curr = mixture_case(max(n, 1), 1920 + n)
    za_compare(nk, prev[:n], curr[:n], 1e-3, 5, label=f"n={n}")


def test_za_all_invalid(nk):
    za_compare(nk, np.zeros(9000), np.linspace(-1, 1, 9000), 1e-3, 6, label="all invalid")


@pytest.mark.parametrize("dt", [np.float64, np.float32])
def test_za_adversarial(nk, dt):
    p, q = adversarial_case(dt)
    za_compare(nk, np.tile(p, 300), np.tile(q, 300), 1e-3, 4,
               label=f"adversarial {np.dtype(dt).name}", ranges=[(0, 6000), (7, 33)])


@pytest.mark.parametrize("bb", [64, 1000])
def test_za_small_blocks(nk, bb):
    prev, curr = mixture_case(50_000, 1930 + bb)
    za_compare(nk, prev, curr, 1e-3, 7, block_bytes=bb, label=f"bb={bb}",
               ranges=[(0, 50_000), (123, 4567)])


def test_za_flash_like(nk):
    s = inputs.FlashSeries(edge=64, seed=31)
    prev = s.x.clone().numpy()
    curr = s.step().numpy()
    za_compare(nk, prev, curr, 1e-3, 8, label="flash 64^3", ranges=[(0, prev.size)])


def test_za_climate_outliers(nk):
    s = inputs.ClimateSeries(nlat=180, nlon=360, seed=32, outlier_lo=-0.9, outlier_hi=1.5)
    prev = s.x.clone().numpy()
    curr = s.step().numpy()
    za_compare(nk, prev, curr, 1e-4, 10, label="climate outliers", ranges=[(0, prev.size)])


def test_za_equals_topk_when_min_is_minus_E(nk):
    """With the smallest valid ratio exactly -E both anchors coincide: the two
    GPU paths give the same index table, centres and reconstruction."""
    E = 2.0 ** -10
    rng = np.random.default_rng(9)
    n = 300_000
    r = np.maximum(np.round(rng.normal(0, 4 * E, n) * 2 ** 20) / 2 ** 20, -E)
    r[1234] = -E
    p = (2.0 ** rng.integers(-3, 4, n)) * np.where(rng.random(n) < 0.3, -1, 1)
    q = p * (1.0 + r)
    dev = torch.device("cuda:0")
    pt, qt = torch.from_numpy(p).to(dev), torch.from_numpy(q).to(dev)
    a = nk.compress_zero_anchored(pt, qt, E, 8, recon=True)
    b = nk.compress(pt, qt, E, 8, recon=True)
    torch.cuda.synchronize()
    ha, hb = a.header().as_dict(), b.header().as_dict()
    assert hb["lo"] == -E and ha["lo"] == -E
    for f in ("n_inc", "n_nonzero", "k_used", "tau"):
        assert ha[f] == hb[f], f
    nw = (n * 8 + 31) // 32
    assert torch.equal(a.packed[:nw], b.packed[:nw])
    assert torch.equal(a.centers.view(torch.int64), b.centers.view(torch.int64))
    assert torch.equal(a.recon.view(torch.int64), b.recon.view(torch.int64))
    assert np.array_equal(to_np(a.incomp)[: ha["n_inc"]].view(np.int64),
                          to_np(b.incomp)[: hb["n_inc"]].view(np.int64))


def test_za_plans(nk):
    """Zero-anchored plans: time chains, unchained jobs, both element types
    and several B in one batch; every job equals its plain zero-anchored
    compression on every run, and some equal the oracle."""
    def series(n, dt, seed, steps):
        rng = np.random.default_rng(seed)
        x = rng.lognormal(0, 1, n)
        out = [x.astype(dt)]
        for _ in range(steps):
            x = x * (1 + rng.normal(0, 2e-3, n)) + np.where(rng.random(n) < 0.01,
                                                            rng.normal(0, 0.3, n), 0)
            out.append(x.astype(dt))
        return [torch.from_numpy(v).cuda() for v in out]

    fa = series(100_003, np.float64, 61, 4)
    fb = series(262_147, np.float32, 62, 3)
    other = series(50_001, np.float64, 63, 1)
    jobs = [(fa[t], fa[t + 1], 1e-3, 8) for t in range(4)]
    jobs.append((other[0], other[1], 1e-3, 12))
    jobs += [(fb[t], fb[t + 1], 1e-3, 10) for t in range(3)]
    plan = nk.Plan([nk.BatchJob(p, q, E, B) for p, q, E, B in jobs], recon=True, bin_ids=True,
                   zero_anchored=True)
    for rep in range(2):
        res = plan.run()
        torch.cuda.synchronize()
        for i, ((p, q, E, B), c) in enumerate(zip(jobs, res)):
            ref = nk.compress_zero_anchored(p, q, E, B, recon=True, bin_ids=True)
            assert_same_compression(c, ref, f"za plan job {i} rep {rep}")
    orc = oracle.get()
    for i in (0, 4, 6):
        p, q, E, B = jobs[i]
        pn, qn = to_np(p), to_np(q)
        assert_matches_oracle(nk, res[i], orc.compress(pn, qn, E, B, binning="zero_anchored"),
                              pn, qn, E, B, check_hist=False, label=f"za plan job {i}")
    # captured as a HIP graph and replayed, with eager work between replays
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.capture(s)
    for rep in range(3):
        with torch.cuda.stream(s):
            res = plan.replay(s)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        _ = (jobs[0][0] * 2).sum().item()  # eager work between replays
        for i, ((p, q, E, B), c) in enumerate(zip(jobs, res)):
            ref = nk.compress_zero_anchored(p, q, E, B, recon=True, bin_ids=True)
            assert_same_compression(c, ref, f"za graph job {i} replay {rep}")
    plan.close()
