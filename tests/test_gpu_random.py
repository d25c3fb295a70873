"""Randomised configurations through the C ABI against the oracle: 40 seeded
cases drawing the size (1 to 300,000, ragged), the type, E, B (1 to 16), the
block size and the shape of the ratio distribution (narrow or wide Gaussian
cores, a uniform spill of random width and weight, zeros, runs of equal
values, huge outliers), so that windows, tails, ties and escapes combine in
ways the hand-made cases do not.  Every case compares every compression
output bit for bit, the full decompression and three ranges, and the
lossless stage of the index table."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import compare_compress, compare_decompress, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nk():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1703_02438_amd.numarck as nk
    return nk


def _case(seed):
    rng = np.random.default_rng(9000 + seed)
    n = int(rng.choice([1, 7, 64, 1023, 4097, 65535, 100_003, 300_000]))
    n = max(1, n + int(rng.integers(-3, 4)))
    dt = np.float32 if rng.random() < 0.5 else np.float64
    E = float(10.0 ** rng.uniform(-4, -1))
    B = int(rng.integers(1, 17))
    bb = int(rng.choice([0, 1, 3, 64, 4096, 1 << 20]))
    bb = 2 if 0 < bb and 8 * bb < B else bb  # a block holds at least one index
    prev = rng.lognormal(0.0, rng.uniform(0.1, 2.0), n)
    prev[rng.random(n) < rng.uniform(0, 0.01)] = 0.0
    prev *= np.where(rng.random(n) < 0.2, -1.0, 1.0)
    core = rng.normal(rng.uniform(-5, 5) * E, rng.uniform(0.2, 20) * E, n)
    spill_w = rng.uniform(0, 0.3)
    spill = rng.uniform(-rng.uniform(0.01, 2.0), rng.uniform(0.01, 2.0), n)
    r = np.where(rng.random(n) < spill_w, spill, core)
    if rng.random() < 0.3:  # runs of equal ratios
        r = np.repeat(r[: n // 8 + 1], 8)[:n]
    if rng.random() < 0.2:  # a few huge changes
        idx = rng.choice(n, max(1, n // 5000), replace=False)
        r[idx] = rng.choice([1e6, -1e6, 1e30, -1e30], idx.size)
    curr = prev * (1.0 + r)
    with np.errstate(over="ignore"):
        prev, curr = prev.astype(dt), curr.astype(dt)
    return prev, curr, E, B, bb


@pytest.mark.parametrize("seed", range(40))
def test_random_configuration(nk, seed):
    prev, curr, E, B, bb = _case(seed)
    label = f"random {seed}"
    c, o, p = compare_compress(nk, prev, curr, E, B, block_bytes=bb, label=label)
    rng = np.random.default_rng(seed)
    n = prev.size
    ranges = []
    for _ in range(3):
        s = int(rng.integers(0, n + 1))
        ranges.append((s, int(rng.integers(0, n - s + 1))))
    compare_decompress(nk, c, o, p, prev, ranges, label=label)
    # the lossless stage of the same index table
    ol = oracle.get().lossless_encode(o.packed, n, B)
    e = nk.lossless_encode(c.packed, n, B)
    h = e.header()
    assert h.k == ol["k"] and h.stream_words == len(ol["stream"]), label
    sw = h.stream_words
    assert np.array_equal(to_np(e.stream)[:sw].view(np.uint32), ol["stream"]), f"{label} stream"
    back, fl = nk.lossless_decode(e)
    assert int(fl.item()) == 0
    words = (n * B + 31) // 32
    assert np.array_equal(to_np(back)[:words].view(np.uint32), o.packed[:words]), label
