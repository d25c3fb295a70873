"""Lossless stage of the index table (numarck_lossless_encode / _decode)
through the C ABI against the CPU oracle: the code ranks, the order k, the
sub-block offsets and every stream word bit for bit, and decoding returns
the table."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import to_np
from paper_1703_02438_amd import inputs
from pins import mixture_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nk():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1703_02438_amd.numarck as nk
    return nk


def _table(codes, B):
    """Pack B-bit codes LSB-first into 32-bit words."""
    n = len(codes)
    words = np.zeros(max((n * B + 31) // 32, 1), np.uint64)
    bit = np.arange(n, dtype=np.uint64) * np.uint64(B)
    for b in range(B):
        on = ((codes >> b) & 1).astype(bool)
        pos = bit[on] + np.uint64(b)
        np.bitwise_or.at(words, (pos >> np.uint64(5)).astype(np.int64),
                         np.left_shift(np.uint64(1), pos & np.uint64(31)))
    return words.astype(np.uint32)[: (n * B + 31) // 32]


def ll_compare(nk, packed, n, B, label="", shift_words=0):
    """Encode on the GPU (the table `shift_words` words past a 16-byte
    boundary when nonzero), compare with the oracle, decode back."""
    orc = oracle.get()
    o = orc.lossless_encode(packed, n, B)
    dev = torch.device("cuda:0")
    src = np.ascontiguousarray(packed if packed.size else np.zeros(1, np.uint32))
    base = torch.zeros(src.size + 4, dtype=torch.int32, device=dev)
    t = base[shift_words:shift_words + src.size]
    t.copy_(torch.from_numpy(src.view(np.int32)))
    assert (t.data_ptr() % 16 == 0) == (shift_words % 4 == 0)
    e = nk.lossless_encode(t, n, B)
    h = e.header()
    tag = f"[{label} n={n} B={B}]"
    assert h.k == o["k"], f"{tag} order"
    assert h.bits == o["bits_k"][o["k"]], f"{tag} bits"
    assert h.n_sub == len(o["sub_off"]) - 1 and h.stream_words == len(o["stream"]), tag
    assert np.array_equal(to_np(e.code_of_rank).view(np.uint16), o["code_of_rank"]), f"{tag} ranks"
    assert np.array_equal(to_np(e.sub_off).view(np.uint64), o["sub_off"]), f"{tag} offsets"
    sw = h.stream_words
    assert np.array_equal(to_np(e.stream)[:sw].view(np.uint32), o["stream"]), f"{tag} stream"
    assert h.bytes == (2 << B) + 8 * (h.n_sub + 1) + 4 * sw + 56
    assert (h.sub_log2, h.group_log2) == (10, 7), tag
    out, fl = nk.lossless_decode(e)
    assert int(fl.item()) == 0, tag
    words = (n * B + 31) // 32
    assert np.array_equal(to_np(out)[:words].view(np.uint32), packed[:words]), f"{tag} decode"
    return e, o


@pytest.mark.parametrize("B", [1, 2, 3, 5, 8, 10, 12, 13, 14, 16])
def test_lossless_random_tables(nk, B):
    rng = np.random.default_rng(70 + B)
    n = 3 * 1024 + 1234
    w = rng.pareto(1.1, 1 << B) + 1e-3
    codes = rng.choice(1 << B, n, p=w / w.sum())
    ll_compare(nk, _table(codes, B), n, B, label="pareto")


@pytest.mark.parametrize("B", [4, 6, 8, 16])
@pytest.mark.parametrize("n", [0, 1, 31, 127, 128, 129, 1024, 1025, 2048 + 5, 40_000])
def test_lossless_sizes(nk, n, B):
    """Short and ragged tables: partial groups and sub-blocks, for the
    word-aligned widths (4, 8, 16) and one that straddles words (6)."""
    rng = np.random.default_rng(n + 100 * B)
    codes = rng.integers(0, 1 << min(B, 6), n) if n else np.zeros(0, np.int64)
    ll_compare(nk, _table(codes, B), n, B, label="uniform")


@pytest.mark.parametrize("B", [4, 8, 16])
@pytest.mark.parametrize("shift", [1, 2, 3])
def test_lossless_table_off_16_byte_boundary(nk, B, shift):
    """A table that does not start on a 16-byte boundary takes the kernels
    that read it word by word: the same stream."""
    rng = np.random.default_rng(7 * B + shift)
    n = 5 * 1024 + 77
    w = rng.pareto(1.3, 1 << B) + 1e-3
    codes = rng.choice(1 << B, n, p=w / w.sum())
    ll_compare(nk, _table(codes, B), n, B, label="unaligned", shift_words=shift)


def test_lossless_single_symbol(nk):
    n = 100_000
    ll_compare(nk, _table(np.full(n, 9), 4), n, 4, label="one symbol")


@pytest.mark.parametrize("dt,B", [(np.float64, 8), (np.float32, 11), (np.float64, 16)])
def test_lossless_of_compressions(nk, dt, B):
    """The index tables the compressor writes (mixtures, with escapes)."""
    prev, curr = mixture_case(300_001, 81 + B, dt)
    o = oracle.get().compress(prev, curr, 1e-3, B)
    e, lo = ll_compare(nk, o.packed, prev.size, B, label=f"mixture {np.dtype(dt).name}")
    assert e.header().bytes < o.packed.size * 4 or B == 16


def test_lossless_flash_table_gpu_compressed(nk):
    """A FLASH-like 64^3 float64 pair compressed on the GPU, its table
    encoded and decoded on the GPU; the oracle agrees on the stream."""
    s = inputs.FlashSeries(edge=64, seed=91)
    p = s.x.clone().cuda()
    q = s.step().cuda()
    c = nk.compress(p, q, 1e-3, 8)
    n = p.numel()
    packed = to_np(c.packed)[: (n * 8 + 31) // 32].view(np.uint32).copy()
    e, o = ll_compare(nk, packed, n, 8, label="flash 64^3")
    assert e.header().bytes < 0.7 * packed.size * 4  # about 5 bits per 8-bit code here


@pytest.mark.parametrize("B", [4, 5])
def test_lossless_corrupt_stream_flagged(nk, B):
    """A stream of zeros (every codeword's leading one missing) and offsets
    past the stream are reported in the flag word, with every access in
    bounds (B = 4: the word-aligned decoder; 5: the general one)."""
    rng = np.random.default_rng(5)
    n = 2 * 1024 + 7
    codes = rng.integers(0, 16, n)
    t = torch.from_numpy(_table(codes, B).view(np.int32)).cuda()
    e = nk.lossless_encode(t, n, B)
    e.header()
    e.stream.zero_()
    _, fl = nk.lossless_decode(e)
    assert int(fl.item()) & nk.FLAG_BAD_STREAM
    e2 = nk.lossless_encode(t, n, B)
    e2.header()
    e2.sub_off[1] = 1 << 40
    _, fl = nk.lossless_decode(e2)
    assert int(fl.item()) & nk.FLAG_BAD_STREAM
    # a group offset moved by one bit: group 2 of sub-block 0 starts late, so
    # group 1 ends before its successor (and group 2 runs short)
    e3 = nk.lossless_encode(t, n, B)
    e3.header()
    e3.stream[1] += 1
    _, fl = nk.lossless_decode(e3)
    assert int(fl.item()) & nk.FLAG_BAD_STREAM
    # a group table with an offset inside the table itself
    e4 = nk.lossless_encode(t, n, B)
    e4.header()
    e4.stream[0] = 5
    _, fl = nk.lossless_decode(e4)
    assert int(fl.item()) & nk.FLAG_BAD_STREAM
    # a sound group table over codewords of zeros (no leading ones)
    e5 = nk.lossless_encode(t, n, B)
    e5.header()
    e5.stream[4:int(e5.sub_off[1].item()) // 32] = 0
    _, fl = nk.lossless_decode(e5)
    assert int(fl.item()) & nk.FLAG_BAD_STREAM


def test_lossless_partial_decode_then_range(nk):
    """Partial decompression through the lossless stage: only the sub-blocks
    from the start of the range's index-table block to its end are decoded,
    and the range decompressed from that partial table equals the range
    decompressed from the full table; words outside those sub-blocks stay
    untouched."""
    prev, curr = mixture_case(300_001, 99)
    p = torch.from_numpy(prev).cuda()
    q = torch.from_numpy(curr).cuda()
    B, bb = 8, 4096
    c = nk.compress(p, q, 1e-3, B, bb)
    n = p.numel()
    enc = nk.lossless_encode(c.packed, n, B)
    epb = c.header().elems_per_block
    for s, ln in ((0, 10), (123_456, 5_000), (299_990, 11), (40_960, 4096), (77_777, 0)):
        first = (s // epb) * epb
        table = torch.zeros_like(c.packed)
        fl = nk.lossless_decode_codes(enc, first, s + ln, table)
        assert int(fl.item()) == 0
        c2 = nk.Compressed(table, c.centers, c.incomp, c.block_inc_off, None, None, c.hdr, None,
                           c.n, c.dtype)
        a, afl = nk.decompress_range(c, p, s, ln)
        b, bfl = nk.decompress_range(c2, p, s, ln)
        assert int(afl.item()) == int(bfl.item()) == 0
        assert torch.equal(a[:ln].view(torch.int64), b[:ln].view(torch.int64)), (s, ln)
        w0 = (first // 1024) * 1024 * B // 32
        assert int(table[:w0].abs().sum().item()) == 0, (s, ln)
