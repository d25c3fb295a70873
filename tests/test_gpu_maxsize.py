"""The largest input the library accepts: n = 2^32 - 1 float32 points
(16 GiB per snapshot), B = 8.  The CPU oracle cannot run at this size, so
the checks are properties that hold at any size, evaluated chunk by chunk
with torch on the device:

- the header's sizes follow their formulas and no flag is set;
- with B = 8 the index of point j is byte j of the index table; the escape
  code marks exactly n_inc points, and every other index is below k_used;
- decompression returns an escaped point's value bit for bit, and for every
  other point T(p * (1 + c)) of its centre c, within E * |p| of the value;
- lo and hi are the smallest and largest valid ratio;
- each block offset is the number of escapes before the block;
- range decompressions at the far end of the array (offsets past 2^31 and
  up to the last point) equal the full decompression there.

This exercises every 32-bit quantity of the path at its limit (element
offsets, packed words, unit ranges, escape offsets)."""
import pytest
import torch

pytestmark = pytest.mark.gpu

N = (1 << 32) - 1
E, B = 1e-3, 8
CH = 1 << 28  # elements per checking chunk


@pytest.fixture(scope="module")
def nk():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1703_02438_amd.numarck as nk
    return nk


def _inputs():
    g = torch.Generator(device="cuda")
    g.manual_seed(1712)
    prev = torch.empty(N, dtype=torch.float32, device="cuda")
    curr = torch.empty(N, dtype=torch.float32, device="cuda")
    for s in range(0, N, CH):
        e = min(s + CH, N)
        z = torch.randn(e - s, generator=g, device="cuda", dtype=torch.float32)
        p = torch.exp(0.5 * z)
        p[::997] = 0.0  # invalid points
        r = 0.002 * torch.randn(e - s, generator=g, device="cuda", dtype=torch.float32)
        jump = torch.rand(e - s, generator=g, device="cuda") < 0.01
        r = torch.where(jump, 0.05 * (2 * torch.rand(e - s, generator=g, device="cuda") - 1), r)
        prev[s:e] = p
        curr[s:e] = (p.double() * (1 + r.double())).float()
    return prev, curr


@pytest.mark.timeout(900)
def test_max_size_float32(nk):
    prev, curr = _inputs()
    o = nk.alloc_outputs(N, torch.float32, B, bin_ids=True)
    ws = torch.empty(nk.numarck_workspace_bytes_tail(N, nk.F32, 1 << 20), dtype=torch.uint8,
                     device="cuda")
    c = nk.compress(prev, curr, E, B, ws=ws, outputs=o)
    h = c.header()
    epb = nk.numarck_elems_per_block(B, 0)
    assert h.n == N and h.flags == 0 and h.B == B
    assert h.elems_per_block == epb and h.n_blocks == -(-N // epb)
    assert h.packed_bytes == 4 * (-(-N * B // 32))
    assert 1 <= h.k_used <= 255
    del ws

    out, fl = nk.decompress(c, prev)
    assert int(fl.item()) == 0
    codes = c.packed.view(torch.uint8)
    cent = c.centers.double()
    n_inc = 0
    lo, hi = float("inf"), float("-inf")
    blk = c.block_inc_off[: h.n_blocks].cpu()
    for s in range(0, N, CH):
        e = min(s + CH, N)
        k = codes[s:e].long()
        p, q, r = prev[s:e], curr[s:e], out[s:e]
        esc = k == 255
        assert bool((k[~esc] < h.k_used).all())
        assert torch.equal(r[esc].view(torch.int32), q[esc].view(torch.int32))
        pd = p.double()
        exp = (pd * (1.0 + cent[k.clamp(max=254)])).float()
        ok = ~esc
        assert torch.equal(r[ok].view(torch.int32), exp[ok].view(torch.int32))
        assert bool(((r[ok].double() - q[ok].double()).abs() <= E * pd[ok].abs()).all())
        d = (q.double() - pd) / pd
        valid = torch.isfinite(pd) & (pd != 0) & torch.isfinite(d) & (d.abs() <= E * 2.0 ** 50)
        assert bool(esc[~valid].all())
        if bool(valid.any()):
            lo = min(lo, float(d[valid].min()))
            hi = max(hi, float(d[valid].max()))
        # block offsets of the blocks starting in this chunk
        b0, b1 = -(-s // epb), -(-e // epb)
        cnt = torch.cumsum(esc.long(), 0)
        first = torch.arange(b0, b1, device="cuda") * epb - s
        before = n_inc + torch.where(first > 0, cnt[(first - 1).clamp(min=0)],
                                     torch.zeros_like(first))
        assert torch.equal(before.cpu(), blk[b0:b1]), f"block offsets in [{b0}, {b1})"
        n_inc += int(cnt[-1])
    assert h.n_inc == n_inc
    assert (h.lo, h.hi) == (lo, hi)

    for s, ln in [(N - 1, 1), (N - 777, 777), ((1 << 31) + 12345, 1 << 20),
                  (N - (1 << 24) - 3, 1 << 24)]:
        part, pf = nk.decompress_range(c, prev, s, ln)
        assert int(pf.item()) == 0
        assert torch.equal(part[:ln].view(torch.int32), out[s:s + ln].view(torch.int32)), (s, ln)
