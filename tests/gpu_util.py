"""Helpers for the GPU parity tests: run the HIP library and the CPU oracle on
the same inputs and compare every output bit for bit."""
from __future__ import annotations

import numpy as np
import torch

import oracle


def bits(a: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(a)
    if a.dtype == np.float32:
        return a.view(np.uint32)
    if a.dtype == np.float64:
        return a.view(np.uint64)
    return a


def to_np(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy()


def gpu_compress(nk, prev: np.ndarray, curr: np.ndarray, E, B, block_bytes=0, ws=None):
    dev = torch.device("cuda:0")
    p = torch.from_numpy(np.ascontiguousarray(prev)).to(dev)
    q = torch.from_numpy(np.ascontiguousarray(curr)).to(dev)
    c = nk.compress(p, q, E, B, block_bytes=block_bytes, recon=True, bin_ids=True, ws=ws)
    return c, p, q


HEADER_FIELDS = ["n", "n_valid", "n_invalid", "n_inc", "n_blocks", "elems_per_block",
                 "block_bytes", "M", "n_nonzero", "B", "k_used", "tau", "packed_bytes",
                 "compressed_bytes"]


def assert_matches_oracle(nk, c, o, prev, curr, E, B, block_bytes=0, check_hist=True,
                          label=""):
    """Assert that the GPU compression `c` equals the oracle's `o` in every output."""
    orc = oracle.get()
    h = c.header().as_dict()
    tag = f"[{label} n={prev.size} {prev.dtype} E={E} B={B} bb={block_bytes}]"
    for f in HEADER_FIELDS:
        assert h[f] == o.info[f], f"{tag} header {f}: gpu {h[f]} oracle {o.info[f]}"
    assert h["flags"] == 0, f"{tag} flags {h['flags']}"
    assert h["dtype"] == o.info["dtype"]
    assert bits(np.array([h["lo"], h["hi"]])).tolist() == \
        bits(np.array([o.info["lo"], o.info["hi"]])).tolist(), f"{tag} lo/hi"
    n = prev.size
    nw = o.info["packed_words"]
    assert np.array_equal(to_np(c.packed)[:nw].view(np.uint32), o.packed), f"{tag} packed"
    # buffers may be sized for a larger B (the automatic choice of B)
    assert np.array_equal(bits(to_np(c.centers)[: 1 << B]), bits(o.centers)), f"{tag} centers"
    ninc = o.info["n_inc"]
    assert np.array_equal(bits(to_np(c.incomp)[:ninc]), bits(o.incomp)), f"{tag} incomp"
    nb = o.info["n_blocks"]
    assert np.array_equal(to_np(c.block_inc_off)[:nb], o.block_inc_off), f"{tag} blocks"
    if n and c.recon is not None:
        assert np.array_equal(bits(to_np(c.recon)[:n]), bits(o.recon)), f"{tag} recon"
    if c.bin_ids is not None:
        ku = o.info["k_used"]
        gb = to_np(c.bin_ids)[: (1 << B) - 1]
        assert np.array_equal(gb[:ku], o.sel_ids), f"{tag} selected bins"
        assert np.all(gb[ku:] == -1), f"{tag} unused bin ids"
    if check_hist:
        ids, cnt, k = nk.histogram(c)
        assert k == o.info["n_nonzero"], f"{tag} nonzero bins"
        gi, gc = to_np(ids), to_np(cnt).view(np.uint32)
        order = np.argsort(gi, kind="stable")
        d, v = orc.ratio(prev, curr, E)
        if o.info["n_valid"]:
            m = orc.bin_ids(d, v, o.info["lo"], E)
            oi, oc = orc.histogram(m, v)
        else:
            oi, oc = np.zeros(0, np.int64), np.zeros(0, np.uint32)
        assert np.array_equal(gi[order], oi), f"{tag} histogram ids"
        assert np.array_equal(gc[order], oc), f"{tag} histogram counts"


def compare_compress(nk, prev, curr, E, B, block_bytes=0, check_hist=True, label=""):
    """Compress on both sides and assert every output is identical: once with
    the reconstruction (the encoder that reads both snapshots) and once
    without (the precoded encoder, from the histogram pass's window codes)."""
    o = oracle.get().compress(prev, curr, E, B, block_bytes=block_bytes)
    c, p, q = gpu_compress(nk, prev, curr, E, B, block_bytes)
    assert_matches_oracle(nk, c, o, prev, curr, E, B, block_bytes, check_hist, label)
    c2 = nk.compress(p, q, E, B, block_bytes=block_bytes, bin_ids=True)
    assert c2.recon is None
    assert_matches_oracle(nk, c2, o, prev, curr, E, B, block_bytes, False, label + " precoded")
    return c, o, p


def assert_same_compression(a, b, label=""):
    """Two GPU compressions of the same input are identical in every output."""
    ha, hb = a.header().as_dict(), b.header().as_dict()
    for f in HEADER_FIELDS + ["flags", "lo", "hi", "tail_count", "window_base"]:
        assert bits(np.array([ha[f]])).tolist() == bits(np.array([hb[f]])).tolist(), \
            f"[{label}] header {f}: {ha[f]} vs {hb[f]}"
    nw = ha["packed_bytes"] // 4
    assert torch.equal(a.packed[:nw], b.packed[:nw]), f"[{label}] packed"
    assert torch.equal(a.centers.view(torch.int32) if a.centers.dtype == torch.float32
                       else a.centers.view(torch.int64),
                       b.centers.view(torch.int32) if b.centers.dtype == torch.float32
                       else b.centers.view(torch.int64)), f"[{label}] centers"
    ni = ha["n_inc"]
    ia, ib = a.incomp[:ni], b.incomp[:ni]
    iv = torch.int32 if ia.dtype == torch.float32 else torch.int64
    assert torch.equal(ia.view(iv), ib.view(iv)), f"[{label}] incomp"
    nb = ha["n_blocks"]
    assert torch.equal(a.block_inc_off[:nb], b.block_inc_off[:nb]), f"[{label}] blocks"


def compare_decompress(nk, c, o, p, prev, ranges=(), label=""):
    orc = oracle.get()
    out, fl = nk.decompress(c, p)
    ref, rfl = orc.decompress(o, prev)
    assert int(fl.item()) == rfl == 0, label
    assert np.array_equal(bits(to_np(out)), bits(ref)), f"[{label}] full decompress"
    for s, ln in ranges:
        g, gfl = nk.decompress_range(c, p, s, ln)
        r, rfl = orc.decompress_range(o, prev, s, ln)
        assert int(gfl.item()) == rfl == 0
        assert np.array_equal(bits(to_np(g)[:ln]), bits(r)), f"[{label}] range {s},{ln}"
