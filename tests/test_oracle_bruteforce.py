"""A second, independent CPU implementation of the whole compression, written
as plain Python loops over Python floats (binary64, round-to-nearest, no
fused operations), compared byte for byte with the C oracle on small inputs:
the change ratios and validity of eq. (1), the range, the 2E bins and their
counts, top-k by sorting (count descending, bin id ascending), centres, the
verify against E, escapes, the index bit string written out character by
character, the block offsets and the header counts.  It shares nothing with
the C oracle but the seeded inputs."""
import math

import numpy as np
import pytest

import oracle
from pins import adversarial_case, mixture_case


def _to_type(x: float, dt) -> float:
    if dt != np.float32:
        return x
    with np.errstate(over="ignore"):  # values past the float32 range round to infinity
        return float(np.float32(x))


def brute_compress(prev, curr, E, B, block_bytes=1 << 20, binning="topk"):
    dt = prev.dtype.type
    n = prev.size
    k = (1 << B) - 1
    p = [float(v) for v in prev]
    q = [float(v) for v in curr]
    cap = math.ldexp(E, 50)
    d, valid = [], []
    for pj, qj in zip(p, q):
        ok = math.isfinite(pj) and pj != 0.0 and math.isfinite(qj)
        r = (qj - pj) / pj if ok else float("nan")
        ok = ok and math.isfinite(r) and abs(r) <= cap
        d.append(r)
        valid.append(ok)
    vals = [x for x, v in zip(d, valid) if v]
    n_valid = len(vals)
    lo = min(vals) if vals else 0.0
    hi = max(vals) if vals else 0.0
    if binning == "zero_anchored":
        lo, hi = -E, 0.0
    cand = [-1] * n
    info = {"n_valid": n_valid, "n_nonzero": 0, "tau": 0, "k_used": 0, "M": 0}
    if binning == "equal_width":
        w = (hi - lo) / k
        centres = [lo + (i + 0.5) * w for i in range(k)] if n_valid else []
        for j in range(n):
            if valid[j]:
                cand[j] = min(math.floor((d[j] - lo) / w), k - 1) if w > 0 else 0
        info["k_used"] = info["M"] = k if n_valid else 0
    else:
        counts = {}
        bins = [0] * n
        for j in range(n):
            if valid[j]:
                bins[j] = math.floor((d[j] - lo) / (2.0 * E))
                counts[bins[j]] = counts.get(bins[j], 0) + 1
        ranked = sorted(counts.items(), key=lambda kv: (-kv[1], kv[0]))
        chosen = sorted(m for m, _ in ranked[:k])
        info["n_nonzero"] = len(counts)
        info["k_used"] = len(chosen)
        info["tau"] = ranked[k - 1][1] if len(ranked) > k else 0
        if n_valid and binning == "topk":
            info["M"] = math.floor((hi - lo) / (2.0 * E)) + 1
        rank = {m: i for i, m in enumerate(chosen)}
        centres = [lo + (2 * m + 1) * E for m in chosen]
        for j in range(n):
            if valid[j] and bins[j] in rank:
                cand[j] = rank[bins[j]]
    if not n_valid and binning == "topk":
        lo = hi = 0.0
    cen = [_to_type(c, dt) for c in centres] + [0.0] * ((1 << B) - len(centres))
    codes, incomp, recon = [], [], []
    for j in range(n):
        code = k
        if cand[j] >= 0:
            r = _to_type(p[j] * (1.0 + cen[cand[j]]), dt)
            if abs(r - q[j]) <= E * abs(p[j]):
                code = cand[j]
                recon.append(r)
        if code == k:
            incomp.append(curr[j])
            recon.append(curr[j])
        codes.append(code)
    bitstr = "".join(format(c, f"0{B}b")[::-1] for c in codes)
    bitstr += "0" * (-len(bitstr) % 32)
    packed = [int(bitstr[i:i + 32][::-1], 2) for i in range(0, len(bitstr), 32)]
    epb = 8 * block_bytes // B
    blocks = [sum(1 for c in codes[:b0] if c == k) for b0 in range(0, n, epb)]
    info.update(n_inc=len(incomp), lo=lo, hi=hi, n_blocks=len(blocks))
    return info, packed, cen, incomp, recon, codes, blocks


CASES = [
    ("mixture f64 B=4", lambda: mixture_case(300, 11), 1e-3, 4, 1 << 20),
    ("mixture f64 B=8 small blocks", lambda: mixture_case(257, 12), 1e-3, 8, 16),
    ("mixture f32 B=6", lambda: mixture_case(200, 13, np.float32), 1e-3, 6, 40),
    ("mixture f64 B=1", lambda: mixture_case(150, 14), 1e-2, 1, 1 << 20),
    ("mixture f64 B=13", lambda: mixture_case(120, 15), 1e-4, 13, 1 << 20),
    ("adversarial f64", lambda: adversarial_case(np.float64), 1e-3, 3, 8),
    ("adversarial f32", lambda: adversarial_case(np.float32), 1e-3, 5, 8),
    ("all invalid", lambda: (np.zeros(40), np.ones(40)), 1e-3, 4, 1 << 20),
]


@pytest.mark.parametrize("binning", ["topk", "zero_anchored", "equal_width"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_bruteforce_equals_oracle(case, binning):
    _, make, E, B, bb = case
    prev, curr = make()
    info, packed, cen, incomp, recon, codes, blocks = brute_compress(prev, curr, E, B, bb,
                                                                    binning)
    o = oracle.get().compress(prev, curr, E, B, block_bytes=bb, binning=binning)
    for f in ("n_valid", "n_nonzero", "tau", "k_used", "M", "n_inc", "n_blocks"):
        assert o.info[f] == info[f], f
    assert np.float64(o.info["lo"]).tobytes() == np.float64(info["lo"]).tobytes()
    assert np.float64(o.info["hi"]).tobytes() == np.float64(info["hi"]).tobytes()
    assert o.packed.tolist() == packed
    assert o.index.tolist() == codes
    dt = prev.dtype
    assert o.centers.tobytes() == np.array(cen, dt).tobytes()
    assert o.incomp.tobytes() == np.array(incomp, dt).tobytes()
    assert o.recon.tobytes() == np.array(recon, dt).tobytes()
    assert o.block_inc_off.tolist() == blocks
