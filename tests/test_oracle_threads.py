"""The oracle's threaded per-element loops give the same bytes as one thread:
every output of the three binnings and of the choice of B, on mixtures,
adversarial values and an all-invalid input, at several thread counts."""
import numpy as np
import pytest

import oracle
from pins import adversarial_case, mixture_case

OUTS = ("packed", "centers", "incomp", "block_inc_off", "recon", "index", "sel_ids")


def _case(name):
    if name == "mixture_f64":
        return mixture_case(200_003, 61, np.float64)
    if name == "mixture_f32":
        return mixture_case(150_001, 62, np.float32)
    if name == "adversarial":
        pa, qa = adversarial_case(np.float64)
        pm, qm = mixture_case(50_000, 63, np.float64)
        return np.concatenate([pm, pa, pm]), np.concatenate([qm, qa, qm])
    z = np.zeros(4_099)
    return z, z + 1.0


def _bytes(res):
    out = {f: getattr(res, f) for f in OUTS if getattr(res, f, None) is not None}
    return {k: np.ascontiguousarray(v).tobytes() for k, v in out.items()}, res.info


@pytest.mark.parametrize("case", ["mixture_f64", "mixture_f32", "adversarial", "all_invalid"])
@pytest.mark.parametrize("binning", ["topk", "zero_anchored", "equal_width"])
def test_threads_give_identical_bytes(case, binning):
    orc = oracle.get()
    prev, curr = _case(case)
    try:
        orc.set_threads(1)
        ref_bytes, ref_info = _bytes(orc.compress(prev, curr, 1e-3, 8, block_bytes=1 << 12,
                                                  binning=binning))
        ref_B = orc.choose_B(prev, curr, 1e-3)
        for t in (2, 3, 8):
            assert orc.set_threads(t) == t, "the oracle was built without OpenMP"
            got_bytes, got_info = _bytes(orc.compress(prev, curr, 1e-3, 8, block_bytes=1 << 12,
                                                      binning=binning))
            assert got_info == ref_info, (t, case, binning)
            for k in ref_bytes:
                assert got_bytes[k] == ref_bytes[k], (t, case, binning, k)
            assert orc.choose_B(prev, curr, 1e-3) == ref_B, (t, case)
    finally:
        orc.set_threads(1)
