"""The C-ABI library: it loads, exports every entry point include/numarck.h
declares, and its host-only functions (sizes, validation) behave as
documented.  No kernel is launched here (no GPU)."""
import ctypes
import math
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "numarck.h")


@pytest.fixture(scope="module")
def nk():
    from paper_1703_02438_amd import build

    if not os.path.exists(build.LIB):
        build.build()
    import paper_1703_02438_amd.numarck as nk
    return nk


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(numarck_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_entry_points():
    names = declared_functions()
    for must in ("numarck_compress", "numarck_decompress", "numarck_decompress_range"):
        assert must in names


def test_library_exports_every_declared_symbol(nk):
    out = subprocess.run(["nm", "-D", "--defined-only", nk.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (numarck_\w+)", out))
    missing = [f for f in declared_functions() if f not in exported]
    assert not missing, missing
    lib = ctypes.CDLL(nk.LIB_PATH)
    for f in declared_functions():
        assert hasattr(lib, f)


def test_sizes(nk):
    assert nk.numarck_packed_bytes(0, 8) == 0
    assert nk.numarck_packed_bytes(3, 8) == 4
    assert nk.numarck_packed_bytes(33, 1) == 8
    assert nk.numarck_packed_bytes(1000, 13) == 4 * math.ceil(13000 / 32)
    assert nk.numarck_centers_bytes(13, nk.F32) == 8192 * 4
    assert nk.numarck_centers_bytes(8, nk.F64) == 256 * 8
    assert nk.numarck_centers_bytes(0, nk.F64) == 0
    # Fig. 2: 13-bit indices, 1 MB blocks -> 645,277 per block, 6 blocks for 3,758,400
    assert nk.numarck_elems_per_block(13, 1 << 20) == 645277
    assert nk.numarck_block_count(3758400, 13, 0) == 6
    assert nk.numarck_block_count(0, 13, 0) == 0
    w_full = nk.numarck_workspace_bytes(1 << 20, nk.F64, 8)
    w_none = nk.numarck_workspace_bytes_tail(1 << 20, nk.F64, 0)
    assert w_full > w_none > 0
    assert nk.numarck_workspace_bytes_tail(1 << 20, nk.F64, 1 << 20) == w_full
    assert nk.numarck_decompress_workspace_bytes(0) > 0


class _FakeOut(ctypes.Structure):
    pass


def _out(nk, base=0x100000):
    return nk.NumarckOut(base, base + 0x1000, base + 0x2000, base + 0x3000, None, None,
                         base + 0x4000)


def test_compress_validation_without_gpu(nk):
    o = _out(nk)
    ws = 0x200000
    p, q = 0x300000, 0x400000
    big = 1 << 40
    call = lambda *a: nk.numarck_compress(*a)
    assert call(p, q, 10, 7, 1e-3, 8, 0, ctypes.byref(o), ws, big, None) == nk.EDTYPE
    assert call(p, q, 10, nk.F64, 1e-3, 0, 0, ctypes.byref(o), ws, big, None) == nk.EBITS
    assert call(p, q, 10, nk.F64, 1e-3, 17, 0, ctypes.byref(o), ws, big, None) == nk.EBITS
    for bad_e in (0.0, -1e-3, 1.5, float("nan"), float("inf")):
        assert call(p, q, 10, nk.F64, bad_e, 8, 0, ctypes.byref(o), ws, big, None) == nk.EBOUND
    assert call(p, q, 1 << 32, nk.F64, 1e-3, 8, 0, ctypes.byref(o), ws, big, None) == nk.EINVAL
    assert call(p, q, 10, nk.F64, 1e-3, 8, 0, None, ws, big, None) == nk.EINVAL
    assert call(None, q, 10, nk.F64, 1e-3, 8, 0, ctypes.byref(o), ws, big, None) == nk.EINVAL
    assert call(p + 8, q, 10, nk.F64, 1e-3, 8, 0, ctypes.byref(o), ws, big, None) == nk.EALIGN
    assert call(p, q, 10, nk.F64, 1e-3, 8, 0, ctypes.byref(o), ws + 64, big, None) == nk.EALIGN
    assert call(p, q, 10, nk.F64, 1e-3, 8, 0, ctypes.byref(o), ws, 1024, None) == nk.ECAPACITY
    assert call(p, q, 10, nk.F64, 1e-3, 16, 1, ctypes.byref(o), ws, big, None) == nk.EINVAL


def _header(nk, n=1000, B=8, bb=1 << 20):
    h = nk.NumarckHeader()
    h.n, h.B, h.dtype, h.block_bytes = n, B, nk.F64, bb
    h.elems_per_block = 8 * bb // B
    h.n_blocks = -(-n // h.elems_per_block)
    h.k_used, h.n_inc = 10, 5
    return h


def test_compress_auto_validation_without_gpu(nk):
    o = _out(nk)
    ws, big = 0x200000, 1 << 40
    p, q = 0x300000, 0x400000
    B = ctypes.c_uint32(0)
    bits = (ctypes.c_uint64 * 17)()
    call = lambda lo, hi, **kw: nk.numarck_compress_auto(
        kw.get("p", p), q, 10, nk.F64, kw.get("E", 1e-3), lo, hi, 0, ctypes.byref(o), ws, big,
        None, kw.get("B", ctypes.byref(B)), bits)
    assert call(0, 8) == nk.EBITS
    assert call(1, 17) == nk.EBITS
    assert call(9, 8) == nk.EBITS
    assert call(1, 16, B=None) == nk.EINVAL
    assert call(1, 16, E=0.0) == nk.EBOUND
    assert call(1, 16, p=p + 8) == nk.EALIGN


@pytest.mark.parametrize("entry", ["numarck_compress_equal_width",
                                   "numarck_compress_zero_anchored"])
def test_compress_variant_validation_without_gpu(nk, entry):
    o = _out(nk)
    ws, big = 0x200000, 1 << 40
    p, q = 0x300000, 0x400000
    call = lambda **kw: getattr(nk, entry)(
        kw.get("p", p), q, 10, nk.F64, kw.get("E", 1e-3), kw.get("B", 8), 0, ctypes.byref(o),
        kw.get("ws", ws), big, None)
    assert call(B=0) == nk.EBITS
    assert call(B=17) == nk.EBITS
    assert call(E=0.0) == nk.EBOUND
    assert call(p=p + 8) == nk.EALIGN
    assert call(ws=ws + 16) == nk.EALIGN
    assert call(ws=None) == nk.EINVAL


def test_decompress_validation_without_gpu(nk):
    h = _header(nk)
    ws, big = 0x200000, 1 << 30
    args = lambda hh, s, ln: (ctypes.byref(hh), 0x300000, 0x400000, 0x500000, 0x600000,
                              0x700000, s, ln, 0x800000, 0x900000, ws, big, None)
    assert nk.numarck_decompress_range(*args(h, 900, 101)) == nk.ERANGE
    assert nk.numarck_decompress_range(*args(h, 1001, 0)) == nk.ERANGE
    bad = _header(nk)
    bad.elems_per_block += 1
    assert nk.numarck_decompress_range(*args(bad, 0, 10)) == nk.EINVAL
    bad = _header(nk)
    bad.B = 0
    assert nk.numarck_decompress_range(*args(bad, 0, 10)) == nk.EBITS
    bad = _header(nk)
    bad.k_used = 300
    assert nk.numarck_decompress_range(*args(bad, 0, 10)) == nk.EINVAL
    small = list(args(h, 0, 1000))
    small[11] = 16
    assert nk.numarck_decompress_range(*small) == nk.ECAPACITY


def test_status_strings(nk):
    for s in range(9):
        assert nk.numarck_status_str(s)
    assert nk.numarck_status_str(99) == b"unknown status"


def _job(nk, n=1000, dtype=None, E=1e-3, B=8, base=0x300000):
    return nk.NumarckJob(base, base + 0x100000, n, nk.F64 if dtype is None else dtype, E, B, 0,
                         _out(nk))


def test_plan_validation_without_gpu(nk):
    jobs = (nk.NumarckJob * 3)(_job(nk), _job(nk, 5000, nk.F32, 1e-4, 12), _job(nk, 0))
    need = nk.numarck_batch_workspace_bytes(jobs, 3)
    single = sum(nk.numarck_workspace_bytes(j.n, j.dtype, j.B) for j in jobs)
    assert need > single  # job table and prefix arrays come first
    h = ctypes.c_void_p()
    ws = 0x10000000
    create = lambda js, nj, w=ws, wb=need, t=None: nk.numarck_plan_create(
        js, nj, t, w, wb, None, ctypes.byref(h))
    assert create(jobs, 0) == nk.EINVAL
    assert create(jobs, nk.MAX_JOBS + 1) == nk.EINVAL
    assert create(jobs, 3, w=ws + 16) == nk.EALIGN
    assert create(jobs, 3, wb=need - 1) == nk.ECAPACITY
    bad = (nk.NumarckJob * 2)(_job(nk), _job(nk, B=0))
    assert create(bad, 2) == nk.EBITS
    assert b"job 1" in nk.numarck_last_error()
    bad = (nk.NumarckJob * 2)(_job(nk, E=2.0), _job(nk))
    assert create(bad, 2) == nk.EBOUND
    bad = (nk.NumarckJob * 1)(_job(nk, base=0x300008))
    assert create(bad, 1) == nk.EALIGN
    t = nk.NumarckTuning(8, 2, 1, 4096, 0, 0)  # unit_pct 0
    assert create(jobs, 3, t=ctypes.byref(t)) == nk.EINVAL
    assert not h.value
    assert nk.numarck_plan_run(None, None) == nk.EINVAL
    assert nk.numarck_plan_replay(None, None) == nk.EINVAL
    nk.numarck_plan_destroy(None)


def test_tuning_defaults_and_files(nk, tmp_path):
    t = nk.default_tuning()
    assert t.as_dict() == {"range_blocks_per_cu": 2, "hist_blocks_per_cu": 2, "hist_lds": 1,
                           "chunk_vec": 0, "unit_pct": 100, "stream_loads": 0}
    good = tmp_path / "good.txt"
    good.write_text("# comment\nf64 27 4 2 1 8192 75 1\nf32 20 8 4 0 2048 100\n")
    assert nk.numarck_tuning_load(str(good).encode()) == nk.OK
    out = tmp_path / "out.txt"
    assert nk.numarck_tuning_save(str(out).encode()) == nk.OK
    lines = [ln for ln in out.read_text().splitlines() if not ln.startswith("#")]
    assert "f64 27 4 2 1 8192 75 1" in lines and "f32 20 8 4 0 2048 100 0" in lines
    for bad in ("f16 3 1 1 1 64 1\n", "f64 3 0 1 1 64 1\n", "f64 3 1 1 2 64 1\n",
                "f64 3 1 1 1 63 1\n", "f64 3 1 1 1 64 101\n", "f64 3 1 1\n",
                "f64 3 1 1 1 64 1 3\n"):
        p = tmp_path / "bad.txt"
        p.write_text(bad)
        assert nk.numarck_tuning_load(str(p).encode()) == nk.EINVAL, bad
    assert nk.numarck_tuning_load(str(tmp_path / "missing.txt").encode()) == nk.EINVAL


def test_compress_tuned_validation_without_gpu(nk):
    o = _out(nk)
    bad = nk.NumarckTuning(8, 2, 1, 32, 100, 0)  # chunk_vec below 64
    st = nk.numarck_compress_tuned(0x300000, 0x400000, 10, nk.F64, 1e-3, 8, 0, ctypes.byref(o),
                                   0x200000, 1 << 40, ctypes.byref(bad), None)
    assert st == nk.EINVAL


def test_flag_constants_match_header():
    """The binding's flag values are the header's."""
    import re
    import paper_1703_02438_amd.numarck as nk
    h = open(os.path.join(os.path.dirname(__file__), "..", "include", "numarck.h")).read()
    flags = {k: int(v.rstrip("u")) for k, v in re.findall(r"#define NUMARCK_(FLAG_\w+) (\w+)", h)}
    assert flags and all(getattr(nk, k) == v for k, v in flags.items()), flags


def test_lossless_validation_without_gpu(nk):
    """Argument checks of the lossless stage return before any device work."""
    import paper_1703_02438_amd.numarck as m
    ws, big = 0x200000, 1 << 30
    enc = lambda B=8, n=100, sb=big, wsb=big, **kw: m.numarck_lossless_encode(
        kw.get("packed", 0x300000), n, B, 0x400000, 0x500000, 0x600000, sb,
        kw.get("hdr", 0x700000), ws, wsb, None)
    assert enc(B=0) == nk.EBITS and enc(B=17) == nk.EBITS
    assert enc(n=1 << 32) == nk.EINVAL
    assert enc(hdr=None) == nk.EINVAL and enc(packed=None) == nk.EINVAL
    assert enc(sb=m.numarck_lossless_stream_bytes(100, 8) - 4) == nk.ECAPACITY
    assert enc(wsb=m.numarck_lossless_workspace_bytes(8) - 1) == nk.ECAPACITY
    assert m.numarck_lossless_subblocks(0) == 0 and m.numarck_lossless_subblocks(1025) == 2
    assert m.numarck_lossless_stream_bytes(4096, 8) == 4 * (4096 * 9 // 32 + 5 * 4)
    h = m.NumarckLosslessHeader(n=10, n_sub=1, stream_words=5, bits=10, B=8, k=9, sub_log2=10,
                                group_log2=7)
    dec = lambda hh: m.numarck_lossless_decode(ctypes.byref(hh), 0x400000, 0x500000, 0x600000,
                                               0x800000, 0x900000, None)
    assert dec(h) == nk.EINVAL  # k > B
    h.k, h.n_sub = 0, 2
    assert dec(h) == nk.EINVAL  # n_sub inconsistent with n
    h.n_sub, h.B = 1, 0
    assert dec(h) == nk.EBITS
    h.B = 8
    h.sub_log2 = 12  # a stream of another layout
    assert dec(h) == nk.EINVAL
    h.sub_log2, h.group_log2 = 10, 6
    assert dec(h) == nk.EINVAL
    h.group_log2 = 7
    misaligned = m.numarck_lossless_decode(ctypes.byref(h), 0x400000, 0x500000, 0x600004,
                                           0x800000, 0x900000, None)
    assert misaligned == nk.EALIGN
    rng = lambda b, c: m.numarck_lossless_decode_range(ctypes.byref(h), 0x400000, 0x500000,
                                                       0x600000, b, c, 0x800000, 0x900000, None)
    assert rng(0, 2) == nk.ERANGE and rng(2, 0) == nk.ERANGE and rng(1 << 63, 1 << 63) == nk.ERANGE


def test_decompress_noalloc_validation_without_gpu(nk):
    """The no-allocation range decompression checks its arguments like the
    workspace form, before it touches the device."""
    h = _header(nk)
    args = lambda hh, s, ln, fl=0x900000: (ctypes.byref(hh), 0x300000, 0x400000, 0x500000,
                                           0x600000, 0x700000, s, ln, 0x800000, fl, None)
    assert nk.numarck_decompress_range_noalloc(*args(h, 900, 101)) == nk.ERANGE
    assert nk.numarck_decompress_range_noalloc(*args(h, 1001, 0)) == nk.ERANGE
    assert nk.numarck_decompress_range_noalloc(*args(h, 0, 10, fl=None)) == nk.EINVAL
    bad = _header(nk)
    bad.B = 17
    assert nk.numarck_decompress_range_noalloc(*args(bad, 0, 10)) == nk.EBITS
    assert nk.numarck_decompress_range_noalloc(None, *args(h, 0, 10)[1:]) == nk.EINVAL
    assert nk.numarck_static_scratch_bytes() >= nk.numarck_decompress_workspace_bytes(1 << 31)


def test_stream_kernel_validation_without_gpu(nk):
    a, b = 0x300000, 0x400000
    assert nk.numarck_stream_kernel(8, a, b, 1 << 20, 8, None) == nk.EINVAL
    for kind in (nk.STREAM_READ2_WRITE16, nk.STREAM_READ2_WRITE8):
        assert nk.numarck_stream_kernel(kind, a, b, (1 << 20) + 16, 8, None) == nk.EINVAL
    assert nk.numarck_stream_kernel(-1, a, b, 1 << 20, 8, None) == nk.EINVAL
    assert nk.numarck_stream_kernel(nk.STREAM_COPY, a, b, (1 << 20) + 8, 8, None) == nk.EINVAL
    assert nk.numarck_stream_kernel(nk.STREAM_COPY, a, b, 1 << 20, 0, None) == nk.EINVAL
    assert nk.numarck_stream_kernel(nk.STREAM_COPY, a, b, 1 << 20, 65, None) == nk.EINVAL
    assert nk.numarck_stream_kernel(nk.STREAM_COPY, None, b, 1 << 20, 8, None) == nk.EINVAL
    assert nk.numarck_stream_kernel(nk.STREAM_COPY, a + 8, b, 1 << 20, 8, None) == nk.EALIGN
    assert nk.numarck_stream_kernel(nk.STREAM_WRITE, None, b + 4, 1 << 20, 8, None) == nk.EALIGN
    assert nk.numarck_stream_kernel(nk.STREAM_READ, a, None, 1 << 20, 8, None) == nk.EINVAL


def test_plan_autotune_validation_without_gpu(nk):
    arr = (nk.NumarckJob * 1)()
    assert nk.numarck_plan_autotune(arr, 1, 0x200000, 1 << 30, 2, 0, None, None) == nk.EINVAL
