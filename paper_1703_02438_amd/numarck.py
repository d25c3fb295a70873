"""ctypes binding of libnumarck.so (the C ABI declared in include/numarck.h).

The functions named ``numarck_*`` take exactly the arguments of the C entry
points of the same name (integers for device pointers and streams) and return
the status code.  The helpers below them (:func:`compress`,
:func:`decompress`, :func:`decompress_range`, :func:`histogram`) only
allocate device tensors with torch, pass their pointers and the current HIP
stream, and wrap the results; every step of the method runs in the library's
kernels.  There is no CPU fallback: if the library is missing this module
fails to import.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch  # loads torch's HIP runtime before the library binds to it

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnumarck.so")

F32, F64 = 0, 1
OK, EINVAL, EDTYPE, EBITS, EBOUND, EALIGN, ECAPACITY, EHIP, ERANGE = range(9)
FLAG_BAD_INDEX, FLAG_INC_OVERRUN, FLAG_TAIL_OVERFLOW, FLAG_BAD_STREAM = 1, 2, 4, 8


class NumarckHeader(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_uint64), ("n_valid", ctypes.c_uint64), ("n_invalid", ctypes.c_uint64),
        ("n_inc", ctypes.c_uint64), ("n_blocks", ctypes.c_uint64),
        ("elems_per_block", ctypes.c_uint64), ("block_bytes", ctypes.c_uint64),
        ("M", ctypes.c_int64), ("n_nonzero", ctypes.c_uint64),
        ("B", ctypes.c_uint32), ("k_used", ctypes.c_uint32), ("dtype", ctypes.c_uint32),
        ("flags", ctypes.c_uint32), ("tau", ctypes.c_uint32), ("reserved0", ctypes.c_uint32),
        ("E", ctypes.c_double), ("lo", ctypes.c_double), ("hi", ctypes.c_double),
        ("packed_bytes", ctypes.c_uint64), ("compressed_bytes", ctypes.c_uint64),
        ("tail_count", ctypes.c_uint64), ("window_base", ctypes.c_int64),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class NumarckLosslessHeader(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_uint64), ("n_sub", ctypes.c_uint64), ("stream_words", ctypes.c_uint64),
        ("bits", ctypes.c_uint64), ("B", ctypes.c_uint32), ("k", ctypes.c_uint32),
        ("flags", ctypes.c_uint32), ("sub_log2", ctypes.c_uint16),
        ("group_log2", ctypes.c_uint16), ("bytes", ctypes.c_uint64),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class NumarckOut(ctypes.Structure):
    _fields_ = [
        ("packed", ctypes.c_void_p), ("centers", ctypes.c_void_p), ("incomp", ctypes.c_void_p),
        ("block_inc_off", ctypes.c_void_p), ("recon", ctypes.c_void_p),
        ("bin_ids", ctypes.c_void_p), ("hdr", ctypes.c_void_p),
    ]


class NumarckTuning(ctypes.Structure):
    _fields_ = [
        ("range_blocks_per_cu", ctypes.c_uint32), ("hist_blocks_per_cu", ctypes.c_uint32),
        ("hist_lds", ctypes.c_uint32), ("chunk_vec", ctypes.c_uint32),
        ("unit_pct", ctypes.c_uint32), ("stream_loads", ctypes.c_uint32),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class NumarckJob(ctypes.Structure):
    _fields_ = [
        ("prev", ctypes.c_void_p), ("curr", ctypes.c_void_p), ("n", ctypes.c_uint64),
        ("dtype", ctypes.c_int), ("E", ctypes.c_double), ("B", ctypes.c_uint32),
        ("block_bytes", ctypes.c_uint64), ("out", NumarckOut), ("tail_cap", ctypes.c_uint64),
    ]


class NumarckPlanGroup(ctypes.Structure):
    _fields_ = [(name, ctypes.c_uint32) for name in
                ("pass_", "dtype", "cls", "first_job", "njobs", "chain", "load_hint", "hist_lds")]

    def as_dict(self) -> dict:
        d = {name: getattr(self, name) for name, _ in self._fields_}
        d["pass"] = ("range", "hist", "encode")[d.pop("pass_")]
        return d


class NumarckServerConfig(ctypes.Structure):
    _fields_ = [
        ("budget_bytes", ctypes.c_uint64), ("arena_bytes", ctypes.c_uint64),
        ("slots", ctypes.c_uint32), ("max_batch", ctypes.c_uint32), ("device", ctypes.c_int32),
        ("reserved", ctypes.c_uint32),
    ]


class NumarckRequest(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_uint32), ("var", ctypes.c_uint32), ("curr", ctypes.c_void_p),
        ("start", ctypes.c_uint64), ("len", ctypes.c_uint64), ("out", ctypes.c_void_p),
        ("ready", ctypes.c_void_p),
    ]


class NumarckCompletion(ctypes.Structure):
    _fields_ = [
        ("ticket", ctypes.c_uint64), ("var", ctypes.c_uint32), ("kind", ctypes.c_uint32),
        ("status", ctypes.c_int32), ("flags", ctypes.c_uint32), ("bytes", ctypes.c_uint64),
        ("batch", ctypes.c_uint64), ("submit_us", ctypes.c_double),
        ("start_us", ctypes.c_double), ("done_us", ctypes.c_double),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class NumarckServerStats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_uint64) for f in (
        "submitted", "completed", "batches", "max_batch_seen", "arena_capacity", "arena_peak",
        "resident_bytes", "waits_for_memory", "tail_retries")]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


HEADER_BYTES = ctypes.sizeof(NumarckHeader)
MAX_JOBS = 65535
REQ_COMPRESS, REQ_RANGE = 0, 1

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                      "(the NUMARCK path has no CPU fallback)")
_lib = ctypes.CDLL(LIB_PATH)

_u64, _u32, _sz, _vp, _d = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_double
_i = ctypes.c_int


def _bind(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


numarck_packed_bytes = _bind("numarck_packed_bytes", _sz, [_u64, _u32])
numarck_centers_bytes = _bind("numarck_centers_bytes", _sz, [_u32, _i])
numarck_elems_per_block = _bind("numarck_elems_per_block", _u64, [_u32, _u64])
numarck_block_count = _bind("numarck_block_count", _u64, [_u64, _u32, _u64])
numarck_workspace_bytes = _bind("numarck_workspace_bytes", _sz, [_u64, _i, _u32])
numarck_workspace_bytes_tail = _bind("numarck_workspace_bytes_tail", _sz, [_u64, _i, _u64])
numarck_decompress_workspace_bytes = _bind("numarck_decompress_workspace_bytes", _sz, [_u64])
numarck_compress = _bind("numarck_compress", _i,
                         [_vp, _vp, _u64, _i, _d, _u32, _u64, ctypes.POINTER(NumarckOut), _vp,
                          _sz, _vp])
numarck_lossless_subblocks = _bind("numarck_lossless_subblocks", _u64, [_u64])
numarck_lossless_stream_bytes = _bind("numarck_lossless_stream_bytes", _sz, [_u64, _u32])
numarck_lossless_workspace_bytes = _bind("numarck_lossless_workspace_bytes", _sz, [_u32])
numarck_lossless_encode = _bind("numarck_lossless_encode", _i,
                                [_vp, _u64, _u32, _vp, _vp, _vp, _sz, _vp, _vp, _sz, _vp])
numarck_lossless_decode = _bind("numarck_lossless_decode", _i,
                                [ctypes.POINTER(NumarckLosslessHeader), _vp, _vp, _vp, _vp, _vp,
                                 _vp])
numarck_lossless_decode_range = _bind("numarck_lossless_decode_range", _i,
                                      [ctypes.POINTER(NumarckLosslessHeader), _vp, _vp, _vp,
                                       _u64, _u64, _vp, _vp, _vp])
numarck_compress_zero_anchored = _bind("numarck_compress_zero_anchored", _i,
                                       [_vp, _vp, _u64, _i, _d, _u32, _u64,
                                        ctypes.POINTER(NumarckOut), _vp, _sz, _vp])
numarck_compress_equal_width = _bind("numarck_compress_equal_width", _i,
                                     [_vp, _vp, _u64, _i, _d, _u32, _u64,
                                      ctypes.POINTER(NumarckOut), _vp, _sz, _vp])
numarck_compress_auto = _bind("numarck_compress_auto", _i,
                              [_vp, _vp, _u64, _i, _d, _u32, _u32, _u64,
                               ctypes.POINTER(NumarckOut), _vp, _sz, _vp,
                               ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint64)])
numarck_decompress = _bind("numarck_decompress", _i,
                           [ctypes.POINTER(NumarckHeader), _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                            _vp, _sz, _vp])
numarck_decompress_range = _bind("numarck_decompress_range", _i,
                                 [ctypes.POINTER(NumarckHeader), _vp, _vp, _vp, _vp, _vp, _u64,
                                  _u64, _vp, _vp, _vp, _sz, _vp])
numarck_stream_kernel = _bind("numarck_stream_kernel", _i, [_i, _vp, _vp, _u64, _u32, _vp])
(STREAM_READ, STREAM_READ_NT, STREAM_WRITE, STREAM_WRITE_NT, STREAM_COPY, STREAM_COPY_NT,
 STREAM_READ2_WRITE16, STREAM_READ2_WRITE8) = range(8)
numarck_static_scratch_bytes = _bind("numarck_static_scratch_bytes", _sz, [])
numarck_decompress_range_noalloc = _bind("numarck_decompress_range_noalloc", _i,
                                         [ctypes.POINTER(NumarckHeader), _vp, _vp, _vp, _vp,
                                          _vp, _u64, _u64, _vp, _vp, _vp])
numarck_histogram_export = _bind("numarck_histogram_export", _i,
                                 [_vp, _sz, _u64, _i, _vp, _vp, _u64, _vp, _vp])
numarck_tuning_default = _bind("numarck_tuning_default", None, [ctypes.POINTER(NumarckTuning)])
numarck_compress_tuned = _bind("numarck_compress_tuned", _i,
                               [_vp, _vp, _u64, _i, _d, _u32, _u64, ctypes.POINTER(NumarckOut),
                                _vp, _sz, ctypes.POINTER(NumarckTuning), _vp])
numarck_autotune = _bind("numarck_autotune", _i,
                         [_vp, _vp, _u64, _i, _d, _u32, _u64, ctypes.POINTER(NumarckOut), _vp,
                          _sz, _u32, _vp, ctypes.POINTER(NumarckTuning)])
numarck_tuning_save = _bind("numarck_tuning_save", _i, [ctypes.c_char_p])
numarck_tuning_load = _bind("numarck_tuning_load", _i, [ctypes.c_char_p])
numarck_batch_workspace_bytes = _bind("numarck_batch_workspace_bytes", _sz,
                                      [ctypes.POINTER(NumarckJob), _u32])
numarck_plan_create = _bind("numarck_plan_create", _i,
                            [ctypes.POINTER(NumarckJob), _u32, ctypes.POINTER(NumarckTuning), _vp,
                             _sz, _vp, ctypes.POINTER(_vp)])
numarck_plan_create_zero_anchored = _bind("numarck_plan_create_zero_anchored", _i,
                                          [ctypes.POINTER(NumarckJob), _u32,
                                           ctypes.POINTER(NumarckTuning), _vp, _sz, _vp,
                                           ctypes.POINTER(_vp)])
numarck_plan_run = _bind("numarck_plan_run", _i, [_vp, _vp])
numarck_plan_capture = _bind("numarck_plan_capture", _i, [_vp, _vp])
numarck_plan_replay = _bind("numarck_plan_replay", _i, [_vp, _vp])
numarck_plan_destroy = _bind("numarck_plan_destroy", None, [_vp])
numarck_plan_autotune = _bind("numarck_plan_autotune", _i,
                              [ctypes.POINTER(NumarckJob), _u32, _vp, _sz, _u32, _u32, _vp,
                               ctypes.POINTER(NumarckTuning)])
numarck_plan_groups = _bind("numarck_plan_groups", _u32,
                            [_vp, ctypes.POINTER(NumarckPlanGroup), _u32])
numarck_compress_batch = _bind("numarck_compress_batch", _i,
                               [ctypes.POINTER(NumarckJob), _u32, _vp, _sz, _vp])
numarck_server_create = _bind("numarck_server_create", _i,
                              [ctypes.POINTER(NumarckServerConfig), ctypes.POINTER(_vp)])
numarck_server_add_variable = _bind("numarck_server_add_variable", _i,
                                    [_vp, _u64, _i, _d, _u32, _u64, _vp, ctypes.POINTER(_u32)])
numarck_server_submit = _bind("numarck_server_submit", _i,
                              [_vp, ctypes.POINTER(NumarckRequest), ctypes.POINTER(_u64)])
numarck_server_poll = _bind("numarck_server_poll", _u32,
                            [_vp, ctypes.POINTER(NumarckCompletion), _u32])
numarck_server_drain = _bind("numarck_server_drain", _i, [_vp])
numarck_server_fetch = _bind("numarck_server_fetch", _i, [_vp, _u32, ctypes.POINTER(NumarckOut), _vp])
numarck_server_get_stats = _bind("numarck_server_get_stats", _i,
                                 [_vp, ctypes.POINTER(NumarckServerStats)])
numarck_server_destroy = _bind("numarck_server_destroy", None, [_vp])
numarck_status_str = _bind("numarck_status_str", ctypes.c_char_p, [_i])
numarck_last_error = _bind("numarck_last_error", ctypes.c_char_p, [])
numarck_timing_enable = _bind("numarck_timing_enable", None, [_i])
numarck_timing_read = _bind("numarck_timing_read", _i,
                            [ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(_u32),
                             ctypes.POINTER(_d), _i])


class NumarckError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = numarck_status_str(status).decode()
        if status == EHIP:
            msg += ": " + numarck_last_error().decode()
        super().__init__(f"{where}: {msg} (status {status})")
        self.status = status


def _check(st: int, where: str):
    if st != OK:
        raise NumarckError(st, where)


def _ptr(t):
    return None if t is None else t.data_ptr()


def _stream(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def dtype_code(t: torch.dtype) -> int:
    if t == torch.float32:
        return F32
    if t == torch.float64:
        return F64
    raise ValueError(f"unsupported dtype {t}")


def header_from_device(hdr: torch.Tensor) -> NumarckHeader:
    """Copy a device header (uint8 tensor) to the host; synchronises its stream."""
    raw = hdr.cpu().numpy().tobytes()
    return NumarckHeader.from_buffer_copy(raw)


@dataclass
class Compressed:
    """Device buffers of one compression.  ``incomp`` has room for n values;
    its first ``header().n_inc`` entries are meaningful."""
    packed: torch.Tensor
    centers: torch.Tensor
    incomp: torch.Tensor
    block_inc_off: torch.Tensor
    recon: torch.Tensor | None
    bin_ids: torch.Tensor | None
    hdr: torch.Tensor
    ws: torch.Tensor | None  # the workspace of a plain compression (histogram export)
    n: int
    dtype: torch.dtype
    _host: NumarckHeader | None = None

    def header(self) -> NumarckHeader:
        if self._host is None:
            self._host = header_from_device(self.hdr)
        return self._host


def alloc_outputs(n: int, dtype: torch.dtype, B: int, block_bytes: int = 0, recon=False,
                  bin_ids=False, device="cuda"):
    L = 4 if dtype == torch.float32 else 8
    pw = numarck_packed_bytes(n, B) // 4
    nb = numarck_block_count(n, B, block_bytes)
    return dict(
        packed=torch.empty(max(pw, 1), dtype=torch.int32, device=device),
        centers=torch.empty(1 << B, dtype=dtype, device=device),
        incomp=torch.empty(max(n, 1), dtype=dtype, device=device),
        block_inc_off=torch.empty(max(nb, 1), dtype=torch.int64, device=device),
        recon=torch.empty(max(n, 1), dtype=dtype, device=device) if recon else None,
        bin_ids=torch.empty(max((1 << B) - 1, 1), dtype=torch.int64, device=device) if bin_ids else None,
        hdr=torch.empty(HEADER_BYTES, dtype=torch.uint8, device=device),
    )


def out_struct(o: dict) -> NumarckOut:
    return NumarckOut(_ptr(o["packed"]), _ptr(o["centers"]), _ptr(o["incomp"]),
                      _ptr(o["block_inc_off"]), _ptr(o["recon"]), _ptr(o["bin_ids"]),
                      _ptr(o["hdr"]))


def compress(prev: torch.Tensor, curr: torch.Tensor, E: float, B: int, block_bytes: int = 0,
             recon: bool = False, bin_ids: bool = False, ws: torch.Tensor | None = None,
             outputs: dict | None = None, stream=None, _tune=None) -> Compressed:
    """Compress `curr` against `prev` (1-D contiguous float32/float64 device tensors)."""
    if prev.dtype != curr.dtype or prev.numel() != curr.numel():
        raise ValueError("prev and curr must have the same dtype and size")
    if not (prev.is_cuda and curr.is_cuda):
        raise ValueError("prev and curr must be device tensors")
    prev = prev.reshape(-1)
    curr = curr.reshape(-1)
    n = prev.numel()
    dt = dtype_code(prev.dtype)
    o = outputs if outputs is not None else alloc_outputs(n, prev.dtype, B, block_bytes, recon,
                                                          bin_ids, prev.device)
    if ws is None:
        ws = torch.empty(numarck_workspace_bytes(n, dt, B), dtype=torch.uint8, device=prev.device)
    out = out_struct(o)
    if _tune is None:
        st = numarck_compress(_ptr(prev), _ptr(curr), n, dt, float(E), int(B), int(block_bytes),
                              ctypes.byref(out), _ptr(ws), ws.numel(), _stream(stream))
    else:
        st = numarck_compress_tuned(_ptr(prev), _ptr(curr), n, dt, float(E), int(B),
                                    int(block_bytes), ctypes.byref(out), _ptr(ws), ws.numel(),
                                    ctypes.byref(_tune) if _tune is not False else None,
                                    _stream(stream))
    _check(st, "numarck_compress")
    return Compressed(o["packed"], o["centers"], o["incomp"], o["block_inc_off"], o["recon"],
                      o["bin_ids"], o["hdr"], ws, n, prev.dtype)


def compress_zero_anchored(prev: torch.Tensor, curr: torch.Tensor, E: float, B: int,
                           block_bytes: int = 0, recon: bool = False, bin_ids: bool = False,
                           ws: torch.Tensor | None = None, outputs: dict | None = None,
                           stream=None) -> Compressed:
    """:func:`compress` with the fine bins anchored at -E, centred on multiples
    of 2E (numarck_compress_zero_anchored): two passes over the snapshots."""
    return _compress_variant(numarck_compress_zero_anchored, "numarck_compress_zero_anchored",
                             prev, curr, E, B, block_bytes, recon, bin_ids, ws, outputs, stream)


def compress_equal_width(prev: torch.Tensor, curr: torch.Tensor, E: float, B: int,
                         block_bytes: int = 0, recon: bool = False, bin_ids: bool = False,
                         ws: torch.Tensor | None = None, outputs: dict | None = None,
                         stream=None) -> Compressed:
    """:func:`compress` with equal-width binning (numarck_compress_equal_width):
    the 2^B - 1 bins cut evenly from the range of the ratios."""
    return _compress_variant(numarck_compress_equal_width, "numarck_compress_equal_width",
                             prev, curr, E, B, block_bytes, recon, bin_ids, ws, outputs, stream)


def _compress_variant(fn, name, prev, curr, E, B, block_bytes, recon, bin_ids, ws, outputs,
                      stream) -> Compressed:
    if prev.dtype != curr.dtype or prev.numel() != curr.numel():
        raise ValueError("prev and curr must have the same dtype and size")
    if not (prev.is_cuda and curr.is_cuda):
        raise ValueError("prev and curr must be device tensors")
    prev = prev.reshape(-1)
    curr = curr.reshape(-1)
    n = prev.numel()
    dt = dtype_code(prev.dtype)
    o = outputs if outputs is not None else alloc_outputs(n, prev.dtype, B, block_bytes, recon,
                                                          bin_ids, prev.device)
    if ws is None:
        ws = torch.empty(numarck_workspace_bytes(n, dt, B), dtype=torch.uint8, device=prev.device)
    out = out_struct(o)
    st = fn(_ptr(prev), _ptr(curr), n, dt, float(E), int(B), int(block_bytes), ctypes.byref(out),
            _ptr(ws), ws.numel(), _stream(stream))
    _check(st, name)
    return Compressed(o["packed"], o["centers"], o["incomp"], o["block_inc_off"], o["recon"],
                      o["bin_ids"], o["hdr"], ws, n, prev.dtype)


def compress_auto(prev: torch.Tensor, curr: torch.Tensor, E: float, B_min: int = 1,
                  B_max: int = 16, block_bytes: int = 0, recon: bool = False,
                  bin_ids: bool = False, ws: torch.Tensor | None = None,
                  outputs: dict | None = None, stream=None):
    """:func:`compress` with B chosen in [B_min, B_max] from the histogram
    (numarck_compress_auto).  Returns (Compressed, B, est_bits): est_bits[B]
    is the estimated compressed size in bits of each B of the range."""
    if prev.dtype != curr.dtype or prev.numel() != curr.numel():
        raise ValueError("prev and curr must have the same dtype and size")
    prev = prev.reshape(-1)
    curr = curr.reshape(-1)
    n = prev.numel()
    dt = dtype_code(prev.dtype)
    o = outputs if outputs is not None else alloc_outputs(n, prev.dtype, B_max, block_bytes,
                                                          recon, bin_ids, prev.device)
    if ws is None:
        ws = torch.empty(numarck_workspace_bytes(n, dt, B_max), dtype=torch.uint8,
                         device=prev.device)
    out = out_struct(o)
    B = ctypes.c_uint32(0)
    bits = (ctypes.c_uint64 * 17)()
    st = numarck_compress_auto(_ptr(prev), _ptr(curr), n, dt, float(E), int(B_min), int(B_max),
                               int(block_bytes), ctypes.byref(out), _ptr(ws), ws.numel(),
                               _stream(stream), ctypes.byref(B), bits)
    _check(st, "numarck_compress_auto")
    c = Compressed(o["packed"], o["centers"], o["incomp"], o["block_inc_off"], o["recon"],
                   o["bin_ids"], o["hdr"], ws, n, prev.dtype)
    return c, int(B.value), [int(x) for x in bits]


def default_tuning() -> NumarckTuning:
    t = NumarckTuning()
    numarck_tuning_default(ctypes.byref(t))
    return t


def compress_tuned(prev: torch.Tensor, curr: torch.Tensor, E: float, B: int,
                   tune: NumarckTuning | None, block_bytes: int = 0, ws: torch.Tensor | None = None,
                   outputs: dict | None = None, stream=None) -> Compressed:
    """:func:`compress` with explicit launch tuning (None: the recorded one)."""
    return compress(prev, curr, E, B, block_bytes, ws=ws, outputs=outputs, stream=stream,
                    _tune=tune if tune is not None else False)


def autotune(prev: torch.Tensor, curr: torch.Tensor, E: float, B: int, block_bytes: int = 0,
             reps: int = 3, stream=None) -> NumarckTuning:
    """Measure launch tunings on one compression; records and returns the fastest."""
    prev, curr = prev.reshape(-1), curr.reshape(-1)
    n, dt = prev.numel(), dtype_code(prev.dtype)
    o = alloc_outputs(n, prev.dtype, B, block_bytes, device=prev.device)
    ws = torch.empty(numarck_workspace_bytes(n, dt, B), dtype=torch.uint8, device=prev.device)
    out = out_struct(o)
    best = NumarckTuning()
    st = numarck_autotune(_ptr(prev), _ptr(curr), n, dt, float(E), int(B), int(block_bytes),
                          ctypes.byref(out), _ptr(ws), ws.numel(), int(reps), _stream(stream),
                          ctypes.byref(best))
    _check(st, "numarck_autotune")
    return best


@dataclass
class BatchJob:
    """One compression of a batch: curr against prev with its own E, B and block size."""
    prev: torch.Tensor
    curr: torch.Tensor
    E: float
    B: int
    block_bytes: int = 0
    tail_cap: int = 0  # 0: n (never overflows)


@dataclass
class Lossless:
    """Device buffers of the lossless stage of one index table."""
    code_of_rank: torch.Tensor  # int16 view of 2^B uint16
    sub_off: torch.Tensor       # int64 view of n_sub + 1 uint64 (bits)
    stream: torch.Tensor        # int32 view of the codeword words
    hdr: torch.Tensor           # uint8 device header
    n: int
    B: int
    _host: NumarckLosslessHeader | None = None

    def header(self) -> NumarckLosslessHeader:
        if self._host is None:
            raw = self.hdr.cpu().numpy().tobytes()
            self._host = NumarckLosslessHeader.from_buffer_copy(raw)
        return self._host


def lossless_encode(packed: torch.Tensor, n: int, B: int, ws: torch.Tensor | None = None,
                    stream=None) -> Lossless:
    """Lossless stage of an index table of n B-bit codes (numarck_lossless_encode);
    `packed` is e.g. ``Compressed.packed``."""
    dev = packed.device
    nsub = int(numarck_lossless_subblocks(n))
    sb = numarck_lossless_stream_bytes(n, B)
    cor = torch.empty(1 << B, dtype=torch.int16, device=dev)
    sub = torch.empty(nsub + 1, dtype=torch.int64, device=dev)
    st = torch.empty(max(sb // 4, 1), dtype=torch.int32, device=dev)
    hdr = torch.empty(ctypes.sizeof(NumarckLosslessHeader), dtype=torch.uint8, device=dev)
    if ws is None:
        ws = torch.empty(numarck_lossless_workspace_bytes(B), dtype=torch.uint8, device=dev)
    r = numarck_lossless_encode(_ptr(packed), n, B, _ptr(cor), _ptr(sub), _ptr(st), st.numel() * 4,
                                _ptr(hdr), _ptr(ws), ws.numel(), _stream(stream))
    _check(r, "numarck_lossless_encode")
    return Lossless(cor, sub, st, hdr, n, B)


def lossless_decode(enc: Lossless, out: torch.Tensor | None = None, stream=None):
    """The index table of a lossless stream; returns (packed int32 words, flags)."""
    h = enc.header()
    dev = enc.stream.device
    words = (enc.n * enc.B + 31) // 32
    if out is None:
        out = torch.empty(max(words, 1), dtype=torch.int32, device=dev)
    flags = torch.zeros(1, dtype=torch.int32, device=dev)
    r = numarck_lossless_decode(ctypes.byref(h), _ptr(enc.code_of_rank), _ptr(enc.sub_off),
                                _ptr(enc.stream), _ptr(out), _ptr(flags), _stream(stream))
    _check(r, "numarck_lossless_decode")
    return out[:words], flags


def lossless_decode_codes(enc: Lossless, first: int, last: int, out: torch.Tensor, stream=None):
    """Decode only the sub-blocks holding codes [first, last) into their places
    in the full-size table `out` (numarck_lossless_decode_range); returns the
    flags tensor."""
    h = enc.header()
    sb = 1 << h.sub_log2  # codes per sub-block, as the stream records it
    s0 = first // sb
    s1 = min((last + sb - 1) // sb, h.n_sub) if last > first else s0
    flags = torch.zeros(1, dtype=torch.int32, device=out.device)
    r = numarck_lossless_decode_range(ctypes.byref(h), _ptr(enc.code_of_rank), _ptr(enc.sub_off),
                                      _ptr(enc.stream), s0, s1 - s0, _ptr(out), _ptr(flags),
                                      _stream(stream))
    _check(r, "numarck_lossless_decode_range")
    return flags


class ClosedLoop:
    """Closed-loop compression of a time series: each snapshot is compressed
    against the reconstruction of the one before (which a reader rebuilds
    from the records), not against the original, so the reconstruction error
    of every step stays within E of the reconstructed previous value instead
    of compounding.  Each call is one numarck_compress (or the zero-anchored
    or equal-width entry) writing its reconstruction, which becomes the next
    call's previous snapshot; two reconstruction buffers alternate.  The
    first snapshot is kept as given (the series' full checkpoint)."""

    _FNS = {"topk": "compress", "zero_anchored": "compress_zero_anchored",
            "equal_width": "compress_equal_width"}

    def __init__(self, first: torch.Tensor, E: float, B: int, block_bytes: int = 0,
                 binning: str = "topk", stream=None):
        if binning not in self._FNS:
            raise ValueError(f"unknown binning {binning}")
        x = first.reshape(-1)
        self.E, self.B, self.block_bytes, self.stream = E, B, block_bytes, stream
        self._fn = globals()[self._FNS[binning]]
        n = x.numel()
        self._bufs = [x.clone(), torch.empty_like(x)]
        self._cur = 0
        self._ws = torch.empty(numarck_workspace_bytes(n, dtype_code(x.dtype), B),
                               dtype=torch.uint8, device=x.device)

    @property
    def reconstruction(self) -> torch.Tensor:
        """The reconstruction of the latest snapshot (what a reader decodes)."""
        return self._bufs[self._cur]

    def push(self, curr: torch.Tensor) -> Compressed:
        """Compress `curr` against the current reconstruction; the returned
        record's `recon` is the new reconstruction (valid until the call
        after next)."""
        prev = self._bufs[self._cur]
        nxt = self._bufs[1 - self._cur]
        n = prev.numel()
        o = alloc_outputs(n, prev.dtype, self.B, self.block_bytes, False, False, prev.device)
        o["recon"] = nxt
        c = self._fn(prev, curr.reshape(-1), self.E, self.B, self.block_bytes, ws=self._ws,
                     outputs=o, stream=self.stream)
        c.ws = None  # the workspace is reused by the next call
        self._cur = 1 - self._cur
        return c


def _job_array(jobs: list[BatchJob], recon: bool, bin_ids: bool, outputs: list[dict] | None):
    """The numarck_job array of a batch, its outputs and its workspace."""
    if not jobs:
        raise ValueError("empty batch")
    kept, outs = [], []
    arr = (NumarckJob * len(jobs))()
    for i, j in enumerate(jobs):
        p, q = j.prev.reshape(-1), j.curr.reshape(-1)
        if p.dtype != q.dtype or p.numel() != q.numel() or not (p.is_cuda and q.is_cuda):
            raise ValueError(f"job {i}: prev and curr must be device tensors of one dtype and size")
        o = outputs[i] if outputs is not None else alloc_outputs(
            p.numel(), p.dtype, j.B, j.block_bytes, recon, bin_ids, p.device)
        arr[i] = NumarckJob(_ptr(p), _ptr(q), p.numel(), dtype_code(p.dtype), float(j.E),
                            int(j.B), int(j.block_bytes), out_struct(o), int(j.tail_cap))
        kept.append((p, q, j))
        outs.append(o)
    ws = torch.empty(max(numarck_batch_workspace_bytes(arr, len(jobs)), 1), dtype=torch.uint8,
                     device=jobs[0].prev.device)
    return kept, outs, arr, ws


def plan_autotune(jobs: list[BatchJob], reps: int = 3, zero_anchored: bool = False,
                  outputs: list[dict] | None = None, stream=None) -> NumarckTuning:
    """numarck_plan_autotune: the fastest launch tuning for this batch."""
    kept, outs, arr, ws = _job_array(jobs, False, False, outputs)
    best = NumarckTuning()
    _check(numarck_plan_autotune(arr, len(jobs), _ptr(ws), ws.numel(), int(reps),
                                 1 if zero_anchored else 0, _stream(stream), ctypes.byref(best)),
           "numarck_plan_autotune")
    return best


class Plan:
    """A batch plan (numarck_plan_*): the jobs' outputs are allocated here (or
    passed in), the descriptors are uploaded once; :meth:`run` launches the
    chain, :meth:`capture` / :meth:`replay` use a HIP graph of it."""

    def __init__(self, jobs: list[BatchJob], recon: bool = False, bin_ids: bool = False,
                 outputs: list[dict] | None = None, tune: NumarckTuning | None = None,
                 stream=None, zero_anchored: bool = False):
        self.jobs, self.outputs, arr, self.ws = _job_array(jobs, recon, bin_ids, outputs)
        self._arr = arr
        h = _vp()
        create = numarck_plan_create_zero_anchored if zero_anchored else numarck_plan_create
        st = create(arr, len(jobs), ctypes.byref(tune) if tune is not None else None,
                    _ptr(self.ws), self.ws.numel(), _stream(stream), ctypes.byref(h))
        _check(st, "numarck_plan_create")
        self._h = h

    def results(self) -> list[Compressed]:
        return [Compressed(o["packed"], o["centers"], o["incomp"], o["block_inc_off"],
                           o["recon"], o["bin_ids"], o["hdr"], None, p.numel(), p.dtype)
                for (p, _, _), o in zip(self.jobs, self.outputs)]

    def run(self, stream=None) -> list[Compressed]:
        _check(numarck_plan_run(self._h, _stream(stream)), "numarck_plan_run")
        return self.results()

    def groups(self) -> list[dict]:
        """The plan's launch groups (numarck_plan_groups), in launch order."""
        k = numarck_plan_groups(self._h, None, 0)
        arr = (NumarckPlanGroup * max(k, 1))()
        numarck_plan_groups(self._h, arr, k)
        return [arr[i].as_dict() for i in range(k)]

    def capture(self, stream):
        _check(numarck_plan_capture(self._h, _stream(stream)), "numarck_plan_capture")

    def replay(self, stream=None) -> list[Compressed]:
        _check(numarck_plan_replay(self._h, _stream(stream)), "numarck_plan_replay")
        return self.results()

    def close(self):
        if self._h:
            numarck_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def compress_batch(jobs: list[BatchJob], recon: bool = False, bin_ids: bool = False,
                   stream=None) -> list[Compressed]:
    """One-shot batch through numarck_compress_batch."""
    arr = (NumarckJob * len(jobs))()
    outs = []
    for i, j in enumerate(jobs):
        p, q = j.prev.reshape(-1), j.curr.reshape(-1)
        o = alloc_outputs(p.numel(), p.dtype, j.B, j.block_bytes, recon, bin_ids, p.device)
        arr[i] = NumarckJob(_ptr(p), _ptr(q), p.numel(), dtype_code(p.dtype), float(j.E),
                            int(j.B), int(j.block_bytes), out_struct(o), int(j.tail_cap))
        outs.append((p, o))
    dev = jobs[0].prev.device
    ws = torch.empty(max(numarck_batch_workspace_bytes(arr, len(jobs)), 1), dtype=torch.uint8,
                     device=dev)
    _check(numarck_compress_batch(arr, len(jobs), _ptr(ws), ws.numel(), _stream(stream)),
           "numarck_compress_batch")
    res = [Compressed(o["packed"], o["centers"], o["incomp"], o["block_inc_off"], o["recon"],
                      o["bin_ids"], o["hdr"], None, p.numel(), p.dtype) for p, o in outs]
    for c in res:
        c._batch_ws = ws  # keep the workspace alive until the chain has run
    return res


class Server:
    """The serving loop (numarck_server_*): variables keep their previous
    snapshot resident; compression and range requests of different variables
    are batched by the library's scheduler thread under a device memory
    budget.  This wrapper only keeps the tensors it hands to the library
    alive while the library may still read or write them."""

    def __init__(self, budget_bytes: int, arena_bytes: int, slots: int = 2, max_batch: int = 64,
                 device: int = 0):
        cfg = NumarckServerConfig(int(budget_bytes), int(arena_bytes), int(slots), int(max_batch),
                                  int(device), 0)
        h = _vp()
        _check(numarck_server_create(ctypes.byref(cfg), ctypes.byref(h)), "numarck_server_create")
        self._h = h
        self.vars = []        # (n, torch dtype, E, B, block_bytes)
        # snapshot k of a variable is the reference of its record k + 1, so it
        # stays referenced until compression k + 2 has completed
        self._keep = {}       # var -> [(sequence number, snapshot)]
        self._seq = {}        # var -> snapshots handed over so far
        self._done = {}       # var -> compressions completed
        self._inflight = {}   # ticket -> tensors / events the request uses
        self._kind = {}       # ticket -> (var, kind)

    def add_variable(self, initial: torch.Tensor, E: float, B: int, block_bytes: int = 0) -> int:
        x = initial.reshape(-1)
        v = _u32()
        st = numarck_server_add_variable(self._h, x.numel(), dtype_code(x.dtype), float(E), int(B),
                                         int(block_bytes), _ptr(x), ctypes.byref(v))
        _check(st, "numarck_server_add_variable")
        self.vars.append((x.numel(), x.dtype, float(E), int(B), int(block_bytes)))
        self._keep[v.value] = [(0, x)]  # (sequence number, snapshot)
        self._seq[v.value] = 0
        self._done[v.value] = 0
        return v.value

    def _submit(self, req: NumarckRequest, keep) -> int:
        t = _u64()
        _check(numarck_server_submit(self._h, ctypes.byref(req), ctypes.byref(t)),
               "numarck_server_submit")
        self._inflight[t.value] = keep
        return t.value

    def compress(self, var: int, curr: torch.Tensor, ready: "torch.cuda.Event | None" = None) -> int:
        x = curr.reshape(-1)
        req = NumarckRequest(REQ_COMPRESS, var, _ptr(x), 0, 0, None,
                             ready.cuda_event if ready is not None else None)
        t = self._submit(req, (x, ready))
        self._seq[var] += 1
        self._keep[var].append((self._seq[var], x))
        self._kind[t] = (var, REQ_COMPRESS)
        return t

    def range(self, var: int, start: int, length: int, out: torch.Tensor | None = None,
              ready: "torch.cuda.Event | None" = None):
        n, dt = self.vars[var][0], self.vars[var][1]
        if out is None:
            out = torch.empty(max(length, 1), dtype=dt, device="cuda")
        req = NumarckRequest(REQ_RANGE, var, None, int(start), int(length), _ptr(out),
                             ready.cuda_event if ready is not None else None)
        return self._submit(req, (out, ready)), out

    def poll(self, cap: int = 4096) -> list[dict]:
        buf = (NumarckCompletion * cap)()
        k = numarck_server_poll(self._h, buf, cap)
        res = [buf[i].as_dict() for i in range(k)]
        for c in res:
            self._inflight.pop(c["ticket"], None)
            var, kind = self._kind.pop(c["ticket"], (c["var"], c["kind"]))
            if kind == REQ_COMPRESS and c["status"] == OK:
                self._done[var] += 1
                lim = self._done[var] - 1
                self._keep[var] = [(q, x) for q, x in self._keep[var] if q >= lim]
        return res

    def drain(self):
        _check(numarck_server_drain(self._h), "numarck_server_drain")

    def fetch(self, var: int, stream=None) -> Compressed:
        n, dt, E, B, bb = self.vars[var]
        o = alloc_outputs(n, dt, B, bb)
        out = out_struct(o)
        _check(numarck_server_fetch(self._h, var, ctypes.byref(out), _stream(stream)),
               "numarck_server_fetch")
        return Compressed(o["packed"], o["centers"], o["incomp"], o["block_inc_off"], None, None,
                          o["hdr"], None, n, dt)

    def stats(self) -> dict:
        st = NumarckServerStats()
        _check(numarck_server_get_stats(self._h, ctypes.byref(st)), "numarck_server_get_stats")
        return st.as_dict()

    def close(self):
        if self._h:
            numarck_server_destroy(self._h)
            self._h = None
            self._inflight.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def decompress(c: Compressed, prev: torch.Tensor, out: torch.Tensor | None = None,
               stream=None):
    """Full decompression; returns (values, flags tensor)."""
    h = c.header()
    if out is None:
        out = torch.empty(max(h.n, 1), dtype=c.dtype, device=prev.device)
    flags = torch.zeros(1, dtype=torch.int32, device=prev.device)
    ws = torch.empty(numarck_decompress_workspace_bytes(h.n), dtype=torch.uint8, device=prev.device)
    st = numarck_decompress(ctypes.byref(h), _ptr(prev), _ptr(c.packed), _ptr(c.centers),
                            _ptr(c.incomp), _ptr(c.block_inc_off), _ptr(out), _ptr(flags),
                            _ptr(ws), ws.numel(), _stream(stream))
    _check(st, "numarck_decompress")
    return out[: h.n], flags


def decompress_range(c: Compressed, prev: torch.Tensor, start: int, length: int,
                     out: torch.Tensor | None = None, stream=None):
    """Partial decompression of [start, start + length); returns (values, flags)."""
    h = c.header()
    if out is None:
        out = torch.empty(max(length, 1), dtype=c.dtype, device=prev.device)
    flags = torch.zeros(1, dtype=torch.int32, device=prev.device)
    ws = torch.empty(numarck_decompress_workspace_bytes(length), dtype=torch.uint8,
                     device=prev.device)
    st = numarck_decompress_range(ctypes.byref(h), _ptr(prev), _ptr(c.packed), _ptr(c.centers),
                                  _ptr(c.incomp), _ptr(c.block_inc_off), int(start), int(length),
                                  _ptr(out), _ptr(flags), _ptr(ws), ws.numel(), _stream(stream))
    _check(st, "numarck_decompress_range")
    return out[:length], flags


def decompress_range_noalloc(c: Compressed, prev: torch.Tensor, start: int, length: int,
                             out: torch.Tensor, flags: torch.Tensor, stream=None):
    """numarck_decompress_range_noalloc into caller-provided `out` and `flags`
    (the library allocates nothing; its workspace is a device-global array)."""
    h = c.header()
    st = numarck_decompress_range_noalloc(ctypes.byref(h), _ptr(prev), _ptr(c.packed),
                                          _ptr(c.centers), _ptr(c.incomp), _ptr(c.block_inc_off),
                                          int(start), int(length), _ptr(out), _ptr(flags),
                                          _stream(stream))
    _check(st, "numarck_decompress_range_noalloc")
    return out[:length], flags


def histogram(c: Compressed, capacity: int | None = None, stream=None):
    """Nonzero fine bins of the compression `c` (unordered ids, counts)."""
    if capacity is None:
        capacity = max(c.n, 1)
    ids = torch.empty(max(capacity, 1), dtype=torch.int64, device=c.hdr.device)
    counts = torch.empty(max(capacity, 1), dtype=torch.int32, device=c.hdr.device)
    cnt = torch.zeros(1, dtype=torch.int64, device=c.hdr.device)
    st = numarck_histogram_export(_ptr(c.ws), c.ws.numel(), c.n, dtype_code(c.dtype), _ptr(ids),
                                  _ptr(counts), capacity, _ptr(cnt), _stream(stream))
    _check(st, "numarck_histogram_export")
    k = int(cnt.item())
    return ids[:min(k, capacity)], counts[:min(k, capacity)], k


def stream_kernel(kind: int, src: torch.Tensor | None, dst: torch.Tensor, nbytes: int,
                  per_cu: int = 8, stream=None):
    """One reference read / write / copy launch (numarck_stream_kernel)."""
    _check(numarck_stream_kernel(int(kind), _ptr(src), _ptr(dst), int(nbytes), int(per_cu),
                                 _stream(stream)), "numarck_stream_kernel")


def timing_enable(on: bool = True):
    numarck_timing_enable(1 if on else 0)


def timing_read(cap: int = 32) -> dict:
    names = (ctypes.c_char_p * cap)()
    launches = (_u32 * cap)()
    ms = (_d * cap)()
    k = numarck_timing_read(names, launches, ms, cap)
    return {names[i].decode(): (int(launches[i]), float(ms[i])) for i in range(k)}
