"""Python access to the plain CPU oracle of the NUMARCK compression path.

TEST INFRASTRUCTURE ONLY.  The oracle is a slow, plain C implementation of the
method of "Parallel Implementation of Lossy Data Compression for Temporal Data
Sets" (Yuan et al., arXiv 1703.02438); it exists so the tests, the smoke check
and the CPU-baseline leg of the benchmark can check the HIP library against an
independent implementation.  The product package never imports this module.

The C source (``numarck_oracle.c``) carries the step-by-step citations of the
paper; this module only marshals numpy arrays through ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "numarck_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libnumarck_oracle.so")

F32, F64 = 0, 1
FLAG_BAD_INDEX = 1
FLAG_INC_OVERRUN = 2

# Compile flags: binary64 evaluated as written (no FMA contraction, no fast-math).
# -fopenmp: the per-element loops may run on several threads (orc_set_threads;
# one by default), with identical results.
CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
          "-shared"]


def build(src: str = _SRC, out: str = _LIB_PATH, extra=()) -> str:
    """Compile the oracle with gcc into a shared library and return its path."""
    cmd = ["gcc", *CFLAGS, *extra, "-o", out, src, "-lm"]
    subprocess.run(cmd, check=True)
    return out


class _Info(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_uint64), ("n_valid", ctypes.c_uint64),
        ("n_invalid", ctypes.c_uint64), ("n_inc", ctypes.c_uint64),
        ("n_blocks", ctypes.c_uint64), ("elems_per_block", ctypes.c_uint64),
        ("block_bytes", ctypes.c_uint64), ("M", ctypes.c_int64),
        ("n_nonzero", ctypes.c_uint64),
        ("B", ctypes.c_uint32), ("k", ctypes.c_uint32), ("k_used", ctypes.c_uint32),
        ("dtype", ctypes.c_uint32), ("tau", ctypes.c_uint32),
        ("E", ctypes.c_double), ("lo", ctypes.c_double), ("hi", ctypes.c_double),
        ("packed_words", ctypes.c_uint64), ("packed_bytes", ctypes.c_uint64),
        ("compressed_bytes", ctypes.c_uint64),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


_VP = ctypes.c_void_p


class Oracle:
    """ctypes wrapper around one compiled oracle library (the default one, or
    a variant compiled from another source file)."""

    def __init__(self, path: str = _LIB_PATH):
        if not os.path.exists(path):
            if path != _LIB_PATH:
                raise FileNotFoundError(path)
            build()
        lib = ctypes.CDLL(path)
        lib.orc_set_threads.argtypes = [ctypes.c_int]
        lib.orc_set_threads.restype = ctypes.c_int
        lib.orc_ratio.argtypes = [_VP, _VP, ctypes.c_uint64, ctypes.c_int, ctypes.c_double, _VP, _VP]
        lib.orc_ratio.restype = ctypes.c_int
        lib.orc_range.argtypes = [_VP, _VP, ctypes.c_uint64, _VP, _VP]
        lib.orc_range.restype = ctypes.c_uint64
        lib.orc_bin_ids.argtypes = [_VP, _VP, ctypes.c_uint64, ctypes.c_double, ctypes.c_double, _VP]
        lib.orc_bin_ids.restype = None
        lib.orc_histogram.argtypes = [_VP, _VP, ctypes.c_uint64, _VP, _VP]
        lib.orc_histogram.restype = ctypes.c_int64
        lib.orc_topk.argtypes = [_VP, _VP, ctypes.c_int64, ctypes.c_uint32, _VP, _VP]
        lib.orc_topk.restype = ctypes.c_int64
        lib.orc_compress.argtypes = [_VP, _VP, ctypes.c_uint64, ctypes.c_int, ctypes.c_double,
                                     ctypes.c_uint32, ctypes.c_uint64, _VP, _VP, _VP, _VP, _VP,
                                     _VP, _VP, ctypes.POINTER(_Info)]
        lib.orc_compress.restype = ctypes.c_int
        lib.orc_lossless_subblocks.argtypes = [ctypes.c_uint64]
        lib.orc_lossless_subblocks.restype = ctypes.c_uint64
        lib.orc_lossless_encode.argtypes = [_VP, ctypes.c_uint64, ctypes.c_uint32, _VP,
                                            ctypes.POINTER(ctypes.c_uint32), _VP, _VP, _VP,
                                            ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint64)]
        lib.orc_lossless_encode.restype = ctypes.c_int
        lib.orc_lossless_decode.argtypes = [_VP, ctypes.c_uint32, _VP, _VP, ctypes.c_uint64,
                                            ctypes.c_uint32, _VP]
        lib.orc_lossless_decode.restype = ctypes.c_int
        lib.orc_compress_za.argtypes = lib.orc_compress.argtypes
        lib.orc_compress_za.restype = ctypes.c_int
        lib.orc_compress_ew.argtypes = [_VP, _VP, ctypes.c_uint64, ctypes.c_int, ctypes.c_double,
                                        ctypes.c_uint32, ctypes.c_uint64, _VP, _VP, _VP, _VP, _VP,
                                        _VP, ctypes.POINTER(_Info)]
        lib.orc_compress_ew.restype = ctypes.c_int
        lib.orc_choose_B.argtypes = [_VP, _VP, ctypes.c_uint64, ctypes.c_int, ctypes.c_double,
                                     ctypes.c_uint32, ctypes.c_uint32, _VP,
                                     ctypes.POINTER(ctypes.c_uint32)]
        lib.orc_choose_B.restype = ctypes.c_int
        lib.orc_decompress.argtypes = [ctypes.POINTER(_Info), _VP, _VP, _VP, _VP, _VP,
                                       ctypes.POINTER(ctypes.c_uint32)]
        lib.orc_decompress.restype = ctypes.c_int
        lib.orc_decompress_range.argtypes = [ctypes.POINTER(_Info), _VP, _VP, _VP, _VP, _VP,
                                             ctypes.c_uint64, ctypes.c_uint64, _VP,
                                             ctypes.POINTER(ctypes.c_uint32)]
        lib.orc_decompress_range.restype = ctypes.c_int
        self.lib = lib

    # -- individual steps ----------------------------------------------------
    def set_threads(self, n: int) -> int:
        """Threads of the per-element loops; returns the count in effect.
        Results are identical for every count (tests/test_oracle_threads.py)."""
        return int(self.lib.orc_set_threads(int(n)))

    def ratio(self, prev: np.ndarray, curr: np.ndarray, E: float):
        prev, curr, dt = _pair(prev, curr)
        n = prev.size
        d = np.empty(max(n, 1), np.float64)
        v = np.empty(max(n, 1), np.uint8)
        self.lib.orc_ratio(_p(prev), _p(curr), n, dt, E, _p(d), _p(v))
        return d[:n], v[:n].astype(bool)

    def range(self, d: np.ndarray, valid: np.ndarray):
        d = np.ascontiguousarray(d, np.float64)
        v = np.ascontiguousarray(valid, np.uint8)
        lo, hi = ctypes.c_double(0), ctypes.c_double(0)
        nv = self.lib.orc_range(_p(d), _p(v), d.size, ctypes.byref(lo), ctypes.byref(hi))
        return int(nv), lo.value, hi.value

    def bin_ids(self, d: np.ndarray, valid: np.ndarray, lo: float, E: float):
        d = np.ascontiguousarray(d, np.float64)
        v = np.ascontiguousarray(valid, np.uint8)
        m = np.empty(max(d.size, 1), np.int64)
        self.lib.orc_bin_ids(_p(d), _p(v), d.size, lo, E, _p(m))
        return m[:d.size]

    def histogram(self, m: np.ndarray, valid: np.ndarray):
        m = np.ascontiguousarray(m, np.int64)
        v = np.ascontiguousarray(valid, np.uint8)
        n = m.size
        ids = np.empty(max(n, 1), np.int64)
        cnt = np.empty(max(n, 1), np.uint32)
        nb = self.lib.orc_histogram(_p(m), _p(v), n, _p(ids), _p(cnt))
        return ids[:nb].copy(), cnt[:nb].copy()

    def topk(self, ids: np.ndarray, counts: np.ndarray, k: int):
        ids = np.ascontiguousarray(ids, np.int64)
        counts = np.ascontiguousarray(counts, np.uint32)
        sel = np.empty(max(k, 1), np.int64)
        tau = ctypes.c_uint32(0)
        t = self.lib.orc_topk(_p(ids), _p(counts), ids.size, k, _p(sel), ctypes.byref(tau))
        return sel[:t].copy(), int(tau.value)

    # -- whole path ----------------------------------------------------------
    def compress(self, prev: np.ndarray, curr: np.ndarray, E: float, B: int,
                 block_bytes: int = 0, recon: bool = True,
                 binning: str = "topk") -> "OracleResult":
        """The whole compression; binning "topk" (Sec. IV-B-1), "zero_anchored"
        (top-k over bins centred on multiples of 2E) or "equal_width" (Sec.
        IV-B-3)."""
        prev, curr, dt = _pair(prev, curr)
        n = prev.size
        T = prev.dtype
        packed = np.zeros(max((n * B + 31) // 32, 1), np.uint32)
        centers = np.zeros(1 << B, T)
        incomp = np.empty(max(n, 1), T)
        bb = block_bytes or (1 << 20)
        epb = (8 * bb) // B
        nblk = (n + epb - 1) // epb
        # room for any block length >= bytes/16 (the smallest B-bit block), so a
        # miscomputed block length cannot write past the table
        blk = np.zeros(max(nblk, (16 * n) // bb + 2), np.int64)
        rec = np.empty(max(n, 1), T) if recon else None
        index = np.empty(max(n, 1), np.uint16)
        sel = np.zeros(max((1 << B) - 1, 1), np.int64)
        info = _Info()
        if binning == "topk":
            st = self.lib.orc_compress(_p(prev), _p(curr), n, dt, E, B, block_bytes, _p(packed),
                                       _p(centers), _p(incomp), _p(blk),
                                       _p(rec) if rec is not None else None, _p(index), _p(sel),
                                       ctypes.byref(info))
        elif binning == "zero_anchored":
            st = self.lib.orc_compress_za(_p(prev), _p(curr), n, dt, E, B, block_bytes,
                                          _p(packed), _p(centers), _p(incomp), _p(blk),
                                          _p(rec) if rec is not None else None, _p(index),
                                          _p(sel), ctypes.byref(info))
        elif binning == "equal_width":
            st = self.lib.orc_compress_ew(_p(prev), _p(curr), n, dt, E, B, block_bytes,
                                          _p(packed), _p(centers), _p(incomp), _p(blk),
                                          _p(rec) if rec is not None else None, _p(index),
                                          ctypes.byref(info))
        else:
            raise ValueError(f"unknown binning {binning}")
        if st != 0:
            raise ValueError(f"oracle compress failed with status {st}")
        h = info.as_dict()
        return OracleResult(
            info=h, _info=info,
            packed=packed[: h["packed_words"]].copy(), centers=centers,
            incomp=incomp[: h["n_inc"]].copy(), block_inc_off=blk[: h["n_blocks"]].copy(),
            recon=None if rec is None else rec[:n].copy(), index=index[:n].copy(),
            sel_ids=(sel[: h["k_used"]].copy() if binning != "equal_width"
                     else np.zeros(0, np.int64)),
        )

    def choose_B(self, prev: np.ndarray, curr: np.ndarray, E: float, b_lo: int = 1,
                 b_hi: int = 16):
        """(B, bits): the B of eqs. (5)-(6) and the estimated size in bits of
        every B (index B; 0 outside [b_lo, b_hi])."""
        prev, curr, dt = _pair(prev, curr)
        bits = np.zeros(17, np.uint64)
        B = ctypes.c_uint32(0)
        st = self.lib.orc_choose_B(_p(prev), _p(curr), prev.size, dt, E, b_lo, b_hi, _p(bits),
                                   ctypes.byref(B))
        if st != 0:
            raise ValueError(f"oracle choose_B failed with status {st}")
        return int(B.value), [int(x) for x in bits]

    def lossless_encode(self, packed: np.ndarray, n: int, B: int) -> dict:
        """Lossless stage of an index table of n B-bit codes: code_of_rank,
        k, bits_k (total bits of every order k in [0, B]), sub_off (bits) and
        the stream words."""
        packed = _nonempty(np.ascontiguousarray(packed, np.uint32), np.uint32)
        nsub = int(self.lib.orc_lossless_subblocks(n))
        cor = np.zeros(1 << B, np.uint16)
        bits_k = np.zeros(B + 1, np.uint64)
        sub_off = np.zeros(nsub + 1, np.uint64)
        k = ctypes.c_uint32(0)
        words = ctypes.c_uint64(0)
        cap = n * 33 // 32 + 5 * nsub + 2  # codewords, a group table and a padding word each
        stream = np.zeros(max(cap, 1), np.uint32)
        st = self.lib.orc_lossless_encode(_p(packed), n, B, _p(cor), ctypes.byref(k), _p(bits_k),
                                          _p(sub_off), _p(stream), stream.size, ctypes.byref(words))
        if st != 0:
            raise ValueError(f"oracle lossless_encode failed with status {st}")
        return {"code_of_rank": cor, "k": int(k.value), "bits_k": [int(x) for x in bits_k],
                "sub_off": sub_off, "stream": stream[: words.value].copy(), "n": n, "B": B}

    def lossless_decode(self, enc: dict) -> np.ndarray:
        """The index table (packed words) of a lossless_encode result."""
        n, B = enc["n"], enc["B"]
        packed = np.zeros(max((n * B + 31) // 32, 1), np.uint32)
        stream = _nonempty(enc["stream"], np.uint32)
        st = self.lib.orc_lossless_decode(_p(np.ascontiguousarray(enc["code_of_rank"], np.uint16)),
                                          enc["k"], _p(np.ascontiguousarray(enc["sub_off"],
                                                                            np.uint64)),
                                          _p(stream), n, B, _p(packed))
        if st != 0:
            raise ValueError(f"oracle lossless_decode failed with status {st}")
        return packed[: (n * B + 31) // 32]

    def decompress(self, res: "OracleResult", prev: np.ndarray):
        prev = np.ascontiguousarray(prev)
        n = res.info["n"]
        out = np.empty(max(n, 1), prev.dtype)
        flags = ctypes.c_uint32(0)
        packed = _nonempty(res.packed, np.uint32)
        incomp = _nonempty(res.incomp, prev.dtype)
        st = self.lib.orc_decompress(ctypes.byref(res._info), _p(prev), _p(packed),
                                     _p(res.centers), _p(incomp), _p(out), ctypes.byref(flags))
        if st != 0:
            raise ValueError(f"oracle decompress failed with status {st}")
        return out[:n], int(flags.value)

    def decompress_range(self, res: "OracleResult", prev: np.ndarray, start: int, length: int):
        prev = np.ascontiguousarray(prev)
        out = np.empty(max(length, 1), prev.dtype)
        flags = ctypes.c_uint32(0)
        packed = _nonempty(res.packed, np.uint32)
        incomp = _nonempty(res.incomp, prev.dtype)
        blk = _nonempty(res.block_inc_off, np.int64)
        st = self.lib.orc_decompress_range(ctypes.byref(res._info), _p(prev), _p(packed),
                                           _p(res.centers), _p(incomp), _p(blk), start, length,
                                           _p(out), ctypes.byref(flags))
        if st != 0:
            raise ValueError(f"oracle decompress_range failed with status {st}")
        return out[:length], int(flags.value)


@dataclass
class OracleResult:
    info: dict
    _info: _Info
    packed: np.ndarray
    centers: np.ndarray
    incomp: np.ndarray
    block_inc_off: np.ndarray
    recon: np.ndarray | None
    index: np.ndarray
    sel_ids: np.ndarray


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _nonempty(a, dtype):
    a = np.ascontiguousarray(a, dtype)
    return a if a.size else np.zeros(1, dtype)


def _pair(prev, curr):
    prev = np.ascontiguousarray(prev).reshape(-1)
    curr = np.ascontiguousarray(curr).reshape(-1)
    if prev.dtype != curr.dtype or prev.size != curr.size:
        raise ValueError("prev and curr must have the same dtype and size")
    if prev.dtype == np.float32:
        dt = F32
    elif prev.dtype == np.float64:
        dt = F64
    else:
        raise ValueError(f"unsupported dtype {prev.dtype}")
    if prev.size == 0:
        prev = np.zeros(1, prev.dtype)[:0]
    return prev, curr, dt


_default: Oracle | None = None


def get() -> Oracle:
    """The oracle compiled from this directory's source (built on first use)."""
    global _default
    if _default is None:
        _default = Oracle()
    return _default
