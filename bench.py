"""Benchmark of the NUMARCK compression hot path on one MI355X.

Workload: FLASH-like 3-D turbulence variable, 512^3 float64 (1 GiB per
snapshot), 10 consecutive snapshots (9 pairs), E = 1e-3, B = 8, one plain
compression per pair (a "step" compresses one pair: range pass, histogram,
top-k selection, encode/pack/compaction).  Inputs are synthetic and already
resident in HBM when the timed region starts.

Prints one JSON line: whole-job input throughput (GB/s of the compressed
snapshot, n * 8 bytes), per-step latency p50/p99, the roofline of the
dominant kernel (algorithmic bytes per launch / its average duration from HIP
events on the compression stream) and the CPU oracle timed on a bounded
sample of the same workload.
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E peak
EDGE, E, B, SNAPSHOTS = 512, 1e-3, 8, 10

# Algorithmic bytes per element of each kernel (float64, B index bits,
# incompressible fraction alpha): what the kernel must move at minimum.
#   range, hist : read prev + curr                      = 16
#   encode      : write B/8 + alpha*8 (the index table and the incompressible
#                 values); the method's index + verify step also reads both
#                 snapshots, which the precoded encoding does in the histogram
#                 pass, so here the encoder's own share is counted
# The precoded encoding's window codes (2 bytes per element written by the
# histogram pass and read by the encoder) and the staging of the
# incompressible points (their indices written by the encoder, read by the
# placement kernel, which then reads the values) are overhead of this
# design, measured by the counters and reported beside these figures.
ALGO = {
    "range": lambda a: 16.0,
    "hist": lambda a: 16.0,
    "encode": lambda a: B / 8 + 8 * a,
}
# The whole compression's minimum: read both snapshots once, write the index
# table and the incompressible values.
ALGO_CALL = lambda a: 16.0 + B / 8 + 8 * a

# Kernels of one compression call (the library's k_* names; the precoded
# encoder k_encode_pre counts as the encode pass).
PIPELINE_KERNELS = ("init", "range", "hist", "hclear", "hinsert", "select",
                    "tailrank", "encode", "gather")


def pass_name(kernel: str) -> str:
    """Pass of a library kernel name (the part after nk::k_)."""
    return "encode" if kernel == "encode_pre" else kernel


# The sources the compression and decompression kernels are built from: the
# committed counters are taken as stale when any of them changes.
KERNEL_SOURCES = ("compress_kernels.hip", "decompress_kernels.hip", "nk_device.h", "nk_internal.h")


def source_digest() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1703_02438_amd", "csrc")
    for f in KERNEL_SOURCES:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def load_pmc(kernel: str, workload: str):
    """The committed rocprofv3 counter summary of `kernel` (or "pipeline"),
    if it was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", f"pmc_{kernel}_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_digest") != source_digest():
        return None
    return rec


def load_traffic(kernel: str, workload: str):
    """HBM traffic of `kernel` measured with rocprofv3 counters, if the
    committed measurement matches the current kernel sources."""
    rec = load_pmc(kernel, workload)
    return rec.get("bytes_per_launch") if rec else None


COPY_CALIB_BYTES = 1 << 30


def calib_copy(torch, nk, dev):
    """The library's reference copy of 1 GiB (numarck_stream_kernel, cached
    loads and stores): a kernel of known traffic for scaling the FETCH_SIZE /
    WRITE_SIZE counters."""
    src = torch.empty(COPY_CALIB_BYTES // 8, dtype=torch.float64, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(3):
        nk.stream_kernel(nk.STREAM_COPY, src, dst, COPY_CALIB_BYTES)
    torch.cuda.synchronize()
    del src, dst


def summarize_pmc(fetch_dir: str, write_dir: str, workload: str, cmd: str):
    """Turn two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) of
    `bench.py --calib-copy` into HBM bytes per launch of every library kernel,
    scaled by what the counters read for the 1 GiB calibration copy; writes
    profiles/pmc_{range,hist,encode,decode}_* (the streaming kernels) and
    pmc_pipeline_* (every kernel of one compression call)."""
    import csv
    import glob
    import re

    def per_kernel(d, counter):
        vals = {}
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            with open(f) as fh:
                for row in csv.DictReader(fh):
                    if row.get("Counter_Name") != counter:
                        continue
                    name = row["Kernel_Name"]
                    m = re.search(r"nk::k_(\w+)", name)
                    if m:
                        k = pass_name(m.group(1))
                        if k.startswith("stream_") and "<true>" in name:
                            k += "_nt"
                        vals.setdefault(k, []).append(float(row["Counter_Value"]))
        return vals

    rec = {}
    for d, counter in ((fetch_dir, "FETCH_SIZE"), (write_dir, "WRITE_SIZE")):
        v = per_kernel(d, counter)
        copy = [x for x in v.get("stream_copy", []) if x * 1024 > 0.25 * COPY_CALIB_BYTES]
        if not copy:
            raise SystemExit(f"no {counter} samples of the calibration copy")
        copy_kib = sorted(copy)[len(copy) // 2]
        scale = (COPY_CALIB_BYTES / 1024) / copy_kib
        for k, xs in v.items():
            # full-size launches only (range decompressions launch the decoder on 1 %)
            xs = [x for x in xs if x >= 0.5 * max(xs)] if k in ("decode", "dcount") else xs
            rec.setdefault(k, {})[counter] = {"kernel_kib": sum(xs) / len(xs),
                                              "copy_kib": copy_kib, "scale": scale,
                                              "dispatches": len(xs)}
    base = {"workload": workload, "command": cmd, "source_digest": source_digest(),
            "copy_bytes": COPY_CALIB_BYTES, "copy_kernel": "nk::k_stream_copy<false>"}

    def bytes_of(k):
        r = rec[k]
        return sum(r[c]["kernel_kib"] * r[c]["scale"] * 1024 for c in ("FETCH_SIZE", "WRITE_SIZE"))

    for kernel in ("range", "hist", "encode", "decode"):
        if kernel not in rec:
            raise SystemExit(f"no samples of k_{kernel}")
        out = dict(base, kernel=kernel, **rec[kernel])
        out["bytes_per_launch"] = int(bytes_of(kernel))
        path = os.path.join(ROOT, "profiles", f"pmc_{kernel}_{workload}.json")
        with open(path, "w") as f:
            json.dump(out, f, indent=1)
        print(path)
    per = {}
    for k in PIPELINE_KERNELS:
        if k not in rec:
            if k == "tailrank":  # not launched when k_select ranks the tail bins
                continue
            raise SystemExit(f"no samples of k_{k}")
        r = rec[k]
        per[k] = {"fetch_bytes": int(r["FETCH_SIZE"]["kernel_kib"] * r["FETCH_SIZE"]["scale"] * 1024),
                  "write_bytes": int(r["WRITE_SIZE"]["kernel_kib"] * r["WRITE_SIZE"]["scale"] * 1024),
                  "dispatches": r["FETCH_SIZE"]["dispatches"]}
    out = dict(base, kernel="pipeline", kernels=per,
               bytes_per_call=sum(v["fetch_bytes"] + v["write_bytes"] for v in per.values()))
    path = os.path.join(ROOT, "profiles", f"pmc_pipeline_{workload}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path)


SQ_COUNTERS = ("SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_INSTS_VMEM_RD",
               "SQ_INSTS_VMEM_WR")


def summarize_sq(sq_dir: str, workload: str, n: int, cmd: str):
    """Instruction counts per element of the compression and decompression
    kernels from one rocprofv3 --pmc run of SQ counters: wave instructions
    times 64 lanes over the n elements of the call (decoder: full-size
    launches only); writes profiles/sq_counters_<workload>.md."""
    import csv
    import glob
    import re

    vals = {}
    for f in glob.glob(os.path.join(sq_dir, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            for row in csv.DictReader(fh):
                m = re.search(r"nk::k_(\w+)", row["Kernel_Name"])
                if not m or row.get("Counter_Name") not in SQ_COUNTERS:
                    continue
                key = (pass_name(m.group(1)), int(row.get("Dispatch_Id", 0) or 0))
                vals.setdefault(key, {})[row["Counter_Name"]] = float(row["Counter_Value"])
    per = {}
    for (k, _), c in vals.items():
        per.setdefault(k, []).append(c)
    lines = [f"# SQ instruction counters, {workload} (n = {n})", "",
             "Command (from the repository root, on one MI355X):", "", "```", cmd, "```", "",
             "Wave-level instruction counts times 64 lanes, per element of the call "
             "(averaged over the dispatches; the decoder's full-size launches only).", "",
             "| kernel | dispatches | waves | VALU / elem | SALU / elem | LDS / elem "
             "| VMEM rd / elem | VMEM wr / elem |",
             "|---|---:|---:|---:|---:|---:|---:|---:|"]
    order = list(PIPELINE_KERNELS) + ["dcount", "decode"]
    for k in order:
        xs = per.get(k, [])
        if k in ("decode", "dcount") and xs:
            top = max(x.get("SQ_WAVES", 0.0) for x in xs)
            xs = [x for x in xs if x.get("SQ_WAVES", 0.0) >= 0.5 * top]
        if not xs:
            continue
        avg = {c: sum(x.get(c, 0.0) for x in xs) / len(xs) for c in SQ_COUNTERS}
        pe = {c: avg[c] * 64 / n for c in SQ_COUNTERS[1:]}
        lines.append(f"| `k_{k}` | {len(xs)} | {avg['SQ_WAVES']:.0f} | {pe['SQ_INSTS_VALU']:.2f} "
                     f"| {pe['SQ_INSTS_SALU']:.2f} | {pe['SQ_INSTS_LDS']:.2f} "
                     f"| {pe['SQ_INSTS_VMEM_RD']:.3f} | {pe['SQ_INSTS_VMEM_WR']:.3f} |")
    path = os.path.join(ROOT, "profiles", f"sq_counters_{workload}.md")
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(path)


def summarize_trace(trace_csv: str, out_md: str, title: str, cmd: str):
    """A rocprofv3 --kernel-trace CSV to a markdown table of the library's
    kernels, one row per kernel and grid size (a range decompression and a
    full one launch the same decoder with different grids), and the sum of
    the compression call's kernels."""
    import csv

    rows = {}
    for r in csv.DictReader(open(trace_csv)):
        name = r["Kernel_Name"]
        if "nk::k_" not in name:
            continue
        name = name.replace("void ", "", 1)
        grid = int(r.get("Grid_Size_X") or r.get("Grid_Size") or 0)
        wg = int(r.get("Workgroup_Size_X") or r.get("Workgroup_Size") or 1)
        d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        rows.setdefault(name, []).append((grid // max(wg, 1), d))
    # a kernel launched with several grids: the largest grid (the whole
    # array) and the smaller ones (partial decompressions) are kept apart
    split = {}
    for name, xs in rows.items():
        gmax = max(g for g, _ in xs)
        one = len({g for g, _ in xs}) == 1
        for g, d in xs:
            key = (name, "one size" if one else "largest" if g == gmax else "smaller")
            split.setdefault(key, []).append(d)
    rows = split
    lines = [f"# {title}", "", "Command (from the repository root, on one MI355X):", "", "```",
             cmd, "```", "",
             "Per-dispatch kernel trace (rocprofv3 `--kernel-trace`), library kernels only.  A",
             "kernel launched with several grids has a row for its largest grid (the whole array)",
             "and one for the smaller grids (range decompressions).", "",
             "| kernel | grid | calls | avg us | min us | max us |",
             "|---|---|---:|---:|---:|---:|"]
    call = 0.0
    for (name, wgs), ds in sorted(rows.items(), key=lambda kv: -sum(kv[1])):
        avg = sum(ds) / len(ds)
        lines.append(f"| `{name}` | {wgs} | {len(ds)} | {avg:.1f} | {min(ds):.1f} | {max(ds):.1f} |")
    comp = {}
    for (name, wgs), ds in rows.items():
        for k in PIPELINE_KERNELS:
            if any(f"nk::k_{x}{c}" in name for x in ((k, "encode_pre") if k == "encode" else (k,))
                   for c in "<("):
                comp.setdefault(k, []).extend(ds)
    if comp:
        lines += ["", "Compression call (average of each kernel, summed):", ""]
        for k in PIPELINE_KERNELS:
            if k in comp:
                a = sum(comp[k]) / len(comp[k])
                call += a
                lines.append(f"- `k_{k}`: {a:.1f} us")
        lines.append(f"- sum: {call:.1f} us")
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(out_md)


STREAM_KINDS = ("read", "read_nt", "write", "write_nt", "copy", "copy_nt", "read2_write16",
                "read2_write8")


def stream_section(torch, nk, reps: int, nbytes: int = 1 << 30) -> dict:
    """The library's reference streaming kernels (numarck_stream_kernel) on
    1 GiB: read, write and copy, cached and non-temporal, and two read and
    write mixes (two arrays read, 1/16 of that written: an encoder reading
    both snapshots; 1/8: the histogram pass writing window codes), at 2..16
    workgroups per compute unit; GB/s of bytes moved (a copy moves 2 x
    nbytes), the best launch of each."""
    src = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream()
    out = {}
    for kind, name in enumerate(STREAM_KINDS):
        moved = (2 * nbytes if name.startswith("copy") else
                 nbytes + nbytes // 16 if name == "read2_write16" else
                 nbytes + nbytes // 8 if name == "read2_write8" else nbytes)
        best = None
        for per_cu in (2, 4, 8, 16):
            t = time_ms(torch, lambda: nk.stream_kernel(kind, src, dst, nbytes, per_cu, stream),
                        reps, stream)
            gbs = moved / t / 1e6
            if best is None or gbs > best[0]:
                best = (gbs, per_cu)
        out[name] = {"gbs": round(best[0], 1), "per_cu": best[1]}
    del src, dst
    torch.cuda.empty_cache()
    return out


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# Host threads of the CPU baseline: the host's share for one GPU.
CPU_THREADS_MAX = 16


def cpu_baseline(prev, curr, sample_elems: int, n_total: int):
    """The C oracle on the host cores: the whole compression of pair 0 (or
    its first `sample_elems` values), once with the per-element loops on all
    threads of the host's share and once on one thread (identical results;
    the histogram sort, selection, packing and placement are serial)."""
    import oracle

    p = prev[:sample_elems].cpu().numpy()
    q = curr[:sample_elems].cpu().numpy()
    o = oracle.get()
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    threads = o.set_threads(min(avail, CPU_THREADS_MAX))
    t = time.perf_counter()
    o.compress(p, q, E, B, recon=False)
    dt_mt = time.perf_counter() - t
    o.set_threads(1)
    t = time.perf_counter()
    o.compress(p, q, E, B, recon=False)
    dt_1 = time.perf_counter() - t
    what = "all of pair 0" if p.size == n_total else f"first {p.size} elements of pair 0"
    return {
        "value": round(p.size * 8 / dt_mt / 1e9, 4),
        "unit": "GB/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"{what} ({p.size * 8 / 2**20:.0f} MiB), C oracle, per-element loops on "
                  f"{threads} threads: {dt_mt:.2f} s",
        "cpu_model": cpu_model(),
        "host_cpus": avail,
        "single_thread": {"value": round(p.size * 8 / dt_1 / 1e9, 4), "seconds": round(dt_1, 2)},
    }


def decompress_section(torch, nk, c, prev, reps: int, stream, workload: str) -> dict:
    """Full decompression of one 512^3 float64 record and range decompressions
    of 1 % of it at seeded offsets: output GB/s, and the decode kernel against
    its algorithmic bytes (read prev 8 + index B/8 + incompressible 8 alpha,
    write 8 per element)."""
    import random

    h = c.header()
    n = h.n
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    flags = torch.zeros(1, dtype=torch.int32, device="cuda")
    dws = torch.empty(nk.numarck_decompress_workspace_bytes(n), dtype=torch.uint8, device="cuda")
    st = stream.cuda_stream

    def full():
        nk._check(nk.numarck_decompress(ctypes.byref(h), prev.data_ptr(), c.packed.data_ptr(),
                                        c.centers.data_ptr(), c.incomp.data_ptr(),
                                        c.block_inc_off.data_ptr(), out.data_ptr(),
                                        flags.data_ptr(), dws.data_ptr(), dws.numel(), st),
                  "numarck_decompress")

    t_full = time_ms(torch, full, reps, stream)
    nk.timing_enable(True)
    for _ in range(reps):
        full()
    torch.cuda.synchronize()
    tk = nk.timing_read()
    nk.timing_enable(False)
    dl, dms = tk["decode"]
    ln = n // 100
    rnd = random.Random(1711)
    starts = [rnd.randrange(0, n - ln) for _ in range(max(reps, 2))]
    it = iter(starts * 2)

    def part():
        s0 = next(it)
        nk._check(nk.numarck_decompress_range(ctypes.byref(h), prev.data_ptr(), c.packed.data_ptr(),
                                              c.centers.data_ptr(), c.incomp.data_ptr(),
                                              c.block_inc_off.data_ptr(), s0, ln, out.data_ptr(),
                                              flags.data_ptr(), dws.data_ptr(), dws.numel(), st),
                  "numarck_decompress_range")

    t_part = time_ms(torch, part, max(reps - 1, 1), stream)
    assert int(flags.item()) == 0
    alpha = h.n_inc / n
    algo = (8 + 8 + h.B / 8 + 8 * alpha) * n
    dec_s = dms / dl / 1e3
    return {
        "full_gbs": round(n * 8 / t_full / 1e6, 1),
        "full_ms": round(t_full, 4),
        "range_1pct_ms": round(t_part, 4),
        "range_1pct_gbs": round(ln * 8 / t_part / 1e6, 1),
        "decode_kernel": {"achieved": round(algo / dec_s / 1e9, 1), "peak": HBM_PEAK_GBS,
                          "unit": "GB/s", "frac": round(algo / dec_s / 1e9 / HBM_PEAK_GBS, 4),
                          "traffic": load_traffic("decode", workload),
                          "algorithmic_bytes_per_launch": int(algo),
                          "avg_launch_us": round(dec_s * 1e6, 2)},
    }


def auto_b_section(torch, nk, prev, curr, outs_max, ws, reps: int, stream) -> dict:
    """Compression with B chosen in [1, 16] from the histogram (eqs. 5-6) on
    the benchmark pair: the choice, every B's estimated size against the
    compression's actual size, and the time of the automatic call (which
    waits once on the stream for the choice) against a plain call with the
    chosen B."""
    n = prev.numel()
    c, B, est = nk.compress_auto(prev, curr, E, 1, 16, ws=ws, outputs=outs_max, stream=stream)
    h = c.header()
    t_auto = time_ms(torch, lambda: nk.compress_auto(prev, curr, E, 1, 16, ws=ws,
                                                      outputs=outs_max, stream=stream), reps, stream)
    outs = nk.alloc_outputs(n, torch.float64, B)
    t_plain = time_ms(torch, lambda: nk.compress(prev, curr, E, B, ws=ws, outputs=outs,
                                                 stream=stream), reps, stream)
    return {
        "B": B,
        "est_bytes": {b: est[b] // 8 for b in range(1, 17)},
        "actual_compressed_bytes": int(h.compressed_bytes),
        "est_n_inc": (est[B] - 8 * (1 << B) * 8 - n * B) // 64,
        "actual_n_inc": int(h.n_inc),
        "auto_ms": round(t_auto, 4),
        "plain_ms_same_B": round(t_plain, 4),
        "auto_gbs": round(n * 8 / t_auto / 1e6, 1),
    }


def variant_section(torch, nk, fn, prev, curr, topk_hdr, ws, reps: int, stream) -> dict:
    """Another binning on the benchmark pair with the same E and B (equal-width
    binning, Sec. III-B, IV-B-3, or the zero-anchored top-k bins): the time
    and input rate of the call, its kernels, and its incompressible count and
    size against the paper's top-k."""
    n = prev.numel()
    outs = nk.alloc_outputs(n, torch.float64, B)
    run = lambda: fn(prev, curr, E, B, ws=ws, outputs=outs, stream=stream)
    c = run()
    torch.cuda.synchronize()
    h = c.header()
    t = time_ms(torch, run, reps, stream)
    nk.timing_enable(True)
    for _ in range(reps):
        run()
    torch.cuda.synchronize()
    tk = nk.timing_read()
    nk.timing_enable(False)
    return {
        "ms": round(t, 4),
        "gbs": round(n * 8 / t / 1e6, 1),
        "kernels_us": {k: round(v[1] / v[0] * 1e3, 1) for k, v in tk.items()},
        "n_inc": int(h.n_inc),
        "compressed_bytes": int(h.compressed_bytes),
        "topk_n_inc": int(topk_hdr.n_inc),
        "topk_compressed_bytes": int(topk_hdr.compressed_bytes),
        "size_vs_topk": round(h.compressed_bytes / topk_hdr.compressed_bytes, 3),
    }


def lossless_section(torch, nk, c, n: int, reps: int, stream) -> dict:
    """The lossless stage on the benchmark pair's index table: encode and
    decode times, and the stored size against the packed table's."""
    ws = torch.empty(nk.numarck_lossless_workspace_bytes(B), dtype=torch.uint8, device="cuda")
    e = nk.lossless_encode(c.packed, n, B, ws=ws, stream=stream)
    h = e.header()
    t_enc = time_ms(torch, lambda: nk.lossless_encode(c.packed, n, B, ws=ws, stream=stream),
                    reps, stream)
    out = torch.empty_like(c.packed)
    t_dec = time_ms(torch, lambda: nk.lossless_decode(e, out=out, stream=stream), reps, stream)
    _, fl = nk.lossless_decode(e, out=out, stream=stream)
    words = (n * B + 31) // 32
    assert int(fl.item()) == 0 and torch.equal(out[:words], c.packed[:words])
    hdr = c.header()
    packed_bytes = int(hdr.packed_bytes)
    file_plain = int(hdr.compressed_bytes)
    file_ll = file_plain - packed_bytes + int(h.bytes)
    return {
        "order_k": int(h.k),
        "bits_per_code": round(h.bits / n, 3),
        "index_bytes": packed_bytes,
        "lossless_bytes": int(h.bytes),
        "index_ratio": round(packed_bytes / h.bytes, 3),
        "file_cr_without": round(n * 8 / file_plain, 3),
        "file_cr_with": round(n * 8 / file_ll, 3),
        "encode_ms": round(t_enc, 4),
        "decode_ms": round(t_dec, 4),
    }


def time_ms(torch, fn, reps: int, stream) -> float:
    """Average ms of fn() over reps runs, HIP events on `stream` (after one warm run)."""
    fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        fn()
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def batched_vs_plain(torch, nk, jobs, reps: int) -> dict:
    """One workload of many jobs: plain per-job launches (directly, and
    captured in one HIP graph and replayed), one batched plan, the plan
    replayed as a HIP graph, and the batch with zero-anchored bins (input
    GB/s of each)."""
    stream = torch.cuda.current_stream()
    in_bytes = sum(j.curr.numel() * j.curr.element_size() for j in jobs)
    wss = [torch.empty(nk.numarck_workspace_bytes(j.curr.numel(), nk.dtype_code(j.curr.dtype), j.B),
                       dtype=torch.uint8, device="cuda") for j in jobs]
    outs = [nk.alloc_outputs(j.curr.numel(), j.curr.dtype, j.B, j.block_bytes) for j in jobs]

    def plain():
        for j, w, o in zip(jobs, wss, outs):
            nk.compress(j.prev, j.curr, j.E, j.B, j.block_bytes, ws=w, outputs=o, stream=stream)

    t_plain = time_ms(torch, plain, reps, stream)
    ref = [(h.n_inc, h.compressed_bytes) for h in
           (nk.header_from_device(o["hdr"]) for o in outs)]
    # the same plain calls captured in one HIP graph and replayed (every
    # launch recorded, no launch latency between them); the headers of the
    # last replay must equal the direct calls'
    t_plain_graph = None
    g = torch.cuda.CUDAGraph()
    gst = torch.cuda.Stream()
    gst.wait_stream(stream)
    with torch.cuda.graph(g, stream=gst):
        for j, w, o in zip(jobs, wss, outs):
            nk.compress(j.prev, j.curr, j.E, j.B, j.block_bytes, ws=w, outputs=o, stream=gst)
    stream.wait_stream(gst)
    t_plain_graph = time_ms(torch, g.replay, reps, stream)
    torch.cuda.synchronize()
    got = [(h.n_inc, h.compressed_bytes) for h in (nk.header_from_device(o["hdr"]) for o in outs)]
    assert got == ref, "graph-replayed plain calls differ from the direct calls"
    del g, wss
    plan = nk.Plan(jobs, outputs=outs, stream=stream)
    t_plan = time_ms(torch, lambda: plan.run(stream), reps, stream)
    gs = torch.cuda.Stream()
    gs.wait_stream(stream)
    with torch.cuda.stream(gs):
        plan.capture(gs)
        t_graph = time_ms(torch, lambda: plan.replay(gs), reps, gs)
    stream.wait_stream(gs)
    flags = [plan.results()[i].header().flags for i in range(len(jobs))]
    assert not any(flags), flags
    plan.close()
    # the same batch with the bins anchored at -E (no range pass)
    zplan = nk.Plan(jobs, outputs=outs, stream=stream, zero_anchored=True)
    t_za = time_ms(torch, lambda: zplan.run(stream), reps, stream)
    zplan.close()
    return {
        "za_batched_gbs": round(in_bytes / t_za / 1e6, 1),
        "za_batched_ms": round(t_za, 3),
        "jobs": len(jobs),
        "input_bytes": in_bytes,
        "plain_gbs": round(in_bytes / t_plain / 1e6, 1),
        "plain_graph_gbs": round(in_bytes / t_plain_graph / 1e6, 1),
        "batched_gbs": round(in_bytes / t_plan / 1e6, 1),
        "graph_gbs": round(in_bytes / t_graph / 1e6, 1),
        "plain_ms": round(t_plain, 3),
        "batched_ms": round(t_plan, 3),
        "graph_ms": round(t_graph, 3),
        "speedup": round(t_plain / t_plan, 2),
    }


CLIMATE_SNAPSHOTS, CLIMATE_PER_LAUNCH = 192, 16


def climate_series_section(torch, nk, inputs, reps: int, spill: bool) -> dict:
    """The climate-like time series at full length: 192 snapshots of 3600 x
    1800 float32 (E = 1e-4, B = 10), its 191 consecutive pairs compressed as
    191 plain calls, and as 12 batched launches of at most 16 pairs (time
    chains: each plan reads a shared snapshot once per range pass); also
    with zero-anchored bins, with the histogram's window counts forced to
    global memory, and with the batch autotuner's choice.  `spill`: outliers
    U[-0.9, 1.5] on 1 % of the cells (about 12,000 fine bins, ties at the
    k-th count) instead of U[-0.05, 0.05]."""
    kw = {"outlier_lo": -0.9, "outlier_hi": 1.5} if spill else {}
    s = inputs.ClimateSeries(nlat=1800, nlon=3600, seed=1707, device="cuda", **kw)
    snaps = [s.x.clone()] + [s.step().clone() for _ in range(CLIMATE_SNAPSHOTS - 1)]
    del s
    E_c, B_c = 1e-4, 10
    jobs = [nk.BatchJob(snaps[t], snaps[t + 1], E_c, B_c) for t in range(CLIMATE_SNAPSHOTS - 1)]
    n = snaps[0].numel()
    in_bytes = len(jobs) * n * 4
    stream = torch.cuda.current_stream()
    outs = [nk.alloc_outputs(n, torch.float32, B_c) for _ in jobs]
    ws = torch.empty(nk.numarck_workspace_bytes(n, nk.F32, B_c), dtype=torch.uint8, device="cuda")

    def plain():
        for j, o in zip(jobs, outs):
            nk.compress(j.prev, j.curr, E_c, B_c, ws=ws, outputs=o, stream=stream)

    t_plain = time_ms(torch, plain, reps, stream)
    del ws
    groups = [list(range(i, min(i + CLIMATE_PER_LAUNCH, len(jobs))))
              for i in range(0, len(jobs), CLIMATE_PER_LAUNCH)]

    def plans(za=False, tune=None):
        return [nk.Plan([jobs[i] for i in g], outputs=[outs[i] for i in g], stream=stream,
                        zero_anchored=za, tune=tune) for g in groups]

    def run_all(ps):
        for p in ps:
            p.run(stream)

    res = {"pairs": len(jobs), "launches": len(groups), "input_bytes": in_bytes,
           "plain_ms": round(t_plain, 3), "plain_gbs": round(in_bytes / t_plain / 1e6, 1)}
    first = [jobs[i] for i in groups[0]]
    tuned = nk.plan_autotune(first, reps=2, outputs=[outs[i] for i in groups[0]], stream=stream)
    glob = nk.default_tuning()
    glob.hist_lds, glob.hist_blocks_per_cu = 0, 8
    for name, za, tune in (("batched", False, None), ("za_batched", True, None),
                           ("global_hist_batched", False, glob), ("tuned_batched", False, tuned)):
        ps = plans(za, tune)
        t = time_ms(torch, lambda: run_all(ps), reps, stream)
        for p in ps:
            p.close()
        res[f"{name}_ms"] = round(t, 3)
        res[f"{name}_gbs"] = round(in_bytes / t / 1e6, 1)
    h = nk.header_from_device(outs[0]["hdr"])
    assert h.flags == 0
    res["speedup"] = round(res["plain_ms"] / res["batched_ms"], 2)
    res["tuning"] = tuned.as_dict()
    res["pair0"] = {"M": int(h.M), "n_nonzero": int(h.n_nonzero), "alpha": round(h.n_inc / n, 5),
                    "tau": int(h.tau)}
    del snaps, jobs, outs
    torch.cuda.empty_cache()
    return res


def small_call_section(torch, nk, inputs, reps: int = 200) -> dict:
    """The 64^3 float64 mixture pair (E = 1e-3, B = 8; 4 MiB of input, which
    the caches hold): latency of one plain compression and of one full
    decompression, HIP events around each call."""
    n = 64 ** 3
    p, q = inputs.mixture_pair(n, seed=1704)
    p, q = p.cuda(), q.cuda()
    stream = torch.cuda.current_stream()
    ws = torch.empty(nk.numarck_workspace_bytes(n, nk.F64, 8), dtype=torch.uint8, device="cuda")
    outs = nk.alloc_outputs(n, torch.float64, 8)
    c = nk.compress(p, q, 1e-3, 8, ws=ws, outputs=outs, stream=stream)
    out = torch.empty(n, dtype=torch.float64, device="cuda")

    def per_call(fn):
        for _ in range(10):
            fn()
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(reps)]
        for a, b in evs:
            a.record(stream)
            fn()
            b.record(stream)
        torch.cuda.synchronize()
        return [a.elapsed_time(b) * 1e3 for a, b in evs]

    lc = per_call(lambda: nk.compress(p, q, 1e-3, 8, ws=ws, outputs=outs, stream=stream))
    ld = per_call(lambda: nk.decompress(c, p, out=out, stream=stream))
    import numpy as np

    q50 = lambda x: round(float(np.percentile(x, 50)), 1)
    q99 = lambda x: round(float(np.percentile(x, 99)), 1)
    return {"workload": "mixture 64^3 f64, E=1e-3, B=8", "n": n,
            "compress_us": {"p50": q50(lc), "p99": q99(lc)},
            "decompress_us": {"p50": q50(ld), "p99": q99(ld)},
            "compress_gbs_p50": round(n * 8 / q50(lc) / 1e3, 1)}


def batched_section(torch, nk, inputs, reps: int) -> dict:
    """The uneven 64-variable workload (cube edges log-uniform in [32, 384],
    60 % float64, E in {1e-4, 1e-3, 1e-2}, B in {8, 10, 12}), the 191
    consecutive pairs of a 3600 x 1800 float32 climate-like series (E = 1e-4,
    B = 10; and its outlier-heavy variant), and the 9 consecutive pairs of
    the 512^3 float64 FLASH-like series."""
    out = {}
    jobs = []
    for sp in inputs.batched_specs(64):
        p, q = inputs.mixture_pair(sp.n, seed=sp.seed, dtype=sp.dtype, device="cuda")
        jobs.append(nk.BatchJob(p, q, sp.E, sp.B))
    out["uneven_64vars"] = batched_vs_plain(torch, nk, jobs, reps)
    del jobs
    torch.cuda.empty_cache()
    out["climate_191pairs"] = climate_series_section(torch, nk, inputs, reps, spill=False)
    out["climate_191pairs_spill"] = climate_series_section(torch, nk, inputs, reps, spill=True)
    # the 9 consecutive pairs of the 512^3 float64 FLASH-like series as one
    # batch (a time chain: its range pass reads each snapshot once)
    s = inputs.FlashSeries(edge=512, seed=1705, device="cuda")
    snaps = [s.x.clone()] + [s.step().clone() for _ in range(SNAPSHOTS - 1)]
    del s
    out["flash3d_512cubed_9pairs"] = batched_vs_plain(
        torch, nk, [nk.BatchJob(snaps[t], snaps[t + 1], E, B) for t in range(SNAPSHOTS - 1)],
        max(2, reps // 4))
    del snaps
    torch.cuda.empty_cache()
    return out


SERVE_BUDGET = 200 << 30
SERVE_RATE = 200.0
SERVE_REQUESTS = 12000
SERVE_SPEEDUPS = (1, 5, 25)
RANGE_POOL = 4  # output buffers of the range requests, reused round robin
SERVE_SLOTS = 4  # batches in flight (one stream each; the device has four hardware queues)
# compressions per batch: at 25x the rate, batches of up to 8 on 4 streams
# sustained 923 GB/s against 775 for batches of every runnable variable
# (about 23) on 2 streams
SERVE_MAX_BATCH = 8


def _lat(xs):
    import numpy as np

    if not xs:
        return None
    a = np.asarray(xs)
    return {"p50": round(float(np.percentile(a, 50)), 3), "p99": round(float(np.percentile(a, 99)), 3),
            "max": round(float(a.max()), 3)}


def serving_section(torch, nk, inputs, requests: int, rate: float = SERVE_RATE) -> dict:
    """The serving loop: 32 live variables (sizes log-uniform 16 MB .. 4 GB,
    float32/float64, E in {1e-4, 1e-3}, B = 8), `requests` Poisson arrivals
    at `rate` per second, 5 % of them range decompressions of 20/40/60/80 %
    of a variable, admission under a 200 GB budget (the arena plus two
    pinned snapshots per variable).  The same request list is replayed at 1x,
    5x and 25x the rate, then the server is saturated (every variable's next
    compression at once); then the 25x list is served one request at a time
    through plain numarck_compress / numarck_decompress_range calls, each
    waited for, as the serial baseline.  Latency is arrival to completion."""
    specs = inputs.serving_specs()
    snaps = []
    for sp in specs:  # two snapshots per variable; compressions alternate between them
        p, q = inputs.mixture_pair(sp.n, seed=sp.seed, dtype=sp.dtype, device="cuda")
        snaps.append((p, q))
    max_range = max(int(sp.n * 0.8) * sp.dtype.itemsize for sp in specs)
    pool = [torch.empty(max_range // 8 + 1, dtype=torch.float64, device="cuda")
            for _ in range(RANGE_POOL)]
    torch.cuda.synchronize()
    resident = sum(2 * sp.n * sp.dtype.itemsize for sp in specs)
    free, _ = torch.cuda.mem_get_info()
    arena = min(SERVE_BUDGET - resident, free - (8 << 30))
    srv = nk.Server(budget_bytes=SERVE_BUDGET, arena_bytes=arena, slots=SERVE_SLOTS,
                    max_batch=SERVE_MAX_BATCH)

    def poll_all():
        got = []
        while True:
            part = srv.poll(4096)
            if not part:
                return got
            got += part

    for sp, (p, q) in zip(specs, snaps):
        srv.add_variable(p, sp.E, sp.B)
    state = [0] * len(specs)  # index of the resident snapshot
    # live variables already hold a record: one compression each first
    for v in range(len(specs)):
        state[v] ^= 1
        srv.compress(v, snaps[v][state[v]])
    srv.drain()
    assert all(c["status"] == 0 for c in poll_all())
    reqs = inputs.serving_requests(specs, rate, requests)
    n_range = sum(1 for r in reqs if r[2] == 1)

    def range_out(i, v, ln):
        buf = pool[i % RANGE_POOL]
        return buf.view(specs[v].dtype)[:max(ln, 1)]

    def replay(speed: float) -> dict:
        done, ri = [], 0
        t0 = time.perf_counter()
        for (t, v, kind, st, ln) in reqs:
            while time.perf_counter() - t0 < t / speed:
                time.sleep(2e-5)
            if kind == 0:
                state[v] ^= 1
                srv.compress(v, snaps[v][state[v]])
            else:
                srv.range(v, st, ln, out=range_out(ri, v, ln))
                ri += 1
            done += srv.poll(256)
        srv.drain()
        done += poll_all()
        assert len(done) == len(reqs), (len(done), len(reqs))
        assert all(c["status"] == 0 and c["flags"] == 0 for c in done), \
            [c for c in done if c["status"] or c["flags"]][:3]
        comp = [c for c in done if c["kind"] == 0]
        rng = [c for c in done if c["kind"] == 1]
        span_s = (max(c["done_us"] for c in done) - min(c["submit_us"] for c in done)) / 1e6
        in_bytes = sum(c["bytes"] for c in comp)
        return {"offered_gbs": round(in_bytes / (reqs[-1][0] / speed) / 1e9, 1),
                "sustained_gbs": round(in_bytes / span_s / 1e9, 1),
                "latency_ms": _lat([(c["done_us"] - c["submit_us"]) / 1e3 for c in comp]),
                "range_latency_ms": _lat([(c["done_us"] - c["submit_us"]) / 1e3 for c in rng]),
                "seconds": round(span_s, 2)}

    out = {"workload": "32 live variables, 16 MB..4 GB log-uniform, f32/f64, E in {1e-4,1e-3}, "
                       f"B=8; {len(reqs)} Poisson requests at {rate:g}/s (x1), replayed at x5 and "
                       "x25; 5% range decompressions of 20/40/60/80% of a variable",
           "requests": len(reqs), "range": n_range}
    for sp_ in SERVE_SPEEDUPS:
        out[f"x{sp_}"] = replay(float(sp_))
        print(f"# serving x{sp_}: {json.dumps(out[f'x{sp_}'])}", file=sys.stderr, flush=True)
    # saturated: one compression of every variable submitted at once
    srv.drain()
    poll_all()
    sat_t0 = time.perf_counter()
    for v in range(len(specs)):
        state[v] ^= 1
        srv.compress(v, snaps[v][state[v]])
    srv.drain()
    sat_s = time.perf_counter() - sat_t0
    sat = poll_all()
    assert len(sat) == len(specs) and all(c["status"] == 0 and c["flags"] == 0 for c in sat)
    out["saturated_gbs"] = round(sum(c["bytes"] for c in sat) / sat_s / 1e9, 1)
    stats = srv.stats()
    srv.close()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    out.update({"budget_gb": SERVE_BUDGET / 2**30, "resident_gb": round(resident / 2**30, 2),
                "arena_gb": round(arena / 2**30, 2),
                "arena_peak_gb": round(stats["arena_peak"] / 2**30, 2),
                "batches": stats["batches"], "max_batch": stats["max_batch_seen"],
                "waits_for_memory": stats["waits_for_memory"],
                "tail_retries": stats["tail_retries"]})

    # serial baseline: the 25x request list, one plain call at a time
    speed = float(SERVE_SPEEDUPS[-1])
    nmax = max(sp.n for sp in specs)
    ws = torch.empty(nk.numarck_workspace_bytes(nmax, nk.F64, 8), dtype=torch.uint8, device="cuda")
    recs, outs = [], []
    for v, sp in enumerate(specs):
        o = nk.alloc_outputs(sp.n, sp.dtype, sp.B, device="cuda")
        outs.append(o)
        c = nk.compress(snaps[v][state[v] ^ 1], snaps[v][state[v]], sp.E, sp.B, ws=ws, outputs=o)
        recs.append([c, snaps[v][state[v] ^ 1]])  # the record and its reference
    torch.cuda.synchronize()
    for r in recs:
        r[0].header()
    lat_c, lat_r, in_bytes, ri = [], [], 0, 0
    t0 = time.perf_counter()
    for (t, v, kind, st, ln) in reqs:
        arrive = t / speed
        while time.perf_counter() - t0 < arrive:
            time.sleep(2e-5)
        sp = specs[v]
        if kind == 0:
            prev, curr = snaps[v][state[v]], snaps[v][state[v] ^ 1]
            state[v] ^= 1
            c = nk.compress(prev, curr, sp.E, sp.B, ws=ws, outputs=outs[v])
            torch.cuda.synchronize()
            c.header()
            recs[v] = [c, prev]
            lat_c.append((time.perf_counter() - t0 - arrive) * 1e3)
            in_bytes += sp.n * sp.dtype.itemsize
        else:
            c, ref = recs[v]
            _, fl = nk.decompress_range(c, ref, st, ln, out=range_out(ri, v, ln))
            ri += 1
            assert int(fl.item()) == 0
            lat_r.append((time.perf_counter() - t0 - arrive) * 1e3)
    span = time.perf_counter() - t0
    out["serial_x25"] = {"sustained_gbs": round(in_bytes / span / 1e9, 1),
                         "latency_ms": _lat(lat_c), "range_latency_ms": _lat(lat_r),
                         "seconds": round(span, 2)}
    out["served_over_serial_x25"] = round(out["x25"]["sustained_gbs"] /
                                          out["serial_x25"]["sustained_gbs"], 2)
    del snaps, pool, ws, recs, outs
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=27)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--edge", type=int, default=EDGE)
    ap.add_argument("--cpu-sample", type=int, default=1 << 27,
                    help="elements of the oracle's CPU-baseline sample (0 = skip; the default "
                         "is all of pair 0 at 512^3)")
    ap.add_argument("--small-reps", type=int, default=200,
                    help="timed calls of the 64^3 latency measurement (0 = skip)")
    ap.add_argument("--batched-reps", type=int, default=10,
                    help="timed runs of each batched-vs-plain comparison (0 = skip)")
    ap.add_argument("--serve-requests", type=int, default=SERVE_REQUESTS,
                    help="Poisson requests of the serving measurement (0 = skip)")
    ap.add_argument("--variant-reps", type=int, default=-1,
                    help="timed runs of the auto-B, equal-width and zero-anchored sections "
                         "(-1 = max(3, steps / 3), 0 = skip)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run a 1 GiB device copy first (counter calibration)")
    ap.add_argument("--stream-reps", type=int, default=5,
                    help="timed runs of each reference streaming kernel (0 = skip)")
    ap.add_argument("--summarize-pmc", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "CMD"),
                    help="write profiles/pmc_{encode,decode,pipeline}_<workload>.json from two "
                         "rocprofv3 runs")
    ap.add_argument("--summarize-trace", nargs=4, metavar=("TRACE_CSV", "OUT_MD", "TITLE", "CMD"),
                    help="write a markdown summary of a rocprofv3 kernel trace")
    ap.add_argument("--summarize-sq", nargs=2, metavar=("SQ_DIR", "CMD"),
                    help="write profiles/sq_counters_<workload>.md from a rocprofv3 run of "
                         "the SQ instruction counters")
    args = ap.parse_args()
    if args.summarize_trace:
        summarize_trace(*args.summarize_trace)
        return
    if args.summarize_sq:
        summarize_sq(args.summarize_sq[0], f"flash3d_{args.edge}cubed_f64", args.edge ** 3,
                     args.summarize_sq[1])
        return
    if args.summarize_pmc:
        fd, wd, cmd = args.summarize_pmc
        summarize_pmc(fd, wd, f"flash3d_{args.edge}cubed_f64", cmd)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark measures one GPU; --gpus must be 1"}))
        sys.exit(2)

    import torch

    import paper_1703_02438_amd.numarck as nk
    from paper_1703_02438_amd import inputs

    dev = torch.device("cuda:0")
    if args.calib_copy:
        calib_copy(torch, nk, dev)
    stream_ref = stream_section(torch, nk, args.stream_reps) if args.stream_reps > 0 else None
    t_gen = time.time()
    series = inputs.FlashSeries(edge=args.edge, seed=1705, device="cuda")
    snaps = [series.x.clone()]
    for _ in range(SNAPSHOTS - 1):
        snaps.append(series.step().clone())
    del series
    torch.cuda.synchronize()
    # the CPU baseline's sample (host copies taken before the GPU buffers go)
    cs = min(args.cpu_sample, snaps[0].numel()) if args.cpu_sample > 0 else 0
    cpu_prev, cpu_curr = snaps[0][:cs].cpu(), snaps[1][:cs].cpu()
    print(f"# generated {SNAPSHOTS} snapshots of {args.edge}^3 float64 in "
          f"{time.time() - t_gen:.1f}s", file=sys.stderr, flush=True)
    n = snaps[0].numel()
    pairs = SNAPSHOTS - 1
    ws = torch.empty(nk.numarck_workspace_bytes(n, nk.F64, B), dtype=torch.uint8, device=dev)
    outs = nk.alloc_outputs(n, torch.float64, B, device=dev)
    stream = torch.cuda.current_stream()

    def step(i):
        return nk.compress(snaps[i % pairs], snaps[i % pairs + 1], E, B, ws=ws, outputs=outs,
                           stream=stream)

    # warmup with every kernel timed: finds the dominant kernel
    nk.timing_enable(True)
    alphas = []
    for i in range(max(args.warmup, 1)):
        c = step(i)
        h = c.header()
        c._host = None
        assert h.flags == 0, h.flags
        alphas.append(h.n_inc / n)
    torch.cuda.synchronize()
    per_kernel = nk.timing_read()
    nk.timing_enable(False)
    dominant = max(per_kernel, key=lambda k: per_kernel[k][1] / per_kernel[k][0])

    # timed region: K steps, per-step events, no other host work
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    t0 = time.perf_counter()
    for i in range(args.steps):
        evs[i][0].record(stream)
        step(i)
        evs[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat = sorted(a.elapsed_time(b) for a, b in evs)
    ms_per_step = wall * 1e3 / args.steps

    # dominant kernel timed live over the same K steps with HIP events
    nk.timing_enable(True)
    for i in range(args.steps):
        step(i)
    torch.cuda.synchronize()
    tk = nk.timing_read()
    nk.timing_enable(False)
    launches, kms = tk[dominant]
    avg_s = kms / launches / 1e3
    alpha = sum(alphas) / len(alphas)
    algo_bytes = ALGO.get(dominant, lambda a: 16.0)(alpha) * n
    achieved = algo_bytes / avg_s / 1e9
    workload = f"flash3d_{args.edge}cubed_f64"
    traffic = load_traffic(dominant, workload)

    in_bytes = n * 8
    value = in_bytes * args.steps / wall / 1e9
    # the whole call: the method's bytes and the bytes the counters measured
    # over every kernel of one call, against the call's time
    call_algo = ALGO_CALL(alpha) * n
    pipe_rec = load_pmc("pipeline", workload)
    call_meas = pipe_rec["bytes_per_call"] if pipe_rec else None
    call_s = ms_per_step / 1e3
    pipeline = {
        "algorithmic_bytes_per_call": int(call_algo),
        "algorithmic_bytes_per_element": round(ALGO_CALL(alpha), 4),
        "measured_bytes_per_call": call_meas,
        "measured_bytes_per_element": round(call_meas / n, 3) if call_meas else None,
        "ms_per_call": round(ms_per_step, 4),
        "frac_algorithmic": round(call_algo / call_s / 1e9 / HBM_PEAK_GBS, 4),
        "frac_measured": round(call_meas / call_s / 1e9 / HBM_PEAK_GBS, 4) if call_meas else None,
        # design traffic beyond the method's bytes: the window codes (written,
        # then read) and the staged indices of the incompressible points
        # (written, then read before their values are fetched)
        "window_code_bytes_per_call": int(2 * 2 * n),
        "staging_bytes_per_call": int(2 * 4 * alpha * n),
    }
    if stream_ref:
        pipeline["frac_measured_of_stream_read"] = (
            round(call_meas / call_s / 1e9 / stream_ref["read_nt"]["gbs"], 4) if call_meas else None)
    dec = decompress_section(torch, nk, step(0), snaps[0], args.steps, stream, workload)
    vreps = max(3, args.steps // 3) if args.variant_reps < 0 else args.variant_reps
    auto_b = ew = za = ll = None
    if vreps > 0:
        ll = lossless_section(torch, nk, step(0), n, vreps, stream)
        auto_b = auto_b_section(torch, nk, snaps[0], snaps[1],
                                nk.alloc_outputs(n, torch.float64, 16, device=dev), ws, vreps,
                                stream)
        topk_hdr = step(0).header()
        ew = variant_section(torch, nk, nk.compress_equal_width, snaps[0], snaps[1], topk_hdr,
                             ws, vreps, stream)
        za = variant_section(torch, nk, nk.compress_zero_anchored, snaps[0], snaps[1], topk_hdr,
                             ws, vreps, stream)
    del snaps, ws, outs, c
    torch.cuda.empty_cache()
    small = small_call_section(torch, nk, inputs, args.small_reps) if args.small_reps > 0 else None
    batched = None
    if args.batched_reps > 0:
        batched = batched_section(torch, nk, inputs, args.batched_reps)
        print(f"# batched: {json.dumps(batched)}", file=sys.stderr, flush=True)
    serving = None
    if args.serve_requests > 0:
        serving = serving_section(torch, nk, inputs, args.serve_requests)
        print(f"# serving: {json.dumps(serving)}", file=sys.stderr, flush=True)
    cpu = None
    if args.cpu_sample > 0:
        cpu = cpu_baseline(cpu_prev, cpu_curr, min(args.cpu_sample, n), n)

    p50 = lat[len(lat) // 2]
    p99 = lat[min(len(lat) - 1, int(round(0.99 * (len(lat) - 1))))]
    line = {
        "metric": "input GB/s compressed at 1 GPU (% HBM peak), batched vs plain; p50/p99 latency",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": workload,
            "form": "plain per-variable launches",
            "n": n, "E": E, "B": B, "snapshots": SNAPSHOTS, "pairs": pairs,
            "alpha": round(alpha, 5),
        },
        "latency_ms": {"p50": round(p50, 4), "p99": round(p99, 4)},
        "small_call": small,
        "decompress": dec,
        "auto_b": auto_b,
        "equal_width": ew,
        "zero_anchored": za,
        "lossless": ll,
        "batched": batched,
        "serving": serving,
        "kernels_us": {k: round(v[1] / v[0] * 1e3, 1) for k, v in per_kernel.items()},
        "roofline": {
            "bound": "hbm",
            "kernel": dominant,
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "algorithmic_bytes_per_launch": int(algo_bytes),
            "avg_launch_us": round(avg_s * 1e6, 2),
            "pipeline": pipeline,
        },
        "stream": stream_ref,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
