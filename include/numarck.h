/*
 * numarck.h -- C ABI of the MI355X (gfx950) NUMARCK compression library.
 *
 * NUMARCK ("Parallel Implementation of Lossy Data Compression for Temporal
 * Data Sets", Yuan et al., arXiv 1703.02438) compresses a snapshot D_i of a
 * simulation variable against the previous snapshot D_{i-1}:
 *   - change ratio of every point, d_j = (D_i,j - D_i-1,j) / D_i-1,j   (eq. 1)
 *   - a fine histogram of the ratios in bins of width 2E over their range,
 *     and the k = 2^B - 1 bins holding the most points     (Sec. IV-A, IV-B-1)
 *   - every point whose ratio falls in a selected bin is replaced by its
 *     B-bit bin index; the others get the escape index 2^B - 1 and their
 *     value is kept as is, in order, in the incompressible array (Sec. III-C)
 *   - the indices are bit-packed into the index table, which is cut into
 *     blocks; for each block the number of earlier incompressible points is
 *     recorded so that any range can be decompressed on its own (Sec. IV-C)
 *   - decompression multiplies the previous value by one plus the bin centre
 *     of its index (eq. 4, Sec. III-E), fully or for a range (Sec. V-C).
 * Around that path: the choice of B from the histogram (eqs. 5-6,
 * numarck_compress_auto), bins anchored at -E that need no range pass
 * (numarck_compress_zero_anchored, numarck_plan_create_zero_anchored),
 * equal-width binning (Sec. III-B, IV-B-3, numarck_compress_equal_width),
 * batches and plans of many compressions, a serving loop, and a lossless
 * stage for the index table in place of the paper's ZLIB
 * (numarck_lossless_encode / numarck_lossless_decode / _decode_range).
 *
 * Conventions shared by every entry point:
 *   - All data buffers are device memory owned by the caller.  The
 *     compression and decompression entry points never allocate device
 *     memory; a serving loop (numarck_server_*) allocates its arena once,
 *     at creation.  State kept between calls: a per-device count of compute
 *     units, the tunings recorded by numarck_autotune, and the optional
 *     timing records.
 *   - Calls are asynchronous on `stream` (a hipStream_t; NULL = the null
 *     stream).  The returned status reports argument validation and launch
 *     errors only; data-dependent results (counts, flags) are written to
 *     device memory and are valid once the stream reaches that point.
 *   - Concurrent calls must use distinct workspaces and outputs.
 *   - Arithmetic: binary64 for both snapshot types, round-to-nearest-even,
 *     no contraction, subnormals kept.
 *   - Readings of the paper used here: a point is valid when its previous
 *     value is nonzero and finite, its new value is finite, and its ratio is
 *     finite with |d| <= E * 2^50; invalid points are always incompressible.
 *     Bin m holds the ratios with floor((d - lo) / (2E)) == m, lo being the
 *     smallest valid ratio.  Ties between bins of equal count go to the
 *     lower bin id; empty bins are never selected; selected bins are indexed
 *     in ascending bin-id order.  Bin centre c_m = lo + (2m + 1) E rounded to
 *     the snapshot type.  A point is indexed only if its reconstruction
 *     T(p * (1 + c)) is within E * |p| of its value.
 */
#ifndef NUMARCK_H
#define NUMARCK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Snapshot element type. */
typedef enum { NUMARCK_F32 = 0, NUMARCK_F64 = 1 } numarck_dtype;

/* Status returned by every entry point. */
typedef enum {
  NUMARCK_OK = 0,
  NUMARCK_EINVAL = 1,    /* a required pointer is NULL, n >= 2^32, or a header is inconsistent */
  NUMARCK_EDTYPE = 2,    /* dtype is not NUMARCK_F32 / NUMARCK_F64 */
  NUMARCK_EBITS = 3,     /* B outside [1, 16] */
  NUMARCK_EBOUND = 4,    /* E is not a number in (0, 1] */
  NUMARCK_EALIGN = 5,    /* a snapshot pointer is not 16-byte aligned */
  NUMARCK_ECAPACITY = 6, /* the workspace is smaller than the minimum for this call */
  NUMARCK_EHIP = 7,      /* a HIP runtime call or kernel launch failed (see numarck_last_error) */
  NUMARCK_ERANGE = 8     /* start + len > n */
} numarck_status;

/* Bits of numarck_header.flags (compression) and of the decompression flag word. */
#define NUMARCK_FLAG_BAD_INDEX 1u     /* decompression met an index in [k_used, 2^B - 1) */
#define NUMARCK_FLAG_INC_OVERRUN 2u   /* decompression met more escapes than n_inc */
#define NUMARCK_FLAG_BAD_STREAM 8u    /* lossless decoding met a corrupt codeword stream */
#define NUMARCK_FLAG_TAIL_OVERFLOW 4u /* compression: more points outside the on-chip bin
                                         window than the workspace's tail capacity; the
                                         outputs of that call are not valid */

/* Result summary of one compression, written by the device (Fig. 2 holds the
 * paper's version of these fields). */
typedef struct numarck_header {
  uint64_t n;                /* points */
  uint64_t n_valid;          /* points with a valid change ratio */
  uint64_t n_invalid;        /* n - n_valid */
  uint64_t n_inc;            /* incompressible points (entries of incomp) */
  uint64_t n_blocks;         /* index-table blocks = ceil(n / elems_per_block) */
  uint64_t elems_per_block;  /* floor(8 * block_bytes / B) */
  uint64_t block_bytes;      /* index-table block size used */
  int64_t M;                 /* fine bins floor((hi - lo) / 2E) + 1; 0 if no valid point */
  uint64_t n_nonzero;        /* fine bins holding at least one point */
  uint32_t B;                /* index bits */
  uint32_t k_used;           /* selected bins = min(2^B - 1, n_nonzero) */
  uint32_t dtype;            /* numarck_dtype */
  uint32_t flags;            /* NUMARCK_FLAG_* */
  uint32_t tau;              /* smallest selected count; 0 when all nonzero bins are selected */
  uint32_t reserved0;
  double E;                  /* error bound */
  double lo, hi;             /* range of the valid ratios; 0, 0 when none is valid */
  uint64_t packed_bytes;     /* 4 * ceil(n * B / 32) */
  uint64_t compressed_bytes; /* 2^B * L + packed_bytes + n_inc * L, eq. (6) with actual sizes */
  uint64_t tail_count;       /* valid points whose bin lay outside the on-chip window */
  int64_t window_base;       /* first bin id of the on-chip window */
} numarck_header;

/* Output buffers of numarck_compress (all device memory, caller-owned). */
typedef struct numarck_out {
  uint32_t* packed;        /* numarck_packed_bytes(n, B) bytes: index table */
  void* centers;           /* numarck_centers_bytes(B, dtype) bytes: 2^B bin centres */
  void* incomp;            /* n * L bytes (worst case): incompressible values in element order */
  int64_t* block_inc_off;  /* numarck_block_count(n, B, block_bytes) entries */
  void* recon;             /* optional (NULL): n * L bytes, the value decompression will return */
  int64_t* bin_ids;        /* optional (NULL): 2^B - 1 entries, the fine bin of each index
                              (-1 past k_used) */
  numarck_header* hdr;     /* one header */
} numarck_out;

/* ---- sizes (host only, no device access) ---- */

/* Bytes of the packed index table: 4 * ceil(n * B / 32) (Sec. IV-C). */
size_t numarck_packed_bytes(uint64_t n, uint32_t B);
/* Bytes of the bin-centre table: 2^B * L (Sec. IV-B-2). 0 on a bad argument. */
size_t numarck_centers_bytes(uint32_t B, numarck_dtype dtype);
/* Indices per index-table block: floor(8 * block_bytes / B); block_bytes 0 means 2^20. */
uint64_t numarck_elems_per_block(uint32_t B, uint64_t block_bytes);
/* Number of index-table blocks: ceil(n / numarck_elems_per_block(B, block_bytes)). */
uint64_t numarck_block_count(uint64_t n, uint32_t B, uint64_t block_bytes);
/* Workspace bytes for numarck_compress that never overflow (tail capacity n). */
size_t numarck_workspace_bytes(uint64_t n, numarck_dtype dtype, uint32_t B);
/* Workspace bytes for a tail capacity of tail_cap points (clamped to n).  With a
 * smaller workspace numarck_compress uses the largest tail capacity that fits and
 * reports NUMARCK_FLAG_TAIL_OVERFLOW in the header if the data needs more. */
size_t numarck_workspace_bytes_tail(uint64_t n, numarck_dtype dtype, uint64_t tail_cap);
/* Workspace bytes for decompressing len points (full or range). */
size_t numarck_decompress_workspace_bytes(uint64_t len);

/* ---- compression (Sec. III-A..C, IV-A..C) ----
 * prev, curr : n values of `dtype`, 16-byte aligned (D_{i-1} and D_i)
 * E          : error bound in (0, 1]
 * B          : index bits in [1, 16]
 * block_bytes: index-table block size in bytes (0 = 2^20, the paper's 1 MB)
 * out        : host pointer to the output descriptor (device buffers)
 * ws         : device workspace of ws_bytes (>= numarck_workspace_bytes_tail(n, 0))
 * Inputs are only read; outputs are fully written (packed padding bits are 0,
 * centre slots past k_used are 0).  Without out->recon the snapshots are read
 * twice: the histogram pass also stores each point's bin place and the
 * outcome of its error check (Sec. III-C) in the workspace, 2 bytes a point,
 * and the indexing pass reads those; with out->recon, which needs both values
 * of every point, the indexing pass reads the snapshots a third time.  The
 * outputs are the same either way. */
numarck_status numarck_compress(const void* prev, const void* curr, uint64_t n,
                                numarck_dtype dtype, double E, uint32_t B,
                                uint64_t block_bytes, const numarck_out* out, void* ws,
                                size_t ws_bytes, void* stream);

/* ---- compression with zero-anchored bins (two passes instead of three) ----
 * As numarck_compress, with the fine bins of width 2E (Sec. IV-B-1) anchored
 * at -E instead of at the smallest valid ratio: bin m holds the ratios with
 * floor((d + E) / 2E) == m (m may be negative) and is centred on 2mE
 * (lo + (2m + 1) E with lo = -E).  Without a range to find first, the call
 * reads the snapshots once fewer than numarck_compress (once without
 * out->recon, twice with it).  Top-k, verification, escapes, packing and blocks are
 * unchanged, and so is the output format: numarck_decompress and
 * numarck_decompress_range read it.  Header: lo = -E, hi = 0, M = 0;
 * window_base is the first bin of the on-chip window, -8192.  bin_ids, if
 * given, holds the selected (signed) bin ids.  Same arguments, errors and
 * workspace as numarck_compress. */
numarck_status numarck_compress_zero_anchored(const void* prev, const void* curr, uint64_t n,
                                              numarck_dtype dtype, double E, uint32_t B,
                                              uint64_t block_bytes, const numarck_out* out,
                                              void* ws, size_t ws_bytes, void* stream);

/* ---- compression with equal-width binning (Sec. III-B, IV-B-3) ----
 * As numarck_compress, with the k = 2^B - 1 bins cut evenly from the range of
 * the valid ratios instead of chosen by count: w = (hi - lo) / k, a valid
 * point's index is min(floor((d - lo) / w), k - 1) (0 when w is 0), the centre
 * of index i is lo + (i + 1/2) w, and the same verification against E keeps
 * or escapes every point.  The output format is unchanged, so numarck_decompress
 * and numarck_decompress_range read it.  Header: M = k_used = k (0 with no
 * valid point), n_nonzero = tau = tail_count = window_base = 0; bin_ids, if
 * given, is filled with -1.  Same arguments, errors and workspace as
 * numarck_compress. */
numarck_status numarck_compress_equal_width(const void* prev, const void* curr, uint64_t n,
                                            numarck_dtype dtype, double E, uint32_t B,
                                            uint64_t block_bytes, const numarck_out* out,
                                            void* ws, size_t ws_bytes, void* stream);

/* ---- compression with B chosen from the histogram (Sec. IV-B-2, eqs. 5-6) ----
 * As numarck_compress, with the index width chosen in [B_min, B_max]
 * (1 <= B_min <= B_max <= 16): for each B the estimated size
 *   file_size(B) = 2^B L + n B / 8 + n alpha(B) L,
 * alpha(B) n being the points outside the 2^B - 1 fullest bins (invalid points
 * included), is computed from the histogram, which does not depend on B; the
 * smallest size wins (the smaller B on equal sizes) and the compression runs
 * with that B.  The estimate ignores the error-bound check, so the actual
 * n_inc can be larger.  Exact while the out-of-window bins fit the workspace's
 * tail capacity (otherwise the header reports NUMARCK_FLAG_TAIL_OVERFLOW).
 * out.packed, out.centers and out.block_inc_off must be sized for B_max.
 * The call waits once on the stream (the chosen B sizes the passes after
 * top-k): it returns with the histogram done and the rest queued.
 * B_out    : host; the chosen B.
 * est_bits : NULL, or 17 host uint64: 8 * file_size(B) at index B for
 *            B_min <= B <= B_max, 0 elsewhere. */
numarck_status numarck_compress_auto(const void* prev, const void* curr, uint64_t n,
                                     numarck_dtype dtype, double E, uint32_t B_min,
                                     uint32_t B_max, uint64_t block_bytes,
                                     const numarck_out* out, void* ws, size_t ws_bytes,
                                     void* stream, uint32_t* B_out, uint64_t* est_bits);

/* ---- full decompression (eq. 4, Sec. III-E) ----
 * hdr   : host copy of the header numarck_compress wrote
 * prev  : n values, the snapshot the data was compressed against
 * out   : n values
 * flags : device uint32; set to 0, then ORed with NUMARCK_FLAG_BAD_INDEX /
 *         NUMARCK_FLAG_INC_OVERRUN.  An escape past n_inc decodes to 0; an index
 *         in [k_used, ESC) decodes with its (zero) centre.
 * ws    : device workspace of >= numarck_decompress_workspace_bytes(n) bytes */
numarck_status numarck_decompress(const numarck_header* hdr, const void* prev,
                                  const uint32_t* packed, const void* centers,
                                  const void* incomp, const int64_t* block_inc_off, void* out,
                                  uint32_t* flags, void* ws, size_t ws_bytes, void* stream);

/* ---- partial decompression of [start, start + len) (Sec. IV-C, V-C) ----
 * Uses the block table to find the escapes before the range; reads the packed
 * table only from the start of the block holding `start`.
 * prev : the whole previous snapshot (n values); out : len values.
 * ws   : >= numarck_decompress_workspace_bytes(len) bytes.
 * Same flag behaviour as numarck_decompress.  start + len > n -> NUMARCK_ERANGE. */
numarck_status numarck_decompress_range(const numarck_header* hdr, const void* prev,
                                        const uint32_t* packed, const void* centers,
                                        const void* incomp, const int64_t* block_inc_off,
                                        uint64_t start, uint64_t len, void* out,
                                        uint32_t* flags, void* ws, size_t ws_bytes,
                                        void* stream);

/* ---- partial decompression that allocates nothing ----
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * operation, arguments, result and flags as numarck_decompress_range, with no
 * workspace argument.  The workspace is a device-global array of the library
 * (numarck_static_scratch_bytes() bytes, one copy per device, held until the
 * process ends); its device address is looked up once per device with
 * hipGetSymbolAddress on the first call made with that device current.  The
 * stream must belong to the current device.  The call never allocates:
 * no hipMalloc, no hipFree, no allocating library routine.
 * Every call on one device shares that device's array: calls that overlap on
 * one device (different streams, or different host threads, without ordering
 * between them) race and give undefined results.  Calls ordered on one stream
 * are safe; everything the array holds is written before it is read.
 * NUMARCK_ECAPACITY (with numarck_last_error() saying so) if the call's
 * workspace would exceed the array; the decompression workspace does not
 * grow with len, so this cannot happen for a valid header. */
size_t numarck_static_scratch_bytes(void);
numarck_status numarck_decompress_range_noalloc(const numarck_header* hdr, const void* prev,
                                                const uint32_t* packed, const void* centers,
                                                const void* incomp,
                                                const int64_t* block_inc_off, uint64_t start,
                                                uint64_t len, void* out, uint32_t* flags,
                                                void* stream);

/* ---- inspection of the last compression's histogram (Sec. IV-B-1) ----
 * After numarck_compress on the same workspace, size and dtype and on the same
 * stream, writes the nonzero fine bins (id, count), in no particular order, to
 * ids/counts (device, room for `capacity` entries) and their number to
 * *count_dev (device uint64).  Entries beyond `capacity` are dropped (the count
 * is still exact). */
numarck_status numarck_histogram_export(const void* ws, size_t ws_bytes, uint64_t n,
                                        numarck_dtype dtype, int64_t* ids, uint32_t* counts,
                                        uint64_t capacity, uint64_t* count_dev, void* stream);

/* ---- launch tuning ----
 * Launch parameters of the passes.  No setting changes any output; they only
 * trade occupancy, atomic traffic and work granularity.  Filled with the
 * defaults by numarck_tuning_default; numarck_autotune measures candidates. */
typedef struct numarck_tuning {
  uint32_t range_blocks_per_cu; /* pass-1 workgroups per compute unit */
  uint32_t hist_blocks_per_cu;  /* histogram workgroups per compute unit */
  uint32_t hist_lds;            /* 1: window counts in LDS (64 KB per workgroup); 0: in global
                                   memory, and the indexing pass reads the snapshots again
                                   (no window codes) */
  uint32_t chunk_vec;           /* 16-byte vectors per streaming chunk of the first two passes;
                                   0: automatic, about four chunks per compute unit for each
                                   element type's group (a power of two in [4096, 65536]) */
  uint32_t unit_pct;            /* encoder waves as a percentage of the resident capacity (1..100) */
  uint32_t stream_loads;        /* input loads of the three passes: 0 automatic (non-temporal when
                                   a pass streams at least 512 MB and no input is shared between
                                   jobs), 1 non-temporal, 2 cached */
} numarck_tuning;

void numarck_tuning_default(numarck_tuning* t);

/* numarck_compress with explicit launch tuning (NULL = the tuning recorded by
 * numarck_autotune for this size class and dtype, else the defaults). */
numarck_status numarck_compress_tuned(const void* prev, const void* curr, uint64_t n,
                                      numarck_dtype dtype, double E, uint32_t B,
                                      uint64_t block_bytes, const numarck_out* out, void* ws,
                                      size_t ws_bytes, const numarck_tuning* tune, void* stream);

/* Measure candidate tunings on one compression (inputs as for numarck_compress,
 * `reps` timed runs per candidate), write the fastest to *best and record it
 * for the size class (floor(log2 n)) and dtype.  Synchronises `stream`.  The
 * outputs buffers are overwritten by the trial runs. */
numarck_status numarck_autotune(const void* prev, const void* curr, uint64_t n,
                                numarck_dtype dtype, double E, uint32_t B, uint64_t block_bytes,
                                const numarck_out* out, void* ws, size_t ws_bytes, uint32_t reps,
                                void* stream, numarck_tuning* best);
/* Save / load the recorded tunings as text (one line per size class). */
numarck_status numarck_tuning_save(const char* path);
numarck_status numarck_tuning_load(const char* path);

/* ---- batched compression: many variables / time steps in one chain ----
 * Each job is one numarck_compress (its own inputs, E, B, block size and
 * outputs).  All jobs go through the same passes with one launch per pass and
 * element type (the encoder: per index-width class), whatever their number;
 * results are identical to compressing each job alone. */
typedef struct numarck_job {
  const void* prev;
  const void* curr;
  uint64_t n;
  numarck_dtype dtype;
  double E;
  uint32_t B;
  uint64_t block_bytes;  /* 0 = 2^20 */
  numarck_out out;
  uint64_t tail_cap;     /* points outside the on-chip bin window the job's workspace can hold
                            (0 or >= n: n, which never overflows); a smaller capacity shrinks the
                            workspace, and data needing more sets NUMARCK_FLAG_TAIL_OVERFLOW */
} numarck_job;

/* Most jobs in one batch (one grid row per job in the per-job passes). */
#define NUMARCK_MAX_JOBS 65535u

/* A plan: the static description of a batch (job table, per-job workspace,
 * work partition) written once into the workspace; running it only launches
 * kernels, so it can be captured into a HIP graph and replayed. */
typedef struct numarck_plan numarck_plan;

/* Workspace bytes for a batch (each job with its tail_cap). */
size_t numarck_batch_workspace_bytes(const numarck_job* jobs, uint32_t njobs);
/* Validate the jobs, lay out the workspace and copy the job table to it on
 * `stream` (asynchronous).  tune = NULL: defaults.  *plan is host memory owned
 * by the caller until numarck_plan_destroy. */
numarck_status numarck_plan_create(const numarck_job* jobs, uint32_t njobs,
                                   const numarck_tuning* tune, void* ws, size_t ws_bytes,
                                   void* stream, numarck_plan** plan);
/* As numarck_plan_create, with every job's bins anchored at -E as in
 * numarck_compress_zero_anchored (two reads of each snapshot instead of
 * three; same outputs as that call for each job). */
numarck_status numarck_plan_create_zero_anchored(const numarck_job* jobs, uint32_t njobs,
                                                 const numarck_tuning* tune, void* ws,
                                                 size_t ws_bytes, void* stream,
                                                 numarck_plan** plan);
/* Compress every job of the plan on `stream`. */
numarck_status numarck_plan_run(const numarck_plan* plan, void* stream);
/* The launch groups a plan runs, in launch order: the range-pass groups (none
 * in a zero-anchored plan), the histogram groups, then the encoder groups.
 * Each group covers consecutive jobs of the plan's internal order, which is
 * the caller's order stably sorted by (dtype, encoder index-width class).
 * Writes up to `cap` records to `out` (may be NULL) and returns the number of
 * groups.  For tests and tuning reports; no device work. */
typedef enum {
  NUMARCK_PASS_RANGE = 0, NUMARCK_PASS_HIST = 1, NUMARCK_PASS_ENCODE = 2
} numarck_pass;
typedef struct numarck_plan_group {
  uint32_t pass;       /* numarck_pass */
  uint32_t dtype;      /* numarck_dtype of the group's jobs */
  uint32_t cls;        /* encoder: 0 B < 8, 1 B = 8, 2 8 < B < 16, 3 B = 16; else 0 */
  uint32_t first_job;  /* caller's index of the group's first job */
  uint32_t njobs;      /* jobs in the group */
  uint32_t chain;      /* 1: a time chain (each job's prev is the previous job's curr):
                          the range pass sweeps it once, the histogram walks its
                          jobs in step; 0 otherwise (always 0 for the encoder) */
  uint32_t load_hint;  /* loads the group's kernels issue: 0 both inputs cached,
                          1 both non-temporal, 2 prev non-temporal and curr cached */
  uint32_t hist_lds;   /* histogram: 1 LDS window counts, 0 global counts; else 0 */
} numarck_plan_group;
uint32_t numarck_plan_groups(const numarck_plan* plan, numarck_plan_group* out, uint32_t cap);
/* Capture numarck_plan_run on `stream` (not the null stream) into a HIP graph
 * kept by the plan; numarck_plan_replay launches it.  Inputs and outputs are
 * the plan's buffers: replays compress whatever they hold at that time. */
numarck_status numarck_plan_capture(numarck_plan* plan, void* stream);
numarck_status numarck_plan_replay(const numarck_plan* plan, void* stream);
void numarck_plan_destroy(numarck_plan* plan);
/* One-shot batch: plan, run, destroy. */
/* Launch tuning of a batch: a coordinate descent over the numarck_tuning
 * fields (range and histogram workgroups per compute unit, histogram window
 * counts in LDS or in global memory, chunk size, encoder waves), each
 * candidate timed over `reps` runs of a plan of these jobs (a candidate more
 * than twice as slow as the best after one run is dropped).  Writes the
 * fastest to *best, for numarck_plan_create / _zero_anchored
 * (zero_anchored != 0 times zero-anchored plans).  Runs the jobs many times:
 * their outputs hold the last run's results.  Synchronises the stream. */
numarck_status numarck_plan_autotune(const numarck_job* jobs, uint32_t njobs, void* ws,
                                     size_t ws_bytes, uint32_t reps, uint32_t zero_anchored,
                                     void* stream, numarck_tuning* best);
numarck_status numarck_compress_batch(const numarck_job* jobs, uint32_t njobs, void* ws,
                                      size_t ws_bytes, void* stream);

/* ---- serving loop: continuous batching under a device memory budget ----
 * A server owns a device arena (one allocation at creation) for compressed
 * records and workspaces, a scheduler thread and `slots` HIP streams.
 * Variables are registered with their first snapshot; each compression
 * request brings the variable's next snapshot and is compressed against the
 * previous one, which stays resident on the device (zero copy: the snapshot
 * buffers are the caller's).  Requests of one variable run in submission
 * order; requests of different variables are batched together (one plan per
 * batch, numarck_plan_*) and batches on different slots overlap: a batch
 * takes at most max_batch compressions and at most its share of the
 * runnable ones (their count over the free slots, rounded up), so a full
 * queue keeps every slot busy.  A request
 * is admitted when its record and workspace fit in the arena; otherwise it
 * waits for memory to be released.  Range requests decompress part of the
 * variable's latest record (the record of its last compression submitted
 * before the range request).  A compression first runs with a bounded tail
 * capacity (n / 16 points outside the on-chip bin window, at least 2^20),
 * which keeps its workspace near n * L bytes; if the data needs more, it is
 * run again with full capacity before anything else of its variable.
 * Results are identical to numarck_compress / numarck_decompress_range
 * called on each request alone. */
typedef struct numarck_server numarck_server;

typedef struct numarck_server_config {
  uint64_t budget_bytes; /* device bytes the server may account for: the arena plus the
                            registered variables' snapshots, two per variable (the latest
                            record's reference and the next previous snapshot, both
                            pinned by the request contract below) */
  uint64_t arena_bytes;  /* device arena for records and workspaces (<= budget_bytes) */
  uint32_t slots;        /* batches in flight at once, one HIP stream each (1..8) */
  uint32_t max_batch;    /* compression requests per batch (1..NUMARCK_MAX_JOBS) */
  int32_t device;        /* HIP device of the server */
  uint32_t reserved;
} numarck_server_config;

typedef enum numarck_req_kind {
  NUMARCK_REQ_COMPRESS = 0,
  NUMARCK_REQ_RANGE = 1
} numarck_req_kind;

typedef struct numarck_request {
  uint32_t kind;   /* numarck_req_kind */
  uint32_t var;    /* variable id from numarck_server_add_variable */
  const void* curr; /* COMPRESS: the next snapshot (device, n elements, 16-byte aligned).  It
                       becomes the variable's resident previous snapshot, and it is the
                       reference of the new record: keep it unchanged until the variable's
                       second-next compression has completed. */
  uint64_t start;  /* RANGE: first element */
  uint64_t len;    /* RANGE: element count */
  void* out;       /* RANGE: destination (device, len elements, 16-byte aligned) */
  void* ready;     /* optional hipEvent_t: the request's stream waits for it before reading
                      curr / writing out (the event must outlive the request); NULL: the
                      caller has made the data ready before submitting */
} numarck_request;

typedef struct numarck_completion {
  uint64_t ticket;
  uint32_t var;
  uint32_t kind;
  int32_t status;    /* numarck_status of the request */
  uint32_t flags;    /* record flags (COMPRESS) or decode flags (RANGE) */
  uint64_t bytes;    /* input bytes (COMPRESS) or output bytes (RANGE) */
  uint64_t batch;    /* serial number of the batch that ran it */
  double submit_us;  /* host clock, microseconds since the server's creation */
  double start_us;   /* launch of its batch */
  double done_us;    /* completion observed by the scheduler */
} numarck_completion;

typedef struct numarck_server_stats {
  uint64_t submitted, completed, batches, max_batch_seen;
  uint64_t arena_capacity, arena_peak, resident_bytes;
  uint64_t waits_for_memory; /* scheduler passes that left an eligible request queued for lack of memory */
  uint64_t tail_retries;     /* compressions run again with full tail capacity (see below) */
} numarck_server_stats;

/* Create a server (allocates the arena with hipMalloc, creates the streams
 * and starts the scheduler thread).  ECAPACITY if arena_bytes > budget_bytes. */
numarck_status numarck_server_create(const numarck_server_config* cfg, numarck_server** out);
/* Register a variable of n elements with its first snapshot `initial` (device,
 * caller-owned, kept unchanged until the variable's second compression has
 * completed).  ECAPACITY if its two pinned snapshots (2 n L bytes) would take
 * the resident snapshots plus the arena past the budget, or if one
 * compression of it could never fit in the arena. */
numarck_status numarck_server_add_variable(numarck_server* s, uint64_t n, numarck_dtype dtype,
                                           double E, uint32_t B, uint64_t block_bytes,
                                           const void* initial, uint32_t* var_id);
/* Queue a request (thread-safe, non-blocking); *ticket identifies its completion. */
numarck_status numarck_server_submit(numarck_server* s, const numarck_request* r,
                                     uint64_t* ticket);
/* Completed requests since the last poll, oldest first (at most cap); returns the count. */
uint32_t numarck_server_poll(numarck_server* s, numarck_completion* out, uint32_t cap);
/* Block until every submitted request has completed. */
numarck_status numarck_server_drain(numarck_server* s);
/* Copy the variable's latest record to caller buffers (sized as for
 * numarck_compress of the variable; recon and bin_ids are not copied) on
 * `stream`, synchronously.  EINVAL if it has none yet.  Call it when no
 * request of the variable is queued (e.g. after numarck_server_drain). */
numarck_status numarck_server_fetch(numarck_server* s, uint32_t var, const numarck_out* dst,
                                    void* stream);
numarck_status numarck_server_get_stats(numarck_server* s, numarck_server_stats* st);
/* Drain, stop the scheduler, release the arena and streams. */
void numarck_server_destroy(numarck_server* s);

/* ---- reference streaming kernels (measurement, not part of the path) ----
 * The HBM roofline the compression passes are measured against: a read, a
 * write or a copy of `bytes` bytes with 16-byte vector accesses, cached or
 * non-temporal, `per_cu` workgroups of 256 threads per compute unit (1..64),
 * each thread walking the vectors grid-strided.
 *   READ, READ_NT   : reads src; writes one 32-bit word per wave to dst,
 *                     which must hold 16 * per_cu * (compute units) bytes
 *   WRITE, WRITE_NT : writes dst (every 32-bit word 0x3FF00000); src unused
 *   COPY, COPY_NT   : copies src to dst (distinct buffers)
 *   READ2_WRITE16   : the encoder's traffic: src is two arrays of bytes/2
 *                     each, read in step (non-temporal); for every 16-byte
 *                     position one 16-bit word goes to dst (bytes/16 bytes
 *                     written, 1/16 of the read volume)
 *   READ2_WRITE8    : the same with one 32-bit word per position (bytes/8
 *                     bytes written, 1/8 of the read volume: the histogram
 *                     pass writing the window codes of 64-bit values)
 * bytes must be a multiple of 16 (of 32 for the READ2 kinds), src and dst
 * 16-byte aligned.  EINVAL on a bad kind, size, pointer or per_cu;
 * asynchronous on `stream`. */
typedef enum {
  NUMARCK_STREAM_READ = 0, NUMARCK_STREAM_READ_NT = 1,
  NUMARCK_STREAM_WRITE = 2, NUMARCK_STREAM_WRITE_NT = 3,
  NUMARCK_STREAM_COPY = 4, NUMARCK_STREAM_COPY_NT = 5,
  NUMARCK_STREAM_READ2_WRITE16 = 6, NUMARCK_STREAM_READ2_WRITE8 = 7
} numarck_stream_kind;
numarck_status numarck_stream_kernel(int kind, const void* src, void* dst, uint64_t bytes,
                                     uint32_t per_cu, void* stream);

/* ---- diagnostics ---- */
const char* numarck_status_str(numarck_status s);
/* Text of the last HIP error seen by this thread ("" if none). */
const char* numarck_last_error(void);

/* Per-kernel timing with HIP events on the calls' streams (for benchmarks).
 * numarck_timing_enable(1) starts recording every kernel launch of later calls;
 * numarck_timing_read synchronises the recorded events and returns, for up to
 * `cap` kernel kinds, the name, launch count and summed milliseconds, then
 * clears the records.  Not thread-safe; disabled by default. */
void numarck_timing_enable(int on);
int numarck_timing_read(const char** names, uint32_t* launches, double* ms, int cap);

/* ---- lossless stage of the index table (in place of Sec. IV-C's ZLIB) ----
 * The paper passes each block of the index table through ZLIB.  This stage is
 * a prefix code without a tree, every step a pass on the device:
 *   - the 2^B codes are ranked by how often they occur in the table (more
 *     often first, equal counts by the smaller code); code_of_rank lists them;
 *   - rank v is written as an exponential-Golomb codeword of order k: with
 *     x = v + 2^k and nb = floor(log2 x), nb - k zero bits, a one bit, then the
 *     low nb bits of x least significant first (2 nb - k + 1 bits);
 *   - k in [0, B] is the order with the fewest bits (the smaller k on ties);
 *   - sub-blocks of 1024 codes each start on a 32-bit word (the one before is
 *     padded with zeros); sub_off[s] is the first bit of sub-block s and
 *     sub_off[n_sub] the stream's length in bits, so any sub-block decodes on
 *     its own;
 *   - a sub-block opens with eight 16-bit offsets (4 words): the first bit of
 *     each group of 128 consecutive codes, relative to the sub-block's first
 *     bit (an empty group past n: where the codewords end); the groups'
 *     codewords follow without gaps, so each group decodes on its own too
 *     (the decoder gives each group to one lane);
 *   - bits are numbered least significant first in little-endian words. */
typedef struct numarck_lossless_header {
  uint64_t n;            /* codes in the table */
  uint64_t n_sub;        /* sub-blocks: ceil(n / 1024) */
  uint64_t stream_words; /* 32-bit words of the stream (group tables, codewords, padding) */
  uint64_t bits;         /* codeword bits, without the group tables and the padding */
  uint32_t B;            /* index width */
  uint32_t k;            /* exponential-Golomb order */
  uint32_t flags;        /* 0 */
  uint16_t sub_log2;     /* log2 of the codes per sub-block: 10 */
  uint16_t group_log2;   /* log2 of the codes per group: 7 */
  uint64_t bytes;        /* stored size: 2 * 2^B + 8 (n_sub + 1) + 4 stream_words + this header */
} numarck_lossless_header;

/* Sub-blocks of a table of n codes: ceil(n / 1024). */
uint64_t numarck_lossless_subblocks(uint64_t n);
/* Stream bytes that always suffice: 4 (ceil(n (B + 1) / 32) + 5 n_sub).  (Order
 * k = B costs at most B + 1 bits per code, and the chosen order no more; each
 * sub-block adds its 4-word group table and at most one padding word.) */
size_t numarck_lossless_stream_bytes(uint64_t n, uint32_t B);
/* Workspace bytes of numarck_lossless_encode. */
size_t numarck_lossless_workspace_bytes(uint32_t B);

/* Encode the index table `packed` (n codes of B bits, device) into
 * code_of_rank (2^B uint16), sub_off (n_sub + 1 uint64, bits) and stream
 * (stream_bytes >= numarck_lossless_stream_bytes(n, B)); hdr is a device
 * numarck_lossless_header.  All device buffers, written in full; the call
 * only enqueues work on `stream_`.  Errors: NUMARCK_EBITS (B), NUMARCK_EINVAL
 * (NULL pointer, n >= 2^32), NUMARCK_ECAPACITY (stream or workspace too
 * small), NUMARCK_EHIP. */
numarck_status numarck_lossless_encode(const uint32_t* packed, uint64_t n, uint32_t B,
                                       uint16_t* code_of_rank, uint64_t* sub_off,
                                       uint32_t* stream, size_t stream_bytes,
                                       numarck_lossless_header* hdr, void* ws, size_t ws_bytes,
                                       void* stream_);
/* Decode back to the B-bit index table `packed` ((n B + 31) / 32 words,
 * device).  hdr is a HOST copy of the encoder's header; the other pointers
 * are device buffers (stream and packed 16-byte aligned); flags (device
 * uint32) is set to 0, then ORed with
 * NUMARCK_FLAG_BAD_STREAM if a sub-block's offsets or codewords are corrupt
 * (that sub-block's codes are then incomplete).  Reads stay within the
 * stream's hdr->stream_words words and writes within the table.  Errors:
 * NUMARCK_EBITS, NUMARCK_EINVAL (NULL pointer, inconsistent header, a
 * sub-block or group size other than this library's), NUMARCK_EALIGN,
 * NUMARCK_EHIP. */
numarck_status numarck_lossless_decode(const numarck_lossless_header* hdr,
                                       const uint16_t* code_of_rank, const uint64_t* sub_off,
                                       const uint32_t* stream, uint32_t* packed, uint32_t* flags,
                                       void* stream_);

/* Partial decoding (the lossless counterpart of Sec. IV-C's independent
 * blocks): sub-blocks [sub_begin, sub_begin + sub_count) only, each written
 * to its own place in the full-size table `packed`; the rest of `packed` is
 * not touched.  Sub-block s holds codes [1024 s, 1024 (s + 1)).  For
 * numarck_decompress_range of [start, start + len) decode the sub-blocks
 * covering the codes from the start of start's index-table block
 * (floor(start / elems_per_block) * elems_per_block) to start + len.
 * Errors as numarck_lossless_decode, plus NUMARCK_ERANGE when the
 * sub-blocks run past n_sub. */
numarck_status numarck_lossless_decode_range(const numarck_lossless_header* hdr,
                                             const uint16_t* code_of_rank,
                                             const uint64_t* sub_off, const uint32_t* stream,
                                             uint64_t sub_begin, uint64_t sub_count,
                                             uint32_t* packed, uint32_t* flags, void* stream_);

#ifdef __cplusplus
}
#endif
#endif
