// nk_internal.h -- internal definitions shared by the gfx950 kernels and the
// C-ABI layer of the NUMARCK library.  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/numarck.h"

namespace nk {

// ---------------------------------------------------------------- constants
// On-chip (LDS) window of fine bins used by the histogram and the encoder.
// Bins outside it are counted exactly through the tail list + hash table.
constexpr int WIN = 16384;
constexpr uint32_t HEMPTY = 0xFFFFFFFFu;  // empty hash slot
constexpr int MAX_SEL = 65535;            // k for B = 16

// The encoder and decoder are range-partitioned by wave: each wave ("unit")
// owns a contiguous run of wave tiles and keeps a running count of
// incompressible points, so no wave ever waits for another.  A wave tile is
// 4 rounds of one 16-byte vector per lane: 512 float64 or 1024 float32.
// Tuning knobs (compile-time; every setting computes identical outputs).
#ifndef NK_ENC_ROUNDS
#define NK_ENC_ROUNDS 2      // vector rounds per encoder wave tile
#endif
#ifndef NK_ENC_PREFETCH
#define NK_ENC_PREFETCH 1    // issue the next tile's loads before computing
#endif
#ifndef NK_DEC_ROUNDS
#define NK_DEC_ROUNDS 4      // vector rounds per decoder wave tile
#endif
#ifndef NK_DEC_DIRECT
#define NK_DEC_DIRECT 0      // decoder reads index bits from global, not via LDS
#endif
#ifndef NK_HIST_REVERSE
#define NK_HIST_REVERSE 0    // histogram sweep from the end of the arrays
#endif
#ifndef NK_HIST_TPB
#define NK_HIST_TPB 512
#endif
// Encoder lanes with nothing to store write to a per-wave slot here instead,
// so every full tile issues the same number of stores (see k_encode).
constexpr int SINK_SLOTS = 256;
constexpr int UNIT_TPB = 256;      // 4 units per workgroup
constexpr int ENC_ROUNDS = NK_ENC_ROUNDS;
constexpr int DEC_ROUNDS = NK_DEC_ROUNDS;
constexpr int MAX_UNITS = 8192;
// Pieces of the part of a block before a decompression range, counted in
// parallel, at most.
constexpr int MAX_PRE_UNITS = 1024;

// ------------------------------------------------ device control block
// Lives at the start of the compression workspace.  Fields above `lo` are
// reset by k_init at the start of every call.
struct Ctl {
  unsigned long long lo_key;      // order key of the smallest valid ratio (atomicMin)
  unsigned long long hi_key;      // order key of the largest valid ratio (atomicMax)
  unsigned long long n_invalid;   // points that are not valid
  unsigned long long tail_count;  // points outside the window (may exceed capacity)
  unsigned int tile_ticket;       // encoder tile tickets
  unsigned int flags;             // NUMARCK_FLAG_*
  unsigned int tail_bins;         // distinct tail bins (k_hinsert)
  unsigned int tail_max;          // largest tail-bin count (k_hinsert)
  // derived from the range (derive_job): written by k_hclear, read by the
  // kernels after it (the histogram derives them itself)
  double lo, hi;
  long long M;
  long long wbase;
  unsigned long long n_valid;
  unsigned int win_len;
  unsigned int empty;
  // hash table in use
  unsigned long long H;
  unsigned long long tail_used;   // min(tail_count, capacity)
  // selection
  unsigned long long n_nonzero;
  long long cut;                  // tie cut: selected ties have id <= cut
  unsigned int tau;               // k-th count (0: every nonzero bin selected)
  unsigned int k_used;
  unsigned int nsel_window;
  unsigned int nsel_tail;
  unsigned int nsel_tail_below;
  unsigned int n_inc;             // incompressible points (k_gather)
  // choice of B (k_autob): estimated size in bits per B
  unsigned long long est_bits[17];
  // equal-width binning (k_ewprep): chunk width and its reciprocal
  double ew_w, ew_inv;
};

// Control block of a decompression call.
struct DCtl {
  unsigned long long base;  // escapes before `start`
};

// Workspace layout of one compression (byte offsets from the workspace base).
struct Layout {
  size_t ctl, gwin, lut, sel_tail, sorted_tail, unit_cnt, sink, scratch, wcode, tail, hslot,
      hcnt, total;
  uint64_t tail_cap, hcap;
};
Layout compress_layout(uint64_t n, uint64_t elem_bytes, uint64_t tail_cap);

// Everything a compression kernel needs (passed by value).
struct CParams {
  const void* prev;
  const void* curr;
  uint64_t n;
  double E, twoE, cap;
  double inv2E;      // binary64 1/(2E), used with an exactness check
  uint32_t B;
  uint32_t k;        // 2^B - 1 (also the escape code)
  uint64_t epb;      // elements per index-table block
  uint64_t n_blocks;
  uint64_t n_tiles;
  uint64_t packed_words;
  Ctl* ctl;
  uint32_t* gwin;
  uint16_t* lut;      // window bin -> index, or the escape code if not selected
  uint32_t mulB;      // ceil(2^32 / B) for B > 1: floor(x / B) = mulhi(x, mulB) for x < 2^15
  int64_t* tail;
  uint64_t tail_cap;
  uint32_t* hslot;
  uint32_t* hcnt;
  uint64_t hcap;
  int64_t* sel_tail;
  int64_t* sorted_tail;
  uint32_t* unit_cnt;  // incompressible points per encoder unit, then their offsets
  void* scratch;       // incompressible values (or, precoded, their element
                       // indices) staged per unit range
  // Precoded encoding (pre != 0): the histogram pass also writes each
  // point's window code (WC_* below) and the encoder reads those 2 bytes in
  // place of the 2L bytes of the snapshots.
  uint16_t* wcode;
  uint32_t pre;
  uint32_t tile_elems;  // elements of an encoder wave tile
  void* sink;          // SINK_SLOTS x 256 bytes written by masked-off lanes (never read)
  uint32_t n_units;
  uint64_t tiles_per_unit;
  uint32_t* packed;
  void* centers;
  void* incomp;
  int64_t* block_inc_off;
  void* recon;
  int64_t* bin_ids;
  numarck_header* hdr;
  uint64_t block_bytes;
  int dtype;
};

struct DParams {
  const void* prev;
  const uint32_t* packed;
  const void* centers;
  const void* incomp;
  const int64_t* block_inc_off;
  void* out;
  uint32_t* flags;
  uint64_t n, start, len, n_inc, epb, packed_words;
  uint32_t B, k_used;
  int dtype;
  DCtl* dctl;
  uint32_t* unit_cnt;  // escapes per decoder unit range, then their offsets
  uint32_t* pre_cnt;   // escapes per piece of start's block before start
  uint32_t n_units;
  uint32_t pre_units;  // pieces of [start of start's block, start)
  uint64_t pre_elems;  // indices per piece
  uint64_t tiles_per_unit;
  uint64_t n_tiles;
  uint64_t tile_elems;  // elements of a wave tile
};

// Launch geometry of the streaming kernels for the current device.
struct Geometry {
  int cus;
};
Geometry geometry();

// Where a launch's work items come from: for a batch, the device prefix
// arrays map a streaming chunk or an encoder unit to its job; for one job
// they are null and everything belongs to job_begin.
struct Geo {
  const uint64_t* chunk0;  // first streaming chunk of each job, then the total
  const uint32_t* unit0;   // first encoder unit of each job, then the total
  uint32_t job_begin, job_end;
  uint64_t c_begin, c_end;  // streaming chunks of this launch
  uint32_t u_begin, u_end;  // encoder units of this launch
  uint32_t chunk_vec;       // 16-byte vectors per streaming chunk
  uint32_t stream_nt;       // load hints of the streaming passes (stream_nt_for)
  uint32_t chain;           // the jobs are a time chain (see JobGroup::chain)
  uint32_t za;              // zero-anchored bins: the window is set before the
                            // histogram (k_init), not derived from the range
};

// Launch parameters a tuner may change (none changes any output).
struct Tuning {
  uint32_t range_blocks_per_cu;  // k_range grid = this x CUs (capped by chunks)
  uint32_t hist_blocks_per_cu;   // k_hist grid
  uint32_t hist_lds;             // 1: LDS window counts, 0: global window counts
  uint32_t chunk_vec;            // 16-byte vectors per streaming chunk (0: automatic)
  uint32_t unit_pct;             // encoder units, % of the resident capacity
  uint32_t stream_loads;         // 0: automatic, 1: non-temporal, 2: cached
};
Tuning default_tuning();

// A contiguous group of jobs of one element type (and, for the encoder, one
// index-width class: 0 = B < 8, 1 = B == 8, 2 = 8 < B < 16, 3 = B == 16).
struct JobGroup {
  int dtype;
  int cls;
  uint32_t nt;         // load hints of the streaming passes (stream_nt_for)
  uint32_t chunk_vec;  // 16-byte vectors per streaming chunk of this group
  uint32_t job_begin, job_end;
  uint64_t c_begin, c_end;
  uint32_t u_begin, u_end;
  // The jobs are a time chain (job i's curr is job i+1's prev, one n).  In
  // a range-pass group it is read as one sweep over the snapshots and
  // c_begin/c_end count the chain's own chunks from 0; in a histogram group
  // the chunks keep the batch numbering and each workgroup stays on one job,
  // consecutive jobs in step.
  uint32_t chain;
  // Encoder groups: the jobs take the precoded encoding (CParams::pre).
  uint32_t pre;
};
inline int enc_class(uint32_t B) { return B < 8 ? 0 : B == 8 ? 1 : B < 16 ? 2 : 3; }

// Input bytes per pass above which a streaming pass gains nothing from
// caching its inputs (well past the 256 MB Infinity Cache).
constexpr uint64_t NT_STREAM_BYTES = 512ull << 20;
// Load hints of a group streaming `bytes` per pass: 0 both inputs cached,
// 1 both non-temporal, 2 prev non-temporal and curr cached.  The last is for
// batches whose jobs share snapshots (time-ordered pairs): a pair's prev was
// the previous pair's curr and is read for the last time, while its curr is
// read again by the next pair.
inline uint32_t stream_nt_for(uint32_t mode, uint64_t bytes, bool shared_inputs) {
  if (mode == 1) return 1u;
  if (mode == 2) return 0u;
  if (bytes < NT_STREAM_BYTES) return 0u;
  return shared_inputs ? 2u : 1u;
}

// Pairs of one time chain in the range pass, at most (longer chains are cut).
constexpr uint32_t CHAIN_MAX = 64;
// 16-byte vectors per thread per step of a time chain's sweep.
constexpr uint32_t CHAIN_K = 4;
// Streaming chunk of a time chain of `pairs` pairs over `vecs` vectors per
// snapshot: about four chunks per compute unit, a power of two from one
// sweep step of a workgroup (CHAIN_K * 256 vectors) to 65536.
inline uint32_t chain_chunk_vec(uint64_t vecs, int cus) {
  const uint64_t want = vecs / (4 * (uint64_t)(cus > 0 ? cus : 1));
  uint32_t c = CHAIN_K * 256;
  while (c < 65536 && (uint64_t)c * 2 <= want) c *= 2;
  return c;
}

// Streaming chunk of a launch group moving `vecs` 16-byte vectors per pass:
// `fixed` when the tuning sets one, else about four chunks per compute unit
// (a power of two in [4096, 65536]): long chunks keep a workgroup on one
// contiguous stretch of each array, enough of them keep every workgroup busy.
inline uint32_t chunk_vec_for(uint32_t fixed, uint64_t vecs, int cus) {
  if (fixed) return fixed;
  const uint64_t want = vecs / ((uint64_t)cus * 4);
  uint32_t c = 4096;
  while (c < 65536 && (uint64_t)c * 2 <= want) c *= 2;
  return c;
}

// Elements of one encoder / decoder wave tile for an element size (16-byte vectors).
inline uint64_t enc_wave_tile(uint64_t elem_bytes) { return ENC_ROUNDS * 64 * (16 / elem_bytes); }

// Window codes of the precoded encoding, one 16-bit word per point: a valid
// point inside the histogram window holds its window place w (bits 0-13,
// WIN = 2^14) and, in bit 14, whether the reconstruction from its own bin's
// centre passes the error check of Sec. III-C (the check the encoder makes
// when that bin is selected); an invalid point holds WC_INVALID, a valid
// point outside the window WC_TAIL.
constexpr uint16_t WC_OK = 0x4000;
constexpr uint16_t WC_INVALID = 0x8000;
constexpr uint16_t WC_TAIL = 0xC000;
static_assert(WIN == 1 << 14, "window places fit 14 bits");
// Rounds of 8 codes (one 16-byte load) per lane in a precoded encoder tile.
constexpr int PRE_ROUNDS = 2;
constexpr uint64_t PRE_WAVE_TILE = PRE_ROUNDS * 64 * 8;
inline uint64_t dec_wave_tile(uint64_t elem_bytes) { return DEC_ROUNDS * 64 * (16 / elem_bytes); }
// Units (waves) of a range-partitioned pass over `tiles` wave tiles, at most
// `resident` (the waves that fit on the device at once); a multiple of the 4
// units of a workgroup.
inline uint32_t range_units(uint64_t tiles, int resident) {
  uint64_t u = (uint64_t)resident;
  if (u > (uint64_t)MAX_UNITS) u = MAX_UNITS;
  if (u > tiles) u = tiles;
  if (u < 1) u = 1;
  return (uint32_t)((u + 3) / 4 * 4);
}

// Kernel kinds for the optional event timing.
enum KernelKind {
  KK_INIT = 0, KK_RANGE, KK_DERIVE, KK_HIST, KK_HCLEAR, KK_HINSERT, KK_SELECT,
  KK_TAILRANK, KK_ENCODE, KK_USCAN, KK_GATHER, KK_DCOUNT, KK_DSCAN, KK_DECODE, KK_EXPORT,
  KK_COUNT
};
void timing_begin(KernelKind k, hipStream_t s);
void timing_end(KernelKind k, hipStream_t s);

// Launch wrappers (compress_kernels.hip / decompress_kernels.hip).  Each
// returns the hipError_t of the launch.
hipError_t launch_compress(const CParams& p, const Tuning& tn, hipStream_t s);
// A batch: the job table and prefix arrays live in device memory; groups are
// contiguous runs of jobs sorted by (dtype, class).
struct BatchLaunch {
  const CParams* jobs_dev;
  const uint64_t* chunk0_dev;
  const uint32_t* unit0_dev;
  uint32_t njobs;
  const JobGroup* dgroups;  // by dtype
  uint32_t n_dgroups;
  const JobGroup* egroups;  // by (dtype, class)
  uint32_t n_egroups;
  const JobGroup* rgroups;  // range pass: runs of unchained jobs and time chains
  uint32_t n_rgroups;
  const JobGroup* hgroups;  // histogram pass: the same runs and chains
  uint32_t n_hgroups;
  Tuning tune;
  uint32_t za;  // 1: bins anchored at -E (no range pass)
};
hipError_t launch_compress_batch(const BatchLaunch& b, hipStream_t s);
// One compression in two halves around the choice of B: phase 1 runs the
// passes that do not depend on B (ratios, range, histogram, tail hash),
// phase 2 the rest; launch_autob estimates the size of every B in
// [b_lo, b_hi] from phase 1's histogram (eqs. 5-6) into the control block.
hipError_t launch_compress_phase(const CParams& P, const Tuning& tn, hipStream_t s,
                                 unsigned phases);
hipError_t launch_autob(const CParams& P, uint32_t b_lo, uint32_t b_hi, hipStream_t s);
// Lossless stage of an index table (lossless_kernels.hip).
struct LLParams {
  const uint32_t* packed;  // the B-bit index table
  uint64_t n, n_sub;
  uint32_t B;
  uint32_t* counts;        // workspace: 2^B code counts
  uint32_t* rank_of;       // workspace: 2^B ranks
  unsigned long long* bits_k;  // workspace: 17 totals
  uint32_t* order;         // workspace: the chosen order k
  uint64_t* parts;         // workspace: per-tile totals of the offset scan
  uint16_t* code_of_rank;  // out: 2^B
  uint64_t* sub_off;       // out: n_sub + 1 bit offsets
  uint32_t* stream;        // out
  numarck_lossless_header* hdr;  // out (device)
};
struct LLDecodeParams {
  uint64_t n, n_sub, stream_words;
  uint64_t s_begin, s_end;  // the sub-blocks to decode
  uint32_t B, k;
  const uint16_t* code_of_rank;
  const uint64_t* sub_off;
  const uint32_t* stream;
  uint32_t* packed;        // out: the B-bit index table
  uint32_t* flags;         // out: NUMARCK_FLAG_BAD_STREAM
};
hipError_t launch_lossless_encode(const LLParams& p, hipStream_t s);
hipError_t launch_lossless_decode(const LLDecodeParams& p, hipStream_t s);
constexpr uint64_t LL_SUB_CODES = 1024;
constexpr uint64_t LL_GROUP_CODES = 128;

// One compression with the fine bins anchored at -E (centred on multiples of
// 2E): no range pass; histogram, top-k and the rest as launch_compress.
hipError_t launch_compress_za(const CParams& P, const Tuning& tn, hipStream_t s);
// One compression with equal-width binning (Sec. III-B, IV-B-3): the range
// pass, the chunk width and centres, then the same index/pack/gather passes.
hipError_t launch_compress_ew(const CParams& P, const Tuning& tn, hipStream_t s);
// Resident workgroups per CU of one encoder specialisation (for sizing units).
int encoder_occupancy(int dtype, int cls, bool table);
int encoder_pre_occupancy(int dtype, int cls, bool table);
// Streaming chunks of a job (0 for an empty job, at least 1 otherwise).
uint64_t stream_chunks(uint64_t n, int dtype, uint32_t chunk_vec);
hipError_t launch_decompress(const DParams& p, hipStream_t s);
// Reference read / write / copy kernels (numarck_stream_kernel).
hipError_t launch_stream(int kind, const void* src, void* dst, uint64_t bytes, unsigned per_cu,
                         hipStream_t s);
hipError_t launch_histogram_export(Ctl* ctl, const uint32_t* gwin, const uint32_t* hslot,
                                   const uint32_t* hcnt, const int64_t* tail, int64_t* ids,
                                   uint32_t* counts, uint64_t capacity, uint64_t* count_dev,
                                   hipStream_t s);

}  // namespace nk
