// api.hip -- C-ABI entry points of the NUMARCK library: argument validation,
// workspace layout, launch of the kernel chains, diagnostics.  The entry
// points are declared and documented in include/numarck.h.
#include <math.h>
#include <string.h>

#include <stdio.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "nk_internal.h"

namespace nk {

static thread_local std::string g_last_error;

static numarck_status hip_fail(hipError_t e) {
  g_last_error = hipGetErrorString(e);
  return NUMARCK_EHIP;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static uint64_t next_pow2_u64(uint64_t x) {
  uint64_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

Layout compress_layout(uint64_t n, uint64_t elem_bytes, uint64_t tail_cap) {
  Layout L{};
  if (tail_cap > n) tail_cap = n;
  L.tail_cap = tail_cap;
  L.hcap = next_pow2_u64(2 * tail_cap > 1024 ? 2 * tail_cap : 1024);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  L.ctl = take(sizeof(Ctl));
  L.gwin = take((size_t)WIN * 4);
  L.lut = take((size_t)WIN * 2);
  L.sel_tail = take((size_t)(MAX_SEL + 1) * 8);
  L.sorted_tail = take((size_t)(MAX_SEL + 1) * 8);
  L.unit_cnt = take((size_t)MAX_UNITS * 4);
  L.sink = take((size_t)SINK_SLOTS * 256);
  L.scratch = take((size_t)n * elem_bytes);
  L.wcode = take((size_t)n * 2);
  L.tail = take((size_t)tail_cap * 8);
  L.hslot = take((size_t)L.hcap * 4);
  L.hcnt = take((size_t)L.hcap * 4);
  L.total = off;
  return L;
}

// Largest tail capacity whose layout fits ws_bytes; false if none does.
static bool fit_layout(uint64_t n, uint64_t elem_bytes, size_t ws_bytes, Layout* out) {
  Layout full = compress_layout(n, elem_bytes, n);
  if (full.total <= ws_bytes) {
    *out = full;
    return true;
  }
  Layout none = compress_layout(n, elem_bytes, 0);
  if (none.total > ws_bytes) return false;
  uint64_t a = 0, b = n;  // capacity a fits, b does not
  while (b - a > 1) {
    const uint64_t m = a + (b - a) / 2;
    if (compress_layout(n, elem_bytes, m).total <= ws_bytes) a = m; else b = m;
  }
  *out = compress_layout(n, elem_bytes, a);
  return true;
}

static size_t decompress_layout_bytes(uint64_t len, size_t* cnt_off, size_t* pre_off = nullptr) {
  (void)len;
  const size_t s = align256(sizeof(DCtl));
  const size_t p = s + align256((size_t)MAX_UNITS * 4);
  if (cnt_off) *cnt_off = s;
  if (pre_off) *pre_off = p;
  return p + align256((size_t)MAX_PRE_UNITS * 4);
}

static int g_cus[128];

Geometry geometry() {
  int dev = 0;
  (void)hipGetDevice(&dev);
  if (dev < 0 || dev >= 128) dev = 0;
  if (g_cus[dev] == 0) {
    int c = 0;
    if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        c <= 0)
      c = 256;
    g_cus[dev] = c;
  }
  return Geometry{g_cus[dev]};
}

// ------------------------------------------------------------- event timing
static const char* kKindNames[KK_COUNT] = {
    "init", "range", "derive", "hist", "hash_clear", "hash_insert", "select", "tail_rank",
    "encode", "unit_scan", "gather", "dec_count", "dec_scan", "decode", "export"};
static bool g_timing = false;
struct EvPair {
  hipEvent_t a, b;
  int kind;
};
static std::vector<EvPair> g_pairs;
static std::vector<hipEvent_t> g_pool;
static hipEvent_t g_open[KK_COUNT];

static hipEvent_t get_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

void timing_begin(KernelKind k, hipStream_t s) {
  if (!g_timing) return;
  g_open[k] = get_event();
  (void)hipEventRecord(g_open[k], s);
}

void timing_end(KernelKind k, hipStream_t s) {
  if (!g_timing || !g_open[k]) return;
  hipEvent_t b = get_event();
  (void)hipEventRecord(b, s);
  g_pairs.push_back(EvPair{g_open[k], b, (int)k});
  g_open[k] = nullptr;
}

}  // namespace nk

using namespace nk;

extern "C" {

size_t numarck_packed_bytes(uint64_t n, uint32_t B) {
  return (size_t)(((n * (uint64_t)B) + 31) / 32 * 4);
}

size_t numarck_centers_bytes(uint32_t B, numarck_dtype dtype) {
  if (B < 1 || B > 16) return 0;
  if (dtype != NUMARCK_F32 && dtype != NUMARCK_F64) return 0;
  return ((size_t)1 << B) * (dtype == NUMARCK_F32 ? 4 : 8);
}

uint64_t numarck_elems_per_block(uint32_t B, uint64_t block_bytes) {
  if (B < 1 || B > 16) return 0;
  if (block_bytes == 0) block_bytes = (uint64_t)1 << 20;
  return 8 * block_bytes / B;
}

uint64_t numarck_block_count(uint64_t n, uint32_t B, uint64_t block_bytes) {
  const uint64_t epb = numarck_elems_per_block(B, block_bytes);
  if (epb == 0) return 0;
  return (n + epb - 1) / epb;
}

static uint64_t elem_bytes_of(numarck_dtype dtype) { return dtype == NUMARCK_F32 ? 4 : 8; }

size_t numarck_workspace_bytes(uint64_t n, numarck_dtype dtype, uint32_t B) {
  (void)B;
  return compress_layout(n, elem_bytes_of(dtype), n).total;
}

size_t numarck_workspace_bytes_tail(uint64_t n, numarck_dtype dtype, uint64_t tail_cap) {
  return compress_layout(n, elem_bytes_of(dtype), tail_cap).total;
}

size_t numarck_decompress_workspace_bytes(uint64_t len) {
  return decompress_layout_bytes(len, nullptr);
}

static bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

// Validate one compression's arguments (the checks every entry point makes).
static numarck_status check_job(const void* prev, const void* curr, uint64_t n,
                                numarck_dtype dtype, double E, uint32_t B,
                                uint64_t block_bytes, const numarck_out* out) {
  if (dtype != NUMARCK_F32 && dtype != NUMARCK_F64) return NUMARCK_EDTYPE;
  if (B < 1 || B > 16) return NUMARCK_EBITS;
  if (!(E > 0.0 && E <= 1.0)) return NUMARCK_EBOUND;
  if (n >= ((uint64_t)1 << 32)) return NUMARCK_EINVAL;
  if (!out || !out->hdr || !out->centers) return NUMARCK_EINVAL;
  if (n > 0 && (!prev || !curr || !out->packed || !out->incomp || !out->block_inc_off))
    return NUMARCK_EINVAL;
  if (block_bytes == 0) block_bytes = (uint64_t)1 << 20;
  if (8 * block_bytes < B) return NUMARCK_EINVAL;
  if (!aligned16(prev) || !aligned16(curr) || !aligned16(out->recon)) return NUMARCK_EALIGN;
  return NUMARCK_OK;
}

// Kernel parameters of one checked compression whose workspace slice starts
// at `base` with layout L (encoder units are set by the launcher).
static CParams make_params(const void* prev, const void* curr, uint64_t n, numarck_dtype dtype,
                           double E, uint32_t B, uint64_t block_bytes, const numarck_out* out,
                           char* base, const Layout& L) {
  if (block_bytes == 0) block_bytes = (uint64_t)1 << 20;
  const uint64_t eb = elem_bytes_of(dtype);
  CParams P{};
  P.prev = prev;
  P.curr = curr;
  P.n = n;
  P.E = E;
  P.twoE = 2.0 * E;
  P.cap = ldexp(E, 50);
  P.inv2E = 1.0 / P.twoE;
  P.B = B;
  P.k = (1u << B) - 1u;
  P.block_bytes = block_bytes;
  P.epb = 8 * block_bytes / B;
  P.n_blocks = (n + P.epb - 1) / P.epb;
  const uint64_t tile = enc_wave_tile(eb);
  P.n_tiles = (n + tile - 1) / tile;
  P.packed_words = (n * B + 31) / 32;
  P.ctl = reinterpret_cast<Ctl*>(base + L.ctl);
  P.gwin = reinterpret_cast<uint32_t*>(base + L.gwin);
  P.lut = reinterpret_cast<uint16_t*>(base + L.lut);
  P.mulB = B > 1 ? (uint32_t)((((uint64_t)1 << 32) + B - 1) / B) : 0u;  // unused for B = 1
  P.unit_cnt = reinterpret_cast<uint32_t*>(base + L.unit_cnt);
  P.scratch = base + L.scratch;
  P.wcode = reinterpret_cast<uint16_t*>(base + L.wcode);
  P.pre = 0;  // the launcher decides
  P.tile_elems = (uint32_t)tile;
  P.sink = base + L.sink;
  P.tail = reinterpret_cast<int64_t*>(base + L.tail);
  P.tail_cap = L.tail_cap;
  P.hslot = reinterpret_cast<uint32_t*>(base + L.hslot);
  P.hcnt = reinterpret_cast<uint32_t*>(base + L.hcnt);
  P.hcap = L.hcap;
  P.sel_tail = reinterpret_cast<int64_t*>(base + L.sel_tail);
  P.sorted_tail = reinterpret_cast<int64_t*>(base + L.sorted_tail);
  P.packed = out->packed;
  P.centers = out->centers;
  P.incomp = out->incomp;
  P.block_inc_off = out->block_inc_off;
  P.recon = out->recon;
  P.bin_ids = out->bin_ids;
  P.hdr = out->hdr;
  P.dtype = (int)dtype;
  return P;
}

}  // extern "C"

// ------------------------------------------------------------- tuning table
namespace nk {

static std::mutex g_tune_mu;
// recorded tunings by (dtype, floor(log2 n))
static std::map<std::pair<int, int>, Tuning> g_tune;

static int size_class(uint64_t n) {
  int c = 0;
  while (n > 1) {
    n >>= 1;
    ++c;
  }
  return c;
}

static bool tuning_valid(const Tuning& t) {
  return t.range_blocks_per_cu >= 1 && t.range_blocks_per_cu <= 64 &&
         t.hist_blocks_per_cu >= 1 && t.hist_blocks_per_cu <= 16 && t.hist_lds <= 1 &&
         (t.chunk_vec == 0 || (t.chunk_vec >= 64 && t.chunk_vec <= (1u << 20))) &&
         t.unit_pct >= 1 &&
         t.unit_pct <= 100 && t.stream_loads <= 2;
}

static Tuning to_internal(const numarck_tuning& t) {
  return Tuning{t.range_blocks_per_cu, t.hist_blocks_per_cu, t.hist_lds, t.chunk_vec,
                t.unit_pct, t.stream_loads};
}

static numarck_tuning to_public(const Tuning& t) {
  numarck_tuning o;
  o.range_blocks_per_cu = t.range_blocks_per_cu;
  o.hist_blocks_per_cu = t.hist_blocks_per_cu;
  o.hist_lds = t.hist_lds;
  o.chunk_vec = t.chunk_vec;
  o.unit_pct = t.unit_pct;
  o.stream_loads = t.stream_loads;
  return o;
}

static Tuning recorded_tuning(int dtype, uint64_t n) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune.find({dtype, size_class(n)});
  return it == g_tune.end() ? default_tuning() : it->second;
}

}  // namespace nk

extern "C" {

void numarck_tuning_default(numarck_tuning* t) {
  if (t) *t = to_public(default_tuning());
}

numarck_status numarck_compress_tuned(const void* prev, const void* curr, uint64_t n,
                                      numarck_dtype dtype, double E, uint32_t B,
                                      uint64_t block_bytes, const numarck_out* out, void* ws,
                                      size_t ws_bytes, const numarck_tuning* tune, void* stream) {
  const numarck_status st = check_job(prev, curr, n, dtype, E, B, block_bytes, out);
  if (st != NUMARCK_OK) return st;
  if (!ws) return NUMARCK_EINVAL;
  if (((uintptr_t)ws & 255u) != 0) return NUMARCK_EALIGN;
  Tuning tn = tune ? to_internal(*tune) : recorded_tuning((int)dtype, n);
  if (!tuning_valid(tn)) return NUMARCK_EINVAL;
  Layout L;
  if (!fit_layout(n, elem_bytes_of(dtype), ws_bytes, &L)) return NUMARCK_ECAPACITY;
  const CParams P = make_params(prev, curr, n, dtype, E, B, block_bytes, out,
                                static_cast<char*>(ws), L);
  const hipError_t e = launch_compress(P, tn, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e);
  return NUMARCK_OK;
}

numarck_status numarck_compress(const void* prev, const void* curr, uint64_t n,
                                numarck_dtype dtype, double E, uint32_t B,
                                uint64_t block_bytes, const numarck_out* out, void* ws,
                                size_t ws_bytes, void* stream) {
  return numarck_compress_tuned(prev, curr, n, dtype, E, B, block_bytes, out, ws, ws_bytes,
                                nullptr, stream);
}

uint64_t numarck_lossless_subblocks(uint64_t n) { return (n + LL_SUB_CODES - 1) / LL_SUB_CODES; }

size_t numarck_lossless_stream_bytes(uint64_t n, uint32_t B) {
  if (B < 1 || B > 16) return 0;
  // the codewords (order B costs at most B + 1 bits per code, the chosen
  // order no more), and per sub-block its group table (4 words) and a
  // padding word
  return 4 * ((n * (B + 1) + 31) / 32 + 5 * numarck_lossless_subblocks(n));
}

size_t numarck_lossless_workspace_bytes(uint32_t B) {
  if (B < 1 || B > 16) return 0;
  // counts and ranks, the order totals, the scan's per-tile totals (n < 2^32
  // makes at most 2^22 sub-blocks: 1024 tiles of 4096)
  return align256((size_t)8 << B) + 256 + 8 * 1024;
}

numarck_status numarck_lossless_encode(const uint32_t* packed, uint64_t n, uint32_t B,
                                       uint16_t* code_of_rank, uint64_t* sub_off,
                                       uint32_t* stream, size_t stream_bytes,
                                       numarck_lossless_header* hdr, void* ws, size_t ws_bytes,
                                       void* stream_) {
  if (B < 1 || B > 16) return NUMARCK_EBITS;
  if (n >= ((uint64_t)1 << 32) || !code_of_rank || !sub_off || !hdr || !ws ||
      (n && (!packed || !stream)))
    return NUMARCK_EINVAL;
  if (stream_bytes < numarck_lossless_stream_bytes(n, B) ||
      ws_bytes < numarck_lossless_workspace_bytes(B))
    return NUMARCK_ECAPACITY;
  char* base = static_cast<char*>(ws);
  LLParams p{};
  p.packed = packed;
  p.n = n;
  p.n_sub = numarck_lossless_subblocks(n);
  p.B = B;
  p.counts = reinterpret_cast<uint32_t*>(base);
  p.rank_of = reinterpret_cast<uint32_t*>(base + ((size_t)4 << B));
  p.bits_k = reinterpret_cast<unsigned long long*>(base + align256((size_t)8 << B));
  p.order = reinterpret_cast<uint32_t*>(base + align256((size_t)8 << B) + 17 * 8);
  p.parts = reinterpret_cast<uint64_t*>(base + align256((size_t)8 << B) + 256);
  p.code_of_rank = code_of_rank;
  p.sub_off = sub_off;
  p.stream = stream;
  p.hdr = hdr;
  const hipError_t e = launch_lossless_encode(p, static_cast<hipStream_t>(stream_));
  return e == hipSuccess ? NUMARCK_OK : hip_fail(e);
}

numarck_status numarck_lossless_decode(const numarck_lossless_header* hdr,
                                       const uint16_t* code_of_rank, const uint64_t* sub_off,
                                       const uint32_t* stream, uint32_t* packed, uint32_t* flags,
                                       void* stream_) {
  if (!hdr) return NUMARCK_EINVAL;
  return numarck_lossless_decode_range(hdr, code_of_rank, sub_off, stream, 0, hdr->n_sub, packed,
                                       flags, stream_);
}

numarck_status numarck_lossless_decode_range(const numarck_lossless_header* hdr,
                                             const uint16_t* code_of_rank,
                                             const uint64_t* sub_off, const uint32_t* stream,
                                             uint64_t sub_begin, uint64_t sub_count,
                                             uint32_t* packed, uint32_t* flags, void* stream_) {
  if (!hdr || !code_of_rank || !sub_off || !flags) return NUMARCK_EINVAL;
  if (hdr->B < 1 || hdr->B > 16) return NUMARCK_EBITS;
  if (hdr->n >= ((uint64_t)1 << 32) || hdr->k > hdr->B ||
      hdr->n_sub != numarck_lossless_subblocks(hdr->n) || (hdr->n && (!stream || !packed)))
    return NUMARCK_EINVAL;
  // the stream's layout must be this library's
  if (hdr->sub_log2 >= 32 || hdr->group_log2 >= 32 ||
      (1ull << hdr->sub_log2) != LL_SUB_CODES || (1ull << hdr->group_log2) != LL_GROUP_CODES) {
    g_last_error = "lossless stream with sub-blocks of 2^" + std::to_string(hdr->sub_log2) +
                   " codes and groups of 2^" + std::to_string(hdr->group_log2) +
                   "; this library reads 1024 and 128";
    return NUMARCK_EINVAL;
  }
  if (((uintptr_t)stream & 15u) || ((uintptr_t)packed & 15u)) return NUMARCK_EALIGN;
  if (sub_begin > hdr->n_sub || sub_count > hdr->n_sub - sub_begin) return NUMARCK_ERANGE;
  LLDecodeParams p{};
  p.n = hdr->n;
  p.n_sub = hdr->n_sub;
  p.s_begin = sub_begin;
  p.s_end = sub_begin + sub_count;
  p.stream_words = hdr->stream_words;
  p.B = hdr->B;
  p.k = hdr->k;
  p.code_of_rank = code_of_rank;
  p.sub_off = sub_off;
  p.stream = stream;
  p.packed = packed;
  p.flags = flags;
  const hipError_t e = launch_lossless_decode(p, static_cast<hipStream_t>(stream_));
  return e == hipSuccess ? NUMARCK_OK : hip_fail(e);
}

numarck_status numarck_compress_zero_anchored(const void* prev, const void* curr, uint64_t n,
                                              numarck_dtype dtype, double E, uint32_t B,
                                              uint64_t block_bytes, const numarck_out* out,
                                              void* ws, size_t ws_bytes, void* stream) {
  const numarck_status st = check_job(prev, curr, n, dtype, E, B, block_bytes, out);
  if (st != NUMARCK_OK) return st;
  if (!ws) return NUMARCK_EINVAL;
  if (((uintptr_t)ws & 255u) != 0) return NUMARCK_EALIGN;
  const Tuning tn = recorded_tuning((int)dtype, n);
  Layout L;
  if (!fit_layout(n, elem_bytes_of(dtype), ws_bytes, &L)) return NUMARCK_ECAPACITY;
  const CParams P = make_params(prev, curr, n, dtype, E, B, block_bytes, out,
                                static_cast<char*>(ws), L);
  const hipError_t e = launch_compress_za(P, tn, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? NUMARCK_OK : hip_fail(e);
}

numarck_status numarck_compress_equal_width(const void* prev, const void* curr, uint64_t n,
                                            numarck_dtype dtype, double E, uint32_t B,
                                            uint64_t block_bytes, const numarck_out* out,
                                            void* ws, size_t ws_bytes, void* stream) {
  const numarck_status st = check_job(prev, curr, n, dtype, E, B, block_bytes, out);
  if (st != NUMARCK_OK) return st;
  if (!ws) return NUMARCK_EINVAL;
  if (((uintptr_t)ws & 255u) != 0) return NUMARCK_EALIGN;
  const Tuning tn = recorded_tuning((int)dtype, n);
  Layout L;
  if (!fit_layout(n, elem_bytes_of(dtype), ws_bytes, &L)) return NUMARCK_ECAPACITY;
  const CParams P = make_params(prev, curr, n, dtype, E, B, block_bytes, out,
                                static_cast<char*>(ws), L);
  const hipError_t e = launch_compress_ew(P, tn, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? NUMARCK_OK : hip_fail(e);
}

numarck_status numarck_compress_auto(const void* prev, const void* curr, uint64_t n,
                                     numarck_dtype dtype, double E, uint32_t B_min,
                                     uint32_t B_max, uint64_t block_bytes,
                                     const numarck_out* out, void* ws, size_t ws_bytes,
                                     void* stream, uint32_t* B_out, uint64_t* est_bits) {
  if (!B_out) return NUMARCK_EINVAL;
  if (B_min < 1 || B_max > 16 || B_min > B_max) return NUMARCK_EBITS;
  numarck_status st = check_job(prev, curr, n, dtype, E, B_max, block_bytes, out);
  if (st != NUMARCK_OK) return st;
  if (!ws) return NUMARCK_EINVAL;
  if (((uintptr_t)ws & 255u) != 0) return NUMARCK_EALIGN;
  const Tuning tn = recorded_tuning((int)dtype, n);
  Layout L;
  if (!fit_layout(n, elem_bytes_of(dtype), ws_bytes, &L)) return NUMARCK_ECAPACITY;
  char* base = static_cast<char*>(ws);
  hipStream_t s = static_cast<hipStream_t>(stream);
  // the passes before top-k do not depend on B
  const CParams P1 = make_params(prev, curr, n, dtype, E, B_max, block_bytes, out, base, L);
  hipError_t e = launch_compress_phase(P1, tn, s, 1);
  if (e == hipSuccess) e = launch_autob(P1, B_min, B_max, s);
  unsigned long long bits[17] = {};
  if (e == hipSuccess)
    e = hipMemcpyAsync(bits, P1.ctl->est_bits, sizeof(bits), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e);
  // the smallest estimate, the smaller B on equal estimates
  uint32_t B = B_min;
  for (uint32_t b = B_min + 1; b <= B_max; ++b)
    if (bits[b] < bits[B]) B = b;
  *B_out = B;
  if (est_bits)
    for (int b = 0; b <= 16; ++b) est_bits[b] = bits[b];
  const CParams P2 = make_params(prev, curr, n, dtype, E, B, block_bytes, out, base, L);
  e = launch_compress_phase(P2, tn, s, 2);
  return e == hipSuccess ? NUMARCK_OK : hip_fail(e);
}

numarck_status numarck_autotune(const void* prev, const void* curr, uint64_t n,
                                numarck_dtype dtype, double E, uint32_t B, uint64_t block_bytes,
                                const numarck_out* out, void* ws, size_t ws_bytes, uint32_t reps,
                                void* stream, numarck_tuning* best) {
  if (reps < 1) reps = 1;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipEvent_t a = nullptr, b = nullptr;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)
    return hip_fail(hipGetLastError());
  numarck_status st = NUMARCK_OK;
  auto measure = [&](const Tuning& t, uint32_t nrep, float* ms) -> numarck_status {
    const numarck_tuning pt = to_public(t);
    numarck_status r = numarck_compress_tuned(prev, curr, n, dtype, E, B, block_bytes, out, ws,
                                              ws_bytes, &pt, stream);  // warm
    if (r != NUMARCK_OK) return r;
    hipError_t e = hipEventRecord(a, s);
    for (uint32_t i = 0; i < nrep && r == NUMARCK_OK && e == hipSuccess; ++i)
      r = numarck_compress_tuned(prev, curr, n, dtype, E, B, block_bytes, out, ws, ws_bytes,
                                 &pt, stream);
    if (r != NUMARCK_OK) return r;
    if (e == hipSuccess) e = hipEventRecord(b, s);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, a, b);
    if (e == hipSuccess) *ms /= (float)nrep;
    return e == hipSuccess ? NUMARCK_OK : hip_fail(e);
  };
  // coordinate descent from the defaults, one parameter family at a time
  Tuning cur = default_tuning();
  float cur_ms = 0.f;
  st = measure(cur, reps, &cur_ms);
  const uint32_t rbpc[] = {1, 2, 4, 8};
  // histogram placement: the LDS window at 1..3 workgroups per compute unit,
  // or global window counts at 4 or 8 (no 64 KB of LDS per workgroup, so
  // more workgroups; their atomics serialise on the hot bins of concentrated
  // ratio distributions, which the single timed run below drops early)
  const uint32_t hist[][2] = {{1, 1}, {1, 2}, {1, 3}, {0, 4}, {0, 8}};
  const uint32_t cvec[] = {4096, 16384, 65536, 131072};
  const uint32_t upct[] = {40, 60, 80, 100};
  const uint32_t sload[] = {1, 2};
  auto try_one = [&](const Tuning& t) {
    if (st != NUMARCK_OK) return;
    // one timed run first: a candidate more than twice as slow as the best
    // so far is dropped without its repetitions
    float ms = 0.f;
    st = measure(t, 1, &ms);
    if (st != NUMARCK_OK || ms > 2.f * cur_ms) return;
    st = measure(t, reps, &ms);
    if (st == NUMARCK_OK && ms < cur_ms) {
      cur = t;
      cur_ms = ms;
    }
  };
  for (uint32_t v : rbpc) { Tuning t = cur; t.range_blocks_per_cu = v; try_one(t); }
  for (auto& h : hist) { Tuning t = cur; t.hist_lds = h[0]; t.hist_blocks_per_cu = h[1]; try_one(t); }
  for (uint32_t v : cvec) { Tuning t = cur; t.chunk_vec = v; try_one(t); }
  for (uint32_t v : upct) { Tuning t = cur; t.unit_pct = v; try_one(t); }
  for (uint32_t v : sload) { Tuning t = cur; t.stream_loads = v; try_one(t); }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (st != NUMARCK_OK) return st;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[{(int)dtype, size_class(n)}] = cur;
  }
  if (best) *best = to_public(cur);
  return NUMARCK_OK;
}

numarck_status numarck_tuning_save(const char* path) {
  if (!path) return NUMARCK_EINVAL;
  FILE* f = fopen(path, "w");
  if (!f) {
    g_last_error = std::string("cannot write ") + path;
    return NUMARCK_EINVAL;
  }
  std::lock_guard<std::mutex> lk(g_tune_mu);
  fprintf(f, "# dtype log2n range_blocks_per_cu hist_blocks_per_cu hist_lds chunk_vec unit_pct "
             "stream_loads\n");
  for (const auto& kv : g_tune) {
    const Tuning& t = kv.second;
    fprintf(f, "%s %d %u %u %u %u %u %u\n", kv.first.first == NUMARCK_F32 ? "f32" : "f64",
            kv.first.second, t.range_blocks_per_cu, t.hist_blocks_per_cu, t.hist_lds,
            t.chunk_vec, t.unit_pct, t.stream_loads);
  }
  fclose(f);
  return NUMARCK_OK;
}

numarck_status numarck_tuning_load(const char* path) {
  if (!path) return NUMARCK_EINVAL;
  FILE* f = fopen(path, "r");
  if (!f) {
    g_last_error = std::string("cannot read ") + path;
    return NUMARCK_EINVAL;
  }
  std::map<std::pair<int, int>, Tuning> got;
  char line[256];
  numarck_status st = NUMARCK_OK;
  while (fgets(line, sizeof line, f)) {
    if (line[0] == '#' || line[0] == '\n') continue;
    char dt[8];
    int cls = 0;
    Tuning t{};
    const int got_n = sscanf(line, "%7s %d %u %u %u %u %u %u", dt, &cls, &t.range_blocks_per_cu,
                             &t.hist_blocks_per_cu, &t.hist_lds, &t.chunk_vec, &t.unit_pct,
                             &t.stream_loads);
    if (got_n == 7) t.stream_loads = 0;  // lines without the last column: automatic
    if ((got_n != 7 && got_n != 8) ||
        (strcmp(dt, "f32") != 0 && strcmp(dt, "f64") != 0) || cls < 0 || cls > 63 ||
        !tuning_valid(t)) {
      g_last_error = std::string("malformed tuning line: ") + line;
      st = NUMARCK_EINVAL;
      break;
    }
    got[{strcmp(dt, "f32") == 0 ? (int)NUMARCK_F32 : (int)NUMARCK_F64, cls}] = t;
  }
  fclose(f);
  if (st != NUMARCK_OK) return st;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (const auto& kv : got) g_tune[kv.first] = kv.second;
  return NUMARCK_OK;
}

}  // extern "C"

// ------------------------------------------------------------- batch plans
struct numarck_plan {
  uint32_t njobs;
  std::vector<CParams> table;        // sorted by (dtype, encoder class)
  std::vector<uint64_t> chunk0;      // njobs + 1
  std::vector<uint32_t> unit0;       // njobs + 1
  std::vector<nk::JobGroup> dgroups, egroups, rgroups, hgroups;
  std::vector<uint32_t> order;       // caller's index of each job of `table`
  nk::BatchLaunch bl;
  hipEvent_t uploaded = nullptr;     // the descriptor copy has completed
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace nk {

// Batch workspace: the job table, the two prefix arrays, then one
// compression layout (full tail capacity) per job.
static size_t batch_head_bytes(uint32_t njobs) {
  return align256((size_t)njobs * sizeof(CParams)) + align256((size_t)(njobs + 1) * 8) +
         align256((size_t)(njobs + 1) * 4);
}

static uint64_t job_tail_cap(const numarck_job& j) {
  return (j.tail_cap == 0 || j.tail_cap > j.n) ? j.n : j.tail_cap;
}

static size_t job_slice_bytes(const numarck_job& j) {
  return align256(compress_layout(j.n, j.dtype == NUMARCK_F32 ? 4 : 8, job_tail_cap(j)).total);
}

}  // namespace nk

extern "C" {

size_t numarck_batch_workspace_bytes(const numarck_job* jobs, uint32_t njobs) {
  if (!jobs || njobs == 0) return 0;
  size_t total = batch_head_bytes(njobs);
  for (uint32_t i = 0; i < njobs; ++i) total += job_slice_bytes(jobs[i]);
  return total;
}

static numarck_status plan_create(const numarck_job* jobs, uint32_t njobs,
                                  const numarck_tuning* tune, void* ws, size_t ws_bytes,
                                  void* stream, numarck_plan** plan_out, uint32_t za) {
  if (!plan_out) return NUMARCK_EINVAL;
  *plan_out = nullptr;
  if (!jobs || njobs == 0 || njobs > NUMARCK_MAX_JOBS || !ws) return NUMARCK_EINVAL;
  if (((uintptr_t)ws & 255u) != 0) return NUMARCK_EALIGN;
  const Tuning tn = tune ? to_internal(*tune) : default_tuning();
  if (!tuning_valid(tn)) return NUMARCK_EINVAL;
  for (uint32_t i = 0; i < njobs; ++i) {
    const numarck_job& j = jobs[i];
    const numarck_status st =
        check_job(j.prev, j.curr, j.n, j.dtype, j.E, j.B, j.block_bytes, &j.out);
    if (st != NUMARCK_OK) {
      g_last_error = "job " + std::to_string(i) + ": " + numarck_status_str(st);
      return st;
    }
  }
  if (numarck_batch_workspace_bytes(jobs, njobs) > ws_bytes) return NUMARCK_ECAPACITY;

  // order: element type, then encoder class, then the encoding (precoded
  // unless a reconstruction is asked for); each launch covers a contiguous run
  auto pre_of = [&](uint32_t i) { return tn.hist_lds && jobs[i].out.recon == nullptr ? 1 : 0; };
  std::vector<uint32_t> order(njobs);
  for (uint32_t i = 0; i < njobs; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
    const int ka = (int)jobs[a].dtype * 16 + enc_class(jobs[a].B) * 2 + pre_of(a);
    const int kb = (int)jobs[b].dtype * 16 + enc_class(jobs[b].B) * 2 + pre_of(b);
    return ka < kb;
  });

  numarck_plan* pl = new numarck_plan();
  pl->njobs = njobs;
  pl->order = order;
  pl->table.resize(njobs);
  pl->chunk0.assign(njobs + 1, 0);
  pl->unit0.assign(njobs + 1, 0);
  char* base = static_cast<char*>(ws);
  size_t off = batch_head_bytes(njobs);
  for (uint32_t r = 0; r < njobs; ++r) {
    const numarck_job& j = jobs[order[r]];
    const uint64_t eb = j.dtype == NUMARCK_F32 ? 4 : 8;
    const Layout L = compress_layout(j.n, eb, job_tail_cap(j));
    pl->table[r] = make_params(j.prev, j.curr, j.n, j.dtype, j.E, j.B, j.block_bytes, &j.out,
                               base + off, L);
    if (pre_of(order[r])) {
      CParams& P = pl->table[r];
      P.pre = 1;
      P.tile_elems = (uint32_t)PRE_WAVE_TILE;
      P.n_tiles = (P.n + PRE_WAVE_TILE - 1) / PRE_WAVE_TILE;
    }
    off += align256(L.total);
  }
  // streaming chunks: each element type's group gets its own chunk size
  const Geometry G0 = geometry();
  std::vector<uint32_t> cvec_of(njobs);
  for (uint32_t r = 0; r < njobs;) {
    uint32_t e = r + 1;
    while (e < njobs && pl->table[e].dtype == pl->table[r].dtype) ++e;
    uint64_t vecs = 0;
    for (uint32_t q = r; q < e; ++q)
      vecs += pl->table[q].n / (pl->table[q].dtype == NUMARCK_F32 ? 4 : 2);
    const uint32_t cv = chunk_vec_for(tn.chunk_vec, vecs, G0.cus);
    for (uint32_t q = r; q < e; ++q) cvec_of[q] = cv;
    r = e;
  }
  for (uint32_t r = 0; r < njobs; ++r)
    pl->chunk0[r + 1] =
        pl->chunk0[r] + stream_chunks(pl->table[r].n, pl->table[r].dtype, cvec_of[r]);

  // a snapshot read by two jobs (consecutive time pairs) is better kept in
  // the caches between its two reads than streamed past them
  bool shared_inputs = false;
  {
    std::vector<const void*> in;
    for (uint32_t i = 0; i < njobs; ++i)
      if (jobs[i].n) {
        in.push_back(jobs[i].prev);
        in.push_back(jobs[i].curr);
      }
    std::sort(in.begin(), in.end());
    for (size_t i = 1; i < in.size() && !shared_inputs; ++i) shared_inputs = in[i] == in[i - 1];
  }

  // groups, and encoder units split within each encoder group in proportion
  // to the jobs' tiles (a multiple of 4 per job, at least 4)
  const Geometry G = geometry();
  for (uint32_t r = 0; r < njobs;) {
    uint32_t e = r + 1;
    const int dt = pl->table[r].dtype, cls = enc_class(pl->table[r].B);
    const uint32_t pre = pl->table[r].pre;
    while (e < njobs && pl->table[e].dtype == dt && enc_class(pl->table[e].B) == cls &&
           pl->table[e].pre == pre)
      ++e;
    uint64_t tiles = 0;
    for (uint32_t q = r; q < e; ++q) tiles += pl->table[q].n_tiles;
    const int occ = pre ? encoder_pre_occupancy(dt, cls, true) : encoder_occupancy(dt, cls, true);
    uint64_t resident = (uint64_t)G.cus * occ * 4 * tn.unit_pct / 100;
    if (resident < 4) resident = 4;
    for (uint32_t q = r; q < e; ++q) {
      CParams& P = pl->table[q];
      const uint64_t share =
          tiles ? (resident * P.n_tiles + tiles - 1) / tiles : 1;  // ceil
      P.n_units = range_units(P.n_tiles, (int)(share < 4 ? 4 : share));
      P.tiles_per_unit = (P.n_tiles + P.n_units - 1) / P.n_units;
      pl->unit0[q + 1] = pl->unit0[q] + P.n_units;
    }
    uint64_t gbytes = 0;
    for (uint32_t q = r; q < e; ++q)
      gbytes += 2 * pl->table[q].n * (dt == NUMARCK_F32 ? 4 : 8);
    JobGroup g{};
    g.dtype = dt;
    g.cls = cls;
    g.pre = pre;
    g.nt = stream_nt_for(tn.stream_loads, gbytes, shared_inputs);
    g.chunk_vec = cvec_of[r];
    g.job_begin = r;
    g.job_end = e;
    g.c_begin = pl->chunk0[r];
    g.c_end = pl->chunk0[e];
    g.u_begin = pl->unit0[r];
    g.u_end = pl->unit0[e];
    pl->egroups.push_back(g);
    if (!pl->dgroups.empty() && pl->dgroups.back().dtype == dt) {
      pl->dgroups.back().job_end = e;
      pl->dgroups.back().c_end = g.c_end;
      pl->dgroups.back().u_end = g.u_end;
    } else {
      pl->dgroups.push_back(g);
    }
    r = e;
  }
  for (JobGroup& dg : pl->dgroups) {  // the streaming passes decide per element type
    uint64_t bytes = 0;
    for (uint32_t q = dg.job_begin; q < dg.job_end; ++q)
      bytes += 2 * pl->table[q].n * (dg.dtype == NUMARCK_F32 ? 4 : 8);
    dg.nt = stream_nt_for(tn.stream_loads, bytes, shared_inputs);
  }
  // range pass: a time chain (consecutive jobs of one n, each job's prev the
  // previous job's curr) is swept once, every snapshot read once; the other
  // jobs stream per run as in the other passes
  for (const JobGroup& dg : pl->dgroups) {
    uint32_t run = dg.job_begin, q = dg.job_begin;
    // the histogram pass takes the same runs and chains, in the batch's
    // chunk numbering
    auto hist_group = [&](uint32_t a, uint32_t b, uint32_t chain) {
      JobGroup h = dg;
      h.job_begin = a;
      h.job_end = b;
      h.c_begin = pl->chunk0[a];
      h.c_end = pl->chunk0[b];
      h.chunk_vec = cvec_of[a];
      h.chain = chain;
      pl->hgroups.push_back(h);
    };
    auto plain_run = [&](uint32_t a, uint32_t b) {
      if (a == b) return;
      JobGroup r = dg;
      r.job_begin = a;
      r.job_end = b;
      r.c_begin = pl->chunk0[a];
      r.c_end = pl->chunk0[b];
      r.chunk_vec = cvec_of[a];
      r.chain = 0;
      pl->rgroups.push_back(r);
      hist_group(a, b, 0);
    };
    while (q < dg.job_end) {
      uint32_t e = q + 1;
      while (e < dg.job_end && e - q < CHAIN_MAX && pl->table[q].n > 0 &&
             pl->table[e].n == pl->table[q].n && pl->table[e].prev == pl->table[e - 1].curr)
        ++e;
      if (e - q < 2) {
        ++q;
        continue;
      }
      plain_run(run, q);
      JobGroup r = dg;
      r.job_begin = q;
      r.job_end = e;
      const uint64_t nvec = pl->table[q].n / (dg.dtype == NUMARCK_F32 ? 4 : 2);
      r.chunk_vec = chain_chunk_vec(nvec, G.cus);
      r.c_begin = 0;
      r.c_end = stream_chunks(pl->table[q].n, dg.dtype, r.chunk_vec);
      r.chain = 1;
      // the sweep reads each snapshot once: nothing to keep in the caches
      r.nt = stream_nt_for(tn.stream_loads,
                           (uint64_t)(e - q + 1) * pl->table[q].n * (dg.dtype == NUMARCK_F32 ? 4 : 8),
                           false);
      pl->rgroups.push_back(r);
      hist_group(q, e, 1);
      run = q = e;
    }
    plain_run(run, dg.job_end);
  }
  if ((uint64_t)pl->unit0[njobs] / 4 > 0x7FFFFFFFull) {
    delete pl;
    return NUMARCK_EINVAL;
  }

  // descriptors to the workspace head
  const size_t t_off = 0;
  const size_t c_off = align256((size_t)njobs * sizeof(CParams));
  const size_t u_off = c_off + align256((size_t)(njobs + 1) * 8);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(base + t_off, pl->table.data(), njobs * sizeof(CParams),
                                hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(base + c_off, pl->chunk0.data(), (njobs + 1) * 8, hipMemcpyHostToDevice,
                       s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(base + u_off, pl->unit0.data(), (njobs + 1) * 4, hipMemcpyHostToDevice,
                       s);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&pl->uploaded, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventRecord(pl->uploaded, s);
  if (e != hipSuccess) {
    if (pl->uploaded) (void)hipEventDestroy(pl->uploaded);
    delete pl;
    return hip_fail(e);
  }
  BatchLaunch& bl = pl->bl;
  bl.jobs_dev = reinterpret_cast<const CParams*>(base + t_off);
  bl.chunk0_dev = reinterpret_cast<const uint64_t*>(base + c_off);
  bl.unit0_dev = reinterpret_cast<const uint32_t*>(base + u_off);
  bl.njobs = njobs;
  bl.dgroups = pl->dgroups.data();
  bl.n_dgroups = (uint32_t)pl->dgroups.size();
  bl.egroups = pl->egroups.data();
  bl.n_egroups = (uint32_t)pl->egroups.size();
  bl.rgroups = pl->rgroups.data();
  bl.n_rgroups = (uint32_t)pl->rgroups.size();
  bl.hgroups = pl->hgroups.data();
  bl.n_hgroups = (uint32_t)pl->hgroups.size();
  bl.tune = tn;
  bl.za = za;
  *plan_out = pl;
  return NUMARCK_OK;
}

numarck_status numarck_plan_create(const numarck_job* jobs, uint32_t njobs,
                                   const numarck_tuning* tune, void* ws, size_t ws_bytes,
                                   void* stream, numarck_plan** plan_out) {
  return plan_create(jobs, njobs, tune, ws, ws_bytes, stream, plan_out, 0);
}

numarck_status numarck_plan_create_zero_anchored(const numarck_job* jobs, uint32_t njobs,
                                                 const numarck_tuning* tune, void* ws,
                                                 size_t ws_bytes, void* stream,
                                                 numarck_plan** plan_out) {
  return plan_create(jobs, njobs, tune, ws, ws_bytes, stream, plan_out, 1);
}

uint32_t numarck_plan_groups(const numarck_plan* plan, numarck_plan_group* out, uint32_t cap) {
  if (!plan) return 0;
  uint32_t w = 0;
  auto put = [&](uint32_t pass, const JobGroup& g, uint32_t hint, uint32_t lds) {
    if (out && w < cap) {
      numarck_plan_group r{};
      r.pass = pass;
      r.dtype = (uint32_t)g.dtype;
      r.cls = pass == NUMARCK_PASS_ENCODE ? (uint32_t)g.cls : 0u;
      r.first_job = g.job_begin < plan->njobs ? plan->order[g.job_begin] : 0u;
      r.njobs = g.job_end - g.job_begin;
      r.chain = pass == NUMARCK_PASS_ENCODE ? 0u : g.chain;
      r.load_hint = hint;
      r.hist_lds = lds;
      out[w] = r;
    }
    ++w;
  };
  // the hints each pass's kernels take (run_chain): the range and LDS
  // histogram passes stream non-temporally for hint 1 only, global
  // histogram counts always read cached, the encoder takes all three
  if (!plan->bl.za)
    for (const JobGroup& g : plan->rgroups) put(NUMARCK_PASS_RANGE, g, g.nt == 1 ? 1u : 0u, 0u);
  const uint32_t lds = plan->bl.tune.hist_lds;
  for (const JobGroup& g : plan->hgroups)
    put(NUMARCK_PASS_HIST, g, (lds && g.nt == 1) ? 1u : 0u, lds);
  for (const JobGroup& g : plan->egroups) put(NUMARCK_PASS_ENCODE, g, g.nt, 0u);
  return w;
}

numarck_status numarck_plan_run(const numarck_plan* plan, void* stream) {
  if (!plan) return NUMARCK_EINVAL;
  const hipError_t e = launch_compress_batch(plan->bl, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? NUMARCK_OK : hip_fail(e);
}

numarck_status numarck_plan_capture(numarck_plan* plan, void* stream) {
  if (!plan || !stream) return NUMARCK_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (plan->exec) {
    (void)hipGraphExecDestroy(plan->exec);
    plan->exec = nullptr;
  }
  if (plan->graph) {
    (void)hipGraphDestroy(plan->graph);
    plan->graph = nullptr;
  }
  // the descriptors must be in place before the graph's first replay
  hipError_t e = hipStreamWaitEvent(s, plan->uploaded, 0);
  if (e != hipSuccess) return hip_fail(e);
  const bool timing = g_timing;
  g_timing = false;  // no event records inside the graph
  e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
  hipError_t le = hipSuccess;
  if (e == hipSuccess) {
    le = launch_compress_batch(plan->bl, s);
    e = hipStreamEndCapture(s, &plan->graph);
  }
  g_timing = timing;
  if (le != hipSuccess) e = le;
  if (e == hipSuccess) e = hipGraphInstantiate(&plan->exec, plan->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    if (plan->graph) (void)hipGraphDestroy(plan->graph);
    plan->graph = nullptr;
    plan->exec = nullptr;
    return hip_fail(e);
  }
  return NUMARCK_OK;
}

numarck_status numarck_plan_replay(const numarck_plan* plan, void* stream) {
  if (!plan || !plan->exec) return NUMARCK_EINVAL;
  const hipError_t e = hipGraphLaunch(plan->exec, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? NUMARCK_OK : hip_fail(e);
}

void numarck_plan_destroy(numarck_plan* plan) {
  if (!plan) return;
  if (plan->uploaded) {
    (void)hipEventSynchronize(plan->uploaded);  // the host tables feed the copy
    (void)hipEventDestroy(plan->uploaded);
  }
  if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
  if (plan->graph) (void)hipGraphDestroy(plan->graph);
  delete plan;
}

numarck_status numarck_plan_autotune(const numarck_job* jobs, uint32_t njobs, void* ws,
                                     size_t ws_bytes, uint32_t reps, uint32_t zero_anchored,
                                     void* stream, numarck_tuning* best) {
  if (!best) return NUMARCK_EINVAL;
  if (reps < 1) reps = 1;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipEvent_t a = nullptr, b = nullptr;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)
    return hip_fail(hipGetLastError());
  // time `nrep` runs of a plan built with tuning t (after one warm run)
  auto measure = [&](const Tuning& t, uint32_t nrep, float* ms) -> numarck_status {
    const numarck_tuning pt = to_public(t);
    numarck_plan* pl = nullptr;
    numarck_status r = plan_create(jobs, njobs, &pt, ws, ws_bytes, stream, &pl, zero_anchored);
    if (r != NUMARCK_OK) return r;
    r = numarck_plan_run(pl, stream);
    hipError_t e = r == NUMARCK_OK ? hipEventRecord(a, s) : hipSuccess;
    for (uint32_t i = 0; i < nrep && r == NUMARCK_OK && e == hipSuccess; ++i)
      r = numarck_plan_run(pl, stream);
    if (r == NUMARCK_OK && e == hipSuccess) e = hipEventRecord(b, s);
    if (r == NUMARCK_OK && e == hipSuccess) e = hipEventSynchronize(b);
    if (r == NUMARCK_OK && e == hipSuccess) e = hipEventElapsedTime(ms, a, b);
    numarck_plan_destroy(pl);
    if (r != NUMARCK_OK) return r;
    if (e != hipSuccess) return hip_fail(e);
    *ms /= (float)nrep;
    return NUMARCK_OK;
  };
  // coordinate descent from the defaults, as numarck_autotune; histogram
  // placement is where a batch of many small jobs can gain (global counts
  // need no 64 KB of LDS per workgroup), and where concentrated ratios lose
  // badly, which the single timed run drops early
  Tuning cur = default_tuning();
  float cur_ms = 0.f;
  numarck_status st = measure(cur, reps, &cur_ms);
  auto try_one = [&](const Tuning& t) {
    if (st != NUMARCK_OK) return;
    float ms = 0.f;
    st = measure(t, 1, &ms);
    if (st != NUMARCK_OK || ms > 2.f * cur_ms) return;
    st = measure(t, reps, &ms);
    if (st == NUMARCK_OK && ms < cur_ms) {
      cur = t;
      cur_ms = ms;
    }
  };
  const uint32_t rbpc[] = {1, 2, 4, 8};
  const uint32_t hist[][2] = {{1, 1}, {1, 2}, {1, 3}, {0, 4}, {0, 8}};
  const uint32_t cvec[] = {4096, 16384, 65536};
  const uint32_t upct[] = {40, 60, 80, 100};
  for (uint32_t v : rbpc) { Tuning t = cur; t.range_blocks_per_cu = v; try_one(t); }
  for (auto& h : hist) { Tuning t = cur; t.hist_lds = h[0]; t.hist_blocks_per_cu = h[1]; try_one(t); }
  for (uint32_t v : cvec) { Tuning t = cur; t.chunk_vec = v; try_one(t); }
  for (uint32_t v : upct) { Tuning t = cur; t.unit_pct = v; try_one(t); }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (st != NUMARCK_OK) return st;
  *best = to_public(cur);
  return NUMARCK_OK;
}

numarck_status numarck_compress_batch(const numarck_job* jobs, uint32_t njobs, void* ws,
                                      size_t ws_bytes, void* stream) {
  numarck_plan* pl = nullptr;
  numarck_status st = numarck_plan_create(jobs, njobs, nullptr, ws, ws_bytes, stream, &pl);
  if (st != NUMARCK_OK) return st;
  st = numarck_plan_run(pl, stream);
  numarck_plan_destroy(pl);
  return st;
}

static numarck_status check_header(const numarck_header* h) {
  if (!h) return NUMARCK_EINVAL;
  if (h->dtype != NUMARCK_F32 && h->dtype != NUMARCK_F64) return NUMARCK_EDTYPE;
  if (h->B < 1 || h->B > 16) return NUMARCK_EBITS;
  if (h->n >= ((uint64_t)1 << 32)) return NUMARCK_EINVAL;
  if (h->block_bytes == 0 || 8 * h->block_bytes < h->B) return NUMARCK_EINVAL;
  if (h->elems_per_block != 8 * h->block_bytes / h->B) return NUMARCK_EINVAL;
  if (h->n_blocks != (h->n + h->elems_per_block - 1) / h->elems_per_block) return NUMARCK_EINVAL;
  if (h->k_used > (1u << h->B) - 1u) return NUMARCK_EINVAL;
  if (h->n_inc > h->n) return NUMARCK_EINVAL;
  return NUMARCK_OK;
}

// Argument checks of a (range) decompression, the workspace aside.
static numarck_status check_decompress_args(const numarck_header* hdr, const void* prev,
                                            const uint32_t* packed, const void* centers,
                                            const void* incomp, const int64_t* block_inc_off,
                                            uint64_t start, uint64_t len, const void* out,
                                            const uint32_t* flags) {
  numarck_status st = check_header(hdr);
  if (st != NUMARCK_OK) return st;
  if (start > hdr->n || len > hdr->n - start) return NUMARCK_ERANGE;
  if (!flags) return NUMARCK_EINVAL;
  if (len > 0 && (!prev || !packed || !centers || !out || !block_inc_off)) return NUMARCK_EINVAL;
  if (len > 0 && hdr->n_inc > 0 && !incomp) return NUMARCK_EINVAL;
  return NUMARCK_OK;
}

static numarck_status decompress_impl(const numarck_header* hdr, const void* prev,
                                      const uint32_t* packed, const void* centers,
                                      const void* incomp, const int64_t* block_inc_off,
                                      uint64_t start, uint64_t len, void* out, uint32_t* flags,
                                      void* ws, size_t ws_bytes, void* stream) {
  numarck_status st = check_decompress_args(hdr, prev, packed, centers, incomp, block_inc_off,
                                            start, len, out, flags);
  if (st != NUMARCK_OK) return st;
  if (!ws) return NUMARCK_EINVAL;
  if (((uintptr_t)ws & 255u) != 0) return NUMARCK_EALIGN;
  size_t cnt_off = 0, pre_off = 0;
  if (ws_bytes < decompress_layout_bytes(len, &cnt_off, &pre_off)) return NUMARCK_ECAPACITY;
  char* base = static_cast<char*>(ws);
  DParams P{};
  P.prev = prev;
  P.packed = packed;
  P.centers = centers;
  P.incomp = incomp;
  P.block_inc_off = block_inc_off;
  P.out = out;
  P.flags = flags;
  P.n = hdr->n;
  P.start = start;
  P.len = len;
  P.n_inc = hdr->n_inc;
  P.epb = hdr->elems_per_block;
  P.packed_words = (hdr->n * hdr->B + 31) / 32;
  P.B = hdr->B;
  P.k_used = hdr->k_used;
  P.dtype = (int)hdr->dtype;
  P.dctl = reinterpret_cast<DCtl*>(base);
  P.unit_cnt = reinterpret_cast<uint32_t*>(base + cnt_off);
  P.pre_cnt = reinterpret_cast<uint32_t*>(base + pre_off);
  P.tile_elems = dec_wave_tile(hdr->dtype == NUMARCK_F32 ? 4 : 8);
  P.n_tiles = (len + P.tile_elems - 1) / P.tile_elems;
  const hipError_t e = launch_decompress(P, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e);
  return NUMARCK_OK;
}

numarck_status numarck_decompress(const numarck_header* hdr, const void* prev,
                                  const uint32_t* packed, const void* centers,
                                  const void* incomp, const int64_t* block_inc_off, void* out,
                                  uint32_t* flags, void* ws, size_t ws_bytes, void* stream) {
  if (!hdr) return NUMARCK_EINVAL;
  return decompress_impl(hdr, prev, packed, centers, incomp, block_inc_off, 0, hdr->n, out,
                         flags, ws, ws_bytes, stream);
}

numarck_status numarck_decompress_range(const numarck_header* hdr, const void* prev,
                                        const uint32_t* packed, const void* centers,
                                        const void* incomp, const int64_t* block_inc_off,
                                        uint64_t start, uint64_t len, void* out,
                                        uint32_t* flags, void* ws, size_t ws_bytes,
                                        void* stream) {
  return decompress_impl(hdr, prev, packed, centers, incomp, block_inc_off, start, len, out,
                         flags, ws, ws_bytes, stream);
}

}  // extern "C"

namespace nk {

// Workspace of numarck_decompress_range_noalloc: the decompression layout (a
// control word, the unit escape counts and the counts of the pieces before
// the range; its size does not depend on the range) in a device-global array.
// Each device holds its own copy until the process ends.  In host code the
// array's name is only a host-side stand-in: kernels get the device address
// that hipGetSymbolAddress returns on that device.
constexpr size_t NK_STATIC_SCRATCH_BYTES = 64 * 1024;
static __device__ __align__(256) unsigned char scratch[NK_STATIC_SCRATCH_BYTES];

constexpr int NK_MAX_DEVICES = 128;
static std::mutex g_scratch_mu;
static void* g_scratch_dev[NK_MAX_DEVICES];

// The current device's address of `scratch`, looked up once per device.
static numarck_status static_scratch(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e);
  if (dev < 0 || dev >= NK_MAX_DEVICES) {
    g_last_error = "device ordinal beyond the static scratch table";
    return NUMARCK_EINVAL;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e);
    if (!p) {
      g_last_error = "hipGetSymbolAddress returned no address for the static scratch";
      return NUMARCK_EHIP;
    }
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return NUMARCK_OK;
}

}  // namespace nk

extern "C" {

size_t numarck_static_scratch_bytes(void) { return NK_STATIC_SCRATCH_BYTES; }

numarck_status numarck_decompress_range_noalloc(const numarck_header* hdr, const void* prev,
                                                const uint32_t* packed, const void* centers,
                                                const void* incomp,
                                                const int64_t* block_inc_off, uint64_t start,
                                                uint64_t len, void* out, uint32_t* flags,
                                                void* stream) {
  numarck_status st = check_decompress_args(hdr, prev, packed, centers, incomp, block_inc_off,
                                            start, len, out, flags);
  if (st != NUMARCK_OK) return st;
  const size_t need = decompress_layout_bytes(len, nullptr);
  if (need > NK_STATIC_SCRATCH_BYTES) {
    g_last_error = "decompression workspace of " + std::to_string(need) +
                   " bytes exceeds the static scratch of " +
                   std::to_string(NK_STATIC_SCRATCH_BYTES);
    return NUMARCK_ECAPACITY;
  }
  void* ws = nullptr;
  st = static_scratch(&ws);
  if (st != NUMARCK_OK) return st;
  return decompress_impl(hdr, prev, packed, centers, incomp, block_inc_off, start, len, out,
                         flags, ws, NK_STATIC_SCRATCH_BYTES, stream);
}

numarck_status numarck_histogram_export(const void* ws, size_t ws_bytes, uint64_t n,
                                        numarck_dtype dtype, int64_t* ids, uint32_t* counts,
                                        uint64_t capacity, uint64_t* count_dev, void* stream) {
  if (!ws || !count_dev || (capacity > 0 && (!ids || !counts))) return NUMARCK_EINVAL;
  if (n >= ((uint64_t)1 << 32)) return NUMARCK_EINVAL;
  if (dtype != NUMARCK_F32 && dtype != NUMARCK_F64) return NUMARCK_EDTYPE;
  Layout L;
  if (!fit_layout(n, elem_bytes_of(dtype), ws_bytes, &L)) return NUMARCK_ECAPACITY;
  const char* base = static_cast<const char*>(ws);
  const hipError_t e = launch_histogram_export(
      reinterpret_cast<Ctl*>(const_cast<char*>(base) + L.ctl),
      reinterpret_cast<const uint32_t*>(base + L.gwin),
      reinterpret_cast<const uint32_t*>(base + L.hslot),
      reinterpret_cast<const uint32_t*>(base + L.hcnt),
      reinterpret_cast<const int64_t*>(base + L.tail), ids, counts, capacity, count_dev,
      static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e);
  return NUMARCK_OK;
}

const char* numarck_status_str(numarck_status s) {
  switch (s) {
    case NUMARCK_OK: return "ok";
    case NUMARCK_EINVAL: return "invalid argument";
    case NUMARCK_EDTYPE: return "unsupported dtype";
    case NUMARCK_EBITS: return "B outside [1, 16]";
    case NUMARCK_EBOUND: return "E outside (0, 1]";
    case NUMARCK_EALIGN: return "misaligned pointer";
    case NUMARCK_ECAPACITY: return "workspace too small";
    case NUMARCK_EHIP: return "HIP error";
    case NUMARCK_ERANGE: return "range outside the data";
  }
  return "unknown status";
}

const char* numarck_last_error(void) { return g_last_error.c_str(); }

numarck_status numarck_stream_kernel(int kind, const void* src, void* dst, uint64_t bytes,
                                     uint32_t per_cu, void* stream) {
  if (kind < NUMARCK_STREAM_READ || kind > NUMARCK_STREAM_READ2_WRITE8) return NUMARCK_EINVAL;
  const uint64_t unit =
      kind == NUMARCK_STREAM_READ2_WRITE16 || kind == NUMARCK_STREAM_READ2_WRITE8 ? 32 : 16;
  if (bytes % unit != 0 || per_cu < 1 || per_cu > 64 || !dst) return NUMARCK_EINVAL;
  const bool reads = kind != NUMARCK_STREAM_WRITE && kind != NUMARCK_STREAM_WRITE_NT;
  if (reads && !src) return NUMARCK_EINVAL;
  if (!aligned16(dst) || (reads && !aligned16(src))) return NUMARCK_EALIGN;
  if (bytes == 0) return NUMARCK_OK;
  const hipError_t e = launch_stream(kind, src, dst, bytes, per_cu, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? NUMARCK_OK : hip_fail(e);
}

void numarck_timing_enable(int on) { g_timing = on != 0; }

int numarck_timing_read(const char** names, uint32_t* launches, double* ms, int cap) {
  double tot[KK_COUNT] = {0};
  uint32_t cnt[KK_COUNT] = {0};
  for (const EvPair& p : g_pairs) {
    float t = 0.f;
    if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&t, p.a, p.b) == hipSuccess) {
      tot[p.kind] += t;
      cnt[p.kind] += 1;
    }
    g_pool.push_back(p.a);
    g_pool.push_back(p.b);
  }
  g_pairs.clear();
  int w = 0;
  for (int k = 0; k < KK_COUNT && w < cap; ++k) {
    if (!cnt[k]) continue;
    if (names) names[w] = kKindNames[k];
    if (launches) launches[w] = cnt[k];
    if (ms) ms[w] = tot[k];
    ++w;
  }
  return w;
}

}  // extern "C"
