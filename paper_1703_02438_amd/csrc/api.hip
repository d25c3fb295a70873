// api.hip -- C-ABI entry points of the NUMARCK library: argument validation,
// workspace layout, launch of the kernel chains, diagnostics.  The entry
// points are declared and documented in include/numarck.h.
#include <math.h>
#include <string.h>

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
  L.scratch = take((size_t)n * elem_bytes);
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

static size_t decompress_layout_bytes(uint64_t len, size_t* cnt_off) {
  (void)len;
  const size_t s = align256(sizeof(DCtl));
  if (cnt_off) *cnt_off = s;
  return s + align256((size_t)MAX_UNITS * 4);
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
    "encode", "unit_scan", "gather", "dec_init", "dec_prefix", "dec_count",
    "dec_scan", "decode", "export"};
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

numarck_status numarck_compress(const void* prev, const void* curr, uint64_t n,
                                numarck_dtype dtype, double E, uint32_t B,
                                uint64_t block_bytes, const numarck_out* out, void* ws,
                                size_t ws_bytes, void* stream) {
  if (dtype != NUMARCK_F32 && dtype != NUMARCK_F64) return NUMARCK_EDTYPE;
  if (B < 1 || B > 16) return NUMARCK_EBITS;
  if (!(E > 0.0 && E <= 1.0)) return NUMARCK_EBOUND;
  if (n >= ((uint64_t)1 << 32)) return NUMARCK_EINVAL;
  if (!out || !out->hdr || !out->centers || !ws) return NUMARCK_EINVAL;
  if (n > 0 && (!prev || !curr || !out->packed || !out->incomp || !out->block_inc_off))
    return NUMARCK_EINVAL;
  if (block_bytes == 0) block_bytes = (uint64_t)1 << 20;
  if (8 * block_bytes < B) return NUMARCK_EINVAL;
  if (!aligned16(prev) || !aligned16(curr) || !aligned16(out->recon)) return NUMARCK_EALIGN;
  if (((uintptr_t)ws & 255u) != 0) return NUMARCK_EALIGN;
  Layout L;
  const uint64_t eb = elem_bytes_of(dtype);
  if (!fit_layout(n, eb, ws_bytes, &L)) return NUMARCK_ECAPACITY;

  char* base = static_cast<char*>(ws);
  CParams P{};
  P.prev = prev;
  P.curr = curr;
  P.n = n;
  P.E = E;
  P.twoE = 2.0 * E;
  P.cap = ldexp(E, 50);
  P.inv2E = 1.0 / P.twoE;
  P.fastbin = (isfinite(P.inv2E) && P.inv2E >= 2.2250738585072014e-308) ? 1 : 0;
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
  const hipError_t e = launch_compress(P, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e);
  return NUMARCK_OK;
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

static numarck_status decompress_impl(const numarck_header* hdr, const void* prev,
                                      const uint32_t* packed, const void* centers,
                                      const void* incomp, const int64_t* block_inc_off,
                                      uint64_t start, uint64_t len, void* out, uint32_t* flags,
                                      void* ws, size_t ws_bytes, void* stream) {
  numarck_status st = check_header(hdr);
  if (st != NUMARCK_OK) return st;
  if (start > hdr->n || len > hdr->n - start) return NUMARCK_ERANGE;
  if (!flags || !ws) return NUMARCK_EINVAL;
  if (len > 0 && (!prev || !packed || !centers || !out || !block_inc_off)) return NUMARCK_EINVAL;
  if (len > 0 && hdr->n_inc > 0 && !incomp) return NUMARCK_EINVAL;
  if (((uintptr_t)ws & 255u) != 0) return NUMARCK_EALIGN;
  size_t cnt_off = 0;
  if (ws_bytes < decompress_layout_bytes(len, &cnt_off)) return NUMARCK_ECAPACITY;
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
