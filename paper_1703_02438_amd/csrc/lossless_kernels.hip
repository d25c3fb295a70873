// lossless_kernels.hip -- lossless stage of the index table.
//
// The paper passes each block of the index table through ZLIB (Sec. IV-C,
// V-A).  Here a prefix code without a tree takes its place, so that every
// step is a data-parallel pass:
//   - the 2^B codes are ranked by how often they occur (more often first,
//     equal counts by the smaller code);
//   - a rank v is written as an exponential-Golomb codeword of order k: with
//     x = v + 2^k and nb = floor(log2 x), nb - k zero bits, a one bit, then
//     the low nb bits of x least significant first (2 nb - k + 1 bits);
//   - k in [0, B] is the order with the fewest bits in total (the smaller k on
//     equal totals);
//   - sub-blocks of LL_SUB codes start on 32-bit words (the previous one is
//     padded with zeros), and sub_off[s] is the first bit of sub-block s, so
//     any sub-block decodes on its own;
//   - a sub-block opens with LL_GROUPS 16-bit offsets: the first bit of each
//     group of LL_GROUP consecutive codes relative to the sub-block's (an
//     empty group past n: where the codewords end); the codewords follow
//     without gaps, so any group decodes on its own too.
// Bits are numbered least significant first in little-endian 32-bit words,
// as in the index table.
//
// Encode: k_llclear, k_llhist (code counts), k_llrank (rank of every code by
// counting the codes before it), k_llorder (bits of every order, the choice;
// the two in one launch, k_llrankorder, up to 1024 codes), k_llsub (bits of
// every sub-block), k_llscan_tiles, k_llscan_parts and k_llscan_add (offsets
// and the header), k_llwrite.  Decode: k_llflags, k_lldecode.  The encoder's
// per-sub-block passes give each sub-block to a wave (each lane a 128-bit
// chunk of the table per round); the decoder gives each group to one lane,
// which walks its codewords in order (where a codeword starts is known only
// after the one before).  B = 4, 8 and 16 have kernels of their own (below).
#include "nk_device.h"

namespace nk {

constexpr int LL_SUB = (int)LL_SUB_CODES;  // codes per sub-block
constexpr int LL_GROUP = (int)LL_GROUP_CODES;  // codes per group (restart point)
constexpr int LL_GROUPS = LL_SUB / LL_GROUP;
constexpr uint32_t LL_HEAD_BITS = 16u * LL_GROUPS;  // the group offsets at a sub-block's start
constexpr int LL_TPB = 256;
constexpr int LL_LDS_BINS = 8192;   // code counts kept in LDS up to this many codes
constexpr int LL_ORD_TPB = 1024;
constexpr int LL_LDS_RANKS = 1024;  // rank / code tables kept in LDS up to this many codes (small: occupancy)
constexpr int LL_SCAN_TPB = 1024;
constexpr int LL_SCAN_PER = 4;  // offsets per thread and tile (16 was twice as slow)

__device__ __forceinline__ uint32_t ll_log2(uint32_t x) { return 31u - (uint32_t)__clz(x); }

__device__ __forceinline__ uint32_t ll_len(uint32_t v, uint32_t k) {
  return 2u * ll_log2(v + (1u << k)) - k + 1u;
}

__global__ void __launch_bounds__(LL_TPB) k_llclear(LLParams p) {
  const uint32_t K = 1u << p.B;
  const uint32_t i = blockIdx.x * LL_TPB + threadIdx.x;
  if (i < K) p.counts[i] = 0u;
  if (i < 17) p.bits_k[i] = 0ull;
}

// Code counts.  Each lane takes 128 bits of the table per step (four words,
// and the word after them for a code that runs past them) and counts the
// codes that start in those bits: a step then moves 1 KiB per wave.
__device__ __forceinline__ uint32_t ll_pick(uint32_t w0, uint32_t w1, uint32_t w2, uint32_t w3,
                                            uint32_t w4, uint32_t i) {
  return i == 0 ? w0 : i == 1 ? w1 : i == 2 ? w2 : i == 3 ? w3 : w4;
}

// The 128-bit chunk t of sub-block s: words (plus the one after, for a code
// that runs past them) and the range [a, b) of the sub-block's codes that
// start in it.
struct SubChunk {
  uint32_t w[5];
  uint32_t a, b;
  __device__ __forceinline__ void load(const uint32_t* packed, uint64_t words, uint64_t ws,
                                       uint32_t t, uint32_t ncode, uint32_t B) {
#pragma unroll
    for (int u = 0; u < 5; ++u) {
      const uint64_t i = ws + 4ull * t + u;
      w[u] = i < words ? packed[i] : 0u;
    }
    a = (t * 128u + B - 1) / B;
    b = ((t + 1) * 128u + B - 1) / B;
    a = a < ncode ? a : ncode;
    b = b < ncode ? b : ncode;
  }
  // code a + i (i < b - a)
  __device__ __forceinline__ uint32_t code(uint32_t t, uint32_t i, uint32_t B) const {
    const uint32_t off = (a + i) * B - t * 128u;  // < 128
    const uint32_t wi = off >> 5, sh = off & 31;
    const unsigned long long two =
        (unsigned long long)ll_pick(w[0], w[1], w[2], w[3], w[4], wi) |
        ((unsigned long long)ll_pick(w[0], w[1], w[2], w[3], w[4], wi + 1) << 32);
    return (uint32_t)(two >> sh) & ((1u << B) - 1u);
  }
};

__global__ void __launch_bounds__(LL_TPB) k_llhist(LLParams p) {
  __shared__ uint32_t h[LL_LDS_BINS];
  const uint32_t K = 1u << p.B, B = p.B;
  const bool lds = K <= (uint32_t)LL_LDS_BINS;
  if (lds) {
    for (uint32_t i = threadIdx.x; i < K; i += LL_TPB) h[i] = 0u;
    __syncthreads();
  }
  const uint64_t words = (p.n * B + 31) / 32;
  const uint64_t chunks = (words + 3) / 4;
  const uint32_t maxc = (128u + B - 1) / B;  // codes that can start in 128 bits
  // Each lane counts runs of equal codes and adds a run with one atomic: the
  // index table of a smooth field holds long runs (neighbouring points fall
  // in the same bin).  Aggregating the codes of a wave instead cost more
  // than it saved, since a wave's codes spread over many values.
  uint32_t last = 0, run = 0;
  uint32_t* const cnt = lds ? h : p.counts;
  for (uint64_t base = (uint64_t)blockIdx.x * LL_TPB; base < chunks;
       base += (uint64_t)gridDim.x * LL_TPB) {
    const uint64_t t = base + threadIdx.x;
    const bool live = t < chunks;
    const uint64_t w0 = t * 4;
    uint32_t w[5];
#pragma unroll
    for (int u = 0; u < 5; ++u) w[u] = live && w0 + u < words ? p.packed[w0 + u] : 0u;
    // codes j with j * B in [128 t, 128 t + 128)
    const uint64_t jlo = (t * 128 + B - 1) / B;
    for (uint32_t i = 0; i < maxc; ++i) {
      const uint64_t j = jlo + i;
      const bool on = live && j < p.n && j * B < t * 128 + 128;
      uint32_t c = 0;
      if (on) {
        const uint32_t off = (uint32_t)(j * B - t * 128);  // < 128
        const uint32_t wi = off >> 5, sh = off & 31;
        const unsigned long long two =
            (unsigned long long)ll_pick(w[0], w[1], w[2], w[3], w[4], wi) |
            ((unsigned long long)ll_pick(w[0], w[1], w[2], w[3], w[4], wi + 1) << 32);
        c = (uint32_t)(two >> sh) & (K - 1u);
      }
      if (on) {
        if (c == last) {
          ++run;
        } else {
          if (run) atomicAdd(&cnt[last], run);
          last = c;
          run = 1;
        }
      }
    }
  }
  if (run) atomicAdd(&cnt[last], run);
  if (lds) {
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < K; i += LL_TPB)
      if (h[i]) atomicAdd(&p.counts[i], h[i]);
  }
}

// rank(c) = #codes with a larger count, or the same count and a smaller code.
__global__ void __launch_bounds__(LL_TPB) k_llrank(LLParams p) {
  __shared__ uint32_t tile[LL_TPB];
  const uint32_t K = 1u << p.B;
  const uint32_t c = blockIdx.x * LL_TPB + threadIdx.x;
  const uint32_t mine = c < K ? p.counts[c] : 0u;
  uint32_t r = 0;
  for (uint32_t t0 = 0; t0 < K; t0 += LL_TPB) {
    __syncthreads();
    tile[threadIdx.x] = t0 + threadIdx.x < K ? p.counts[t0 + threadIdx.x] : 0u;
    __syncthreads();
    const uint32_t lim = K - t0 < (uint32_t)LL_TPB ? K - t0 : (uint32_t)LL_TPB;
    for (uint32_t i = 0; i < lim; ++i) {
      const uint32_t o = tile[i];
      r += (o > mine || (o == mine && t0 + i < c)) ? 1u : 0u;
    }
  }
  if (c < K) {
    p.rank_of[c] = r;
    p.code_of_rank[r] = (uint16_t)c;
  }
}

// Total bits of every order k in [0, B]; the order with the fewest.
__global__ void __launch_bounds__(LL_ORD_TPB) k_llorder(LLParams p) {
  __shared__ unsigned long long part[LL_ORD_TPB / 64][17];
  const uint32_t K = 1u << p.B;
  unsigned long long acc[17];
#pragma unroll
  for (int k = 0; k < 17; ++k) acc[k] = 0ull;
  for (uint32_t c = threadIdx.x; c < K; c += LL_ORD_TPB) {
    const uint32_t cnt = p.counts[c];
    if (!cnt) continue;
    const uint32_t r = p.rank_of[c];
#pragma unroll
    for (int k = 0; k < 17; ++k)
      if ((uint32_t)k <= p.B) acc[k] += (unsigned long long)cnt * ll_len(r, (uint32_t)k);
  }
#pragma unroll
  for (int k = 0; k < 17; ++k) {
    const unsigned long long v = wave_sum_u64(acc[k]);
    if (lane_id() == 0) part[threadIdx.x / 64][k] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t best_k = 0;
    unsigned long long best = 0;
    for (uint32_t k = 0; k <= p.B; ++k) {
      unsigned long long t = 0;
      for (int w = 0; w < LL_ORD_TPB / 64; ++w) t += part[w][k];
      p.bits_k[k] = t;
      if (k == 0 || t < best) {
        best = t;
        best_k = k;
      }
    }
    *p.order = best_k;
  }
}

// Up to LL_ORD_TPB codes (B <= 10), ranks and order in one workgroup: the
// counts in LDS; the P = LL_ORD_TPB / K consecutive threads of a code each
// count the codes ahead of it among every P-th code, and add up with
// shuffles (P is a power of two up to 64: within a wave).  Same results as
// k_llrank + k_llorder.
__global__ void __launch_bounds__(LL_ORD_TPB) k_llrankorder(LLParams p) {
  __shared__ uint32_t cnt[LL_ORD_TPB];
  __shared__ unsigned long long part[LL_ORD_TPB / 64][17];
  const uint32_t K = 1u << p.B;
  const uint32_t lP = p.B >= 10 ? 0u : 10u - p.B;  // log2 of P (LL_ORD_TPB = 1024)
  const uint32_t P = 1u << (lP < 6 ? lP : 6u);
  const uint32_t c = threadIdx.x / P, part_i = threadIdx.x % P;
  cnt[threadIdx.x] = threadIdx.x < K ? p.counts[threadIdx.x] : 0u;
  __syncthreads();
  const uint32_t mine = c < K ? cnt[c] : 0u;
  uint32_t r = 0;
#pragma unroll 4
  for (uint32_t i = part_i; i < K; i += P) {
    const uint32_t o = cnt[i];
    r += (o > mine || (o == mine && i < c)) ? 1u : 0u;
  }
  for (uint32_t o = 1; o < P; o <<= 1) r += (uint32_t)__shfl_xor((int)r, (int)o, 64);
  unsigned long long acc[17];
#pragma unroll
  for (int k = 0; k < 17; ++k) acc[k] = 0ull;
  if (c < K && part_i == 0) {
    p.rank_of[c] = r;
    p.code_of_rank[r] = (uint16_t)c;
    if (mine) {
#pragma unroll
      for (int k = 0; k < 17; ++k)
        if ((uint32_t)k <= p.B) acc[k] = (unsigned long long)mine * ll_len(r, (uint32_t)k);
    }
  }
#pragma unroll
  for (int k = 0; k < 17; ++k) {
    const unsigned long long v = wave_sum_u64(acc[k]);
    if (lane_id() == 0) part[threadIdx.x / 64][k] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t best_k = 0;
    unsigned long long best = 0;
    for (uint32_t k = 0; k <= p.B; ++k) {
      unsigned long long t = 0;
      for (int w = 0; w < LL_ORD_TPB / 64; ++w) t += part[w][k];
      p.bits_k[k] = t;
      if (k == 0 || t < best) {
        best = t;
        best_k = k;
      }
    }
    *p.order = best_k;
  }
}

// Bits of sub-block s (its group offsets and codewords), rounded up to a
// word, into sub_off[s + 1].  One wave
// per sub-block; each lane takes the codes that start in its 128-bit chunks
// of the sub-block's words (16-byte loads).
__global__ void __launch_bounds__(LL_TPB) k_llsub(LLParams p) {
  __shared__ uint32_t s_rank[LL_LDS_RANKS];
  const uint32_t K = 1u << p.B;
  const bool lds = K <= (uint32_t)LL_LDS_RANKS;
  if (lds) {
    for (uint32_t i = threadIdx.x; i < K; i += LL_TPB) s_rank[i] = p.rank_of[i];
    __syncthreads();
  }
  const uint32_t* rank_of = lds ? s_rank : p.rank_of;
  const uint64_t s = (uint64_t)blockIdx.x * (LL_TPB / 64) + threadIdx.x / 64;
  if (s >= p.n_sub) return;  // whole waves leave
  const int lane = lane_id();
  const uint32_t k = *p.order;
  const uint64_t j0 = s * LL_SUB;
  const uint64_t j1 = j0 + LL_SUB < p.n ? j0 + LL_SUB : p.n;
  const uint32_t B = p.B, ncode = (uint32_t)(j1 - j0);
  const uint64_t ws = j0 * B / 32, words = (p.n * B + 31) / 32;
  const uint32_t nch = (ncode * B + 127) / 128;
  unsigned long long bits = 0;
  for (uint32_t t = lane; t < nch; t += 64) {
    SubChunk ch;
    ch.load(p.packed, words, ws, t, ncode, B);
    for (uint32_t i = 0; i < ch.b - ch.a; ++i) bits += ll_len(rank_of[ch.code(t, i, B)], k);
  }
  bits = wave_sum_u64(bits);
  if (lane == 0) p.sub_off[s + 1] = (LL_HEAD_BITS + bits + 31) / 32 * 32;
}

// Offsets of the sub-blocks: an inclusive scan of their sizes, held in
// sub_off[1..n_sub], in three launches.  k_llscan_tiles scans tiles of
// LL_SCAN_TILE sizes in place, one workgroup each, and records each tile's
// total; k_llscan_parts turns the totals into exclusive tile offsets (one
// workgroup) and writes the header; k_llscan_add adds them to the tiles.
constexpr int LL_SCAN_TILE = LL_SCAN_TPB * LL_SCAN_PER;
// n < 2^32 codes: the tile totals fit one tile and the 1024 workspace slots
static_assert(LL_ORD_TPB == 1024, "k_llrankorder spreads 1024 threads over the codes");
static_assert((((uint64_t)1 << 32) / LL_SUB_CODES + LL_SCAN_TILE - 1) / LL_SCAN_TILE <= 1024 &&
                  1024 <= LL_SCAN_TILE,
              "tile totals of the offset scan");

// Inclusive scan of v[0..cnt) (cnt <= LL_SCAN_TILE) in place by one
// workgroup, each thread LL_SCAN_PER consecutive entries; returns the total
// to every thread.
__device__ unsigned long long ll_tile_scan(uint64_t* v, uint64_t cnt) {
  __shared__ unsigned long long s_wave[LL_SCAN_TPB / 64];
  const int lane = lane_id(), wave = threadIdx.x / 64;
  const uint64_t i0 = (uint64_t)threadIdx.x * LL_SCAN_PER;
  unsigned long long x[LL_SCAN_PER];
  unsigned long long mine = 0;
#pragma unroll
  for (int u = 0; u < LL_SCAN_PER; ++u) {
    x[u] = i0 + u < cnt ? v[i0 + u] : 0ull;
    mine += x[u];
  }
  // exclusive prefix of the thread sums over the workgroup
  unsigned long long inc = mine;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const unsigned long long t = __shfl_up(inc, o, 64);
    if (lane >= o) inc += t;
  }
  if (lane == 63) s_wave[wave] = inc;
  __syncthreads();
  unsigned long long before = 0, total = 0;
  for (int w = 0; w < LL_SCAN_TPB / 64; ++w) {
    const unsigned long long y = s_wave[w];
    before += w < wave ? y : 0ull;
    total += y;
  }
  unsigned long long run = before + inc - mine;
#pragma unroll
  for (int u = 0; u < LL_SCAN_PER; ++u) {
    run += x[u];
    if (i0 + u < cnt) v[i0 + u] = run;
  }
  return total;
}

__global__ void __launch_bounds__(LL_SCAN_TPB) k_llscan_tiles(LLParams p) {
  const uint64_t t0 = (uint64_t)blockIdx.x * LL_SCAN_TILE;
  const uint64_t cnt = p.n_sub - t0 < (uint64_t)LL_SCAN_TILE ? p.n_sub - t0 : LL_SCAN_TILE;
  const unsigned long long total = ll_tile_scan(p.sub_off + 1 + t0, cnt);
  if (threadIdx.x == 0) p.parts[blockIdx.x] = total;
}

__global__ void __launch_bounds__(LL_SCAN_TPB) k_llscan_parts(LLParams p, uint32_t ntiles) {
  // running sums of the tile totals (ntiles <= LL_SCAN_TILE)
  const unsigned long long total = ntiles ? ll_tile_scan(p.parts, ntiles) : 0ull;
  __syncthreads();
  if (threadIdx.x == 0) {
    p.sub_off[0] = 0;
    const uint32_t k = *p.order;
    numarck_lossless_header* h = p.hdr;
    h->n = p.n;
    h->n_sub = p.n_sub;
    h->stream_words = total / 32;
    h->bits = p.bits_k[k];
    h->B = p.B;
    h->k = k;
    h->flags = 0;
    h->sub_log2 = 10;
    h->group_log2 = 7;
    h->bytes = ((uint64_t)2 << p.B) + 8 * (p.n_sub + 1) + 4 * (total / 32) +
               sizeof(numarck_lossless_header);
  }
}

__global__ void __launch_bounds__(LL_SCAN_TPB) k_llscan_add(LLParams p) {
  // tile b >= 1 adds the tiles before it (parts[b] is now inclusive)
  const uint64_t t0 = (uint64_t)(blockIdx.x + 1) * LL_SCAN_TILE;
  const unsigned long long add = p.parts[blockIdx.x];
  for (uint64_t i = t0 + threadIdx.x; i < p.n_sub && i < t0 + LL_SCAN_TILE; i += LL_SCAN_TPB)
    p.sub_off[1 + i] += add;
}

// Sub-block s's codewords, from word sub_off[s] / 32 on.  One wave per
// sub-block, each lane a 128-bit chunk of the table per round: a wave prefix
// sum of the lanes' codeword bits places each lane's codewords, in order, in
// the wave's LDS copy of the sub-block's stream (ORed into at most two words
// each; ORs commute, so rounds need no ordering), and the wave stores the
// finished copy with consecutive lanes on consecutive words.
constexpr int LL_WIN = (LL_HEAD_BITS + LL_SUB * 33 + 31) / 32 + 1;  // words of the longest sub-block

__global__ void __launch_bounds__(LL_TPB) k_llwrite(LLParams p) {
  __shared__ uint32_t s_win[LL_TPB / 64][LL_WIN];
  __shared__ uint32_t s_rank[LL_LDS_RANKS];
  const uint32_t K = 1u << p.B;
  const bool lds = K <= (uint32_t)LL_LDS_RANKS;
  if (lds) {
    for (uint32_t i = threadIdx.x; i < K; i += LL_TPB) s_rank[i] = p.rank_of[i];
    __syncthreads();
  }
  const uint32_t* rank_of = lds ? s_rank : p.rank_of;
  const uint64_t s = (uint64_t)blockIdx.x * (LL_TPB / 64) + threadIdx.x / 64;
  if (s >= p.n_sub) return;  // whole waves leave; no workgroup barrier below
  const int lane = lane_id();
  uint32_t* win = s_win[threadIdx.x / 64];
  const uint32_t k = *p.order;
  const uint64_t j0 = s * LL_SUB;
  const uint64_t j1 = j0 + LL_SUB < p.n ? j0 + LL_SUB : p.n;
  const uint64_t gw = p.sub_off[s] / 32;
  const uint32_t words = (uint32_t)(p.sub_off[s + 1] / 32 - gw);  // <= LL_WIN - 1
  for (int i = lane; i < LL_WIN; i += 64) win[i] = 0u;
  wave_lds_sync();
  const uint32_t B = p.B, ncode = (uint32_t)(j1 - j0);
  const uint64_t ws = j0 * B / 32, twords = (p.n * B + 31) / 32;
  const uint32_t nch = (ncode * B + 127) / 128;
  uint32_t off = LL_HEAD_BITS;  // bits placed so far: the group offsets come first
  for (uint32_t t0 = 0; t0 < nch; t0 += 64) {
    const uint32_t t = t0 + lane;
    SubChunk ch;
    ch.a = ch.b = 0;
    if (t < nch) ch.load(p.packed, twords, ws, t, ncode, B);
    uint32_t mine = 0;
    for (uint32_t i = 0; i < ch.b - ch.a; ++i) mine += ll_len(rank_of[ch.code(t, i, B)], k);
    // inclusive prefix sum of the lanes' bits over the wave
    uint32_t inc = mine;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t v = __shfl_up(inc, o, 64);
      if (lane >= o) inc += v;
    }
    uint32_t pos = off + inc - mine;
    for (uint32_t i = 0; i < ch.b - ch.a; ++i) {
      const uint32_t c = ch.a + i;  // code within the sub-block
      if (c % LL_GROUP == 0)        // a group starts here: its offset
        atomicOr(&win[c / LL_GROUP / 2], pos << (16 * ((c / LL_GROUP) & 1)));
      const uint32_t x = rank_of[ch.code(t, i, B)] + (1u << k);
      const uint32_t nb = ll_log2(x);
      const uint32_t q = nb - k;
      const unsigned long long cw =
          (1ull << q) | ((unsigned long long)(x ^ (1u << nb)) << (q + 1));
      const uint32_t len = q + 1 + nb;
      const uint32_t w = pos >> 5, sh = pos & 31;
      atomicOr(&win[w], (uint32_t)(cw << sh));
      if (sh + len > 32) atomicOr(&win[w + 1], (uint32_t)((cw << sh) >> 32));
      pos += len;
    }
    off += __shfl(inc, 63, 64);
  }
  // groups past the table's end: the offset where the codewords end
  if (lane < LL_GROUPS && (uint32_t)lane * LL_GROUP >= ncode)
    atomicOr(&win[lane / 2], off << (16 * (lane & 1)));
  wave_lds_sync();
  for (uint32_t i = lane; i < words; i += 64) p.stream[gw + i] = win[i];
}

__global__ void k_llflags(uint32_t* flags) { *flags = 0u; }

// Decoding gives each group to one lane.  A group's offsets out of order or
// outside its sub-block, a codeword that runs past its group, one of more
// than 33 bits, a rank of 2^B or more, or a group that does not end where the
// next one starts set the flag (the group's codes are then incomplete).

// Group g of sub-block s and its bits [gs, ge): its offset, and the next
// group's (or the sub-block's end).  1: decode it; 0: past the sub-blocks
// asked for; -1: a malformed sub-block or group table (flag set).
struct LLGroup {
  uint64_t s, gs, ge;
  uint32_t g;
};
__device__ __forceinline__ int ll_group_of(const LLDecodeParams& p, LLGroup& G) {
  const uint64_t gi = (uint64_t)blockIdx.x * LL_TPB + threadIdx.x;
  G.s = p.s_begin + gi / LL_GROUPS;
  G.g = (uint32_t)(gi % LL_GROUPS);
  if (G.s >= p.s_end) return 0;
  const uint64_t start = p.sub_off[G.s], end = p.sub_off[G.s + 1];
  if (start > end || end > p.stream_words * 32 || (start & 31) || (end & 31) ||
      end - start < LL_HEAD_BITS) {
    atomicOr(p.flags, NUMARCK_FLAG_BAD_STREAM);
    return -1;
  }
  const uint32_t g = G.g;
  const uint64_t hw = start / 32;
  const uint32_t off = (p.stream[hw + g / 2] >> (16 * (g & 1))) & 0xFFFFu;
  G.gs = start + off;
  G.ge = g + 1 < LL_GROUPS
             ? start + ((p.stream[hw + (g + 1) / 2] >> (16 * ((g + 1) & 1))) & 0xFFFFu)
             : end;
  if (off < LL_HEAD_BITS || G.gs > G.ge || G.ge > end) {
    atomicOr(p.flags, NUMARCK_FLAG_BAD_STREAM);
    return -1;
  }
  return 1;
}

// Any B and any group (also the table's last, short one): true if malformed.
__device__ bool ll_decode_group(const LLDecodeParams& p, const uint16_t* code_of_rank,
                                const LLGroup& G) {
  const uint32_t K = 1u << p.B, k = p.k, B = p.B;
  const uint64_t gs = G.gs, ge = G.ge;
  uint64_t j0 = G.s * LL_SUB + (uint64_t)G.g * LL_GROUP;
  uint64_t j1 = j0 + LL_GROUP;
  j0 = j0 < p.n ? j0 : p.n;
  j1 = j1 < p.n ? j1 : p.n;
  // bits from gs on, 32 at a time into a 64-bit buffer; `pos` is the
  // absolute position of the buffer's first bit
  uint64_t iw = gs / 32;
  const uint64_t ew = (ge + 31) / 32;
  uint64_t pos = gs;
  unsigned long long buf = 0;
  uint32_t nbits = 0;
  if (iw < ew) {
    buf = p.stream[iw] >> (gs & 31);
    nbits = 32 - (uint32_t)(gs & 31);
    ++iw;
  }
  // the group's codes are 4B whole words of the table (128 codes of B bits),
  // written 16 bytes at a time
  uint64_t ow = j0 * B / 32;
  unsigned long long ob = 0;
  uint32_t on = 0, o0 = 0, o1 = 0, o2 = 0, o3 = 0, oc = 0;
  auto put_word = [&](uint32_t w) {
    o0 = oc == 0 ? w : o0;
    o1 = oc == 1 ? w : o1;
    o2 = oc == 2 ? w : o2;
    o3 = oc == 3 ? w : o3;
    if (++oc == 4) {
      *reinterpret_cast<uint4*>(p.packed + ow) = make_uint4(o0, o1, o2, o3);
      ow += 4;
      oc = 0;
    }
  };
  for (uint64_t j = j0; j < j1; ++j) {
    while (nbits <= 32 && iw < ew) {
      buf |= (unsigned long long)p.stream[iw] << nbits;
      nbits += 32;
      ++iw;
    }
    const uint64_t left = ge - pos;  // bits of the group not yet taken
    const uint32_t avail = (uint64_t)nbits < left ? nbits : (uint32_t)left;
    const unsigned long long live = avail >= 64 ? buf : (buf & ((1ull << avail) - 1ull));
    const uint32_t q = live ? (uint32_t)__builtin_ctzll(live) : 64u;
    const uint32_t nb = q + k;
    if (nb > 16 || q + 1 + nb > avail) return true;
    const uint32_t low = (uint32_t)(buf >> (q + 1)) & ((1u << nb) - 1u);
    buf >>= (q + 1 + nb);
    nbits -= q + 1 + nb;
    pos += q + 1 + nb;
    const uint32_t v = ((1u << nb) | low) - (1u << k);
    if (v >= K) return true;
    ob |= (unsigned long long)code_of_rank[v] << on;
    on += B;
    if (on >= 32) {
      put_word((uint32_t)ob);
      ob >>= 32;
      on -= 32;
    }
  }
  if (G.g + 1 < LL_GROUPS && pos != ge) return true;
  if (oc > 0) p.packed[ow] = o0;
  if (oc > 1) p.packed[ow + 1] = o1;
  if (oc > 2) p.packed[ow + 2] = o2;
  if (on) p.packed[ow + oc] = (uint32_t)ob;
  return false;
}

__global__ void __launch_bounds__(LL_TPB) k_lldecode(LLDecodeParams p) {
  __shared__ uint16_t s_code[LL_LDS_RANKS];
  const uint32_t Kt = 1u << p.B;
  const bool lds = Kt <= (uint32_t)LL_LDS_RANKS;
  if (lds) {
    for (uint32_t i = threadIdx.x; i < Kt; i += LL_TPB) s_code[i] = p.code_of_rank[i];
    __syncthreads();
  }
  LLGroup G;
  if (ll_group_of(p, G) <= 0) return;  // no workgroup barrier below
  if (ll_decode_group(p, lds ? s_code : p.code_of_rank, G))
    atomicOr(p.flags, NUMARCK_FLAG_BAD_STREAM);
}

// ---- Word-aligned codes: B = 4, 8 or 16 ----
// No code straddles a 32-bit word, so a 16-byte vector of the table (the
// table starting on a 16-byte boundary) holds VC = 128 / B whole codes,
// unpacked with constant shifts.  The kernels below give the same results as
// the ones above with a fraction of their instructions:
//   - counts: each lane adds into one of LL_HCOPIES copies of the counts in
//     LDS, the copies one bank apart, so the many lanes of a wave that hold
//     the same code (neighbouring points fall in the same bins) meet in
//     different banks;
//   - sizes and writing: the codeword and length of every code come from
//     tables in LDS; each lane assembles its codewords in a 64-bit register
//     and ORs whole words into the wave's LDS copy of the stream;
//   - decoding: the next stream word is loaded one word ahead, and a group's
//     codes are put together a 16-byte vector at a time.
constexpr int LL_HCOPIES = 16;

template <int BT>
struct LLWa {
  static constexpr uint32_t K = 1u << BT;
  static constexpr int CPW = 32 / BT;             // codes per word
  static constexpr int VC = 4 * CPW;              // codes per vector
  static constexpr int SUBV = LL_SUB / VC;        // vectors per sub-block
  static constexpr int GRPV = LL_GROUP / VC;      // vectors per group
  static_assert(32 % BT == 0 && LL_GROUP % VC == 0, "word-aligned codes");
  __device__ static __forceinline__ uint32_t code(const nk_u32x4& v, int i) {
    return (v[i / CPW] >> ((i % CPW) * BT)) & (K - 1u);
  }
  // code i (< 4 CPW) of the vector at word w0, for a vector that runs past
  // the table: only its words below `words` are read
  __device__ static __forceinline__ uint32_t code_guarded(const uint32_t* tab, uint64_t w0,
                                                          uint64_t words, int i) {
    const uint64_t w = w0 + (uint32_t)i / CPW;
    return w < words ? (tab[w] >> (((uint32_t)i % CPW) * BT)) & (K - 1u) : 0u;
  }
};

template <int BT>
__global__ void __launch_bounds__(LL_TPB) k_llhist_wa(LLParams p) {
  using W = LLWa<BT>;
  constexpr bool LDS = W::K <= 256;
  constexpr uint32_t STRIDE = W::K + 1;
  __shared__ uint32_t h[LDS ? LL_HCOPIES * STRIDE : 1];
  if constexpr (LDS) {
    for (uint32_t i = threadIdx.x; i < LL_HCOPIES * STRIDE; i += LL_TPB) h[i] = 0u;
    __syncthreads();
  }
  uint32_t* const cnt = LDS ? h + (threadIdx.x % LL_HCOPIES) * STRIDE : p.counts;
  const uint64_t nv = (p.n + W::VC - 1) / W::VC;  // vectors holding codes
  const uint64_t nfull = p.n / W::VC;             // vectors of VC codes below n
  const uint64_t words = (p.n * BT + 31) / 32;
  const nk_u32x4* tab = reinterpret_cast<const nk_u32x4*>(p.packed);
  for (uint64_t t = (uint64_t)blockIdx.x * LL_TPB + threadIdx.x; t < nv;
       t += (uint64_t)gridDim.x * LL_TPB) {
    if (t < nfull) {
      const nk_u32x4 v = gload(tab + t);
#pragma unroll
      for (int i = 0; i < W::VC; ++i) atomicAdd(&cnt[W::code(v, i)], 1u);
    } else {
      const uint32_t left = (uint32_t)(p.n - t * W::VC);  // < VC
      for (uint32_t i = 0; i < left; ++i)
        atomicAdd(&cnt[W::code_guarded(p.packed, t * 4, words, (int)i)], 1u);
    }
  }
  if constexpr (LDS) {
    __syncthreads();
    for (uint32_t c = threadIdx.x; c < W::K; c += LL_TPB) {
      uint32_t sum = 0;
#pragma unroll
      for (int j = 0; j < LL_HCOPIES; ++j) sum += h[j * STRIDE + c];
      if (sum) atomicAdd(&p.counts[c], sum);
    }
  }
}

// Sub-block s's vector t: the codes in it below the sub-block's end (nc of
// them; 0 past it), the vector itself, or the guarded words of a short one.
template <int BT>
__device__ __forceinline__ nk_u32x4 ll_wa_vector(const LLParams& p, uint64_t s, uint32_t t,
                                                 uint32_t ncode, uint32_t& nc) {
  using W = LLWa<BT>;
  const uint32_t c0 = t * W::VC;
  nc = c0 < ncode ? (ncode - c0 < (uint32_t)W::VC ? ncode - c0 : (uint32_t)W::VC) : 0u;
  nk_u32x4 v = {0u, 0u, 0u, 0u};
  const uint64_t vi = s * W::SUBV + t;
  if (nc == (uint32_t)W::VC) {
    v = gload(reinterpret_cast<const nk_u32x4*>(p.packed) + vi);
  } else if (nc) {
    const uint64_t words = (p.n * BT + 31) / 32;
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = vi * 4 + u < words ? p.packed[vi * 4 + u] : 0u;
  }
  return v;
}

// The codeword of code c under order k, least significant bit first, in
// bits [0, 33), and its length in bits [56, 62).
__device__ __forceinline__ unsigned long long ll_cw_entry(uint32_t rank, uint32_t k) {
  const uint32_t x = rank + (1u << k);
  const uint32_t nb = ll_log2(x);
  const uint32_t q = nb - k;
  const unsigned long long cw = (1ull << q) | ((unsigned long long)(x ^ (1u << nb)) << (q + 1));
  return cw | ((unsigned long long)(q + 1 + nb) << 56);
}
constexpr unsigned long long LL_CW_MASK = (1ull << 40) - 1ull;

template <int BT>
__global__ void __launch_bounds__(LL_TPB) k_llsub_wa(LLParams p) {
  using W = LLWa<BT>;
  constexpr bool LDS = W::K <= (uint32_t)LL_LDS_RANKS;
  __shared__ uint8_t s_len[LDS ? W::K : 1];  // codeword length of every code
  const uint32_t k = *p.order;
  if constexpr (LDS) {
    for (uint32_t c = threadIdx.x; c < W::K; c += LL_TPB) s_len[c] = (uint8_t)ll_len(p.rank_of[c], k);
    __syncthreads();
  }
  const uint64_t s = (uint64_t)blockIdx.x * (LL_TPB / 64) + threadIdx.x / 64;
  if (s >= p.n_sub) return;  // whole waves leave
  const int lane = lane_id();
  const uint64_t j0 = s * LL_SUB;
  const uint32_t ncode = (uint32_t)(p.n - j0 < (uint64_t)LL_SUB ? p.n - j0 : LL_SUB);
  uint32_t bits = 0;  // at most 33 per code
  for (uint32_t t = lane; t < (uint32_t)W::SUBV; t += 64) {
    uint32_t nc;
    const nk_u32x4 v = ll_wa_vector<BT>(p, s, t, ncode, nc);
    // every lookup unconditional (a code is below K): the loads go out
    // together and the lengths past nc are masked
    uint32_t len[W::VC];
#pragma unroll
    for (int i = 0; i < W::VC; ++i) {
      const uint32_t c = W::code(v, i);
      if constexpr (LDS) len[i] = s_len[c];
      else len[i] = ll_len(p.rank_of[c], k);
    }
#pragma unroll
    for (int i = 0; i < W::VC; ++i) bits += (uint32_t)i < nc ? len[i] : 0u;
  }
  const unsigned long long all = wave_sum_u64(bits);
  if (lane == 0) p.sub_off[s + 1] = (LL_HEAD_BITS + all + 31) / 32 * 32;
}

template <int BT>
__global__ void __launch_bounds__(LL_TPB) k_llwrite_wa(LLParams p) {
  using W = LLWa<BT>;
  constexpr bool LDS = W::K <= (uint32_t)LL_LDS_RANKS;
  __shared__ uint32_t s_win[LL_TPB / 64][LL_WIN];
  __shared__ unsigned long long s_cw[LDS ? W::K : 1];  // ll_cw_entry of every code
  __shared__ uint8_t s_len[LDS ? W::K : 1];
  const uint32_t k = *p.order;
  if constexpr (LDS) {
    for (uint32_t c = threadIdx.x; c < W::K; c += LL_TPB) {
      const unsigned long long e = ll_cw_entry(p.rank_of[c], k);
      s_cw[c] = e;
      s_len[c] = (uint8_t)(e >> 56);
    }
    __syncthreads();
  }
  auto entry = [&](uint32_t c) -> unsigned long long {
    if constexpr (LDS) return s_cw[c];
    return ll_cw_entry(p.rank_of[c], k);
  };
  auto length = [&](uint32_t c) -> uint32_t {
    if constexpr (LDS) return s_len[c];
    return ll_len(p.rank_of[c], k);
  };
  const uint64_t s = (uint64_t)blockIdx.x * (LL_TPB / 64) + threadIdx.x / 64;
  if (s >= p.n_sub) return;  // whole waves leave; no workgroup barrier below
  const int lane = lane_id();
  uint32_t* win = s_win[threadIdx.x / 64];
  const uint64_t j0 = s * LL_SUB;
  const uint32_t ncode = (uint32_t)(p.n - j0 < (uint64_t)LL_SUB ? p.n - j0 : LL_SUB);
  const uint64_t gw = p.sub_off[s] / 32;
  const uint32_t words = (uint32_t)(p.sub_off[s + 1] / 32 - gw);  // <= LL_WIN - 1
  for (uint32_t i = lane; i < words; i += 64) win[i] = 0u;
  wave_lds_sync();
  uint32_t off = LL_HEAD_BITS;  // bits placed so far: the group offsets come first
  for (uint32_t t0 = 0; t0 < (uint32_t)W::SUBV; t0 += 64) {
    const uint32_t t = t0 + lane;
    uint32_t nc = 0;
    nk_u32x4 v = {0u, 0u, 0u, 0u};
    if (t < (uint32_t)W::SUBV) v = ll_wa_vector<BT>(p, s, t, ncode, nc);
    // the lengths of the lane's codes (every lookup unconditional: a code is
    // below K), masked past nc
    uint32_t mine = 0;
    {
      uint32_t len[W::VC];
#pragma unroll
      for (int i = 0; i < W::VC; ++i) len[i] = length(W::code(v, i));
#pragma unroll
      for (int i = 0; i < W::VC; ++i) mine += (uint32_t)i < nc ? len[i] : 0u;
    }
    // inclusive prefix sum of the lanes' bits over the wave
    uint32_t inc = mine;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(inc, o, 64);
      if (lane >= o) inc += y;
    }
    const uint32_t pos = off + inc - mine;
    const uint32_t c0 = t * W::VC;
    if (nc && c0 % LL_GROUP == 0)  // a group starts here: its offset
      atomicOr(&win[c0 / LL_GROUP / 2], pos << (16 * ((c0 / LL_GROUP) & 1)));
    // the lane's codewords, least significant first, from bit pos & 31 of
    // word pos / 32 on, gathered in a 64-bit accumulator; each word it
    // completes is ORed into the wave's copy (the first and last are shared
    // with the neighbouring lanes)
    uint32_t w = pos >> 5;
    uint32_t nacc = pos & 31;
    unsigned long long acc = 0;
#pragma unroll
    for (int i = 0; i < W::VC; ++i) {
      const unsigned long long e = (uint32_t)i < nc ? entry(W::code(v, i)) : 0ull;
      acc |= (e & LL_CW_MASK) << nacc;  // nacc < 32 and a codeword of at most 33 bits
      nacc += (uint32_t)(e >> 56);
      if (nacc >= 32) {
        atomicOr(&win[w++], (uint32_t)acc);
        acc >>= 32;
        nacc -= 32;
        if (nacc >= 32) {  // 64 bits were held
          atomicOr(&win[w++], (uint32_t)acc);
          acc >>= 32;
          nacc -= 32;
        }
      }
    }
    if (nacc > 0 && mine > 0) atomicOr(&win[w], (uint32_t)acc);
    off += __shfl(inc, 63, 64);
  }
  // groups past the table's end: the offset where the codewords end
  if (lane < LL_GROUPS && (uint32_t)lane * LL_GROUP >= ncode)
    atomicOr(&win[lane / 2], off << (16 * (lane & 1)));
  wave_lds_sync();
  for (uint32_t i = lane; i < words; i += 64) p.stream[gw + i] = win[i];
}

// A whole group of 128 codes from its bits [gs, ge), read from the wave's
// staged copy of the stream (STAGED; words from w0 on) or from the stream
// itself.  True if malformed.
template <int BT, bool STAGED>
__device__ __forceinline__ bool ll_decode_group_wa(const LLDecodeParams& p,
                                                   const uint16_t* code_of_rank,
                                                   const uint32_t* stage, uint64_t w0,
                                                   const LLGroup& G, uint64_t j0) {
  using W = LLWa<BT>;
  auto fetch = [&](uint64_t i) -> uint32_t {
    if constexpr (STAGED) return stage[i - w0];
    return gload(p.stream + i);
  };
  const uint32_t k = p.k;
  uint64_t iw = G.gs / 32;
  const uint64_t ew = (G.ge + 31) / 32;
  unsigned long long buf = 0;
  uint32_t nbits = 0;
  if (iw < ew) {
    buf = fetch(iw) >> (G.gs & 31);
    nbits = 32 - (uint32_t)(G.gs & 31);
    ++iw;
  }
  // the word after the buffer, loaded one word ahead (the last word of the
  // group again once past it: never used then)
  uint32_t nxt = iw < ew ? fetch(iw) : 0u;
  // bits of the group not yet taken; 128 codewords take at most 4224, so a
  // larger count (a malformed last offset) is kept at 2^20
  uint32_t rem = G.ge - G.gs < (1ull << 20) ? (uint32_t)(G.ge - G.gs) : (1u << 20);
  auto refill = [&]() {
    if (nbits <= 32 && iw < ew) {
      buf |= (unsigned long long)nxt << nbits;
      nbits += 32;
      ++iw;
      // unconditional, so the load lands in nxt's register with no wait
      nxt = fetch(iw < ew ? iw : iw - 1);
    }
  };
  bool bad = false;
  nk_u32x4* out = reinterpret_cast<nk_u32x4*>(p.packed) + j0 / W::VC;
  for (int vi = 0; vi < W::GRPV; ++vi) {
    nk_u32x4 o = {0u, 0u, 0u, 0u};
#pragma unroll 1
    for (int u = 0; u < 4; ++u) {
      uint32_t word = 0;
#pragma unroll
      for (int i = 0; i < W::CPW; ++i) {
        refill();
        refill();  // a codeword is up to 33 bits
        // a missing leading one shows as q = 63, then nb > 16
        const uint32_t q = (uint32_t)__builtin_ctzll(buf | 0x8000000000000000ull);
        const uint32_t nb = q + k;
        const uint32_t len = q + 1 + nb;
        const uint32_t avail = nbits < rem ? nbits : rem;
        bad |= (nb > 16) | (len > avail);
        const uint32_t nbc = nb > 16 ? 16u : nb;
        const uint32_t low = (uint32_t)((buf >> q) >> 1) & ((1u << nbc) - 1u);
        const uint32_t v = ((1u << nbc) | low) - (1u << k);
        bad |= v >= W::K;
        const uint32_t lc = len > 63 ? 63u : len;
        buf >>= lc;
        nbits -= lc;
        rem -= lc;
        word |= (uint32_t)code_of_rank[v & (W::K - 1u)] << (i * BT);
      }
      o.x = u == 0 ? word : o.x;
      o.y = u == 1 ? word : o.y;
      o.z = u == 2 ? word : o.z;
      o.w = u == 3 ? word : o.w;
    }
    if (bad) break;
    gstore(out + vi, o);
  }
  return bad || (G.g + 1 < LL_GROUPS && rem != 0);
}

// The lanes of a wave decode 64 consecutive groups, eight sub-blocks whose
// codewords are one stretch of the stream: the wave first copies that
// stretch into LDS with coalesced loads (when it fits and its offsets are in
// order), so the lanes' word-by-word reads, each in a different place, stay
// on chip.  Read straight from the stream, those scattered reads pulled whole
// cache lines from HBM again and again.
template <int BT>
__global__ void __launch_bounds__(LL_TPB) k_lldecode_wa(LLDecodeParams p) {
  using W = LLWa<BT>;
  constexpr bool LDS = W::K <= (uint32_t)LL_LDS_RANKS;
  constexpr int STAGE = BT <= 8 ? 2048 : 4096;  // words per wave
  __shared__ uint16_t s_code[LDS ? W::K : 1];
  __shared__ uint32_t s_stage[LL_TPB / 64][STAGE];
  if constexpr (LDS) {
    for (uint32_t i = threadIdx.x; i < W::K; i += LL_TPB) s_code[i] = p.code_of_rank[i];
    __syncthreads();
  }
  const uint16_t* code_of_rank = LDS ? s_code : p.code_of_rank;
  // the wave's sub-blocks [s0, s1) and their words [w0, w1)
  const uint64_t s0 = p.s_begin + ((uint64_t)blockIdx.x * LL_TPB + (threadIdx.x & ~63u)) / LL_GROUPS;
  if (s0 >= p.s_end) return;  // whole waves; no workgroup barrier below
  const uint64_t s1 = s0 + 64 / LL_GROUPS < p.s_end ? s0 + 64 / LL_GROUPS : p.s_end;
  const uint64_t b0 = p.sub_off[s0], b1 = p.sub_off[s1];
  const uint64_t w0 = b0 / 32, w1 = (b1 + 31) / 32;
  const bool fits = b0 <= b1 && w1 <= p.stream_words && w1 - w0 <= (uint64_t)STAGE;
  uint32_t* stage = s_stage[threadIdx.x / 64];
  if (fits)
    for (uint32_t i = lane_id(); i < (uint32_t)(w1 - w0); i += 64)
      stage[i] = gload(p.stream + w0 + i);
  wave_lds_sync();
  LLGroup G;
  if (ll_group_of(p, G) <= 0) return;
  const uint64_t j0 = G.s * LL_SUB + (uint64_t)G.g * LL_GROUP;
  bool bad;
  if (j0 + LL_GROUP > p.n) {  // the table's last, short group, or one past it
    bad = ll_decode_group(p, code_of_rank, G);
  } else {
    // staged only if every remaining lane's bits lie in the copy (offsets out
    // of order across sub-blocks can place a group elsewhere)
    const bool in = fits && G.gs / 32 >= w0 && (G.ge + 31) / 32 <= w1;
    if (__all(in))
      bad = ll_decode_group_wa<BT, true>(p, code_of_rank, stage, w0, G, j0);
    else
      bad = ll_decode_group_wa<BT, false>(p, code_of_rank, stage, w0, G, j0);
  }
  if (bad) atomicOr(p.flags, NUMARCK_FLAG_BAD_STREAM);
}

#define LL_LAUNCH(kern, grid, block, ...)                                     \
  do {                                                                        \
    hipLaunchKernelGGL(kern, dim3(grid), dim3(block), 0, s, __VA_ARGS__);     \
    hipError_t e_ = hipGetLastError();                                        \
    if (e_ != hipSuccess) return e_;                                          \
  } while (0)

hipError_t launch_lossless_encode(const LLParams& p, hipStream_t s) {
  const uint32_t K = 1u << p.B;
  const uint32_t kb = (K + LL_TPB - 1) / LL_TPB;
  // word-aligned codes on a 16-byte boundary take the kernels that unpack
  // them with constant shifts
  const int wa = ((uintptr_t)p.packed & 15u) == 0 && (p.B == 4 || p.B == 8 || p.B == 16)
                     ? (int)p.B
                     : 0;
  LL_LAUNCH(k_llclear, kb, LL_TPB, p);
  if (p.n) {
    const uint64_t chunks = ((p.n * p.B + 31) / 32 + 3) / 4;
    uint64_t hb = (chunks + LL_TPB - 1) / LL_TPB;
    const uint64_t cap = (uint64_t)geometry().cus * 8;
    hb = hb < cap ? hb : cap;
    switch (wa) {
      case 4: LL_LAUNCH(k_llhist_wa<4>, hb, LL_TPB, p); break;
      case 8: LL_LAUNCH(k_llhist_wa<8>, hb, LL_TPB, p); break;
      case 16: LL_LAUNCH(k_llhist_wa<16>, hb, LL_TPB, p); break;
      default: LL_LAUNCH(k_llhist, hb, LL_TPB, p);
    }
  }
  if (K <= (uint32_t)LL_ORD_TPB) {
    LL_LAUNCH(k_llrankorder, 1, LL_ORD_TPB, p);
  } else {
    LL_LAUNCH(k_llrank, kb, LL_TPB, p);
    LL_LAUNCH(k_llorder, 1, LL_ORD_TPB, p);
  }
  const uint64_t wb = (p.n_sub + LL_TPB / 64 - 1) / (LL_TPB / 64);  // a wave per sub-block
  if (wb) {
    switch (wa) {
      case 4: LL_LAUNCH(k_llsub_wa<4>, wb, LL_TPB, p); break;
      case 8: LL_LAUNCH(k_llsub_wa<8>, wb, LL_TPB, p); break;
      case 16: LL_LAUNCH(k_llsub_wa<16>, wb, LL_TPB, p); break;
      default: LL_LAUNCH(k_llsub, wb, LL_TPB, p);
    }
  }
  const uint32_t ntiles = (uint32_t)((p.n_sub + LL_SCAN_TILE - 1) / LL_SCAN_TILE);
  if (ntiles) LL_LAUNCH(k_llscan_tiles, ntiles, LL_SCAN_TPB, p);
  LL_LAUNCH(k_llscan_parts, 1, LL_SCAN_TPB, p, ntiles);
  if (ntiles > 1) LL_LAUNCH(k_llscan_add, ntiles - 1, LL_SCAN_TPB, p);
  if (wb) {
    switch (wa) {
      case 4: LL_LAUNCH(k_llwrite_wa<4>, wb, LL_TPB, p); break;
      case 8: LL_LAUNCH(k_llwrite_wa<8>, wb, LL_TPB, p); break;
      case 16: LL_LAUNCH(k_llwrite_wa<16>, wb, LL_TPB, p); break;
      default: LL_LAUNCH(k_llwrite, wb, LL_TPB, p);
    }
  }
  return hipSuccess;
}

hipError_t launch_lossless_decode(const LLDecodeParams& p, hipStream_t s) {
  LL_LAUNCH(k_llflags, 1, 1, p.flags);
  const uint64_t sb = ((p.s_end - p.s_begin) * LL_GROUPS + LL_TPB - 1) / LL_TPB;
  if (sb) {
    // the output table is 16-byte aligned (checked by the caller)
    switch (p.B == 4 || p.B == 8 || p.B == 16 ? (int)p.B : 0) {
      case 4: LL_LAUNCH(k_lldecode_wa<4>, sb, LL_TPB, p); break;
      case 8: LL_LAUNCH(k_lldecode_wa<8>, sb, LL_TPB, p); break;
      case 16: LL_LAUNCH(k_lldecode_wa<16>, sb, LL_TPB, p); break;
      default: LL_LAUNCH(k_lldecode, sb, LL_TPB, p);
    }
  }
  return hipSuccess;
}

}  // namespace nk
