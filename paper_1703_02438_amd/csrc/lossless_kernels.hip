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
// counting the codes before it), k_llorder (bits of every order, the
// choice), k_llsub (bits of every sub-block), k_llscan (offsets and the
// header), k_llwrite.  Decode: k_llflags, k_lldecode.  The encoder's
// per-sub-block passes give each sub-block to a wave (each lane a 128-bit
// chunk of the table per round); the decoder gives each group to one lane,
// which walks its codewords in order (where a codeword starts is known only
// after the one before).
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
  // plain LDS atomics: the codes of a wave are spread over many values, and
  // aggregating the first lane's value first cost more than it saved
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
      if (on) atomicAdd(lds ? &h[c] : &p.counts[c], 1u);
    }
  }
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

// Inclusive scan of sub_off[1..n_sub] in place (one workgroup, tiles of
// LL_SCAN_TPB * LL_SCAN_PER entries, each thread LL_SCAN_PER consecutive
// ones), then the header.
__global__ void __launch_bounds__(LL_SCAN_TPB) k_llscan(LLParams p) {
  __shared__ unsigned long long s_wave[LL_SCAN_TPB / 64];
  const uint64_t ns = p.n_sub;
  const int lane = lane_id(), wave = threadIdx.x / 64;
  unsigned long long carry = 0;
  for (uint64_t t0 = 1; t0 <= ns; t0 += (uint64_t)LL_SCAN_TPB * LL_SCAN_PER) {
    const uint64_t i0 = t0 + (uint64_t)threadIdx.x * LL_SCAN_PER;
    unsigned long long v[LL_SCAN_PER];
    unsigned long long mine = 0;
#pragma unroll
    for (int u = 0; u < LL_SCAN_PER; ++u) {
      v[u] = i0 + u <= ns ? p.sub_off[i0 + u] : 0ull;
      mine += v[u];
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
    unsigned long long before = carry, total = carry;
    for (int w = 0; w < LL_SCAN_TPB / 64; ++w) {
      const unsigned long long x = s_wave[w];
      before += w < wave ? x : 0ull;
      total += x;
    }
    unsigned long long run = before + inc - mine;
#pragma unroll
    for (int u = 0; u < LL_SCAN_PER; ++u) {
      run += v[u];
      if (i0 + u <= ns) p.sub_off[i0 + u] = run;
    }
    carry = total;
    __syncthreads();
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    p.sub_off[0] = 0;
    const uint32_t k = *p.order;
    numarck_lossless_header* h = p.hdr;
    const unsigned long long total = ns ? p.sub_off[ns] : 0ull;
    h->n = p.n;
    h->n_sub = ns;
    h->stream_words = total / 32;
    h->bits = p.bits_k[k];
    h->B = p.B;
    h->k = k;
    h->flags = 0;
    h->sub_log2 = 10;
    h->group_log2 = 7;
    h->bytes = ((uint64_t)2 << p.B) + 8 * (ns + 1) + 4 * (total / 32) +
               sizeof(numarck_lossless_header);
  }
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

// Group g of sub-block s back to its B-bit codes, one lane per group.  A
// group's offsets out of order or outside its sub-block, a codeword that runs
// past its group, one of more than 33 bits, a rank of 2^B or more, or a group
// that does not end where the next one starts set the flag (the group's codes
// are then incomplete).
__global__ void __launch_bounds__(LL_TPB) k_lldecode(LLDecodeParams p) {
  __shared__ uint16_t s_code[LL_LDS_RANKS];
  const uint32_t Kt = 1u << p.B;
  const bool lds = Kt <= (uint32_t)LL_LDS_RANKS;
  if (lds) {
    for (uint32_t i = threadIdx.x; i < Kt; i += LL_TPB) s_code[i] = p.code_of_rank[i];
    __syncthreads();
  }
  const uint16_t* code_of_rank = lds ? s_code : p.code_of_rank;
  const uint64_t gi = (uint64_t)blockIdx.x * LL_TPB + threadIdx.x;
  const uint64_t s = p.s_begin + gi / LL_GROUPS;
  const uint32_t g = (uint32_t)(gi % LL_GROUPS);
  if (s >= p.s_end) return;  // no workgroup barrier below
  const uint64_t start = p.sub_off[s], end = p.sub_off[s + 1];
  if (start > end || end > p.stream_words * 32 || (start & 31) || (end & 31) ||
      end - start < LL_HEAD_BITS) {
    atomicOr(p.flags, NUMARCK_FLAG_BAD_STREAM);
    return;
  }
  // the group's bits [gs, ge): its offset, and the next group's (or the
  // sub-block's end)
  const uint64_t hw = start / 32;
  const uint32_t off = (p.stream[hw + g / 2] >> (16 * (g & 1))) & 0xFFFFu;
  const uint64_t gs = start + off;
  const uint64_t ge =
      g + 1 < LL_GROUPS ? start + ((p.stream[hw + (g + 1) / 2] >> (16 * ((g + 1) & 1))) & 0xFFFFu)
                        : end;
  if (off < LL_HEAD_BITS || gs > ge || ge > end) {
    atomicOr(p.flags, NUMARCK_FLAG_BAD_STREAM);
    return;
  }
  const uint32_t K = 1u << p.B, k = p.k, B = p.B;
  uint64_t j0 = s * LL_SUB + (uint64_t)g * LL_GROUP;
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
  bool bad = false;
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
    if (nb > 16 || q + 1 + nb > avail) {
      bad = true;
      break;
    }
    const uint32_t low = (uint32_t)(buf >> (q + 1)) & ((1u << nb) - 1u);
    buf >>= (q + 1 + nb);
    nbits -= q + 1 + nb;
    pos += q + 1 + nb;
    const uint32_t v = ((1u << nb) | low) - (1u << k);
    if (v >= K) {
      bad = true;
      break;
    }
    ob |= (unsigned long long)code_of_rank[v] << on;
    on += B;
    if (on >= 32) {
      put_word((uint32_t)ob);
      ob >>= 32;
      on -= 32;
    }
  }
  if (bad || (g + 1 < LL_GROUPS && pos != ge)) {
    atomicOr(p.flags, NUMARCK_FLAG_BAD_STREAM);
    return;
  }
  if (oc > 0) p.packed[ow] = o0;
  if (oc > 1) p.packed[ow + 1] = o1;
  if (oc > 2) p.packed[ow + 2] = o2;
  if (on) p.packed[ow + oc] = (uint32_t)ob;
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
  LL_LAUNCH(k_llclear, kb, LL_TPB, p);
  if (p.n) {
    const uint64_t chunks = ((p.n * p.B + 31) / 32 + 3) / 4;
    uint64_t hb = (chunks + LL_TPB - 1) / LL_TPB;
    const uint64_t cap = (uint64_t)geometry().cus * 8;
    hb = hb < cap ? hb : cap;
    LL_LAUNCH(k_llhist, hb, LL_TPB, p);
  }
  LL_LAUNCH(k_llrank, kb, LL_TPB, p);
  LL_LAUNCH(k_llorder, 1, LL_ORD_TPB, p);
  const uint64_t wb = (p.n_sub + LL_TPB / 64 - 1) / (LL_TPB / 64);  // a wave per sub-block
  if (wb) LL_LAUNCH(k_llsub, wb, LL_TPB, p);
  LL_LAUNCH(k_llscan, 1, LL_SCAN_TPB, p);
  if (wb) LL_LAUNCH(k_llwrite, wb, LL_TPB, p);
  return hipSuccess;
}

hipError_t launch_lossless_decode(const LLDecodeParams& p, hipStream_t s) {
  LL_LAUNCH(k_llflags, 1, 1, p.flags);
  const uint64_t sb = ((p.s_end - p.s_begin) * LL_GROUPS + LL_TPB - 1) / LL_TPB;
  if (sb) LL_LAUNCH(k_lldecode, sb, LL_TPB, p);
  return hipSuccess;
}

}  // namespace nk
