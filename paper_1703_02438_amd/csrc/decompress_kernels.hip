// decompress_kernels.hip -- full and partial decompression of NUMARCK
// (arXiv 1703.02438, eq. 4 / Sec. III-E, partial decompression Sec. IV-C and
// V-C).
//
// A range [start, start + len) is cut into wave tiles; each wave ("unit")
// owns a contiguous run of them:
//   k_dcount   escapes in each unit's run, and in pieces of the part of
//              start's block before the range (reads the packed indices only)
//   k_decode   each workgroup first sums the escapes before its units (the
//              block table's count at start's block, the counted pieces
//              before start, the counts of the earlier units); then each
//              unit decodes its tiles in order: an escape takes the next
//              incompressible value, any other index gives
//              T(prev * (1 + centre[index]))
#include "nk_device.h"

namespace nk {

__device__ __forceinline__ uint32_t unpack_index(const uint32_t* __restrict__ packed, uint64_t j,
                                                 uint32_t B) {
  const uint64_t bit = j * B;
  const uint64_t w = bit >> 5;
  const uint32_t sh = (uint32_t)(bit & 31);
  uint32_t v = packed[w] >> sh;
  if (sh + B > 32) v |= packed[w + 1] << (32 - sh);
  return v & ((1u << B) - 1u);
}

constexpr int DCOUNT_GROUPS = 4;

// Escapes among the indices of [r0, r1), summed over the calling wave (every
// lane returns the total).  Reads the packed indices only.
__device__ unsigned long long wave_count_escapes(const uint32_t* __restrict__ packed,
                                                 uint64_t packed_words, uint32_t B, uint64_t r0,
                                                 uint64_t r1) {
  const int lane = lane_id();
  const uint32_t esc = (1u << B) - 1u;
  unsigned long long cnt = 0;
  if (r0 < r1 && (32 % B) == 0) {
    // B divides 32: indices never straddle words.  AND-folding a word by 1,
    // 2, 4, ... < B bit positions leaves at the first bit of each field the
    // AND of the field's B bits (1 exactly for the escape code).  Lanes take
    // 16-byte groups of four words when the stream is 16-byte aligned.
    const uint32_t per = 32 / B;
    uint32_t start_mask = 0;
    for (uint32_t b = 0; b < 32; b += B) start_mask |= 1u << b;
    const uint64_t wlo = r0 / per, whi = (r1 + per - 1) / per;  // words [wlo, whi)
    // escapes among the fields of word w that lie in [r0, r1)
    auto word_escapes = [&](uint64_t w, uint32_t x) -> uint32_t {
      for (uint32_t sh = 1; sh < B; sh <<= 1) x &= x >> sh;
      x &= start_mask;
      const uint64_t e0 = w * per;
      if (e0 < r0) x &= ~0u << (uint32_t)((r0 - e0) * B);  // r0 - e0 < per here
      if (e0 + per > r1) x &= (1u << (uint32_t)((r1 - e0) * B)) - 1u;  // < 32 bits kept
      return (uint32_t)__popc(x);
    };
    if (((uintptr_t)packed & 15u) == 0) {
      // Groups of four words wholly inside [r0, r1) count without masks,
      // DCOUNT_GROUPS of them per lane loaded before any is counted; the few
      // words at either end (up to seven a side) take word_escapes.
      const uint64_t cw0 = (r0 + per - 1) / per, cw1 = r1 / per;  // whole words [cw0, cw1)
      const uint64_t gc0 = (cw0 + 3) / 4;
      const uint64_t gc1 = cw1 / 4 > gc0 ? cw1 / 4 : gc0;  // clean groups [gc0, gc1)
      auto clean = [&](uint32_t x) -> uint32_t {
        for (uint32_t sh = 1; sh < B; sh <<= 1) x &= x >> sh;
        return (uint32_t)__popc(x & start_mask);
      };
      for (uint64_t g0 = gc0 + lane; g0 < gc1; g0 += 64 * DCOUNT_GROUPS) {
        nk_u32x4 v[DCOUNT_GROUPS];
#pragma unroll
        for (int u = 0; u < DCOUNT_GROUPS; ++u) {
          const uint64_t g = g0 + 64 * (uint64_t)u;
          v[u] = g < gc1 ? gload(reinterpret_cast<const nk_u32x4*>(packed) + g)
                         : nk_u32x4{0u, 0u, 0u, 0u};
        }
#pragma unroll
        for (int u = 0; u < DCOUNT_GROUPS; ++u)
          cnt += clean(v[u].x) + clean(v[u].y) + clean(v[u].z) + clean(v[u].w);
      }
      // the words outside the clean groups: [wlo, 4 gc0) and [4 gc1, whi)
      const uint64_t a1 = 4 * gc0 < whi ? 4 * gc0 : whi;
      const uint64_t b0 = 4 * gc1 > a1 ? 4 * gc1 : a1;
      const uint64_t na = a1 > wlo ? a1 - wlo : 0, nb = whi > b0 ? whi - b0 : 0;
      for (uint64_t i = lane; i < na + nb; i += 64) {
        const uint64_t w = i < na ? wlo + i : b0 + (i - na);
        cnt += word_escapes(w, packed[w]);
      }
    } else {
      for (uint64_t w = wlo + lane; w < whi; w += 64) cnt += word_escapes(w, packed[w]);
    }
  } else if (r0 < r1) {
    // Lane l takes words w = w_lo + l, w_lo + l + 64, ... and counts the
    // indices that start in word w (those straddling into w + 1 read it
    // too).  The first index starting in w and its bit offset there are
    // advanced from one word to the next without divisions: 64 words are
    // 2048 bits.
    const uint64_t wlo = (r0 * B) >> 5;
    const uint64_t whi = (r1 * B + 31) >> 5;  // exclusive
    uint64_t w = wlo + lane;
    // first index starting at or after bit 32w, and its offset in word w
    uint64_t e = (32 * w + B - 1) / B;
    uint32_t off = (uint32_t)(e * B - 32 * w);
    const uint32_t q = 2048 / B, rem = 2048 % B;
    for (; w < whi; w += 64) {
      const uint32_t lo = packed[w];
      const uint32_t hi = w + 1 < packed_words ? packed[w + 1] : 0u;
      const unsigned long long x = (unsigned long long)lo | ((unsigned long long)hi << 32);
      uint64_t ee = e;
      for (uint32_t o = off; o < 32; o += B, ++ee)
        cnt += (ee >= r0 && ee < r1 && (uint32_t)((x >> o) & esc) == esc) ? 1ull : 0ull;
      // advance by 64 words: offset drops by 2048 bits = q indices + rem bits
      e += q;
      if (off >= rem) {
        off -= rem;
      } else {
        off = off + B - rem;
        e += 1;
      }
    }
  }
  return wave_sum_u64(cnt);
}

// One launch counts escapes for the whole decode.  The first n_units waves
// are the decoder units: wave u counts its tile run of the range.  The
// pre_units waves after them split [start of start's block, start), the part
// of the block before the range, into pieces of pre_elems indices.
__global__ void __launch_bounds__(UNIT_TPB) k_dcount(DParams P) {
  const uint32_t wave = blockIdx.x * (UNIT_TPB / 64) + threadIdx.x / 64;
  if (blockIdx.x == 0 && threadIdx.x == 0) gstore(P.flags, 0u);  // the decoder ORs into it
  uint64_t r0, r1;
  if (wave < P.n_units) {
    const uint64_t end = P.start + P.len;
    r0 = P.start + (uint64_t)wave * P.tiles_per_unit * P.tile_elems;
    r1 = r0 + P.tiles_per_unit * P.tile_elems;
    r0 = r0 < end ? r0 : end;
    r1 = r1 < end ? r1 : end;
  } else {
    const uint32_t i = wave - P.n_units;
    if (i >= P.pre_units) return;
    const uint64_t b0 = P.start / P.epb * P.epb;
    r0 = b0 + (uint64_t)i * P.pre_elems;
    r1 = r0 + P.pre_elems;
    r0 = r0 < P.start ? r0 : P.start;
    r1 = r1 < P.start ? r1 : P.start;
  }
  const unsigned long long cnt = wave_count_escapes(P.packed, P.packed_words, P.B, r0, r1);
  if (lane_id() == 0) {
    if (wave < P.n_units)
      P.unit_cnt[wave] = (uint32_t)cnt;
    else
      P.pre_cnt[wave - P.n_units] = (uint32_t)cnt;
  }
}

// LDS budget for the centre table (used when 2^B entries fit).
constexpr int DEC_CENT_BYTES = 32768;
constexpr uint64_t DEC_NT_BYTES = 256ull << 20;  // output size from which accesses are non-temporal

// Unit u decodes its wave tiles in order.  Each lane handles V consecutive
// elements per round (V = 16 / sizeof(T)); VEC selects 16-byte vector loads
// of prev and stores of out (start a multiple of V, pointers 16-byte
// aligned), otherwise the same elements are moved one by one.
template <typename T, bool VEC, bool NT>
__global__ void __launch_bounds__(UNIT_TPB) k_decode(DParams P) {
  constexpr int V = Traits<T>::V;
  constexpr int R = DEC_ROUNDS;
  constexpr int WT = R * 64 * V;
  constexpr int NWAVE = UNIT_TPB / 64;
  constexpr int TW = NK_DEC_DIRECT ? 1 : WT * 16 / 32 + 2;  // packed words of a tile, at most
  __shared__ uint32_t s_words[NWAVE][TW];
  extern __shared__ unsigned char s_dyn[];  // centre table when it fits
  T* s_cent = reinterpret_cast<T*>(s_dyn);
  const int tid = threadIdx.x;
  const int wave = tid / 64;
  const int lane = lane_id();
  const uint32_t B = P.B;
  const uint32_t esc = (1u << B) - 1u;
  const T* __restrict__ prev = static_cast<const T*>(P.prev);
  const T* __restrict__ centers = static_cast<const T*>(P.centers);
  const T* __restrict__ incomp = static_cast<const T*>(P.incomp);
  T* __restrict__ out = static_cast<T*>(P.out);
  const uint64_t end = P.start + P.len;
  const bool lds_cent = ((uint64_t)1 << B) * sizeof(T) <= (uint64_t)DEC_CENT_BYTES;
  if (lds_cent)
    for (int i = tid; i < (1 << B); i += UNIT_TPB) s_cent[i] = centers[i];
  // Escapes before this workgroup's first unit: those before `start` (the
  // block table's count at start's block plus the counted pieces of that
  // block before start) and the counts of the units before it.
  __shared__ unsigned long long s_part[NWAVE];
  __shared__ uint32_t s_cnt[NWAVE];
  const uint32_t unit0 = blockIdx.x * NWAVE;
  unsigned long long sum = strided_sum_u32(P.unit_cnt, tid, unit0, UNIT_TPB) +
                           strided_sum_u32(P.pre_cnt, tid, P.pre_units, UNIT_TPB);
  sum = wave_sum_u64(sum);
  if (lane == 0) {
    s_part[wave] = sum;
    s_cnt[wave] = unit0 + wave < P.n_units ? gload(P.unit_cnt + unit0 + wave) : 0u;
  }
  __syncthreads();
  unsigned long long run =
      P.len ? (unsigned long long)gload(P.block_inc_off + P.start / P.epb) : 0ull;
#pragma unroll
  for (int w = 0; w < NWAVE; ++w) run += s_part[w] + (w < wave ? s_cnt[w] : 0u);

  const uint32_t unit = unit0 + wave;
  uint32_t* words = s_words[wave];
  const uint64_t tb = (uint64_t)unit * P.tiles_per_unit;
  uint64_t te = tb + P.tiles_per_unit;
  te = te < P.n_tiles ? te : P.n_tiles;
  const unsigned long long lt = lanemask_lt();
  bool bad = false, over = false;
  for (uint64_t tile = tb; tile < te; ++tile) {
    const uint64_t t0 = P.start + tile * WT;
    const uint64_t rem = end - t0;
    const uint32_t tn = rem < (uint64_t)WT ? (uint32_t)rem : (uint32_t)WT;
    const uint64_t wlo = (t0 * B) >> 5;
    const uint32_t nw = (uint32_t)((((t0 + tn) * B + 31) >> 5) - wlo);
    if (!NK_DEC_DIRECT)
      for (uint32_t i = lane; i < nw; i += 64) words[i] = P.packed[wlo + i];

    T pv[R][V];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint32_t e = ((uint32_t)r * 64 + lane) * V;
      if (VEC && e + V <= tn) {
        load_vec_t<NT>(prev, (t0 + e) / V, pv[r]);
      } else {
#pragma unroll
        for (int v = 0; v < V; ++v) pv[r][v] = e + v < tn ? prev[t0 + e + v] : (T)0;
      }
    }
    if (!NK_DEC_DIRECT) wave_lds_sync();

    const uint32_t bitbase = (uint32_t)(t0 * B - wlo * 32);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint32_t e = ((uint32_t)r * 64 + lane) * V;
      uint32_t code[V];
      unsigned long long emask[V];
      unsigned below = 0, all = 0;
#pragma unroll
      for (int v = 0; v < V; ++v) {
        uint32_t cd = 0;
        if (e + v < tn) {
          if (NK_DEC_DIRECT) {
            cd = unpack_index(P.packed, t0 + e + v, B);
          } else {
            const uint32_t bit = bitbase + (e + v) * B;
            const uint32_t w = bit >> 5, sh = bit & 31;
            uint32_t x = words[w] >> sh;
            if (sh + B > 32) x |= words[w + 1] << (32 - sh);
            cd = x & esc;
          }
        }
        code[v] = cd;
        emask[v] = __ballot(e + v < tn && cd == esc);
        below += (unsigned)__popcll(emask[v] & lt);
        all += (unsigned)__popcll(emask[v]);
      }
      unsigned long long rank = run + below;
      T ov[V];
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const uint32_t cd = code[v];
        if ((emask[v] >> lane) & 1ull) {
          if (rank < P.n_inc) {
            ov[v] = incomp[rank];
          } else {
            over = true;
            ov[v] = (T)0;
          }
          rank += 1;
        } else {
          bad |= (e + v < tn) && cd >= P.k_used;
          const double c = (double)(lds_cent ? s_cent[cd] : centers[cd]);
          ov[v] = (T)((double)pv[r][v] * (1.0 + c));
        }
      }
      const uint64_t o = t0 + e - P.start;
      if (VEC && e + V <= tn) {
        nk_u32x4 x;
        __builtin_memcpy(&x, ov, 16);
        NK_GLOBAL nk_u32x4* dst = (NK_GLOBAL nk_u32x4*)out + o / V;
        if constexpr (NT) __builtin_nontemporal_store(x, dst);
        else *dst = x;
      } else {
#pragma unroll
        for (int v = 0; v < V; ++v)
          if (e + v < tn) out[o + v] = ov[v];
      }
      run += all;
    }
    if (!NK_DEC_DIRECT) wave_lds_sync();
  }
  if (__ballot(bad) && lane == 0) atomicOr(P.flags, NUMARCK_FLAG_BAD_INDEX);
  if (__ballot(over) && lane == 0) atomicOr(P.flags, NUMARCK_FLAG_INC_OVERRUN);
}

#define NK_DLAUNCH(kind, kern, grid, block, lds, ...)                            \
  do {                                                                           \
    timing_begin(kind, s);                                                       \
    hipLaunchKernelGGL(kern, dim3(grid), dim3(block), lds, s, __VA_ARGS__);      \
    timing_end(kind, s);                                                         \
    hipError_t e_ = hipGetLastError();                                           \
    if (e_ != hipSuccess) return e_;                                             \
  } while (0)

template <typename T, bool VEC, bool NT>
static hipError_t launch_decode_chain(DParams P, size_t cent_lds, hipStream_t s) {
  const Geometry g = geometry();
  // as many units as can be resident at once (4 per workgroup)
  int occ = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_decode<T, VEC, NT>, UNIT_TPB,
                                                   cent_lds) != hipSuccess || occ < 1)
    occ = 1;
  P.n_units = range_units(P.n_tiles, g.cus * occ * 4);
  P.tiles_per_unit = (P.n_tiles + P.n_units - 1) / P.n_units;
  // the part of start's block before the range, in pieces of at least 8192
  // indices, at most MAX_PRE_UNITS of them
  const uint64_t pre = P.len ? P.start % P.epb : 0;
  uint64_t piece = (pre + MAX_PRE_UNITS - 1) / MAX_PRE_UNITS;
  piece = piece < 8192 ? 8192 : piece;
  P.pre_units = (uint32_t)((pre + piece - 1) / piece);
  P.pre_elems = piece;
  const uint32_t waves = P.n_units + P.pre_units;
  NK_DLAUNCH(KK_DCOUNT, k_dcount, (waves + 3) / 4, UNIT_TPB, 0, P);
  NK_DLAUNCH(KK_DECODE, (k_decode<T, VEC, NT>), P.n_units / 4, UNIT_TPB, cent_lds, P);
  return hipSuccess;
}

template <typename T>
static hipError_t launch_decompress_t(const DParams& P, hipStream_t s) {
  const size_t cent = ((size_t)1 << P.B) * sizeof(T);
  const size_t cent_lds = cent <= (size_t)DEC_CENT_BYTES ? cent : 0;
  const bool vec = (P.start % Traits<T>::V) == 0 && ((uintptr_t)P.prev & 15u) == 0 &&
                   ((uintptr_t)P.out & 15u) == 0;
  // a large decompression streams prev and out once: non-temporal accesses
  // keep them from displacing each other in the caches (as in the
  // compression passes)
  const bool nt = vec && P.len * sizeof(T) >= DEC_NT_BYTES;
  return nt ? launch_decode_chain<T, true, true>(P, cent_lds, s)
            : vec ? launch_decode_chain<T, true, false>(P, cent_lds, s)
                  : launch_decode_chain<T, false, false>(P, cent_lds, s);
}

hipError_t launch_decompress(const DParams& P, hipStream_t s) {
  return P.dtype == NUMARCK_F32 ? launch_decompress_t<float>(P, s)
                                : launch_decompress_t<double>(P, s);
}

}  // namespace nk
