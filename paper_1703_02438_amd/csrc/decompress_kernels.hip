// decompress_kernels.hip -- full and partial decompression of NUMARCK
// (arXiv 1703.02438, eq. 4 / Sec. III-E, partial decompression Sec. IV-C and
// V-C).
//
// A range [start, start + len) is decoded in tiles taken in ticket order:
//   k_dinit    reset the control block, the flag word and the look-back words
//   k_dprefix  escapes before `start`: the block table gives the count up to
//              the start of start's block, the rest is counted from the
//              packed indices (at most one block)
//   k_decode   unpack each index; an escape takes the next incompressible
//              value (its rank comes from a decoupled look-back over tiles),
//              any other index gives T(prev * (1 + centre[index]))
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

__global__ void k_dinit(DParams P) {
  const uint64_t gt = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t gs = (uint64_t)gridDim.x * blockDim.x;
  if (gt == 0) {
    P.dctl->base = 0ull;
    P.dctl->ticket = 0u;
    *P.flags = 0u;
  }
  for (uint64_t i = gt; i < P.n_tiles; i += gs) P.status[i] = 0ull;
}

__global__ void k_dprefix(DParams P) {
  if (P.len == 0) return;
  const uint64_t blk = P.start / P.epb;
  const uint64_t b0 = blk * P.epb;
  const uint32_t esc = (1u << P.B) - 1u;
  const uint64_t gt = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t gs = (uint64_t)gridDim.x * blockDim.x;
  unsigned long long cnt = 0;
  if (gt == 0) cnt += (unsigned long long)P.block_inc_off[blk];
  for (uint64_t j = b0 + gt; j < P.start; j += gs)
    cnt += unpack_index(P.packed, j, P.B) == esc ? 1ull : 0ull;
  cnt = wave_sum_u64(cnt);
  if (lane_id() == 0 && cnt) atomicAdd(&P.dctl->base, cnt);
}

template <typename T>
__global__ void __launch_bounds__(DEC_TPB) k_decode(DParams P) {
  constexpr int R = DEC_TILE / DEC_TPB;
  constexpr int NW = DEC_TPB / 64;
  __shared__ unsigned s_wcnt[R][NW];
  __shared__ unsigned long long s_prefix;
  __shared__ uint64_t s_tile;
  const int tid = threadIdx.x;
  const int wave = tid / 64;
  const int lane = lane_id();
  const uint32_t esc = (1u << P.B) - 1u;
  const T* __restrict__ prev = static_cast<const T*>(P.prev);
  const T* __restrict__ centers = static_cast<const T*>(P.centers);
  const T* __restrict__ incomp = static_cast<const T*>(P.incomp);
  T* __restrict__ out = static_cast<T*>(P.out);
  const uint64_t end = P.start + P.len;

  while (true) {
    __syncthreads();
    if (tid == 0) s_tile = atomicAdd(&P.dctl->ticket, 1u);
    __syncthreads();
    const uint64_t tile = s_tile;
    if (tile >= P.n_tiles) break;
    const uint64_t t0 = P.start + tile * DEC_TILE;

    uint32_t code[R];
    unsigned long long emask[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint64_t j = t0 + (uint64_t)r * DEC_TPB + tid;
      const bool inr = j < end;
      code[r] = inr ? unpack_index(P.packed, j, P.B) : 0u;
      emask[r] = __ballot(inr && code[r] == esc);
      if (lane == 0) s_wcnt[r][wave] = (unsigned)__popcll(emask[r]);
    }
    __syncthreads();
    if (tid < 64) {
      unsigned long long tot = 0;
      if (tid == 0) {
        for (int r = 0; r < R; ++r)
          for (int w = 0; w < NW; ++w) {
            const unsigned t = s_wcnt[r][w];
            s_wcnt[r][w] = (unsigned)tot;
            tot += t;
          }
      }
      tot = __shfl(tot, 0, 64);
      const unsigned long long ex = lookback(P.status, tile, tot);
      if (tid == 0) s_prefix = ex;
    }
    __syncthreads();
    const unsigned long long base = P.dctl->base + s_prefix;
    const unsigned long long lt = lanemask_lt();
    bool bad = false, over = false;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint64_t j = t0 + (uint64_t)r * DEC_TPB + tid;
      if (j < end) {
        T v;
        if (code[r] == esc) {
          const unsigned long long rank =
              base + s_wcnt[r][wave] + (unsigned long long)__popcll(emask[r] & lt);
          if (rank < P.n_inc) {
            v = incomp[rank];
          } else {
            over = true;
            v = (T)0;
          }
        } else {
          bad |= code[r] >= P.k_used;
          const double c = (double)centers[code[r]];
          v = (T)((double)prev[j] * (1.0 + c));
        }
        out[j - P.start] = v;
      }
    }
    if (__ballot(bad) && lane == 0) atomicOr(P.flags, NUMARCK_FLAG_BAD_INDEX);
    if (__ballot(over) && lane == 0) atomicOr(P.flags, NUMARCK_FLAG_INC_OVERRUN);
  }
}

#define NK_DLAUNCH(kind, kern, grid, block, ...)                                 \
  do {                                                                           \
    timing_begin(kind, s);                                                       \
    hipLaunchKernelGGL(kern, dim3(grid), dim3(block), 0, s, __VA_ARGS__);        \
    timing_end(kind, s);                                                         \
    hipError_t e_ = hipGetLastError();                                           \
    if (e_ != hipSuccess) return e_;                                             \
  } while (0)

template <typename T>
static hipError_t launch_decompress_t(const DParams& P, hipStream_t s) {
  const Geometry g = geometry();
  uint64_t init_blocks = (P.n_tiles + 255) / 256;
  if (init_blocks < 1) init_blocks = 1;
  if (init_blocks > (uint64_t)g.cus) init_blocks = g.cus;
  uint64_t pre_blocks = P.len ? ((P.start % P.epb) + 255) / 256 : 1;
  if (pre_blocks < 1) pre_blocks = 1;
  if (pre_blocks > (uint64_t)g.cus * 2) pre_blocks = (uint64_t)g.cus * 2;
  uint64_t dec_blocks = P.n_tiles;
  if (dec_blocks > (uint64_t)g.cus * 4) dec_blocks = (uint64_t)g.cus * 4;
  if (dec_blocks < 1) dec_blocks = 1;
  NK_DLAUNCH(KK_DINIT, k_dinit, init_blocks, 256, P);
  NK_DLAUNCH(KK_DPREFIX, k_dprefix, pre_blocks, 256, P);
  NK_DLAUNCH(KK_DECODE, k_decode<T>, dec_blocks, DEC_TPB, P);
  return hipSuccess;
}

hipError_t launch_decompress(const DParams& P, hipStream_t s) {
  return P.dtype == NUMARCK_F32 ? launch_decompress_t<float>(P, s)
                                : launch_decompress_t<double>(P, s);
}

}  // namespace nk
