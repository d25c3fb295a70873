// stream_kernels.hip -- reference kernels for the HBM roofline the
// compression passes are measured against: a read, a write and a copy of a
// large buffer with 16-byte vector accesses, each with cached or
// non-temporal accesses, and the encoder's shape (two arrays read, a
// 1/16-sized stream written).  Not part of the compression path; the benchmark
// times them beside it and uses the copy as the kernel of known traffic that
// scales the hardware byte counters.
#include "nk_device.h"

namespace nk {

constexpr int STREAM_TPB = 256;
constexpr int STREAM_UNROLL = 4;  // vectors in flight per thread

template <bool NT>
__device__ __forceinline__ nk_u32x4 sload(const nk_u32x4* p) {
  if constexpr (NT) return __builtin_nontemporal_load((const NK_GLOBAL nk_u32x4*)p);
  return *((const NK_GLOBAL nk_u32x4*)p);
}
template <bool NT>
__device__ __forceinline__ void sstore(nk_u32x4* p, nk_u32x4 v) {
  if constexpr (NT) __builtin_nontemporal_store(v, (NK_GLOBAL nk_u32x4*)p);
  else *((NK_GLOBAL nk_u32x4*)p) = v;
}

// Each thread walks the vectors grid-strided, STREAM_UNROLL at a time: all
// loads of a step are issued before their uses.
template <bool NT>
__global__ void __launch_bounds__(STREAM_TPB) k_stream_read(const nk_u32x4* __restrict__ src,
                                                            uint64_t nvec,
                                                            unsigned int* __restrict__ sink) {
  const uint64_t stride = (uint64_t)gridDim.x * STREAM_TPB;
  uint64_t i = (uint64_t)blockIdx.x * STREAM_TPB + threadIdx.x;
  unsigned int acc = 0;
  for (; i + (STREAM_UNROLL - 1) * stride < nvec; i += STREAM_UNROLL * stride) {
    nk_u32x4 v[STREAM_UNROLL];
#pragma unroll
    for (int u = 0; u < STREAM_UNROLL; ++u) v[u] = sload<NT>(src + i + u * stride);
#pragma unroll
    for (int u = 0; u < STREAM_UNROLL; ++u) acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
  }
  for (; i < nvec; i += stride) {
    const nk_u32x4 v = sload<NT>(src + i);
    acc ^= v.x ^ v.y ^ v.z ^ v.w;
  }
  // one word per wave keeps the loads live
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc ^= (unsigned int)__shfl_xor((int)acc, o, 64);
  if (lane_id() == 0) gstore(sink + (blockIdx.x * STREAM_TPB + threadIdx.x) / 64, acc);
}

template <bool NT>
__global__ void __launch_bounds__(STREAM_TPB) k_stream_write(nk_u32x4* __restrict__ dst,
                                                             uint64_t nvec, unsigned int value) {
  const uint64_t stride = (uint64_t)gridDim.x * STREAM_TPB;
  const nk_u32x4 v = {value, value, value, value};
  for (uint64_t i = (uint64_t)blockIdx.x * STREAM_TPB + threadIdx.x; i < nvec; i += stride)
    sstore<NT>(dst + i, v);
}

template <bool NT>
__global__ void __launch_bounds__(STREAM_TPB) k_stream_copy(const nk_u32x4* __restrict__ src,
                                                            nk_u32x4* __restrict__ dst,
                                                            uint64_t nvec) {
  const uint64_t stride = (uint64_t)gridDim.x * STREAM_TPB;
  uint64_t i = (uint64_t)blockIdx.x * STREAM_TPB + threadIdx.x;
  for (; i + (STREAM_UNROLL - 1) * stride < nvec; i += STREAM_UNROLL * stride) {
    nk_u32x4 v[STREAM_UNROLL];
#pragma unroll
    for (int u = 0; u < STREAM_UNROLL; ++u) v[u] = sload<NT>(src + i + u * stride);
#pragma unroll
    for (int u = 0; u < STREAM_UNROLL; ++u) sstore<NT>(dst + i + u * stride, v[u]);
  }
  for (; i < nvec; i += stride) sstore<NT>(dst + i, sload<NT>(src + i));
}

// Two arrays of nvec vectors each (the two snapshots, src and src + nvec)
// read in step, and one word W written per vector position: a 16-bit word is
// the shape of an encoder that reads both snapshots (a 1/16 write stream, the
// index table of 8-bit codes of 64-bit values); a 32-bit word that of the
// histogram pass writing window codes (1/8: two 16-bit codes per vector of
// 64-bit values).
template <bool NT, typename W>
__global__ void __launch_bounds__(STREAM_TPB) k_stream_mix(const nk_u32x4* __restrict__ src,
                                                           uint64_t nvec, W* __restrict__ dst) {
  const uint64_t stride = (uint64_t)gridDim.x * STREAM_TPB;
  const nk_u32x4* __restrict__ a = src;
  const nk_u32x4* __restrict__ b = src + nvec;
  uint64_t i = (uint64_t)blockIdx.x * STREAM_TPB + threadIdx.x;
  for (; i + stride < nvec; i += 2 * stride) {
    const nk_u32x4 x0 = sload<NT>(a + i), y0 = sload<NT>(b + i);
    const nk_u32x4 x1 = sload<NT>(a + i + stride), y1 = sload<NT>(b + i + stride);
    gstore(dst + i, (W)(x0.x ^ y0.y));
    gstore(dst + i + stride, (W)(x1.x ^ y1.y));
  }
  for (; i < nvec; i += stride) {
    const nk_u32x4 x = sload<NT>(a + i), y = sload<NT>(b + i);
    gstore(dst + i, (W)(x.x ^ y.y));
  }
}

// Workgroups of a streaming launch: `per_cu` per compute unit, no more than
// the vectors need.
static unsigned stream_grid(uint64_t nvec, unsigned per_cu) {
  const uint64_t want = (uint64_t)geometry().cus * per_cu;
  const uint64_t need = (nvec + STREAM_TPB - 1) / STREAM_TPB;
  const uint64_t g = want < need ? want : need;
  return (unsigned)(g < 1 ? 1 : g);
}

hipError_t launch_stream(int kind, const void* src, void* dst, uint64_t bytes, unsigned per_cu,
                         hipStream_t s) {
  const uint64_t nvec = bytes / 16;
  const unsigned grid = stream_grid(nvec, per_cu);
  const nk_u32x4* in = static_cast<const nk_u32x4*>(src);
  nk_u32x4* out = static_cast<nk_u32x4*>(dst);
  switch (kind) {
    case NUMARCK_STREAM_READ:
      hipLaunchKernelGGL(k_stream_read<false>, dim3(grid), dim3(STREAM_TPB), 0, s, in, nvec,
                         static_cast<unsigned int*>(dst));
      break;
    case NUMARCK_STREAM_READ_NT:
      hipLaunchKernelGGL(k_stream_read<true>, dim3(grid), dim3(STREAM_TPB), 0, s, in, nvec,
                         static_cast<unsigned int*>(dst));
      break;
    case NUMARCK_STREAM_WRITE:
      hipLaunchKernelGGL(k_stream_write<false>, dim3(grid), dim3(STREAM_TPB), 0, s, out, nvec,
                         0x3FF00000u);
      break;
    case NUMARCK_STREAM_WRITE_NT:
      hipLaunchKernelGGL(k_stream_write<true>, dim3(grid), dim3(STREAM_TPB), 0, s, out, nvec,
                         0x3FF00000u);
      break;
    case NUMARCK_STREAM_COPY:
      hipLaunchKernelGGL(k_stream_copy<false>, dim3(grid), dim3(STREAM_TPB), 0, s, in, out, nvec);
      break;
    case NUMARCK_STREAM_COPY_NT:
      hipLaunchKernelGGL(k_stream_copy<true>, dim3(grid), dim3(STREAM_TPB), 0, s, in, out, nvec);
      break;
    case NUMARCK_STREAM_READ2_WRITE16: {
      const unsigned g2 = stream_grid(nvec / 2, per_cu);
      hipLaunchKernelGGL((k_stream_mix<true, unsigned short>), dim3(g2), dim3(STREAM_TPB), 0, s,
                         in, nvec / 2, static_cast<unsigned short*>(dst));
      break;
    }
    case NUMARCK_STREAM_READ2_WRITE8: {
      const unsigned g2 = stream_grid(nvec / 2, per_cu);
      hipLaunchKernelGGL((k_stream_mix<true, unsigned int>), dim3(g2), dim3(STREAM_TPB), 0, s,
                         in, nvec / 2, static_cast<unsigned int*>(dst));
      break;
    }
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace nk
