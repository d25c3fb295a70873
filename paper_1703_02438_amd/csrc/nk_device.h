// nk_device.h -- device helpers shared by the NUMARCK kernels: element
// traits, the change ratio and its validity, bin ids and centres, wave
// reductions and the decoupled look-back used for order-preserving scans.
#pragma once

#include "nk_internal.h"

#pragma clang fp contract(off)

namespace nk {

template <typename T>
struct Traits;
template <>
struct Traits<double> {
  static constexpr int V = 2;  // elements per 16-byte vector
  using U = unsigned long long;
};
template <>
struct Traits<float> {
  static constexpr int V = 4;
  using U = unsigned int;
};

// 16-byte vector load of V elements (the snapshot pointers are 16-byte aligned).
template <typename T>
__device__ __forceinline__ void load_vec(const T* __restrict__ base, uint64_t vi, T* out) {
  const uint4 x = reinterpret_cast<const uint4*>(base)[vi];
  __builtin_memcpy(out, &x, 16);
}

// Order-preserving map of binary64 to uint64: numeric order, -0 below +0.
__device__ __forceinline__ unsigned long long order_key(double x) {
  unsigned long long b = (unsigned long long)__double_as_longlong(x);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double key_value(unsigned long long k) {
  unsigned long long b = (k >> 63) ? (k & 0x7FFFFFFFFFFFFFFFull) : ~k;
  return __longlong_as_double((long long)b);
}

// eq. (1): change ratio d = (q - p) / p in binary64; returns validity
// (nonzero finite p, finite q, finite d, |d| <= cap = E * 2^50).
__device__ __forceinline__ bool ratio_of(double p, double q, double cap, double& d) {
  d = (q - p) / p;
  return (p != 0.0) & __builtin_isfinite(p) & __builtin_isfinite(q) & __builtin_isfinite(d) &
         (fabs(d) <= cap);
}

// Fine bin of a valid ratio: bins of width 2E anchored at lo.
__device__ __forceinline__ long long bin_of(double d, double lo, double twoE) {
  return (long long)floor((d - lo) / twoE);
}

// Bin centre lo + (2m + 1) E, rounded to the snapshot type and widened back.
template <typename T>
__device__ __forceinline__ double centre_of(long long m, double lo, double E) {
  double c = lo + (double)(2 * m + 1) * E;
  return (double)(T)c;
}

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

__device__ __forceinline__ unsigned long long lanemask_lt() {
  const int l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ unsigned long long wave_min_u64(unsigned long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    unsigned long long w = __shfl_xor(v, o, 64);
    v = w < v ? w : v;
  }
  return v;
}
__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    unsigned long long w = __shfl_xor(v, o, 64);
    v = w > v ? w : v;
  }
  return v;
}

__device__ __forceinline__ unsigned long long ld_status(unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_status(unsigned long long* p, unsigned long long v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Decoupled look-back over tiles taken in ticket order.  Called by all 64
// lanes of one wave; `agg` is the tile's own total.  Publishes the tile's
// aggregate, walks back over the predecessors 64 at a time until it meets an
// inclusive prefix, publishes its own inclusive prefix and returns the
// exclusive one.  Every predecessor holds an earlier ticket, so its block is
// resident and publishes its aggregate without waiting: every wait ends.
__device__ __forceinline__ unsigned long long lookback(unsigned long long* status,
                                                       uint64_t tile,
                                                       unsigned long long agg) {
  const int lane = lane_id();
  if (tile == 0) {
    if (lane == 0) st_status(&status[0], LB_INC | agg);
    return 0;
  }
  if (lane == 0) st_status(&status[tile], LB_AGG | agg);
  unsigned long long excl = 0;
  long long j = (long long)tile - 1 - lane;
  while (true) {
    unsigned long long s = LB_INC;  // before tile 0: inclusive prefix 0
    if (j >= 0) {
      s = ld_status(&status[j]);
      while ((s >> 62) == 0) {
        __builtin_amdgcn_s_sleep(1);
        s = ld_status(&status[j]);
      }
    }
    const unsigned long long incl = __ballot((s >> 62) == 2);
    unsigned long long v = s & LB_VAL;
    if (incl) {
      const int first = __ffsll((long long)incl) - 1;  // nearest inclusive predecessor
      excl += wave_sum_u64(lane <= first ? v : 0ull);
      break;
    }
    excl += wave_sum_u64(v);
    j -= 64;
  }
  if (lane == 0) st_status(&status[tile], LB_INC | (excl + agg));
  return excl;
}

}  // namespace nk
