// nk_device.h -- device helpers shared by the NUMARCK kernels: element
// traits, the change ratio and its validity, bin ids and centres, wave
// reductions.
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
// Global-memory access through a generic pointer.  Pointers that kernels
// read from memory (a batch's job table) carry no address space, and the
// compiler would otherwise access through them with flat instructions, which
// also count against the LDS counter: every LDS wait then waits for the
// streamed loads as well.
#define NK_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ void gstore(T* p, T v) {
  *((NK_GLOBAL T*)p) = v;  // a C-style cast: it may change the address space
}
template <typename T>
__device__ __forceinline__ T gload(const T* p) {
  return *((const NK_GLOBAL T*)p);
}

typedef unsigned int nk_u32x4 __attribute__((ext_vector_type(4)));

template <typename T>
__device__ __forceinline__ void load_vec(const T* __restrict__ base, uint64_t vi, T* out) {
  const nk_u32x4 x = ((const NK_GLOBAL nk_u32x4*)base)[vi];
  __builtin_memcpy(out, &x, 16);
}

// The same load, marked non-temporal when NT: streamed data that will not
// be read again then does not displace what will (the written outputs,
// inputs shared with another job of a batch).  A compile-time choice: the
// compiler merges a run-time choice between the two into one cached load.
template <bool NT, typename T>
__device__ __forceinline__ void load_vec_t(const T* __restrict__ base, uint64_t vi, T* out) {
  if constexpr (NT) {
    const nk_u32x4 x = __builtin_nontemporal_load(((const NK_GLOBAL nk_u32x4*)base) + vi);
    __builtin_memcpy(out, &x, 16);
  } else {
    load_vec(base, vi, out);
  }
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

// eq. (1): change ratio d = (q - p) / p in binary64; returns validity:
// p nonzero and finite, q finite, d finite and |d| <= cap = E * 2^50.
// Evaluated as isfinite(p) && |d| <= cap, which is the same predicate: the
// comparison is false for a NaN or infinite d, and with p finite a zero p
// (division by zero) or a non-finite q always yields such a d.
__device__ __forceinline__ bool ratio_of(double p, double q, double cap, double& d) {
  d = (q - p) / p;
  return __builtin_isfinite(p) & (fabs(d) <= cap);
}

// Fine bin of a valid ratio: bins of width 2E anchored at lo.
__device__ __forceinline__ long long bin_of(double d, double lo, double twoE) {
  return (long long)floor((d - lo) / twoE);
}

// floor(x / twoE) for x of either sign, as a double, bit-identical to
// flooring the correctly rounded quotient.  The fast path multiplies by
// inv = fl(1/twoE): t' = fl(x * inv) is within 2^-51 |t'| of t = fl(x / twoE)
// (three roundings of at most 2^-53 each), so floor(t') == floor(t) unless an
// integer lies within that distance of t'.  Those cases take the exact
// division, and so does every x when 2E is subnormal: inv is then infinite,
// t' infinite or NaN, and the check fails.  The distance to the integer
// below, t' - floor(t'), is exact (Sterbenz) for t' >= 0 and for t' <= -1/2;
// in (-1/2, 0) it is above 1/2 and only its distance 1 - frac to 0 matters,
// which is at least |t'| (t and t' then share their sign, so both floors are
// -1).  For |x| below 2^51 * twoE, as every valid ratio gives, t' cannot
// overflow, and neither quotient is subnormal: x = d - lo is 0 or, with d a
// ratio (0 or at least 2^-53 in magnitude) and lo a ratio or -E, at least
// about 2^-55 * twoE in magnitude.
__device__ __forceinline__ double bin_floor(double x, double twoE, double inv) {
  const double t = x * inv;
  const double f = floor(t);
  const double frac = t - f;
  const double thr = fabs(t) * 0x1p-49;
  if ((frac > thr) && ((1.0 - frac) > thr)) return f;
  return floor(x / twoE);
}

// The fast part of bin_floor: floor(x * inv) and whether it is certain.
// When `sure` is false the caller takes floor(x / twoE).
__device__ __forceinline__ double bin_floor_fast(double x, double inv, bool& sure) {
  const double t = x * inv;
  const double f = floor(t);
  const double frac = t - f;
  const double thr = fabs(t) * 0x1p-49;
  sure = (frac > thr) && ((1.0 - frac) > thr);
  return f;
}

// Fine bin of the change ratio without the correctly rounded division, for
// the passes that need only the bin and the validity of a point (the
// histogram and the encoder).  The exact definition is
//   d = fl(fl(q - p) / p),  valid = isfinite(p) && |d| <= cap,
//   m = floor(fl(fl(d - lo) / bw)).
// The fast path takes r0 = the hardware reciprocal of p, one Newton step
// r1 = r0 + r0 (1 - p r0), and d1 = fl(q - p) * r1.  When |1 - p r0| <= 2^-20,
// r1 is within 2^-39.9 of 1/p, so d1 is within 2^-39.6 |d1| of d (the
// division's own rounding included).  Then:
//   - validity is certain unless |d1| lies within 2^-36 of cap;
//   - with x1 = fl(d1 - lo) and t1 = fl(x1 * inv), t1 differs from the exact
//     quotient fl(fl(d - lo) / bw) by at most 2^-38 |d1| inv (the ratio's
//     error, scaled) plus 2^-49 |t1| (the roundings, as in bin_floor), so
//     floor(t1) is the exact bin unless an integer lies within
//     thr = 2^-36 |d1| inv + 2^-48 |t1| of t1 (both terms taken twice over).
// A point is `sure` when its reciprocal is that good and neither test is
// close.  A zero, infinite or NaN p makes 1 - p r0 a NaN and a p whose
// reciprocal overflows makes it infinite, so such points are never sure;
// neither is a ratio at the cap or a bin edge.  The caller recomputes the
// points that are not sure with ratio_of and floor((d - lo) / bw).  When a
// point is sure, `valid` is its validity and the result its bin.  inv_err is
// inv * 2^-36.
__device__ __forceinline__ double ratio_bin_fast(double p, double q, double cap_lo,
                                                 double cap_hi, double lo, double inv,
                                                 double inv_err, bool& valid, bool& sure) {
  const double qp = q - p;
  const double r0 = __builtin_amdgcn_rcp(p);
  const double e0 = __builtin_fma(-p, r0, 1.0);
  const double r1 = __builtin_fma(r0, e0, r0);
  const double d1 = qp * r1;
  const double ad = fabs(d1);
  const bool in_lo = ad <= cap_lo;  // false for a NaN ratio
  const bool in_hi = ad <= cap_hi;
  valid = in_lo;
  const double t = (d1 - lo) * inv;
  const double f = floor(t);
  const double frac = t - f;
  const double thr = __builtin_fma(ad, inv_err, fabs(t) * 0x1p-48);
  const bool bin_ok = (frac > thr) & ((1.0 - frac) > thr);
  // in_lo implies in_hi: a valid point needs its bin certain, an invalid one
  // a ratio clearly past the cap
  sure = (fabs(e0) <= 0x1p-20) & ((in_lo & bin_ok) | !in_hi);
  return f;
}

// The fine bin and validity of a point, bit-identical to the exact
// definition: ratio_bin_fast, and the exact division where it is unsure.
__device__ __forceinline__ double ratio_bin(double p, double q, double cap, double cap_lo,
                                            double cap_hi, double lo, double bw, double inv,
                                            double inv_err, bool& valid) {
  bool sure;
  double m = ratio_bin_fast(p, q, cap_lo, cap_hi, lo, inv, inv_err, valid, sure);
  if (!sure) {
    double d;
    valid = ratio_of(p, q, cap, d);
    m = floor((d - lo) / bw);
  }
  return m;
}

// Margins of ratio_bin_fast's validity test: cap (1 -+ 2^-36).
__device__ __forceinline__ double cap_below(double cap) { return cap * (1.0 - 0x1p-36); }
__device__ __forceinline__ double cap_above(double cap) { return cap * (1.0 + 0x1p-36); }

// Bin centre lo + (2m + 1) E from a bin id held as a double (an integer below
// 2^51, so 2m + 1 is exact), rounded to the snapshot type and widened back.
template <typename T>
__device__ __forceinline__ double centre_of_d(double m, double lo, double E) {
  const double c = lo + (2.0 * m + 1.0) * E;
  return (double)(T)c;
}

// Bin centre lo + (2m + 1) E, rounded to the snapshot type and widened back.
template <typename T>
__device__ __forceinline__ double centre_of(long long m, double lo, double E) {
  double c = lo + (double)(2 * m + 1) * E;
  return (double)(T)c;
}

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// Add one to counter `key` of an LDS histogram for every lane with `on`.
// The wave's most common case -- the key of its first active lane -- takes a
// single atomic for all lanes that share it; the other lanes add directly.
__device__ __forceinline__ void lds_count(uint32_t* hist, bool on, unsigned key) {
  const unsigned long long act = __ballot(on);
  if (!act) return;
  const int leader = __ffsll((long long)act) - 1;
  const unsigned lk = (unsigned)__builtin_amdgcn_readlane((int)key, leader);
  const bool same = on && key == lk;
  const unsigned long long sm = __ballot(same);
  if (lane_id() == leader) atomicAdd(&hist[lk], (unsigned)__popcll(sm));
  if (on && !same) atomicAdd(&hist[key], 1u);
}

// Order this wave's LDS accesses before and after: LDS instructions of one
// wave execute in order, so a compiler barrier plus waiting for the wave's
// own LDS operations is enough for lanes to read what other lanes wrote.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

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
// Sum of a[i] over i = first, first + step, ... below lim (one thread's
// share of a workgroup-strided sum), eight loads in flight at a time: a
// plain loop waits for each load before the next, a chain of dependent
// round trips to L2 that cost the kernels summing a few thousand counts
// ahead of their work about 10 us.
__device__ __forceinline__ unsigned long long strided_sum_u32(const uint32_t* a, uint32_t first,
                                                              uint32_t lim, uint32_t step) {
  unsigned long long s = 0;
  uint32_t i = first;
  for (; i + 7 * step < lim; i += 8 * step) {
    uint32_t x[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) x[u] = gload(a + i + u * step);
#pragma unroll
    for (int u = 0; u < 8; ++u) s += x[u];
  }
  for (; i < lim; i += step) s += gload(a + i);
  return s;
}

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    unsigned long long w = __shfl_xor(v, o, 64);
    v = w > v ? w : v;
  }
  return v;
}

constexpr int USCAN_TPB = 1024;

// Exclusive scan of cnt[0..n) in place (n <= MAX_UNITS) by one workgroup of
// USCAN_TPB threads; every thread returns the total.
__device__ __forceinline__ unsigned long long unit_scan(uint32_t* cnt, uint32_t n) {
  constexpr int PER = MAX_UNITS / USCAN_TPB;
  constexpr int Q = USCAN_TPB / 64;
  __shared__ unsigned long long s_part[Q];
  const int tid = threadIdx.x;
  uint32_t v[PER];
  unsigned long long mine = 0;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const uint32_t k = (uint32_t)tid * PER + i;
    v[i] = k < n ? gload(cnt + k) : 0u;
    mine += v[i];
  }
  // exclusive prefix of `mine` over the workgroup: wave scans, then the
  // wave totals (every thread reads all Q of them: broadcast, no conflicts)
  const int lane = tid & 63, w = tid >> 6;
  unsigned long long inc = mine;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const unsigned long long t = __shfl_up(inc, o, 64);
    if (lane >= o) inc += t;
  }
  if (lane == 63) s_part[w] = inc;
  __syncthreads();
  unsigned long long base = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const unsigned long long r = s_part[i];
    base += i < w ? r : 0ull;
    tot += r;
  }
  unsigned long long run = base + inc - mine;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const uint32_t k = (uint32_t)tid * PER + i;
    if (k < n) gstore(cnt + k, (uint32_t)run);
    run += v[i];
  }
  return tot;
}

}  // namespace nk
