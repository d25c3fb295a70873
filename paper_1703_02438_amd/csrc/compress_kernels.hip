// compress_kernels.hip -- the gfx950 compression path of NUMARCK
// (arXiv 1703.02438, Sec. III-A..C and IV-A..C).
//
// One compression is a chain of kernels on one stream; every data-dependent
// quantity stays in device memory, so the host never waits between them:
//
//   k_init      reset the control block
//   k_range     pass 1: ratio + validity of every point, min/max of the valid
//               ratios, number of invalid points (Sec. IV-A); also clears the
//               window counts and the look-back status words
//   k_derive    lo, hi, M = floor((hi-lo)/2E)+1 and the on-chip bin window
//   k_hist      pass 2: fine histogram (Sec. IV-B-1).  Bins inside a
//               16384-bin window are counted in LDS with wave-aggregated
//               atomics; the ids of points outside it go to a tail list
//   k_hclear / k_hinsert   exact counts of the tail bins in a hash table
//   k_select    top-k over window + tail counts: the k-th largest count tau by
//               radix select, the lowest-id ties, indices in bin order, the
//               window LUT and the centres (Sec. IV-B-1, III-B)
//   k_tailrank  rank of the selected tail bins (rare; O(t^2) over t <= 65535)
//   k_encode    pass 3: index + verify every point, pack the B-bit indices,
//               write incompressible values in element order through a
//               decoupled look-back over tiles, and the per-block offsets
//               (Sec. III-C, IV-C)
//   k_final     write the header
#include "nk_device.h"

namespace nk {

// =====================================================================
// k_init
// =====================================================================
__global__ void k_init(Ctl* ctl) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    ctl->lo_key = ~0ull;
    ctl->hi_key = 0ull;
    ctl->n_invalid = 0ull;
    ctl->tail_count = 0ull;
    ctl->tile_ticket = 0u;
    ctl->flags = 0u;
    ctl->sel_tail_count = 0u;
  }
}

// =====================================================================
// k_range: pass 1 over prev/curr
// =====================================================================
constexpr int RNG_TPB = 256;
constexpr int RNG_UNROLL = 4;

template <typename T>
__global__ void __launch_bounds__(RNG_TPB) k_range(CParams P) {
  constexpr int V = Traits<T>::V;
  const T* __restrict__ prev = static_cast<const T*>(P.prev);
  const T* __restrict__ curr = static_cast<const T*>(P.curr);
  const uint64_t nvec = P.n / V;
  const int tid = threadIdx.x;

  // side job: clear the global window counts and the look-back words
  {
    const uint64_t gt = (uint64_t)blockIdx.x * RNG_TPB + tid;
    const uint64_t gs = (uint64_t)gridDim.x * RNG_TPB;
    for (uint64_t i = gt; i < (uint64_t)WIN; i += gs) P.gwin[i] = 0u;
    for (uint64_t i = gt; i < P.n_tiles; i += gs) P.status[i] = 0ull;
  }

  unsigned long long kmin = ~0ull, kmax = 0ull, ninv = 0ull;
  for (uint64_t vb = (uint64_t)blockIdx.x * (RNG_TPB * RNG_UNROLL) + tid; vb < nvec;
       vb += (uint64_t)gridDim.x * (RNG_TPB * RNG_UNROLL)) {
    T pv[RNG_UNROLL][V], qv[RNG_UNROLL][V];
#pragma unroll
    for (int u = 0; u < RNG_UNROLL; ++u) {
      const uint64_t vi = vb + (uint64_t)u * RNG_TPB;
      if (vi < nvec) {
        load_vec(prev, vi, pv[u]);
        load_vec(curr, vi, qv[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < RNG_UNROLL; ++u) {
      const uint64_t vi = vb + (uint64_t)u * RNG_TPB;
      if (vi < nvec) {
#pragma unroll
        for (int v = 0; v < V; ++v) {
          double d;
          if (ratio_of((double)pv[u][v], (double)qv[u][v], P.cap, d)) {
            const unsigned long long k = order_key(d);
            kmin = k < kmin ? k : kmin;
            kmax = k > kmax ? k : kmax;
          } else {
            ninv += 1;
          }
        }
      }
    }
  }
  // scalar remainder (n not a multiple of V)
  if (blockIdx.x == 0) {
    const uint64_t j = nvec * V + tid;
    if (j < P.n) {
      double d;
      if (ratio_of((double)prev[j], (double)curr[j], P.cap, d)) {
        const unsigned long long k = order_key(d);
        kmin = k < kmin ? k : kmin;
        kmax = k > kmax ? k : kmax;
      } else {
        ninv += 1;
      }
    }
  }

  kmin = wave_min_u64(kmin);
  kmax = wave_max_u64(kmax);
  ninv = wave_sum_u64(ninv);
  __shared__ unsigned long long smin[RNG_TPB / 64], smax[RNG_TPB / 64], sinv[RNG_TPB / 64];
  const int w = tid / 64;
  if (lane_id() == 0) {
    smin[w] = kmin;
    smax[w] = kmax;
    sinv[w] = ninv;
  }
  __syncthreads();
  if (tid == 0) {
    for (int i = 1; i < RNG_TPB / 64; ++i) {
      kmin = smin[i] < kmin ? smin[i] : kmin;
      kmax = smax[i] > kmax ? smax[i] : kmax;
      ninv += sinv[i];
    }
    if (kmin != ~0ull) atomicMin(&P.ctl->lo_key, kmin);
    if (kmax != 0ull) atomicMax(&P.ctl->hi_key, kmax);
    if (ninv) atomicAdd(&P.ctl->n_invalid, ninv);
  }
}

// =====================================================================
// k_derive: lo, hi, M and the bin window
// =====================================================================
__global__ void k_derive(CParams P) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  Ctl* c = P.ctl;
  const unsigned long long n_valid = P.n - c->n_invalid;
  c->n_valid = n_valid;
  if (n_valid == 0) {
    c->lo = 0.0;
    c->hi = 0.0;
    c->M = 0;
    c->wbase = 0;
    c->win_len = 0;
    c->empty = 1;
    return;
  }
  const double lo = key_value(c->lo_key);
  const double hi = key_value(c->hi_key);
  c->lo = lo;
  c->hi = hi;
  const long long M = (long long)floor((hi - lo) / P.twoE) + 1;
  c->M = M;
  c->empty = 0;
  if (M <= WIN) {
    c->wbase = 0;
    c->win_len = (unsigned)M;
  } else {
    // centre the window on the bin of ratio 0 (clamped to the range): the
    // ratios of temporal data concentrate around no change.  Placement only
    // affects speed; bins outside the window are counted exactly elsewhere.
    double z = 0.0;
    z = z < lo ? lo : z;
    z = z > hi ? hi : z;
    long long m0 = bin_of(z, lo, P.twoE);
    long long b = m0 - WIN / 2;
    b = b < 0 ? 0 : b;
    b = b > M - WIN ? M - WIN : b;
    c->wbase = b;
    c->win_len = WIN;
  }
}

// =====================================================================
// k_hist: pass 2, fine histogram
// =====================================================================
constexpr int HIST_TPB = 512;
constexpr int HIST_UNROLL = 2;

// Count one element per lane: window bins in LDS (one atomic per distinct bin
// per wave), other valid points appended to the tail list (one global atomic
// per wave).
__device__ __forceinline__ void hist_count(uint32_t* lds, bool valid, long long m, long long wbase,
                                           unsigned win_len, const CParams& P) {
  const long long w = m - wbase;
  const bool inwin = valid && w >= 0 && w < (long long)win_len;
  const bool tail = valid && !inwin;
  const unsigned key = inwin ? (unsigned)w : 0xFFFFFFFFu;
  unsigned long long act = __ballot(inwin);
  while (act) {
    const int leader = __ffsll((long long)act) - 1;
    const unsigned lk = (unsigned)__builtin_amdgcn_readlane((int)key, leader);
    const unsigned long long same = __ballot(key == lk);
    if (lane_id() == leader) atomicAdd(&lds[lk], (unsigned)__popcll(same));
    act &= ~same;
  }
  const unsigned long long tm = __ballot(tail);
  if (tm) {
    const int leader = __ffsll((long long)tm) - 1;
    unsigned long long base = 0;
    if (lane_id() == leader) base = atomicAdd(&P.ctl->tail_count, (unsigned long long)__popcll(tm));
    base = __shfl(base, leader, 64);
    if (tail) {
      const unsigned long long pos = base + (unsigned long long)__popcll(tm & lanemask_lt());
      if (pos < P.tail_cap) P.tail[pos] = m;
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(HIST_TPB) k_hist(CParams P) {
  constexpr int V = Traits<T>::V;
  __shared__ uint32_t lds[WIN];
  const Ctl* c = P.ctl;
  if (c->empty) return;
  const double lo = c->lo;
  const long long wbase = c->wbase;
  const unsigned win_len = c->win_len;
  const int tid = threadIdx.x;
  for (int i = tid; i < WIN; i += HIST_TPB) lds[i] = 0u;
  __syncthreads();

  const T* __restrict__ prev = static_cast<const T*>(P.prev);
  const T* __restrict__ curr = static_cast<const T*>(P.curr);
  const uint64_t nvec = P.n / V;
  for (uint64_t vb = (uint64_t)blockIdx.x * (HIST_TPB * HIST_UNROLL) + tid; vb < nvec;
       vb += (uint64_t)gridDim.x * (HIST_TPB * HIST_UNROLL)) {
    T pv[HIST_UNROLL][V], qv[HIST_UNROLL][V];
#pragma unroll
    for (int u = 0; u < HIST_UNROLL; ++u) {
      const uint64_t vi = vb + (uint64_t)u * HIST_TPB;
      if (vi < nvec) {
        load_vec(prev, vi, pv[u]);
        load_vec(curr, vi, qv[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < HIST_UNROLL; ++u) {
      const uint64_t vi = vb + (uint64_t)u * HIST_TPB;
      const bool inr = vi < nvec;
#pragma unroll
      for (int v = 0; v < V; ++v) {
        double d = 0.0;
        const bool valid =
            inr && ratio_of((double)pv[u][v], (double)qv[u][v], P.cap, d);
        const long long m = valid ? bin_of(d, lo, P.twoE) : 0;
        hist_count(lds, valid, m, wbase, win_len, P);
      }
    }
  }
  if (blockIdx.x == 0) {
    const uint64_t j = nvec * V + tid;
    double d = 0.0;
    bool valid = false;
    if (j < P.n) valid = ratio_of((double)prev[j], (double)curr[j], P.cap, d);
    const long long m = valid ? bin_of(d, lo, P.twoE) : 0;
    hist_count(lds, valid, m, wbase, win_len, P);
  }
  __syncthreads();
  for (unsigned i = tid; i < win_len; i += HIST_TPB) {
    const uint32_t v = lds[i];
    if (v) atomicAdd(&P.gwin[i], v);
  }
}

// =====================================================================
// tail bins: exact counts in an open-addressing hash table
// =====================================================================
__device__ __forceinline__ unsigned long long hash_id(long long id) {
  unsigned long long x = (unsigned long long)id * 0x9E3779B97F4A7C15ull;
  return x ^ (x >> 29);
}

__device__ __forceinline__ unsigned long long next_pow2(unsigned long long x) {
  unsigned long long p = 1;
  while (p < x) p <<= 1;
  return p;
}

__global__ void k_hclear(CParams P) {
  Ctl* c = P.ctl;
  const unsigned long long T = c->tail_count;
  const unsigned long long used = T < P.tail_cap ? T : P.tail_cap;
  unsigned long long H = next_pow2(2 * used > 1024 ? 2 * used : 1024);
  H = H < P.hcap ? H : P.hcap;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    c->H = H;
    c->tail_used = used;
    if (T > P.tail_cap) c->flags |= NUMARCK_FLAG_TAIL_OVERFLOW;
  }
  if (used == 0) return;
  const uint64_t gt = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t gs = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = gt; i < H; i += gs) {
    P.hslot[i] = HEMPTY;
    P.hcnt[i] = 0u;
  }
}

__global__ void k_hinsert(CParams P) {
  const Ctl* c = P.ctl;
  const unsigned long long used = c->tail_used;
  const unsigned long long mask = c->H - 1;
  const uint64_t gt = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t gs = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = gt; i < used; i += gs) {
    const long long id = P.tail[i];
    unsigned long long h = hash_id(id) & mask;
    while (true) {  // load factor <= 1/2: a free or matching slot exists
      const uint32_t old = atomicCAS(&P.hslot[h], HEMPTY, (uint32_t)i);
      if (old == HEMPTY || P.tail[old] == id) {
        atomicAdd(&P.hcnt[h], 1u);
        break;
      }
      h = (h + 1) & mask;
    }
  }
}

// =====================================================================
// k_select: top-k over the window and the tail bins (one workgroup)
// =====================================================================
constexpr int SEL_TPB = 1024;
constexpr int SEL_DIGIT = 11;
constexpr int SEL_BUCKETS = 1 << SEL_DIGIT;

struct Cand {
  long long id;
  uint32_t cnt;
};

// Candidate i: i < win_len is window bin wbase + i, otherwise hash slot
// i - win_len (count 0 when the slot is empty).
__device__ __forceinline__ Cand cand_at(const CParams& P, uint64_t i, long long wbase,
                                        unsigned win_len) {
  Cand c;
  if (i < win_len) {
    c.id = wbase + (long long)i;
    c.cnt = P.gwin[i];
  } else {
    const uint64_t s = i - win_len;
    const uint32_t slot = P.hslot[s];
    if (slot == HEMPTY) {
      c.id = -1;
      c.cnt = 0;
    } else {
      c.id = P.tail[slot];
      c.cnt = P.hcnt[s];
    }
  }
  return c;
}

// Block-wide sum of one value per thread (SEL_TPB threads).
__device__ unsigned long long sel_block_sum(unsigned long long v, unsigned long long* red) {
  v = wave_sum_u64(v);
  const int w = threadIdx.x / 64;
  __syncthreads();
  if (lane_id() == 0) red[w] = v;
  __syncthreads();
  unsigned long long t = 0;
  for (int i = 0; i < SEL_TPB / 64; ++i) t += red[i];
  __syncthreads();
  return t;
}

// Add one to bucket `b` for every lane with `on`, one LDS atomic per distinct bucket.
__device__ __forceinline__ void bucket_add(uint32_t* hist, bool on, unsigned b) {
  const unsigned key = on ? b : 0xFFFFFFFFu;
  unsigned long long act = __ballot(on);
  while (act) {
    const int leader = __ffsll((long long)act) - 1;
    const unsigned lk = (unsigned)__builtin_amdgcn_readlane((int)key, leader);
    const unsigned long long same = __ballot(key == lk);
    if (lane_id() == leader) atomicAdd(&hist[lk], (unsigned)__popcll(same));
    act &= ~same;
  }
}

// Find, scanning buckets from the top (descending=true) or bottom, the bucket
// where the running count reaches `target` (1-based).  Returns the bucket and
// the count strictly before it in scan order.
__device__ void scan_buckets(const uint32_t* hist, unsigned long long target, bool descending,
                             unsigned* out_bucket, unsigned long long* out_before,
                             unsigned long long* red) {
  // one wave: each lane owns 32 consecutive buckets in scan order
  __shared__ unsigned s_bucket;
  __shared__ unsigned long long s_before;
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    unsigned long long mine = 0;
    for (int i = 0; i < SEL_BUCKETS / 64; ++i) {
      const int pos = lane * (SEL_BUCKETS / 64) + i;
      const int b = descending ? SEL_BUCKETS - 1 - pos : pos;
      mine += hist[b];
    }
    // inclusive scan over lanes
    unsigned long long inc = mine;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      unsigned long long t = __shfl_up(inc, o, 64);
      if (lane >= o) inc += t;
    }
    const unsigned long long exc = inc - mine;
    const bool here = exc < target && inc >= target;
    if (here) {
      unsigned long long run = exc;
      for (int i = 0; i < SEL_BUCKETS / 64; ++i) {
        const int pos = lane * (SEL_BUCKETS / 64) + i;
        const int b = descending ? SEL_BUCKETS - 1 - pos : pos;
        if (run + hist[b] >= target) {
          s_bucket = (unsigned)b;
          s_before = run;
          break;
        }
        run += hist[b];
      }
    }
  }
  __syncthreads();
  *out_bucket = s_bucket;
  *out_before = s_before;
  (void)red;
}

template <typename T>
__global__ void __launch_bounds__(SEL_TPB) k_select(CParams P) {
  __shared__ uint32_t hist[SEL_BUCKETS];
  __shared__ unsigned long long red[SEL_TPB / 64];
  __shared__ unsigned long long s_scan[SEL_TPB];
  Ctl* c = P.ctl;
  const int tid = threadIdx.x;
  const uint32_t k = P.k;
  const uint64_t ncent = (uint64_t)k + 1;

  // centres and bin ids start cleared
  T* centers = static_cast<T*>(P.centers);
  for (uint64_t i = tid; i < ncent; i += SEL_TPB) centers[i] = (T)0;
  if (P.bin_ids)
    for (uint64_t i = tid; i < k; i += SEL_TPB) P.bin_ids[i] = -1;

  const bool empty = c->empty != 0;
  const long long wbase = empty ? 0 : c->wbase;
  const unsigned win_len = empty ? 0u : c->win_len;
  const unsigned long long H = (empty || c->tail_used == 0) ? 0ull : c->H;
  const uint64_t ncand = (uint64_t)win_len + H;
  const double lo = empty ? 0.0 : c->lo;

  // ---- pass 0: number of nonzero bins and the largest count
  unsigned long long nz = 0, mx = 0;
  for (uint64_t i = tid; i < ncand; i += SEL_TPB) {
    const Cand cd = cand_at(P, i, wbase, win_len);
    if (cd.cnt) {
      nz += 1;
      mx = cd.cnt > mx ? cd.cnt : mx;
    }
  }
  nz = sel_block_sum(nz, red);
  {
    mx = wave_max_u64(mx);
    if (lane_id() == 0) red[tid / 64] = mx;
    __syncthreads();
    unsigned long long t = 0;
    for (int i = 0; i < SEL_TPB / 64; ++i) t = red[i] > t ? red[i] : t;
    mx = t;
    __syncthreads();
  }

  unsigned tau = 0;
  long long cut = -1;
  if (nz > k) {
    // ---- tau = k-th largest count, radix select from the top digit
    unsigned long long target = k;  // rank from the top, 1-based
    unsigned prefix = 0;
    int top = 0;
    while (top < 32 && (mx >> top) != 0) top += SEL_DIGIT;
    for (int shift = top - SEL_DIGIT; shift >= 0; shift -= SEL_DIGIT) {
      for (int i = tid; i < SEL_BUCKETS; i += SEL_TPB) hist[i] = 0u;
      __syncthreads();
      const unsigned long long hmask = (shift + SEL_DIGIT >= 32) ? 0ull
                                       : (~0ull << (shift + SEL_DIGIT)) & 0xFFFFFFFFull;
      for (uint64_t i0 = 0; i0 < ncand; i0 += SEL_TPB) {
        const uint64_t i = i0 + tid;
        Cand cd;
        cd.cnt = 0;
        if (i < ncand) cd = cand_at(P, i, wbase, win_len);
        const bool on = cd.cnt != 0 && ((cd.cnt & hmask) == (prefix & hmask));
        bucket_add(hist, on, (cd.cnt >> shift) & (SEL_BUCKETS - 1));
      }
      __syncthreads();
      unsigned b;
      unsigned long long before;
      scan_buckets(hist, target, true, &b, &before, red);
      target -= before;
      prefix |= b << shift;
      __syncthreads();
    }
    tau = prefix;
    // ---- ties: the r lowest ids among count == tau
    unsigned long long gt = 0, ties = 0, tmin = ~0ull, tmax = 0;
    for (uint64_t i = tid; i < ncand; i += SEL_TPB) {
      const Cand cd = cand_at(P, i, wbase, win_len);
      if (cd.cnt > tau) gt += 1;
      if (cd.cnt == tau && cd.cnt) {
        ties += 1;
        tmin = (unsigned long long)cd.id < tmin ? (unsigned long long)cd.id : tmin;
        tmax = (unsigned long long)cd.id > tmax ? (unsigned long long)cd.id : tmax;
      }
    }
    gt = sel_block_sum(gt, red);
    ties = sel_block_sum(ties, red);
    tmin = wave_min_u64(tmin);
    tmax = wave_max_u64(tmax);
    if (lane_id() == 0) red[tid / 64] = tmin;
    __syncthreads();
    unsigned long long t0 = ~0ull;
    for (int i = 0; i < SEL_TPB / 64; ++i) t0 = red[i] < t0 ? red[i] : t0;
    __syncthreads();
    if (lane_id() == 0) red[tid / 64] = tmax;
    __syncthreads();
    unsigned long long t1 = 0;
    for (int i = 0; i < SEL_TPB / 64; ++i) t1 = red[i] > t1 ? red[i] : t1;
    __syncthreads();
    tmin = t0;
    tmax = t1;
    const unsigned long long r = (unsigned long long)k - gt;  // ties to take, >= 1
    if (r >= ties) {
      cut = (long long)tmax;
    } else {
      // radix select the r-th smallest (id - tmin) among the ties
      const unsigned long long span = tmax - tmin;
      int topb = 0;
      while (topb < 64 && (span >> topb) != 0) topb += SEL_DIGIT;
      unsigned long long pre = 0;
      unsigned long long tgt = r;
      for (int shift = topb - SEL_DIGIT; shift >= 0; shift -= SEL_DIGIT) {
        for (int i = tid; i < SEL_BUCKETS; i += SEL_TPB) hist[i] = 0u;
        __syncthreads();
        const unsigned long long hmask =
            (shift + SEL_DIGIT >= 64) ? 0ull : (~0ull << (shift + SEL_DIGIT));
        for (uint64_t i0 = 0; i0 < ncand; i0 += SEL_TPB) {
          const uint64_t i = i0 + tid;
          Cand cd;
          cd.cnt = 0;
          cd.id = 0;
          if (i < ncand) cd = cand_at(P, i, wbase, win_len);
          const unsigned long long rel = (unsigned long long)cd.id - tmin;
          const bool on = cd.cnt == tau && cd.cnt != 0 && ((rel & hmask) == (pre & hmask));
          bucket_add(hist, on, (unsigned)((rel >> shift) & (SEL_BUCKETS - 1)));
        }
        __syncthreads();
        unsigned b;
        unsigned long long before;
        scan_buckets(hist, tgt, false, &b, &before, red);
        tgt -= before;
        pre |= (unsigned long long)b << shift;
        __syncthreads();
      }
      cut = (long long)(tmin + pre);
    }
  }
  // selected <=> cnt > tau, or cnt == tau (nonzero) and id <= cut
  // ---- selected tail bins: counts and the ones below the window
  unsigned long long sel_tail = 0, sel_below = 0;
  __shared__ unsigned s_tail_pos;
  if (tid == 0) s_tail_pos = 0;
  __syncthreads();
  for (uint64_t i = (uint64_t)win_len + tid; i < ncand; i += SEL_TPB) {
    const Cand cd = cand_at(P, i, wbase, win_len);
    const bool s = cd.cnt != 0 && (cd.cnt > tau || (cd.cnt == tau && cd.id <= cut));
    if (s) {
      sel_tail += 1;
      if (cd.id < wbase) sel_below += 1;
      const unsigned pos = atomicAdd(&s_tail_pos, 1u);
      P.sel_tail[pos] = cd.id;
    }
  }
  sel_tail = sel_block_sum(sel_tail, red);
  sel_below = sel_block_sum(sel_below, red);

  // ---- window: LUT and ranks.  Thread t owns bins [t*per, (t+1)*per).
  constexpr int PER = WIN / SEL_TPB;
  unsigned mine = 0;
  for (int q = 0; q < PER; ++q) {
    const unsigned w = tid * PER + q;
    if (w < win_len) {
      const uint32_t cn = P.gwin[w];
      const long long id = wbase + (long long)w;
      mine += (cn != 0 && (cn > tau || (cn == tau && id <= cut))) ? 1u : 0u;
    }
  }
  s_scan[tid] = mine;
  __syncthreads();
  if (tid == 0) {  // exclusive scan over 1024 partial counts
    unsigned long long run = 0;
    for (int i = 0; i < SEL_TPB; ++i) {
      const unsigned long long t = s_scan[i];
      s_scan[i] = run;
      run += t;
    }
    c->nsel_window = (unsigned)run;
  }
  __syncthreads();
  unsigned rank = (unsigned)(sel_below + s_scan[tid]);
  for (int q = 0; q < PER; ++q) {
    const unsigned w = tid * PER + q;
    uint16_t l = NOSEL;
    if (w < win_len) {
      const uint32_t cn = P.gwin[w];
      const long long id = wbase + (long long)w;
      if (cn != 0 && (cn > tau || (cn == tau && id <= cut))) {
        l = (uint16_t)rank;
        centers[rank] = (T)centre_of<T>(id, lo, P.E);
        if (P.bin_ids) P.bin_ids[rank] = id;
        rank += 1;
      }
    }
    P.lut[w] = l;
  }
  if (tid == 0) {
    c->n_nonzero = nz;
    c->tau = tau;
    c->cut = cut;
    c->k_used = (unsigned)(nz < k ? nz : k);
    c->nsel_tail = (unsigned)sel_tail;
    c->nsel_tail_below = (unsigned)sel_below;
  }
}

// =====================================================================
// k_tailrank: order the selected tail bins (t <= 65535, usually 0)
// =====================================================================
constexpr int TR_TPB = 256;

template <typename T>
__global__ void __launch_bounds__(TR_TPB) k_tailrank(CParams P) {
  __shared__ long long chunk[TR_TPB];
  const Ctl* c = P.ctl;
  const unsigned t = c->nsel_tail;
  if (t == 0) return;
  const long long wbase = c->wbase;
  const unsigned nwin = c->nsel_window;
  const double lo = c->lo;
  T* centers = static_cast<T*>(P.centers);
  for (uint64_t base = (uint64_t)blockIdx.x * TR_TPB; base < t;
       base += (uint64_t)gridDim.x * TR_TPB) {
    const uint64_t i = base + threadIdx.x;
    const long long id = i < t ? P.sel_tail[i] : 0;
    unsigned r = 0;
    for (unsigned j0 = 0; j0 < t; j0 += TR_TPB) {
      __syncthreads();
      if (j0 + threadIdx.x < t) chunk[threadIdx.x] = P.sel_tail[j0 + threadIdx.x];
      __syncthreads();
      const unsigned lim = t - j0 < (unsigned)TR_TPB ? t - j0 : (unsigned)TR_TPB;
      for (unsigned j = 0; j < lim; ++j) r += chunk[j] < id ? 1u : 0u;
    }
    if (i < t) {
      P.sorted_tail[r] = id;
      const unsigned idx = r + (id > wbase ? nwin : 0u);
      centers[idx] = (T)centre_of<T>(id, lo, P.E);
      if (P.bin_ids) P.bin_ids[idx] = id;
    }
  }
}

// =====================================================================
// k_encode: pass 3, index + verify + pack + compaction + block offsets
// =====================================================================
template <typename T>
__global__ void __launch_bounds__(ENC_TPB) k_encode(CParams P) {
  constexpr int V = Traits<T>::V;
  constexpr int R = ENC_TILE / (ENC_TPB * V);  // vector rounds per tile
  constexpr int NW = ENC_TPB / 64;
  using U = typename Traits<T>::U;
  __shared__ uint16_t s_lut[WIN];
  __shared__ uint16_t s_idx[ENC_TILE];
  __shared__ unsigned s_wcnt[R][NW];
  __shared__ unsigned long long s_prefix;
  __shared__ uint64_t s_tile;

  const Ctl* c = P.ctl;
  const int tid = threadIdx.x;
  const int wave = tid / 64;
  const int lane = lane_id();
  const bool empty = c->empty != 0;
  const double lo = empty ? 0.0 : c->lo;
  const long long wbase = empty ? 0 : c->wbase;
  const unsigned win_len = empty ? 0u : c->win_len;
  const unsigned nsel_tail = empty ? 0u : c->nsel_tail;
  const unsigned nsel_win = empty ? 0u : c->nsel_window;
  const uint32_t esc = P.k;
  for (unsigned i = tid; i < win_len; i += ENC_TPB) s_lut[i] = P.lut[i];

  const T* __restrict__ prev = static_cast<const T*>(P.prev);
  const T* __restrict__ curr = static_cast<const T*>(P.curr);
  T* __restrict__ incomp = static_cast<T*>(P.incomp);
  T* __restrict__ recon = static_cast<T*>(P.recon);
  const uint64_t nvec = P.n / V;
  const uint64_t tile_words = (uint64_t)ENC_TILE * P.B / 32;

  while (true) {
    __syncthreads();
    if (tid == 0) s_tile = atomicAdd(&P.ctl->tile_ticket, 1u);
    __syncthreads();
    const uint64_t tile = s_tile;
    if (tile >= P.n_tiles) break;
    const uint64_t t0 = tile * ENC_TILE;

    T pv[R][V], qv[R][V];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint64_t vi = t0 / V + (uint64_t)r * ENC_TPB + tid;
      if (vi < nvec) {
        load_vec(prev, vi, pv[r]);
        load_vec(curr, vi, qv[r]);
      } else {
#pragma unroll
        for (int v = 0; v < V; ++v) {
          const uint64_t j = vi * V + v;
          pv[r][v] = j < P.n ? prev[j] : (T)0;
          qv[r][v] = j < P.n ? curr[j] : (T)0;
        }
      }
    }

    unsigned long long emask[R][V];
    unsigned my_esc_bits[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      my_esc_bits[r] = 0;
      const uint64_t e0 = ((uint64_t)r * ENC_TPB + tid) * V;  // tile-local element
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const uint64_t j = t0 + e0 + v;
        const bool inr = j < P.n;
        const double p = (double)pv[r][v];
        const double q = (double)qv[r][v];
        double d = 0.0;
        const bool valid = inr && ratio_of(p, q, P.cap, d);
        uint32_t code = esc;
        T rv = qv[r][v];
        if (valid) {
          const long long m = bin_of(d, lo, P.twoE);
          const long long w = m - wbase;
          int sel = -1;
          if (w >= 0 && w < (long long)win_len) {
            const uint16_t l = s_lut[w];
            if (l != NOSEL) sel = l;
          } else if (nsel_tail) {
            // binary search among the selected tail bins
            unsigned a = 0, b = nsel_tail;
            while (a < b) {
              const unsigned mid = (a + b) >> 1;
              if (P.sorted_tail[mid] < m) a = mid + 1; else b = mid;
            }
            if (a < nsel_tail && P.sorted_tail[a] == m) sel = (int)(a + (m > wbase ? nsel_win : 0u));
          }
          if (sel >= 0) {
            const double cc = centre_of<T>(m, lo, P.E);
            const T r_t = (T)(p * (1.0 + cc));
            if (fabs((double)r_t - q) <= P.E * fabs(p)) {
              code = (uint32_t)sel;
              rv = r_t;
            }
          }
        }
        const bool is_esc = inr && code == esc;
        if (!inr) code = 0;
        s_idx[e0 + v] = (uint16_t)code;
        emask[r][v] = __ballot(is_esc);
        my_esc_bits[r] |= (is_esc ? 1u : 0u) << v;
        if (recon) pv[r][v] = rv;  // reuse the register for the reconstruction
      }
      unsigned wc = 0;
#pragma unroll
      for (int v = 0; v < V; ++v) wc += (unsigned)__popcll(emask[r][v]);
      if (lane == 0) s_wcnt[r][wave] = wc;
    }
    if (recon) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const uint64_t vi = t0 / V + (uint64_t)r * ENC_TPB + tid;
        if (vi < nvec) {
          uint4 x;
          __builtin_memcpy(&x, pv[r], 16);
          reinterpret_cast<uint4*>(recon)[vi] = x;
        } else {
#pragma unroll
          for (int v = 0; v < V; ++v) {
            const uint64_t j = vi * V + v;
            if (j < P.n) recon[j] = pv[r][v];
          }
        }
      }
    }
    __syncthreads();
    // exclusive offsets of (round, wave) groups in element order, tile total
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
    const unsigned long long tprefix = s_prefix;
    const unsigned long long lt = lanemask_lt();

    // incompressible values and block offsets
    const bool single_boundary = P.epb >= (uint64_t)ENC_TILE;
    const uint64_t first_b = (t0 + P.epb - 1) / P.epb * P.epb;  // first boundary >= t0
#pragma unroll
    for (int r = 0; r < R; ++r) {
      unsigned below = 0;
#pragma unroll
      for (int v = 0; v < V; ++v) below += (unsigned)__popcll(emask[r][v] & lt);
      unsigned long long rank = tprefix + s_wcnt[r][wave] + below;
      const uint64_t e0 = ((uint64_t)r * ENC_TPB + tid) * V;
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const uint64_t j = t0 + e0 + v;
        if (j < P.n) {
          const bool at_b = single_boundary ? (j == first_b) : (j % P.epb == 0);
          if (at_b) P.block_inc_off[j / P.epb] = (long long)rank;
        }
        if ((my_esc_bits[r] >> v) & 1u) {
          incomp[rank] = qv[r][v];
          rank += 1;
        }
      }
    }

    // bit-pack the tile: word w holds bits [32w, 32w + 32) of the tile's stream
    const uint64_t word0 = t0 * P.B / 32;
    for (uint64_t w = tid; w < tile_words; w += ENC_TPB) {
      if (word0 + w >= P.packed_words) break;
      const uint64_t bit0 = w * 32;
      const uint32_t e_first = (uint32_t)(bit0 / P.B);
      const uint32_t e_last = (uint32_t)((bit0 + 31) / P.B);
      uint32_t word = 0;
      for (uint32_t e = e_first; e <= e_last; ++e) {
        const uint32_t v = s_idx[e];
        const long long sh = (long long)e * P.B - (long long)bit0;
        word |= sh >= 0 ? (v << sh) : (v >> (-sh));
      }
      P.packed[word0 + w] = word;
    }
  }
}

// =====================================================================
// k_final: header
// =====================================================================
__global__ void k_final(CParams P) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const Ctl* c = P.ctl;
  numarck_header* h = P.hdr;
  const uint64_t L = P.dtype == NUMARCK_F32 ? 4 : 8;
  const unsigned long long n_inc = P.n_tiles ? (P.status[P.n_tiles - 1] & LB_VAL) : 0ull;
  h->n = P.n;
  h->n_valid = c->n_valid;
  h->n_invalid = P.n - c->n_valid;
  h->n_inc = n_inc;
  h->n_blocks = P.n_blocks;
  h->elems_per_block = P.epb;
  h->block_bytes = P.block_bytes;
  h->M = c->M;
  h->n_nonzero = c->n_nonzero;
  h->B = P.B;
  h->k_used = c->k_used;
  h->dtype = (uint32_t)P.dtype;
  h->flags = c->flags;
  h->tau = c->tau;
  h->reserved0 = 0;
  h->E = P.E;
  h->lo = c->lo;
  h->hi = c->hi;
  h->packed_bytes = P.packed_words * 4;
  h->compressed_bytes = ((uint64_t)1 << P.B) * L + P.packed_words * 4 + n_inc * L;
  h->tail_count = c->empty ? 0ull : c->tail_count;
  h->window_base = c->wbase;
}

// =====================================================================
// launch sequence
// =====================================================================
#define NK_LAUNCH(kind, kern, grid, block, ...)                                  \
  do {                                                                           \
    timing_begin(kind, s);                                                       \
    hipLaunchKernelGGL(kern, dim3(grid), dim3(block), 0, s, __VA_ARGS__);        \
    timing_end(kind, s);                                                         \
    hipError_t e_ = hipGetLastError();                                           \
    if (e_ != hipSuccess) return e_;                                             \
  } while (0)

template <typename T>
static hipError_t launch_compress_t(const CParams& P, hipStream_t s) {
  const Geometry g = geometry();
  constexpr int V = Traits<T>::V;
  const uint64_t nvec = P.n / V;
  uint64_t rng_blocks = (nvec + RNG_TPB * RNG_UNROLL - 1) / (RNG_TPB * RNG_UNROLL);
  const uint64_t rng_cap = (uint64_t)g.cus * 8;
  if (rng_blocks > rng_cap) rng_blocks = rng_cap;
  if (rng_blocks < 8) rng_blocks = 8;  // also clears WIN window counts
  uint64_t hist_blocks = (nvec + HIST_TPB * HIST_UNROLL - 1) / (HIST_TPB * HIST_UNROLL);
  const uint64_t hist_cap = (uint64_t)g.cus * 2;
  if (hist_blocks > hist_cap) hist_blocks = hist_cap;
  if (hist_blocks < 1) hist_blocks = 1;
  uint64_t enc_blocks = P.n_tiles;
  const uint64_t enc_cap = (uint64_t)g.cus * 3;
  if (enc_blocks > enc_cap) enc_blocks = enc_cap;
  if (enc_blocks < 1) enc_blocks = 1;
  const uint64_t aux_blocks = (uint64_t)g.cus * 2;

  NK_LAUNCH(KK_INIT, k_init, 1, 64, P.ctl);
  NK_LAUNCH(KK_RANGE, k_range<T>, rng_blocks, RNG_TPB, P);
  NK_LAUNCH(KK_DERIVE, k_derive, 1, 64, P);
  NK_LAUNCH(KK_HIST, k_hist<T>, hist_blocks, HIST_TPB, P);
  NK_LAUNCH(KK_HCLEAR, k_hclear, aux_blocks, 256, P);
  NK_LAUNCH(KK_HINSERT, k_hinsert, aux_blocks, 256, P);
  NK_LAUNCH(KK_SELECT, k_select<T>, 1, SEL_TPB, P);
  NK_LAUNCH(KK_TAILRANK, k_tailrank<T>, 256, TR_TPB, P);
  NK_LAUNCH(KK_ENCODE, k_encode<T>, enc_blocks, ENC_TPB, P);
  NK_LAUNCH(KK_FINAL, k_final, 1, 64, P);
  return hipSuccess;
}

hipError_t launch_compress(const CParams& P, hipStream_t s) {
  return P.dtype == NUMARCK_F32 ? launch_compress_t<float>(P, s)
                                : launch_compress_t<double>(P, s);
}

// =====================================================================
// histogram export (inspection)
// =====================================================================
__global__ void k_export(const Ctl* ctl, const uint32_t* gwin, const uint32_t* hslot,
                         const uint32_t* hcnt, const int64_t* tail, int64_t* ids,
                         uint32_t* counts, uint64_t capacity, unsigned long long* count) {
  const bool empty = ctl->empty != 0;
  const unsigned win_len = empty ? 0u : ctl->win_len;
  const long long wbase = empty ? 0 : ctl->wbase;
  const unsigned long long H = (empty || ctl->tail_used == 0) ? 0ull : ctl->H;
  const uint64_t ncand = (uint64_t)win_len + H;
  const uint64_t gt = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t gs = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = gt; i < ncand; i += gs) {
    long long id;
    uint32_t cn;
    if (i < win_len) {
      id = wbase + (long long)i;
      cn = gwin[i];
    } else {
      const uint32_t slot = hslot[i - win_len];
      if (slot == HEMPTY) continue;
      id = tail[slot];
      cn = hcnt[i - win_len];
    }
    if (!cn) continue;
    const unsigned long long pos = atomicAdd(count, 1ull);
    if (pos < capacity) {
      ids[pos] = id;
      counts[pos] = cn;
    }
  }
}

__global__ void k_zero_u64(unsigned long long* p) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0ull;
}

hipError_t launch_histogram_export(Ctl* ctl, const uint32_t* gwin, const uint32_t* hslot,
                                   const uint32_t* hcnt, const int64_t* tail, int64_t* ids,
                                   uint32_t* counts, uint64_t capacity, uint64_t* count_dev,
                                   hipStream_t s) {
  const Geometry g = geometry();
  unsigned long long* cnt = reinterpret_cast<unsigned long long*>(count_dev);
  NK_LAUNCH(KK_EXPORT, k_zero_u64, 1, 64, cnt);
  NK_LAUNCH(KK_EXPORT, k_export, (uint64_t)g.cus * 2, 256, ctl, gwin, hslot, hcnt, tail, ids,
            counts, capacity, cnt);
  return hipSuccess;
}

}  // namespace nk
