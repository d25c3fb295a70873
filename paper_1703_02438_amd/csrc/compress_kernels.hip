// compress_kernels.hip -- the gfx950 compression path of NUMARCK
// (arXiv 1703.02438, Sec. III-A..C and IV-A..C).
//
// One compression is a chain of kernels on one stream; every data-dependent
// quantity stays in device memory, so the host never waits between them:
//
//   k_init      reset the control block
//   k_range     pass 1: ratio + validity of every point, min/max of the valid
//               ratios, number of invalid points (Sec. IV-A); also clears the
//               window counts
//   k_hist      pass 2: fine histogram (Sec. IV-B-1), after each workgroup
//               derives lo, hi, M = floor((hi-lo)/2E)+1 and the on-chip bin
//               window from the range pass's results.  Bins inside a
//               16384-bin window are counted with LDS atomics; the ids of
//               points outside it go to a tail list
//   k_hclear / k_hinsert   exact counts of the tail bins in a hash table
//               (k_hclear also records the derived lo, hi, M and window)
//   k_select    top-k over window + tail counts: the k-th largest count tau by
//               radix select, the lowest-id ties, indices in bin order, the
//               window LUT and the centres (Sec. IV-B-1, III-B); the tail is
//               skipped when no tail bin can reach the window's k-th count
//   k_tailrank  rank of the selected tail bins (rare; O(t^2) over t <= 65535)
//   k_encode    pass 3: index + verify every point, pack the B-bit indices,
//               stage incompressible values per wave range with
//               range-relative block offsets (Sec. III-C, IV-C)
//   k_gather    each workgroup sums the escape counts of the units before its
//               own, moves the staged values to their final, element-order
//               offsets and completes the block offsets; the job's first
//               workgroup sums them all and writes the header
#include <type_traits>

#include "nk_device.h"

namespace nk {

// Job sources: the plain path passes its one job by value, a batch reads the
// job table in device memory.
struct OneJob {
  CParams p;
  __device__ __forceinline__ const CParams& job(uint32_t) const { return p; }
};
struct JobTable {
  const CParams* t;
  __device__ __forceinline__ const CParams& job(uint32_t j) const { return t[j]; }
};

// Largest j in [lo, hi) with starts[j] <= x (starts ascending).
template <typename U>
__device__ __forceinline__ uint32_t find_job(const U* starts, uint32_t lo, uint32_t hi, U x) {
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (starts[mid] <= x) lo = mid; else hi = mid;
  }
  return lo;
}

// A streaming workgroup's current job and that job's chunk span, kept in
// registers: chunks rise monotonically per workgroup, so the prefix array is
// searched only when a chunk lies past the span.
struct ChunkCursor {
  uint32_t j = 0xFFFFFFFFu;
  uint64_t first = 0, end = 0;  // chunks of job j: [first, end)

  // Moves to the job of chunk c; true if that is another job than before.
  __device__ __forceinline__ bool seek(const Geo& g, uint64_t c) {
    if (j != 0xFFFFFFFFu && c < end) return false;
    if (!g.chunk0) {
      j = g.job_begin;
      first = 0;
      end = ~0ull;
      return true;
    }
    j = find_job(g.chunk0, j == 0xFFFFFFFFu ? g.job_begin : j + 1, g.job_end, c);
    first = g.chunk0[j];
    end = g.chunk0[j + 1];
    return true;
  }
};

// =====================================================================
// k_init
// =====================================================================
template <typename S>
__global__ void k_init(S src, Geo g) {
  const CParams& P = src.job(g.job_begin + blockIdx.x);
  Ctl* ctl = P.ctl;
  if (threadIdx.x == 0) {
    ctl->lo_key = ~0ull;
    ctl->hi_key = 0ull;
    ctl->n_invalid = 0ull;
    ctl->tail_count = 0ull;
    ctl->tile_ticket = 0u;
    ctl->flags = 0u;
    ctl->tail_bins = 0u;
    ctl->tail_max = 0u;
    if (g.za) {
      // zero-anchored bins: lo = -E and the 2^14 bins around ratio 0, with
      // no range pass before the histogram; k_zafin counts the valid points
      // after it.  The header reports lo = -E, hi = 0, M = 0.
      ctl->lo = -P.E;
      ctl->hi = 0.0;
      ctl->M = 0;
      ctl->wbase = -(long long)(WIN / 2);
      ctl->win_len = WIN;
      ctl->empty = 0;
    }
  }
  for (int i = threadIdx.x; i < WIN; i += blockDim.x) gstore(P.gwin + i, 0u);
}

// =====================================================================
// k_range: pass 1 over prev/curr
// =====================================================================
constexpr int RNG_TPB = 256;
constexpr int RNG_UNROLL = 4;

// Block reduction of the running extremes and invalid count, added to the
// job's control block.  Every thread of the block calls it.
__device__ void range_flush(Ctl* ctl, unsigned long long& kmin, unsigned long long& kmax,
                            unsigned long long& ninv) {
  __shared__ unsigned long long smin[RNG_TPB / 64], smax[RNG_TPB / 64], sinv[RNG_TPB / 64];
  kmin = wave_min_u64(kmin);
  kmax = wave_max_u64(kmax);
  ninv = wave_sum_u64(ninv);
  const int w = threadIdx.x / 64;
  __syncthreads();
  if (lane_id() == 0) {
    smin[w] = kmin;
    smax[w] = kmax;
    sinv[w] = ninv;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < RNG_TPB / 64; ++i) {
      kmin = smin[i] < kmin ? smin[i] : kmin;
      kmax = smax[i] > kmax ? smax[i] : kmax;
      ninv += sinv[i];
    }
    if (kmin != ~0ull) atomicMin(&ctl->lo_key, kmin);
    if (kmax != 0ull) atomicMax(&ctl->hi_key, kmax);
    if (ninv) atomicAdd(&ctl->n_invalid, ninv);
  }
  kmin = ~0ull;
  kmax = 0ull;
  ninv = 0ull;
}

// Streaming chunks [c_begin, c_end), block-strided; a chunk is chunk_vec
// vectors of one job, and a job's last chunk also takes its scalar tail.
template <typename T, typename S, bool NT>
__global__ void __launch_bounds__(RNG_TPB) k_range(S src, Geo g) {
  constexpr int V = Traits<T>::V;
  const int tid = threadIdx.x;
  unsigned long long kmin = ~0ull, kmax = 0ull, ninv = 0ull;
  ChunkCursor cu;
  // the current job's parameters, loaded when the workgroup reaches it
  Ctl* ctl = nullptr;
  const T* prev = nullptr;
  const T* curr = nullptr;
  uint64_t n = 0, nvec = 0;
  double cap = 0.0;
  for (uint64_t c = g.c_begin + blockIdx.x; c < g.c_end; c += gridDim.x) {
    if (cu.seek(g, c)) {
      if (ctl) range_flush(ctl, kmin, kmax, ninv);
      const CParams& P = src.job(cu.j);
      ctl = P.ctl;
      prev = static_cast<const T*>(P.prev);
      curr = static_cast<const T*>(P.curr);
      n = P.n;
      nvec = n / V;
      cap = P.cap;
    }
    const uint64_t v0 = (c - cu.first) * g.chunk_vec;
    uint64_t v1 = v0 + g.chunk_vec;
    v1 = v1 < nvec ? v1 : nvec;
    for (uint64_t vb = v0 + tid; vb < v1; vb += RNG_TPB * RNG_UNROLL) {
      T pv[RNG_UNROLL][V], qv[RNG_UNROLL][V];
#pragma unroll
      for (int u = 0; u < RNG_UNROLL; ++u) {
        const uint64_t vi = vb + (uint64_t)u * RNG_TPB;
        if (vi < v1) {
          load_vec_t<NT>(prev, vi, pv[u]);
          load_vec_t<NT>(curr, vi, qv[u]);
        }
      }
#pragma unroll
      for (int u = 0; u < RNG_UNROLL; ++u) {
        const uint64_t vi = vb + (uint64_t)u * RNG_TPB;
        if (vi < v1) {
#pragma unroll
          for (int v = 0; v < V; ++v) {
            double d;
            if (ratio_of((double)pv[u][v], (double)qv[u][v], cap, d)) {
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
    if (v1 == nvec) {  // the job's last chunk: scalar remainder
      const uint64_t jj = nvec * V + tid;
      if (jj < n) {
        double d;
        if (ratio_of((double)prev[jj], (double)curr[jj], cap, d)) {
          const unsigned long long k = order_key(d);
          kmin = k < kmin ? k : kmin;
          kmax = k > kmax ? k : kmax;
        } else {
          ninv += 1;
        }
      }
    }
  }
  if (ctl) range_flush(ctl, kmin, kmax, ninv);
}

// Pass 1 over a time chain: jobs j0 .. j0 + T - 1 (T <= CHAIN_MAX) with
// one n, job t comparing snapshot t with snapshot t + 1.  Each thread holds
// CHAIN_K vectors of snapshots t and t + 1 in registers, takes the ratios of
// pair t while the same positions of snapshot t + 2 load, and moves on to
// pair t + 1: every snapshot is read once per sweep instead of twice.  A
// wave folds its extremes and invalid count of pair t into its own LDS slot
// after each step; the workgroup adds the slots to the jobs' control blocks
// once, at the end.
static_assert(RNG_TPB == 256, "chain chunks are sized for 256-thread workgroups");

template <typename T, bool NT>
__global__ void __launch_bounds__(RNG_TPB) k_range_chain(JobTable src, Geo g) {
  constexpr int V = Traits<T>::V;
  constexpr int NW = RNG_TPB / 64;
  constexpr int K = (int)CHAIN_K;
  __shared__ const T* s_in[CHAIN_MAX + 1];
  __shared__ double s_cap[CHAIN_MAX];
  __shared__ unsigned long long s_min[CHAIN_MAX][NW], s_max[CHAIN_MAX][NW], s_inv[CHAIN_MAX][NW];
  const int tid = threadIdx.x;
  const int wave = tid / 64;
  const int lane = lane_id();
  const uint32_t j0 = g.job_begin;
  const uint32_t npair = g.job_end - g.job_begin;
  for (uint32_t t = tid; t < npair; t += RNG_TPB) {
    const CParams& P = src.job(j0 + t);
    if (t == 0) s_in[0] = static_cast<const T*>(P.prev);
    s_in[t + 1] = static_cast<const T*>(P.curr);
    s_cap[t] = P.cap;
  }
  for (uint32_t i = tid; i < npair * NW; i += RNG_TPB) {
    s_min[i / NW][i % NW] = ~0ull;
    s_max[i / NW][i % NW] = 0ull;
    s_inv[i / NW][i % NW] = 0ull;
  }
  __syncthreads();
  const uint64_t n = src.job(j0).n;
  const uint64_t nvec = n / V;

  // pair t's extremes and invalid count of one step into the wave's slot
  // (the whole wave calls it)
  auto fold = [&](uint32_t t, unsigned long long kmin, unsigned long long kmax,
                  unsigned long long ninv) {
    kmin = wave_min_u64(kmin);
    kmax = wave_max_u64(kmax);
    ninv = wave_sum_u64(ninv);
    if (lane == 0) {
      s_min[t][wave] = kmin < s_min[t][wave] ? kmin : s_min[t][wave];
      s_max[t][wave] = kmax > s_max[t][wave] ? kmax : s_max[t][wave];
      s_inv[t][wave] += ninv;
    }
  };

  for (uint64_t c = g.c_begin + blockIdx.x; c < g.c_end; c += gridDim.x) {
    const uint64_t v0 = (c - g.c_begin) * g.chunk_vec;
    uint64_t v1 = v0 + g.chunk_vec;
    v1 = v1 < nvec ? v1 : nvec;
    for (uint64_t vb = v0; vb < v1; vb += (uint64_t)RNG_TPB * K) {
      // positions past the chunk load its last vector (every load is issued,
      // so the waits below count a fixed number of loads) and are skipped
      uint64_t vl[K];
      bool on[K];
#pragma unroll
      for (int u = 0; u < K; ++u) {
        const uint64_t vi = vb + (uint64_t)u * RNG_TPB + tid;
        on[u] = vi < v1;
        vl[u] = on[u] ? vi : v1 - 1;
      }
      // snapshot t in cur, t + 1 in nxt; t + 2 is loaded while pair t is
      // computed
      T cur[K][V], nxt[K][V];
#pragma unroll
      for (int u = 0; u < K; ++u) load_vec_t<NT>(s_in[0], vl[u], cur[u]);
#pragma unroll
      for (int u = 0; u < K; ++u) load_vec_t<NT>(s_in[1], vl[u], nxt[u]);
      const T* ahead = s_in[2 <= npair ? 2 : npair];
      for (uint32_t t = 0; t < npair; ++t) {
        T nn[K][V];
#pragma unroll
        for (int u = 0; u < K; ++u) load_vec_t<NT>(ahead, vl[u], nn[u]);
        // the loads go out before the arithmetic of this step
        __builtin_amdgcn_sched_barrier(0);
        ahead = s_in[t + 3 <= npair ? t + 3 : npair];
        const double cap = s_cap[t];
        unsigned long long kmin = ~0ull, kmax = 0ull, ninv = 0ull;
#pragma unroll
        for (int u = 0; u < K; ++u) {
#pragma unroll
          for (int v = 0; v < V; ++v) {
            double d;
            const bool ok = ratio_of((double)cur[u][v], (double)nxt[u][v], cap, d);
            const unsigned long long k = ok ? order_key(d) : 0ull;
            kmin = on[u] && ok && k < kmin ? k : kmin;
            kmax = on[u] && ok && k > kmax ? k : kmax;
            ninv += on[u] && !ok ? 1ull : 0ull;
          }
        }
        fold(t, kmin, kmax, ninv);
#pragma unroll
        for (int u = 0; u < K; ++u)
#pragma unroll
          for (int v = 0; v < V; ++v) {
            cur[u][v] = nxt[u][v];
            nxt[u][v] = nn[u][v];
          }
      }
    }
    if (v1 == nvec && wave == 0) {  // the last chunk: scalar remainder (< V points)
      const uint64_t jj = nvec * V + lane;
      for (uint32_t t = 0; t < npair; ++t) {
        unsigned long long kmin = ~0ull, kmax = 0ull, ninv = 0ull;
        if (jj < n) {
          double d;
          if (ratio_of((double)s_in[t][jj], (double)s_in[t + 1][jj], s_cap[t], d)) {
            kmin = kmax = order_key(d);
          } else {
            ninv = 1;
          }
        }
        fold(t, kmin, kmax, ninv);
      }
    }
  }
  __syncthreads();
  for (uint32_t t = tid; t < npair; t += RNG_TPB) {
    unsigned long long kmin = ~0ull, kmax = 0ull, ninv = 0ull;
    for (int w = 0; w < NW; ++w) {
      kmin = s_min[t][w] < kmin ? s_min[t][w] : kmin;
      kmax = s_max[t][w] > kmax ? s_max[t][w] : kmax;
      ninv += s_inv[t][w];
    }
    Ctl* ctl = src.job(j0 + t).ctl;
    if (kmin != ~0ull) atomicMin(&ctl->lo_key, kmin);
    if (kmax != 0ull) atomicMax(&ctl->hi_key, kmax);
    if (ninv) atomicAdd(&ctl->n_invalid, ninv);
  }
}

// =====================================================================
// derive_job: lo, hi, M and the bin window from the range pass's results
// =====================================================================
struct Derived {
  double lo, hi;
  long long M, wbase;
  unsigned long long n_valid;
  unsigned win_len, empty;
};

__device__ __forceinline__ Derived derive_job(const CParams& P, const Ctl* c) {
  Derived d{};
  d.n_valid = P.n - c->n_invalid;
  if (d.n_valid == 0) {
    d.empty = 1;
    return d;
  }
  d.lo = key_value(c->lo_key);
  d.hi = key_value(c->hi_key);
  d.M = (long long)floor((d.hi - d.lo) / P.twoE) + 1;
  if (d.M <= WIN) {
    d.wbase = 0;
    d.win_len = (unsigned)d.M;
  } else {
    // centre the window on the bin of ratio 0 (clamped to the range): the
    // ratios of temporal data concentrate around no change.  Placement only
    // affects speed; bins outside the window are counted exactly elsewhere.
    double z = 0.0;
    z = z < d.lo ? d.lo : z;
    z = z > d.hi ? d.hi : z;
    const long long m0 = bin_of(z, d.lo, P.twoE);
    long long b = m0 - WIN / 2;
    b = b < 0 ? 0 : b;
    b = b > d.M - WIN ? d.M - WIN : b;
    d.wbase = b;
    d.win_len = WIN;
  }
  return d;
}

// The derived fields in the control block, for the kernels after the
// histogram.
__device__ __forceinline__ void store_derived(Ctl* c, const Derived& d) {
  c->n_valid = d.n_valid;
  c->lo = d.lo;
  c->hi = d.hi;
  c->M = d.M;
  c->wbase = d.wbase;
  c->win_len = d.win_len;
  c->empty = d.empty;
}

// =====================================================================
// zero-anchored bins: the anchor is -E, so no range pass precedes the
// histogram.  k_init sets the window to the 2^14 bins around ratio 0 (lo =
// -E); k_zafin, after the histogram, counts the valid points (window counts
// plus the points outside the window).
// =====================================================================
template <typename S>
__global__ void __launch_bounds__(256) k_zafin(S src, Geo g) {
  const CParams& P = src.job(g.job_begin + blockIdx.x);
  Ctl* c = P.ctl;
  unsigned long long v = strided_sum_u32(P.gwin, threadIdx.x, WIN, 256);
  v = wave_sum_u64(v);
  __shared__ unsigned long long part[4];
  if (lane_id() == 0) part[threadIdx.x / 64] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned long long n_valid = part[0] + part[1] + part[2] + part[3] + c->tail_count;
    c->n_valid = n_valid;
    c->n_invalid = P.n - n_valid;
    if (n_valid == 0) {
      c->empty = 1;
      c->win_len = 0;
      c->wbase = 0;
    }
  }
}

// =====================================================================
// k_ewprep: equal-width binning (Sec. III-B, IV-B-3) -- the range [lo, hi]
// cut into k = 2^B - 1 chunks of width w = (hi - lo) / k, chunk i's centre
// lo + (i + 1/2) w; it takes the place of the histogram and the top-k
// selection, and leaves the control block as the encoder and the header
// expect it (no fine-bin window, k bins in use when a point is valid)
// =====================================================================
template <typename T, typename S>
__global__ void __launch_bounds__(256) k_ewprep(S src, Geo g) {
  const CParams& P = src.job(g.job_begin + blockIdx.x);
  Ctl* c = P.ctl;
  const unsigned long long n_valid = P.n - c->n_invalid;
  const bool any = n_valid != 0;
  const double lo = any ? key_value(c->lo_key) : 0.0;
  const double hi = any ? key_value(c->hi_key) : 0.0;
  const double w = (hi - lo) / (double)P.k;
  T* cen = static_cast<T*>(P.centers);
  for (uint32_t i = threadIdx.x; i <= P.k; i += blockDim.x)
    gstore(cen + i, (any && i < P.k) ? (T)(lo + ((double)i + 0.5) * w) : (T)0);
  if (P.bin_ids)
    for (uint32_t i = threadIdx.x; i < P.k; i += blockDim.x) gstore(P.bin_ids + i, (int64_t)-1);
  if (threadIdx.x == 0) {
    c->n_valid = n_valid;
    c->lo = lo;
    c->hi = hi;
    c->M = any ? (long long)P.k : 0;
    c->empty = any ? 0u : 1u;
    c->wbase = 0;
    c->win_len = 0;
    c->n_nonzero = 0;
    c->tau = 0;
    c->k_used = any ? P.k : 0u;
    c->nsel_window = 0;
    c->nsel_tail = 0;
    c->nsel_tail_below = 0;
    c->ew_w = w;
    c->ew_inv = 1.0 / w;
  }
}

// =====================================================================
// k_hist: pass 2, fine histogram
// =====================================================================
constexpr int HIST_TPB = NK_HIST_TPB;
constexpr int HIST_UNROLL = 2;

// Where a job's out-of-window points go: the tail list and its fill count.
struct TailSink {
  unsigned long long* count;
  int64_t* list;
  uint64_t cap;
};

// Append the bin id m of every lane with `tail` to the tail list (one global
// atomic per wave).  The whole wave calls it.
__device__ __forceinline__ void tail_append(bool tail, double m, const TailSink& ts) {
  const unsigned long long tm = __ballot(tail);
  if (tm) {
    const int leader = __ffsll((long long)tm) - 1;
    unsigned long long base = 0;
    if (lane_id() == leader) base = atomicAdd(ts.count, (unsigned long long)__popcll(tm));
    const unsigned lo32 = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)base, leader);
    const unsigned hi32 = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(base >> 32), leader);
    base = ((unsigned long long)hi32 << 32) | lo32;
    if (tail) {
      const unsigned long long pos = base + (unsigned long long)__popcll(tm & lanemask_lt());
      if (pos < ts.cap) gstore(ts.list + pos, (int64_t)m);
    }
  }
}

// Count one element per lane: window bins with atomics on `win` (LDS or the
// job's global window counts), other valid points appended to the tail list.
__device__ __forceinline__ void hist_count(uint32_t* win, bool valid, double m, double wbase_d,
                                           double wlen_d, const TailSink& ts) {
  const double w = m - wbase_d;  // exact: both are integers below 2^51
  const bool inwin = valid && w >= 0.0 && w < wlen_d;
  if (inwin) atomicAdd(&win[(int)w], 1u);
  tail_append(valid && !inwin, m, ts);
}

// LDSH: count window bins in an LDS copy flushed to the job's global counts
// when the block moves to another job (or finishes); otherwise count
// directly in the global counts (more atomic traffic, no LDS, higher
// occupancy).  Same counts either way.
template <typename T, typename S, bool LDSH, int NT>
__global__ void __launch_bounds__(HIST_TPB) k_hist(S src, Geo g) {
  constexpr int V = Traits<T>::V;
  // the window, then one slot per lane for points outside it (never read):
  // every lane adds to some slot, so the count needs no branch
  __shared__ uint32_t lds[LDSH ? WIN + 64 : 1];
  const int tid = threadIdx.x;
  if (LDSH) {
    for (int i = tid; i < WIN; i += HIST_TPB) lds[i] = 0u;
    __syncthreads();
  }
  ChunkCursor cu;
  // The current job's parameters and window, loaded once when the workgroup
  // reaches the job: inside a saturated stream a dependent load per chunk
  // would stall every wave of the workgroup.
  bool have = false, empty = true;
  double lo = 0.0, wbase_d = 0.0, wlen_d = 0.0, cap = 0.0, twoE = 1.0, inv2E = 1.0;
  double cap_lo = 0.0, cap_hi = 0.0, inv_err = 0.0, E = 0.0;
  unsigned wl = 0;
  uint32_t* gwin = nullptr;
  uint16_t* wc = nullptr;  // window codes to write (precoded encoding), or null
  const T* prev = nullptr;
  const T* curr = nullptr;
  uint64_t n = 0, nvec = 0;
  TailSink ts{nullptr, nullptr, 0};
  // Points outside the window: each wave gathers their bin ids in its own
  // LDS buffer and appends a full buffer to the job's tail list with one
  // global atomic (a returning atomic per point on the one tail counter
  // stalls the stream wherever the tail is dense).
  __shared__ long long s_tbuf[LDSH ? HIST_TPB / 64 : 1][64];
  const int wave = tid / 64;
  const int lane = tid & 63;
  unsigned tbn = 0;  // entries in this wave's buffer (wave-uniform)
  auto tail_flush = [&]() {  // the whole wave calls it
    if (tbn == 0) return;
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(ts.count, (unsigned long long)tbn);
    const unsigned lo32 = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)base, 0);
    const unsigned hi32 = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(base >> 32), 0);
    base = ((unsigned long long)hi32 << 32) | lo32;
    wave_lds_sync();
    if ((unsigned)lane < tbn && base + lane < ts.cap) gstore(ts.list + base + lane, (int64_t)s_tbuf[wave][lane]);
    wave_lds_sync();
    tbn = 0;
  };
  auto tail_push = [&](bool tail, double m) {  // the whole wave calls it
    const unsigned long long tm = __ballot(tail);
    if (!tm) return;
    const unsigned cnt = (unsigned)__popcll(tm);
    if (tbn + cnt > 64u) tail_flush();
    if (tail) s_tbuf[wave][tbn + (unsigned)__popcll(tm & lanemask_lt())] = (long long)m;
    tbn += cnt;
  };
  auto flush = [&]() {  // LDS window counts to the job's global counts
    if (!LDSH) return;
    tail_flush();
    __syncthreads();
    for (unsigned i = tid; i < (unsigned)WIN; i += HIST_TPB) {
      const uint32_t v = lds[i];
      if (v && i < wl) atomicAdd(&gwin[i], v);
      lds[i] = 0u;
    }
    __syncthreads();
  };
  // Chunks block-strided over the group.  In a time chain, workgroup b works
  // on job (b mod T) only, taking its chunks b / T, b / T + G / T, ... (G / T
  // workgroups per job): consecutive jobs read the snapshot they share at the
  // same positions at about the same time, and its second read can hit the
  // Infinity Cache.  Workgroups past (G / T) T have nothing to do.
  uint64_t c0 = g.c_begin + blockIdx.x, cend = g.c_end, cstep = gridDim.x;
  if (g.chain) {
    const uint32_t nj = g.job_end - g.job_begin;
    const uint32_t per = gridDim.x / nj;
    const uint32_t j = g.job_begin + blockIdx.x % nj;
    cend = g.chunk0[j + 1];
    c0 = blockIdx.x < per * nj ? g.chunk0[j] + blockIdx.x / nj : cend;
    cstep = per;
  }
  for (uint64_t c = c0; c < cend; c += cstep) {
    if (cu.seek(g, c)) {
      if (have) flush();
      have = true;
      const CParams& P = src.job(cu.j);
      const Ctl* ctl = P.ctl;
      Derived d;
      if (g.za) {  // set by k_init
        d.empty = ctl->empty;
        d.win_len = ctl->win_len;
        d.lo = ctl->lo;
        d.wbase = ctl->wbase;
      } else {
        d = derive_job(P, ctl);
      }
      empty = d.empty != 0;
      wl = empty ? 0u : d.win_len;
      lo = d.lo;
      wbase_d = (double)d.wbase;
      wlen_d = (double)wl;
      gwin = P.gwin;
      prev = static_cast<const T*>(P.prev);
      curr = static_cast<const T*>(P.curr);
      n = P.n;
      nvec = n / V;
      cap = P.cap;
      cap_lo = cap_below(cap);
      cap_hi = cap_above(cap);
      twoE = P.twoE;
      inv2E = P.inv2E;
      inv_err = inv2E * 0x1p-36;
      E = P.E;
      wc = LDSH && P.pre ? P.wcode : nullptr;
      ts = TailSink{&P.ctl->tail_count, P.tail, P.tail_cap};
    }
    if (empty) continue;  // uniform: the whole chunk belongs to this job
    uint32_t* win = LDSH ? lds : gwin;
    const uint64_t v0 = (c - cu.first) * g.chunk_vec;
    uint64_t v1 = v0 + g.chunk_vec;
    v1 = v1 < nvec ? v1 : nvec;
    // every lane runs every step (the bound is the workgroup's, not the
    // lane's): the tail buffer's flush needs the whole wave
    for (uint64_t vs = v0; vs < v1; vs += HIST_TPB * HIST_UNROLL) {
      const uint64_t vb = vs + tid;
      T pv[HIST_UNROLL][V], qv[HIST_UNROLL][V];
#pragma unroll
      for (int u = 0; u < HIST_UNROLL; ++u) {
        const uint64_t vi = vb + (uint64_t)u * HIST_TPB;
        if (vi < v1) {
          load_vec_t<NT != 0>(prev, vi, pv[u]);
          load_vec_t<NT == 1>(curr, vi, qv[u]);
        }
      }
      if constexpr (LDSH) {
        // window points counted without branches; the (rare) points outside
        // the window go to the tail list after one test for the whole step
        double mt[HIST_UNROLL][V];
        bool tl[HIST_UNROLL][V];
        bool anyt = false;
#pragma unroll
        for (int u = 0; u < HIST_UNROLL; ++u) {
          const uint64_t vi = vb + (uint64_t)u * HIST_TPB;
          const bool inr = vi < v1;
          // the vector's window codes, element v in bits [16 v, 16 v + 16)
          typename std::conditional<V == 2, uint32_t, unsigned long long>::type cw = 0;
#pragma unroll
          for (int v = 0; v < V; ++v) {
            bool vf;
            const double mf = ratio_bin((double)pv[u][v], (double)qv[u][v], cap, cap_lo, cap_hi,
                                        lo, twoE, inv2E, inv_err, vf);
            const bool valid = inr && vf;
            const double m = valid ? mf : 0.0;
            const double w = m - wbase_d;  // exact: both are integers below 2^51
            const bool inwin = valid && w >= 0.0 && w < wlen_d;
            atomicAdd(&lds[inwin ? (int)w : WIN + (tid & 63)], 1u);
            mt[u][v] = m;
            tl[u][v] = valid && !inwin;
            anyt |= tl[u][v];
            if (wc) {  // uniform
              uint32_t code = valid ? WC_TAIL : WC_INVALID;
              if (inwin) {
                // the check the encoder makes with this bin's centre (Sec. III-C)
                const double p = (double)pv[u][v], q = (double)qv[u][v];
                const T r_t = (T)(p * (1.0 + centre_of_d<T>(m, lo, E)));
                const bool ok = fabs((double)r_t - q) <= E * fabs(p);
                code = (uint32_t)(int)w | (ok ? WC_OK : 0u);
              }
              cw |= (decltype(cw))code << (16 * v);
            }
          }
          if (wc && inr) gstore(reinterpret_cast<decltype(cw)*>(wc) + vi, cw);
        }
        if (__ballot(anyt)) {
#pragma unroll
          for (int u = 0; u < HIST_UNROLL; ++u)
#pragma unroll
            for (int v = 0; v < V; ++v) tail_push(tl[u][v], mt[u][v]);
        }
      } else {
#pragma unroll
        for (int u = 0; u < HIST_UNROLL; ++u) {
          const uint64_t vi = vb + (uint64_t)u * HIST_TPB;
          const bool inr = vi < v1;
#pragma unroll
          for (int v = 0; v < V; ++v) {
            bool vf;
            const double mf = ratio_bin((double)pv[u][v], (double)qv[u][v], cap, cap_lo, cap_hi,
                                        lo, twoE, inv2E, inv_err, vf);
            const bool valid = inr && vf;
            const double m = valid ? mf : 0.0;
            hist_count(win, valid, m, wbase_d, wlen_d, ts);
          }
        }
      }
    }
    if (v1 == nvec) {  // the job's last chunk: scalar remainder
      const uint64_t jj = nvec * V + tid;
      double d = 0.0;
      bool valid = false;
      if (jj < n) valid = ratio_of((double)prev[jj], (double)curr[jj], cap, d);
      const double m = valid ? bin_floor(d - lo, twoE, inv2E) : 0.0;
      hist_count(win, valid, m, wbase_d, wlen_d, ts);
      if (wc && jj < n) {
        const double w = m - wbase_d;
        const bool inwin = valid && w >= 0.0 && w < wlen_d;
        uint16_t code = valid ? WC_TAIL : WC_INVALID;
        if (inwin) {
          const double p = (double)prev[jj], q = (double)curr[jj];
          const T r_t = (T)(p * (1.0 + centre_of_d<T>(m, lo, E)));
          code = (uint16_t)((int)w | (fabs((double)r_t - q) <= E * fabs(p) ? WC_OK : 0));
        }
        gstore(wc + jj, code);
      }
    }
  }
  if (have) flush();
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

template <typename S>
__global__ void k_hclear(S src, Geo g) {
  const CParams& P = src.job(g.job_begin + blockIdx.y);
  Ctl* c = P.ctl;
  if (!g.za && blockIdx.x == 0 && threadIdx.x == 0) store_derived(c, derive_job(P, c));
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

// One tail point per thread and step; the distinct-bin count and the
// largest count are reduced per workgroup before one pair of atomics on the
// control block.
template <typename S>
__global__ void __launch_bounds__(256) k_hinsert(S src, Geo g) {
  const CParams& P = src.job(g.job_begin + blockIdx.y);
  const Ctl* c = P.ctl;
  const unsigned long long used = c->tail_used;
  const unsigned long long mask = c->H - 1;
  const uint64_t gt = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t gs = (uint64_t)gridDim.x * blockDim.x;
  if ((uint64_t)blockIdx.x * blockDim.x >= used) return;  // whole workgroups
  unsigned long long fresh = 0, top = 0;
  for (uint64_t i = gt; i < used; i += gs) {
    const long long id = P.tail[i];
    unsigned long long h = hash_id(id) & mask;
    while (true) {  // load factor <= 1/2: a free or matching slot exists
      const uint32_t old = atomicCAS(&P.hslot[h], HEMPTY, (uint32_t)i);
      if (old == HEMPTY || P.tail[old] == id) {
        const uint32_t before = atomicAdd(&P.hcnt[h], 1u);
        top = before + 1 > top ? before + 1 : top;
        fresh += old == HEMPTY ? 1 : 0;
        break;
      }
      h = (h + 1) & mask;
    }
  }
  // distinct tail bins and the largest final count (the last increment of a
  // bin returns its final count minus one), per workgroup
  __shared__ unsigned long long s_f[4], s_t[4];
  fresh = wave_sum_u64(fresh);
  top = wave_max_u64(top);
  if (lane_id() == 0) {
    s_f[threadIdx.x / 64] = fresh;
    s_t[threadIdx.x / 64] = top;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long f = 0, t = 0;
    for (int w = 0; w < 4; ++w) {
      f += s_f[w];
      t = s_t[w] > t ? s_t[w] : t;
    }
    if (f) atomicAdd(&P.ctl->tail_bins, (unsigned)f);
    if (t) atomicMax(&P.ctl->tail_max, (unsigned)t);
  }
}

// =====================================================================
// k_select: top-k over the window and the tail bins (one workgroup)
// =====================================================================
// The window counts are staged in LDS.  tau (the k-th largest count) and the
// tie cut are found by MSD radix select with 2048-bucket LDS histograms.  If
// the window alone holds k nonzero bins, its k-th count tau_w bounds tau from
// below; when every tail bin count is smaller than tau_w (k_hinsert records
// the largest), no tail bin can be selected or tie, and the tail is never
// read.  Otherwise the hash table's slots are visited too.
constexpr int SEL_TPB = 1024;
constexpr int SEL_DIGIT = 11;
constexpr int SEL_BUCKETS = 1 << SEL_DIGIT;

struct SelShared {
  uint32_t win[WIN];
  uint32_t hist[SEL_BUCKETS];
  unsigned long long red[SEL_TPB / 64];
  unsigned long long red4[SEL_TPB / 64][4];
  unsigned bucket;
  unsigned long long before;
  unsigned tail_pos;
};

// Four block-wide reductions at once: sums of a and b, min of c, max of d.
__device__ void sel_reduce4(unsigned long long& a, unsigned long long& b, unsigned long long& c,
                            unsigned long long& d, SelShared& S) {
  a = wave_sum_u64(a);
  b = wave_sum_u64(b);
  c = wave_min_u64(c);
  d = wave_max_u64(d);
  __syncthreads();
  if (lane_id() == 0) {
    const int w = threadIdx.x / 64;
    S.red4[w][0] = a;
    S.red4[w][1] = b;
    S.red4[w][2] = c;
    S.red4[w][3] = d;
  }
  __syncthreads();
  a = 0;
  b = 0;
  c = ~0ull;
  d = 0;
  for (int i = 0; i < SEL_TPB / 64; ++i) {
    a += S.red4[i][0];
    b += S.red4[i][1];
    c = S.red4[i][2] < c ? S.red4[i][2] : c;
    d = S.red4[i][3] > d ? S.red4[i][3] : d;
  }
  __syncthreads();
}

// Block-wide exclusive prefix sum of one value per thread (thread order);
// *total gets the sum over the block.
__device__ unsigned long long sel_excl_scan(unsigned long long v, SelShared& S,
                                            unsigned long long* total) {
  const int lane = lane_id();
  const int w = threadIdx.x / 64;
  unsigned long long inc = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const unsigned long long t = __shfl_up(inc, o, 64);
    if (lane >= o) inc += t;
  }
  __syncthreads();
  if (lane == 63) S.red[w] = inc;
  __syncthreads();
  unsigned long long base = 0, tot = 0;
  for (int i = 0; i < SEL_TPB / 64; ++i) {
    const unsigned long long r = S.red[i];
    base += i < w ? r : 0ull;
    tot += r;
  }
  __syncthreads();
  *total = tot;
  return base + inc - v;
}

// Bucket where the running count, scanned from the top (descending) or the
// bottom, reaches `target` (1-based); S.before = count strictly before it.
// Thread t takes scan positions 2t and 2t + 1.
__device__ void sel_scan(SelShared& S, unsigned long long target, bool descending) {
  static_assert(SEL_BUCKETS == 2 * SEL_TPB, "two buckets per thread");
  const int p0 = 2 * (int)threadIdx.x;
  const int b0 = descending ? SEL_BUCKETS - 1 - p0 : p0;
  const int b1 = descending ? b0 - 1 : b0 + 1;
  const unsigned long long c0 = S.hist[b0], c1 = S.hist[b1];
  unsigned long long tot;
  const unsigned long long ex = sel_excl_scan(c0 + c1, S, &tot);
  if (ex < target && ex + c0 >= target) {
    S.bucket = (unsigned)b0;
    S.before = ex;
  } else if (ex + c0 < target && ex + c0 + c1 >= target) {
    S.bucket = (unsigned)b1;
    S.before = ex + c0;
  }
  __syncthreads();
}

// Visit the candidates (id, count): the window from LDS, then, if `tail`,
// the hash slots.  Every lane of the workgroup makes the same number of
// calls (wave-level counting inside f); count 0 means "no candidate".
template <typename F>
__device__ __forceinline__ void sel_visit(const CParams& P, const SelShared& S, long long wbase,
                                          unsigned win_len, bool tail, unsigned long long H, F f) {
  (void)win_len;
  for (unsigned w = threadIdx.x; w < (unsigned)WIN; w += SEL_TPB)
    f(wbase + (long long)w, S.win[w]);  // bins past win_len hold 0
  if (tail) {
    for (unsigned long long s0 = 0; s0 < H; s0 += (unsigned long long)SEL_TPB * 4) {
      uint32_t slot[4], cn[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const unsigned long long si = s0 + (unsigned long long)u * SEL_TPB + threadIdx.x;
        slot[u] = si < H ? gload(P.hslot + si) : HEMPTY;
        cn[u] = si < H ? gload(P.hcnt + si) : 0u;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const bool ok = slot[u] != HEMPTY && cn[u] != 0;
        f(ok ? (long long)gload(P.tail + slot[u]) : 0ll, ok ? cn[u] : 0u);
      }
    }
  }
}

// Order-preserving 11-bit key of a count c >= 1 on a log scale: c itself
// below 64, else its exponent e = floor(log2 c) and the six bits after the
// leading one.  Key b >= 64 holds the counts [(64 + b % 64) << s,
// (65 + b % 64) << s) with s = b / 64 - 1.
__device__ __forceinline__ unsigned sel_log_key(uint32_t c) {
  if (c < 64u) return c;
  const unsigned e = 31u - (unsigned)__clz(c);
  return ((e - 5u) << 6) | ((c >> (e - 6u)) & 63u);
}

// k-th largest count among the window's bins (mx >= 1: their largest) and
// its place among the bins of that count (*r, 1-based).  A first pass over
// log-scale keys leaves only the bins of one key's narrow range of counts,
// usually few, for the passes over the low bits: with a few bins holding
// most points, a first digit cut from the top of the largest count puts
// nearly every bin in its lowest bucket and narrows nothing.
template <typename Visit>
__device__ unsigned sel_kth_count_log(SelShared& S, unsigned long long k, Visit visit,
                                      unsigned long long* r) {
  for (int i = threadIdx.x; i < SEL_BUCKETS; i += SEL_TPB) S.hist[i] = 0u;
  __syncthreads();
  visit([&](long long, uint32_t cn) { lds_count(S.hist, cn != 0, cn ? sel_log_key(cn) : 0u); });
  __syncthreads();
  sel_scan(S, k, true);
  unsigned long long target = k - S.before;
  const unsigned b = S.bucket;
  __syncthreads();
  if (b < 64u) {  // exact
    *r = target;
    return b;
  }
  const unsigned low = b / 64u - 1u;                       // bits below the key's range
  const uint32_t base = (64u + (b & 63u)) << low;          // its smallest count
  unsigned prefix = 0;                                     // offset from base
  const int top = ((int)low + SEL_DIGIT - 1) / SEL_DIGIT * SEL_DIGIT;
  for (int shift = top - SEL_DIGIT; shift >= 0; shift -= SEL_DIGIT) {
    for (int i = threadIdx.x; i < SEL_BUCKETS; i += SEL_TPB) S.hist[i] = 0u;
    __syncthreads();
    visit([&](long long, uint32_t cn) {
      const uint32_t o = cn - base;  // wraps for counts below base
      const bool on = cn >= base && ((unsigned long long)o >> low) == 0ull &&
                      ((unsigned long long)(o ^ prefix) >> (shift + SEL_DIGIT)) == 0ull;
      lds_count(S.hist, on, (o >> shift) & (SEL_BUCKETS - 1));
    });
    __syncthreads();
    sel_scan(S, target, true);
    target -= S.before;
    prefix |= S.bucket << shift;
    __syncthreads();
  }
  *r = target;
  return base + prefix;
}

// tau and the tie cut over the window alone (more than k nonzero bins): the
// ties are bins of the window, whose ids are wbase + their place, so the
// r-th tie in id order is found with one scan of per-thread tie counts
// (thread t takes places [16 t, 16 t + 16)) instead of a count of the bins
// above tau and a radix select over the ties' ids.
template <typename Visit>
__device__ void sel_threshold_window(SelShared& S, unsigned long long k, long long wbase,
                                     Visit visit, unsigned* tau_out, long long* cut_out) {
  static_assert(WIN == 16 * SEL_TPB, "16 window bins per thread");
  unsigned long long r = 0;
  const unsigned tau = sel_kth_count_log(S, k, visit, &r);
  const unsigned w0 = 16u * threadIdx.x;
  unsigned mine = 0;
#pragma unroll
  for (int i = 0; i < 16; ++i) mine += S.win[w0 + i] == tau ? 1u : 0u;
  unsigned long long tot;
  const unsigned long long ex = sel_excl_scan(mine, S, &tot);
  if (ex < r && r <= ex + mine) {
    unsigned left = (unsigned)(r - ex);
    unsigned at = w0;
    for (int i = 0; i < 16; ++i) {
      const bool t = S.win[w0 + i] == tau;
      if (t && left == 1) {
        at = w0 + i;
        break;
      }
      left -= t ? 1u : 0u;
    }
    S.bucket = at;
  }
  __syncthreads();
  *tau_out = tau;
  *cut_out = wbase + (long long)S.bucket;
  __syncthreads();
}

// Bin ids as order-preserving unsigned keys (ids may be negative when the
// bins are anchored at -E).
constexpr unsigned long long ID_SIGN = 1ull << 63;
__device__ __forceinline__ unsigned long long id_key(long long id) {
  return (unsigned long long)id ^ ID_SIGN;
}

// The r-th smallest id (1-based) among candidates with count == tau, given
// the smallest and largest such id as keys.
template <typename Visit>
__device__ long long sel_rth_tie(SelShared& S, unsigned tau, unsigned long long r,
                                 unsigned long long tmin, unsigned long long tmax, Visit visit) {
  const unsigned long long span = tmax - tmin;
  int topb = 0;
  while (topb < 64 && (span >> topb) != 0) topb += SEL_DIGIT;
  unsigned long long pre = 0, tgt = r;
  for (int shift = topb - SEL_DIGIT; shift >= 0; shift -= SEL_DIGIT) {
    for (int i = threadIdx.x; i < SEL_BUCKETS; i += SEL_TPB) S.hist[i] = 0u;
    __syncthreads();
    const unsigned long long hmask =
        (shift + SEL_DIGIT >= 64) ? 0ull : (~0ull << (shift + SEL_DIGIT));
    visit([&](long long id, uint32_t cn) {
      const unsigned long long rel = id_key(id) - tmin;
      const bool on = cn != 0 && cn == tau && (rel & hmask) == (pre & hmask);
      lds_count(S.hist, on, (unsigned)((rel >> shift) & (SEL_BUCKETS - 1)));
    });
    __syncthreads();
    sel_scan(S, tgt, false);
    tgt -= S.before;
    pre |= (unsigned long long)S.bucket << shift;
    __syncthreads();
  }
  return (long long)((tmin + pre) ^ ID_SIGN);
}

// tau and the tie cut over the visited candidates (nz nonzero of them, nz > k).
template <typename Visit>
__device__ void sel_threshold(SelShared& S, unsigned long long k,
                              Visit visit, unsigned* tau_out, long long* cut_out) {
  unsigned long long r_unused;
  const unsigned tau = sel_kth_count_log(S, k, visit, &r_unused);
  unsigned long long gt = 0, ties = 0, tmin = ~0ull, tmax = 0;
  visit([&](long long id, uint32_t cn) {
    if (cn == 0) return;
    if (cn > tau) gt += 1;
    if (cn == tau) {
      ties += 1;
      const unsigned long long key = id_key(id);
      tmin = key < tmin ? key : tmin;
      tmax = key > tmax ? key : tmax;
    }
  });
  sel_reduce4(gt, ties, tmin, tmax, S);
  const unsigned long long r = k - gt;  // ties to take, >= 1
  *tau_out = tau;
  *cut_out = r >= ties ? (long long)(tmax ^ ID_SIGN) : sel_rth_tie(S, tau, r, tmin, tmax, visit);
}

// The window counts to LDS (16-byte loads, all in flight at once), with the
// number of nonzero bins and the largest count; the buffer holds WIN counts,
// zero past win_len.  The whole workgroup calls it.
__device__ void sel_load_window(const CParams& P, SelShared& S, unsigned win_len,
                                unsigned long long& nzw, unsigned long long& mxw) {
  constexpr int G4 = WIN / 4 / SEL_TPB;
  const int tid = threadIdx.x;
  unsigned long long unused0 = ~0ull, unused1 = 0;
  nzw = 0;
  mxw = 0;
  nk_u32x4 x[G4];
#pragma unroll
  for (int i = 0; i < G4; ++i)
    x[i] = gload(reinterpret_cast<const nk_u32x4*>(P.gwin) + (tid + i * SEL_TPB));
#pragma unroll
  for (int i = 0; i < G4; ++i) {
    const unsigned w0 = 4u * (unsigned)(tid + i * SEL_TPB);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const uint32_t cn = w0 + e < win_len ? x[i][e] : 0u;
      x[i][e] = cn;
      nzw += cn ? 1 : 0;
      mxw = cn > mxw ? cn : mxw;
    }
    reinterpret_cast<nk_u32x4*>(S.win)[tid + i * SEL_TPB] = x[i];
  }
  sel_reduce4(nzw, unused1, unused0, mxw, S);  // also orders the LDS writes
}

template <typename T, typename SRC>
__global__ void __launch_bounds__(SEL_TPB) k_select(SRC src, Geo g) {
  const CParams& P = src.job(g.job_begin + blockIdx.x);
  __shared__ SelShared S;
  Ctl* c = P.ctl;
  const int tid = threadIdx.x;
  const uint32_t k = P.k;
  const uint64_t ncent = (uint64_t)k + 1;

  // centres and bin ids start cleared
  T* centers = static_cast<T*>(P.centers);
  for (uint64_t i = tid; i < ncent; i += SEL_TPB) gstore(centers + i, (T)0);
  if (P.bin_ids)
    for (uint64_t i = tid; i < k; i += SEL_TPB) gstore(P.bin_ids + i, (int64_t)-1);

  const bool empty = c->empty != 0;
  const long long wbase = empty ? 0 : c->wbase;
  const unsigned win_len = empty ? 0u : c->win_len;
  const bool has_tail = !empty && c->tail_used > 0;
  const unsigned long long H = has_tail ? c->H : 0ull;
  const unsigned long long tail_bins = has_tail ? c->tail_bins : 0ull;
  const unsigned long long tail_max = has_tail ? c->tail_max : 0ull;
  const double lo = empty ? 0.0 : c->lo;
  if (tid == 0) S.tail_pos = 0;
  unsigned long long nzw = 0, mxw = 0;
  sel_load_window(P, S, win_len, nzw, mxw);
  const unsigned long long nz = nzw + tail_bins;

  auto visit_win = [&](auto f) { sel_visit(P, S, wbase, win_len, false, 0ull, f); };
  auto visit_all = [&](auto f) { sel_visit(P, S, wbase, win_len, has_tail, H, f); };

  unsigned tau = 0;
  long long cut = -1;
  bool tail_matters = has_tail;
  if (nz > k) {
    bool done = false;
    if (nzw >= k) {
      unsigned tw;
      long long cw;
      sel_threshold_window(S, k, wbase, visit_win, &tw, &cw);
      if (tail_max < tw) {  // no tail bin reaches the window's k-th count
        tau = tw;
        cut = cw;
        done = true;
        tail_matters = false;
      }
    }
    if (!done) sel_threshold(S, k, visit_all, &tau, &cut);
  }
  // selected <=> cnt > tau, or cnt == tau and id <= cut (cnt nonzero).
  // With k <= SEL_TPB the selected tail ids also go to LDS (the radix
  // histogram's space, free from here on) and are ranked at the end of this
  // kernel; larger k leaves them to k_tailrank.
  const bool rank_here = k <= (uint32_t)SEL_TPB;
  long long* s_tail = reinterpret_cast<long long*>(S.hist);
  static_assert(sizeof(S.hist) >= SEL_TPB * sizeof(long long), "tail ids fit");
  unsigned long long sel_tail = 0, sel_below = 0;
  if (tail_matters) {
    for (unsigned long long si = tid; si < H; si += SEL_TPB) {
      const uint32_t slot = gload(P.hslot + si);
      if (slot == HEMPTY) continue;
      const uint32_t cn = gload(P.hcnt + si);
      const long long id = gload(P.tail + slot);
      if (cn != 0 && (cn > tau || (cn == tau && id <= cut))) {
        sel_tail += 1;
        if (id < wbase) sel_below += 1;
        const unsigned pos = atomicAdd(&S.tail_pos, 1u);
        gstore(P.sel_tail + pos, (int64_t)id);
        if (rank_here) s_tail[pos] = id;  // pos < k
      }
    }
  }
  if (tail_matters) {  // uniform; otherwise both counts are 0 everywhere
    unsigned long long u0 = ~0ull, u1 = 0;
    sel_reduce4(sel_tail, sel_below, u0, u1, S);
  }

  // window: LUT, centres and bin ids in ascending bin order.  Wave v owns
  // the window bins [v * SEL_WBINS, (v + 1) * SEL_WBINS), read as 64-bin
  // segments (lane l takes bin l of a segment: no LDS bank conflicts); a
  // segment's selected bins are ranked by ballot, the waves by one scan.
  constexpr int SEL_WBINS = WIN / (SEL_TPB / 64);
  constexpr int SEGS = SEL_WBINS / 64;
  const int wv = tid / 64, ln = tid & 63;
  auto chosen = [&](unsigned w) {
    const uint32_t cn = S.win[w];
    const long long id = wbase + (long long)w;
    return cn != 0 && (cn > tau || (cn == tau && id <= cut));
  };
  unsigned mine = 0;
#pragma unroll
  for (int q = 0; q < SEGS; ++q)
    mine += (unsigned)__popcll(__ballot(chosen((unsigned)(wv * SEL_WBINS + q * 64 + ln))));
  // exclusive prefix of the wave totals (every lane holds its wave's total)
  __syncthreads();
  if (ln == 0) S.red[wv] = mine;
  __syncthreads();
  unsigned long long wbefore = 0, nwin_sel = 0;
  for (int i = 0; i < SEL_TPB / 64; ++i) {
    const unsigned long long r = S.red[i];
    wbefore += i < wv ? r : 0ull;
    nwin_sel += r;
  }
  if (tid == 0) c->nsel_window = (unsigned)nwin_sel;
  unsigned rank = (unsigned)sel_below + (unsigned)wbefore;
#pragma unroll 4
  for (int q = 0; q < SEGS; ++q) {
    const unsigned w = (unsigned)(wv * SEL_WBINS + q * 64 + ln);
    const unsigned long long mk = __ballot(chosen(w));
    const unsigned r = rank + __builtin_amdgcn_mbcnt_hi((unsigned)(mk >> 32),
                                                        __builtin_amdgcn_mbcnt_lo((unsigned)mk, 0u));
    uint32_t l = k;  // escape code: not selected
    if ((mk >> ln) & 1ull) {
      l = r;
      gstore(centers + r, (T)centre_of<T>(wbase + (long long)w, lo, P.E));
      if (P.bin_ids) gstore(P.bin_ids + r, (int64_t)(wbase + (long long)w));
    }
    S.win[w] = l;  // each lane rewrites only the bin it read
    rank += (unsigned)__popcll(mk);
  }
  __syncthreads();
  uint32_t* lut2 = reinterpret_cast<uint32_t*>(P.lut);  // two 16-bit codes per word
  for (int i = tid; i < WIN / 2; i += SEL_TPB) {
    const uint2 pr = reinterpret_cast<const uint2*>(S.win)[i];
    gstore(lut2 + i, (pr.x & 0xFFFFu) | (pr.y << 16));
  }
  if (tid == 0) {
    c->n_nonzero = nz;
    c->tau = tau;
    c->cut = cut;
    c->k_used = (unsigned)(nz < k ? nz : k);
    c->nsel_tail = (unsigned)sel_tail;
    c->nsel_tail_below = (unsigned)sel_below;
  }
  // the selected tail bins in id order (what k_tailrank does for larger k):
  // thread i ranks the i-th id by counting the smaller ones (ids distinct)
  if (rank_here && sel_tail != 0) {  // uniform
    const unsigned t = (unsigned)sel_tail;
    if ((unsigned)tid < t) {
      const long long id = s_tail[tid];
      unsigned r = 0;
      for (unsigned j = 0; j < t; ++j) r += s_tail[j] < id ? 1u : 0u;
      gstore(P.sorted_tail + r, (int64_t)id);
      const unsigned idx = r + (id > wbase ? (unsigned)nwin_sel : 0u);
      gstore(centers + idx, (T)centre_of<T>(id, lo, P.E));
      if (P.bin_ids) gstore(P.bin_ids + idx, (int64_t)id);
    }
  }
}

// =====================================================================
// k_autob: choice of B from the histogram (Sec. IV-B-2, eqs. 5-6)
// =====================================================================
// Workgroup b estimates B = b_lo + b: the points held by the 2^B - 1
// fullest bins (all valid points when there are no more nonzero bins than
// that; otherwise the counts above the (2^B - 1)-th largest count tau, plus
// tau for each of the remaining places), and the estimated size
// 2^B L + n B / 8 + n alpha L in bits, alpha n being the points not held.
// Exact while the tail fits its capacity.  The caller picks the smallest.
// Tail-bin counts held in LDS for the repeated visits (80 KB beside the
// window); a larger tail is visited in the hash table instead.
constexpr int AUTOB_TAIL_LDS = 20480;

template <typename SRC>
__global__ void __launch_bounds__(SEL_TPB) k_autob(SRC src, Geo g, uint32_t b_lo, uint32_t b_hi) {
  const CParams& P = src.job(g.job_begin);
  __shared__ SelShared S;
  __shared__ uint32_t s_tc[AUTOB_TAIL_LDS];
  __shared__ unsigned s_ntc;
  Ctl* c = P.ctl;
  const int tid = threadIdx.x;
  const bool empty = c->empty != 0;
  const long long wbase = empty ? 0 : c->wbase;
  const unsigned win_len = empty ? 0u : c->win_len;
  const bool has_tail = !empty && c->tail_used > 0;
  const unsigned long long H = has_tail ? c->H : 0ull;
  const unsigned long long tail_bins = has_tail ? c->tail_bins : 0ull;
  const unsigned long long tail_max = has_tail ? c->tail_max : 0ull;
  const unsigned long long n = P.n;
  const unsigned long long n_valid = empty ? 0ull : c->n_valid;
  const unsigned long long L = P.dtype == NUMARCK_F32 ? 4ull : 8ull;
  unsigned long long nzw, mxw;
  if (tid == 0) s_ntc = 0;
  sel_load_window(P, S, win_len, nzw, mxw);  // its barriers also publish s_ntc
  const unsigned long long nz = nzw + tail_bins;
  // the nonzero tail-bin counts (their ids are not needed here) into LDS,
  // when the window alone cannot decide
  unsigned ntc = 0;
  bool tail_lds = false;
  auto gather_tail = [&]() {
    for (unsigned long long si = tid; si < H; si += SEL_TPB) {
      const uint32_t slot = gload(P.hslot + si);
      const uint32_t cn = slot == HEMPTY ? 0u : gload(P.hcnt + si);
      if (cn != 0) {
        const unsigned pos = atomicAdd(&s_ntc, 1u);
        if (pos < (unsigned)AUTOB_TAIL_LDS) s_tc[pos] = cn;
      }
    }
    __syncthreads();
    ntc = s_ntc;
    tail_lds = ntc <= (unsigned)AUTOB_TAIL_LDS;
  };
  auto visit_win = [&](auto f) { sel_visit(P, S, wbase, win_len, false, 0ull, f); };
  auto visit_all = [&](auto f) {
    if (tail_lds) {  // every lane makes the same number of calls (count 0: none)
      sel_visit(P, S, wbase, win_len, false, 0ull, f);
      const unsigned rounds = (ntc + SEL_TPB - 1) / SEL_TPB;
      for (unsigned r = 0; r < rounds; ++r) {
        const unsigned i = r * SEL_TPB + tid;
        f(0ll, i < ntc ? s_tc[i] : 0u);
      }
    } else {
      sel_visit(P, S, wbase, win_len, has_tail, H, f);
    }
  };

  {
    const uint32_t B = b_lo + blockIdx.x;
    const unsigned long long k = (1ull << B) - 1ull;
    unsigned long long held = n_valid, r_unused;
    if (nz > k) {
      // tau from the window alone when no tail bin reaches its k-th count
      bool win_only = false;
      unsigned tau = 0;
      if (nzw >= k) {
        tau = sel_kth_count_log(S, k, visit_win, &r_unused);
        win_only = tail_max < tau;
      }
      if (!win_only) {
        gather_tail();
        tau = sel_kth_count_log(S, k, visit_all, &r_unused);
      }
      unsigned long long sum_gt = 0, n_gt = 0, u0 = ~0ull, u1 = 0;
      auto above = [&](long long, uint32_t cn) {
        if (cn > tau) {
          sum_gt += cn;
          n_gt += 1;
        }
      };
      if (win_only) visit_win(above); else visit_all(above);
      sel_reduce4(sum_gt, n_gt, u0, u1, S);
      held = sum_gt + (k - n_gt) * (unsigned long long)tau;
    }
    const unsigned long long bits =
        8ull * (1ull << B) * L + n * (unsigned long long)B + 8ull * L * (n - held);
    if (tid == 0) c->est_bits[B] = bits;
  }
  if (blockIdx.x == 0 && tid < 17 && (tid < (int)b_lo || tid > (int)b_hi))
    c->est_bits[tid] = 0ull;
}

// =====================================================================
// k_tailrank: order the selected tail bins (t <= 65535, usually 0)
// =====================================================================
constexpr int TR_TPB = 256;

template <typename T, typename S>
__global__ void __launch_bounds__(TR_TPB) k_tailrank(S src, Geo g) {
  const CParams& P = src.job(g.job_begin + blockIdx.y);
  __shared__ long long chunk[TR_TPB];
  const Ctl* c = P.ctl;
  const unsigned t = c->nsel_tail;
  if (t == 0 || P.k <= (uint32_t)SEL_TPB) return;  // none, or ranked by k_select
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
// k_encode: pass 3, index + verify + pack + staged compaction
// =====================================================================
// Wave u owns wave tiles [u*tpu, (u+1)*tpu).  It keeps a running count of
// the incompressible points of its range: their values go to scratch at
// (first element of the range + running rank), each block boundary in the
// range gets its range-relative count, and the count of the range goes to
// unit_cnt[u].  k_gather then places every range.  No wave waits
// for another and the loop has no workgroup barrier.
//
// LT: element type of the window LUT in LDS (uint8_t when B <= 8, else
// uint16_t); a LUT entry is the bin's index or the escape code.
// PACK: 8 or 16 when B is 8 or 16 -- the LDS index array is then already the
// packed stream -- or 0 for any B.
constexpr int ENC_CTAB = 2048;  // LDS centre table when 2^B <= this

// Waves per SIMD the float64 B = 8 top-k encoders are compiled for (their
// registers fit five without spilling); others take what they need.
template <typename T, int PACK, bool EW>
constexpr int enc_min_waves = (sizeof(T) == 8 && PACK == 8 && !EW) ? 5 : 1;

// EW: equal-width chunks (k_ewprep) instead of the selected fine bins: a
// valid point's code is min(floor((d - lo) / w), k - 1), 0 when w is 0.
template <typename T, typename LT, int PACK, typename S, int NT, bool EW = false>
__global__ void __launch_bounds__(UNIT_TPB, (enc_min_waves<T, PACK, EW>)) k_encode(S src, Geo g) {
  constexpr int V = Traits<T>::V;
  constexpr int R = ENC_ROUNDS;
  constexpr int WT = R * 64 * V;  // elements of a wave tile
  constexpr int NWAVE = UNIT_TPB / 64;
  using IT = typename std::conditional<PACK == 8, uint8_t, uint16_t>::type;
  constexpr int NCTAB = sizeof(LT) == 1 ? 256 : ENC_CTAB;
  __shared__ LT s_lut[WIN];
  __shared__ double s_ctab[NCTAB];
  // the tile's indices, for widths that are packed from LDS (8- and 16-bit
  // codes go from registers straight to the packed stream)
  __shared__ IT s_idx[NWAVE][PACK == 0 ? WT : 1];
  // float64 full tiles stage up to 64 escapes in LDS and write them with one
  // store; float32 tiles (8 element slots per lane, a compute-bound loop)
  // store each slot directly, lanes without an escape writing the sink
  constexpr bool STAGE = V == 2;
  constexpr int ESC_STAGE = 64;
  __shared__ T s_esc[NWAVE][STAGE ? ESC_STAGE : 1];

  // the 4 units of a workgroup belong to one job (jobs own multiples of 4)
  const uint32_t ublk = g.u_begin + blockIdx.x * NWAVE;
  const uint32_t jb = g.unit0 ? find_job(g.unit0, g.job_begin, g.job_end, ublk) : g.job_begin;
  const CParams P = src.job(jb);  // a copy: stores below cannot alias it
  const Ctl* c = P.ctl;
  const int tid = threadIdx.x;
  const int wave = tid / 64;
  const int lane = lane_id();
  const bool empty = c->empty != 0;
  const double lo = empty ? 0.0 : c->lo;
  const long long wbase = empty ? 0 : c->wbase;
  const double wbase_d = (double)wbase;
  const unsigned win_len = empty ? 0u : c->win_len;
  const double wlen_d = (double)win_len;
  // wave-uniform: kept in a scalar register, so the test per point below is a
  // scalar branch
  const unsigned nsel_tail =
      (unsigned)__builtin_amdgcn_readfirstlane((int)(empty ? 0u : c->nsel_tail));
  const unsigned nsel_win = empty ? 0u : c->nsel_window;
  const uint32_t esc = P.k;
  const uint32_t B = P.B;
  // bin width and its reciprocal: 2E, or the equal-width chunk
  const double bw = EW ? (empty ? 0.0 : c->ew_w) : P.twoE;
  const double binv = EW ? (empty ? 0.0 : c->ew_inv) : P.inv2E;
  const bool wzero = !(bw > 0.0);
  // margins of the fast bin (ratio_bin_fast)
  const double cap_lo = cap_below(P.cap), cap_hi = cap_above(P.cap);
  const double binv_err = binv * 0x1p-36;
  const double kmax_d = (double)(P.k - 1u);
  // with one-byte codes (B <= 8) every centre fits the table
  const bool use_ctab = sizeof(LT) == 1 || ((uint32_t)1 << B) <= (uint32_t)NCTAB;
  if constexpr (!EW)
    for (int i = tid; i < WIN; i += UNIT_TPB) s_lut[i] = (LT)gload(P.lut + i);
  if (use_ctab) {
    const T* cen = static_cast<const T*>(P.centers);
    for (int i = tid; i < (1 << B); i += UNIT_TPB) s_ctab[i] = (double)gload(cen + i);
  }
  __syncthreads();

  const T* __restrict__ prev = static_cast<const T*>(P.prev);
  const T* __restrict__ curr = static_cast<const T*>(P.curr);
  T* __restrict__ scratch = static_cast<T*>(P.scratch);
  T* __restrict__ recon = static_cast<T*>(P.recon);
  IT* idx = s_idx[wave];
  const uint64_t nvec = P.n / V;
  const uint32_t tile_words = (uint32_t)(WT * B / 32);
  const uint32_t unit = ublk + wave - (g.unit0 ? g.unit0[jb] : 0u);  // unit within the job
  const uint64_t tb = (uint64_t)unit * P.tiles_per_unit;
  uint64_t te = tb + P.tiles_per_unit;
  te = te < P.n_tiles ? te : P.n_tiles;
  const uint64_t e_base = tb * WT;
  unsigned run = 0;  // incompressible points so far in this range

  auto load_tile = [&](uint64_t t0, T (&pa)[R][V], T (&qa)[R][V]) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint64_t vi = t0 / V + (uint64_t)r * 64 + lane;
      if (vi < nvec) {
        load_vec_t<NT != 0>(prev, vi, pa[r]);
        load_vec_t<NT == 1>(curr, vi, qa[r]);
      } else {
#pragma unroll
        for (int v = 0; v < V; ++v) {
          const uint64_t j = vi * V + v;
          pa[r][v] = j < P.n ? gload(prev + j) : (T)0;
          qa[r][v] = j < P.n ? gload(curr + j) : (T)0;
        }
      }
    }
  };

  // Lanes with nothing to store in a full tile write here (one 256-byte slot
  // per wave, never read).
  T* const sinkp = reinterpret_cast<T*>(static_cast<char*>(P.sink) +
                                        (size_t)(unit % SINK_SLOTS) * 256);

  // One wave tile: index, verify, stage escapes, pack.  The common path is
  // branch-free; the exact division and the tail-bin search run only when a
  // lane of the wave needs them.  FULL: the tile lies wholly in the vector
  // part of the arrays.  A full tile then issues a fixed set of stores (the
  // packed words, one store per element slot for the escapes, lanes without
  // an escape writing the sink): the loop's wait for the next tile's loads
  // can leave exactly those stores outstanding, instead of waiting for all
  // of them as it must when their number depends on the data.
  auto process = [&](auto full, uint64_t tile, T (&pv)[R][V], T (&qv)[R][V]) {
    constexpr bool FULL = decltype(full)::value;
    const uint64_t t0 = tile * WT;
    const uint64_t left = P.n - t0;
    const uint32_t lim = FULL ? (uint32_t)WT
                              : (left < (uint64_t)WT ? (uint32_t)left : (uint32_t)WT);
    unsigned long long emask[R][V];
    // 8- or 16-bit codes: a lane's V codes of round r, in stream order
    using CW = typename std::conditional<V * (PACK ? PACK : 8) <= 32, uint32_t,
                                         unsigned long long>::type;
    CW cw[R];
    // float64 tiles (four points per lane) take the bins of all their points
    // first -- the multiply by 1/(2E), then, if any lane needs it, the exact
    // division where it is unsure -- so that one wave-wide test covers the
    // tile; float32 tiles (eight points per lane) test point by point, which
    // keeps their registers within four waves per SIMD
    constexpr bool SPLIT = false;
    constexpr int RS = SPLIT ? R : 1, VS = SPLIT ? V : 1;
    double mb[RS][VS];
    bool vb[RS][VS], ex[RS][VS];
    if constexpr (SPLIT) {
      bool need = false;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const uint32_t e0 = ((uint32_t)r * 64 + lane) * V;
#pragma unroll
        for (int v = 0; v < V; ++v) {
          const bool inr = e0 + v < lim;
          bool valid, sure;
          mb[r][v] = ratio_bin_fast((double)pv[r][v], (double)qv[r][v], cap_lo, cap_hi, lo,
                                    binv, binv_err, valid, sure);
          vb[r][v] = valid & inr;
          ex[r][v] = inr & !sure;
          need |= ex[r][v];
        }
      }
      if (__ballot(need)) {
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
          for (int v = 0; v < V; ++v)
            if (ex[r][v]) {
              double d;
              vb[r][v] = ratio_of((double)pv[r][v], (double)qv[r][v], P.cap, d);
              mb[r][v] = floor((d - lo) / bw);
            }
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint32_t e0 = ((uint32_t)r * 64 + lane) * V;  // tile-local element
      cw[r] = 0;
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const bool inr = e0 + v < lim;
        const double p = (double)pv[r][v];
        const double q = (double)qv[r][v];
        bool valid;
        double m;
        if constexpr (SPLIT) {
          valid = vb[r][v];
          m = mb[r][v];
        } else {
          bool vf, sure;
          m = ratio_bin_fast(p, q, cap_lo, cap_hi, lo, binv, binv_err, vf, sure);
          valid = vf & inr;
          const bool exact = inr & !sure;
          if (__ballot(exact)) {
            if (exact) {
              double d;
              valid = ratio_of(p, q, P.cap, d);
              m = floor((d - lo) / bw);
            }
          }
        }
        uint32_t code;
        if constexpr (EW) {
          const double mc = (wzero | !valid) ? 0.0 : (m < kmax_d ? m : kmax_d);
          code = valid ? (uint32_t)mc : esc;
        } else {
        const double w = m - wbase_d;  // exact
        const bool inwin = valid & (w >= 0.0) & (w < wlen_d);
        code = s_lut[inwin ? (int)w : 0];
        code = inwin ? code : esc;
        if (nsel_tail != 0) {  // uniform: selected bins outside the window exist
          const bool tail = valid & !inwin;
          if (__ballot(tail)) {
            if (tail) {  // binary search among the selected tail bins
              const long long mi = (long long)m;
              unsigned a = 0, b = nsel_tail;
              while (a < b) {
                const unsigned mid = (a + b) >> 1;
                if (gload(P.sorted_tail + mid) < mi) a = mid + 1; else b = mid;
              }
              if (a < nsel_tail && gload(P.sorted_tail + a) == mi)
                code = a + (mi > wbase ? nsel_win : 0u);
            }
          }
        }
        }
        const bool sel = code != esc;
        double cc;
        if (use_ctab) {
          cc = s_ctab[sel ? code : 0u];
        } else if constexpr (EW) {
          cc = (double)gload(static_cast<const T*>(P.centers) + (sel ? code : 0u));
        } else {
          cc = centre_of_d<T>(m, lo, P.E);
        }
        const T r_t = (T)(p * (1.0 + cc));
        const bool ok = sel & (fabs((double)r_t - q) <= P.E * fabs(p));
        code = ok ? code : esc;
        if constexpr (PACK == 0)
          idx[e0 + v] = (IT)(inr ? code : 0u);
        else
          cw[r] |= (CW)(inr ? code : 0u) << (v * PACK);
        emask[r][v] = __ballot(inr & !ok);
        if (recon) pv[r][v] = ok ? r_t : qv[r][v];  // the register now holds the reconstruction
      }
    }
    if constexpr (PACK != 0) {
      // element j's code is at bit j * PACK: a lane's V codes of a round are
      // V * PACK / 8 contiguous bytes (2, 4 or 8), stored as 16- or 32-bit
      // words; a partial tile stores code by code up to the stream's end
      // (its padding codes are zero)
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const uint64_t j0 = t0 + ((uint64_t)r * 64 + lane) * V;  // first element
        if (FULL) {
          if constexpr (V * PACK == 16) {
            gstore(reinterpret_cast<uint16_t*>(P.packed) + j0 / 2, (uint16_t)cw[r]);
          } else {
#pragma unroll
            for (int h = 0; h < V * PACK / 32; ++h)
              gstore(P.packed + j0 * PACK / 32 + h, (uint32_t)(cw[r] >> (32 * h)));
          }
        } else {
          const uint64_t pe = (uint64_t)P.packed_words * (32 / PACK);  // codes in the stream
#pragma unroll
          for (int v = 0; v < V; ++v)
            if (j0 + v < pe)
              gstore(reinterpret_cast<IT*>(P.packed) + j0 + v, (IT)(cw[r] >> (v * PACK)));
        }
      }
    }
    if (recon) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const uint64_t vi = t0 / V + (uint64_t)r * 64 + lane;
        if (FULL || vi < nvec) {
          uint4 xv;
          __builtin_memcpy(&xv, pv[r], 16);
          nk_u32x4 yv;
          __builtin_memcpy(&yv, &xv, 16);
          gstore(reinterpret_cast<nk_u32x4*>(recon) + vi, yv);
        } else {
#pragma unroll
          for (int v = 0; v < V; ++v) {
            const uint64_t j = vi * V + v;
            if (j < P.n) gstore(recon + j, pv[r][v]);
          }
        }
      }
    }

    // incompressible values and block offsets, in element order (round,
    // lane, vector slot); ranks are range-relative
    const uint64_t first_b = (t0 + P.epb - 1) / P.epb * P.epb;  // first boundary >= t0
    const bool any_b = first_b < t0 + lim;
    const bool one_b = P.epb >= (uint64_t)WT;
    const uint32_t b_local = (uint32_t)(first_b - t0);
    const unsigned run0 = run;  // escapes of the range before this tile
#pragma unroll
    for (int r = 0; r < R; ++r) {
      unsigned below = 0, all = 0;
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const unsigned long long mk = emask[r][v];
        below += __builtin_amdgcn_mbcnt_hi((unsigned)(mk >> 32),
                                           __builtin_amdgcn_mbcnt_lo((unsigned)mk, 0u));
        all += (unsigned)__popcll(mk);
      }
      unsigned rank = run + below;
      const uint32_t e0 = ((uint32_t)r * 64 + lane) * V;
#pragma unroll
      for (int v = 0; v < V; ++v) {
        if (any_b) {
          const uint64_t j = t0 + e0 + v;
          const bool at_b =
              e0 + v < lim && (one_b ? (e0 + v == b_local) : (j % P.epb == 0));
          if (at_b) gstore(P.block_inc_off + j / P.epb, (int64_t)rank);
        }
        const bool escp = (emask[r][v] >> lane) & 1ull;
        if (FULL && !STAGE) {  // every lane stores: the escape, or into the sink
          gstore(escp ? scratch + e_base + rank : sinkp, qv[r][v]);
        } else if (escp) {
          const unsigned tl = rank - run0;  // rank within the tile
          if (FULL && tl < (unsigned)ESC_STAGE)
            s_esc[wave][tl] = qv[r][v];  // written below, one store for the tile
          else
            gstore(scratch + e_base + rank, qv[r][v]);
        }
        rank += escp ? 1u : 0u;
      }
      run += all;
    }

    // bit-pack the wave tile: word w holds bits [32w, 32w + 32) of its stream
    constexpr bool USE_LDS = PACK == 0 || STAGE;  // LDS written above, read below
    if (USE_LDS) wave_lds_sync();
    if (FULL && STAGE) {  // the staged escapes: lane i writes the tile's i-th, the others the sink
      const bool has = (unsigned)lane < run - run0;
      const T val = s_esc[wave][lane];
      gstore(has ? scratch + e_base + run0 + lane : sinkp, val);
    }
    const uint64_t word0 = t0 * B / 32;
    if (PACK != 0) {
      // stored from registers above
    } else if (FULL) {
      // at most B = 7 (u8 indices) or 15 (u16) bits: a fixed number of store
      // rounds, lanes past the tile's words writing the sink
      constexpr uint32_t BMAX = sizeof(LT) == 1 ? 7u : 15u;
      constexpr uint32_t KW = (uint32_t)((WT * BMAX / 32 + 63) / 64);
#pragma unroll
      for (uint32_t k = 0; k < KW; ++k) {
        const uint32_t w = lane + 64 * k;
        const bool in = w < tile_words;
        uint32_t word = 0;
        if (in) {
          const uint32_t bit0 = w * 32;
          const uint32_t e_first = B == 1 ? bit0 : __umulhi(bit0, P.mulB);
          const uint32_t e_last = B == 1 ? bit0 + 31 : __umulhi(bit0 + 31, P.mulB);
          for (uint32_t e = e_first; e <= e_last; ++e) {
            const uint32_t v = idx[e];
            const int sh = (int)(e * B) - (int)bit0;
            word |= sh >= 0 ? (v << sh) : (v >> (-sh));
          }
        }
        gstore(in ? P.packed + word0 + w : reinterpret_cast<uint32_t*>(sinkp), word);
      }
    } else {
      for (uint32_t w = lane; w < tile_words; w += 64) {
        if (word0 + w >= P.packed_words) break;
        const uint32_t bit0 = w * 32;
        // floor(bit0 / B) and floor((bit0 + 31) / B); mulB does not exist for B = 1
        const uint32_t e_first = B == 1 ? bit0 : __umulhi(bit0, P.mulB);
        const uint32_t e_last = B == 1 ? bit0 + 31 : __umulhi(bit0 + 31, P.mulB);
        uint32_t word = 0;
        for (uint32_t e = e_first; e <= e_last; ++e) {
          const uint32_t v = idx[e];
          const int sh = (int)(e * B) - (int)bit0;
          word |= sh >= 0 ? (v << sh) : (v >> (-sh));
        }
        gstore(P.packed + word0 + w, word);
      }
    }
    if (USE_LDS) wave_lds_sync();
  };

  // Two register sets: the loads of one tile are in flight while the other
  // is processed.  Tiles wholly inside the vector part of the arrays load
  // without bounds checks and the next tile's loads are issued on every
  // iteration (the last one re-reads its own tile), so the loop has a fixed
  // number of loads in flight and the wait before processing a tile leaves
  // the following tile's loads outstanding.  A ragged last tile takes the
  // checked loads.
  auto load_full = [&](uint64_t t0, T (&pa)[R][V], T (&qa)[R][V]) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint64_t vi = t0 / V + (uint64_t)r * 64 + lane;
      load_vec_t<NT != 0>(prev, vi, pa[r]);
      load_vec_t<NT == 1>(curr, vi, qa[r]);
    }
  };
  const uint64_t full_tiles = nvec / (WT / V);  // tiles with every vector in range
  const uint64_t tf = te < full_tiles ? te : (tb > full_tiles ? tb : full_tiles);
  T pa[R][V], qa[R][V], pb[R][V], qb[R][V];
  if (tb < tf) {
    load_full(tb * WT, pa, qa);
    {
      // A tile's wait counts the stores issued after its loads and takes the
      // smallest count over the paths reaching it.  Entering the loop, as
      // many stores follow the first tile's loads as follow any later
      // tile's (a full tile issues at most R*V escape stores and 4 rounds of
      // packed words, plus rare extra ones), so the entry path does not
      // lower that count.
      __builtin_amdgcn_sched_barrier(0);  // keep them after the loads
#pragma unroll
      for (int i = 0; i < R * V + 4; ++i) gstore(sinkp + 2 * i, (T)i);  // distinct, never merged
      __builtin_amdgcn_sched_barrier(0);
    }
    for (uint64_t tile = tb;; tile += 2) {
      const uint64_t n1 = tile + 1 < tf ? tile + 1 : tile;
      load_full(n1 * WT, pb, qb);
      process(std::true_type{}, tile, pa, qa);
      if (tile + 1 >= tf) break;
      const uint64_t n2 = tile + 2 < tf ? tile + 2 : tile + 1;
      load_full(n2 * WT, pa, qa);
      process(std::true_type{}, tile + 1, pb, qb);
      if (tile + 2 >= tf) break;
    }
  }
  for (uint64_t tile = tf; tile < te; ++tile) {  // at most the array's last tile
    load_tile(tile * WT, pa, qa);
    process(std::false_type{}, tile, pa, qa);
  }
  if (lane == 0 && unit < P.n_units) gstore(P.unit_cnt + unit, run);
}

// =====================================================================
// k_gather: move each unit's incompressible values to their final offset
// =====================================================================
__device__ void write_header(const CParams& P);

// =====================================================================
// k_encode_pre: pass 3 from the window codes (precoded encoding)
// =====================================================================
// The index of point j, valid and outside the histogram window, among the
// selected tail bins: its bin from its values (ratio_bin), a binary search
// in the sorted selected tail ids, and the check of Sec. III-C with that
// bin's centre; the escape code when the bin is not selected or the check
// fails.  It runs only for such points, and only when selected tail bins
// exist; the encoder calls it from one loop per tile over such points rather
// than at each of its code slots, which keeps the tile loop short.
template <typename T>
__device__ __forceinline__ uint32_t pre_tail_index(
    const T* prev, const T* curr, uint64_t j, const int64_t* sorted_tail, unsigned nsel_tail,
    unsigned nsel_win, long long wbase, double lo, double E, double cap, double twoE,
    double inv2E, uint32_t esc) {
  const double p = (double)gload(prev + j), q = (double)gload(curr + j);
  bool vf;
  const double m = ratio_bin(p, q, cap, cap_below(cap), cap_above(cap), lo, twoE, inv2E,
                             inv2E * 0x1p-36, vf);
  const long long mi = (long long)m;
  unsigned a = 0, b = nsel_tail;
  while (a < b) {
    const unsigned mid = (a + b) >> 1;
    if (gload(sorted_tail + mid) < mi) a = mid + 1; else b = mid;
  }
  if (!vf || a >= nsel_tail || gload(sorted_tail + a) != mi) return esc;
  const T r_t = (T)(p * (1.0 + centre_of_d<T>(m, lo, E)));
  return fabs((double)r_t - q) <= E * fabs(p) ? a + (mi > wbase ? nsel_win : 0u) : esc;
}

// The histogram pass has written each point's window code (WC_*): its
// place in the window and whether its own bin's centre passes the check of
// Sec. III-C.  A point's index is the window LUT entry of that place when
// the entry is a selected bin and the check passed, else the escape code.
// A point outside the window is looked up among the selected tail bins from
// its values, and only when such bins exist (otherwise it escapes).  So the
// pass reads 2 bytes per point instead of both snapshots.  It stages the
// element indices of the incompressible points; k_gather fetches their
// values and derives the block offsets from them.  Units and compaction
// follow k_encode; lane l of round r holds the 8 codes of elements
// t0 + (r * 64 + l) * 8 + [0, 8).
template <typename T, typename LT, int PACK, typename S>
__global__ void __launch_bounds__(UNIT_TPB) k_encode_pre(S src, Geo g) {
  constexpr int V = 8;
  constexpr int R = PRE_ROUNDS;
  constexpr int WT = (int)PRE_WAVE_TILE;
  constexpr int NWAVE = UNIT_TPB / 64;
  // codes kept in LDS for bit-packing (widths other than 8 and 16)
  using IT = LT;
  constexpr int PK = PACK ? PACK : 8 * (int)sizeof(IT);  // bits per code in cw
  constexpr int CWN = V * PK / 32;                         // 32-bit words per lane-round
  __shared__ LT s_lut[WIN];
  __shared__ __align__(16) IT s_idx[NWAVE][PACK == 0 ? WT : 1];
  constexpr int ESC_STAGE = 256;
  __shared__ uint32_t s_esc[NWAVE][ESC_STAGE];

  const uint32_t ublk = g.u_begin + blockIdx.x * NWAVE;
  const uint32_t jb = g.unit0 ? find_job(g.unit0, g.job_begin, g.job_end, ublk) : g.job_begin;
  const CParams P = src.job(jb);
  const Ctl* c = P.ctl;
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid / 64);
  const int lane = lane_id();
  const bool empty = c->empty != 0;
  const double lo = empty ? 0.0 : c->lo;
  const long long wbase = empty ? 0 : c->wbase;
  const unsigned nsel_tail =
      (unsigned)__builtin_amdgcn_readfirstlane((int)(empty ? 0u : c->nsel_tail));
  const unsigned nsel_win = empty ? 0u : c->nsel_window;
  const uint32_t esc = P.k;
  const uint32_t B = P.B;
  // the LUT's 16-bit entries, eight per 16-byte load
  for (int i = tid; i < WIN / 8; i += UNIT_TPB) {
    const nk_u32x4 x = gload(reinterpret_cast<const nk_u32x4*>(P.lut) + i);
#pragma unroll
    for (int h = 0; h < 8; ++h) s_lut[8 * i + h] = (LT)(x[h / 2] >> (16 * (h & 1)));
  }
  __syncthreads();

  const T* __restrict__ prev = static_cast<const T*>(P.prev);
  const T* __restrict__ curr = static_cast<const T*>(P.curr);
  const nk_u32x4* __restrict__ wv = reinterpret_cast<const nk_u32x4*>(P.wcode);
  uint32_t* __restrict__ stage = static_cast<uint32_t*>(P.scratch);
  IT* idx = s_idx[wave];
  const uint64_t nvec = P.n / V;
  const uint32_t tile_words = (uint32_t)(WT * B / 32);
  const uint32_t unit = ublk + wave - (g.unit0 ? g.unit0[jb] : 0u);
  const uint64_t tb = (uint64_t)unit * P.tiles_per_unit;
  uint64_t te = tb + P.tiles_per_unit;
  te = te < P.n_tiles ? te : P.n_tiles;
  const uint64_t e_base = tb * WT;
  unsigned run = 0;  // incompressible points so far in this range

  auto process = [&](auto full, uint64_t tile, const nk_u32x4 (&cv)[R]) {
    constexpr bool FULL = decltype(full)::value;
    const uint64_t t0 = tile * WT;
    const uint64_t left = P.n - t0;
    const uint32_t lim = FULL ? (uint32_t)WT
                              : (left < (uint64_t)WT ? (uint32_t)left : (uint32_t)WT);
    // code slot sl = r * V + v of a lane: element e0(r) + v.  inm: the slots
    // in range; okm: the slots indexed (selected bin, check passed)
    uint32_t cw[R][CWN];
    uint32_t okm = 0, inm = FULL ? (1u << (R * V)) - 1u : 0u;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint32_t e0 = ((uint32_t)r * 64 + lane) * V;  // tile-local element
#pragma unroll
      for (int h = 0; h < CWN; ++h) cw[r][h] = 0;
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const bool inr = FULL || e0 + v < lim;
        const uint32_t c16 = (cv[r][v / 2] >> (16 * (v & 1))) & 0xFFFFu;
        const uint32_t l = s_lut[c16 & (uint32_t)(WIN - 1)];
        // bits 15-14 = 01: valid, inside the window, check passed
        const uint32_t code = (c16 >> 14) == 1u ? l : esc;
        if (!FULL) inm |= inr ? 1u << (r * V + v) : 0u;
        okm |= inr & (code != esc) ? 1u << (r * V + v) : 0u;
        cw[r][(v * PK) / 32] |= (inr ? code : 0u) << ((v * PK) % 32);
      }
    }
    if (nsel_tail != 0) {  // uniform: points outside the window may be indexed
      uint32_t tm = 0;
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int v = 0; v < V; ++v) {
          const uint32_t c16 = (cv[r][v / 2] >> (16 * (v & 1))) & 0xFFFFu;
          tm |= c16 == WC_TAIL ? 1u << (r * V + v) : 0u;
        }
      tm &= inm;
      while (tm) {
        const int sl = __builtin_ctz(tm);
        tm &= tm - 1u;
        const int v = sl % V;
        const uint32_t e = ((uint32_t)(sl / V) * 64 + lane) * V + v;
        const uint32_t code = pre_tail_index<T>(prev, curr, t0 + e, P.sorted_tail, nsel_tail,
                                                nsel_win, wbase, lo, P.E, P.cap, P.twoE,
                                                P.inv2E, esc);
        if (code != esc) {  // the slot held the escape code: put the index there
          okm |= 1u << sl;
          const int hw = (sl / V) * CWN + (v * PK) / 32;
          const int sh = (v * PK) % 32;
#pragma unroll
          for (int r = 0; r < R; ++r)
#pragma unroll
            for (int h = 0; h < CWN; ++h)
              if (r * CWN + h == hw)
                cw[r][h] = (cw[r][h] & ~(esc << sh)) | (code << sh);
        }
      }
    }
    // the indices: 8- and 16-bit codes straight to the packed stream (a
    // lane's 8 codes are 8 or 16 contiguous bytes), others to LDS
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint64_t j0 = t0 + ((uint64_t)r * 64 + lane) * V;  // first element
      if constexpr (PACK != 0) {
        if (FULL) {
          if constexpr (CWN == 4) {
            nk_u32x4 x;
            x[0] = cw[r][0]; x[1] = cw[r][1]; x[2] = cw[r][2]; x[3] = cw[r][3];
            gstore(reinterpret_cast<nk_u32x4*>(P.packed) + j0 / 8, x);
          } else {
            const unsigned long long x = ((unsigned long long)cw[r][1] << 32) | cw[r][0];
            gstore(reinterpret_cast<unsigned long long*>(P.packed) + j0 / 8, x);
          }
        } else {
          using PT = typename std::conditional<PACK == 8, uint8_t, uint16_t>::type;
          const uint64_t pe = (uint64_t)P.packed_words * (32 / PACK);  // codes in the stream
#pragma unroll
          for (int v = 0; v < V; ++v)
            if (j0 + v < pe)
              gstore(reinterpret_cast<PT*>(P.packed) + j0 + v,
                     (PT)(cw[r][(v * PACK) / 32] >> ((v * PACK) % 32)));
        }
      } else {
        IT* dst = idx + ((uint32_t)r * 64 + lane) * V;
        if constexpr (CWN == 4) {
          nk_u32x4 x;
          x[0] = cw[r][0]; x[1] = cw[r][1]; x[2] = cw[r][2]; x[3] = cw[r][3];
          *reinterpret_cast<nk_u32x4*>(dst) = x;
        } else {
          *reinterpret_cast<unsigned long long*>(dst) =
              ((unsigned long long)cw[r][1] << 32) | cw[r][0];
        }
      }
    }

    // incompressible points in element order (round, lane, code slot);
    // ranks are range-relative.  A lane's escapes of a round number at most
    // 8: the escapes of the lanes below it are counted bit by bit of those
    // counts (four ballots), then each lane stages its own in order.
    const uint32_t em = inm & ~okm;
    const unsigned run0 = run;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint32_t er = (em >> (r * V)) & ((1u << V) - 1u);
      const uint32_t cnt = (uint32_t)__builtin_popcount(er);
      unsigned below = 0, all = 0;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const unsigned long long bm = __ballot((cnt >> b) & 1u);
        below += __builtin_amdgcn_mbcnt_hi((unsigned)(bm >> 32),
                                           __builtin_amdgcn_mbcnt_lo((unsigned)bm, 0u)) << b;
        all += (unsigned)__popcll(bm) << b;
      }
      unsigned rank = run + below;
      const uint32_t e0 = ((uint32_t)r * 64 + lane) * V;
      uint32_t e = er;
      while (e) {
        const uint32_t v = (uint32_t)__builtin_ctz(e);
        e &= e - 1u;
        const unsigned tl = rank - run0;  // rank within the tile
        const uint32_t j = (uint32_t)(t0 + e0 + v);
        if (FULL && tl < (unsigned)ESC_STAGE) s_esc[wave][tl] = j;
        else gstore(stage + e_base + rank, j);
        ++rank;
      }
      run += all;
    }

    wave_lds_sync();
    if (FULL) {  // the staged escape indices, in order
      const unsigned cnt = run - run0 < (unsigned)ESC_STAGE ? run - run0 : (unsigned)ESC_STAGE;
      for (unsigned i = (unsigned)lane; i < cnt; i += 64)
        gstore(stage + e_base + run0 + i, s_esc[wave][i]);
    }
    if constexpr (PACK == 0) {
      // bit-pack the wave tile: word w holds bits [32w, 32w + 32) of its stream
      const uint64_t word0 = t0 * B / 32;
      for (uint32_t w = lane; w < tile_words; w += 64) {
        if (word0 + w >= P.packed_words) break;
        const uint32_t bit0 = w * 32;
        // floor(bit0 / B) and floor((bit0 + 31) / B); mulB does not exist for B = 1
        const uint32_t e_first = B == 1 ? bit0 : __umulhi(bit0, P.mulB);
        const uint32_t e_last = B == 1 ? bit0 + 31 : __umulhi(bit0 + 31, P.mulB);
        uint32_t word = 0;
        for (uint32_t e = e_first; e <= e_last && e < (uint32_t)WT; ++e) {
          const uint32_t v = idx[e];
          const int sh = (int)(e * B) - (int)bit0;
          word |= sh >= 0 ? (v << sh) : (v >> (-sh));
        }
        gstore(P.packed + word0 + w, word);
      }
    }
    wave_lds_sync();
  };

  auto load_full = [&](uint64_t tile, nk_u32x4 (&cv)[R]) {
#pragma unroll
    for (int r = 0; r < R; ++r) cv[r] = gload(wv + tile * (WT / V) + (uint64_t)r * 64 + lane);
  };
  auto load_part = [&](uint64_t tile, nk_u32x4 (&cv)[R]) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint64_t vi = tile * (WT / V) + (uint64_t)r * 64 + lane;
      if (vi < nvec) {
        cv[r] = gload(wv + vi);
      } else {
#pragma unroll
        for (int h = 0; h < 4; ++h) {
          const uint64_t j = vi * V + 2 * h;
          const uint32_t a = j < P.n ? gload(P.wcode + j) : WC_INVALID;
          const uint32_t b = j + 1 < P.n ? gload(P.wcode + j + 1) : WC_INVALID;
          cv[r][h] = a | (b << 16);
        }
      }
    }
  };
  const uint64_t full_tiles = nvec / (WT / V);  // tiles with every vector in range
  const uint64_t tf = te < full_tiles ? te : (tb > full_tiles ? tb : full_tiles);
  nk_u32x4 ca[R], cb[R];
  if (tb < tf) {
    load_full(tb, ca);
    for (uint64_t tile = tb;; tile += 2) {
      const uint64_t n1 = tile + 1 < tf ? tile + 1 : tile;
      load_full(n1, cb);
      process(std::true_type{}, tile, ca);
      if (tile + 1 >= tf) break;
      const uint64_t n2 = tile + 2 < tf ? tile + 2 : tile + 1;
      load_full(n2, ca);
      process(std::true_type{}, tile + 1, cb);
      if (tile + 2 >= tf) break;
    }
  }
  for (uint64_t tile = tf; tile < te; ++tile) {  // at most the array's last tile
    load_part(tile, ca);
    process(std::false_type{}, tile, ca);
  }
  if (lane == 0 && unit < P.n_units) gstore(P.unit_cnt + unit, run);
}

template <typename T, typename S>
__global__ void __launch_bounds__(UNIT_TPB) k_gather(S src, Geo g) {
  constexpr int NWAVE = UNIT_TPB / 64;
  __shared__ unsigned long long s_part[NWAVE];
  __shared__ uint32_t s_cnt[NWAVE];
  // the workgroup's NWAVE units are consecutive units of one job (jobs own
  // multiples of four)
  const uint32_t ublk = g.u_begin + blockIdx.x * NWAVE;
  if (ublk >= g.u_end) return;
  const uint32_t jb = g.unit0 ? find_job(g.unit0, g.job_begin, g.job_end, ublk) : g.job_begin;
  const CParams& P = src.job(jb);
  const uint32_t unit0 = ublk - (g.unit0 ? g.unit0[jb] : 0u);
  const int tid = threadIdx.x, wave = tid / 64, lane = lane_id();
  // the escapes of the job's units before unit0 (the first workgroup of the
  // job sums all of them: the job's total)
  const bool first = unit0 == 0;
  const uint32_t lim = first ? P.n_units : (unit0 < P.n_units ? unit0 : P.n_units);
  unsigned long long sum = strided_sum_u32(P.unit_cnt, tid, lim, UNIT_TPB);
  sum = wave_sum_u64(sum);
  if (lane == 0) {
    s_part[wave] = sum;
    s_cnt[wave] = unit0 + wave < P.n_units ? gload(P.unit_cnt + unit0 + wave) : 0u;
  }
  __syncthreads();
  unsigned long long before = 0;
#pragma unroll
  for (int w = 0; w < NWAVE; ++w) before += s_part[w];
  if (first && tid == 0) {
    P.ctl->n_inc = (unsigned)before;  // the job's total
    write_header(P);
  }
  unsigned long long off = first ? 0ull : before;
  for (int w = 0; w < wave; ++w) off += s_cnt[w];
  const uint32_t unit = unit0 + wave;
  if (unit >= P.n_units) return;
  const uint64_t span = P.tiles_per_unit * P.tile_elems;  // elements of a unit range
  const uint64_t e0 = (uint64_t)unit * span;
  if (e0 >= P.n) return;
  uint64_t e1 = e0 + span;
  e1 = e1 < P.n ? e1 : P.n;
  const unsigned cnt = s_cnt[wave];
  T* __restrict__ incomp = static_cast<T*>(P.incomp);
  if (P.pre) {
    // staged element indices: fetch the values from curr, eight per lane
    // in flight (the fetches are scattered: each waits a full memory latency)
    const uint32_t* __restrict__ st = static_cast<const uint32_t*>(P.scratch);
    const T* __restrict__ curr = static_cast<const T*>(P.curr);
    constexpr int GU = 8;
    for (unsigned i0 = 0; i0 < cnt; i0 += 64 * GU) {
      uint32_t jx[GU];
      T vx[GU];
#pragma unroll
      for (int u = 0; u < GU; ++u) {
        const unsigned i = i0 + (unsigned)u * 64 + (unsigned)lane;
        jx[u] = i < cnt ? gload(st + e0 + i) : 0u;
      }
#pragma unroll
      for (int u = 0; u < GU; ++u) {
        const unsigned i = i0 + (unsigned)u * 64 + (unsigned)lane;
        vx[u] = i < cnt ? gload(curr + jx[u]) : (T)0;
      }
#pragma unroll
      for (int u = 0; u < GU; ++u) {
        const unsigned i = i0 + (unsigned)u * 64 + (unsigned)lane;
        if (i < cnt) gstore(incomp + off + i, vx[u]);
      }
    }
    // block b starting in the range: off plus the range's incompressible
    // points before its first element (the staged indices ascend)
    const uint64_t b0 = (e0 + P.epb - 1) / P.epb;
    for (uint64_t b = b0 + lane; b * P.epb < e1; b += 64) {
      const uint64_t first = b * P.epb;
      unsigned a = 0, z = cnt;
      while (a < z) {
        const unsigned mid = (a + z) >> 1;
        if ((uint64_t)gload(st + e0 + mid) < first) a = mid + 1; else z = mid;
      }
      gstore(P.block_inc_off + b, (int64_t)(off + a));
    }
  } else {
    const T* __restrict__ scratch = static_cast<const T*>(P.scratch);
    for (unsigned i = lane; i < cnt; i += 64) gstore(incomp + off + i, gload(scratch + e0 + i));
    const uint64_t b0 = (e0 + P.epb - 1) / P.epb;
    for (uint64_t b = b0 + lane; b * P.epb < e1; b += 64)
      gstore(P.block_inc_off + b, gload(P.block_inc_off + b) + (int64_t)off);
  }
}

// Header of the call (Fig. 2's attributes plus this library's counts).
__device__ void write_header(const CParams& P) {
  const Ctl* c = P.ctl;
  numarck_header* h = P.hdr;
  const uint64_t L = P.dtype == NUMARCK_F32 ? 4 : 8;
  const unsigned long long n_inc = c->n_inc;
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

// Kernel of an encoder specialisation.
template <typename T, typename S, int NT>
static void (*encoder_kernel_nt(int cls))(S, Geo) {
  switch (cls) {
    case 0: return k_encode<T, uint8_t, 0, S, NT>;
    case 1: return k_encode<T, uint8_t, 8, S, NT>;
    case 2: return k_encode<T, uint16_t, 0, S, NT>;
    default: return k_encode<T, uint16_t, 16, S, NT>;
  }
}
template <typename T, int NT>
static void (*encoder_kernel_ew_nt(int cls))(OneJob, Geo) {
  switch (cls) {
    case 0: return k_encode<T, uint8_t, 0, OneJob, NT, true>;
    case 1: return k_encode<T, uint8_t, 8, OneJob, NT, true>;
    case 2: return k_encode<T, uint16_t, 0, OneJob, NT, true>;
    default: return k_encode<T, uint16_t, 16, OneJob, NT, true>;
  }
}
template <typename T, typename S>
static void (*encoder_kernel(int cls, uint32_t nt))(S, Geo) {
  if constexpr (std::is_same<S, JobTable>::value)
    if (nt == 2) return encoder_kernel_nt<T, S, 2>(cls);
  return nt == 1 ? encoder_kernel_nt<T, S, 1>(cls) : encoder_kernel_nt<T, S, 0>(cls);
}

// Kernel of a precoded encoder specialisation.
template <typename T, typename S>
static void (*encoder_pre_kernel(int cls))(S, Geo) {
  switch (cls) {
    case 0: return k_encode_pre<T, uint8_t, 0, S>;
    case 1: return k_encode_pre<T, uint8_t, 8, S>;
    case 2: return k_encode_pre<T, uint16_t, 0, S>;
    default: return k_encode_pre<T, uint16_t, 16, S>;
  }
}

template <typename S>
static int encoder_pre_occupancy_t(int dtype, int cls) {
  void (*k)(S, Geo) = dtype == NUMARCK_F32 ? encoder_pre_kernel<float, S>(cls)
                                           : encoder_pre_kernel<double, S>(cls);
  int occ = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k, UNIT_TPB, 0) != hipSuccess || occ < 1)
    occ = 1;
  return occ;
}

int encoder_pre_occupancy(int dtype, int cls, bool table) {
  return table ? encoder_pre_occupancy_t<JobTable>(dtype, cls)
               : encoder_pre_occupancy_t<OneJob>(dtype, cls);
}

template <typename S>
static int encoder_occupancy_t(int dtype, int cls) {
  void (*k)(S, Geo) = dtype == NUMARCK_F32 ? encoder_kernel<float, S>(cls, 0)
                                           : encoder_kernel<double, S>(cls, 0);
  int occ = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k, UNIT_TPB, 0) != hipSuccess || occ < 1)
    occ = 1;
  return occ;
}

int encoder_occupancy(int dtype, int cls, bool table) {
  return table ? encoder_occupancy_t<JobTable>(dtype, cls) : encoder_occupancy_t<OneJob>(dtype, cls);
}

// Two range-pass workgroups per compute unit: fewer concurrent streams read
// HBM faster (512^3 float64: 310 us against 334 at eight).
Tuning default_tuning() { return Tuning{2u, 2u, 1u, 0u, 100u, 0u}; }

static Geo group_geo(const Geo& base, const JobGroup& jg) {
  Geo g = base;
  g.stream_nt = jg.nt;
  g.chain = jg.chain;
  if (jg.chunk_vec) g.chunk_vec = jg.chunk_vec;
  g.job_begin = jg.job_begin;
  g.job_end = jg.job_end;
  g.c_begin = jg.c_begin;
  g.c_end = jg.c_end;
  g.u_begin = jg.u_begin;
  g.u_end = jg.u_end;
  return g;
}

static uint64_t clamp_blocks(uint64_t want, uint64_t cap) {
  if (want > cap) want = cap;
  return want < 1 ? 1 : want;
}

// The compression chain over all jobs of `src`: one launch per pass and per
// element type (per index-width class for the encoder), whatever the number
// of jobs.
// phases: 1 = the passes before top-k (they do not depend on B), 2 = top-k
// and after.
// phases bit: the zero-anchored form (k_init sets the window in place of the
// range pass, k_zafin after the histogram)
constexpr unsigned PH_ZA = 8;
constexpr uint32_t CHAIN_BLOCKS_PER_CU = 8;

template <typename S>
static hipError_t run_chain(S src, const Geo& base, uint32_t njobs, const JobGroup* rg,
                            uint32_t nrg, const JobGroup* hg, uint32_t nhg, const JobGroup* dg,
                            uint32_t ndg, const JobGroup* eg, uint32_t neg, const Tuning& tn,
                            hipStream_t s, unsigned phases = 3) {
  const Geometry G = geometry();
  Geo all = base;
  all.job_begin = 0;
  all.job_end = njobs;
  const uint64_t aux = njobs == 1 ? (uint64_t)G.cus * 2
                                  : clamp_blocks((uint64_t)G.cus * 2 / njobs, 64) < 8
                                        ? 8
                                        : clamp_blocks((uint64_t)G.cus * 2 / njobs, 64);
  const bool za = (phases & PH_ZA) != 0;
  all.za = za ? 1u : 0u;
  if (phases & 1) {
  NK_LAUNCH(KK_INIT, k_init<S>, njobs, 256, src, all);
  for (uint32_t i = 0; i < (za ? 0u : nrg); ++i) {
    const Geo g = group_geo(base, rg[i]);
    const uint64_t chunks = g.c_end - g.c_begin;
    if (!chunks) continue;
    // a time chain's sweep keeps two snapshots per thread in flight and
    // reads the next: it wants at least eight workgroups per compute unit
    const uint32_t rbpc = rg[i].chain && tn.range_blocks_per_cu < CHAIN_BLOCKS_PER_CU
                              ? CHAIN_BLOCKS_PER_CU
                              : tn.range_blocks_per_cu;
    const uint64_t blocks = clamp_blocks(chunks, (uint64_t)G.cus * rbpc);
    const bool f32 = rg[i].dtype == NUMARCK_F32;
    if (rg[i].chain) {
      if constexpr (std::is_same<S, JobTable>::value) {
        if (g.stream_nt == 1) {
          if (f32) NK_LAUNCH(KK_RANGE, (k_range_chain<float, true>), blocks, RNG_TPB, src, g);
          else NK_LAUNCH(KK_RANGE, (k_range_chain<double, true>), blocks, RNG_TPB, src, g);
        } else {
          if (f32) NK_LAUNCH(KK_RANGE, (k_range_chain<float, false>), blocks, RNG_TPB, src, g);
          else NK_LAUNCH(KK_RANGE, (k_range_chain<double, false>), blocks, RNG_TPB, src, g);
        }
      } else {
        return hipErrorInvalidValue;  // chains exist in batches only
      }
    } else if (g.stream_nt == 1) {
      if (f32) NK_LAUNCH(KK_RANGE, (k_range<float, S, true>), blocks, RNG_TPB, src, g);
      else NK_LAUNCH(KK_RANGE, (k_range<double, S, true>), blocks, RNG_TPB, src, g);
    } else {
      if (f32) NK_LAUNCH(KK_RANGE, (k_range<float, S, false>), blocks, RNG_TPB, src, g);
      else NK_LAUNCH(KK_RANGE, (k_range<double, S, false>), blocks, RNG_TPB, src, g);
    }
  }
  for (uint32_t i = 0; i < nhg; ++i) {
    Geo g = group_geo(base, hg[i]);
    g.za = all.za;
    const uint64_t chunks = g.c_end - g.c_begin;
    if (!chunks) continue;
    uint64_t blocks = clamp_blocks(chunks, (uint64_t)G.cus * tn.hist_blocks_per_cu);
    if (g.chain && blocks < g.job_end - g.job_begin) blocks = g.job_end - g.job_begin;
    const bool f32 = hg[i].dtype == NUMARCK_F32;
    const uint32_t nt = g.stream_nt;
    if (tn.hist_lds) {
      // shared snapshots (mode 2) are read cached here: the histogram's
      // workgroups walk consecutive pairs in step and hit both reads
      if (f32) {
        if (nt == 1) NK_LAUNCH(KK_HIST, (k_hist<float, S, true, 1>), blocks, HIST_TPB, src, g);
        else NK_LAUNCH(KK_HIST, (k_hist<float, S, true, 0>), blocks, HIST_TPB, src, g);
      } else {
        if (nt == 1) NK_LAUNCH(KK_HIST, (k_hist<double, S, true, 1>), blocks, HIST_TPB, src, g);
        else NK_LAUNCH(KK_HIST, (k_hist<double, S, true, 0>), blocks, HIST_TPB, src, g);
      }
    } else {  // global counts: the chosen few; streamed inputs are cached
      if (f32) NK_LAUNCH(KK_HIST, (k_hist<float, S, false, 0>), blocks, HIST_TPB, src, g);
      else NK_LAUNCH(KK_HIST, (k_hist<double, S, false, 0>), blocks, HIST_TPB, src, g);
    }
  }
  if (za) NK_LAUNCH(KK_DERIVE, k_zafin<S>, njobs, 256, src, all);
  NK_LAUNCH(KK_HCLEAR, k_hclear<S>, dim3((unsigned)aux, njobs), 256, src, all);
  NK_LAUNCH(KK_HINSERT, k_hinsert<S>, dim3((unsigned)aux, njobs), 256, src, all);
  }
  if (!(phases & 2)) return hipSuccess;
  for (uint32_t i = 0; i < ndg; ++i) {
    const Geo g = group_geo(base, dg[i]);
    const uint32_t nj = g.job_end - g.job_begin;
    // k_select ranks the selected tail bins itself when k <= SEL_TPB
    bool tailrank = true;
    if constexpr (std::is_same<S, OneJob>::value) tailrank = src.p.k > (uint32_t)SEL_TPB;
    if (dg[i].dtype == NUMARCK_F32) {
      NK_LAUNCH(KK_SELECT, (k_select<float, S>), nj, SEL_TPB, src, g);
      if (tailrank) NK_LAUNCH(KK_TAILRANK, (k_tailrank<float, S>), dim3(64, nj), TR_TPB, src, g);
    } else {
      NK_LAUNCH(KK_SELECT, (k_select<double, S>), nj, SEL_TPB, src, g);
      if (tailrank) NK_LAUNCH(KK_TAILRANK, (k_tailrank<double, S>), dim3(64, nj), TR_TPB, src, g);
    }
  }
  for (uint32_t i = 0; i < neg; ++i) {
    const Geo g = group_geo(base, eg[i]);
    const uint32_t blocks = (g.u_end - g.u_begin) / 4;
    if (!blocks) continue;
    void (*k)(S, Geo) = eg[i].dtype == NUMARCK_F32
                            ? encoder_kernel<float, S>(eg[i].cls, g.stream_nt)
                            : encoder_kernel<double, S>(eg[i].cls, g.stream_nt);
    if (eg[i].pre)
      k = eg[i].dtype == NUMARCK_F32 ? encoder_pre_kernel<float, S>(eg[i].cls)
                                     : encoder_pre_kernel<double, S>(eg[i].cls);
    NK_LAUNCH(KK_ENCODE, k, blocks, UNIT_TPB, src, g);
  }
  for (uint32_t i = 0; i < ndg; ++i) {
    const Geo g = group_geo(base, dg[i]);
    const uint32_t blocks = (g.u_end - g.u_begin) / 4;
    if (!blocks) continue;
    if (dg[i].dtype == NUMARCK_F32)
      NK_LAUNCH(KK_GATHER, (k_gather<float, S>), blocks, UNIT_TPB, src, g);
    else
      NK_LAUNCH(KK_GATHER, (k_gather<double, S>), blocks, UNIT_TPB, src, g);
  }
  return hipSuccess;
}

uint64_t stream_chunks(uint64_t n, int dtype, uint32_t chunk_vec) {
  if (n == 0) return 0;
  const uint64_t nvec = n / (dtype == NUMARCK_F32 ? 4 : 2);
  const uint64_t c = (nvec + chunk_vec - 1) / chunk_vec;
  return c < 1 ? 1 : c;
}

hipError_t launch_compress(const CParams& P0, const Tuning& tn, hipStream_t s) {
  return launch_compress_phase(P0, tn, s, 3);
}

hipError_t launch_autob(const CParams& P, uint32_t b_lo, uint32_t b_hi, hipStream_t s) {
  Geo g{};
  g.job_begin = 0;
  g.job_end = 1;
  NK_LAUNCH(KK_SELECT, k_autob<OneJob>, b_hi - b_lo + 1, SEL_TPB, OneJob{P}, g, b_lo, b_hi);
  return hipSuccess;
}

hipError_t launch_compress_phase(const CParams& P0, const Tuning& tn, hipStream_t s,
                                 unsigned phases) {
  const Geometry G = geometry();
  CParams P = P0;
  const int cls = enc_class(P.B);
  // Precoded encoding wherever the histogram counts in LDS and no
  // reconstruction is asked for (the encoder then never reads the values of
  // its compressible points).
  P.pre = tn.hist_lds && P.recon == nullptr ? 1u : 0u;
  if (P.pre) {
    P.tile_elems = (uint32_t)PRE_WAVE_TILE;
    P.n_tiles = (P.n + PRE_WAVE_TILE - 1) / PRE_WAVE_TILE;
  }
  const int occ = P.pre ? encoder_pre_occupancy(P.dtype, cls, false)
                        : encoder_occupancy(P.dtype, cls, false);
  const uint64_t resident = (uint64_t)G.cus * occ * 4 * tn.unit_pct / 100;
  P.n_units = range_units(P.n_tiles, (int)(resident < 4 ? 4 : resident));
  P.tiles_per_unit = (P.n_tiles + P.n_units - 1) / P.n_units;
  Geo base{};
  base.chunk_vec = chunk_vec_for(tn.chunk_vec, P.n / (P.dtype == NUMARCK_F32 ? 4 : 2), G.cus);
  JobGroup grp{};
  grp.dtype = P.dtype;
  grp.cls = cls;
  grp.job_begin = 0;
  grp.job_end = 1;
  grp.c_begin = 0;
  grp.chunk_vec = base.chunk_vec;
  grp.c_end = stream_chunks(P.n, P.dtype, base.chunk_vec);
  grp.u_begin = 0;
  grp.u_end = P.n_units;
  grp.pre = P.pre;
  grp.nt = stream_nt_for(tn.stream_loads, 2 * P.n * (P.dtype == NUMARCK_F32 ? 4 : 8),
                         P.prev == P.curr);
  if (grp.nt == 2) grp.nt = 0;  // one job: its two inputs are one snapshot
  return run_chain(OneJob{P}, base, 1, &grp, 1, &grp, 1, &grp, 1, &grp, 1, tn, s, phases);
}

hipError_t launch_compress_za(const CParams& P, const Tuning& tn, hipStream_t s) {
  return launch_compress_phase(P, tn, s, 3 | PH_ZA);
}

hipError_t launch_compress_ew(const CParams& P0, const Tuning& tn, hipStream_t s) {
  const Geometry G = geometry();
  CParams P = P0;
  const int cls = enc_class(P.B);
  const int occ = encoder_occupancy(P.dtype, cls, false);
  const uint64_t resident = (uint64_t)G.cus * occ * 4 * tn.unit_pct / 100;
  P.n_units = range_units(P.n_tiles, (int)(resident < 4 ? 4 : resident));
  P.tiles_per_unit = (P.n_tiles + P.n_units - 1) / P.n_units;
  const bool f32 = P.dtype == NUMARCK_F32;
  Geo g{};
  g.chunk_vec = chunk_vec_for(tn.chunk_vec, P.n / (f32 ? 4 : 2), G.cus);
  g.job_begin = 0;
  g.job_end = 1;
  g.c_begin = 0;
  g.c_end = stream_chunks(P.n, P.dtype, g.chunk_vec);
  g.u_begin = 0;
  g.u_end = P.n_units;
  uint32_t nt = stream_nt_for(tn.stream_loads, 2 * P.n * (f32 ? 4 : 8), P.prev == P.curr);
  g.stream_nt = nt == 1 ? 1u : 0u;
  const OneJob src{P};
  NK_LAUNCH(KK_INIT, k_init<OneJob>, 1, 256, src, g);
  if (g.c_end) {
    const uint64_t blocks = clamp_blocks(g.c_end, (uint64_t)G.cus * tn.range_blocks_per_cu);
    if (g.stream_nt == 1) {
      if (f32) NK_LAUNCH(KK_RANGE, (k_range<float, OneJob, true>), blocks, RNG_TPB, src, g);
      else NK_LAUNCH(KK_RANGE, (k_range<double, OneJob, true>), blocks, RNG_TPB, src, g);
    } else {
      if (f32) NK_LAUNCH(KK_RANGE, (k_range<float, OneJob, false>), blocks, RNG_TPB, src, g);
      else NK_LAUNCH(KK_RANGE, (k_range<double, OneJob, false>), blocks, RNG_TPB, src, g);
    }
  }
  if (f32) NK_LAUNCH(KK_DERIVE, (k_ewprep<float, OneJob>), 1, 256, src, g);
  else NK_LAUNCH(KK_DERIVE, (k_ewprep<double, OneJob>), 1, 256, src, g);
  const uint32_t eblocks = (g.u_end - g.u_begin) / 4;
  if (eblocks) {
    void (*k)(OneJob, Geo) =
        f32 ? (g.stream_nt == 1 ? encoder_kernel_ew_nt<float, 1>(cls)
                                : encoder_kernel_ew_nt<float, 0>(cls))
            : (g.stream_nt == 1 ? encoder_kernel_ew_nt<double, 1>(cls)
                                : encoder_kernel_ew_nt<double, 0>(cls));
    NK_LAUNCH(KK_ENCODE, k, eblocks, UNIT_TPB, src, g);
  }
  if (eblocks) {
    if (f32) NK_LAUNCH(KK_GATHER, (k_gather<float, OneJob>), eblocks, UNIT_TPB, src, g);
    else NK_LAUNCH(KK_GATHER, (k_gather<double, OneJob>), eblocks, UNIT_TPB, src, g);
  }
  return hipSuccess;
}

hipError_t launch_compress_batch(const BatchLaunch& b, hipStream_t s) {
  Geo base{};
  base.chunk0 = b.chunk0_dev;
  base.unit0 = b.unit0_dev;
  base.chunk_vec = b.tune.chunk_vec ? b.tune.chunk_vec : 4096;  // groups carry their own
  return run_chain(JobTable{b.jobs_dev}, base, b.njobs, b.rgroups, b.n_rgroups, b.hgroups,
                   b.n_hgroups, b.dgroups, b.n_dgroups, b.egroups, b.n_egroups, b.tune, s,
                   3u | (b.za ? PH_ZA : 0u));
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
