/*
 * numarck_oracle.c -- plain, slow CPU reference of the NUMARCK compression path
 * ("Parallel Implementation of Lossy Data Compression for Temporal Data Sets",
 * Yuan et al., arXiv 1703.02438).
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark.  The product library never calls it and
 * shares no code with it.
 *
 * The method is a heuristic (top-k coverage is not optimal, Sec. V-D), so this
 * file spells its steps out in the paper's order:
 *   1. change ratio of every point, eq. (1)                    (Sec. III-A, IV-A)
 *   2. range [lo, hi] of the ratios                              (Sec. IV-A)
 *   3. fine bins of width 2E anchored at lo, histogram           (Sec. IV-B-1)
 *   4. top-k bins, k = 2^B - 1, by count                         (Sec. IV-B-1)
 *   5. index each point by its bin, escape code 2^B - 1 otherwise (Sec. III-C)
 *   6. incompressible values kept as they are, in element order  (Sec. III-C)
 *   7. B-bit packing of the index table                          (Sec. IV-C)
 *   8. per-block count of earlier incompressible points          (Sec. IV-C)
 *   9. decompression by eq. (4), full and partial                (Sec. III-E, V-C)
 * plus the choice of B by eqs. (5)-(6) (Sec. IV-B-2) and, as an alternative to
 * steps 3-4, equal-width binning (Sec. III-B, IV-B-3); bins anchored at -E
 * (centred on multiples of 2E) in place of the smallest ratio, which needs no
 * range before the histogram; and a lossless stage for the index table (an
 * exponential-Golomb code over frequency ranks in place of ZLIB, Sec. IV-C).
 *
 * Readings taken where the paper is silent or garbled:
 *   - a point is valid when its previous value is nonzero and finite, the new
 *     value is finite, the ratio is finite and |ratio| <= E * 2^50; invalid
 *     points are always stored as incompressible values;
 *   - bin m holds ratios with floor((d - lo) / (2E)) == m, evaluated in binary64;
 *   - ties in the top-k order go to the lower bin id; empty bins are never
 *     selected; the selected bins get indices in ascending bin-id order;
 *   - bin centre c_m = lo + (2m + 1) E in binary64, stored in the snapshot type;
 *   - reconstruction R = T(p * (1 + c)) (the only reading of eq. (4) consistent
 *     with eq. (1)); a point is kept only if |R - q| <= E |p| after rounding;
 *   - zero-anchored bins: lo is taken as -E, so bin m is floor((d + E) / 2E),
 *     computed as floor((d - lo) / 2E), with centre lo + (2m + 1) E; the
 *     header then reports lo = -E, hi = 0 and M = 0 (no range is formed);
 *   - equal-width binning: w = (hi - lo) / k, chunk i = min(floor((d - lo) / w),
 *     k - 1) (0 when w is 0), centre lo + (i + 1/2) w; the rest as above;
 *   - index bits are written least-significant first into a contiguous stream
 *     of little-endian 32-bit words; elements per block = floor(8 * bytes / B).
 *
 * All arithmetic is binary64, round-to-nearest-even, evaluated exactly as
 * written; build with -ffp-contract=off and without fast-math.
 */
#include "numarck_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads of the per-element loops (ratios, range, bin ids, candidate
 * indices, verification).  Every such loop writes element j's results from
 * element j's inputs only, and the range's min/max is a total order, so any
 * thread count gives the same bytes; the histogram, the selection, the
 * placement of the incompressible values, the packing and the block offsets
 * stay serial.  1 by default. */
static int g_threads = 1;

int orc_set_threads(int n) {
#ifdef _OPENMP
  g_threads = n < 1 ? 1 : n;
#else
  (void)n;
  g_threads = 1;
#endif
  return g_threads;
}

/* ---------------------------------------------------------------- helpers */

static double load_as_double(const void* base, int dtype, uint64_t j) {
  if (dtype == ORC_F32) {
    float v;
    memcpy(&v, (const char*)base + 4 * j, 4);
    return (double)v;
  }
  double v;
  memcpy(&v, (const char*)base + 8 * j, 8);
  return v;
}

/* Round a binary64 value to the snapshot type (nearest-even) and store it. */
static void store_rounded(void* base, int dtype, uint64_t j, double v) {
  if (dtype == ORC_F32) {
    float f = (float)v;
    memcpy((char*)base + 4 * j, &f, 4);
  } else {
    memcpy((char*)base + 8 * j, &v, 8);
  }
}

/* The value as stored in the snapshot type, read back as binary64. */
static double rounded_to_type(int dtype, double v) {
  if (dtype == ORC_F32) return (double)(float)v;
  return v;
}

/* Copy one element bit for bit (keeps NaN payloads and signed zeros). */
static void copy_elem(void* dst, uint64_t dj, const void* src, uint64_t sj, int dtype) {
  size_t L = dtype == ORC_F32 ? 4 : 8;
  memcpy((char*)dst + L * dj, (const char*)src + L * sj, L);
}

static void zero_elem(void* dst, uint64_t dj, int dtype) {
  size_t L = dtype == ORC_F32 ? 4 : 8;
  memset((char*)dst + L * dj, 0, L);
}

static size_t elem_size(int dtype) { return dtype == ORC_F32 ? 4 : 8; }

static int check_args(int dtype, double E, uint32_t B) {
  if (dtype != ORC_F32 && dtype != ORC_F64) return ORC_EDTYPE;
  if (B < 1 || B > 16) return ORC_EBITS;
  if (!(E > 0.0 && E <= 1.0)) return ORC_EBOUND;
  return ORC_OK;
}

/* ------------------------------------------------ step 1: change ratio, eq. (1) */

int orc_ratio(const void* prev, const void* curr, uint64_t n, int dtype, double E,
              double* d, uint8_t* valid) {
  double cap = ldexp(E, 50);
#pragma omp parallel for schedule(static) num_threads(g_threads)
  for (uint64_t j = 0; j < n; j++) {
    double p = load_as_double(prev, dtype, j);
    double q = load_as_double(curr, dtype, j);
    double r = (q - p) / p;
    d[j] = r;
    valid[j] = (p != 0.0) && isfinite(p) && isfinite(q) && isfinite(r) && fabs(r) <= cap;
  }
  return ORC_OK;
}

/* ------------------------------------------------ step 2: range of the ratios */

/* a precedes b in the order used for lo/hi: numeric order, -0 before +0. */
static int precedes(double a, double b) {
  if (a < b) return 1;
  return a == b && signbit(a) && !signbit(b);
}

uint64_t orc_range(const double* d, const uint8_t* valid, uint64_t n, double* lo, double* hi) {
  uint64_t nv = 0;
  double mn = 0.0, mx = 0.0;
#pragma omp parallel num_threads(g_threads)
  {
    uint64_t tnv = 0;
    double tmn = 0.0, tmx = 0.0;
#pragma omp for schedule(static)
    for (uint64_t j = 0; j < n; j++) {
      if (!valid[j]) continue;
      if (tnv == 0) {
        tmn = d[j];
        tmx = d[j];
      } else {
        if (precedes(d[j], tmn)) tmn = d[j];
        if (precedes(tmx, d[j])) tmx = d[j];
      }
      tnv++;
    }
#pragma omp critical
    if (tnv) {
      if (nv == 0) {
        mn = tmn;
        mx = tmx;
      } else {
        if (precedes(tmn, mn)) mn = tmn;
        if (precedes(mx, tmx)) mx = tmx;
      }
      nv += tnv;
    }
  }
  *lo = mn;
  *hi = mx;
  return nv;
}

/* ------------------------------------------------ step 3: fine bins of width 2E */

void orc_bin_ids(const double* d, const uint8_t* valid, uint64_t n, double lo, double E,
                 int64_t* m) {
  double width = 2.0 * E;
#pragma omp parallel for schedule(static) num_threads(g_threads)
  for (uint64_t j = 0; j < n; j++) {
    if (valid[j])
      m[j] = (int64_t)floor((d[j] - lo) / width);
    else
      m[j] = -1;
  }
}

/* ------------------------------------------------ step 4: histogram */

static int cmp_i64(const void* a, const void* b) {
  int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
  return (x > y) - (x < y);
}

int64_t orc_histogram(const int64_t* m, const uint8_t* valid, uint64_t n, int64_t* ids,
                      uint32_t* counts) {
  int64_t* s = (int64_t*)malloc((n ? n : 1) * sizeof(int64_t));
  if (!s) return -1;
  uint64_t nv = 0;
  for (uint64_t j = 0; j < n; j++)
    if (valid[j]) s[nv++] = m[j];
  qsort(s, nv, sizeof(int64_t), cmp_i64);
  int64_t nb = 0;
  for (uint64_t i = 0; i < nv; i++) {
    if (nb > 0 && ids[nb - 1] == s[i]) {
      counts[nb - 1] += 1;
    } else {
      ids[nb] = s[i];
      counts[nb] = 1;
      nb++;
    }
  }
  free(s);
  return nb;
}

/* ------------------------------------------------ step 5: top-k selection */

typedef struct {
  int64_t id;
  uint32_t count;
} bin_t;

/* Larger count first; equal counts: lower bin id first. */
static int cmp_rank(const void* a, const void* b) {
  const bin_t* x = (const bin_t*)a;
  const bin_t* y = (const bin_t*)b;
  if (x->count != y->count) return x->count > y->count ? -1 : 1;
  return (x->id > y->id) - (x->id < y->id);
}

int64_t orc_topk(const int64_t* ids, const uint32_t* counts, int64_t nbins, uint32_t k,
                 int64_t* sel, uint32_t* tau) {
  bin_t* b = (bin_t*)malloc((nbins ? nbins : 1) * sizeof(bin_t));
  if (!b) return -1;
  for (int64_t i = 0; i < nbins; i++) {
    b[i].id = ids[i];
    b[i].count = counts[i];
  }
  qsort(b, (size_t)nbins, sizeof(bin_t), cmp_rank);
  int64_t take = nbins < (int64_t)k ? nbins : (int64_t)k;
  for (int64_t i = 0; i < take; i++) sel[i] = b[i].id;
  *tau = nbins > (int64_t)k ? b[take - 1].count : 0;
  free(b);
  qsort(sel, (size_t)take, sizeof(int64_t), cmp_i64);
  return take;
}

/* ------------------------------------------------ choice of B, eqs. (5)-(6) */

/* Larger count first. */
static int cmp_count_desc(const void* a, const void* b) {
  uint32_t x = *(const uint32_t*)a, y = *(const uint32_t*)b;
  return (x < y) - (x > y);
}

/* The histogram does not depend on B, so one histogram serves every B: with
 * the counts sorted in decreasing order, the points the 2^B - 1 selected bins
 * hold are the sum of the first 2^B - 1 counts (all of them when there are
 * fewer bins), and every other point -- the invalid ones included -- is
 * counted as incompressible, eq. (5).  Eq. (6) in bits: 8 * 2^B L for the
 * centre table, n B for the index table, 8 L per incompressible point. */
int orc_choose_B(const void* prev, const void* curr, uint64_t n, int dtype, double E,
                 uint32_t b_lo, uint32_t b_hi, uint64_t* bits, uint32_t* B_out) {
  if (b_lo < 1 || b_hi > 16 || b_lo > b_hi) return ORC_EBITS;
  int st = check_args(dtype, E, b_lo);
  if (st != ORC_OK) return st;
  if (n >= ((uint64_t)1 << 32)) return ORC_EINVAL;
  if (!bits || !B_out || (n && (!prev || !curr))) return ORC_EINVAL;
  const uint64_t L = elem_size(dtype);
  const uint64_t nn = n ? n : 1;
  double* d = (double*)malloc(nn * sizeof(double));
  uint8_t* valid = (uint8_t*)malloc(nn);
  int64_t* m = (int64_t*)malloc(nn * sizeof(int64_t));
  int64_t* hid = (int64_t*)malloc(nn * sizeof(int64_t));
  uint32_t* hcnt = (uint32_t*)malloc(nn * sizeof(uint32_t));
  if (!d || !valid || !m || !hid || !hcnt) {
    free(d); free(valid); free(m); free(hid); free(hcnt);
    return ORC_ENOMEM;
  }
  orc_ratio(prev, curr, n, dtype, E, d, valid);
  double lo = 0.0, hi = 0.0;
  const uint64_t n_valid = orc_range(d, valid, n, &lo, &hi);
  int64_t nbins = 0;
  if (n_valid > 0) {
    orc_bin_ids(d, valid, n, lo, E, m);
    nbins = orc_histogram(m, valid, n, hid, hcnt);
  }
  qsort(hcnt, (size_t)nbins, sizeof(uint32_t), cmp_count_desc);
  for (uint32_t B = 0; B <= 16; B++) bits[B] = 0;
  uint64_t best = 0;
  uint32_t bestB = 0;
  for (uint32_t B = b_lo; B <= b_hi; B++) {
    const int64_t k = ((int64_t)1 << B) - 1;
    uint64_t covered = 0;
    for (int64_t i = 0; i < nbins && i < k; i++) covered += hcnt[i];
    const uint64_t incompressible = n - covered;
    bits[B] = 8 * ((uint64_t)1 << B) * L + n * (uint64_t)B + 8 * L * incompressible;
    if (bestB == 0 || bits[B] < best) {
      best = bits[B];
      bestB = B;
    }
  }
  *B_out = bestB;
  free(d); free(valid); free(m); free(hid); free(hcnt);
  return ORC_OK;
}

/* ------------------------------------------------ bit packing (Sec. IV-C) */

static void put_index(uint32_t* packed, uint64_t j, uint32_t B, uint32_t idx) {
  for (uint32_t b = 0; b < B; b++) {
    uint64_t bit = j * B + b;
    if ((idx >> b) & 1u) packed[bit >> 5] |= 1u << (bit & 31);
  }
}

static uint32_t get_index(const uint32_t* packed, uint64_t j, uint32_t B) {
  uint32_t idx = 0;
  for (uint32_t b = 0; b < B; b++) {
    uint64_t bit = j * B + b;
    idx |= ((packed[bit >> 5] >> (bit & 31)) & 1u) << b;
  }
  return idx;
}

static int64_t find_sorted(const int64_t* a, int64_t len, int64_t key) {
  const int64_t* hit = (const int64_t*)bsearch(&key, a, (size_t)len, sizeof(int64_t), cmp_i64);
  return hit ? (int64_t)(hit - a) : -1;
}

/* ------------------------------------------------ steps 5-8 for any binning */

/* cand[j]: the index of point j's bin among the bin centres, or -1 (invalid
 * point, or a bin without a centre).  Each candidate is kept only if its
 * reconstruction T(p (1 + c)) is within E |p| of the new value (Sec. III-C);
 * every other point gets the escape code and its value is stored as it is.
 * Then the B-bit packing and the block offsets (Sec. IV-C), and the header:
 * `part` brings the binning's fields (n_valid, M, n_nonzero, k_used, tau,
 * lo, hi).  idx: n scratch words. */
static int index_and_pack(const void* prev, const void* curr, uint64_t n, int dtype, double E,
                          uint32_t B, uint64_t block_bytes, const int64_t* cand,
                          const void* centers, uint32_t* packed, void* incomp,
                          int64_t* block_inc_off, void* recon, uint16_t* index, uint32_t* idx,
                          const orc_info* part, orc_info* info) {
  const uint32_t k = (1u << B) - 1u;
  const uint32_t esc = k;
  const size_t L = elem_size(dtype);
  uint64_t n_inc = 0;
#pragma omp parallel for schedule(static) num_threads(g_threads)
  for (uint64_t j = 0; j < n; j++) {
    uint32_t code = esc;
    const int64_t i = cand[j];
    if (i >= 0) {
      double p = load_as_double(prev, dtype, j);
      double q = load_as_double(curr, dtype, j);
      double c = load_as_double(centers, dtype, (uint64_t)i);
      double r = rounded_to_type(dtype, p * (1.0 + c));
      if (fabs(r - q) <= E * fabs(p)) {
        code = (uint32_t)i;
        if (recon) store_rounded(recon, dtype, j, r);
      }
    }
    if (code == esc && recon) copy_elem(recon, j, curr, j, dtype);
    idx[j] = code;
    if (index) index[j] = (uint16_t)code;
  }
  /* step 6: the incompressible values, in element order */
  for (uint64_t j = 0; j < n; j++) {
    if (idx[j] == esc) {
      copy_elem(incomp, n_inc, curr, j, dtype);
      n_inc++;
    }
  }

  /* step 7: packing */
  uint64_t words = (n * B + 31) / 32;
  memset(packed, 0, words * 4);
  for (uint64_t j = 0; j < n; j++) put_index(packed, j, B, idx[j]);

  /* step 8: per-block offsets into the incompressible array */
  uint64_t epb = (8 * block_bytes) / B;
  uint64_t n_blocks = (n + epb - 1) / epb;
  {
    uint64_t seen = 0;
    for (uint64_t j = 0; j < n; j++) {
      if (j % epb == 0 && block_inc_off) block_inc_off[j / epb] = (int64_t)seen;
      if (idx[j] == esc) seen++;
    }
  }

  *info = *part;
  info->n = n;
  info->n_invalid = n - part->n_valid;
  info->n_inc = n_inc;
  info->n_blocks = n_blocks;
  info->elems_per_block = epb;
  info->block_bytes = block_bytes;
  info->B = B;
  info->k = k;
  info->dtype = (uint32_t)dtype;
  info->E = E;
  info->packed_words = words;
  info->packed_bytes = words * 4;
  /* eq. (6) with the actual packed size: 2^B L + packed + n_inc L */
  info->compressed_bytes = ((uint64_t)1 << B) * L + words * 4 + n_inc * L;
  return ORC_OK;
}

/* ------------------------------------------------ the whole compression */

/* Top-k compression with bins anchored at the smallest valid ratio (the
 * paper's), or, with zero_anchor, at -E: bin m then holds the ratios with
 * floor((d + E) / 2E) == m and is centred on 2mE. */
static int compress_topk(const void* prev, const void* curr, uint64_t n, int dtype, double E,
                         uint32_t B, uint64_t block_bytes, uint32_t* packed, void* centers,
                         void* incomp, int64_t* block_inc_off, void* recon, uint16_t* index,
                         int64_t* sel_ids, orc_info* info, int zero_anchor) {
  int st = check_args(dtype, E, B);
  if (st != ORC_OK) return st;
  if (n >= ((uint64_t)1 << 32)) return ORC_EINVAL;
  if (!info || (n && (!prev || !curr || !incomp || !packed)) || !centers) return ORC_EINVAL;
  if (block_bytes == 0) block_bytes = (uint64_t)1 << 20;

  const uint32_t k = (1u << B) - 1u;
  const size_t L = elem_size(dtype);
  const uint64_t nn = n ? n : 1;

  double* d = (double*)malloc(nn * sizeof(double));
  uint8_t* valid = (uint8_t*)malloc(nn);
  int64_t* m = (int64_t*)malloc(nn * sizeof(int64_t));
  int64_t* hid = (int64_t*)malloc(nn * sizeof(int64_t));
  uint32_t* hcnt = (uint32_t*)malloc(nn * sizeof(uint32_t));
  int64_t* sel = (int64_t*)malloc((size_t)k * sizeof(int64_t));
  uint32_t* idx = (uint32_t*)malloc(nn * sizeof(uint32_t));
  if (!d || !valid || !m || !hid || !hcnt || !sel || !idx) {
    free(d); free(valid); free(m); free(hid); free(hcnt); free(sel); free(idx);
    return ORC_ENOMEM;
  }

  /* steps 1-2 */
  orc_ratio(prev, curr, n, dtype, E, d, valid);
  double lo = 0.0, hi = 0.0;
  uint64_t n_valid = orc_range(d, valid, n, &lo, &hi);
  if (zero_anchor) {  /* no range: the anchor is fixed, M is not known */
    lo = -E;
    hi = 0.0;
  }

  /* steps 3-5 */
  int64_t M = 0, nbins = 0, k_used = 0;
  uint32_t tau = 0;
  if (n_valid > 0) {
    orc_bin_ids(d, valid, n, lo, E, m);
    if (!zero_anchor) M = (int64_t)floor((hi - lo) / (2.0 * E)) + 1;
    nbins = orc_histogram(m, valid, n, hid, hcnt);
    k_used = orc_topk(hid, hcnt, nbins, k, sel, &tau);
  } else if (!zero_anchor) {
    lo = 0.0;
    hi = 0.0;
  }

  /* bin centres: c = lo + (2m + 1) E, stored in the snapshot type; unused slots 0 */
  memset(centers, 0, ((size_t)1 << B) * L);
  for (int64_t i = 0; i < k_used; i++)
    store_rounded(centers, dtype, (uint64_t)i, lo + (double)(2 * sel[i] + 1) * E);

  /* each valid point's candidate index: the rank of its bin among the
     selected ones, or none */
#pragma omp parallel for schedule(static) num_threads(g_threads)
  for (uint64_t j = 0; j < n; j++) m[j] = valid[j] ? find_sorted(sel, k_used, m[j]) : -1;

  orc_info part = {0};
  part.n_valid = n_valid;
  part.M = M;
  part.n_nonzero = (uint64_t)nbins;
  part.k_used = (uint32_t)k_used;
  part.tau = tau;
  part.lo = lo;
  part.hi = hi;
  st = index_and_pack(prev, curr, n, dtype, E, B, block_bytes, m, centers, packed, incomp,
                      block_inc_off, recon, index, idx, &part, info);
  if (st == ORC_OK && sel_ids)
    for (int64_t i = 0; i < k_used; i++) sel_ids[i] = sel[i];

  free(d); free(valid); free(m); free(hid); free(hcnt); free(sel); free(idx);
  return st;
}

int orc_compress(const void* prev, const void* curr, uint64_t n, int dtype, double E,
                 uint32_t B, uint64_t block_bytes, uint32_t* packed, void* centers,
                 void* incomp, int64_t* block_inc_off, void* recon, uint16_t* index,
                 int64_t* sel_ids, orc_info* info) {
  return compress_topk(prev, curr, n, dtype, E, B, block_bytes, packed, centers, incomp,
                       block_inc_off, recon, index, sel_ids, info, 0);
}

int orc_compress_za(const void* prev, const void* curr, uint64_t n, int dtype, double E,
                    uint32_t B, uint64_t block_bytes, uint32_t* packed, void* centers,
                    void* incomp, int64_t* block_inc_off, void* recon, uint16_t* index,
                    int64_t* sel_ids, orc_info* info) {
  return compress_topk(prev, curr, n, dtype, E, B, block_bytes, packed, centers, incomp,
                       block_inc_off, recon, index, sel_ids, info, 1);
}

/* ------------------------------------------------ equal-width binning */

/* The range [lo, hi] of the valid ratios cut into k = 2^B - 1 chunks of width
 * w = (hi - lo) / k (Sec. III-B, Sec. IV-B-3); chunk i holds the ratios with
 * floor((d - lo) / w) == i, the largest ratio (and any rounding past the last
 * chunk) in chunk k - 1, every valid ratio in chunk 0 when w = 0.  The centre
 * of chunk i is its midpoint lo + (i + 1/2) w, stored in the snapshot type.
 * Indexing, verification, packing and blocks as for top-k binning; the
 * header's M and k_used are k (0 without a valid point), n_nonzero and tau
 * are 0. */
int orc_compress_ew(const void* prev, const void* curr, uint64_t n, int dtype, double E,
                    uint32_t B, uint64_t block_bytes, uint32_t* packed, void* centers,
                    void* incomp, int64_t* block_inc_off, void* recon, uint16_t* index,
                    orc_info* info) {
  int st = check_args(dtype, E, B);
  if (st != ORC_OK) return st;
  if (n >= ((uint64_t)1 << 32)) return ORC_EINVAL;
  if (!info || (n && (!prev || !curr || !incomp || !packed)) || !centers) return ORC_EINVAL;
  if (block_bytes == 0) block_bytes = (uint64_t)1 << 20;
  const uint32_t k = (1u << B) - 1u;
  const size_t L = elem_size(dtype);
  const uint64_t nn = n ? n : 1;
  double* d = (double*)malloc(nn * sizeof(double));
  uint8_t* valid = (uint8_t*)malloc(nn);
  int64_t* cand = (int64_t*)malloc(nn * sizeof(int64_t));
  uint32_t* idx = (uint32_t*)malloc(nn * sizeof(uint32_t));
  if (!d || !valid || !cand || !idx) {
    free(d); free(valid); free(cand); free(idx);
    return ORC_ENOMEM;
  }
  orc_ratio(prev, curr, n, dtype, E, d, valid);
  double lo = 0.0, hi = 0.0;
  const uint64_t n_valid = orc_range(d, valid, n, &lo, &hi);
  if (n_valid == 0) {
    lo = 0.0;
    hi = 0.0;
  }
  const double w = (hi - lo) / (double)k;
  memset(centers, 0, ((size_t)1 << B) * L);
  if (n_valid > 0)
    for (uint32_t i = 0; i < k; i++)
      store_rounded(centers, dtype, (uint64_t)i, lo + ((double)i + 0.5) * w);
#pragma omp parallel for schedule(static) num_threads(g_threads)
  for (uint64_t j = 0; j < n; j++) {
    cand[j] = -1;
    if (!valid[j]) continue;
    int64_t i = 0;
    if (w > 0.0) {
      const double t = floor((d[j] - lo) / w);
      i = t < (double)(k - 1) ? (int64_t)t : (int64_t)(k - 1);
    }
    cand[j] = i;
  }
  orc_info part = {0};
  part.n_valid = n_valid;
  part.M = n_valid ? (int64_t)k : 0;
  part.k_used = n_valid ? k : 0;
  part.lo = lo;
  part.hi = hi;
  st = index_and_pack(prev, curr, n, dtype, E, B, block_bytes, cand, centers, packed, incomp,
                      block_inc_off, recon, index, idx, &part, info);
  free(d); free(valid); free(cand); free(idx);
  return st;
}

/* ------------------------------------------------ decompression, eq. (4) */

static void decode_one(const orc_info* info, const void* prev, const uint32_t* packed,
                       const void* centers, const void* incomp, uint64_t j, uint64_t* rank,
                       void* out, uint64_t oj, uint32_t* flags) {
  int dtype = (int)info->dtype;
  uint32_t esc = (1u << info->B) - 1u;
  uint32_t code = get_index(packed, j, info->B);
  if (code == esc) {
    if (*rank < info->n_inc) {
      copy_elem(out, oj, incomp, *rank, dtype);
    } else {
      *flags |= ORC_FLAG_INC_OVERRUN;
      zero_elem(out, oj, dtype);
    }
    *rank += 1;
    return;
  }
  if (code >= info->k_used) *flags |= ORC_FLAG_BAD_INDEX;
  double p = load_as_double(prev, dtype, j);
  double c = load_as_double(centers, dtype, code);
  store_rounded(out, dtype, oj, p * (1.0 + c));
}

int orc_decompress(const orc_info* info, const void* prev, const uint32_t* packed,
                   const void* centers, const void* incomp, void* out, uint32_t* flags) {
  if (!info || !flags) return ORC_EINVAL;
  *flags = 0;
  uint64_t rank = 0;
  for (uint64_t j = 0; j < info->n; j++)
    decode_one(info, prev, packed, centers, incomp, j, &rank, out, j, flags);
  return ORC_OK;
}

int orc_decompress_range(const orc_info* info, const void* prev, const uint32_t* packed,
                         const void* centers, const void* incomp,
                         const int64_t* block_inc_off, uint64_t start, uint64_t len,
                         void* out, uint32_t* flags) {
  if (!info || !flags) return ORC_EINVAL;
  if (start > info->n || len > info->n - start) return ORC_ERANGE;
  *flags = 0;
  if (len == 0) return ORC_OK;
  uint32_t esc = (1u << info->B) - 1u;
  uint64_t epb = info->elems_per_block;
  uint64_t blk = start / epb;
  /* escapes before the block come from the offset table, the rest by counting */
  uint64_t rank = (uint64_t)block_inc_off[blk];
  for (uint64_t j = blk * epb; j < start; j++)
    if (get_index(packed, j, info->B) == esc) rank++;
  for (uint64_t t = 0; t < len; t++)
    decode_one(info, prev, packed, centers, incomp, start + t, &rank, out, t, flags);
  return ORC_OK;
}

/* ------------------------------------------------ lossless index stage */

/* The paper follows the index table with a lossless stage (ZLIB per block,
 * Sec. IV-C and V-A).  This is a tree-free prefix code in its place, so that
 * every step stays a data-parallel pass:
 *   - the 2^B codes are ranked by how often they occur in the table (more
 *     often first, equal counts by the smaller code);
 *   - the rank v of each code is written as an exponential-Golomb codeword of
 *     order k: with x = v + 2^k and q = floor(log2 x) - k, q zero bits, a one
 *     bit, then the low q + k bits of x, least significant first; its length
 *     is 2 floor(log2 x) - k + 1;
 *   - k in [0, B] is the order with the fewest bits in total, the smaller k
 *     on equal totals;
 *   - the table is cut into sub-blocks of ORC_SUB codes; each sub-block's bits
 *     start at a 32-bit word (the previous one padded with zeros) and
 *     sub_off[s] is its first bit, so any sub-block decodes on its own;
 *   - bits are numbered least significant first within little-endian 32-bit
 *     words, as in the index table. */

static uint32_t floor_log2_u64(uint64_t x) {
  uint32_t r = 0;
  while (x >> (r + 1)) r++;
  return r;
}

static uint32_t eg_len(uint64_t v, uint32_t k) {
  return 2 * floor_log2_u64(v + ((uint64_t)1 << k)) - k + 1;
}

typedef struct {
  uint64_t count;
  uint32_t code;
} sym_count;

static int cmp_sym(const void* a, const void* b) {
  const sym_count* x = (const sym_count*)a;
  const sym_count* y = (const sym_count*)b;
  if (x->count != y->count) return (x->count < y->count) - (x->count > y->count);
  return (x->code > y->code) - (x->code < y->code);
}

static void put_bit(uint32_t* w, uint64_t pos, uint32_t bit) {
  if (bit) w[pos >> 5] |= 1u << (pos & 31);
}

static uint32_t get_bit(const uint32_t* w, uint64_t pos) {
  return (w[pos >> 5] >> (pos & 31)) & 1u;
}

uint64_t orc_lossless_subblocks(uint64_t n) { return (n + ORC_SUB - 1) / ORC_SUB; }

/* The 16-bit value at bits [pos, pos + 16) and its store. */
static void put_u16(uint32_t* w, uint64_t pos, uint32_t v) {
  for (uint32_t b = 0; b < 16; b++) put_bit(w, pos + b, (v >> b) & 1u);
}
static uint32_t get_u16(const uint32_t* w, uint64_t pos) {
  uint32_t v = 0;
  for (uint32_t b = 0; b < 16; b++) v |= get_bit(w, pos + b) << b;
  return v;
}

int orc_lossless_encode(const uint32_t* packed, uint64_t n, uint32_t B, uint16_t* code_of_rank,
                        uint32_t* k_out, uint64_t* bits_k, uint64_t* sub_off, uint32_t* stream,
                        uint64_t cap_words, uint64_t* words_out) {
  if (B < 1 || B > 16 || !code_of_rank || !k_out || !sub_off || !words_out) return ORC_EINVAL;
  if (n && (!packed || !stream)) return ORC_EINVAL;
  const uint32_t K = 1u << B;
  sym_count* sc = (sym_count*)calloc(K, sizeof(sym_count));
  uint32_t* rank = (uint32_t*)malloc(K * sizeof(uint32_t));
  if (!sc || !rank) {
    free(sc); free(rank);
    return ORC_ENOMEM;
  }
  for (uint32_t c = 0; c < K; c++) sc[c].code = c;
  for (uint64_t j = 0; j < n; j++) sc[get_index(packed, j, B)].count++;
  /* ranks: more frequent first, ties by the smaller code */
  qsort(sc, K, sizeof(sym_count), cmp_sym);
  for (uint32_t r = 0; r < K; r++) {
    code_of_rank[r] = (uint16_t)sc[r].code;
    rank[sc[r].code] = r;
  }
  /* the order with the fewest bits */
  uint32_t k = 0;
  uint64_t best = 0;
  for (uint32_t kk = 0; kk <= B; kk++) {
    uint64_t bits = 0;
    for (uint32_t r = 0; r < K; r++) bits += sc[r].count * eg_len(r, kk);
    if (bits_k) bits_k[kk] = bits;
    if (kk == 0 || bits < best) {
      best = bits;
      k = kk;
    }
  }
  /* sub-block offsets: the group table, then the codewords, padded to a
     whole word */
  const uint64_t nsub = orc_lossless_subblocks(n);
  sub_off[0] = 0;
  for (uint64_t s = 0; s < nsub; s++) {
    uint64_t bits = ORC_SUB_HEAD_BITS;
    const uint64_t e = (s + 1) * ORC_SUB < n ? (s + 1) * ORC_SUB : n;
    for (uint64_t j = s * ORC_SUB; j < e; j++) bits += eg_len(rank[get_index(packed, j, B)], k);
    sub_off[s + 1] = sub_off[s] + (bits + 31) / 32 * 32;
  }
  const uint64_t words = sub_off[nsub] / 32;
  *words_out = words;
  *k_out = k;
  if (words > cap_words) {
    free(sc); free(rank);
    return ORC_EINVAL;
  }
  if (words) memset(stream, 0, words * 4);
  for (uint64_t s = 0; s < nsub; s++) {
    uint64_t pos = sub_off[s] + ORC_SUB_HEAD_BITS;
    for (uint32_t g = 0; g < ORC_GROUPS; g++) {
      /* group g: codes [s ORC_SUB + g ORC_GROUP, + ORC_GROUP) of the table,
         or none past n; its first bit relative to the sub-block's */
      put_u16(stream, sub_off[s] + 16 * g, (uint32_t)(pos - sub_off[s]));
      uint64_t j0 = s * ORC_SUB + (uint64_t)g * ORC_GROUP;
      uint64_t j1 = j0 + ORC_GROUP;
      j0 = j0 < n ? j0 : n;
      j1 = j1 < n ? j1 : n;
      for (uint64_t j = j0; j < j1; j++) {
        const uint64_t x = (uint64_t)rank[get_index(packed, j, B)] + ((uint64_t)1 << k);
        const uint32_t nb = floor_log2_u64(x); /* x has nb + 1 bits */
        const uint32_t q = nb - k;
        pos += q;                              /* q zeros */
        put_bit(stream, pos++, 1u);            /* the leading one */
        for (uint32_t b = 0; b < nb; b++) put_bit(stream, pos++, (uint32_t)(x >> b) & 1u);
      }
    }
  }
  free(sc); free(rank);
  return ORC_OK;
}

int orc_lossless_decode(const uint16_t* code_of_rank, uint32_t k, const uint64_t* sub_off,
                        const uint32_t* stream, uint64_t n, uint32_t B, uint32_t* packed) {
  if (B < 1 || B > 16 || k > B || !code_of_rank || !sub_off) return ORC_EINVAL;
  if (n && (!stream || !packed)) return ORC_EINVAL;
  const uint64_t nsub = orc_lossless_subblocks(n);
  memset(packed, 0, (n * B + 31) / 32 * 4);
  for (uint64_t s = 0; s < nsub; s++) {
    const uint64_t base = sub_off[s];
    const uint64_t end = sub_off[s + 1];
    if (end < base + ORC_SUB_HEAD_BITS) return ORC_EINVAL;
    /* every group decodes from its own offset and must end where the next
       one starts */
    for (uint32_t g = 0; g < ORC_GROUPS; g++) {
      uint64_t pos = base + get_u16(stream, base + 16 * g);
      const uint64_t gend = g + 1 < ORC_GROUPS ? base + get_u16(stream, base + 16 * (g + 1)) : end;
      if (pos < base + ORC_SUB_HEAD_BITS || gend > end || pos > gend) return ORC_EINVAL;
      uint64_t j0 = s * ORC_SUB + (uint64_t)g * ORC_GROUP;
      uint64_t j1 = j0 + ORC_GROUP;
      j0 = j0 < n ? j0 : n;
      j1 = j1 < n ? j1 : n;
      for (uint64_t j = j0; j < j1; j++) {
        uint32_t q = 0;
        while (pos < gend && !get_bit(stream, pos)) {
          q++;
          pos++;
        }
        if (pos >= gend || q + k > 16) return ORC_EINVAL;
        pos++; /* the leading one */
        const uint32_t nb = q + k;
        if (pos + nb > gend) return ORC_EINVAL;
        uint64_t x = (uint64_t)1 << nb;
        for (uint32_t b = 0; b < nb; b++) x |= (uint64_t)get_bit(stream, pos++) << b;
        const uint64_t v = x - ((uint64_t)1 << k);
        if (v >= ((uint64_t)1 << B)) return ORC_EINVAL;
        put_index(packed, j, B, code_of_rank[v]);
      }
      if (g + 1 < ORC_GROUPS && pos != gend) return ORC_EINVAL;
    }
  }
  return ORC_OK;
}
