/*
 * numarck_oracle.h -- plain CPU reference of the NUMARCK compression path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library includes, links
 * or calls this code; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark use it.  It shares no header, helper or table with the
 * HIP implementation.
 *
 * Every routine works in IEEE-754 binary64 with round-to-nearest-even,
 * evaluates expressions in the order written and must be compiled without
 * floating-point contraction (-ffp-contract=off) and without fast-math.
 *
 * Notation (Sec. III): n points, error bound E, B index bits,
 * k = 2^B - 1 selectable bins, escape code ESC = 2^B - 1, L = sizeof(T).
 */
#ifndef NUMARCK_ORACLE_H
#define NUMARCK_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_F32 = 0, ORC_F64 = 1 };

enum {
  ORC_OK = 0,
  ORC_EINVAL = 1,  /* null pointer or n too large */
  ORC_EDTYPE = 2,  /* dtype not f32/f64 */
  ORC_EBITS = 3,   /* B outside [1, 16] */
  ORC_EBOUND = 4,  /* E not in (0, 1] */
  ORC_ENOMEM = 5,  /* host allocation failed */
  ORC_ERANGE = 6   /* start + len > n */
};

/* Decompression flags (ORed). */
#define ORC_FLAG_BAD_INDEX 1u    /* an index in [k_used, ESC) was found */
#define ORC_FLAG_INC_OVERRUN 2u  /* more escape codes than stored values */

typedef struct {
  uint64_t n, n_valid, n_invalid, n_inc;
  uint64_t n_blocks, elems_per_block, block_bytes;
  int64_t M;            /* number of fine bins, 0 when no point is valid */
  uint64_t n_nonzero;   /* bins with a nonzero count */
  uint32_t B, k, k_used, dtype;
  uint32_t tau;         /* smallest selected count; 0 when every nonzero bin is selected */
  double E, lo, hi;
  uint64_t packed_words, packed_bytes, compressed_bytes;
} orc_info;

/* Step 1, eq. (1): change ratio and validity of every point. */
/* Threads of the per-element loops (1 by default); returns the count set
 * (always 1 when built without OpenMP).  Results do not depend on it. */
int orc_set_threads(int n);

int orc_ratio(const void* prev, const void* curr, uint64_t n, int dtype, double E,
              double* d, uint8_t* valid);

/* Step 2 (Sec. IV-A): range of the valid ratios. Returns the number of valid points. */
uint64_t orc_range(const double* d, const uint8_t* valid, uint64_t n, double* lo, double* hi);

/* Step 3 (Sec. IV-B-1): fine bin id of each valid point (bins of width 2E anchored at lo). */
void orc_bin_ids(const double* d, const uint8_t* valid, uint64_t n, double lo, double E,
                 int64_t* m);

/* Step 4 (Sec. IV-B-1): histogram as ascending (id, count) pairs over nonzero bins.
 * ids/counts need room for n entries.  Returns the number of nonzero bins. */
int64_t orc_histogram(const int64_t* m, const uint8_t* valid, uint64_t n, int64_t* ids,
                      uint32_t* counts);

/* Step 5 (Sec. IV-B-1/2): top-k selection.  sel receives min(k, nbins) ids in
 * ascending order.  Returns that number; *tau gets the smallest selected count
 * (0 when every nonzero bin was selected). */
int64_t orc_topk(const int64_t* ids, const uint32_t* counts, int64_t nbins, uint32_t k,
                 int64_t* sel, uint32_t* tau);

/* orc_compress with the fine bins anchored at -E instead of the smallest
 * valid ratio: bins of width 2E centred on multiples of 2E (bin m holds
 * floor((d + E) / 2E) == m), so no range is needed before the histogram.
 * info->lo = -E, info->hi = 0, info->M = 0. */
int orc_compress_za(const void* prev, const void* curr, uint64_t n, int dtype, double E,
                    uint32_t B, uint64_t block_bytes, uint32_t* packed, void* centers,
                    void* incomp, int64_t* block_inc_off, void* recon, uint16_t* index,
                    int64_t* sel_ids, orc_info* info);

/* Equal-width binning (Sec. III-B, IV-B-3): the compression of orc_compress
 * with the 2^B - 1 bins cut evenly from [lo, hi] instead of the top-k fine
 * bins; same outputs (sel_ids does not apply). */
int orc_compress_ew(const void* prev, const void* curr, uint64_t n, int dtype, double E,
                    uint32_t B, uint64_t block_bytes, uint32_t* packed, void* centers,
                    void* incomp, int64_t* block_inc_off, void* recon, uint16_t* index,
                    orc_info* info);

/* Selection of B (Sec. IV-B-2, eqs. 5-6): for every B in [b_lo, b_hi] the
 * estimated compressed size file_size(B) = 2^B L + n B / 8 + n alpha(B) L,
 * where alpha(B) n = n - (sum of the 2^B - 1 largest bin counts), in bits
 * (8 file_size, an exact integer): bits[B] for b_lo <= B <= b_hi (bits has 17
 * entries, index B).  *B_out gets the B of the smallest size, the smallest
 * such B on equal sizes.  1 <= b_lo <= b_hi <= 16. */
int orc_choose_B(const void* prev, const void* curr, uint64_t n, int dtype, double E,
                 uint32_t b_lo, uint32_t b_hi, uint64_t* bits, uint32_t* B_out);

/* The whole compression of one snapshot pair.
 *   packed         : ceil(n*B/32) u32 words
 *   centers        : 2^B values of the snapshot type
 *   incomp         : room for n values of the snapshot type
 *   block_inc_off  : ceil(n / elems_per_block) int64
 *   recon, index   : optional (NULL) n values / n u16 indices
 *   sel_ids        : optional (NULL) 2^B - 1 int64, selected bin ids in index order
 * block_bytes = 0 means 2^20. */
int orc_compress(const void* prev, const void* curr, uint64_t n, int dtype, double E,
                 uint32_t B, uint64_t block_bytes, uint32_t* packed, void* centers,
                 void* incomp, int64_t* block_inc_off, void* recon, uint16_t* index,
                 int64_t* sel_ids, orc_info* info);

/* Full decompression, eq. (4). *flags receives ORC_FLAG_* bits. */
int orc_decompress(const orc_info* info, const void* prev, const uint32_t* packed,
                   const void* centers, const void* incomp, void* out, uint32_t* flags);

/* Partial decompression of [start, start+len) through the per-block
 * incompressible offsets (Sec. IV-C).  prev is the whole previous snapshot. */
int orc_decompress_range(const orc_info* info, const void* prev, const uint32_t* packed,
                         const void* centers, const void* incomp,
                         const int64_t* block_inc_off, uint64_t start, uint64_t len,
                         void* out, uint32_t* flags);

/* Lossless stage of the index table (in place of the paper's per-block ZLIB,
 * Sec. IV-C): codes ranked by frequency (ties to the smaller code), ranks
 * written as exponential-Golomb codewords of the order k in [0, B] with the
 * fewest bits (ties to the smaller k), in sub-blocks of ORC_SUB codes that
 * each start on a 32-bit word.  A sub-block opens with ORC_GROUPS 16-bit
 * offsets (least significant bit first): the first bit of each group of
 * ORC_GROUP consecutive codes, relative to the sub-block's first bit (an
 * empty group past n: where the codewords end); the groups' codewords follow
 * without gaps, then zero padding to the next word.  Every group decodes on
 * its own.  code_of_rank: 2^B entries; bits_k (optional): B + 1 totals in
 * bits of the codewords alone; sub_off: n_sub + 1 bit offsets (the last is
 * the stream's length in bits); stream: cap_words words.  *words_out gets
 * the stream's words even when they exceed cap_words (then ORC_EINVAL). */
#define ORC_SUB 1024
#define ORC_GROUP 128
#define ORC_GROUPS (ORC_SUB / ORC_GROUP)
#define ORC_SUB_HEAD_BITS (16 * ORC_GROUPS)
uint64_t orc_lossless_subblocks(uint64_t n);
int orc_lossless_encode(const uint32_t* packed, uint64_t n, uint32_t B, uint16_t* code_of_rank,
                        uint32_t* k_out, uint64_t* bits_k, uint64_t* sub_off, uint32_t* stream,
                        uint64_t cap_words, uint64_t* words_out);
/* The inverse: the B-bit index table of n codes.  ORC_EINVAL on a corrupt
 * stream (a group offset out of order or outside its sub-block, a codeword
 * past its group, a group not ending where the next starts, or a rank of
 * 2^B or more). */
int orc_lossless_decode(const uint16_t* code_of_rank, uint32_t k, const uint64_t* sub_off,
                        const uint32_t* stream, uint64_t n, uint32_t B, uint32_t* packed);

#ifdef __cplusplus
}
#endif
#endif
