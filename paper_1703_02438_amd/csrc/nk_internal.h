// nk_internal.h -- internal definitions shared by the gfx950 kernels and the
// C-ABI layer of the NUMARCK library.  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/numarck.h"

namespace nk {

// ---------------------------------------------------------------- constants
// On-chip (LDS) window of fine bins used by the histogram and the encoder.
// Bins outside it are counted exactly through the tail list + hash table.
constexpr int WIN = 16384;
constexpr uint16_t NOSEL = 0xFFFF;       // window LUT entry: bin not selected
constexpr uint32_t HEMPTY = 0xFFFFFFFFu;  // empty hash slot
constexpr int MAX_SEL = 65535;            // k for B = 16

// Tile of the encoder / decoder (elements per tile, threads per block).
constexpr int ENC_TPB = 256;
constexpr int ENC_TILE = 4096;
constexpr int DEC_TPB = 256;
constexpr int DEC_TILE = 4096;

// Look-back status words: 2 flag bits over a 62-bit value.
constexpr uint64_t LB_AGG = 1ull << 62;
constexpr uint64_t LB_INC = 2ull << 62;
constexpr uint64_t LB_VAL = (1ull << 62) - 1;

// ------------------------------------------------ device control block
// Lives at the start of the compression workspace.  Fields above `lo` are
// reset by k_init at the start of every call.
struct Ctl {
  unsigned long long lo_key;      // order key of the smallest valid ratio (atomicMin)
  unsigned long long hi_key;      // order key of the largest valid ratio (atomicMax)
  unsigned long long n_invalid;   // points that are not valid
  unsigned long long tail_count;  // points outside the window (may exceed capacity)
  unsigned int tile_ticket;       // encoder tile tickets
  unsigned int flags;             // NUMARCK_FLAG_*
  unsigned int sel_tail_count;    // selected tail bins appended by k_select
  unsigned int pad0;
  // derived by k_derive
  double lo, hi;
  long long M;
  long long wbase;
  unsigned long long n_valid;
  unsigned int win_len;
  unsigned int empty;
  // hash table in use
  unsigned long long H;
  unsigned long long tail_used;   // min(tail_count, capacity)
  // selection
  unsigned long long n_nonzero;
  long long cut;                  // tie cut: selected ties have id <= cut
  unsigned int tau;               // k-th count (0: every nonzero bin selected)
  unsigned int k_used;
  unsigned int nsel_window;
  unsigned int nsel_tail;
  unsigned int nsel_tail_below;
  unsigned int pad1;
};

// Control block of a decompression call.
struct DCtl {
  unsigned long long base;  // escapes before `start`
  unsigned int ticket;
  unsigned int pad;
};

// Workspace layout of one compression (byte offsets from the workspace base).
struct Layout {
  size_t ctl, gwin, lut, sel_tail, sorted_tail, status, tail, hslot, hcnt, total;
  uint64_t tail_cap, hcap;
  uint64_t n_tiles;
};
Layout compress_layout(uint64_t n, uint64_t tail_cap);

// Everything a compression kernel needs (passed by value).
struct CParams {
  const void* prev;
  const void* curr;
  uint64_t n;
  double E, twoE, cap;
  uint32_t B;
  uint32_t k;        // 2^B - 1 (also the escape code)
  uint64_t epb;      // elements per index-table block
  uint64_t n_blocks;
  uint64_t n_tiles;
  uint64_t packed_words;
  Ctl* ctl;
  uint32_t* gwin;
  uint16_t* lut;
  int64_t* tail;
  uint64_t tail_cap;
  uint32_t* hslot;
  uint32_t* hcnt;
  uint64_t hcap;
  int64_t* sel_tail;
  int64_t* sorted_tail;
  unsigned long long* status;
  uint32_t* packed;
  void* centers;
  void* incomp;
  int64_t* block_inc_off;
  void* recon;
  int64_t* bin_ids;
  numarck_header* hdr;
  uint64_t block_bytes;
  int dtype;
};

struct DParams {
  const void* prev;
  const uint32_t* packed;
  const void* centers;
  const void* incomp;
  const int64_t* block_inc_off;
  void* out;
  uint32_t* flags;
  uint64_t n, start, len, n_inc, epb, packed_words;
  uint32_t B, k_used;
  int dtype;
  DCtl* dctl;
  unsigned long long* status;
  uint64_t n_tiles;
};

// Launch geometry of the streaming kernels for the current device.
struct Geometry {
  int cus;
};
Geometry geometry();

// Kernel kinds for the optional event timing.
enum KernelKind {
  KK_INIT = 0, KK_RANGE, KK_DERIVE, KK_HIST, KK_HCLEAR, KK_HINSERT, KK_SELECT,
  KK_TAILRANK, KK_ENCODE, KK_FINAL, KK_DINIT, KK_DPREFIX, KK_DECODE, KK_EXPORT, KK_COUNT
};
void timing_begin(KernelKind k, hipStream_t s);
void timing_end(KernelKind k, hipStream_t s);

// Launch wrappers (compress_kernels.hip / decompress_kernels.hip).  Each
// returns the hipError_t of the launch.
hipError_t launch_compress(const CParams& p, hipStream_t s);
hipError_t launch_decompress(const DParams& p, hipStream_t s);
hipError_t launch_histogram_export(Ctl* ctl, const uint32_t* gwin, const uint32_t* hslot,
                                   const uint32_t* hcnt, const int64_t* tail, int64_t* ids,
                                   uint32_t* counts, uint64_t capacity, uint64_t* count_dev,
                                   hipStream_t s);

}  // namespace nk
