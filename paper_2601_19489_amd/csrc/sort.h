// Device-wide scan and stable LSD radix sort primitives (internal).
#pragma once

#include "common.h"

namespace gs {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;  // 4096

constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;                         // per thread
constexpr int kSortTile = kSortThreads * kSortItems;   // 4096 keys per block
constexpr int kRadixBits = 8;
constexpr int kRadixBins = 1 << kRadixBits;

// Temporary words scan_u32 needs for n elements.
int64_t scan_tmp_words(int64_t n);

// Exclusive prefix sum of in[0, n) into out (may alias in). If total is not
// null, *total (device) receives the sum.
gs_status scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total, uint32_t* tmp,
                   hipStream_t st);

// Number of sort blocks for up to n keys.
inline int64_t sort_blocks(int64_t n) { return (n + kSortTile - 1) / kSortTile; }

// Words of temporary storage one radix pass needs for up to n keys.
int64_t radix_tmp_words(int64_t n);

// One stable counting pass on digit (key >> shift) & 255 over the first
// count keys, where count = min(*n_dev, n_max) if n_dev is not null, else
// n_max; if *n_dev > n_max the pass sorts nothing. keys_out may be null
// (keys are then not written).
gs_status radix_pass(const uint32_t* keys_in, const uint32_t* vals_in, uint32_t* keys_out,
                     uint32_t* vals_out, int64_t n_max, const uint32_t* n_dev, int shift,
                     uint32_t* tmp, hipStream_t st);

}  // namespace gs
