// Device-wide scan and stable LSD radix sort primitives (internal).
#pragma once

#include "common.h"

namespace gs {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;  // 4096

constexpr int kGridMax = 2048;                         // workgroups of a scan or sort launch

constexpr int kSortThreads = 256;
constexpr int kRadixBits = 8;
constexpr int kRadixBins = 1 << kRadixBits;

// Temporary words scan_u32 needs for n elements.
int64_t scan_tmp_words(int64_t n);

// Exclusive prefix sum of in[0, c) into out (may alias in), c = n, or
// min(*n_dev, n) when n_dev is not null (read on the device); out is written
// for those c elements only. If total is not null, *total (device) receives
// the sum. Each element is read as in[i] >> in_shift.
gs_status scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total, uint32_t* tmp,
                   hipStream_t st, const uint32_t* n_dev = nullptr, int in_shift = 0);

// Words of temporary storage one radix pass needs for up to n keys.
int64_t radix_tmp_words(int64_t n);

// One stable counting pass on digit (key >> shift) & 255 over the first
// count keys, where count = *n_dev if n_dev is not null, else n_max; if
// *n_dev > n_max the pass sorts nothing. keys_out may be null (keys are then
// not written); vals_in may be null (the values are then the key indices); a
// second value array (vals2_in/out) is carried when given. bits (1..8): the
// digit bits that can be set in any key (a cheaper ranking below 8).
// vals2_in is read with a stride of vals2_stride words (1: contiguous).
gs_status radix_pass(const uint32_t* keys_in, const uint32_t* vals_in, uint32_t* keys_out,
                     uint32_t* vals_out, int64_t n_max, const uint32_t* n_dev, int shift,
                     uint32_t* tmp, hipStream_t st, const uint32_t* vals2_in = nullptr,
                     uint32_t* vals2_out = nullptr, int bits = 8, int vals2_stride = 1);

// Keys per tile of a radix pass over up to n_max keys. After a pass, tmp
// holds its scanned histogram laid out [digit][tile] over the
// ceil(count / tile) live tiles: word d * tiles is the first output position
// of digit d.
int64_t radix_tile_keys(int64_t n_max);

__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t v) {
  const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const uint32_t o = __shfl_up(v, d, kWave);
    if (lane >= d) v += o;
  }
  return v;
}

// Exclusive scan over one workgroup of NTH threads (all threads call it):
// returns the exclusive prefix of v; `total` receives the sum. wsum is LDS
// scratch of NTH / 64 words; the call ends with a barrier.
template <int NTH>
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* wsum,
                                                         uint32_t& total) {
  const uint32_t incl = wave_incl_scan_u32(v);
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  if (lane == kWave - 1) wsum[w] = incl;
  __syncthreads();
  uint32_t woff = 0, tot = 0;
#pragma unroll
  for (int j = 0; j < NTH / kWave; ++j) {
    if (j < w) woff += wsum[j];
    tot += wsum[j];
  }
  total = tot;
  __syncthreads();
  return woff + incl - v;
}

}  // namespace gs
