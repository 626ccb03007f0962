// Device-wide exclusive scan (reduce-then-scan) and one stable LSD radix
// sort pass (per-block digit histogram, scan, stable scatter) for 32-bit
// keys with 32-bit values.
#include "sort.h"

namespace gs {

__device__ __forceinline__ int64_t eff_count(int64_t n, const uint32_t* n_dev) {
  if (!n_dev) return n;
  const int64_t c = (int64_t)*n_dev;
  return c < n ? c : n;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_block(const uint32_t* in, uint32_t* out,
                                                            int64_t n, uint32_t* block_sums,
                                                            const uint32_t* n_dev) {
  const int64_t nv = eff_count(n, n_dev);
  if ((int64_t)blockIdx.x * kScanTile >= nv && blockIdx.x > 0) {
    // past the live count: nothing to write but a zero block sum
    if (threadIdx.x == 0 && block_sums) block_sums[blockIdx.x] = 0u;
    return;
  }
  __shared__ uint32_t wsum[kScanThreads / kWave];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t idx = base + k;
    v[k] = idx < nv ? in[idx] : 0u;
    s += v[k];
  }
  const uint32_t incl = wave_incl_scan_u32(s);
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  if (lane == kWave - 1) wsum[w] = incl;
  __syncthreads();
  uint32_t woff = 0;
  for (int j = 0; j < w; ++j) woff += wsum[j];
  uint32_t run = woff + incl - s;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t idx = base + k;
    if (idx < n) out[idx] = run;
    run += v[k];
  }
  if (threadIdx.x == kScanThreads - 1 && block_sums) block_sums[blockIdx.x] = woff + incl;
}

__global__ void k_scan_add(uint32_t* out, int64_t n, const uint32_t* offs,
                           const uint32_t* n_dev) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  if (base >= eff_count(n, n_dev)) return;
  const uint32_t o = offs[blockIdx.x];
  for (int k = threadIdx.x; k < kScanTile; k += blockDim.x) {
    const int64_t idx = base + k;
    if (idx < n) out[idx] += o;
  }
}

__global__ void k_set_u32(uint32_t* p, uint32_t v) { *p = v; }

int64_t scan_tmp_words(int64_t n) {
  const int64_t nb = (n + kScanTile - 1) / kScanTile;
  if (nb <= 1) return 0;
  return nb + scan_tmp_words(nb);
}

gs_status scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total, uint32_t* tmp,
                   hipStream_t st, const uint32_t* n_dev) {
  if (n <= 0) {
    if (total) {
      k_set_u32<<<1, 1, 0, st>>>(total, 0u);
      GS_CHECK_LAUNCH();
    }
    return GS_OK;
  }
  const int64_t nb = (n + kScanTile - 1) / kScanTile;
  if (nb == 1) {
    k_scan_block<<<1, kScanThreads, 0, st>>>(in, out, n, total, n_dev);
    GS_CHECK_LAUNCH();
    return GS_OK;
  }
  k_scan_block<<<(unsigned)nb, kScanThreads, 0, st>>>(in, out, n, tmp, n_dev);
  GS_CHECK_LAUNCH();
  gs_status s = scan_u32(tmp, tmp, nb, total, tmp + nb, st);
  if (s != GS_OK) return s;
  k_scan_add<<<(unsigned)nb, kScanThreads, 0, st>>>(out, n, tmp, n_dev);
  GS_CHECK_LAUNCH();
  return GS_OK;
}

// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t sort_count(int64_t n_max, const uint32_t* n_dev) {
  if (!n_dev) return n_max;
  const uint32_t c = *n_dev;
  return (int64_t)c <= n_max ? (int64_t)c : 0;
}

// Blocks past the live count exit; the histogram is laid out
// [digit][live block] so the scan covers only live entries (its length is
// written to *scan_n by block 0).
__global__ void __launch_bounds__(kSortThreads) k_radix_hist(const uint32_t* __restrict__ keys,
                                                             int64_t n_max,
                                                             const uint32_t* __restrict__ n_dev,
                                                             int shift, uint32_t* __restrict__ hist,
                                                             uint32_t* __restrict__ scan_n) {
  __shared__ uint32_t h[kRadixBins];
  const int64_t count = sort_count(n_max, n_dev);
  const int64_t nb = sort_blocks(count);
  if (blockIdx.x == 0 && threadIdx.x == 0) *scan_n = (uint32_t)(nb * kRadixBins);
  if ((int64_t)blockIdx.x >= nb) return;
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  if (base < count) {
    for (int k = threadIdx.x; k < kSortTile; k += kSortThreads) {
      const int64_t idx = base + k;
      if (idx < count) atomicAdd(&h[(keys[idx] >> shift) & (kRadixBins - 1)], 1u);
    }
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter: wave w of the block owns the contiguous segment
// [w*1024, (w+1)*1024) of the block's 4096 keys and walks it in 16 rounds of
// 64 in order. Lanes holding the same digit in a round find each other with
// 8 ballots (one per digit bit); the lowest of them advances the wave's
// running count for that digit. Ranks are then offset by the counts of the
// lower waves and by the digit's global offset for this block.
__global__ void __launch_bounds__(kSortThreads) k_radix_scatter(
    const uint32_t* __restrict__ keys_in, const uint32_t* __restrict__ vals_in,
    uint32_t* __restrict__ keys_out, uint32_t* __restrict__ vals_out, int64_t n_max,
    const uint32_t* __restrict__ n_dev, int shift, const uint32_t* __restrict__ hist,
    const uint32_t* __restrict__ vals2_in, uint32_t* __restrict__ vals2_out) {
  __shared__ uint32_t cnt[kSortThreads / kWave][kRadixBins];
  __shared__ uint32_t gbase[kRadixBins];
  const int64_t count = sort_count(n_max, n_dev);
  const int64_t nb = sort_blocks(count);
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  if (base >= count) return;  // uniform over the block
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  for (int j = threadIdx.x; j < (kSortThreads / kWave) * kRadixBins; j += kSortThreads)
    (&cnt[0][0])[j] = 0;
  __syncthreads();
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
  uint32_t key[kSortItems], val[kSortItems], val2[kSortItems], rank[kSortItems];
  const int64_t seg = base + (int64_t)w * (kWave * kSortItems);
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const int64_t idx = seg + (int64_t)r * kWave + lane;
    const bool valid = idx < count;
    key[r] = valid ? keys_in[idx] : 0u;
    val[r] = valid ? vals_in[idx] : 0u;
    val2[r] = (valid && vals2_in) ? vals2_in[idx] : 0u;
    const uint32_t d = (key[r] >> shift) & (kRadixBins - 1);
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < kRadixBits; ++bit) {
      const bool set = (d >> bit) & 1u;
      const uint64_t bal = __ballot(set);
      peers &= set ? bal : ~bal;
    }
    uint32_t old = 0;
    if (valid) {
      old = cnt[w][d];
      const uint64_t below = peers & lt;
      rank[r] = old + (uint32_t)__popcll(below);
      if (below == 0) cnt[w][d] = old + (uint32_t)__popcll(peers);
    } else {
      rank[r] = 0;
    }
  }
  __syncthreads();
  {
    const int d = threadIdx.x;  // one digit per thread (256 threads)
    uint32_t run = 0;
#pragma unroll
    for (int j = 0; j < kSortThreads / kWave; ++j) {
      const uint32_t c = cnt[j][d];
      cnt[j][d] = run;
      run += c;
    }
    gbase[d] = hist[(int64_t)d * nb + blockIdx.x];
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const int64_t idx = seg + (int64_t)r * kWave + lane;
    if (idx < count) {
      const uint32_t d = (key[r] >> shift) & (kRadixBins - 1);
      const uint32_t pos = gbase[d] + cnt[w][d] + rank[r];
      if ((int64_t)pos < count) {  // always true for a correct ranking
        if (keys_out) keys_out[pos] = key[r];
        vals_out[pos] = val[r];
        if (vals2_out) vals2_out[pos] = val2[r];
      }
    }
  }
}

int64_t radix_tmp_words(int64_t n) {
  const int64_t nb = sort_blocks(n);
  return nb * kRadixBins + scan_tmp_words(nb * kRadixBins) + 1;
}

gs_status radix_pass(const uint32_t* keys_in, const uint32_t* vals_in, uint32_t* keys_out,
                     uint32_t* vals_out, int64_t n_max, const uint32_t* n_dev, int shift,
                     uint32_t* tmp, hipStream_t st, const uint32_t* vals2_in,
                     uint32_t* vals2_out) {
  if (n_max <= 0) return GS_OK;
  const int64_t nb = sort_blocks(n_max);
  uint32_t* hist = tmp;
  uint32_t* scan_n = tmp + nb * kRadixBins + scan_tmp_words(nb * kRadixBins);
  GS_TIMED("radix_hist", st, k_radix_hist<<<(unsigned)nb, kSortThreads, 0, st>>>(keys_in, n_max, n_dev, shift, hist, scan_n));
  GS_CHECK_LAUNCH();
  gs_status s = scan_u32(hist, hist, nb * kRadixBins, nullptr, tmp + nb * kRadixBins, st, scan_n);
  if (s != GS_OK) return s;
  GS_TIMED("radix_scatter", st, k_radix_scatter<<<(unsigned)nb, kSortThreads, 0, st>>>(keys_in, vals_in, keys_out, vals_out,
                                                         n_max, n_dev, shift, hist,
                                                         vals2_in, vals2_out));
  GS_CHECK_LAUNCH();
  return GS_OK;
}

}  // namespace gs
