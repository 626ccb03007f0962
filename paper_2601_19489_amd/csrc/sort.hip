// Device-wide exclusive scan and one stable LSD radix sort pass for 32-bit
// keys with 32-bit values. The live count is read on the device; a bounded
// grid walks the live tiles (block b takes tiles b, b + grid, ...), so that
// a capacity far above the live count costs no empty workgroups.
//
// Scan: reduce each tile to its sum, then scan each tile from its offset,
// which its workgroup sums from the earlier tiles' sums itself (input read
// twice, two launches at any size).
// Radix pass: per-tile digit histogram laid out [digit][live tile], scanned,
// then each tile's keys are ranked stably and scattered.
#include "sort.h"

namespace gs {

__device__ __forceinline__ int64_t eff_count(int64_t n, const uint32_t* n_dev) {
  if (!n_dev) return n;
  const int64_t c = (int64_t)*n_dev;
  return c < n ? c : n;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_reduce(const uint32_t* __restrict__ in,
                                                             int64_t n, const uint32_t* n_dev,
                                                             uint32_t* __restrict__ partial,
                                                             int in_shift) {
  __shared__ uint32_t wsum[kScanThreads / kWave];
  const int64_t count = eff_count(n, n_dev);
  for (int64_t tile = blockIdx.x; tile * kScanTile < count; tile += gridDim.x) {
    const int64_t lo = tile * kScanTile;
    const int64_t hi = lo + kScanTile < count ? lo + kScanTile : count;
    // all of the thread's loads are issued before the first is used
    uint32_t v[kScanItems];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      const int64_t i = lo + threadIdx.x + (int64_t)k * kScanThreads;
      v[k] = in[i < hi ? i : lo];
    }
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
      if (lo + threadIdx.x + (int64_t)k * kScanThreads < hi) s += v[k] >> in_shift;
    uint32_t tot;
    block_exclusive_scan<kScanThreads>(s, wsum, tot);
    if (threadIdx.x == 0) partial[tile] = tot;
  }
}

// Each tile's offset is the sum of the earlier tiles' sums, added up by the
// tile's own workgroup; the workgroup of the last tile writes the total.
__global__ void __launch_bounds__(kScanThreads) k_scan_chunks(const uint32_t* in, uint32_t* out,
                                                             int64_t n, const uint32_t* n_dev,
                                                             const uint32_t* __restrict__ partial,
                                                             int in_shift, uint32_t* total) {
  __shared__ uint32_t wsum[kScanThreads / kWave];
  const int64_t count = eff_count(n, n_dev);
  const bool vec = (((uintptr_t)in | (uintptr_t)out) & 15) == 0;
  const int64_t n_tiles = (count + kScanTile - 1) / kScanTile;
  if (count == 0 && blockIdx.x == 0 && threadIdx.x == 0 && total) *total = 0;
  for (int64_t tile = blockIdx.x; tile * kScanTile < count; tile += gridDim.x) {
    const int64_t lo = tile * kScanTile;
    const int64_t hi = lo + kScanTile < count ? lo + kScanTile : count;
    uint32_t before = 0;
    for (int64_t t = threadIdx.x; t < tile; t += kScanThreads) before += partial[t];
    uint32_t offset;
    block_exclusive_scan<kScanThreads>(before, wsum, offset);
    const int64_t base = lo + (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems], s = 0;
    // whole runs of kScanItems go through 16-byte loads and stores when both
    // arrays are 16-byte aligned (base is a multiple of kScanItems)
    const bool whole = vec && base + kScanItems <= hi;
    if (whole) {
#pragma unroll
      for (int k = 0; k < kScanItems; k += 4) {
        const uint4 q = *reinterpret_cast<const uint4*>(in + base + k);
        v[k] = q.x; v[k + 1] = q.y; v[k + 2] = q.z; v[k + 3] = q.w;
      }
    } else {
#pragma unroll
      for (int k = 0; k < kScanItems; ++k) v[k] = base + k < hi ? in[base + k] : 0u;
    }
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      v[k] >>= in_shift;
      s += v[k];
    }
    uint32_t tot;
    uint32_t run = offset + block_exclusive_scan<kScanThreads>(s, wsum, tot);
    if (tile == n_tiles - 1 && threadIdx.x == 0 && total) *total = offset + tot;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      const uint32_t x = v[k];
      v[k] = run;
      run += x;
    }
    if (whole) {
#pragma unroll
      for (int k = 0; k < kScanItems; k += 4)
        *reinterpret_cast<uint4*>(out + base + k) = make_uint4(v[k], v[k + 1], v[k + 2], v[k + 3]);
    } else {
#pragma unroll
      for (int k = 0; k < kScanItems; ++k)
        if (base + k < hi) out[base + k] = v[k];
    }
  }
}

__global__ void k_set_u32(uint32_t* p, uint32_t v) { *p = v; }

int64_t scan_tmp_words(int64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

gs_status scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total, uint32_t* tmp,
                   hipStream_t st, const uint32_t* n_dev, int in_shift) {
  if (n <= 0) {
    if (total) {
      k_set_u32<<<1, 1, 0, st>>>(total, 0u);
      GS_CHECK_LAUNCH();
    }
    return GS_OK;
  }
  const int64_t tiles = (n + kScanTile - 1) / kScanTile;
  const unsigned g = (unsigned)(tiles < kGridMax ? tiles : kGridMax);
  k_scan_reduce<<<g, kScanThreads, 0, st>>>(in, n, n_dev, tmp, in_shift);
  GS_CHECK_LAUNCH();
  k_scan_chunks<<<g, kScanThreads, 0, st>>>(in, out, n, n_dev, tmp, in_shift, total);
  GS_CHECK_LAUNCH();
  return GS_OK;
}

// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t sort_count(int64_t n_max, const uint32_t* n_dev) {
  if (!n_dev) return n_max;
  const uint32_t c = *n_dev;
  return (int64_t)c <= n_max ? (int64_t)c : 0;
}

// Keys per thread of a radix tile: small tiles for short arrays (enough
// workgroups to fill the chip), long ones for long arrays (less fixed work
// per key).
static int sort_items(int64_t n_max) { return n_max <= ((int64_t)1 << 22) ? 8 : 16; }

template <int ITEMS>
__device__ __forceinline__ int64_t tiles_of(int64_t count) {
  constexpr int64_t T = (int64_t)kSortThreads * ITEMS;
  return (count + T - 1) / T;
}

// Digit histogram of each live tile, laid out [digit][live tile]; block 0
// writes the length of that layout for the scan.
template <int ITEMS>
__global__ void __launch_bounds__(kSortThreads) k_radix_hist(const uint32_t* __restrict__ keys,
                                                             int64_t n_max,
                                                             const uint32_t* __restrict__ n_dev,
                                                             int shift, uint32_t* __restrict__ hist,
                                                             uint32_t* __restrict__ scan_n) {
  constexpr int64_t T = (int64_t)kSortThreads * ITEMS;
  __shared__ uint32_t h[kRadixBins];
  const int64_t count = sort_count(n_max, n_dev);
  const int64_t nb = tiles_of<ITEMS>(count);
  if (blockIdx.x == 0 && threadIdx.x == 0) *scan_n = (uint32_t)(nb * kRadixBins);
  for (int64_t tile = blockIdx.x; tile < nb; tile += gridDim.x) {
    const int64_t lo = tile * T;
    const int64_t hi = lo + T < count ? lo + T : count;
    // all of the thread's loads are issued before the first is used
    uint32_t k[ITEMS];
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
      const int64_t i = lo + threadIdx.x + (int64_t)r * kSortThreads;
      k[r] = keys[i < hi ? i : lo];
    }
    h[threadIdx.x] = 0;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < ITEMS; ++r)
      if (lo + threadIdx.x + (int64_t)r * kSortThreads < hi)
        atomicAdd(&h[(k[r] >> shift) & (kRadixBins - 1)], 1u);
    __syncthreads();
    hist[(int64_t)threadIdx.x * nb + tile] = h[threadIdx.x];
  }
}

// Stable scatter, one tile of 256 * ITEMS keys at a time. Wave w owns the
// contiguous segment [w * 64 * ITEMS, (w + 1) * 64 * ITEMS) of the tile and
// walks it in ITEMS rounds of 64 in order; lanes holding the same digit in a
// round find each other with one ballot per significant digit bit (`bits`,
// at most 8: the digit's higher bits are zero for every key) and the lowest
// of them advances the wave's count for that digit. The tile is first
// reordered in LDS (digit, then the lower waves' keys, then rank): a key's
// slot is its digit's start within the tile + the counts of the lower waves
// + its rank. Consecutive threads then write consecutive slots: each digit's
// keys of the tile go to consecutive positions from the digit's base for the
// tile, so the stores of a wavefront cover few cache lines.
template <int ITEMS>
__global__ void __launch_bounds__(kSortThreads) k_radix_scatter(
    const uint32_t* __restrict__ keys_in, const uint32_t* __restrict__ vals_in,
    uint32_t* __restrict__ keys_out, uint32_t* __restrict__ vals_out, int64_t n_max,
    const uint32_t* __restrict__ n_dev, int shift, const uint32_t* __restrict__ hist,
    const uint32_t* __restrict__ vals2_in, uint32_t* __restrict__ vals2_out, int bits,
    int vals2_stride) {
  constexpr int NW = kSortThreads / kWave;
  constexpr int T = kSortThreads * ITEMS;
  __shared__ uint32_t cnt[NW][kRadixBins];
  __shared__ uint32_t gbase[kRadixBins], tstart[kRadixBins];
  __shared__ uint32_t wsum[NW];
  __shared__ uint32_t skey[T], sval[T], sval2[T];
  const int64_t count = sort_count(n_max, n_dev);
  const int64_t nb = tiles_of<ITEMS>(count);
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
  for (int64_t tile = blockIdx.x; tile < nb; tile += gridDim.x) {
    for (int j = threadIdx.x; j < NW * kRadixBins; j += kSortThreads) (&cnt[0][0])[j] = 0;
    __syncthreads();
    uint32_t key[ITEMS], val[ITEMS], val2[ITEMS], rank[ITEMS];
    const int64_t t0 = tile * (int64_t)T;
    const int n_in = (int)(count - t0 < T ? count - t0 : T);  // keys of this tile
    const int seg = w * (kWave * ITEMS);
    // every load of the tile is issued before the ranking uses the first
    // (out-of-range slots read the tile's first key and are masked below);
    // this thread's digit base for the tile is fetched alongside
    const uint32_t gb = hist[(int64_t)threadIdx.x * nb + tile];
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
      const int li = seg + r * kWave + lane;
      const int64_t idx = t0 + (li < n_in ? li : 0);
      key[r] = keys_in[idx];
      val[r] = vals_in ? vals_in[idx] : (uint32_t)idx;  // null: the index
      val2[r] = vals2_in ? vals2_in[idx * vals2_stride] : 0u;
    }
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
      const int li = seg + r * kWave + lane;
      const bool valid = li < n_in;
      const uint32_t d = (key[r] >> shift) & (kRadixBins - 1);
      uint64_t peers = __ballot(valid);
#pragma unroll
      for (int bit = 0; bit < kRadixBits; ++bit) {
        if (bit >= bits) break;  // uniform
        const bool set = (d >> bit) & 1u;
        const uint64_t bal = __ballot(set);
        peers &= set ? bal : ~bal;
      }
      rank[r] = 0;
      if (valid) {
        const uint32_t old = cnt[w][d];
        const uint64_t below = peers & lt;
        rank[r] = old + (uint32_t)__popcll(below);
        if (below == 0) cnt[w][d] = old + (uint32_t)__popcll(peers);
      }
    }
    __syncthreads();
    {
      const int d = threadIdx.x;  // one digit per thread (256 threads)
      uint32_t run = 0;
#pragma unroll
      for (int j = 0; j < NW; ++j) {
        const uint32_t c = cnt[j][d];
        cnt[j][d] = run;
        run += c;
      }
      uint32_t all;
      tstart[d] = block_exclusive_scan<kSortThreads>(run, wsum, all);
      gbase[d] = gb;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
      const int li = seg + r * kWave + lane;
      if (li < n_in) {
        const uint32_t d = (key[r] >> shift) & (kRadixBins - 1);
        const uint32_t slot = tstart[d] + cnt[w][d] + rank[r];
        skey[slot] = key[r];
        sval[slot] = val[r];
        if (vals2_out) sval2[slot] = val2[r];
      }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n_in; i += kSortThreads) {
      const uint32_t k = skey[i];
      const uint32_t d = (k >> shift) & (kRadixBins - 1);
      const uint32_t pos = gbase[d] + ((uint32_t)i - tstart[d]);
      if ((int64_t)pos < count) {  // always true for a correct ranking
        if (keys_out) keys_out[pos] = k;
        vals_out[pos] = sval[i];
        if (vals2_out) vals2_out[pos] = sval2[i];
      }
    }
    __syncthreads();  // cnt, gbase, tstart and the staging are rewritten for the next tile
  }
}

int64_t radix_tmp_words(int64_t n) {
  const int64_t T = (int64_t)kSortThreads * sort_items(n);
  const int64_t nb = (n + T - 1) / T;
  return nb * kRadixBins + scan_tmp_words(nb * kRadixBins) + 1;
}

template <int ITEMS>
static gs_status radix_pass_t(const uint32_t* keys_in, const uint32_t* vals_in,
                              uint32_t* keys_out, uint32_t* vals_out, int64_t n_max,
                              const uint32_t* n_dev, int shift, uint32_t* tmp, hipStream_t st,
                              const uint32_t* vals2_in, uint32_t* vals2_out, int bits,
                              int vals2_stride) {
  constexpr int64_t T = (int64_t)kSortThreads * ITEMS;
  const int64_t nb = (n_max + T - 1) / T;
  const unsigned g = (unsigned)(nb < kGridMax ? nb : kGridMax);
  uint32_t* hist = tmp;
  uint32_t* scan_n = tmp + nb * kRadixBins + scan_tmp_words(nb * kRadixBins);
  GS_TIMED("radix_hist", st,
           k_radix_hist<ITEMS><<<g, kSortThreads, 0, st>>>(keys_in, n_max, n_dev, shift, hist,
                                                           scan_n));
  GS_CHECK_LAUNCH();
  gs_status s = scan_u32(hist, hist, nb * kRadixBins, nullptr, tmp + nb * kRadixBins, st, scan_n);
  if (s != GS_OK) return s;
  GS_TIMED("radix_scatter", st,
           k_radix_scatter<ITEMS><<<g, kSortThreads, 0, st>>>(keys_in, vals_in, keys_out,
                                                              vals_out, n_max, n_dev, shift, hist,
                                                              vals2_in, vals2_out, bits,
                                                              vals2_stride));
  GS_CHECK_LAUNCH();
  return GS_OK;
}

gs_status radix_pass(const uint32_t* keys_in, const uint32_t* vals_in, uint32_t* keys_out,
                     uint32_t* vals_out, int64_t n_max, const uint32_t* n_dev, int shift,
                     uint32_t* tmp, hipStream_t st, const uint32_t* vals2_in,
                     uint32_t* vals2_out, int bits, int vals2_stride) {
  if (n_max <= 0) return GS_OK;
  if (bits < 1 || bits > kRadixBits || vals2_stride < 1) return GS_EINVAL;
  if (sort_items(n_max) == 8)
    return radix_pass_t<8>(keys_in, vals_in, keys_out, vals_out, n_max, n_dev, shift, tmp, st,
                           vals2_in, vals2_out, bits, vals2_stride);
  return radix_pass_t<16>(keys_in, vals_in, keys_out, vals_out, n_max, n_dev, shift, tmp, st,
                          vals2_in, vals2_out, bits, vals2_stride);
}

int64_t radix_tile_keys(int64_t n_max) { return (int64_t)kSortThreads * sort_items(n_max); }

}  // namespace gs
