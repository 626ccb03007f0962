// Binning and depth sort (Sec. 2.1): every Gaussian writes one pair per tile
// of its compact tile set; the pairs end up ordered by (tile id, depth bits,
// Gaussian index), tiles numbered column-major (id = tx * tiles_y + ty).
//
// The paper's column walk produces, per Gaussian, runs of consecutive tiles
// (one run per column of its SnugBox). Instead of materialising and sorting
// the P pairs, this works on the runs (about P / 15 of them):
//   1. stable sort of the Gaussians by depth (32-bit keys; ties keep index
//      order), carrying each Gaussian's column span (its first column
//      holding tiles and the number of columns to its last, from the
//      preprocess record): one run per column of the span;
//   2. per block of 256 Gaussians in depth order, its runs per column (a
//      difference array over the columns); one scan over (column, block)
//      gives every block's first position in every column;
//   3. each block walks its Gaussians' spans (the load-balanced column walk)
//      and writes each run (first row, length, Gaussian id) at its block's
//      position in the column plus the number of the block's runs of that
//      column before it, so each column lists its runs in depth order with
//      no sort by column;
//   4. each column's runs are cut into segments of kSegRuns runs;
//   5. per segment, its pairs per row (a difference array over the rows);
//   6. per column, one scan over (row, segment) gives every segment's first
//      position in every tile of the column, and the tile ranges;
//   7. each segment walks its runs in order, 64 at a time: for every row the
//      64 runs touch, the runs covering it are ranked by one ballot and write
//      their Gaussian ids to consecutive positions of that tile.
// Only the final 4-byte Gaussian id is written per pair.
#include <algorithm>

#include "binning.h"
#include "common.h"
#include "sort.h"

namespace gs {

namespace {

constexpr int kSegThreads = 256;              // 4 independent wavefronts per workgroup
constexpr int kSegWaves = kSegThreads / kWave;
constexpr int kScanThreads1 = 1024;           // the per-column scan
constexpr int kMaxRows = 256;                 // tiles_y <= 256
constexpr int kMaxCols = 2048;                // tiles_x <= 2048
constexpr int kEmitBlock = 256;               // Gaussians per block of steps 2-3
constexpr int kEmitWaves = kEmitBlock / kWave;
constexpr int64_t kAlign = 256;

inline int64_t al(int64_t b) { return (b + kAlign - 1) / kAlign * kAlign; }
constexpr int kCountBlocks = 1024;  // workgroups of the pair-total partial sums

struct BinLayout {
  int64_t dkA, dkB, dvA, dvB, spA, spB, ptot;
  int64_t runs, colh;
  int64_t cstart, nseg, segfirst, misc, hist, segtot;
  int64_t rtmp, stmp, total;
  int64_t ns_max, nblk;
};

BinLayout layout(int64_t n, int64_t cap, int tiles_x, int tiles_y) {
  BinLayout L;
  int64_t o = 0;
  const int64_t nw = al(4 * std::max<int64_t>(n, 1));
  const int64_t cw = al(4 * std::max<int64_t>(cap, 1));
  const int64_t tw = al(4 * ((int64_t)tiles_x + 2));
  // runs <= cap when they fit (else overflow), so at most cap / kSegRuns
  // full segments plus one partial segment per column
  L.ns_max = (cap + kSegRuns - 1) / kSegRuns + tiles_x;
  L.nblk = (n + kEmitBlock - 1) / kEmitBlock;
  const int64_t ncolh = (int64_t)tiles_x * L.nblk;
  L.dkA = o; o += nw;
  L.dkB = o; o += nw;
  L.dvA = o; o += nw;
  L.dvB = o; o += nw;
  L.spA = o; o += nw;
  L.spB = o; o += nw;
  L.ptot = o; o += al(8 * kCountBlocks);
  L.runs = o; o += 2 * cw;  // uint2 per run: Gaussian id, row word
  L.colh = o; o += al(4 * std::max<int64_t>(ncolh, 1));
  L.cstart = o; o += tw;
  L.nseg = o; o += tw;
  L.segfirst = o; o += tw;
  L.misc = o; o += al(64);
  L.hist = o; o += al(4 * (int64_t)tiles_y * L.ns_max);
  L.segtot = o; o += al(4 * L.ns_max);
  L.rtmp = o; o += al(4 * radix_tmp_words(std::max<int64_t>(n, 1)));
  L.stmp = o; o += al(4 * (scan_tmp_words(std::max<int64_t>(ncolh, 1)) + 1));
  L.total = o;
  return L;
}

// misc words
constexpr int kRunTotal = 0;   // number of runs C
constexpr int kSegTotal = 1;   // number of run segments
constexpr int kPLo = 4;        // exact pair total as uint64 (words 4, 5)

__device__ __forceinline__ uint64_t pair_total(const uint32_t* misc) {
  return *reinterpret_cast<const uint64_t*>(misc + kPLo);
}

// partial sums of the tile counts, one per workgroup (64-bit, so an overflow
// of the capacity is always seen); k_seg_layout adds them up
__global__ void __launch_bounds__(256) k_count_partials(const uint32_t* __restrict__ counts,
                                                        int64_t n,
                                                        unsigned long long* __restrict__ part) {
  __shared__ unsigned long long wp[256 / kWave];
  unsigned long long acc = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  // four loads in flight per thread
  for (; i + 3 * stride < n; i += 4 * stride) {
    const uint32_t c0 = counts[i], c1 = counts[i + stride], c2 = counts[i + 2 * stride],
                   c3 = counts[i + 3 * stride];
    acc += (unsigned long long)c0 + c1 + c2 + c3;
  }
  for (; i < n; i += stride) acc += counts[i];
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) acc += __shfl_xor(acc, d, kWave);
  if ((threadIdx.x & (kWave - 1)) == 0) wp[threadIdx.x / kWave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
#pragma unroll
    for (int w = 0; w < 256 / kWave; ++w) t += wp[w];
    part[blockIdx.x] = t;
  }
}

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) v = min(v, (uint32_t)__shfl_xor(v, d, kWave));
  return v;
}
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) v = max(v, (uint32_t)__shfl_xor(v, d, kWave));
  return v;
}

// A Gaussian's column span from its record word: first column f and the
// number of columns len (0: no tile), clamped to the grid.
__device__ __forceinline__ void span_of(uint32_t w, int tiles_x, uint32_t& f, uint32_t& len) {
  f = w & 0xFFFFu;
  len = w >> 16;
  if (f >= (uint32_t)tiles_x) len = 0;
  else if (f + len > (uint32_t)tiles_x) len = (uint32_t)tiles_x - f;
}

// step 2: runs per column of each block of kEmitBlock Gaussians in depth
// order, colh[tx * nblk + blk]: a difference array over the columns (+1 at a
// span's first column, -1 past its last), summed along the columns.
__global__ void __launch_bounds__(kEmitBlock) k_col_hist(const uint32_t* __restrict__ spans,
                                                         int64_t n, int tiles_x,
                                                         uint32_t* __restrict__ colh) {
  extern __shared__ uint32_t dcol[];  // tiles_x + 1
  __shared__ uint32_t wsum[kEmitWaves];
  const int64_t nblk = gridDim.x, blk = blockIdx.x;
  for (int c = threadIdx.x; c <= tiles_x; c += kEmitBlock) dcol[c] = 0;
  __syncthreads();
  const int64_t r = blk * kEmitBlock + threadIdx.x;
  if (r < n) {
    uint32_t f, len;
    span_of(spans[r], tiles_x, f, len);
    if (len) {
      atomicAdd(&dcol[f], 1u);
      atomicAdd(&dcol[f + len], 0xFFFFFFFFu);  // -1
    }
  }
  __syncthreads();
  // thread t sums columns [t chunk, (t + 1) chunk); a block scan gives each
  // chunk's running start
  const int chunk = (tiles_x + kEmitBlock - 1) / kEmitBlock;
  const int c0 = threadIdx.x * chunk;
  uint32_t sum = 0;
  for (int k = 0; k < chunk; ++k)
    if (c0 + k < tiles_x) sum += dcol[c0 + k];
  uint32_t tot;
  uint32_t run = block_exclusive_scan<kEmitBlock>(sum, wsum, tot);
  for (int k = 0; k < chunk; ++k) {
    const int c = c0 + k;
    if (c < tiles_x) {
      run += dcol[c];
      colh[(int64_t)c * nblk + blk] = run;
    }
  }
}

__device__ __forceinline__ bool load_snug(const float* splats, uint32_t g, Snug& s) {
  const float4* rec = reinterpret_cast<const float4*>(splats + (int64_t)g * GS_SPLAT_FLOATS);
  const float4 r0 = rec[0], r1 = rec[1];
  return snug_setup(r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, s);
}

// Rows [ty0, ty0 + len) of column tx as a run word ty0 | len << 16 (0 when
// the column holds none of the Gaussian's tiles).
__device__ __forceinline__ uint32_t run_word(bool has, const Snug& s, int tx, const CamDev& cam) {
  int ty0 = 1, ty1 = 0;
  if (has) snug_rows(s, tx, cam.tile, cam.tiles_y, ty0, ty1);
  return ty1 >= ty0 ? (uint32_t)ty0 | ((uint32_t)(ty1 - ty0 + 1) << 16) : 0u;
}

// step 3: one block of kEmitBlock Gaussians in depth order. Each wavefront
// keeps, per column, the position of its next run there: the block's first
// position in the column (colh, scanned) plus the runs of the column in the
// block's earlier wavefronts. The wavefront walks its Gaussians' spans as
// one flattened list (owner-major, columns ascending), 64 entries a round:
// entries of equal column find each other with one ballot per bit of the
// column number and take consecutive positions in lane (= owner = depth)
// order, so every column receives its runs in depth order.
// SEQ: each lane walks its own span instead, the wavefront stepping through
// the columns together (the unbalanced walk the ablation compares with).
template <bool SEQ>
__global__ void __launch_bounds__(kEmitBlock) k_runs_emit(
    const uint32_t* __restrict__ order, const uint32_t* __restrict__ spans,
    const float* __restrict__ splats, int64_t n, CamDev cam, const uint32_t* __restrict__ colh,
    int64_t cap, uint2* __restrict__ runs) {
  __shared__ SnugLds walk[kEmitBlock];
  __shared__ uint32_t gid[kEmitBlock];
  extern __shared__ uint32_t cw[];  // [kEmitWaves][tiles_x]
  const int tiles_x = cam.tiles_x;
  const int64_t nblk = gridDim.x, blk = blockIdx.x;
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  const int64_t r = blk * kEmitBlock + threadIdx.x;
  uint32_t g = 0, f = 0, len = 0;
  if (r < n) {
    g = order[r];
    span_of(spans[r], tiles_x, f, len);
  }
  Snug s;
  const bool has = len > 0 && (int64_t)g < n && load_snug(splats, g, s);
  // each wavefront's runs per column, by the wavefront alone: a difference
  // array over the columns, summed along them (lane l sums a contiguous
  // chunk; a wavefront scan gives the chunk's start). A wavefront's LDS
  // operations complete in order, so no barrier is needed until the counts
  // of the other wavefronts are read.
  uint32_t* const next = cw + w * tiles_x;
  for (int c = lane; c < tiles_x; c += kWave) next[c] = 0;
  if (len) {
    atomicAdd(&next[f], 1u);
    if (f + len < (uint32_t)tiles_x) atomicAdd(&next[f + len], 0xFFFFFFFFu);  // -1
  }
  {
    const int chunk = (tiles_x + kWave - 1) / kWave;
    const int c0 = lane * chunk, c1 = min(c0 + chunk, tiles_x);
    uint32_t sum = 0;
    for (int c = c0; c < c1; ++c) sum += next[c];
    uint32_t run = wave_incl_scan_u32(sum) - sum;
    for (int c = c0; c < c1; ++c) {
      run += next[c];
      next[c] = run;
    }
  }
  __syncthreads();
  // per column: the block's first position (colh, scanned), then each
  // wavefront's start after the earlier wavefronts' runs
  for (int c = threadIdx.x; c < tiles_x; c += kEmitBlock) {
    uint32_t pos = colh[(int64_t)c * nblk + blk];
#pragma unroll
    for (int v = 0; v < kEmitWaves; ++v) {
      const uint32_t k = cw[v * tiles_x + c];
      cw[v * tiles_x + c] = pos;
      pos += k;
    }
  }
  __syncthreads();
  const uint32_t cap32 = (uint32_t)cap;  // cap <= 2^32 - 2
  if constexpr (SEQ) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane(wave_min_u32(len ? f : 0xFFFFFFFFu));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(wave_max_u32(len ? f + len : 0u));
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
    for (uint32_t tx = lo; tx < hi; ++tx) {
      const bool act = tx - f < len;
      const uint64_t bal = __ballot(act);
      const uint32_t base = next[tx];
      if (act) {
        const uint32_t pos = base + (uint32_t)__popcll(bal & lt);
        if (pos < cap32) {
          runs[pos] = make_uint2(g, run_word(has, s, (int)tx, cam));
        }
      }
      if (lane == 0) next[tx] = base + (uint32_t)__popcll(bal);
    }
  } else {
    // the flattened list of the wavefront's (owner, column) entries
    SnugLds* lds = walk + w * kWave;
    const uint32_t incl = wave_incl_scan_u32(len);
    const uint32_t total = __builtin_amdgcn_readfirstlane(__shfl(incl, kWave - 1, kWave));
    lds[lane].s = s;
    lds[lane].tx0 = has ? (int)f : -1 - (int)f;  // negative: no rows (record rejected)
    lds[lane].excl = incl - len;
    gid[threadIdx.x] = g;
    __syncthreads();
    int nbits = 1;
    while ((1 << nbits) < tiles_x) ++nbits;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
    for (uint32_t c0 = 0; c0 < total; c0 += kWave) {
      const uint32_t c = c0 + (uint32_t)lane;
      const bool valid = c < total;
      int o = 0;
      uint32_t tx = 0, word = 0;
      if (valid) {
        int a = 0, b = kWave - 1;  // owner: last lane whose first entry is <= c
        while (a < b) {
          const int mid = (a + b + 1) >> 1;
          if (lds[mid].excl <= c) a = mid; else b = mid - 1;
        }
        o = a;
        const int t0 = lds[o].tx0;
        const bool ohas = t0 >= 0;
        tx = (uint32_t)(ohas ? t0 : -1 - t0) + (c - lds[o].excl);
        word = run_word(ohas, lds[o].s, (int)tx, cam);
      }
      uint64_t peers = __ballot(valid);
      for (int bit = 0; bit < nbits; ++bit) {
        const bool set = (tx >> bit) & 1u;
        const uint64_t bal = __ballot(set);
        peers &= set ? bal : ~bal;
      }
      if (valid) {
        const uint64_t below = peers & lt;
        const uint32_t old = next[tx];
        const uint32_t pos = old + (uint32_t)__popcll(below);
        if (below == 0) next[tx] = old + (uint32_t)__popcll(peers);
        if (pos < cap32) {
          runs[pos] = make_uint2(gid[w * kWave + o], word);
        }
      }
    }
  }
}

__device__ __forceinline__ uint32_t upper_bound_u32(const uint32_t* a, uint32_t lo, uint32_t hi,
                                                    uint32_t x) {
  while (lo < hi) {
    const uint32_t mid = lo + ((hi - lo) >> 1);
    if (a[mid] <= x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// The segment `seg` of the layout: column tx and its run range [r0, r1).
__device__ __forceinline__ void seg_runs(uint32_t seg, const uint32_t* segfirst,
                                         const uint32_t* cstart, int tiles_x, int& tx,
                                         uint32_t& r0, uint32_t& r1) {
  tx = (int)upper_bound_u32(segfirst, 0, (uint32_t)tiles_x, seg) - 1;
  r0 = cstart[tx] + (seg - segfirst[tx]) * (uint32_t)kSegRuns;
  r1 = min(r0 + (uint32_t)kSegRuns, cstart[tx + 1]);
}

// step 4: the pair total P (sum of the partial sums), the first run of each
// column (word tx * nblk of the scanned per-(column, block) counts),
// segments per column and their first index, the pair count output. One
// workgroup. On a capacity overflow (pairs or runs above cap) no segment is
// made and the pair count reports the larger of the two.
__global__ void __launch_bounds__(256) k_seg_layout(
    const unsigned long long* __restrict__ part, int nparts, const uint32_t* __restrict__ colh,
    int64_t nblk, uint32_t* __restrict__ cstart, int64_t cap, int tiles_x,
    uint32_t* __restrict__ nseg, uint32_t* __restrict__ segfirst, uint32_t* __restrict__ misc,
    uint32_t* __restrict__ pair_count) {
  __shared__ uint32_t wsum[256 / kWave];
  __shared__ unsigned long long psum[256 / kWave];
  unsigned long long acc = 0;
  for (int i = threadIdx.x; i < nparts; i += 256) acc += part[i];
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) acc += __shfl_xor(acc, d, kWave);
  if ((threadIdx.x & (kWave - 1)) == 0) psum[threadIdx.x / kWave] = acc;
  const uint32_t C = misc[kRunTotal];
  for (int tx = threadIdx.x; tx < tiles_x; tx += 256)
    cstart[tx] = nblk > 0 ? colh[(int64_t)tx * nblk] : 0u;
  if (threadIdx.x == 0) cstart[tiles_x] = C;
  __syncthreads();
  uint64_t P = 0;
#pragma unroll
  for (int w = 0; w < 256 / kWave; ++w) P += psum[w];
  const bool over = P > (uint64_t)cap || (int64_t)C > cap;
  uint32_t run = 0;
  for (int base = 0; base < tiles_x; base += 256) {
    const int tx = base + threadIdx.x;
    uint32_t ns = 0;
    if (tx < tiles_x && !over) ns = (cstart[tx + 1] - cstart[tx] + kSegRuns - 1) / kSegRuns;
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan<256>(ns, wsum, tot);
    if (tx < tiles_x) {
      nseg[tx] = ns;
      segfirst[tx] = run + ex;
    }
    run += tot;
  }
  if (threadIdx.x == 0) {
    segfirst[tiles_x] = run;
    misc[kSegTotal] = run;
    *reinterpret_cast<unsigned long long*>(misc + kPLo) = P;
    const uint64_t need = (int64_t)C > cap && (uint64_t)C > P ? (uint64_t)C : P;
    *pair_count = need > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)need;
  }
}

// step 5: pairs per row of every segment, hist[seg * tiles_y + ty], and its
// pair total segtot[seg]; one wavefront per segment. A run (ty0, len) adds
// one pair to rows ty0 .. ty0 + len - 1: +1 / -1 at the ends of a
// difference array, then a prefix sum over the rows.
__global__ void __launch_bounds__(kSegThreads) k_seg_hist(
    const uint32_t* __restrict__ cstart, const uint32_t* __restrict__ segfirst,
    const uint2* __restrict__ runs, const uint32_t* __restrict__ misc, int tiles_x, int tiles_y,
    uint32_t* __restrict__ hist, uint32_t* __restrict__ segtot) {
  __shared__ uint32_t dhs[kSegWaves][kMaxRows + 1];
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  uint32_t* dh = dhs[w];
  const uint32_t NS = misc[kSegTotal];
  for (uint32_t seg = blockIdx.x * kSegWaves + w; seg < NS; seg += gridDim.x * kSegWaves) {
    int tx;
    uint32_t r0, r1;
    seg_runs(seg, segfirst, cstart, tiles_x, tx, r0, r1);
    // all loads first (slots past the segment's end read its first run)
    uint32_t Ls[kSegSlots];
#pragma unroll
    for (int j = 0; j < kSegSlots; ++j) {
      const uint32_t k = r0 + j * kWave + lane;
      Ls[j] = runs[k < r1 ? k : r0].y;
    }
    for (int q = lane; q <= kMaxRows; q += kWave) dh[q] = 0;
    uint32_t pairs = 0;
#pragma unroll
    for (int j = 0; j < kSegSlots; ++j) {
      const uint32_t k = r0 + j * kWave + lane;
      if (k < r1) {
        const uint32_t L = Ls[j];
        const uint32_t ty0 = L & 0xFFFFu;
        atomicAdd(&dh[ty0], 1u);
        atomicAdd(&dh[ty0 + (L >> 16)], 0xFFFFFFFFu);  // -1
        pairs += L >> 16;
      }
    }
    // lane l owns rows 4 l .. 4 l + 3 (the wavefront's LDS operations complete
    // in order, so the atomics above are seen)
    uint32_t v[4], sum = 0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      sum += dh[4 * lane + e];
      v[e] = sum;
    }
    const uint32_t ex = wave_incl_scan_u32(sum) - sum;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int ty = 4 * lane + e;
      if (ty < tiles_y) hist[(int64_t)seg * tiles_y + ty] = ex + v[e];
    }
    const uint32_t tot = wave_incl_scan_u32(pairs);
    if (lane == kWave - 1) segtot[seg] = tot;
  }
}

// step 6: one workgroup per column. The column's first position is the sum
// of the totals of the earlier columns' segments; rows are scanned in order, and within a
// row the segments in order: hist becomes each (segment, row)'s first
// position; ranges gets each tile's first position. Thread t handles row
// t % tiles_y of the segments of group t / tiles_y (contiguous groups).
__global__ void __launch_bounds__(kScanThreads1) k_col_scan(
    const uint32_t* __restrict__ nseg, const uint32_t* __restrict__ segfirst,
    const uint32_t* __restrict__ segtot, const uint32_t* __restrict__ misc, int64_t cap,
    int tiles_x, int tiles_y, uint32_t* __restrict__ hist, uint32_t* __restrict__ ranges) {
  constexpr int NTH = kScanThreads1;
  __shared__ uint32_t gsum[NTH];
  __shared__ uint32_t rowbase[kMaxRows];
  __shared__ uint32_t wsum[NTH / kWave];
  const int tx = blockIdx.x;
  const uint64_t P = pair_total(misc);
  const int64_t n_tiles = (int64_t)tiles_x * tiles_y;
  if (P > (uint64_t)cap || (int64_t)misc[kRunTotal] > cap) {  // overflow: every tile empty
    for (int t = threadIdx.x; t < tiles_y; t += NTH) ranges[(int64_t)tx * tiles_y + t] = 0;
    if (tx == tiles_x - 1 && threadIdx.x == 0) ranges[n_tiles] = 0;
    return;
  }
  const int G = NTH / tiles_y;  // >= 4 groups (tiles_y <= 256)
  const int ty = threadIdx.x % tiles_y, g = threadIdx.x / tiles_y;
  const bool act = g < G;
  const uint32_t ns = nseg[tx], sf = segfirst[tx];
  // the pairs of the earlier columns: the totals of the segments before sf
  uint32_t part = 0;
  uint32_t t = threadIdx.x;
  for (; t + 3 * NTH < sf; t += 4 * NTH)  // four loads in flight per thread
    part += segtot[t] + segtot[t + NTH] + segtot[t + 2 * NTH] + segtot[t + 3 * NTH];
  for (; t < sf; t += NTH) part += segtot[t];
  uint32_t cbase;
  block_exclusive_scan<NTH>(part, wsum, cbase);
  const uint32_t s0 = act ? (uint32_t)(((uint64_t)ns * g) / G) : 0u;
  const uint32_t s1 = act ? (uint32_t)(((uint64_t)ns * (g + 1)) / G) : 0u;
  uint32_t rs = 0;
#pragma unroll 8
  for (uint32_t s = s0; s < s1; ++s) rs += hist[(int64_t)(sf + s) * tiles_y + ty];
  gsum[threadIdx.x] = rs;
  __syncthreads();
  // row totals (threads of group 0), scanned over the rows in thread order
  uint32_t rowtot = 0;
  if (g == 0)
    for (int j = 0; j < G; ++j) rowtot += gsum[j * tiles_y + ty];
  uint32_t all;
  const uint32_t rex = block_exclusive_scan<NTH>(g == 0 ? rowtot : 0u, wsum, all);
  if (g == 0) rowbase[ty] = rex;
  __syncthreads();
  if (act) {
    uint32_t run = cbase + rowbase[ty];
    if (g == 0) ranges[(int64_t)tx * tiles_y + ty] = run;
    for (int j = 0; j < g; ++j) run += gsum[j * tiles_y + ty];
#pragma unroll 8
    for (uint32_t s = s0; s < s1; ++s) {
      const int64_t i = (int64_t)(sf + s) * tiles_y + ty;
      const uint32_t v = hist[i];
      hist[i] = run;
      run += v;
    }
  }
  if (tx == tiles_x - 1 && threadIdx.x == 0) ranges[n_tiles] = (uint32_t)P;
}


// step 7: one wavefront per segment; lane l holds runs l, 64 + l, 128 + l,
// ... of it (kSegSlots slots, in run order slot by slot). For each row any of
// them covers, one ballot per slot marks the covering runs; they write their
// Gaussian id at the row's position plus the number of covering runs before
// them (lower slots first, then lower lanes), and the row's position
// advances by their number. Runs keep depth order within a row. The rows'
// positions live in registers: lane l holds those of rows l, 64 + l, ...
template <bool KEYS>
__global__ void __launch_bounds__(kSegThreads) k_run_scatter(
    const uint32_t* __restrict__ cstart, const uint32_t* __restrict__ segfirst,
    const uint2* __restrict__ runs,
    const uint32_t* __restrict__ misc, const uint32_t* __restrict__ hist,
    const uint32_t* __restrict__ depth_keys, int64_t n, int64_t cap, int tiles_x, int tiles_y,
    uint32_t* __restrict__ vals, uint64_t* __restrict__ keys_out) {
  constexpr int RB = kMaxRows / kWave;  // row blocks of 64
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  const uint32_t NS = misc[kSegTotal];
  const uint32_t cap32 = (uint32_t)cap;  // cap <= 2^32 - 2
  for (uint32_t seg = blockIdx.x * kSegWaves + w; seg < NS; seg += gridDim.x * kSegWaves) {
    int tx;
    uint32_t r0, r1;
    seg_runs(seg, segfirst, cstart, tiles_x, tx, r0, r1);
    uint32_t off[RB];
#pragma unroll
    for (int b = 0; b < RB; ++b) {
      const int ty = b * kWave + lane;
      off[b] = ty < tiles_y ? hist[(int64_t)seg * tiles_y + ty] : 0u;
    }
    uint32_t ty0[kSegSlots], len[kSegSlots], gid[kSegSlots];
    uint32_t lo = kMaxRows, hi = 0;
    // all loads first (slots past the segment's end read its first run)
#pragma unroll
    for (int j = 0; j < kSegSlots; ++j) {
      const uint32_t k = r0 + j * kWave + lane;
      const uint32_t kk = k < r1 ? k : r0;
      const uint2 q = runs[kk];
      gid[j] = q.x;
      ty0[j] = q.y;
    }
#pragma unroll
    for (int j = 0; j < kSegSlots; ++j) {
      const uint32_t k = r0 + j * kWave + lane;
      const uint32_t L = ty0[j];
      ty0[j] = L & 0xFFFFu;
      len[j] = k < r1 ? L >> 16 : 0u;  // an empty slot covers no row
      if (len[j]) {
        lo = min(lo, ty0[j]);
        hi = max(hi, ty0[j] + len[j]);
      }
    }
    lo = __builtin_amdgcn_readfirstlane(wave_min_u32(lo));
    hi = __builtin_amdgcn_readfirstlane(wave_max_u32(hi));
    uint64_t key_lo[kSegSlots];
#pragma unroll
    for (int j = 0; j < kSegSlots; ++j)
      key_lo[j] = KEYS ? ((int64_t)gid[j] < n ? depth_keys[gid[j]] : 0xFFFFFFFFu) : 0u;
    const uint64_t tbase = (uint64_t)tx * (uint64_t)tiles_y;
#pragma unroll
    for (int b = 0; b < RB; ++b) {
      const uint32_t ya = max(lo, (uint32_t)(b * kWave)), yb = min(hi, (uint32_t)(b * kWave + kWave));
      for (uint32_t ty = ya; ty < yb; ++ty) {
        uint64_t bal[kSegSlots];
        uint32_t tot = 0;
#pragma unroll
        for (int j = 0; j < kSegSlots; ++j) {
          bal[j] = __ballot(ty - ty0[j] < len[j]);
          tot += (uint32_t)__popcll(bal[j]);
        }
        if (tot == 0) continue;
        const int row_lane = (int)(ty - (uint32_t)(b * kWave));
        uint32_t pos = __builtin_amdgcn_readlane(off[b], row_lane);
        if (pos + tot <= cap32) {  // always, for consistent counts
#pragma unroll
          for (int j = 0; j < kSegSlots; ++j) {
            if (ty - ty0[j] < len[j]) {
              const uint32_t below = __builtin_amdgcn_mbcnt_hi(
                  (uint32_t)(bal[j] >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal[j], 0u));
              const uint32_t p = pos + below;
              vals[p] = gid[j];
              if (KEYS) keys_out[p] = ((tbase + ty) << 32) | key_lo[j];
            }
            pos += (uint32_t)__popcll(bal[j]);
          }
        }
        if (lane == row_lane) off[b] += tot;
      }
    }
  }
}

// Tile counts of the tile-set variants that the compact walk is compared
// with: every tile whose closed cell meets the SnugBox rectangle, or the
// square of half-width ceil(3 sqrt(lambda_max(Sigma'))) around the centroid
// that 3DGS bins with (lambda from its clamp max(0.1, mid^2 - det); opacity
// not considered). FP64 on the stored record, in the order written.
__device__ __forceinline__ void box_cells(double lo, double hi, int tile, int n, int& c0, int& c1) {
#pragma clang fp contract(off)
  const double T = (double)tile;
  const double a = fmax(0.0, ceil(lo / T) - 1.0);
  const double b = fmin((double)(n - 1), floor(hi / T));
  if (!(a <= b)) { c0 = 1; c1 = 0; return; }
  c0 = (int)a;
  c1 = (int)b;
}

__global__ void __launch_bounds__(256) k_tile_count_variant(const float* __restrict__ splats,
                                                            int64_t n, CamDev cam, int variant,
                                                            uint32_t* __restrict__ counts) {
#pragma clang fp contract(off)
  __shared__ SnugLds walk[256];
  __shared__ uint32_t cnt[256];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  Snug s;
  bool has = false;
  float4 r0 = make_float4(0.f, 0.f, 0.f, 0.f), r1 = r0;
  if (i < n) {
    const float4* rec = reinterpret_cast<const float4*>(splats + i * GS_SPLAT_FLOATS);
    r0 = rec[0];
    r1 = rec[1];
    has = snug_setup(r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, s);
  }
  if (variant == GS_TILES_COMPACT) {
    cnt[threadIdx.x] = 0;
    const int wbase = threadIdx.x & ~(kWave - 1);
    wave_column_walk(has, s, cam.tile, cam.tiles_x, cam.tiles_y, walk + wbase,
                     [&](int owner, int, int ty0, int ty1) {
                       if (ty1 >= ty0) atomicAdd(&cnt[wbase + owner], (uint32_t)(ty1 - ty0 + 1));
                     });
    if (i < n) counts[i] = cnt[threadIdx.x];
    return;
  }
  if (i >= n) return;
  double u = r0.x, v = r0.y, hx = 0.0, hy = 0.0;
  bool ok = false;
  if (variant == GS_TILES_SNUGBOX) {
    ok = has;
    hx = s.hx;
    hy = s.hy;
  } else {
    const double a = r0.z, b = r0.w, c = r1.x;
    const double det = a * c - b * b;
    if (det > 0.0) {
      const double sxx = c / det, syy = a / det, sxy = -b / det;
      const double mid = 0.5 * (sxx + syy);
      const double lam = mid + sqrt(fmax(0.1, mid * mid - (sxx * syy - sxy * sxy)));
      const double r = ceil(3.0 * sqrt(lam));
      hx = hy = r;
      ok = true;
    }
  }
  uint32_t total = 0;
  if (ok) {
    int x0, x1, y0, y1;
    box_cells(u - hx, u + hx, cam.tile, cam.tiles_x, x0, x1);
    box_cells(v - hy, v + hy, cam.tile, cam.tiles_y, y0, y1);
    if (x1 >= x0 && y1 >= y0) total = (uint32_t)((x1 - x0 + 1) * (y1 - y0 + 1));
  }
  counts[i] = total;
}

}  // namespace

}  // namespace gs

using namespace gs;

extern "C" gs_status gs_bin_sort_workspace(int64_t n, int64_t capacity, const gs_camera* cam,
                                           size_t* bytes) {
  CamDev cd;
  if (n < 0 || capacity < 0 || capacity > 0xFFFFFFFELL || !bytes || !make_cam(cam, &cd))
    return GS_EINVAL;
  *bytes = (size_t)layout(n, capacity, cd.tiles_x, cd.tiles_y).total;
  return GS_OK;
}

bool gs::run_lists(const void* workspace, size_t bytes, int64_t n, int64_t cap, int tiles_x,
                   int tiles_y, RunLists* out) {
  const BinLayout L = layout(n, cap, tiles_x, tiles_y);
  if (!workspace || (int64_t)bytes < L.total) return false;
  const char* ws = (const char*)workspace;
  out->runs = reinterpret_cast<const uint2*>(ws + L.runs);
  out->cstart = reinterpret_cast<const uint32_t*>(ws + L.cstart);
  out->segfirst = reinterpret_cast<const uint32_t*>(ws + L.segfirst);
  out->hist = reinterpret_cast<const uint32_t*>(ws + L.hist);
  return true;
}

// gs_bin_sort, and with scatter = false its deferred form (every step but
// the last, which writes the lists).
static gs_status bin_sort(const float* splats, const uint32_t* depth_keys,
                          const uint32_t* tile_counts, int64_t n, const gs_camera* cam,
                          void* workspace, size_t workspace_bytes, int64_t capacity,
                          uint32_t* vals, uint32_t* ranges, uint64_t* keys_out,
                          uint32_t* pair_count, void* stream, bool scatter) {
  CamDev cd;
  if (n < 0 || n > 0xFFFFFFFELL || capacity < 0 || capacity > 0xFFFFFFFELL || !make_cam(cam, &cd))
    return GS_EINVAL;
  if (cd.tiles_y > kMaxRows || cd.tiles_x > kMaxCols) return GS_EINVAL;
  if (!ranges || !pair_count || (n > 0 && (!splats || !depth_keys || !tile_counts)) ||
      (scatter && capacity > 0 && !vals) || !workspace)
    return GS_EINVAL;
  const BinLayout L = layout(n, capacity, cd.tiles_x, cd.tiles_y);
  if ((int64_t)workspace_bytes < L.total) return GS_ECAPACITY;
  hipStream_t st = (hipStream_t)stream;
  char* ws = (char*)workspace;
  auto U = [&](int64_t off) { return reinterpret_cast<uint32_t*>(ws + off); };
  auto R2 = [&](int64_t off) { return reinterpret_cast<uint2*>(ws + off); };
  const int n_tiles = cd.tiles_x * cd.tiles_y;
  uint32_t* misc = U(L.misc);
  const int64_t cap = capacity;
  gs_status s;

  const int nparts = n > 0 ? (int)std::min<int64_t>(div_up(n, 256), kCountBlocks) : 0;
  unsigned long long* part = reinterpret_cast<unsigned long long*>(ws + L.ptot);
  uint32_t* colh = U(L.colh);
  const int64_t ncolh = (int64_t)cd.tiles_x * L.nblk;
  if (n > 0) {
    k_count_partials<<<nparts, 256, 0, st>>>(tile_counts, n, part);
    GS_CHECK_LAUNCH();
    // 1. stable depth sort (Gaussians without tiles carry 0xFFFFFFFF); the
    // first pass takes the Gaussian indices as its values and each
    // Gaussian's column span (record word 11) as its second values, so the
    // spans come out in depth order
    const uint32_t* kin = depth_keys;
    uint32_t *kA = U(L.dkA), *kB = U(L.dkB), *vA = U(L.dvA), *vB = U(L.dvB);
    uint32_t *sA = U(L.spA), *sB = U(L.spB);
    for (int pass = 0; pass < 4; ++pass) {
      const bool even = (pass % 2) == 0;
      const uint32_t* s2 = pass == 0 ? reinterpret_cast<const uint32_t*>(splats) + 11
                                     : (even ? sA : sB);
      s = radix_pass(kin, pass == 0 ? nullptr : (even ? vA : vB), even ? kB : kA, even ? vB : vA,
                     n, nullptr, pass * 8, U(L.rtmp), st, s2, even ? sB : sA, 8,
                     pass == 0 ? GS_SPLAT_FLOATS : 1);
      if (s != GS_OK) return s;
      kin = even ? kB : kA;
    }
    // 2. runs per (column, block), scanned: each block's first position in
    // each column, and the run total
    k_col_hist<<<(unsigned)L.nblk, kEmitBlock, 4 * (cd.tiles_x + 1), st>>>(sA, n, cd.tiles_x,
                                                                          colh);
    GS_CHECK_LAUNCH();
  }
  s = scan_u32(colh, colh, ncolh, misc + kRunTotal, U(L.stmp), st);
  if (s != GS_OK) return s;
  // 3. the runs, column by column in depth order
  if (n > 0 && cap > 0) {
    GS_TIMED("bin_runs", st,
             (tuning().seq_walk ? k_runs_emit<true> : k_runs_emit<false>)<<<
                 (unsigned)L.nblk, kEmitBlock, 4 * kEmitWaves * cd.tiles_x, st>>>(
                 U(L.dvA), U(L.spA), splats, n, cd, colh, cap, R2(L.runs)));
    GS_CHECK_LAUNCH();
  }
  uint32_t* cstart = U(L.cstart);
  // 4. pair total, column starts, segments per column (and the pair count output)
  k_seg_layout<<<1, 256, 0, st>>>(part, nparts, colh, L.nblk, cstart, cap, cd.tiles_x,
                                  U(L.nseg), U(L.segfirst), misc, pair_count);
  GS_CHECK_LAUNCH();
  uint32_t* hist = U(L.hist);
  // one wavefront per segment, 4 per workgroup, grid-stride over the live ones
  const unsigned sg =
      (unsigned)std::max<int64_t>(1, std::min<int64_t>(div_up(L.ns_max, kSegWaves), 4096));
  // 5. pairs per (segment, row)
  if (cap > 0) {
    GS_TIMED("bin_hist", st,
             k_seg_hist<<<sg, kSegThreads, 0, st>>>(cstart, U(L.segfirst), R2(L.runs), misc,
                                                    cd.tiles_x, cd.tiles_y, hist, U(L.segtot)));
    GS_CHECK_LAUNCH();
  }
  // 6. segment positions and tile ranges
  k_col_scan<<<cd.tiles_x, kScanThreads1, 0, st>>>(U(L.nseg), U(L.segfirst), U(L.segtot),
                                                           misc, cap, cd.tiles_x, cd.tiles_y, hist,
                                                           ranges);
  GS_CHECK_LAUNCH();
  // 7. final positions
  if (scatter && cap > 0) {
    GS_TIMED("bin_scatter", st,
             (keys_out ? k_run_scatter<true> : k_run_scatter<false>)<<<sg, kSegThreads, 0, st>>>(
                 cstart, U(L.segfirst), R2(L.runs), misc, hist, depth_keys, n, cap,
                 cd.tiles_x, cd.tiles_y, vals, keys_out));
    GS_CHECK_LAUNCH();
  }
  return GS_OK;
}

extern "C" gs_status gs_bin_sort(const float* splats, const uint32_t* depth_keys,
                                 const uint32_t* tile_counts, int64_t n, const gs_camera* cam,
                                 void* workspace, size_t workspace_bytes, int64_t capacity,
                                 uint32_t* vals, uint32_t* ranges, uint64_t* keys_out,
                                 uint32_t* pair_count, void* stream) {
  return bin_sort(splats, depth_keys, tile_counts, n, cam, workspace, workspace_bytes, capacity,
                  vals, ranges, keys_out, pair_count, stream, true);
}

extern "C" gs_status gs_bin_sort_deferred(const float* splats, const uint32_t* depth_keys,
                                          const uint32_t* tile_counts, int64_t n,
                                          const gs_camera* cam, void* workspace,
                                          size_t workspace_bytes, int64_t capacity,
                                          uint32_t* ranges, uint32_t* pair_count, void* stream) {
  return bin_sort(splats, depth_keys, tile_counts, n, cam, workspace, workspace_bytes, capacity,
                  nullptr, ranges, nullptr, pair_count, stream, false);
}

extern "C" gs_status gs_bin_sort_batched_workspace(int64_t n, const gs_view* views, int32_t n_views,
                                                   size_t* bytes) {
  if (!views || n_views < 1 || n_views > GS_MAX_VIEWS || !bytes) return GS_EINVAL;
  size_t best = 0;
  for (int v = 0; v < n_views; ++v) {
    size_t b = 0;
    const gs_status s = gs_bin_sort_workspace(n, views[v].capacity, &views[v].cam, &b);
    if (s != GS_OK) return s;
    best = b > best ? b : best;
  }
  *bytes = best;
  return GS_OK;
}

extern "C" gs_status gs_bin_sort_batched_deferred(int64_t n, const gs_view* views,
                                                  int32_t n_views, void* const* workspaces,
                                                  const size_t* workspace_bytes, void* stream) {
  if (!views || n_views < 1 || n_views > GS_MAX_VIEWS || !workspaces || !workspace_bytes)
    return GS_EINVAL;
  for (int v = 0; v < n_views; ++v) {
    const gs_view& w = views[v];
    const gs_status s =
        gs_bin_sort_deferred(w.splats, w.depth_keys, w.tile_counts, n, &w.cam, workspaces[v],
                             workspace_bytes[v], w.capacity, w.ranges, w.pair_count, stream);
    if (s != GS_OK) return s;
  }
  return GS_OK;
}

extern "C" gs_status gs_bin_sort_batched(int64_t n, const gs_view* views, int32_t n_views,
                                         void* workspace, size_t workspace_bytes, void* stream) {
  if (!views || n_views < 1 || n_views > GS_MAX_VIEWS) return GS_EINVAL;
  for (int v = 0; v < n_views; ++v) {
    const gs_view& w = views[v];
    const gs_status s = gs_bin_sort(w.splats, w.depth_keys, w.tile_counts, n, &w.cam, workspace,
                                    workspace_bytes, w.capacity, w.vals, w.ranges, w.keys_out,
                                    w.pair_count, stream);
    if (s != GS_OK) return s;
  }
  return GS_OK;
}

extern "C" gs_status gs_tile_count_variant(const float* splats, int64_t n, const gs_camera* cam,
                                           int32_t variant, uint32_t* counts, void* stream) {
  CamDev cd;
  if (n < 0 || !make_cam(cam, &cd) ||
      (variant != GS_TILES_COMPACT && variant != GS_TILES_SNUGBOX && variant != GS_TILES_3SIGMA) ||
      (n > 0 && (!splats || !counts)))
    return GS_EINVAL;
  if (n == 0) return GS_OK;
  hipStream_t st = (hipStream_t)stream;
  k_tile_count_variant<<<div_up(n, 256), 256, 0, st>>>(splats, n, cd, variant, counts);
  GS_CHECK_LAUNCH();
  return GS_OK;
}
