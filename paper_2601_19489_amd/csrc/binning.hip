// Binning and depth sort (Sec. 2.1): every Gaussian writes one pair per tile
// of its compact tile set; the pairs end up ordered by (tile id, depth bits,
// Gaussian index), tiles numbered column-major (id = tx * tiles_y + ty).
//
// The paper's column walk produces, per Gaussian, runs of consecutive tiles
// (one run per column of its SnugBox). Instead of materialising and sorting
// the P pairs, this works on the runs (about P / 20 of them):
//   1. stable sort of the Gaussians by depth (32-bit keys; ties keep index
//      order);
//   2. per Gaussian, in depth order, its non-empty column runs
//      (column tx, first row ty0, length), written in depth order;
//   3. stable sort of the runs by column: each column now lists its runs in
//      depth order;
//   4. scan of the run lengths: pair positions within the column-major
//      concatenation;
//   5. each column's pairs are cut into blocks of kPairBlock; a block counts
//      its pairs per row, one scan over all (column, row, block) counts gives
//      every block's first position per tile and the tile ranges;
//   6. each block regenerates its pairs, ranks them stably by row and writes
//      the Gaussian ids to their final positions through LDS.
// Only the final 4-byte Gaussian id is written per pair.
#include <algorithm>

#include "common.h"
#include "sort.h"

namespace gs {

namespace {

constexpr int kPairBlock = 2048;  // pairs per block in steps 5-6
constexpr int kPairThreads = 256;
constexpr int kPairItems = kPairBlock / kPairThreads;  // per thread (8)
constexpr int kMaxRows = 256;     // 8-bit row ranking: tiles_y <= 256
constexpr int64_t kAlign = 256;

inline int64_t al(int64_t b) { return (b + kAlign - 1) / kAlign * kAlign; }

struct BinLayout {
  int64_t dkA, dkB, dvA, dvB, nrun, rbase;
  int64_t rk0, rk1, rg0, rg1, rl0, rl1;
  int64_t cstart, colp0, colnb, colbb, misc, hist, binfo;
  int64_t rtmp, stmp, total;
  int64_t nb_max;
};

BinLayout layout(int64_t n, int64_t cap, int tiles_x, int tiles_y) {
  BinLayout L;
  int64_t o = 0;
  const int64_t nw = al(4 * std::max<int64_t>(n, 1));
  const int64_t cw = al(4 * std::max<int64_t>(cap, 1));
  const int64_t tw = al(4 * ((int64_t)tiles_x + 2));
  L.nb_max = (cap + kPairBlock - 1) / kPairBlock + tiles_x;
  L.dkA = o; o += nw;
  L.dkB = o; o += nw;
  L.dvA = o; o += nw;
  L.dvB = o; o += nw;
  L.nrun = o; o += nw;
  L.rbase = o; o += nw;
  L.rk0 = o; o += cw;
  L.rk1 = o; o += cw;
  L.rg0 = o; o += cw;
  L.rg1 = o; o += cw;
  L.rl0 = o; o += cw;
  L.rl1 = o; o += cw;
  L.cstart = o; o += tw;
  L.colp0 = o; o += tw;
  L.colnb = o; o += tw;
  L.colbb = o; o += tw;
  L.misc = o; o += al(64);
  L.hist = o; o += al(4 * (int64_t)tiles_y * L.nb_max);
  L.binfo = o; o += al(32 * L.nb_max);
  const int64_t sortn = std::max(n, cap);
  L.rtmp = o; o += al(4 * radix_tmp_words(sortn));
  L.stmp = o; o += al(4 * (scan_tmp_words(std::max(sortn, (int64_t)tiles_y * L.nb_max)) + 1));
  L.total = o;
  return L;
}

// misc words
constexpr int kRunTotal = 0;   // number of runs C
constexpr int kNbTotal = 1;    // number of pair blocks
constexpr int kHistN = 2;      // tiles_y * blocks
constexpr int kPLo = 4;        // exact pair total as uint64 (words 4, 5)

__device__ __forceinline__ uint64_t pair_total(const uint32_t* misc) {
  return *reinterpret_cast<const uint64_t*>(misc + kPLo);
}

__global__ void k_zero_misc(uint32_t* misc) {
  if (threadIdx.x < 16) misc[threadIdx.x] = 0;
}

// exact total of the tile counts (64-bit, so an overflow of the capacity is
// always seen)
__global__ void __launch_bounds__(256) k_count_total(const uint32_t* __restrict__ counts,
                                                     int64_t n, uint32_t* misc) {
  __shared__ unsigned long long part[256 / kWave];
  unsigned long long acc = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    acc += counts[i];
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) acc += __shfl_xor(acc, d, kWave);
  if ((threadIdx.x & (kWave - 1)) == 0) part[threadIdx.x / kWave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
#pragma unroll
    for (int w = 0; w < 256 / kWave; ++w) t += part[w];
    atomicAdd(reinterpret_cast<unsigned long long*>(misc + kPLo), t);
  }
}

__device__ __forceinline__ bool load_snug(const float* splats, uint32_t g, Snug& s) {
  const float4* rec = reinterpret_cast<const float4*>(splats + (int64_t)g * GS_SPLAT_FLOATS);
  const float4 r0 = rec[0], r1 = rec[1];
  return snug_setup(r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, s);
}

// step 2a: number of column runs of each Gaussian in depth order, as the
// preprocess recorded it in field 11 of the record
__global__ void __launch_bounds__(256) k_runs_count(const uint32_t* __restrict__ order,
                                                    const uint32_t* __restrict__ counts,
                                                    const float* __restrict__ splats, int64_t n,
                                                    uint32_t* __restrict__ nrun) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const uint32_t g = order[r];
  nrun[r] = ((int64_t)g < n && counts[g] > 0)
                ? __float_as_uint(splats[(int64_t)g * GS_SPLAT_FLOATS + 11])
                : 0u;
}

// step 2b: write the runs (key: column; values: Gaussian, row0 | len << 16).
// The order of one Gaussian's runs does not matter (they go to different
// columns); runs of different Gaussians keep the depth order.
template <bool SEQ>
__global__ void __launch_bounds__(256) k_runs_emit(
    const uint32_t* __restrict__ order, const uint32_t* __restrict__ counts,
    const float* __restrict__ splats, int64_t n, CamDev cam, const uint32_t* __restrict__ rbase,
    const uint32_t* __restrict__ misc, int64_t cap, uint32_t* __restrict__ rk,
    uint32_t* __restrict__ rg, uint32_t* __restrict__ rl) {
  __shared__ SnugLds walk[256];
  __shared__ uint32_t ctr[256], base[256], gid[256];
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool over = pair_total(misc) > (uint64_t)cap;  // overflow: nothing is written
  Snug s;
  bool has = false;
  uint32_t g = 0;
  if (r < n && !over) {
    g = order[r];
    has = (int64_t)g < n && counts[g] > 0 && load_snug(splats, g, s);
  }
  ctr[threadIdx.x] = 0;
  base[threadIdx.x] = (r < n) ? rbase[r] : 0u;
  gid[threadIdx.x] = g;
  const int wbase = threadIdx.x & ~(kWave - 1);
  column_walk<SEQ>(has, s, cam.tile, cam.tiles_x, cam.tiles_y, walk + wbase,
                   [&](int owner, int tx, int ty0, int ty1) {
                     if (ty1 < ty0) return;
                     const int q = wbase + owner;
                     const int64_t o = (int64_t)base[q] + atomicAdd(&ctr[q], 1u);
                     if (o < cap) {
                       rk[o] = (uint32_t)tx;
                       rg[o] = gid[q];
                       rl[o] = (uint32_t)ty0 | ((uint32_t)(ty1 - ty0 + 1) << 16);
                     }
                   });
}

// First position of each key in a sorted key array (keys < n_bins), for
// bins [0, n_bins]; empty bins get the position of the next key.
// Grid-stride over a device-side count (the grid is sized for a bound).
__global__ void k_bin_starts(const uint32_t* __restrict__ keys,
                             const uint32_t* __restrict__ cnt_dev, int64_t cap, int n_bins,
                             uint32_t* __restrict__ starts) {
  const int64_t c = std::min<int64_t>((int64_t)*cnt_dev, cap);
  const auto key_at = [&](int64_t j) -> int64_t {
    const uint32_t k = keys[j];
    return k < (uint32_t)n_bins ? (int64_t)k : (int64_t)n_bins - 1;
  };
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= c;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (i < c) {
      const int64_t k = key_at(i);
      const int64_t kp = i ? key_at(i - 1) : -1;
      for (int64_t t = kp + 1; t <= k; ++t) starts[t] = (uint32_t)i;
    } else {
      const int64_t kl = c ? key_at(c - 1) : -1;
      for (int64_t t = kl + 1; t <= n_bins; ++t) starts[t] = (uint32_t)c;
    }
  }
}

inline unsigned bounded_grid(int64_t n) { return (unsigned)std::min<int64_t>(div_up(n, 256), 4096); }

// step 5a: blocks per column. One workgroup.
__global__ void __launch_bounds__(256) k_col_blocks(
    const uint32_t* __restrict__ cstart, const uint32_t* __restrict__ rpos, int64_t cap,
    int tiles_x, int tiles_y, uint32_t* __restrict__ colp0, uint32_t* __restrict__ colnb,
    uint32_t* __restrict__ colbb, uint32_t* __restrict__ misc, uint32_t* __restrict__ pair_count) {
  __shared__ uint32_t wsum[256 / kWave];
  const uint64_t P = pair_total(misc);
  const bool over = P > (uint64_t)cap;
  const uint32_t C = misc[kRunTotal];
  const auto pos = [&](uint32_t i) -> uint32_t { return i < C ? rpos[i] : (uint32_t)P; };
  uint32_t run = 0;
  for (int base = 0; base < tiles_x; base += 256) {
    const int tx = base + threadIdx.x;
    uint32_t nb = 0, p0 = 0;
    if (tx < tiles_x && !over) {
      p0 = pos(cstart[tx]);
      const uint32_t p1 = pos(cstart[tx + 1]);
      nb = (p1 - p0 + kPairBlock - 1) / kPairBlock;
    }
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan<256>(nb, wsum, tot);
    if (tx < tiles_x) {
      colp0[tx] = p0;
      colnb[tx] = nb;
      colbb[tx] = run + ex;
    }
    run += tot;
  }
  if (threadIdx.x == 0) {
    colp0[tiles_x] = over ? 0u : (uint32_t)P;
    colbb[tiles_x] = run;
    misc[kNbTotal] = run;
    misc[kHistN] = run * (uint32_t)tiles_y;
    *pair_count = P > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)P;
  }
}

// Block geometry of steps 5b / 6, shared through LDS.
struct PairBlk {
  int tx;
  uint32_t bl, nb, lo, hi, r0, wcount, seg;
};
static_assert(sizeof(PairBlk) == 32, "8 words");

// step 5b': geometry of every pair block (one thread per block)
__global__ void k_block_info(const uint32_t* __restrict__ cstart,
                             const uint32_t* __restrict__ rpos,
                             const uint32_t* __restrict__ colp0,
                             const uint32_t* __restrict__ colnb,
                             const uint32_t* __restrict__ colbb,
                             const uint32_t* __restrict__ misc, int tiles_x, int tiles_y,
                             PairBlk* __restrict__ binfo);

__device__ uint32_t upper_bound_u32(const uint32_t* a, uint32_t lo, uint32_t hi, uint32_t x) {
  while (lo < hi) {
    const uint32_t mid = lo + ((hi - lo) >> 1);
    if (a[mid] <= x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

__global__ void k_block_info(const uint32_t* __restrict__ cstart,
                             const uint32_t* __restrict__ rpos,
                             const uint32_t* __restrict__ colp0,
                             const uint32_t* __restrict__ colnb,
                             const uint32_t* __restrict__ colbb,
                             const uint32_t* __restrict__ misc, int tiles_x, int tiles_y,
                             PairBlk* __restrict__ binfo) {
  const uint32_t B = blockIdx.x * blockDim.x + threadIdx.x;
  if (B >= misc[kNbTotal]) return;
  PairBlk pb;
  const int tx = (int)upper_bound_u32(colbb, 0, (uint32_t)tiles_x, B) - 1;
  pb.tx = tx;
  pb.bl = B - colbb[tx];
  pb.nb = colnb[tx];
  pb.lo = colp0[tx] + pb.bl * kPairBlock;
  pb.hi = min(pb.lo + (uint32_t)kPairBlock, colp0[tx + 1]);
  const uint32_t c0 = cstart[tx], c1 = cstart[tx + 1];
  pb.r0 = upper_bound_u32(rpos, c0, c1, pb.lo) - 1;
  const uint32_t rlast = upper_bound_u32(rpos, c0, c1, pb.hi - 1) - 1;
  pb.wcount = min(rlast - pb.r0 + 1, (uint32_t)kPairBlock + 1u);
  pb.seg = (uint32_t)tiles_y * colbb[tx];
  binfo[B] = pb;
}

__device__ __forceinline__ uint32_t wave_incl_max_u32(uint32_t v) {
  const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const uint32_t o = __shfl_up(v, d, kWave);
    if (lane >= d) v = max(v, o);
  }
  return v;
}

// Every thread loads the block's run window and builds map[j - lo] = window
// index of the run holding pair j (run starts marked, then an inclusive
// max-scan). A block's pairs come from at most kPairBlock + 1 runs because
// every run holds at least one pair. Per window run k the block keeps
// wty[k] = ty0_k - rpos_k (mod 2^32), so pair j of run k lies in row
// wty[k] + j, and wg[k] = its Gaussian.
__device__ __forceinline__ void pair_block_setup(uint32_t B, const PairBlk* binfo,
                                                 const uint32_t* rpos, const uint32_t* rl,
                                                 const uint32_t* rg, PairBlk& pb, uint32_t* wty,
                                                 uint32_t* wg, uint16_t* map, uint32_t* wmax) {
  static_assert(kPairItems == 8, "the max-scan reads 8 map entries as one 16-byte word");
  if (threadIdx.x < 8)
    reinterpret_cast<uint32_t*>(&pb)[threadIdx.x] =
        reinterpret_cast<const uint32_t*>(binfo + B)[threadIdx.x];
  for (int q = threadIdx.x; q < kPairBlock / 2; q += kPairThreads)
    reinterpret_cast<uint32_t*>(map)[q] = 0;
  __syncthreads();
  for (uint32_t k = threadIdx.x; k < pb.wcount; k += kPairThreads) {
    const uint32_t p = rpos[pb.r0 + k];
    wty[k] = (rl[pb.r0 + k] & 0xFFFFu) - p;
    wg[k] = rg[pb.r0 + k];
    const uint32_t st = p > pb.lo ? p - pb.lo : 0u;
    if (st < (uint32_t)kPairBlock) map[st] = (uint16_t)k;
  }
  __syncthreads();
  // inclusive max-scan of map: kPairItems consecutive entries per thread,
  // read and written as one 16-byte word
  constexpr int NW = kPairThreads / kWave;
  uint32_t loc[kPairItems];
  uint32_t m = 0;
  {
    const uint4 q = reinterpret_cast<const uint4*>(map)[threadIdx.x];
    const uint32_t wds[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int e = 0; e < kPairItems; ++e) {
      m = max(m, (wds[e >> 1] >> (16 * (e & 1))) & 0xFFFFu);
      loc[e] = m;
    }
  }
  const uint32_t incl = wave_incl_max_u32(m);
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  if (lane == kWave - 1) wmax[w] = incl;
  uint32_t prev = __shfl_up(incl, 1, kWave);
  if (lane == 0) prev = 0;
  __syncthreads();
#pragma unroll
  for (int j = 0; j < NW; ++j)
    if (j < w) prev = max(prev, wmax[j]);
  uint32_t wds[4];
#pragma unroll
  for (int e = 0; e < kPairItems; e += 2)
    wds[e >> 1] = max(prev, loc[e]) | (max(prev, loc[e + 1]) << 16);
  reinterpret_cast<uint4*>(map)[threadIdx.x] = make_uint4(wds[0], wds[1], wds[2], wds[3]);
  __syncthreads();
}

// step 5b: per block, pairs per row. A run k of the block's window holds the
// pairs [rpos_k, rpos_k + len_k) at rows ty0_k, ty0_k + 1, ...; clipped to
// the block's pair range it adds one pair to each row of an interval, so
// +1 / -1 at the interval's ends of a difference array and a prefix sum over
// the rows give the counts (two LDS atomics per run instead of one per pair).
__global__ void __launch_bounds__(kPairThreads) k_pair_hist(
    const PairBlk* __restrict__ binfo, const uint32_t* __restrict__ rpos,
    const uint32_t* __restrict__ rl, const uint32_t* __restrict__ misc, int tiles_y,
    uint32_t* __restrict__ hist) {
  __shared__ uint32_t dh[kMaxRows + 1], wsum[kPairThreads / kWave];
  __shared__ PairBlk pb;
  const uint32_t B = blockIdx.x;
  if (B >= misc[kNbTotal]) return;
  if (threadIdx.x < 8)
    reinterpret_cast<uint32_t*>(&pb)[threadIdx.x] =
        reinterpret_cast<const uint32_t*>(binfo + B)[threadIdx.x];
  for (int q = threadIdx.x; q <= kMaxRows; q += kPairThreads) dh[q] = 0;
  __syncthreads();
  for (uint32_t k = threadIdx.x; k < pb.wcount; k += kPairThreads) {
    const uint32_t p = rpos[pb.r0 + k], L = rl[pb.r0 + k];
    const uint32_t e0 = p + (L >> 16);
    const uint32_t s = max(p, pb.lo), e = min(e0, pb.hi);
    if (s < e) {
      const uint32_t ty0 = L & 0xFFFFu;
      atomicAdd(&dh[ty0 + (s - p)], 1u);
      atomicAdd(&dh[ty0 + (e - p)], 0xFFFFFFFFu);  // -1
    }
  }
  __syncthreads();
  const uint32_t d = dh[threadIdx.x];  // rows 0..255; row tiles_y and above carry no pairs
  uint32_t tot;
  const uint32_t c = block_exclusive_scan<kPairThreads>(d, wsum, tot) + d;
  if ((int)threadIdx.x < tiles_y) hist[pb.seg + threadIdx.x * pb.nb + pb.bl] = c;
}

// step 5c: ranges from the scanned counts
__global__ void k_tile_ranges(const uint32_t* __restrict__ hist,
                              const uint32_t* __restrict__ colp0,
                              const uint32_t* __restrict__ colnb,
                              const uint32_t* __restrict__ colbb,
                              const uint32_t* __restrict__ misc, int64_t cap, int tiles_x,
                              int tiles_y, uint32_t* __restrict__ ranges) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n_tiles = (int64_t)tiles_x * tiles_y;
  if (t > n_tiles) return;
  const uint64_t P = pair_total(misc);
  if (P > (uint64_t)cap) {
    ranges[t] = 0;
    return;
  }
  if (t == n_tiles) {
    ranges[t] = (uint32_t)P;
    return;
  }
  const int tx = (int)(t / tiles_y), ty = (int)(t % tiles_y);
  const uint32_t nb = colnb[tx];
  ranges[t] = nb ? hist[(int64_t)tiles_y * colbb[tx] + (int64_t)ty * nb] : colp0[tx];
}

// step 6: regenerate, rank stably by row (BITS ballots: rows < 2^BITS), write
// through LDS
template <int BITS>
__global__ void __launch_bounds__(kPairThreads) k_pair_scatter(
    const PairBlk* __restrict__ binfo, const uint32_t* __restrict__ rpos,
    const uint32_t* __restrict__ rl, const uint32_t* __restrict__ rg,
    const uint32_t* __restrict__ misc, const uint32_t* __restrict__ hist,
    const uint32_t* __restrict__ depth_keys, int64_t n, int64_t cap, int tiles_y,
    uint32_t* __restrict__ vals, uint64_t* __restrict__ keys_out) {
  constexpr int NW = kPairThreads / kWave;
  constexpr int SEG = kPairBlock / NW;  // items per wavefront, walked in order
  constexpr int ROWS = 1 << BITS;
  __shared__ uint32_t wty[kPairBlock + 1], wg[kPairBlock + 1];
  __shared__ __align__(16) uint16_t map[kPairBlock];
  __shared__ uint32_t cnt[NW][ROWS];
  __shared__ uint32_t boff[kMaxRows], gbase[kMaxRows];
  __shared__ uint32_t wsum[NW];
  __shared__ PairBlk pb;
  const uint32_t B = blockIdx.x;
  if (B >= misc[kNbTotal]) return;
  for (int j = threadIdx.x; j < NW * ROWS; j += kPairThreads) (&cnt[0][0])[j] = 0;
  pair_block_setup(B, binfo, rpos, rl, rg, pb, wty, wg, map, wsum);
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (kWave - lane));
  uint32_t gid[kPairItems], row[kPairItems], rank[kPairItems];
  const uint32_t seg0 = pb.lo + (uint32_t)w * SEG;
#pragma unroll
  for (int r = 0; r < kPairItems; ++r) {
    const uint32_t j = seg0 + (uint32_t)r * kWave + lane;
    const bool valid = j < pb.hi;
    uint32_t ty = 0, g = 0;
    if (valid) {
      const uint32_t k = map[j - pb.lo];
      ty = wty[k] + j;
      g = wg[k];
    }
    ty &= ROWS - 1;
    gid[r] = g;
    row[r] = ty;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < BITS; ++bit) {
      const bool set = (ty >> bit) & 1u;
      const uint64_t bal = __ballot(set);
      peers &= set ? bal : ~bal;
    }
    rank[r] = 0;
    if (valid) {
      const uint32_t old = cnt[w][ty];
      const uint64_t below = peers & lt;
      rank[r] = old + (uint32_t)__popcll(below);
      if (below == 0) cnt[w][ty] = old + (uint32_t)__popcll(peers);
    }
  }
  __syncthreads();
  {
    const int t = threadIdx.x;  // one row per thread
    uint32_t tot = 0;
    if (t < ROWS) {
#pragma unroll
      for (int j = 0; j < NW; ++j) {
        const uint32_t c = cnt[j][t];
        cnt[j][t] = tot;
        tot += c;
      }
    }
    uint32_t all;
    boff[t] = block_exclusive_scan<kPairThreads>(tot, wsum, all);
    gbase[t] = t < tiles_y ? hist[pb.seg + (uint32_t)t * pb.nb + pb.bl] : 0u;
  }
  __syncthreads();
  // stage (position, id) in row order; the window is no longer needed
  uint32_t* spos = wty;
  uint32_t* sgid = wg;
#pragma unroll
  for (int r = 0; r < kPairItems; ++r) {
    const uint32_t j = seg0 + (uint32_t)r * kWave + lane;
    if (j < pb.hi) {
      const uint32_t ty = row[r];
      const uint32_t within = cnt[w][ty] + rank[r];
      const uint32_t li = boff[ty] + within;
      spos[li] = gbase[ty] + within;
      sgid[li] = gid[r];
    }
  }
  __syncthreads();
  const uint32_t count = pb.hi - pb.lo;
  for (uint32_t t = threadIdx.x; t < count; t += kPairThreads) {
    const uint32_t pos = spos[t], g = sgid[t];
    if ((int64_t)pos >= cap) continue;  // never for consistent counts
    vals[pos] = g;
    if (keys_out) {
      // the row of staging slot t: the last row whose block offset is <= t
      int lo = 0, hi = ROWS - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (boff[mid] <= t) lo = mid; else hi = mid - 1;
      }
      const uint64_t tid = (uint64_t)pb.tx * (uint64_t)tiles_y + (uint64_t)lo;
      keys_out[pos] = (tid << 32) | (uint64_t)((int64_t)g < n ? depth_keys[g] : 0xFFFFFFFFu);
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

extern "C" gs_status gs_bin_sort(const float* splats, const uint32_t* depth_keys,
                                 const uint32_t* tile_counts, int64_t n, const gs_camera* cam,
                                 void* workspace, size_t workspace_bytes, int64_t capacity,
                                 uint32_t* vals, uint32_t* ranges, uint64_t* keys_out,
                                 uint32_t* pair_count, void* stream) {
  CamDev cd;
  if (n < 0 || n > 0xFFFFFFFELL || capacity < 0 || capacity > 0xFFFFFFFELL || !make_cam(cam, &cd))
    return GS_EINVAL;
  if (cd.tiles_y > kMaxRows) return GS_EINVAL;
  if (!ranges || !pair_count || (n > 0 && (!splats || !depth_keys || !tile_counts)) ||
      (capacity > 0 && !vals) || !workspace)
    return GS_EINVAL;
  const BinLayout L = layout(n, capacity, cd.tiles_x, cd.tiles_y);
  if ((int64_t)workspace_bytes < L.total) return GS_ECAPACITY;
  hipStream_t st = (hipStream_t)stream;
  char* ws = (char*)workspace;
  auto U = [&](int64_t off) { return reinterpret_cast<uint32_t*>(ws + off); };
  const int n_tiles = cd.tiles_x * cd.tiles_y;
  uint32_t* misc = U(L.misc);
  const int64_t cap = capacity;
  gs_status s;

  k_zero_misc<<<1, 64, 0, st>>>(misc);
  GS_CHECK_LAUNCH();
  if (n > 0) {
    k_count_total<<<(unsigned)std::min<int64_t>(div_up(n, 256), 1024), 256, 0, st>>>(tile_counts,
                                                                                      n, misc);
    GS_CHECK_LAUNCH();
    // 1. stable depth sort (Gaussians without tiles carry 0xFFFFFFFF); the
    // first pass takes the Gaussian indices as its values
    const uint32_t* kin = depth_keys;
    uint32_t *kA = U(L.dkA), *kB = U(L.dkB), *vA = U(L.dvA), *vB = U(L.dvB);
    for (int pass = 0; pass < 4; ++pass) {
      const bool even = (pass % 2) == 0;
      s = radix_pass(kin, pass == 0 ? nullptr : (even ? vA : vB), even ? kB : kA, even ? vB : vA,
                     n, nullptr, pass * 8, U(L.rtmp), st);
      if (s != GS_OK) return s;
      kin = even ? kB : kA;
    }
    // 2. column runs in depth order
    GS_TIMED("bin_runs", st,
             k_runs_count<<<div_up(n, 256), 256, 0, st>>>(U(L.dvA), tile_counts, splats, n,
                                                          U(L.nrun)));
    GS_CHECK_LAUNCH();
  }
  s = scan_u32(U(L.nrun), U(L.rbase), n, misc + kRunTotal, U(L.stmp), st);
  if (s != GS_OK) return s;
  if (n > 0 && cap > 0) {
    GS_TIMED("bin_runs", st,
             (tuning().seq_walk ? k_runs_emit<true> : k_runs_emit<false>)<<<div_up(n, 256), 256, 0,
                                                                           st>>>(
                 U(L.dvA), tile_counts, splats, n, cd, U(L.rbase), misc, cap, U(L.rk0), U(L.rg0),
                 U(L.rl0)));
    GS_CHECK_LAUNCH();
  }
  // 3. stable sort of the runs by column (nothing on overflow: runs <= pairs)
  int bits = 1;
  while ((1 << bits) < cd.tiles_x) ++bits;
  const int passes = (bits + 7) / 8;
  uint32_t* rk[2] = {U(L.rk0), U(L.rk1)};
  uint32_t* rg[2] = {U(L.rg0), U(L.rg1)};
  uint32_t* rl[2] = {U(L.rl0), U(L.rl1)};
  int cur = 0;
  if (cap > 0) {
    for (int pass = 0; pass < passes; ++pass) {
      // column keys < tiles_x: only `bits` low bits can be set
      const int pass_bits = bits - pass * 8 < 8 ? bits - pass * 8 : 8;
      s = radix_pass(rk[cur], rg[cur], rk[cur ^ 1], rg[cur ^ 1], cap, misc + kRunTotal, pass * 8,
                     U(L.rtmp), st, rl[cur], rl[cur ^ 1], pass_bits);
      if (s != GS_OK) return s;
      cur ^= 1;
    }
  }
  uint32_t* cstart = U(L.cstart);
  k_bin_starts<<<bounded_grid(cap + 1), 256, 0, st>>>(rk[cur], misc + kRunTotal, cap,
                                                      cd.tiles_x, cstart);
  GS_CHECK_LAUNCH();
  // 4. pair positions of the runs (the other key buffer is free now)
  uint32_t* rpos = rk[cur ^ 1];
  if (cap > 0) {
    // run lengths are the high 16 bits of the run words
    s = scan_u32(rl[cur], rpos, cap, nullptr, U(L.stmp), st, misc + kRunTotal, 16);
    if (s != GS_OK) return s;
  }
  // 5. pair blocks, per-row counts, one scan, tile ranges
  k_col_blocks<<<1, 256, 0, st>>>(cstart, rpos, cap, cd.tiles_x, cd.tiles_y, U(L.colp0),
                                  U(L.colnb), U(L.colbb), misc, pair_count);
  GS_CHECK_LAUNCH();
  uint32_t* hist = U(L.hist);
  const int64_t nbm = L.nb_max;
  PairBlk* binfo = reinterpret_cast<PairBlk*>(ws + L.binfo);
  if (cap > 0) {
    k_block_info<<<div_up(nbm, 256), 256, 0, st>>>(cstart, rpos, U(L.colp0), U(L.colnb),
                                                   U(L.colbb), misc, cd.tiles_x, cd.tiles_y,
                                                   binfo);
    GS_CHECK_LAUNCH();
    GS_TIMED("bin_hist", st, k_pair_hist<<<(unsigned)nbm, kPairThreads, 0, st>>>(
                                 binfo, rpos, rl[cur], misc, cd.tiles_y, hist));
    GS_CHECK_LAUNCH();
    s = scan_u32(hist, hist, (int64_t)cd.tiles_y * nbm, nullptr, U(L.stmp), st, misc + kHistN);
    if (s != GS_OK) return s;
  }
  k_tile_ranges<<<div_up(n_tiles + 1, 256), 256, 0, st>>>(hist, U(L.colp0), U(L.colnb),
                                                           U(L.colbb), misc, cap, cd.tiles_x,
                                                           cd.tiles_y, ranges);
  GS_CHECK_LAUNCH();
  // 6. final positions
  if (cap > 0) {
    GS_TIMED("bin_scatter", st,
             (cd.tiles_y <= 128 ? k_pair_scatter<7> : k_pair_scatter<8>)<<<(unsigned)nbm,
                                                                           kPairThreads, 0, st>>>(
                 binfo, rpos, rl[cur], rg[cur], misc, hist, depth_keys, n, cap, cd.tiles_y, vals,
                 keys_out));
    GS_CHECK_LAUNCH();
  }
  return GS_OK;
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
