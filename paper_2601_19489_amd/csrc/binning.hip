// Binning and depth sort (Sec. 2.1): every Gaussian writes one pair per tile
// of its compact tile set; pairs end up ordered by (tile id, depth bits,
// Gaussian index).
//
// Instead of sorting P pairs on a 64-bit (tile | depth) key, the N Gaussians
// are first sorted by depth (32-bit keys, stable, so equal depths keep index
// order); pairs are then emitted in that depth order and sorted stably by
// tile id alone, which needs ceil(log2(n_tiles) / 8) passes over the pairs
// instead of ceil((32 + log2(n_tiles)) / 8). The result is the same order.
#include <algorithm>

#include "common.h"
#include "sort.h"

namespace gs {

namespace {

constexpr int64_t kAlign = 256;

inline int64_t al(int64_t b) { return (b + kAlign - 1) / kAlign * kAlign; }

struct BinLayout {
  int64_t dkA, dkB, dvA, dvB, cnt, off, pk0, pk1, pv0, pv1, rtmp, stmp, total;
};

BinLayout layout(int64_t n, int64_t cap) {
  BinLayout L;
  int64_t o = 0;
  const int64_t nw = al(4 * std::max<int64_t>(n, 1));
  const int64_t cw = al(4 * std::max<int64_t>(cap, 1));
  L.dkA = o; o += nw;
  L.dkB = o; o += nw;
  L.dvA = o; o += nw;
  L.dvB = o; o += nw;
  L.cnt = o; o += nw;
  L.off = o; o += nw;
  L.pk0 = o; o += cw;
  L.pk1 = o; o += cw;
  L.pv0 = o; o += cw;
  L.pv1 = o; o += cw;
  L.rtmp = o; o += al(4 * radix_tmp_words(std::max(n, cap)));
  L.stmp = o; o += al(4 * (scan_tmp_words(n) + 1));
  L.total = o;
  return L;
}

__global__ void k_iota(uint32_t* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = (uint32_t)i;
}

__global__ void k_gather_counts(const uint32_t* __restrict__ ids,
                                const uint32_t* __restrict__ counts, uint32_t* __restrict__ out,
                                int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = ids[i] < (uint64_t)n ? counts[ids[i]] : 0u;
}

// One thread per Gaussian in depth order writes its tiles (column walk, same
// FP64 arithmetic as the count in preprocess) at its scanned offset.
__global__ void __launch_bounds__(256) k_emit(const uint32_t* __restrict__ ids,
                                              const uint32_t* __restrict__ cnt,
                                              const uint32_t* __restrict__ off,
                                              const float* __restrict__ splats, int64_t n,
                                              CamDev cam, int64_t cap,
                                              const uint32_t* __restrict__ P_dev,
                                              uint32_t* __restrict__ pk, uint32_t* __restrict__ pv) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const uint32_t c = cnt[r];
  if (c == 0) return;
  if ((int64_t)*P_dev > cap) return;
  const uint32_t g = ids[r];
  if ((int64_t)g >= n) return;
  const int64_t o = off[r];
  const float4* rec = reinterpret_cast<const float4*>(splats + (int64_t)g * GS_SPLAT_FLOATS);
  const float4 r0 = rec[0], r1 = rec[1];
  Snug s;
  if (!snug_setup(r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, s)) return;
  int tx0, tx1;
  snug_columns(s, cam.tile, cam.tiles_x, tx0, tx1);
  uint32_t k = 0;
  for (int tx = tx0; tx <= tx1 && k < c; ++tx) {
    int ty0, ty1;
    snug_rows(s, tx, cam.tile, cam.tiles_y, ty0, ty1);
    for (int ty = ty0; ty <= ty1 && k < c; ++ty, ++k) {
      pk[o + k] = (uint32_t)(ty * cam.tiles_x + tx);
      pv[o + k] = g;
    }
  }
}

// ranges[t] = first sorted position with tile >= t, for t in [0, n_tiles].
__global__ void k_ranges(const uint32_t* __restrict__ keys, const uint32_t* __restrict__ P_dev,
                         int64_t cap, int n_tiles, uint32_t* __restrict__ ranges) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t P = *P_dev;
  const int64_t Pe = (int64_t)P <= cap ? (int64_t)P : 0;
  if (i > Pe) return;
  const auto tile_at = [&](int64_t j) -> int64_t {
    const uint32_t k = keys[j];
    return k < (uint32_t)n_tiles ? (int64_t)k : (int64_t)n_tiles - 1;
  };
  if (i < Pe) {
    const int64_t k = tile_at(i);
    const int64_t kp = i ? tile_at(i - 1) : -1;
    for (int64_t t = kp + 1; t <= k; ++t) ranges[t] = (uint32_t)i;
  } else {
    const int64_t kl = Pe ? tile_at(Pe - 1) : -1;
    for (int64_t t = kl + 1; t <= n_tiles; ++t) ranges[t] = (uint32_t)Pe;
  }
}

__global__ void k_keys_out(const uint32_t* __restrict__ tiles, const uint32_t* __restrict__ vals,
                           const uint32_t* __restrict__ depth_keys,
                           const uint32_t* __restrict__ P_dev, int64_t cap, int64_t n,
                           uint64_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t P = *P_dev;
  if ((int64_t)P > cap || i >= (int64_t)P) return;
  const uint32_t g = vals[i];
  out[i] = ((uint64_t)tiles[i] << 32) | (uint64_t)((int64_t)g < n ? depth_keys[g] : 0xFFFFFFFFu);
}

}  // namespace

}  // namespace gs

using namespace gs;

extern "C" gs_status gs_bin_sort_workspace(int64_t n, int64_t capacity, size_t* bytes) {
  if (n < 0 || capacity < 0 || capacity > 0xFFFFFFFELL || !bytes) return GS_EINVAL;
  *bytes = (size_t)layout(n, capacity).total;
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
  if (!ranges || !pair_count || (n > 0 && (!splats || !depth_keys || !tile_counts)) ||
      (capacity > 0 && !vals) || !workspace)
    return GS_EINVAL;
  const BinLayout L = layout(n, capacity);
  if ((int64_t)workspace_bytes < L.total) return GS_ECAPACITY;
  hipStream_t st = (hipStream_t)stream;
  char* ws = (char*)workspace;
  auto U = [&](int64_t off) { return reinterpret_cast<uint32_t*>(ws + off); };
  const int n_tiles = cd.tiles_x * cd.tiles_y;
  gs_status s;

  // 1. stable depth sort of the Gaussians (keys: FP32 depth bits; Gaussians
  //    without tiles carry 0xFFFFFFFF and land at the end with count 0)
  if (n > 0) {
    k_iota<<<div_up(n, 256), 256, 0, st>>>(U(L.dvA), n);
    GS_CHECK_LAUNCH();
    const uint32_t* kin = depth_keys;
    uint32_t *kA = U(L.dkA), *kB = U(L.dkB), *vA = U(L.dvA), *vB = U(L.dvB);
    for (int pass = 0; pass < 4; ++pass) {
      const bool even = (pass % 2) == 0;
      s = radix_pass(kin, even ? vA : vB, even ? kB : kA, even ? vB : vA, n, nullptr, pass * 8,
                     U(L.rtmp), st);
      if (s != GS_OK) return s;
      kin = even ? kB : kA;
    }
    // 2. tile counts in depth order, exclusive scan -> offsets and P
    k_gather_counts<<<div_up(n, 256), 256, 0, st>>>(U(L.dvA), tile_counts, U(L.cnt), n);
    GS_CHECK_LAUNCH();
  }
  s = scan_u32(U(L.cnt), U(L.off), n, pair_count, U(L.stmp), st);
  if (s != GS_OK) return s;
  if (capacity == 0) {
    k_ranges<<<1, 1, 0, st>>>(U(L.pk0), pair_count, 0, n_tiles, ranges);
    GS_CHECK_LAUNCH();
    return GS_OK;
  }
  // 3. emit (tile, Gaussian) pairs in depth order
  if (n > 0) {
    GS_TIMED("bin_emit", st, k_emit<<<div_up(n, 256), 256, 0, st>>>(U(L.dvA), U(L.cnt), U(L.off), splats, n, cd, capacity,
                                           pair_count, U(L.pk0), U(L.pv0)));
    GS_CHECK_LAUNCH();
  }
  // 4. stable LSD sort of the pairs by tile id
  int bits = 1;
  while ((1 << bits) < n_tiles) ++bits;
  const int passes = (bits + 7) / 8;
  uint32_t* kbuf[2] = {U(L.pk0), U(L.pk1)};
  uint32_t* vbuf[2] = {U(L.pv0), U(L.pv1)};
  int cur = 0;
  for (int pass = 0; pass < passes; ++pass) {
    const bool last = pass == passes - 1;
    s = radix_pass(kbuf[cur], vbuf[cur], kbuf[cur ^ 1], last ? vals : vbuf[cur ^ 1], capacity,
                   pair_count, pass * 8, U(L.rtmp), st);
    if (s != GS_OK) return s;
    cur ^= 1;
  }
  // 5. per-tile ranges and optional 64-bit keys
  k_ranges<<<div_up(capacity + 1, 256), 256, 0, st>>>(kbuf[cur], pair_count, capacity, n_tiles,
                                                       ranges);
  GS_CHECK_LAUNCH();
  if (keys_out) {
    k_keys_out<<<div_up(capacity, 256), 256, 0, st>>>(kbuf[cur], vals, depth_keys, pair_count,
                                                       capacity, n, keys_out);
    GS_CHECK_LAUNCH();
  }
  return GS_OK;
}
