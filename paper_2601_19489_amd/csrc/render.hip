// Per-tile compositing (Sec. 2.1, second step) and its backward (Sec. 2.2).
//
// Forward: one workgroup per tile; each lane owns PX pixels. The tile's
// sorted splat records are gathered through `vals` into LDS in batches;
// every pixel walks the batch front to back. The workgroup stops as soon as
// every pixel has reached T < 1e-4.
//
// Backward: one workgroup per tile, PX pixels per lane, walking the tile's
// list back to front from each pixel's last contributor. The transmittance
// in front of each splat is recomputed as T / (1 - alpha) from the stored
// final transmittance (nothing per splat is stored by the forward), and the
// colour and depth behind it are accumulated on the way. The per-splat
// gradient components are summed over each row of 16 lanes with DPP, the
// rows' sums are parked in LDS, and after each batch one FP64 atomic add per
// (splat, component) carries the tile's total.
//
// The FP32 arithmetic here may be contracted to FMAs; alpha is computed by
// the same expression (explicit fmaf) in both kernels, so the backward
// replays exactly the forward's alphas.
#include <math.h>

#include "binning.h"
#include "common.h"
#include "sort.h"

namespace gs {

constexpr float kAlphaMax = 0.99f;
constexpr float kTStop = 1e-4f;
constexpr float kNegHalfLog2e = -0.72134752044448170f;  // -log2(e) / 2

// G = exp(-Q/2) as one v_exp_f32
__device__ __forceinline__ float gauss(float Q) {
  return __builtin_amdgcn_exp2f(Q * kNegHalfLog2e);
}

struct SplatQ {
  float Q, mag, dx, dy;
};

__device__ __forceinline__ SplatQ eval_q(float px, float py, float u, float v, float a, float b2,
                                         float c) {
  SplatQ r;
  r.dx = px - u;
  r.dy = py - v;
  const float s1 = a * r.dx;
  const float t1 = c * r.dy;
  const float td = t1 * r.dy;
  r.Q = fmaf(r.dx, fmaf(b2, r.dy, s1), td);
  r.mag = fmaf(s1, r.dx, td);
  return r;
}

__device__ __attribute__((noinline)) bool splat_skips_exact(float t, float px, float py, float u,
                                                            float v, float a, float b, float c) {
#pragma clang fp contract(off)
  const double dx = (double)px - (double)u;
  const double dy = (double)py - (double)v;
  const double q = dx * ((double)a * dx + 2.0 * ((double)b * dy)) + dy * ((double)c * dy);
  return q > (double)t;
}

// One front-to-back step of the forward at one pixel: skip (alpha < 1/255,
// decided as Q > t), stop (the blend would take T below 1e-4) or blend with
// alpha `al` and new transmittance `Tn`, from a splat staged as (u, v, a,
// 2 b), (c, t, o, skip band). Used by the Eq. (4) replay of the forward's
// decisions.
constexpr int kSkip = 0, kBlend = 1, kStop = 2;
__device__ __forceinline__ int fwd_step(float px, float py, float4 a0, float4 a1, float T,
                                        float& al, float& Tn) {
#pragma clang fp contract(fast)
  const SplatQ q = eval_q(px, py, a0.x, a0.y, a0.z, a0.w, a1.x);
  if (splat_skips_band(q.Q, a1.w, a1.y, px, py, a0.x, a0.y, a0.z, 0.5f * a0.w, a1.x))
    return kSkip;
  al = fminf(kAlphaMax, a1.z * gauss(q.Q));
  Tn = T * (1.f - al);
  return Tn < kTStop ? kStop : kBlend;
}

constexpr int kFwdBatch = 256;  // splats per LDS batch in the forward (default)
template <int NB>
struct FwdLdsT {
  float4 s0[NB], s1[NB], s2[NB];
};
using FwdLds = FwdLdsT<kFwdBatch>;

// The forward that writes its tile lists (from the binning's column runs):
// the batch's Gaussian ids and the block-scan words.
template <int NB, int NTH>
struct DefLds {
  static constexpr int R = 2;  // runs per thread per scan step
  uint32_t sid[NB];
  uint32_t wcnt[2][R][NTH / kWave];  // per-wavefront counts, double-buffered by step
  uint32_t next;
};

// Where a tile's list continues in the column runs: segment `seg` (global
// index), its next run r and run end r1, and the next list position pos.
// The column's segments sf .. se - 1 and runs c0 .. c1 - 1; a window of NTH
// segments from wb on, thread t holding the first list position in row ty
// of segment wb + t (hs; 0xFFFFFFFF past se).
struct DefCursor {
  uint32_t seg, r, r1, pos;
  uint32_t sf, se, c0, c1, wb, hs;
};

__device__ __forceinline__ void def_window(const RunLists& rl, DefCursor& c, int tiles_y, int ty) {
  const uint32_t s = c.wb + threadIdx.x;
  c.hs = s < c.se ? rl.hist[(int64_t)s * tiles_y + ty] : 0xFFFFFFFFu;
}

// Point the cursor at the segment holding list position pos of row ty: the
// last one whose first position in the row is at most pos (a segment with
// no entry in the row shares its first position with the next one), found
// with one block count over the window (moved on when the whole window lies
// at or below pos). se if that is below min_seg (the seek always moves
// forward), which happens only on a list that the run tables do not hold
// (never for tables of the same binning).
template <int NTH>
__device__ __forceinline__ void def_seek(const RunLists& rl, DefCursor& c, int tiles_y, int ty,
                                         uint32_t pos, uint32_t min_seg) {
  uint32_t seg;
  for (;;) {
    const uint32_t k = __builtin_amdgcn_readfirstlane(
        (uint32_t)__syncthreads_count(c.hs <= pos));  // leading segments (monotone)
    if (k == (uint32_t)NTH && c.wb + NTH < c.se) {
      c.wb += NTH;
      def_window(rl, c, tiles_y, ty);
      continue;
    }
    seg = k > 0 && c.wb + k - 1 >= min_seg ? c.wb + k - 1 : c.se;
    break;
  }
  c.seg = seg;
  c.pos = pos;
  if (seg < c.se) {
    c.r = c.c0 + (seg - c.sf) * (uint32_t)kSegRuns;
    c.r1 = min(c.r + (uint32_t)kSegRuns, c.c1);
  } else {
    c.r = c.r1 = 0;
  }
}

// The cursor of a tile (column tx, row ty) at its first list position.
template <int NTH>
__device__ __forceinline__ void def_start(const RunLists& rl, DefCursor& c, int tx, int tiles_y,
                                          int ty, uint32_t start) {
  c.sf = rl.segfirst[tx];
  c.se = rl.segfirst[tx + 1];
  c.c0 = rl.cstart[tx];
  c.c1 = rl.cstart[tx + 1];
  c.wb = c.sf;
  def_window(rl, c, tiles_y, ty);
  def_seek<NTH>(rl, c, tiles_y, ty, start, c.sf);
}

// The next cnt entries of the tile's list (row ty of column tx): the runs
// from the cursor on that cover row ty, in run order (= list order), into
// L.sid[0 .. cnt) and vals[c.pos ..]. Each step scans R NTH runs (run
// c.r + k NTH + t in slot k of thread t) with one barrier: the per-wavefront
// counts alternate between two buffers, so a step's counts are not
// overwritten before every thread has read them. A run left over when the
// batch fills is taken by the next batch. Entries that the tables do not
// hold (never for tables of the same binning) get the id 0xFFFFFFFF, an
// absent splat.
template <int NB, int NTH>
__device__ __forceinline__ void def_fill(const RunLists& rl, DefLds<NB, NTH>& D, DefCursor& c,
                                         int tx, int tiles_y, int ty, int cnt,
                                         uint32_t* __restrict__ vals) {
  constexpr int R = DefLds<NB, NTH>::R, NW = NTH / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  int filled = 0, buf = 0;
  bool full = false;
  while (filled < cnt) {
    if (c.r >= c.r1) {  // segment used up: the one holding the next position
      if (c.seg >= c.se) break;
      def_seek<NTH>(rl, c, tiles_y, ty, c.pos, c.seg + 1);
      if (c.seg >= c.se) break;
    }
    bool cov[R];
    uint32_t gid[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {  // loads first
      const uint32_t rr = c.r + k * NTH + threadIdx.x;
      const uint2 q = rr < c.r1 ? rl.runs[rr] : make_uint2(0u, 0u);
      gid[k] = q.x;
      cov[k] = (uint32_t)ty - (q.y & 0xFFFFu) < (q.y >> 16);
    }
    uint64_t bal[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
      bal[k] = __ballot(cov[k]);
      if (lane == 0) D.wcnt[buf][k][w] = (uint32_t)__popcll(bal[k]);
    }
    __syncthreads();
    // the counts are uniform (per block, and below w per wavefront): scalar
    uint32_t total = 0, rank[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
      uint32_t before = 0, tk = 0;
#pragma unroll
      for (int v = 0; v < NW; ++v) {
        const uint32_t x = __builtin_amdgcn_readfirstlane(D.wcnt[buf][k][v]);
        before += v < w ? x : 0u;
        tk += x;
      }
      rank[k] = total + before +
                __builtin_amdgcn_mbcnt_hi((uint32_t)(bal[k] >> 32),
                                          __builtin_amdgcn_mbcnt_lo((uint32_t)bal[k], 0u));
      total += tk;
    }
    const uint32_t need = (uint32_t)(cnt - filled);
    const uint32_t take = min(total, need);
#pragma unroll
    for (int k = 0; k < R; ++k) {
      if (cov[k] && rank[k] < take) {
        D.sid[filled + (int)rank[k]] = gid[k];
        vals[c.pos + rank[k]] = gid[k];
      }
      if (cov[k] && rank[k] == take) D.next = (uint32_t)(k * NTH) + threadIdx.x;  // first not taken
    }
    c.pos += take;
    filled += (int)take;
    buf ^= 1;
    if (total > need) {
      full = true;
      break;
    }
    c.r = min(c.r + (uint32_t)(R * NTH), c.r1);
  }
  for (int q = filled + (int)threadIdx.x; q < cnt; q += NTH) D.sid[q] = 0xFFFFFFFFu;
  __syncthreads();
  if (full) c.r += __builtin_amdgcn_readfirstlane(D.next);
}

// Checkpoints of the per-splat backward (the design the paper adopts): the
// forward state (T, C0, C1, C2, D) of every pixel before list positions 0,
// 32, 64, ..., laid out [tile][bucket][5][TILE * TILE].
constexpr int kCkptInterval = 32;
constexpr int kCkptVals = 5;

// Forward of one tile (column-major id `tile`) by the whole workgroup; with
// CKPT it also writes the checkpoints of the pixels still compositing at
// each interval boundary below nbk buckets, and sets *ovf if a pixel blends
// a splat at a list position of bucket nbk or later.
// With DEF the lists come from the binning's run tables `rl` (deferred
// binning) and the forward writes each batch's entries to `dvals` (vals is
// not read): every list position up to the last one staged, which covers
// every pixel's n_contrib.
template <int TILE, int PX, bool CKPT = false, int NB = kFwdBatch, bool DEF = false>
__device__ __forceinline__ void fwd_tile(FwdLdsT<NB>& L, int tile,
                                         const float* __restrict__ splats,
                                         const uint32_t* __restrict__ vals,
                                         const uint32_t* __restrict__ ranges, int64_t n, int W,
                                         int H, int tiles_y, float bg0, float bg1, float bg2,
                                         float* __restrict__ image, float* __restrict__ depth,
                                         float* __restrict__ T_final,
                                         uint32_t* __restrict__ n_contrib,
                                         float* __restrict__ ckpt = nullptr, int nbk = 0,
                                         uint32_t* __restrict__ ovf = nullptr,
                                         DefLds<NB, TILE * TILE / PX>* DL = nullptr,
                                         RunLists rl = {}, uint32_t* __restrict__ dvals = nullptr) {
#pragma clang fp contract(fast)
  constexpr int NTH = TILE * TILE / PX;
  float4* s0 = L.s0;
  float4* s1 = L.s1;
  float4* s2 = L.s2;
  const int tx = tile / tiles_y, ty = tile % tiles_y;
  const uint32_t start = ranges[tile], end = ranges[tile + 1];
  float px[PX], py[PX], T[PX], C0[PX], C1[PX], C2[PX], D[PX];
  uint32_t last[PX];  // one past the list position of the last blended splat
  bool done[PX];
  bool alldone = true;
#pragma unroll
  for (int j = 0; j < PX; ++j) {
    const int pi = threadIdx.x + j * NTH;
    const int x = tx * TILE + pi % TILE, y = ty * TILE + pi / TILE;
    px[j] = (float)x + 0.5f;
    py[j] = (float)y + 0.5f;
    T[j] = 1.f; C0[j] = C1[j] = C2[j] = D[j] = 0.f; last[j] = 0;
    done[j] = !(x < W && y < H);
    alldone &= done[j];
  }
  DefCursor cur{};
  if constexpr (DEF) {
    if (start < end) def_start<NTH>(rl, cur, tx, tiles_y, ty, start);
  }
  for (uint32_t b = start; b < end; b += NB) {
    if (__syncthreads_count(!alldone) == 0) break;
    const int cnt = (int)min((uint32_t)NB, end - b);
    if constexpr (DEF) def_fill<NB, NTH>(rl, *DL, cur, tx, tiles_y, ty, cnt, dvals);
    for (int q = threadIdx.x; q < cnt; q += NTH) {
      uint32_t g;
      if constexpr (DEF) g = DL->sid[q]; else g = vals[b + q];
      if ((int64_t)g < n) {
        const float4* r = reinterpret_cast<const float4*>(splats + (size_t)g * GS_SPLAT_FLOATS);
        // staged as (u, v, a, 2 b), (c, t, o, z), (r, g, b, skip band)
        float4 r0 = r[0];
        const float4 r1 = r[1];
        float4 r2 = r[2];
        r2.w = skip_band(r0.z, r0.w, r1.x, r1.y);
        r0.w = r0.w + r0.w;  // exact
        s0[q] = r0;
        s1[q] = r1;
        s2[q] = r2;
      } else {  // never for a correct list: an empty splat (t < 0 skips it)
        s0[q] = make_float4(0.f, 0.f, 1.f, 0.f);
        s1[q] = make_float4(1.f, -1.f, 0.f, 0.f);
        s2[q] = make_float4(0.f, 0.f, 0.f, 0.f);
      }
    }
    __syncthreads();
    for (int k = 0; k < cnt && !alldone; ++k) {
      const float4 a0 = s0[k], a1 = s1[k];
      const float4 a2 = s2[k];
      const float b2 = a0.w;
      if (CKPT) {
        const uint32_t pos = b + (uint32_t)k - start;
        if ((pos % kCkptInterval) == 0) {
          const uint32_t bk = pos / kCkptInterval;
#pragma unroll
          for (int j = 0; j < PX; ++j) {
            if (done[j] || bk >= (uint32_t)nbk) continue;
            constexpr int NP = TILE * TILE;
            float* c = ckpt + ((size_t)tile * nbk + bk) * kCkptVals * NP + threadIdx.x + j * NTH;
            c[0] = T[j];
            c[NP] = C0[j];
            c[2 * NP] = C1[j];
            c[3 * NP] = C2[j];
            c[4 * NP] = D[j];
          }
        }
      }
      // the step in select form: every pixel runs it, and a skipped, stopped
      // or finished pixel changes nothing (the same decisions as fwd_step,
      // without divergent branches)
      alldone = true;
      const uint32_t posn = b + (uint32_t)k - start + 1u;
#pragma unroll
      for (int j = 0; j < PX; ++j) {
        const SplatQ q = eval_q(px[j], py[j], a0.x, a0.y, a0.z, b2, a1.x);
        const bool live = !done[j] && !splat_skips_band(q.Q, a2.w, a1.y, px[j], py[j], a0.x,
                                                        a0.y, a0.z, 0.5f * b2, a1.x);
        const float al = fminf(kAlphaMax, a1.z * gauss(q.Q));
        const float Tn = T[j] * (1.f - al);
        const bool stop = live && Tn < kTStop;
        const bool blend = live && !stop;
        // weight 0 when not blending: adding c * 0 leaves the sums unchanged
        const float w = blend ? al * T[j] : 0.f;
        C0[j] = fmaf(a2.x, w, C0[j]);
        C1[j] = fmaf(a2.y, w, C1[j]);
        C2[j] = fmaf(a2.z, w, C2[j]);
        D[j] = fmaf(a1.w, w, D[j]);
        T[j] = blend ? Tn : T[j];
        last[j] = blend ? posn : last[j];
        done[j] = done[j] || stop;
        // a blend in a bucket without a checkpoint: the backward would need it
        if (CKPT && blend && posn > (uint32_t)nbk * kCkptInterval) atomicOr(ovf, 1u);
        alldone &= done[j];
      }
    }
  }
  const size_t HW = (size_t)H * W;
#pragma unroll
  for (int j = 0; j < PX; ++j) {
    const int pi = threadIdx.x + j * NTH;
    const int x = tx * TILE + pi % TILE, y = ty * TILE + pi / TILE;
    if (x < W && y < H) {
      const size_t p = (size_t)y * W + x;
      image[p] = fmaf(T[j], bg0, C0[j]);
      image[HW + p] = fmaf(T[j], bg1, C1[j]);
      image[2 * HW + p] = fmaf(T[j], bg2, C2[j]);
      depth[p] = D[j];
      T_final[p] = T[j];
      n_contrib[p] = last[j];
    }
  }
}

template <int TILE, int PX>
__global__ void __launch_bounds__(TILE* TILE / PX) k_render_fwd(
    const float* __restrict__ splats, const uint32_t* __restrict__ vals,
    const uint32_t* __restrict__ ranges, int64_t n, int W, int H, int tiles_y, float bg0,
    float bg1, float bg2, float* __restrict__ image, float* __restrict__ depth,
    float* __restrict__ T_final, uint32_t* __restrict__ n_contrib) {
  __shared__ FwdLds L;
  fwd_tile<TILE, PX>(L, blockIdx.x, splats, vals, ranges, n, W, H, tiles_y, bg0, bg1, bg2, image,
                     depth, T_final, n_contrib);
}

template <int TILE, int PX>
__global__ void __launch_bounds__(TILE* TILE / PX) k_render_fwd_def(
    const float* __restrict__ splats, RunLists rl, uint32_t* __restrict__ vals,
    const uint32_t* __restrict__ ranges, int64_t n, int W, int H, int tiles_y, float bg0,
    float bg1, float bg2, float* __restrict__ image, float* __restrict__ depth,
    float* __restrict__ T_final, uint32_t* __restrict__ n_contrib) {
  __shared__ FwdLds L;
  __shared__ DefLds<kFwdBatch, TILE * TILE / PX> DL;
  fwd_tile<TILE, PX, false, kFwdBatch, true>(L, blockIdx.x, splats, nullptr, ranges, n, W, H,
                                             tiles_y, bg0, bg1, bg2, image, depth, T_final,
                                             n_contrib, nullptr, 0, nullptr, &DL, rl, vals);
}

__global__ void __launch_bounds__(256) k_render_fwd_ckpt(
    const float* __restrict__ splats, const uint32_t* __restrict__ vals,
    const uint32_t* __restrict__ ranges, int64_t n, int W, int H, int tiles_y, float bg0,
    float bg1, float bg2, float* __restrict__ image, float* __restrict__ depth,
    float* __restrict__ T_final, uint32_t* __restrict__ n_contrib, float* __restrict__ ckpt,
    int nbk, uint32_t* __restrict__ ovf) {
  __shared__ FwdLds L;
  fwd_tile<16, 1, true>(L, blockIdx.x, splats, vals, ranges, n, W, H, tiles_y, bg0, bg1, bg2,
                        image, depth, T_final, n_contrib, ckpt, nbk, ovf);
}

// Inclusive scans over each half (32 lanes) of the wavefront with DPP: row
// shifts within 16-lane rows, then row 0 (2) carried into row 1 (3).
__device__ __forceinline__ float half_incl_sum(float x) {
  x += dpp_mov<0x111>(0.f, x);
  x += dpp_mov<0x112>(0.f, x);
  x += dpp_mov<0x114>(0.f, x);
  x += dpp_mov<0x118>(0.f, x);
  x += dpp_mov<0x142, 0xa>(0.f, x);
  return x;
}
__device__ __forceinline__ float half_incl_prod(float x) {
  x *= dpp_mov<0x111>(1.f, x);
  x *= dpp_mov<0x112>(1.f, x);
  x *= dpp_mov<0x114>(1.f, x);
  x *= dpp_mov<0x118>(1.f, x);
  x *= dpp_mov<0x142, 0xa>(1.f, x);
  return x;
}
// the value of the next lower lane of the half (1 for its first lane)
__device__ __forceinline__ float half_shift_prod(float x, int lane) {
  const float y = dpp_mov<0x138>(1.f, x);  // wave_shr:1
  return (lane & 31) ? y : 1.f;
}

// Per-splat backward with checkpoints (the paper's design, as an ablation of
// the pixel-parallel backward below): one workgroup per 16 x 16 tile; each
// wavefront takes buckets of 32 list positions, one splat per lane of each
// half, and walks the tile's pixels two at a time (one per half). A lane
// rebuilds the transmittance in front of its splat from the bucket's
// checkpoint and the product of (1 - alpha) over the lower lanes, and the
// colour behind it from the image minus the checkpoint colour and the
// blended colour of the lanes up to it (DPP scans), and accumulates its
// splat's gradient over all pixels in registers (as moments for the conic
// and centroid); the halves are combined and each (splat, tile) gets one
// atomic per component.
template <bool DEPTH>
__global__ void __launch_bounds__(256) k_render_bwd_ckpt(
    const float* __restrict__ splats, const uint32_t* __restrict__ vals,
    const uint32_t* __restrict__ ranges, int W, int H, int tiles_y,
    const float* __restrict__ image, const float* __restrict__ depth,
    const uint32_t* __restrict__ n_contrib, const float* __restrict__ ckpt, int nbk,
    const float* __restrict__ dL_dimage, const float* __restrict__ dL_ddepth,
    double* __restrict__ grad2d, int64_t n) {
#pragma clang fp contract(fast)
  constexpr int TILE = 16, NP = TILE * TILE;
  __shared__ float pim[3][NP], pdc[3][NP], pdep[NP], pdd[NP];
  __shared__ uint32_t pnc[NP];
  __shared__ uint32_t smax;
  const int tile = blockIdx.x;
  const int tx = tile / tiles_y, ty = tile % tiles_y;
  const uint32_t start = ranges[tile], end = ranges[tile + 1];
  const size_t HW = (size_t)H * W;
  {
    const int t = threadIdx.x;
    const int x = tx * TILE + t % TILE, y = ty * TILE + t / TILE;
    const bool in = x < W && y < H;
    const size_t p = (size_t)y * W + x;
    pnc[t] = in ? n_contrib[p] : 0u;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      pim[c][t] = in ? image[c * HW + p] : 0.f;
      pdc[c][t] = in ? dL_dimage[c * HW + p] : 0.f;
    }
    pdep[t] = (DEPTH && in) ? depth[p] : 0.f;
    pdd[t] = (DEPTH && in && dL_ddepth) ? dL_ddepth[p] : 0.f;
    if (t == 0) smax = 0;
    __syncthreads();
    if (pnc[t]) atomicMax(&smax, pnc[t]);
    __syncthreads();
  }
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  const int h = lane >> 5;
  const uint32_t nbt = (smax + kCkptInterval - 1) / kCkptInterval;
  for (uint32_t b = (uint32_t)w; b < nbt; b += 256 / kWave) {
    const uint32_t pos = b * kCkptInterval + (uint32_t)(lane & 31);
    const bool has = pos < smax && start + pos < end;
    uint32_t g = 0xFFFFFFFFu;
    float4 a0 = make_float4(0.f, 0.f, 1.f, 0.f), a1 = make_float4(1.f, -1.f, 0.f, 0.f);
    float4 a2 = make_float4(0.f, 0.f, 0.f, 0.f);
    if (has) {
      g = vals[start + pos];
      if ((int64_t)g < n) {
        const float4* r = reinterpret_cast<const float4*>(splats + (size_t)g * GS_SPLAT_FLOATS);
        a0 = r[0];
        a1 = r[1];
        a2 = r[2];
      }
    }
    const float b2 = a0.w + a0.w;
    float M00 = 0.f, Mx = 0.f, My = 0.f, Mxx = 0.f, Mxy = 0.f, Myy = 0.f;
    float gc0 = 0.f, gc1 = 0.f, gc2 = 0.f, gz = 0.f;
    for (int it = 0; it < NP / 2; ++it) {
      const int pi = 2 * it + h;
      const uint32_t nc = pnc[pi];
      float Tb = 0.f, Cb0 = 0.f, Cb1 = 0.f, Cb2 = 0.f, Db = 0.f;
      // the pixel composites in this bucket (and its checkpoint exists: a
      // caller's bucket count below the forward's need gives wrong values,
      // never an access outside the buffer)
      if (b * kCkptInterval < nc && b < (uint32_t)nbk) {
        const float* c = ckpt + ((size_t)tile * nbk + b) * kCkptVals * NP + pi;
        Tb = c[0];
        Cb0 = c[NP];
        Cb1 = c[2 * NP];
        Cb2 = c[3 * NP];
        if (DEPTH) Db = c[4 * NP];
      }
      const float pxf = (float)(tx * TILE + pi % TILE) + 0.5f;
      const float pyf = (float)(ty * TILE + pi / TILE) + 0.5f;
      const SplatQ q = eval_q(pxf, pyf, a0.x, a0.y, a0.z, b2, a1.x);
      const bool act = has && pos < nc &&
                       !splat_skips(q.Q, q.mag, a1.y, pxf, pyf, a0.x, a0.y, a0.z, a0.w, a1.x);
      const float G = act ? gauss(q.Q) : 0.f;
      const float oG = a1.z * G;
      const float al = fminf(kAlphaMax, oG);
      const float om = 1.f - al;
      const float Ti = Tb * half_shift_prod(half_incl_prod(om), lane);
      const float wgt = al * Ti;
      const float C0i = Cb0 + half_incl_sum(a2.x * wgt);
      const float C1i = Cb1 + half_incl_sum(a2.y * wgt);
      const float C2i = Cb2 + half_incl_sum(a2.z * wgt);
      const float rinv = __builtin_amdgcn_rcpf(om);
      const float d0 = pdc[0][pi], d1 = pdc[1][pi], d2 = pdc[2][pi];
      // colour (with background) behind the splat = image - blended up to it
      float acc = d0 * (Ti * a2.x - (pim[0][pi] - C0i) * rinv) +
                  d1 * (Ti * a2.y - (pim[1][pi] - C1i) * rinv) +
                  d2 * (Ti * a2.z - (pim[2][pi] - C2i) * rinv);
      gc0 += d0 * wgt;
      gc1 += d1 * wgt;
      gc2 += d2 * wgt;
      if (DEPTH) {
        const float Di = Db + half_incl_sum(a1.w * wgt);
        const float dd = pdd[pi];
        acc += dd * (Ti * a1.w - (pdep[pi] - Di) * rinv);
        gz += dd * wgt;
      }
      const float tg = (act && oG <= kAlphaMax) ? acc * G : 0.f;
      const float tx_ = tg * q.dx, ty_ = tg * q.dy;
      M00 += tg;
      Mx += tx_;
      My += ty_;
      Mxx = fmaf(tx_, q.dx, Mxx);
      Mxy = fmaf(tx_, q.dy, Mxy);
      Myy = fmaf(ty_, q.dy, Myy);
    }
    float v[10] = {M00, Mx, My, Mxx, Mxy, Myy, gc0, gc1, gc2, gz};
#pragma unroll
    for (int c = 0; c < 10; ++c) v[c] += __shfl_xor(v[c], 32, kWave);
    // lanes l and l + 32 now hold the same sums for splat l & 31
    constexpr int NC = GS_GRAD2D_COMPONENTS;
    const float o = a1.z, a = a0.z, bb = a0.w, cc = a1.x;
    float out[NC];
    out[0] = o * (a * v[1] + bb * v[2]);
    out[1] = o * (bb * v[1] + cc * v[2]);
    out[2] = -0.5f * o * v[3];
    out[3] = -o * v[4];
    out[4] = -0.5f * o * v[5];
    out[5] = v[0];
    out[6] = v[6];
    out[7] = v[7];
    out[8] = v[8];
    out[9] = v[9];
    const uint32_t gv = (has && (int64_t)g < n) ? g : 0xFFFFFFFFu;
    // one lane per (splat, component), so that an instruction's atomic adds
    // fall in the consecutive records of a few splats; the values come from
    // the splat's lane by wave shuffles
#pragma unroll
    for (int r = 0; r < 32 * NC / kWave; ++r) {
      const int e = r * kWave + lane, sl = e / NC, c = e - NC * sl;
      float val = 0.f;
#pragma unroll
      for (int k = 0; k < NC; ++k) {
        const float t = __shfl(out[k], sl, kWave);
        if (k == c) val = t;
      }
      const uint32_t gs = (uint32_t)__shfl((int)gv, sl, kWave);
      if (gs != 0xFFFFFFFFu && val != 0.f)
        unsafeAtomicAdd(grad2d + (size_t)gs * NC + c, (double)val);
    }
  }
}

// Row sums of eight values by reduce-scatter over a row of 16 lanes: the
// values are halved between partner lanes three times (partners differ in
// lane bit 0, then bit 1, then by a rotation of 4, which flips bit 2) and
// the last partners (rotation by 8) are added. Lane l ends with the row sum
// of v[rs_slot(l)], rs_slot(l) = 4 (l & 1) + 2 ((l >> 1) & 1) + ((l >> 2) & 1),
// in 22 operations where eight all-reduces take 32. b0..b2 are lane bits
// 0..2 and every lane of the row must be active.
__device__ __forceinline__ float row_reduce_scatter8(const float* v, bool b0, bool b1, bool b2) {
  float r1[4], r2[2];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const float keep = b0 ? v[i + 4] : v[i], send = b0 ? v[i] : v[i + 4];
    r1[i] = keep + dpp_mov<0xB1>(0.f, send);  // partner lane ^ 1
  }
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const float keep = b1 ? r1[i + 2] : r1[i], send = b1 ? r1[i] : r1[i + 2];
    r2[i] = keep + dpp_mov<0x4E>(0.f, send);  // partner lane ^ 2
  }
  const float keep = b2 ? r2[1] : r2[0], send = b2 ? r2[0] : r2[1];
  const float r3 = keep + dpp_mov<0x124>(0.f, send);  // row_ror:4
  return r3 + dpp_mov<0x128>(0.f, r3);                 // row_ror:8
}

__host__ __device__ constexpr int rs_slot(int l) {
  return 4 * (l & 1) + 2 * ((l >> 1) & 1) + ((l >> 2) & 1);
}

// splats per LDS batch of the backward by default: 32 for one-wavefront
// workgroups (more of them fit on a compute unit), 64 otherwise (fewer
// barriers per splat)
template <int TILE, int PX>
constexpr int bwd_batch_default() { return TILE * TILE / PX <= 64 ? 32 : 64; }

template <int TILE, int PX, int NBV = bwd_batch_default<TILE, PX>()>
struct BwdLds {
  static constexpr int NR = TILE * TILE / PX / 16;  // rows of 16 lanes
  static constexpr int NB = NBV;
  float4 s0[NB], s1[NB], s2[NB];
  uint32_t sid[NB];
  float red[NR][GS_GRAD2D_COMPONENTS][NB];
  uint32_t smax;
};

// Backward of one tile (column-major id `tile`) by the whole workgroup.
template <int TILE, int PX, bool DEPTH, int NBV = bwd_batch_default<TILE, PX>()>
__device__ __forceinline__ void bwd_tile(BwdLds<TILE, PX, NBV>& L, int tile,
                                         const float* __restrict__ splats,
                                         const uint32_t* __restrict__ vals,
                                         const uint32_t* __restrict__ ranges, int W, int H,
                                         int tiles_y, float bg0, float bg1, float bg2,
                                         const float* __restrict__ T_final,
                                         const uint32_t* __restrict__ n_contrib,
                                         const float* __restrict__ dL_dimage,
                                         const float* __restrict__ dL_ddepth,
                                         double* __restrict__ grad2d, int64_t n) {
#pragma clang fp contract(fast)
  constexpr int NTH = TILE * TILE / PX;   // threads
  constexpr int NR = BwdLds<TILE, PX, NBV>::NR;
  constexpr int NB = BwdLds<TILE, PX, NBV>::NB;
  constexpr int NC = GS_GRAD2D_COMPONENTS;
  static_assert(NTH % kWave == 0, "whole wavefronts");
  float4* s0 = L.s0;
  float4* s1 = L.s1;
  float4* s2 = L.s2;
  uint32_t* sid = L.sid;
  auto& red = L.red;
  uint32_t& smax = L.smax;
  const int tx = tile / tiles_y, ty = tile % tiles_y;
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  const int row = wv * (kWave / 16) + lane / 16;
  // lanes 0..7 of a row store the reduce-scattered sums, lanes 8 and 9 the
  // sums of components 8 and 9
  const int l16 = lane & 15;
  const bool rb0 = l16 & 1, rb1 = l16 & 2, rb2 = l16 & 4;
  const int slot = l16 < 8 ? rs_slot(l16) : l16;
  const bool writer = l16 < (DEPTH ? 10 : 9);
  const uint32_t start = ranges[tile];
  const size_t HW = (size_t)H * W;
  float px[PX], py[PX], T[PX], dC0[PX], dC1[PX], dC2[PX], dD[PX];
  // U = dL/dC . (colour, depth) of everything behind the current splat
  // (background included): dL/dalpha (1 - alpha) = T (dL/dC . c) - U
  float U[PX];
  uint32_t nc[PX];
  uint32_t mymax = 0;
#pragma unroll
  for (int j = 0; j < PX; ++j) {
    const int pi = threadIdx.x + j * NTH;
    const int x = tx * TILE + pi % TILE, y = ty * TILE + pi / TILE;
    px[j] = (float)x + 0.5f;
    py[j] = (float)y + 0.5f;
    T[j] = 1.f; dC0[j] = dC1[j] = dC2[j] = dD[j] = 0.f; nc[j] = 0;
    if (x < W && y < H) {
      const size_t p = (size_t)y * W + x;
      T[j] = T_final[p];
      nc[j] = n_contrib[p];
      dC0[j] = dL_dimage[p];
      dC1[j] = dL_dimage[HW + p];
      dC2[j] = dL_dimage[2 * HW + p];
      if (DEPTH) dD[j] = dL_ddepth ? dL_ddepth[p] : 0.f;
    }
    U[j] = T[j] * (dC0[j] * bg0 + dC1[j] * bg1 + dC2[j] * bg2);  // background depth is 0
    mymax = max(mymax, nc[j]);
  }
  if (threadIdx.x == 0) smax = 0;
  __syncthreads();
  if (mymax) atomicMax(&smax, mymax);
  __syncthreads();
  const uint32_t last = start + smax;
  for (uint32_t bend = last; bend > start;) {
    const uint32_t bstart = bend - start > (uint32_t)NB ? bend - NB : start;
    const int cnt = (int)(bend - bstart);
    for (int q = threadIdx.x; q < cnt; q += NTH) {
      const uint32_t g = vals[bstart + q];
      if ((int64_t)g < n) {
        // staged as (u, v, a, b), (c, t, o, skip band), (r, g, b, z)
        const float4* r = reinterpret_cast<const float4*>(splats + (size_t)g * GS_SPLAT_FLOATS);
        const float4 r0 = r[0];
        float4 r1 = r[1], r2 = r[2];
        r2.w = r1.w;
        r1.w = skip_band(r0.z, r0.w, r1.x, r1.y);
        s0[q] = r0;
        s1[q] = r1;
        s2[q] = r2;
        sid[q] = g;
      } else {  // never for a correct list: an empty splat with no gradient target
        s0[q] = make_float4(0.f, 0.f, 1.f, 0.f);
        s1[q] = make_float4(1.f, -1.f, 0.f, 0.f);
        s2[q] = make_float4(0.f, 0.f, 0.f, 0.f);
        sid[q] = 0xFFFFFFFFu;
      }
    }
    __syncthreads();
    for (int k = cnt - 1; k >= 0; --k) {
      const uint32_t pos = bstart + (uint32_t)k - start;  // position in the tile list
      const float4 a0 = s0[k], a1 = s1[k];
      const float b2 = a0.w + a0.w;
      // the PX pixels of a lane share their column: dx and a dx are common
      const float ex = px[0] - a0.x;
      const float aex = a0.z * ex;
      float Qs[PX], ey[PX];
      bool any = false;
#pragma unroll
      for (int j = 0; j < PX; ++j) {
        ey[j] = py[j] - a0.y;
        const float t1 = a1.x * ey[j];
        const float td = t1 * ey[j];
        const float Q = fmaf(ex, fmaf(b2, ey[j], aex), td);  // same value as eval_q
        const bool act = pos < nc[j] && !splat_skips_band(Q, a1.w, a1.y, px[j], py[j], a0.x,
                                                          a0.y, a0.z, a0.w, a1.x);
        // an inactive pixel runs the same arithmetic with alpha = 0: no change
        Qs[j] = act ? Q : __builtin_huge_valf();
        any |= act;
      }
      float out = 0.f;
      if (__ballot(any) != 0) {
        float g[NC];
        const float4 a2 = s2[k];
        // sums over the lane's pixels of dL/dQ / (-o/2) and its ey, ey^2 moments
        float m0, m1, m2;  // set by the first pixel
#pragma unroll
        for (int j = 0; j < PX; ++j) {
          const float G = gauss(Qs[j]);
          const float oG = a1.z * G;
          const float al = fminf(kAlphaMax, oG);
          const float rinv = __builtin_amdgcn_rcpf(1.f - al);
          const float Tb = T[j] * rinv;  // transmittance in front of this splat
          const float w = al * Tb;
          float dcc = dC0[j] * a2.x + dC1[j] * a2.y + dC2[j] * a2.z;
          if (DEPTH) dcc += dD[j] * a2.w;
          const float dal = rinv * (T[j] * dcc - U[j]);
          const float tg = oG <= kAlphaMax ? dal * G : 0.f;  // no gradient through the clamp
          const float tey = tg * ey[j];
          if (j == 0) {
            g[6] = dC0[j] * w;
            g[7] = dC1[j] * w;
            g[8] = dC2[j] * w;
            if (DEPTH) g[9] = dD[j] * w;
            m0 = tg;
            m1 = tey;
            m2 = tey * ey[j];
          } else {
            g[6] = fmaf(dC0[j], w, g[6]);
            g[7] = fmaf(dC1[j], w, g[7]);
            g[8] = fmaf(dC2[j], w, g[8]);
            if (DEPTH) g[9] = fmaf(dD[j], w, g[9]);
            m0 += tg;
            m1 += tey;
            m2 = fmaf(tey, ey[j], m2);
          }
          U[j] = fmaf(w, dcc, U[j]);
          T[j] = Tb;
        }
        g[5] = m0;
        // dL/dQ = -o/2 tg: centroid and conic terms from the moments
        const float nho = -0.5f * a1.z;
        g[0] = nho * (aex * m0 + a0.w * m1);          // times -2 in the tile sum
        g[1] = nho * (a0.w * ex * m0 + a1.x * m1);    // times -2 in the tile sum
        g[2] = nho * (ex * ex) * m0;
        g[3] = nho * ex * m1;                         // times 2 in the tile sum
        g[4] = nho * m2;
        const float rs = row_reduce_scatter8(g, rb0, rb1, rb2);
        const float s8 = row_sum16(g[8]);
        out = l16 < 8 ? rs : s8;
        if (DEPTH) {
          const float s9 = row_sum16(g[9]);
          if (l16 == 9) out = s9;
        }
      }
      if (writer) red[row][slot][k] = out;
    }
    __syncthreads();
    // one atomic per (splat, component) for this tile, one lane per pair, so
    // that the lanes of an instruction cover the consecutive components of a
    // few splats (a few cache lines of the per-splat records); splats no
    // pixel of the tile blends contribute nothing and are skipped. Without
    // depth, component 9 has no gradient (and no LDS row).
    constexpr int NCU = DEPTH ? NC : NC - 1;
    for (int e = threadIdx.x; e < cnt * NCU; e += NTH) {
      const int q = e / NCU, c = e - q * NCU;
      const uint32_t gidx = sid[q];
      if ((int64_t)gidx >= n) continue;
      float a = 0.f;
#pragma unroll
      for (int r2 = 0; r2 < NR; ++r2) a += red[r2][c][q];
      if (c < 2) a *= -2.f;  // exact: powers of two
      if (c == 3) a *= 2.f;
      if (a != 0.f) unsafeAtomicAdd(grad2d + (size_t)gidx * NC + c, (double)a);
    }
    __syncthreads();
    bend = bstart;
  }
}

// Workgroup b takes tile order[b] (order null: tile b).
template <int TILE, int PX, bool DEPTH>
__global__ void __launch_bounds__(TILE* TILE / PX) k_render_bwd(
    const float* __restrict__ splats, const uint32_t* __restrict__ vals,
    const uint32_t* __restrict__ ranges, int W, int H, int tiles_y, float bg0, float bg1,
    float bg2, const float* __restrict__ T_final, const uint32_t* __restrict__ n_contrib,
    const float* __restrict__ dL_dimage, const float* __restrict__ dL_ddepth,
    double* __restrict__ grad2d, int64_t n, const uint32_t* __restrict__ order) {
  __shared__ BwdLds<TILE, PX> L;
  const int tile = order ? (int)order[blockIdx.x] : (int)blockIdx.x;
  bwd_tile<TILE, PX, DEPTH>(L, tile, splats, vals, ranges, W, H, tiles_y, bg0, bg1, bg2,
                            T_final, n_contrib, dL_dimage, dL_ddepth, grad2d, n);
}

// Longest-first tile order for the backward. The backward of a tile walks
// its list down from the largest n_contrib of its pixels, so that number is
// the tile's work; starting the heaviest tiles first keeps them out of the
// launch's tail. work[t] = max n_contrib over tile t (one workgroup a tile).
template <int TILE>
__global__ void __launch_bounds__(256) k_tile_work(const uint32_t* __restrict__ n_contrib, int W,
                                                   int H, int tiles_y,
                                                   uint32_t* __restrict__ work) {
  __shared__ uint32_t wmax[256 / kWave];
  const int tile = blockIdx.x, tx = tile / tiles_y, ty = tile % tiles_y;
  uint32_t m = 0;
  for (int i = threadIdx.x; i < TILE * TILE; i += 256) {
    const int x = tx * TILE + i % TILE, y = ty * TILE + i / TILE;
    if (x < W && y < H) m = max(m, n_contrib[(size_t)y * W + x]);
  }
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, d, kWave));
  if ((threadIdx.x & (kWave - 1)) == 0) wmax[threadIdx.x / kWave] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int w = 1; w < 256 / kWave; ++w) m = max(m, wmax[w]);
    work[tile] = m;
  }
}

// 1024 work classes, exact below 512 splats, 8 wide above (up to 4600).
__device__ __forceinline__ uint32_t work_class(uint32_t w) {
  return w < 512u ? w : min(512u + ((w - 512u) >> 3), 1023u);
}

// Counting sort of the nt tiles by descending work class (one workgroup);
// tiles of one class keep no particular order.
__global__ void __launch_bounds__(1024) k_tile_rank(const uint32_t* __restrict__ work, int nt,
                                                    uint32_t* __restrict__ order) {
  constexpr int kHeld = 8;  // classes held in registers per thread (nt <= 8192)
  __shared__ uint32_t cnt[1024];
  __shared__ uint32_t wsum[1024 / kWave];
  cnt[threadIdx.x] = 0;
  uint32_t cls[kHeld];
#pragma unroll
  for (int j = 0; j < kHeld; ++j) {
    const int t = threadIdx.x + j * 1024;
    cls[j] = t < nt ? work_class(work[t]) : 0u;
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kHeld; ++j)
    if (threadIdx.x + j * 1024 < nt) atomicAdd(&cnt[cls[j]], 1u);
  for (int t = threadIdx.x + kHeld * 1024; t < nt; t += 1024)
    atomicAdd(&cnt[work_class(work[t])], 1u);
  __syncthreads();
  // thread i holds class 1023 - i, so the exclusive scan gives descending offsets
  const uint32_t c = cnt[1023 - threadIdx.x];
  uint32_t total;
  const uint32_t off = block_exclusive_scan<1024>(c, wsum, total);
  cnt[1023 - threadIdx.x] = off;
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kHeld; ++j) {
    const int t = threadIdx.x + j * 1024;
    if (t < nt) order[atomicAdd(&cnt[cls[j]], 1u)] = (uint32_t)t;
  }
  for (int t = threadIdx.x + kHeld * 1024; t < nt; t += 1024)
    order[atomicAdd(&cnt[work_class(work[t])], 1u)] = (uint32_t)t;
}

// Eq. 4 counts: the forward's decisions replayed per tile; for every splat
// of the list, the number of masked pixels of the tile that blend it is
// summed over the workgroup (wave ballots, then LDS) and added to its score
// with one atomic per (splat, tile).
template <int TILE>
__global__ void __launch_bounds__(TILE* TILE) k_split_score(
    const float* __restrict__ splats, const uint32_t* __restrict__ vals,
    const uint32_t* __restrict__ ranges, int64_t n, int W, int H, int tiles_y,
    const uint8_t* __restrict__ mask, uint32_t* __restrict__ score) {
  constexpr int NTH = TILE * TILE;
  constexpr int NB = 256;
  __shared__ float4 s0[NB], s1[NB];
  __shared__ uint32_t sid[NB], cnt[NB];
  const int tile = blockIdx.x;
  const int tx = tile / tiles_y, ty = tile % tiles_y;
  const uint32_t start = ranges[tile], end = ranges[tile + 1];
  const int x = tx * TILE + threadIdx.x % TILE, y = ty * TILE + threadIdx.x / TILE;
  const bool valid = x < W && y < H;
  const bool masked = valid && mask[(size_t)y * W + x] != 0;
  if (__syncthreads_count(masked) == 0) return;  // uniform: nothing to count here
  const float px = (float)x + 0.5f, py = (float)y + 0.5f;
  float T = 1.f;
  bool done = !valid;
  const int lane = threadIdx.x & (kWave - 1);
  for (uint32_t b = start; b < end; b += NB) {
    if (__syncthreads_count(!done) == 0) break;
    const int nb = (int)min((uint32_t)NB, end - b);
    for (int q = threadIdx.x; q < nb; q += NTH) {
      const uint32_t g = vals[b + q];
      cnt[q] = 0;
      sid[q] = g;
      if ((int64_t)g < n) {  // staged as fwd_step takes it
        const float4* r = reinterpret_cast<const float4*>(splats + (size_t)g * GS_SPLAT_FLOATS);
        float4 r0 = r[0], r1 = r[1];
        r1.w = skip_band(r0.z, r0.w, r1.x, r1.y);
        r0.w = r0.w + r0.w;  // exact
        s0[q] = r0;
        s1[q] = r1;
      } else {  // never for a correct list: an empty splat (t < 0 skips it)
        s0[q] = make_float4(0.f, 0.f, 1.f, 0.f);
        s1[q] = make_float4(1.f, -1.f, 0.f, 0.f);
      }
    }
    __syncthreads();
    for (int k = 0; k < nb; ++k) {
      bool hit = false;
      if (!done) {
        const float4 a0 = s0[k], a1 = s1[k];
        float al, Tn;
        const int st = fwd_step(px, py, a0, a1, T, al, Tn);
        if (st == kStop) {
          done = true;
        } else if (st == kBlend) {
          T = Tn;
          hit = masked;
        }
      }
      const uint64_t bal = __ballot(hit);
      if (hit && lane == __builtin_ctzll(bal)) atomicAdd(&cnt[k], (uint32_t)__popcll(bal));
    }
    __syncthreads();
    for (int q = threadIdx.x; q < nb; q += NTH)
      if (cnt[q] && (int64_t)sid[q] < n) atomicAdd(score + sid[q], cnt[q]);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Batched views: one persistent launch per phase. The (view, tile) work items
// of all views form one queue (view by view, tiles in id order); every
// workgroup takes the next item with one atomic on a device counter until
// the queue is empty.
struct ViewSet {
  int n_views, total;
  int start[GS_MAX_VIEWS + 1];  // first work item of each view
  int W[GS_MAX_VIEWS], H[GS_MAX_VIEWS], tiles_y[GS_MAX_VIEWS];
  const float* splats[GS_MAX_VIEWS];
  const uint32_t* vals[GS_MAX_VIEWS];
  const uint32_t* ranges[GS_MAX_VIEWS];
  float* image[GS_MAX_VIEWS];
  float* depth[GS_MAX_VIEWS];
  float* T_final[GS_MAX_VIEWS];
  uint32_t* n_contrib[GS_MAX_VIEWS];
  const float* dL_dimage[GS_MAX_VIEWS];
  const float* dL_ddepth[GS_MAX_VIEWS];
  double* grad2d[GS_MAX_VIEWS];
  RunLists rl[GS_MAX_VIEWS];  // the deferred binning's run tables (deferred forward only)
};

// Next work item for the whole workgroup (-1 when the queue is empty).
__device__ __forceinline__ int next_item(uint32_t* queue, int total, int* s_item) {
  if (threadIdx.x == 0) *s_item = (int)atomicAdd(queue, 1u);
  __syncthreads();
  const int it = *s_item;
  __syncthreads();
  return it < total ? it : -1;
}

__device__ __forceinline__ int view_of(const ViewSet& vs, int it) {
  int v = 0;
  while (v + 1 < vs.n_views && it >= vs.start[v + 1]) ++v;
  return v;
}

template <int TILE, int PX, int NB>
__global__ void __launch_bounds__(TILE* TILE / PX) k_render_fwd_batched(ViewSet vs, int64_t n,
                                                                         float bg0, float bg1,
                                                                         float bg2,
                                                                         uint32_t* queue) {
  __shared__ FwdLdsT<NB> L;
  __shared__ int s_item;
  for (int it; (it = next_item(queue, vs.total, &s_item)) >= 0;) {
    const int v = view_of(vs, it);
    fwd_tile<TILE, PX, false, NB>(L, it - vs.start[v], vs.splats[v], vs.vals[v], vs.ranges[v], n, vs.W[v],
                       vs.H[v], vs.tiles_y[v], bg0, bg1, bg2, vs.image[v], vs.depth[v],
                       vs.T_final[v], vs.n_contrib[v]);
  }
}

// The batched forward on the lists of the deferred binning (one run table
// per view); each view's vals receives the list positions it stages.
template <int TILE, int PX, int NB>
__global__ void __launch_bounds__(TILE* TILE / PX) k_render_fwd_batched_def(ViewSet vs, int64_t n,
                                                                             float bg0, float bg1,
                                                                             float bg2,
                                                                             uint32_t* queue) {
  __shared__ FwdLdsT<NB> L;
  __shared__ DefLds<NB, TILE * TILE / PX> DL;
  __shared__ int s_item;
  for (int it; (it = next_item(queue, vs.total, &s_item)) >= 0;) {
    const int v = view_of(vs, it);
    uint32_t* vals = const_cast<uint32_t*>(vs.vals[v]);  // the caller's (writable) list array
    fwd_tile<TILE, PX, false, NB, true>(L, it - vs.start[v], vs.splats[v], vals, vs.ranges[v], n,
                                        vs.W[v], vs.H[v], vs.tiles_y[v], bg0, bg1, bg2,
                                        vs.image[v], vs.depth[v], vs.T_final[v], vs.n_contrib[v],
                                        nullptr, 0, nullptr, &DL, vs.rl[v], vals);
  }
}

template <int TILE, int PX, bool DEPTH, int NB>
__global__ void __launch_bounds__(TILE* TILE / PX) k_render_bwd_batched(ViewSet vs, int64_t n,
                                                                         float bg0, float bg1,
                                                                         float bg2,
                                                                         uint32_t* queue,
                                                                         const uint32_t* order) {
  __shared__ BwdLds<TILE, PX, NB> L;
  __shared__ int s_item;
  for (int q; (q = next_item(queue, vs.total, &s_item)) >= 0;) {
    const int it = order ? (int)order[q] : q;
    const int v = view_of(vs, it);
    bwd_tile<TILE, PX, DEPTH, NB>(L, it - vs.start[v], vs.splats[v], vs.vals[v], vs.ranges[v],
                              vs.W[v], vs.H[v], vs.tiles_y[v], bg0, bg1, bg2, vs.T_final[v],
                              vs.n_contrib[v], vs.dL_dimage[v], vs.dL_ddepth[v], vs.grad2d[v],
                              n);
  }
}

__global__ void k_reset_queue(uint32_t* q) { *q = 0u; }

// k_tile_work over the (view, tile) items of a batch: work[it] = largest
// n_contrib of the item's pixels.
template <int TILE>
__global__ void __launch_bounds__(256) k_tile_work_views(ViewSet vs, uint32_t* __restrict__ work) {
  __shared__ uint32_t wmax[256 / kWave];
  const int it = blockIdx.x, v = view_of(vs, it), tile = it - vs.start[v];
  const int W = vs.W[v], H = vs.H[v], tx = tile / vs.tiles_y[v], ty = tile % vs.tiles_y[v];
  const uint32_t* nc = vs.n_contrib[v];
  uint32_t m = 0;
  for (int i = threadIdx.x; i < TILE * TILE; i += 256) {
    const int x = tx * TILE + i % TILE, y = ty * TILE + i / TILE;
    if (x < W && y < H) m = max(m, nc[(size_t)y * W + x]);
  }
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, d, kWave));
  if ((threadIdx.x & (kWave - 1)) == 0) wmax[threadIdx.x / kWave] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int w = 1; w < 256 / kWave; ++w) m = max(m, wmax[w]);
    work[it] = m;
  }
}

__global__ void k_zero_f64(double* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

gs_status launch_preprocess_bwd(const gs_gaussians* g, int64_t n, int deg, const CamDev& cam,
                                const double* grad2d, gs_gaussians* grads, int accumulate,
                                hipStream_t st);
gs_status launch_preprocess_bwd_adam(gs_gaussians* g, int64_t n, int deg, const CamDev& cam,
                                     const double* grad2d, const gs_adam_params* adam,
                                     hipStream_t st);
gs_status launch_preprocess_bwd_views(const gs_gaussians* g, int64_t n, int deg,
                                      const CamDev* cams, const double* const* grad2d,
                                      int n_views, gs_gaussians* grads, int accumulate,
                                      hipStream_t st);

}  // namespace gs

using namespace gs;

extern "C" gs_status gs_render_fwd(const float* splats, int64_t n, const uint32_t* vals,
                                   const uint32_t* ranges, const gs_camera* cam, const float* bg,
                                   float* image, float* depth, float* T_final,
                                   uint32_t* n_contrib, void* stream) {
  CamDev cd;
  if (n < 0 || !make_cam(cam, &cd) || !ranges || !bg || !image || !depth || !T_final ||
      !n_contrib)
    return GS_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const int nt = cd.tiles_x * cd.tiles_y;
  const int px = tuning().fwd_px;
#define GS_FWD(TL, PXV)                                                                        \
  k_render_fwd<TL, PXV><<<nt, TL * TL / PXV, 0, st>>>(splats, vals, ranges, n, cd.W, cd.H,  \
                                                      cd.tiles_y, bg[0], bg[1], bg[2], image, \
                                                      depth, T_final, n_contrib)
  GS_TIMED("render_fwd", st, if (cd.tile == 8) GS_FWD(8, 1);
           else if (cd.tile == 16) {
             if (px == 4) GS_FWD(16, 4); else if (px == 2) GS_FWD(16, 2); else GS_FWD(16, 1);
           } else {
             if (px == 4) GS_FWD(32, 4); else if (px == 2) GS_FWD(32, 2); else GS_FWD(32, 1);
           });
#undef GS_FWD
  GS_CHECK_LAUNCH();
  return GS_OK;
}

extern "C" gs_status gs_render_fwd_deferred(const float* splats, int64_t n, const void* workspace,
                                            size_t workspace_bytes, int64_t capacity,
                                            uint32_t* vals, const uint32_t* ranges,
                                            const gs_camera* cam, const float* bg, float* image,
                                            float* depth, float* T_final, uint32_t* n_contrib,
                                            void* stream) {
  CamDev cd;
  if (n < 0 || capacity < 0 || !make_cam(cam, &cd) || !ranges || !bg || !image || !depth ||
      !T_final || !n_contrib || (capacity > 0 && !vals))
    return GS_EINVAL;
  RunLists rl;
  if (!run_lists(workspace, workspace_bytes, n, capacity, cd.tiles_x, cd.tiles_y, &rl))
    return GS_ECAPACITY;
  hipStream_t st = (hipStream_t)stream;
  const int nt = cd.tiles_x * cd.tiles_y;
  const int px = tuning().fwd_px;
#define GS_FWD(TL, PXV)                                                                        \
  k_render_fwd_def<TL, PXV><<<nt, TL * TL / PXV, 0, st>>>(splats, rl, vals, ranges, n, cd.W,  \
                                                          cd.H, cd.tiles_y, bg[0], bg[1],     \
                                                          bg[2], image, depth, T_final,       \
                                                          n_contrib)
  GS_TIMED("render_fwd", st, if (cd.tile == 8) GS_FWD(8, 1);
           else if (cd.tile == 16) {
             if (px == 4) GS_FWD(16, 4); else if (px == 2) GS_FWD(16, 2); else GS_FWD(16, 1);
           } else {
             if (px == 4) GS_FWD(32, 4); else if (px == 2) GS_FWD(32, 2); else GS_FWD(32, 1);
           });
#undef GS_FWD
  GS_CHECK_LAUNCH();
  return GS_OK;
}

// The image-space backward of gs_render_bwd and gs_render_bwd_adam: grad2d
// zeroed, the tile order measured (when asked), then one launch over the
// tiles accumulating grad2d.
static gs_status image_bwd(int64_t n, const CamDev& cd, const float* splats, const uint32_t* vals,
                           const uint32_t* ranges, const float* bg, const float* T_final,
                           const uint32_t* n_contrib, const float* dL_dimage,
                           const float* dL_ddepth, double* grad2d, uint32_t* tile_order,
                           hipStream_t st) {
  k_zero_f64<<<div_up(n * GS_GRAD2D_COMPONENTS, 256), 256, 0, st>>>(grad2d,
                                                                     n * GS_GRAD2D_COMPONENTS);
  GS_CHECK_LAUNCH();
  const int nt = cd.tiles_x * cd.tiles_y;
  const int px = tuning().bwd_px;
  const uint32_t* order = nullptr;
  if (tile_order) {  // [0, nt): the order; [nt, 2 nt): per-tile work
    uint32_t* work = tile_order + nt;
    GS_TIMED("tile_order", st, {
      if (cd.tile == 8) k_tile_work<8><<<nt, 256, 0, st>>>(n_contrib, cd.W, cd.H, cd.tiles_y, work);
      else if (cd.tile == 16) k_tile_work<16><<<nt, 256, 0, st>>>(n_contrib, cd.W, cd.H, cd.tiles_y, work);
      else k_tile_work<32><<<nt, 256, 0, st>>>(n_contrib, cd.W, cd.H, cd.tiles_y, work);
      k_tile_rank<<<1, 1024, 0, st>>>(work, nt, tile_order);
    });
    GS_CHECK_LAUNCH();
    order = tile_order;
  }
#define GS_BWD2(TL, PXV, DEP)                                                                  \
  k_render_bwd<TL, PXV, DEP><<<nt, TL * TL / PXV, 0, st>>>(                                 \
      splats, vals, ranges, cd.W, cd.H, cd.tiles_y, bg[0], bg[1], bg[2], T_final, n_contrib, \
      dL_dimage, dL_ddepth, grad2d, n, order)
#define GS_BWD(TL, PXV) \
  if (dL_ddepth) GS_BWD2(TL, PXV, true); else GS_BWD2(TL, PXV, false)
  // 32x32 tiles with one pixel per lane would need 160 KB of LDS: use 2
  GS_TIMED("render_bwd", st, if (cd.tile == 8) { GS_BWD(8, 1); }
           else if (cd.tile == 16) {
             if (px == 4) { GS_BWD(16, 4); } else if (px == 2) { GS_BWD(16, 2); }
             else { GS_BWD(16, 1); }
           } else {
             if (px == 4) { GS_BWD(32, 4); } else { GS_BWD(32, 2); }
           });
#undef GS_BWD
#undef GS_BWD2
  GS_CHECK_LAUNCH();
  return GS_OK;
}

extern "C" gs_status gs_render_bwd(const gs_gaussians* g, int64_t n, int32_t sh_degree,
                                   const gs_camera* cam, const float* splats,
                                   const uint32_t* vals, const uint32_t* ranges, const float* bg,
                                   const float* T_final, const uint32_t* n_contrib,
                                   const float* dL_dimage, const float* dL_ddepth, double* grad2d,
                                   gs_gaussians* grads, int32_t accumulate, uint32_t* tile_order,
                                   void* stream) {
  CamDev cd;
  if (n < 0 || sh_degree < GS_DIRECT || sh_degree > 3 || !make_cam(cam, &cd) || !ranges || !bg ||
      !T_final || !n_contrib || !dL_dimage || !grad2d || !aligned16(grad2d) || !g || !grads)
    return GS_EINVAL;
  if (n == 0) return GS_OK;
  hipStream_t st = (hipStream_t)stream;
  const gs_status s = image_bwd(n, cd, splats, vals, ranges, bg, T_final, n_contrib, dL_dimage,
                                dL_ddepth, grad2d, tile_order, st);
  if (s != GS_OK) return s;
  return launch_preprocess_bwd(g, n, sh_degree, cd, grad2d, grads, accumulate, st);
}

static bool gaussians_set(const gs_gaussians& g) {
  return g.means && g.log_scales && g.quats && g.opacity_logits && g.sh;
}

extern "C" gs_status gs_render_bwd_adam(gs_gaussians* g, int64_t n, int32_t sh_degree,
                                        const gs_camera* cam, const float* splats,
                                        const uint32_t* vals, const uint32_t* ranges,
                                        const float* bg, const float* T_final,
                                        const uint32_t* n_contrib, const float* dL_dimage,
                                        const float* dL_ddepth, double* grad2d,
                                        const gs_adam_params* adam, uint32_t* tile_order,
                                        void* stream) {
  CamDev cd;
  if (n < 0 || sh_degree < GS_DIRECT || sh_degree > 3 || !make_cam(cam, &cd) || !ranges || !bg ||
      !T_final || !n_contrib || !dL_dimage || !grad2d || !aligned16(grad2d) || !g || !adam ||
      !adam->step)
    return GS_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  if (n > 0) {
    if (!gaussians_set(*g) || !gaussians_set(adam->m) || !gaussians_set(adam->v))
      return GS_EINVAL;
    gs_status s = image_bwd(n, cd, splats, vals, ranges, bg, T_final, n_contrib, dL_dimage,
                            dL_ddepth, grad2d, tile_order, st);
    if (s != GS_OK) return s;
    s = launch_preprocess_bwd_adam(g, n, sh_degree, cd, grad2d, adam, st);
    if (s != GS_OK) return s;
  }
  return launch_step_advance(adam->step, st);
}

extern "C" gs_status gs_render_fwd_ckpt(const float* splats, int64_t n, const uint32_t* vals,
                                        const uint32_t* ranges, const gs_camera* cam,
                                        const float* bg, float* image, float* depth,
                                        float* T_final, uint32_t* n_contrib, float* ckpt,
                                        int32_t ckpt_buckets, uint32_t* ckpt_overflow,
                                        void* stream) {
  CamDev cd;
  if (n < 0 || !make_cam(cam, &cd) || cd.tile != 16 || ckpt_buckets < 1 || !ranges || !bg ||
      !image || !depth || !T_final || !n_contrib || !ckpt || !ckpt_overflow)
    return GS_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const int nt = cd.tiles_x * cd.tiles_y;
  GS_TIMED("render_fwd", st,
           k_render_fwd_ckpt<<<nt, 256, 0, st>>>(splats, vals, ranges, n, cd.W, cd.H, cd.tiles_y,
                                                 bg[0], bg[1], bg[2], image, depth, T_final,
                                                 n_contrib, ckpt, ckpt_buckets, ckpt_overflow));
  GS_CHECK_LAUNCH();
  return GS_OK;
}

extern "C" gs_status gs_render_bwd_ckpt(const gs_gaussians* g, int64_t n, int32_t sh_degree,
                                        const gs_camera* cam, const float* splats,
                                        const uint32_t* vals, const uint32_t* ranges,
                                        const float* image, const float* depth,
                                        const uint32_t* n_contrib, const float* ckpt,
                                        int32_t ckpt_buckets, const float* dL_dimage,
                                        const float* dL_ddepth, double* grad2d,
                                        gs_gaussians* grads, int32_t accumulate, void* stream) {
  CamDev cd;
  if (n < 0 || sh_degree < GS_DIRECT || sh_degree > 3 || !make_cam(cam, &cd) || cd.tile != 16 ||
      ckpt_buckets < 1 || !ranges || !image || !n_contrib || !ckpt || !dL_dimage || !grad2d ||
      !aligned16(grad2d) ||
      !g || !grads || (dL_ddepth && !depth))
    return GS_EINVAL;
  if (n == 0) return GS_OK;
  hipStream_t st = (hipStream_t)stream;
  k_zero_f64<<<div_up(n * GS_GRAD2D_COMPONENTS, 256), 256, 0, st>>>(grad2d,
                                                                     n * GS_GRAD2D_COMPONENTS);
  GS_CHECK_LAUNCH();
  const int nt = cd.tiles_x * cd.tiles_y;
  GS_TIMED("render_bwd", st, if (dL_ddepth) {
    k_render_bwd_ckpt<true><<<nt, 256, 0, st>>>(splats, vals, ranges, cd.W, cd.H, cd.tiles_y,
                                                image, depth, n_contrib, ckpt, ckpt_buckets,
                                                dL_dimage, dL_ddepth, grad2d, n);
  } else {
    k_render_bwd_ckpt<false><<<nt, 256, 0, st>>>(splats, vals, ranges, cd.W, cd.H, cd.tiles_y,
                                                 image, depth, n_contrib, ckpt, ckpt_buckets,
                                                 dL_dimage, nullptr, grad2d, n);
  });
  GS_CHECK_LAUNCH();
  return launch_preprocess_bwd(g, n, sh_degree, cd, grad2d, grads, accumulate, st);
}

extern "C" gs_status gs_split_score(const float* splats, int64_t n, const uint32_t* vals,
                                    const uint32_t* ranges, const gs_camera* cam,
                                    const uint8_t* mask, uint32_t* score, void* stream) {
  CamDev cd;
  if (n < 0 || !make_cam(cam, &cd) || !ranges || !mask || !score || (n > 0 && !splats))
    return GS_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const int nt = cd.tiles_x * cd.tiles_y;
#define GS_SCORE(TL) \
  k_split_score<TL><<<nt, TL * TL, 0, st>>>(splats, vals, ranges, n, cd.W, cd.H, cd.tiles_y, mask, score)
  GS_TIMED("split_score", st, if (cd.tile == 8) GS_SCORE(8); else if (cd.tile == 16) GS_SCORE(16);
           else GS_SCORE(32));
#undef GS_SCORE
  GS_CHECK_LAUNCH();
  return GS_OK;
}

// ---------------------------------------------------------------------------
namespace {

int cu_count() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (!cached[dev]) {
    int c = 0;
    if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0)
      c = 256;
    cached[dev] = c;
  }
  return cached[dev];
}

// Validates a view batch for the render phases; fills the work queue layout.
bool make_view_set(const gs_view* views, int32_t n_views, bool bwd, ViewSet* vs, int* tile,
                   bool* any_depth) {
  if (!views || n_views < 1 || n_views > GS_MAX_VIEWS) return false;
  vs->n_views = n_views;
  vs->start[0] = 0;
  *any_depth = false;
  for (int v = 0; v < n_views; ++v) {
    CamDev cd;
    const gs_view& w = views[v];
    if (!make_cam(&w.cam, &cd)) return false;
    if (v == 0) *tile = cd.tile;
    if (cd.tile != *tile) return false;
    if (!w.ranges || !w.T_final || !w.n_contrib) return false;
    if (!bwd && (!w.image || !w.depth)) return false;
    if (bwd && (!w.dL_dimage || !w.grad2d || !aligned16(w.grad2d))) return false;
    vs->W[v] = cd.W;
    vs->H[v] = cd.H;
    vs->tiles_y[v] = cd.tiles_y;
    vs->splats[v] = w.splats;
    vs->vals[v] = w.vals;
    vs->ranges[v] = w.ranges;
    vs->image[v] = w.image;
    vs->depth[v] = w.depth;
    vs->T_final[v] = w.T_final;
    vs->n_contrib[v] = w.n_contrib;
    vs->dL_dimage[v] = w.dL_dimage;
    vs->dL_ddepth[v] = w.dL_ddepth;
    vs->grad2d[v] = w.grad2d;
    if (w.dL_ddepth) *any_depth = true;
    vs->start[v + 1] = vs->start[v] + cd.tiles_x * cd.tiles_y;
  }
  vs->total = vs->start[n_views];
  return true;
}

int persistent_grid(int total, int wgs_per_cu) {
  const int g = cu_count() * wgs_per_cu;
  return g < total ? g : total;
}

}  // namespace

extern "C" gs_status gs_render_fwd_batched(int64_t n, const gs_view* views, int32_t n_views,
                                           const float* bg, uint32_t* queue, void* stream) {
  ViewSet vs;
  int tile = 16;
  bool any_depth;
  if (n < 0 || !bg || !queue || !make_view_set(views, n_views, false, &vs, &tile, &any_depth))
    return GS_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const int px = tuning().fwd_px;
  const int grid = persistent_grid(vs.total, tuning().persist_wgs);
  k_reset_queue<<<1, 1, 0, st>>>(queue);
  GS_CHECK_LAUNCH();
  const int fb = tuning().fwd_batch;
#define GS_FWDB3(TL, PXV, NBV)                                                                   \
  k_render_fwd_batched<TL, PXV, NBV><<<grid, TL * TL / PXV, 0, st>>>(vs, n, bg[0], bg[1], bg[2], \
                                                                     queue)
#define GS_FWDB(TL, PXV)                                 \
  do {                                                   \
    if (fb == 64) GS_FWDB3(TL, PXV, 64);                 \
    else if (fb == 128) GS_FWDB3(TL, PXV, 128);          \
    else GS_FWDB3(TL, PXV, 256);                         \
  } while (0)
  GS_TIMED("render_fwd", st, if (tile == 8) GS_FWDB(8, 1);
           else if (tile == 16) {
             if (px == 4) GS_FWDB(16, 4); else if (px == 2) GS_FWDB(16, 2); else GS_FWDB(16, 1);
           } else {
             if (px == 4) GS_FWDB(32, 4); else if (px == 2) GS_FWDB(32, 2); else GS_FWDB(32, 1);
           });
#undef GS_FWDB
#undef GS_FWDB3
  GS_CHECK_LAUNCH();
  return GS_OK;
}

extern "C" gs_status gs_render_fwd_batched_deferred(int64_t n, const gs_view* views,
                                                    int32_t n_views, const void* const* workspaces,
                                                    const size_t* workspace_bytes, const float* bg,
                                                    uint32_t* queue, void* stream) {
  ViewSet vs;
  int tile = 16;
  bool any_depth;
  if (n < 0 || !bg || !queue || !workspaces || !workspace_bytes ||
      !make_view_set(views, n_views, false, &vs, &tile, &any_depth))
    return GS_EINVAL;
  for (int v = 0; v < n_views; ++v) {
    const gs_view& w = views[v];
    if (w.capacity < 0 || (w.capacity > 0 && !w.vals)) return GS_EINVAL;
    CamDev cd;
    if (!make_cam(&w.cam, &cd)) return GS_EINVAL;
    if (!run_lists(workspaces[v], workspace_bytes[v], n, w.capacity, cd.tiles_x, cd.tiles_y,
                   &vs.rl[v]))
      return GS_ECAPACITY;
  }
  hipStream_t st = (hipStream_t)stream;
  const int px = tuning().fwd_px;
  const int grid = persistent_grid(vs.total, tuning().persist_wgs);
  k_reset_queue<<<1, 1, 0, st>>>(queue);
  GS_CHECK_LAUNCH();
  const int fb = tuning().fwd_batch;
#define GS_FWDB3(TL, PXV, NBV)                                                               \
  k_render_fwd_batched_def<TL, PXV, NBV><<<grid, TL * TL / PXV, 0, st>>>(vs, n, bg[0], bg[1], \
                                                                         bg[2], queue)
#define GS_FWDB(TL, PXV)                                 \
  do {                                                   \
    if (fb == 64) GS_FWDB3(TL, PXV, 64);                 \
    else if (fb == 128) GS_FWDB3(TL, PXV, 128);          \
    else GS_FWDB3(TL, PXV, 256);                         \
  } while (0)
  GS_TIMED("render_fwd", st, if (tile == 8) GS_FWDB(8, 1);
           else if (tile == 16) {
             if (px == 4) GS_FWDB(16, 4); else if (px == 2) GS_FWDB(16, 2); else GS_FWDB(16, 1);
           } else {
             if (px == 4) GS_FWDB(32, 4); else if (px == 2) GS_FWDB(32, 2); else GS_FWDB(32, 1);
           });
#undef GS_FWDB
#undef GS_FWDB3
  GS_CHECK_LAUNCH();
  return GS_OK;
}

extern "C" gs_status gs_render_bwd_batched(const gs_gaussians* g, int64_t n, int32_t sh_degree,
                                           const gs_view* views, int32_t n_views,
                                           const float* bg, uint32_t* queue,
                                           gs_gaussians* grads, int32_t accumulate,
                                           uint32_t* tile_order, void* stream) {
  ViewSet vs;
  int tile = 16;
  bool any_depth;
  if (n < 0 || sh_degree < GS_DIRECT || sh_degree > 3 || !bg || !queue || !g || !grads ||
      (accumulate != 0 && accumulate != 1) ||
      !make_view_set(views, n_views, true, &vs, &tile, &any_depth))
    return GS_EINVAL;
  if (n == 0) return GS_OK;
  hipStream_t st = (hipStream_t)stream;
  for (int v = 0; v < n_views; ++v) {
    k_zero_f64<<<div_up(n * GS_GRAD2D_COMPONENTS, 256), 256, 0, st>>>(vs.grad2d[v],
                                                                       n * GS_GRAD2D_COMPONENTS);
    GS_CHECK_LAUNCH();
  }
  const int px = tuning().bwd_px;
  const int grid = persistent_grid(vs.total, tuning().persist_wgs);
  k_reset_queue<<<1, 1, 0, st>>>(queue);
  GS_CHECK_LAUNCH();
  const uint32_t* order = nullptr;
  if (tile_order && vs.total > 0) {  // [0, total): the order; [total, 2 total): the work
    uint32_t* work = tile_order + vs.total;
    GS_TIMED("tile_order", st, {
      if (tile == 8) k_tile_work_views<8><<<vs.total, 256, 0, st>>>(vs, work);
      else if (tile == 16) k_tile_work_views<16><<<vs.total, 256, 0, st>>>(vs, work);
      else k_tile_work_views<32><<<vs.total, 256, 0, st>>>(vs, work);
      k_tile_rank<<<1, 1024, 0, st>>>(work, vs.total, tile_order);
    });
    GS_CHECK_LAUNCH();
    order = tile_order;
  }
  // splat batch: the knob (32, 64, 128; 128 needs 80 KB of LDS at 256 threads
  // and is not built for 512), else the default of the workgroup size
  const int bb = tuning().bwd_batch;
#define GS_BWDB3(TL, PXV, DEP, NBV)                                                          \
  k_render_bwd_batched<TL, PXV, DEP, NBV><<<grid, TL * TL / PXV, 0, st>>>(vs, n, bg[0], bg[1], \
                                                                          bg[2], queue, order)
#define GS_BWDB2(TL, PXV, DEP)                                                        \
  do {                                                                                \
    if (bb == 32) GS_BWDB3(TL, PXV, DEP, 32);                                         \
    else if (bb == 64) GS_BWDB3(TL, PXV, DEP, 64);                                    \
    else if (bb == 128 && TL * TL / PXV <= 256) GS_BWDB3(TL, PXV, DEP, (TL * TL / PXV <= 256 ? 128 : 64)); \
    else GS_BWDB3(TL, PXV, DEP, (bwd_batch_default<TL, PXV>()));                      \
  } while (0)
#define GS_BWDB(TL, PXV) \
  if (any_depth) GS_BWDB2(TL, PXV, true); else GS_BWDB2(TL, PXV, false)
  GS_TIMED("render_bwd", st, if (tile == 8) { GS_BWDB(8, 1); }
           else if (tile == 16) {
             if (px == 4) { GS_BWDB(16, 4); } else if (px == 2) { GS_BWDB(16, 2); }
             else { GS_BWDB(16, 1); }
           } else {
             if (px == 4) { GS_BWDB(32, 4); } else { GS_BWDB(32, 2); }
           });
#undef GS_BWDB
#undef GS_BWDB2
#undef GS_BWDB3
  GS_CHECK_LAUNCH();
  CamDev cds[GS_MAX_VIEWS];
  const double* g2[GS_MAX_VIEWS];
  for (int v = 0; v < n_views; ++v) {
    make_cam(&views[v].cam, &cds[v]);
    g2[v] = vs.grad2d[v];
  }
  return launch_preprocess_bwd_views(g, n, sh_degree, cds, g2, n_views, grads, accumulate, st);
}
