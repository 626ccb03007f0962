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

#include "common.h"

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

// One front-to-back step of the forward at one pixel: skip (alpha < 1/255,
// decided as Q > t), stop (the blend would take T below 1e-4) or blend with
// alpha `al` and new transmittance `Tn`. Shared by every kernel that replays
// the forward's decisions.
constexpr int kSkip = 0, kBlend = 1, kStop = 2;
__device__ __forceinline__ int fwd_step(float px, float py, float4 a0, float4 a1, float b2,
                                        float T, float& al, float& Tn) {
#pragma clang fp contract(fast)
  const SplatQ q = eval_q(px, py, a0.x, a0.y, a0.z, b2, a1.x);
  if (splat_skips(q.Q, q.mag, a1.y, px, py, a0.x, a0.y, a0.z, a0.w, a1.x)) return kSkip;
  al = fminf(kAlphaMax, a1.z * gauss(q.Q));
  Tn = T * (1.f - al);
  return Tn < kTStop ? kStop : kBlend;
}

template <int TILE, int PX>
__global__ void __launch_bounds__(TILE* TILE / PX) k_render_fwd(
    const float* __restrict__ splats, const uint32_t* __restrict__ vals,
    const uint32_t* __restrict__ ranges, int64_t n, int W, int H, int tiles_y, float bg0,
    float bg1, float bg2, float* __restrict__ image, float* __restrict__ depth,
    float* __restrict__ T_final, uint32_t* __restrict__ n_contrib) {
#pragma clang fp contract(fast)
  constexpr int NTH = TILE * TILE / PX;
  constexpr int NB = 256;  // splats per LDS batch
  __shared__ float4 s0[NB], s1[NB], s2[NB];
  const int tile = blockIdx.x;  // column-major tile id
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
  for (uint32_t b = start; b < end; b += NB) {
    if (__syncthreads_count(!alldone) == 0) break;
    const int cnt = (int)min((uint32_t)NB, end - b);
    for (int q = threadIdx.x; q < cnt; q += NTH) {
      const uint32_t g = vals[b + q];
      if ((int64_t)g < n) {
        const float4* r = reinterpret_cast<const float4*>(splats + (size_t)g * GS_SPLAT_FLOATS);
        s0[q] = r[0];
        s1[q] = r[1];
        s2[q] = r[2];
      } else {  // never for a correct list: an empty splat (t < 0 skips it)
        s0[q] = make_float4(0.f, 0.f, 1.f, 0.f);
        s1[q] = make_float4(1.f, -1.f, 0.f, 0.f);
        s2[q] = make_float4(0.f, 0.f, 0.f, 0.f);
      }
    }
    __syncthreads();
    for (int k = 0; k < cnt && !alldone; ++k) {
      const float4 a0 = s0[k], a1 = s1[k];
      const float b2 = a0.w + a0.w;
      alldone = true;
#pragma unroll
      for (int j = 0; j < PX; ++j) {
        if (!done[j]) {
          float al, Tn;
          const int st = fwd_step(px[j], py[j], a0, a1, b2, T[j], al, Tn);
          if (st != kSkip) {
            if (st == kStop) {
              done[j] = true;
            } else {
              const float4 a2 = s2[k];
              const float w = al * T[j];
              C0[j] = fmaf(a2.x, w, C0[j]);
              C1[j] = fmaf(a2.y, w, C1[j]);
              C2[j] = fmaf(a2.z, w, C2[j]);
              D[j] = fmaf(a1.w, w, D[j]);
              T[j] = Tn;
              last[j] = b + (uint32_t)k - start + 1u;
            }
          }
        }
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

template <int TILE, int PX, bool DEPTH>
__global__ void __launch_bounds__(TILE* TILE / PX) k_render_bwd(
    const float* __restrict__ splats, const uint32_t* __restrict__ vals,
    const uint32_t* __restrict__ ranges, int W, int H, int tiles_y, float bg0, float bg1,
    float bg2, const float* __restrict__ T_final, const uint32_t* __restrict__ n_contrib,
    const float* __restrict__ dL_dimage, const float* __restrict__ dL_ddepth,
    double* __restrict__ grad2d, int64_t n) {
#pragma clang fp contract(fast)
  constexpr int NTH = TILE * TILE / PX;   // threads
  constexpr int NW = NTH / kWave;         // wavefronts
  constexpr int NR = NW * (kWave / 16);   // rows of 16 lanes
  constexpr int NB = 64;                  // splats per batch
  constexpr int NC = GS_GRAD2D_COMPONENTS;
  static_assert(NTH % kWave == 0, "whole wavefronts");
  __shared__ float4 s0[NB], s1[NB], s2[NB];
  __shared__ uint32_t sid[NB];
  __shared__ float red[NR][NC][NB];
  __shared__ uint32_t smax;
  const int tile = blockIdx.x;  // column-major tile id
  const int tx = tile / tiles_y, ty = tile % tiles_y;
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  const int row = wv * (kWave / 16) + lane / 16;
  const uint32_t start = ranges[tile];
  const size_t HW = (size_t)H * W;
  float px[PX], py[PX], T[PX], dC0[PX], dC1[PX], dC2[PX], dD[PX];
  float S0[PX], S1[PX], S2[PX], SD[PX];
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
      if (DEPTH) dD[j] = dL_ddepth[p];
    }
    // colour and depth of everything behind the current splat
    S0[j] = T[j] * bg0; S1[j] = T[j] * bg1; S2[j] = T[j] * bg2; SD[j] = 0.f;
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
        const float4* r = reinterpret_cast<const float4*>(splats + (size_t)g * GS_SPLAT_FLOATS);
        s0[q] = r[0];
        s1[q] = r[1];
        s2[q] = r[2];
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
      bool act[PX];
      SplatQ q[PX];
      bool any = false;
#pragma unroll
      for (int j = 0; j < PX; ++j) {
        act[j] = pos < nc[j];
        if (act[j]) {
          q[j] = eval_q(px[j], py[j], a0.x, a0.y, a0.z, b2, a1.x);
          act[j] = !splat_skips(q[j].Q, q[j].mag, a1.y, px[j], py[j], a0.x, a0.y, a0.z, a0.w,
                                a1.x);
        }
        any |= act[j];
      }
      float g[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) g[c] = 0.f;
      if (__ballot(any) != 0) {
        const float4 a2 = s2[k];
        const float nho = -0.5f * a1.z;
#pragma unroll
        for (int j = 0; j < PX; ++j) {
          if (!act[j]) continue;
          const float G = gauss(q[j].Q);
          const float oG = a1.z * G;
          const float al = fminf(kAlphaMax, oG);
          const float rinv = __builtin_amdgcn_rcpf(1.f - al);
          const float Tb = T[j] * rinv;  // transmittance in front of this splat
          const float w = al * Tb;
          float acc = dC0[j] * (T[j] * a2.x - S0[j]) + dC1[j] * (T[j] * a2.y - S1[j]) +
                      dC2[j] * (T[j] * a2.z - S2[j]);
          if (DEPTH) acc += dD[j] * (T[j] * a1.w - SD[j]);
          const float dal = rinv * acc;
          g[6] += dC0[j] * w;
          g[7] += dC1[j] * w;
          g[8] += dC2[j] * w;
          if (DEPTH) g[9] += dD[j] * w;
          if (oG <= kAlphaMax) {
            const float tg = dal * G;
            g[5] += tg;
            const float dQ = tg * nho;
            const float ex = q[j].dx, ey = q[j].dy;
            g[0] += dQ * (a0.z * ex + a0.w * ey);   // times -2 below
            g[1] += dQ * (a0.w * ex + a1.x * ey);   // times -2 below
            g[2] += (dQ * ex) * ex;
            g[3] += (dQ * ex) * ey;                  // times 2 below
            g[4] += (dQ * ey) * ey;
          }
          S0[j] += a2.x * w;
          S1[j] += a2.y * w;
          S2[j] += a2.z * w;
          if (DEPTH) SD[j] += a1.w * w;
          T[j] = Tb;
        }
#pragma unroll
        for (int c = 0; c < NC; ++c)
          if (DEPTH || c != 9) g[c] = row_sum16(g[c]);
      }
      if ((lane & 15) == 15) {
        red[row][0][k] = -2.f * g[0];
        red[row][1][k] = -2.f * g[1];
        red[row][2][k] = g[2];
        red[row][3][k] = 2.f * g[3];
#pragma unroll
        for (int c = 4; c < NC; ++c) red[row][c][k] = g[c];
      }
    }
    __syncthreads();
    // one atomic per (splat, component) for this tile; splats no pixel of the
    // tile blends contribute nothing and are skipped
    for (int q = threadIdx.x; q < cnt; q += NTH) {
      const uint32_t gidx = sid[q];
      if ((int64_t)gidx >= n) continue;
      for (int c = 0; c < NC; ++c) {
        float a = 0.f;
#pragma unroll
        for (int r2 = 0; r2 < NR; ++r2) a += red[r2][c][q];
        if (a != 0.f) unsafeAtomicAdd(grad2d + (size_t)c * n + gidx, (double)a);
      }
    }
    __syncthreads();
    bend = bstart;
  }
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
      if ((int64_t)g < n) {
        const float4* r = reinterpret_cast<const float4*>(splats + (size_t)g * GS_SPLAT_FLOATS);
        s0[q] = r[0];
        s1[q] = r[1];
      } else {
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
        const int st = fwd_step(px, py, a0, a1, a0.w + a0.w, T, al, Tn);
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

__global__ void k_zero_f64(double* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

gs_status launch_preprocess_bwd(const gs_gaussians* g, int64_t n, int deg, const CamDev& cam,
                                const double* grad2d, gs_gaussians* grads, int accumulate,
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

extern "C" gs_status gs_render_bwd(const gs_gaussians* g, int64_t n, int32_t sh_degree,
                                   const gs_camera* cam, const float* splats,
                                   const uint32_t* vals, const uint32_t* ranges, const float* bg,
                                   const float* T_final, const uint32_t* n_contrib,
                                   const float* dL_dimage, const float* dL_ddepth, double* grad2d,
                                   gs_gaussians* grads, int32_t accumulate, void* stream) {
  CamDev cd;
  if (n < 0 || sh_degree < GS_DIRECT || sh_degree > 3 || !make_cam(cam, &cd) || !ranges || !bg ||
      !T_final || !n_contrib || !dL_dimage || !grad2d || !g || !grads)
    return GS_EINVAL;
  if (n == 0) return GS_OK;
  hipStream_t st = (hipStream_t)stream;
  k_zero_f64<<<div_up(n * GS_GRAD2D_COMPONENTS, 256), 256, 0, st>>>(grad2d,
                                                                     n * GS_GRAD2D_COMPONENTS);
  GS_CHECK_LAUNCH();
  const int nt = cd.tiles_x * cd.tiles_y;
  const int px = tuning().bwd_px;
#define GS_BWD2(TL, PXV, DEP)                                                                  \
  k_render_bwd<TL, PXV, DEP><<<nt, TL * TL / PXV, 0, st>>>(                                 \
      splats, vals, ranges, cd.W, cd.H, cd.tiles_y, bg[0], bg[1], bg[2], T_final, n_contrib, \
      dL_dimage, dL_ddepth, grad2d, n)
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
