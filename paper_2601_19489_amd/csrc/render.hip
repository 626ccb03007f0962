// Per-tile compositing (Sec. 2.1, second step) and its backward (Sec. 2.2).
//
// Forward: one workgroup per tile, one thread per pixel. The tile's sorted
// splat records are gathered through `vals` into LDS in batches of one
// record per thread; every pixel walks the batch front to back. The
// workgroup stops as soon as every pixel has reached T < 1e-4.
//
// Backward: one workgroup per tile, one thread per pixel, walking the
// tile's list back to front from each pixel's last contributor. The
// transmittance in front of each splat is recomputed as T / (1 - alpha)
// from the stored final transmittance (nothing per splat is stored by the
// forward), and the colour and depth behind it are accumulated on the way.
// The ten per-splat gradient components are summed over the 64 pixels of a
// wavefront with DPP; per tile, one FP64 atomic add per (splat, component).
#include <math.h>

#include "common.h"

namespace gs {

constexpr float kAlphaMax = 0.99f;
constexpr float kTStop = 1e-4f;

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

template <int TILE>
__global__ void __launch_bounds__(TILE* TILE) k_render_fwd(
    const float* __restrict__ splats, const uint32_t* __restrict__ vals,
    const uint32_t* __restrict__ ranges, int64_t n, int W, int H, int tiles_y, float bg0,
    float bg1, float bg2, float* __restrict__ image, float* __restrict__ depth,
    float* __restrict__ T_final, uint32_t* __restrict__ n_contrib) {
  constexpr int NT = TILE * TILE;
  __shared__ float4 s0[NT], s1[NT], s2[NT];
  const int tile = blockIdx.x;  // column-major tile id
  const int tx = tile / tiles_y, ty = tile % tiles_y;
  const int x = tx * TILE + (int)(threadIdx.x % TILE);
  const int y = ty * TILE + (int)(threadIdx.x / TILE);
  const bool inside = x < W && y < H;
  const float px = (float)x + 0.5f, py = (float)y + 0.5f;
  const uint32_t start = ranges[tile], end = ranges[tile + 1];
  float T = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f, D = 0.f;
  uint32_t last = 0;  // one past the list position of the last blended splat
  bool done = !inside;
  for (uint32_t b = start; b < end; b += NT) {
    if (__syncthreads_count(!done) == 0) break;
    const uint32_t j = b + threadIdx.x;
    if (j < end) {
      const uint32_t g = vals[j];
      if ((int64_t)g < n) {
        const float4* r = reinterpret_cast<const float4*>(splats + (size_t)g * GS_SPLAT_FLOATS);
        s0[threadIdx.x] = r[0];
        s1[threadIdx.x] = r[1];
        s2[threadIdx.x] = r[2];
      } else {  // never for a correct list: an empty splat (t < 0 skips it)
        s0[threadIdx.x] = make_float4(0.f, 0.f, 1.f, 0.f);
        s1[threadIdx.x] = make_float4(1.f, -1.f, 0.f, 0.f);
        s2[threadIdx.x] = make_float4(0.f, 0.f, 0.f, 0.f);
      }
    }
    __syncthreads();
    const int cnt = (int)min((uint32_t)NT, end - b);
    for (int k = 0; k < cnt && !done; ++k) {
      const float4 a0 = s0[k], a1 = s1[k];
      const SplatQ q = eval_q(px, py, a0.x, a0.y, a0.z, a0.w + a0.w, a1.x);
      if (splat_skips(q.Q, q.mag, a1.y, px, py, a0.x, a0.y, a0.z, a0.w, a1.x)) continue;
      const float G = __expf(-0.5f * q.Q);
      const float al = fminf(kAlphaMax, a1.z * G);
      const float Tn = T * (1.f - al);
      if (Tn < kTStop) {
        done = true;
        break;
      }
      const float4 a2 = s2[k];
      const float w = al * T;
      C0 = fmaf(a2.x, w, C0);
      C1 = fmaf(a2.y, w, C1);
      C2 = fmaf(a2.z, w, C2);
      D = fmaf(a1.w, w, D);
      T = Tn;
      last = b + (uint32_t)k - start + 1u;
    }
  }
  if (inside) {
    const size_t p = (size_t)y * W + x, HW = (size_t)H * W;
    image[p] = fmaf(T, bg0, C0);
    image[HW + p] = fmaf(T, bg1, C1);
    image[2 * HW + p] = fmaf(T, bg2, C2);
    depth[p] = D;
    T_final[p] = T;
    n_contrib[p] = last;
  }
}

// Backward, one workgroup per tile. Each lane owns PX pixels of the tile
// (pixel t + j * threads, j < PX) and walks the list back to front. Per splat
// the lane adds its pixels' gradient terms, the wavefront sums the ten
// components with DPP, and the wave's last lane parks the sums in LDS. After
// each batch of splats the workgroup adds the waves' sums and issues one
// atomic per (splat, component) for the tile, 64 splats per instruction.
template <int TILE, int PX>
__global__ void __launch_bounds__(TILE* TILE / PX) k_render_bwd(
    const float* __restrict__ splats, const uint32_t* __restrict__ vals,
    const uint32_t* __restrict__ ranges, int W, int H, int tiles_y, float bg0, float bg1,
    float bg2, const float* __restrict__ T_final, const uint32_t* __restrict__ n_contrib,
    const float* __restrict__ dL_dimage, const float* __restrict__ dL_ddepth,
    double* __restrict__ grad2d, int64_t n) {
  constexpr int NTH = TILE * TILE / PX;   // threads
  constexpr int NW = NTH / kWave;         // wavefronts
  constexpr int NB = NTH < 128 ? NTH : 128;  // splats per batch (keeps LDS under 48 KB)
  static_assert(NTH % kWave == 0, "whole wavefronts");
  __shared__ float4 s0[NB], s1[NB], s2[NB];
  __shared__ uint32_t sid[NB];
  __shared__ float red[NW][GS_GRAD2D_COMPONENTS][NB];
  __shared__ uint32_t smax;
  const int tile = blockIdx.x;  // column-major tile id
  const int tx = tile / tiles_y, ty = tile % tiles_y;
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
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
      if (dL_ddepth) dD[j] = dL_ddepth[p];
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
    for (int q = threadIdx.x; q < cnt; q += NTH) {  // cnt <= NB
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
      float gu = 0.f, gv = 0.f, ga = 0.f, gb = 0.f, gc = 0.f, go = 0.f;
      float gr = 0.f, gg = 0.f, gbc = 0.f, gz = 0.f;
      if (__ballot(any) != 0) {
        const float4 a2 = s2[k];
#pragma unroll
        for (int j = 0; j < PX; ++j) {
          if (!act[j]) continue;
          const float G = __expf(-0.5f * q[j].Q);
          const float oG = a1.z * G;
          const float al = fminf(kAlphaMax, oG);
          const float rinv = __builtin_amdgcn_rcpf(1.f - al);
          const float Tb = T[j] * rinv;  // transmittance in front of this splat
          const float w = al * Tb;
          const float dal = rinv * (dC0[j] * (T[j] * a2.x - S0[j]) + dC1[j] * (T[j] * a2.y - S1[j]) +
                                    dC2[j] * (T[j] * a2.z - S2[j]) + dD[j] * (T[j] * a1.w - SD[j]));
          gr = fmaf(dC0[j], w, gr);
          gg = fmaf(dC1[j], w, gg);
          gbc = fmaf(dC2[j], w, gbc);
          gz = fmaf(dD[j], w, gz);
          if (oG <= kAlphaMax) {
            go = fmaf(dal, G, go);
            const float dQ = -0.5f * G * (dal * a1.z);
            gu += -2.f * dQ * (a0.z * q[j].dx + a0.w * q[j].dy);
            gv += -2.f * dQ * (a0.w * q[j].dx + a1.x * q[j].dy);
            ga += dQ * q[j].dx * q[j].dx;
            gb += 2.f * dQ * q[j].dx * q[j].dy;
            gc += dQ * q[j].dy * q[j].dy;
          }
          S0[j] = fmaf(a2.x, w, S0[j]);
          S1[j] = fmaf(a2.y, w, S1[j]);
          S2[j] = fmaf(a2.z, w, S2[j]);
          SD[j] = fmaf(a1.w, w, SD[j]);
          T[j] = Tb;
        }
        gu = wave_sum_to_last(gu);
        gv = wave_sum_to_last(gv);
        ga = wave_sum_to_last(ga);
        gb = wave_sum_to_last(gb);
        gc = wave_sum_to_last(gc);
        go = wave_sum_to_last(go);
        gr = wave_sum_to_last(gr);
        gg = wave_sum_to_last(gg);
        gbc = wave_sum_to_last(gbc);
        gz = wave_sum_to_last(gz);
      }
      if (lane == kWave - 1) {
        red[wv][0][k] = gu; red[wv][1][k] = gv; red[wv][2][k] = ga; red[wv][3][k] = gb;
        red[wv][4][k] = gc; red[wv][5][k] = go; red[wv][6][k] = gr; red[wv][7][k] = gg;
        red[wv][8][k] = gbc; red[wv][9][k] = gz;
      }
    }
    __syncthreads();
    // one atomic per (splat, component) for this tile; splats no pixel of the
    // tile blends contribute nothing and are skipped
    for (int q = threadIdx.x; q < cnt; q += NTH) {
      const uint32_t g = sid[q];
      float acc[GS_GRAD2D_COMPONENTS];
      bool nz = false;
#pragma unroll
      for (int c = 0; c < GS_GRAD2D_COMPONENTS; ++c) {
        float a = 0.f;
#pragma unroll
        for (int w2 = 0; w2 < NW; ++w2) a += red[w2][c][q];
        acc[c] = a;
        nz |= a != 0.f;
      }
      if (nz && (int64_t)g < n) {
#pragma unroll
        for (int c = 0; c < GS_GRAD2D_COMPONENTS; ++c)
          if (acc[c] != 0.f) unsafeAtomicAdd(grad2d + (size_t)c * n + g, (double)acc[c]);
      }
    }
    __syncthreads();
    bend = bstart;
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
#define GS_FWD(TL)                                                                         \
  k_render_fwd<TL><<<nt, TL * TL, 0, st>>>(splats, vals, ranges, n, cd.W, cd.H, cd.tiles_y, \
                                           bg[0], bg[1], bg[2], image, depth, T_final,    \
                                           n_contrib)
  GS_TIMED("render_fwd", st, if (cd.tile == 8) GS_FWD(8); else if (cd.tile == 16) GS_FWD(16);
           else GS_FWD(32));
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
  if (n < 0 || sh_degree < 0 || sh_degree > 3 || !make_cam(cam, &cd) || !ranges || !bg ||
      !T_final || !n_contrib || !dL_dimage || !grad2d || !g || !grads)
    return GS_EINVAL;
  if (n == 0) return GS_OK;
  hipStream_t st = (hipStream_t)stream;
  k_zero_f64<<<div_up(n * GS_GRAD2D_COMPONENTS, 256), 256, 0, st>>>(grad2d,
                                                                     n * GS_GRAD2D_COMPONENTS);
  GS_CHECK_LAUNCH();
  const int nt = cd.tiles_x * cd.tiles_y;
  const int px = tuning().bwd_px;
#define GS_BWD(TL, PXV)                                                                        \
  k_render_bwd<TL, PXV><<<nt, TL * TL / PXV, 0, st>>>(splats, vals, ranges, cd.W, cd.H,     \
                                                      cd.tiles_y, bg[0], bg[1], bg[2], T_final, \
                                                      n_contrib, dL_dimage, dL_ddepth, grad2d, n)
  // 32x32 tiles with one pixel per lane would need 160 KB of LDS: use 2
  GS_TIMED("render_bwd", st, if (cd.tile == 8) GS_BWD(8, 1);
           else if (cd.tile == 16) {
             if (px == 4) GS_BWD(16, 4); else if (px == 2) GS_BWD(16, 2); else GS_BWD(16, 1);
           } else {
             if (px == 4) GS_BWD(32, 4); else GS_BWD(32, 2);
           });
#undef GS_BWD
  GS_CHECK_LAUNCH();
  return launch_preprocess_bwd(g, n, sh_degree, cd, grad2d, grads, accumulate, st);
}
