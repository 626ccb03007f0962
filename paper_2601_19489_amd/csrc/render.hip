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
// wavefront with DPP before a single atomic add per (splat, wavefront).
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
    const uint32_t* __restrict__ ranges, int64_t n, int W, int H, int tiles_x, float bg0,
    float bg1, float bg2, float* __restrict__ image, float* __restrict__ depth,
    float* __restrict__ T_final, uint32_t* __restrict__ n_contrib) {
  constexpr int NT = TILE * TILE;
  __shared__ float4 s0[NT], s1[NT], s2[NT];
  const int tile = blockIdx.x;
  const int tx = tile % tiles_x, ty = tile / tiles_x;
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

template <int TILE>
__global__ void __launch_bounds__(TILE* TILE) k_render_bwd(
    const float* __restrict__ splats, const uint32_t* __restrict__ vals,
    const uint32_t* __restrict__ ranges, int W, int H, int tiles_x, float bg0, float bg1,
    float bg2, const float* __restrict__ T_final, const uint32_t* __restrict__ n_contrib,
    const float* __restrict__ dL_dimage, const float* __restrict__ dL_ddepth,
    float* __restrict__ grad2d, int64_t n) {
  constexpr int NT = TILE * TILE;
  __shared__ float4 s0[NT], s1[NT], s2[NT];
  __shared__ uint32_t sid[NT];
  __shared__ uint32_t smax;
  const int tile = blockIdx.x;
  const int tx = tile % tiles_x, ty = tile / tiles_x;
  const int x = tx * TILE + (int)(threadIdx.x % TILE);
  const int y = ty * TILE + (int)(threadIdx.x / TILE);
  const bool inside = x < W && y < H;
  const float px = (float)x + 0.5f, py = (float)y + 0.5f;
  const uint32_t start = ranges[tile];
  const size_t p = (size_t)y * W + x, HW = (size_t)H * W;
  float T = 1.f, dC0 = 0.f, dC1 = 0.f, dC2 = 0.f, dD = 0.f;
  uint32_t nc = 0;
  if (inside) {
    T = T_final[p];
    nc = n_contrib[p];
    dC0 = dL_dimage[p];
    dC1 = dL_dimage[HW + p];
    dC2 = dL_dimage[2 * HW + p];
    if (dL_ddepth) dD = dL_ddepth[p];
  }
  if (threadIdx.x == 0) smax = 0;
  __syncthreads();
  if (nc) atomicMax(&smax, nc);
  __syncthreads();
  const uint32_t last = start + smax;
  // colour and depth of everything behind the current splat
  float S0 = T * bg0, S1 = T * bg1, S2 = T * bg2, SD = 0.f;
  const int lane = threadIdx.x & (kWave - 1);
  for (uint32_t bend = last; bend > start;) {
    const uint32_t bstart = bend - start > (uint32_t)NT ? bend - NT : start;
    __syncthreads();
    const uint32_t j = bstart + threadIdx.x;
    if (j < bend) {
      const uint32_t g = vals[j];
      if ((int64_t)g < n) {
        const float4* r = reinterpret_cast<const float4*>(splats + (size_t)g * GS_SPLAT_FLOATS);
        s0[threadIdx.x] = r[0];
        s1[threadIdx.x] = r[1];
        s2[threadIdx.x] = r[2];
        sid[threadIdx.x] = g;
      } else {  // never for a correct list: an empty splat with no gradient target
        s0[threadIdx.x] = make_float4(0.f, 0.f, 1.f, 0.f);
        s1[threadIdx.x] = make_float4(1.f, -1.f, 0.f, 0.f);
        s2[threadIdx.x] = make_float4(0.f, 0.f, 0.f, 0.f);
        sid[threadIdx.x] = 0xFFFFFFFFu;
      }
    }
    __syncthreads();
    for (int k = (int)(bend - bstart) - 1; k >= 0; --k) {
      const uint32_t pos = bstart + (uint32_t)k - start;  // position in the tile list
      const float4 a0 = s0[k], a1 = s1[k];
      bool act = pos < nc;
      SplatQ q;
      if (act) {
        q = eval_q(px, py, a0.x, a0.y, a0.z, a0.w + a0.w, a1.x);
        act = !splat_skips(q.Q, q.mag, a1.y, px, py, a0.x, a0.y, a0.z, a0.w, a1.x);
      }
      if (__ballot(act) == 0) continue;
      float gu = 0.f, gv = 0.f, ga = 0.f, gb = 0.f, gc = 0.f, go = 0.f;
      float gr = 0.f, gg = 0.f, gbc = 0.f, gz = 0.f;
      if (act) {
        const float4 a2 = s2[k];
        const float G = __expf(-0.5f * q.Q);
        const float oG = a1.z * G;
        const float al = fminf(kAlphaMax, oG);
        const float rinv = __builtin_amdgcn_rcpf(1.f - al);
        const float Tb = T * rinv;  // transmittance in front of this splat
        const float w = al * Tb;
        const float dal = rinv * (dC0 * (T * a2.x - S0) + dC1 * (T * a2.y - S1) +
                                  dC2 * (T * a2.z - S2) + dD * (T * a1.w - SD));
        gr = dC0 * w;
        gg = dC1 * w;
        gbc = dC2 * w;
        gz = dD * w;
        if (oG <= kAlphaMax) {
          go = dal * G;
          const float dQ = -0.5f * G * (dal * a1.z);
          gu = -2.f * dQ * (a0.z * q.dx + a0.w * q.dy);
          gv = -2.f * dQ * (a0.w * q.dx + a1.x * q.dy);
          ga = dQ * q.dx * q.dx;
          gb = 2.f * dQ * q.dx * q.dy;
          gc = dQ * q.dy * q.dy;
        }
        S0 = fmaf(a2.x, w, S0);
        S1 = fmaf(a2.y, w, S1);
        S2 = fmaf(a2.z, w, S2);
        SD = fmaf(a1.w, w, SD);
        T = Tb;
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
      if (lane == kWave - 1 && (int64_t)sid[k] < n) {
        float* dst = grad2d + sid[k];
        unsafeAtomicAdd(dst + 0 * n, gu);
        unsafeAtomicAdd(dst + 1 * n, gv);
        unsafeAtomicAdd(dst + 2 * n, ga);
        unsafeAtomicAdd(dst + 3 * n, gb);
        unsafeAtomicAdd(dst + 4 * n, gc);
        unsafeAtomicAdd(dst + 5 * n, go);
        unsafeAtomicAdd(dst + 6 * n, gr);
        unsafeAtomicAdd(dst + 7 * n, gg);
        unsafeAtomicAdd(dst + 8 * n, gbc);
        unsafeAtomicAdd(dst + 9 * n, gz);
      }
    }
    bend = bstart;
  }
}

__global__ void k_zero_f32(float* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.f;
}

gs_status launch_preprocess_bwd(const gs_gaussians* g, int64_t n, int deg, const CamDev& cam,
                                const float* grad2d, gs_gaussians* grads, int accumulate,
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
  k_render_fwd<TL><<<nt, TL * TL, 0, st>>>(splats, vals, ranges, n, cd.W, cd.H, cd.tiles_x, \
                                           bg[0], bg[1], bg[2], image, depth, T_final,    \
                                           n_contrib)
  if (cd.tile == 8) GS_FWD(8);
  else if (cd.tile == 16) GS_FWD(16);
  else GS_FWD(32);
#undef GS_FWD
  GS_CHECK_LAUNCH();
  return GS_OK;
}

extern "C" gs_status gs_render_bwd(const gs_gaussians* g, int64_t n, int32_t sh_degree,
                                   const gs_camera* cam, const float* splats,
                                   const uint32_t* vals, const uint32_t* ranges, const float* bg,
                                   const float* T_final, const uint32_t* n_contrib,
                                   const float* dL_dimage, const float* dL_ddepth, float* grad2d,
                                   gs_gaussians* grads, int32_t accumulate, void* stream) {
  CamDev cd;
  if (n < 0 || sh_degree < 0 || sh_degree > 3 || !make_cam(cam, &cd) || !ranges || !bg ||
      !T_final || !n_contrib || !dL_dimage || !grad2d || !g || !grads)
    return GS_EINVAL;
  if (n == 0) return GS_OK;
  hipStream_t st = (hipStream_t)stream;
  k_zero_f32<<<div_up(n * GS_GRAD2D_COMPONENTS, 256), 256, 0, st>>>(grad2d,
                                                                     n * GS_GRAD2D_COMPONENTS);
  GS_CHECK_LAUNCH();
  const int nt = cd.tiles_x * cd.tiles_y;
#define GS_BWD(TL)                                                                         \
  k_render_bwd<TL><<<nt, TL * TL, 0, st>>>(splats, vals, ranges, cd.W, cd.H, cd.tiles_x, \
                                           bg[0], bg[1], bg[2], T_final, n_contrib,       \
                                           dL_dimage, dL_ddepth, grad2d, n)
  if (cd.tile == 8) GS_BWD(8);
  else if (cd.tile == 16) GS_BWD(16);
  else GS_BWD(32);
#undef GS_BWD
  GS_CHECK_LAUNCH();
  return launch_preprocess_bwd(g, n, sh_degree, cd, grad2d, grads, accumulate, st);
}
