// Photometric loss of Eq. 5 for one view, E = (1 - lambda) L1 + lambda
// (1 - SSIM), and its image gradient; the pruning-score accumulation of
// Eq. 6. SSIM per colour channel under an 11 x 11 Gaussian window (sigma
// 1.5, normalised) with zero padding, C1 = 0.01^2, C2 = 0.03^2; SSIM and L1
// are means over channels and pixels.
//
// Forward: one workgroup per 32 x 32 output tile of one channel. The 42 x 42
// input patch of both images goes to LDS, a horizontal 11-tap pass writes the
// five window sums (x, y, x^2, y^2, xy) per patch row and output column to
// LDS, and a vertical pass finishes them per pixel. With the gradient
// requested, each pixel also writes the three partials of its SSIM term with
// respect to the window's mean, second moment and cross moment of x; the
// backward correlates those maps with the same window (it is symmetric) and
// combines them with x and y at the pixel.
#include <math.h>

#include "common.h"

namespace gs {

namespace {

constexpr int kTile = 32;
constexpr int kRad = 5;
constexpr int kTaps = 2 * kRad + 1;
constexpr int kPatch = kTile + 2 * kRad;  // 42
constexpr float kC1 = 0.01f * 0.01f;
constexpr float kC2 = 0.03f * 0.03f;

struct Window {
  float w[kTaps];
};

// The block's sums of NQ per-thread values, written to out[q * n_blocks +
// block] (summed over the blocks in a fixed order afterwards).
template <int NQ>
__device__ __forceinline__ void block_sum_store(float (&v)[NQ], float* out, int64_t n_blocks,
                                                int64_t block, float* red) {
#pragma unroll
  for (int q = 0; q < NQ; ++q)
    for (int d = 1; d < kWave; d <<= 1) v[q] += __shfl_xor(v[q], d, kWave);
  const int w = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0)
    for (int q = 0; q < NQ; ++q) red[q * 4 + w] = v[q];
  __syncthreads();
  if (threadIdx.x < NQ) {
    const int q = threadIdx.x;
    out[q * n_blocks + block] =
        (red[q * 4 + 0] + red[q * 4 + 1]) + (red[q * 4 + 2] + red[q * 4 + 3]);
  }
}

__global__ void __launch_bounds__(256) k_photo_fwd(const float* __restrict__ img,
                                                   const float* __restrict__ tgt, int H, int W,
                                                   Window win, float* __restrict__ fmaps,
                                                   int64_t plane, float* __restrict__ parts) {
  __shared__ float px[kPatch][kPatch], py[kPatch][kPatch];
  __shared__ float hs[5][kPatch][kTile];
  __shared__ float red[8];
  const int x0 = blockIdx.x * kTile, y0 = blockIdx.y * kTile;
  const int64_t base = (int64_t)blockIdx.z * H * W;
  const int tid = threadIdx.x;
  for (int k = tid; k < kPatch * kPatch; k += 256) {
    const int r = k / kPatch, c = k % kPatch;
    const int gy = y0 + r - kRad, gx = x0 + c - kRad;
    const bool in = gy >= 0 && gy < H && gx >= 0 && gx < W;
    px[r][c] = in ? img[base + (int64_t)gy * W + gx] : 0.f;
    py[r][c] = in ? tgt[base + (int64_t)gy * W + gx] : 0.f;
  }
  __syncthreads();
  for (int k = tid; k < kPatch * kTile; k += 256) {
    const int r = k / kTile, j = k % kTile;
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f, s4 = 0.f;
#pragma unroll
    for (int t = 0; t < kTaps; ++t) {
      const float a = px[r][j + t], b = py[r][j + t], w = win.w[t];
      s0 = fmaf(w, a, s0);
      s1 = fmaf(w, b, s1);
      s2 = fmaf(w, a * a, s2);
      s3 = fmaf(w, b * b, s3);
      s4 = fmaf(w, a * b, s4);
    }
    hs[0][r][j] = s0; hs[1][r][j] = s1; hs[2][r][j] = s2; hs[3][r][j] = s3; hs[4][r][j] = s4;
  }
  __syncthreads();
  const int j = tid % kTile;
  float acc[2] = {0.f, 0.f};  // sum |x - y|, sum S
  for (int i = tid / kTile; i < kTile; i += 256 / kTile) {
    const int gy = y0 + i, gx = x0 + j;
    if (gy >= H || gx >= W) continue;
    float m[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < kTaps; ++t)
#pragma unroll
      for (int q = 0; q < 5; ++q) m[q] = fmaf(win.w[t], hs[q][i + t][j], m[q]);
    const float mx = m[0], my = m[1];
    const float vx = m[2] - mx * mx, vy = m[3] - my * my, cxy = m[4] - mx * my;
    const float A1 = 2.f * mx * my + kC1, A2 = 2.f * cxy + kC2;
    const float B1 = mx * mx + my * my + kC1, B2 = vx + vy + kC2;
    const float inv = 1.f / (B1 * B2);
    const float S = A1 * A2 * inv;
    acc[0] += fabsf(px[i + kRad][j + kRad] - py[i + kRad][j + kRad]);
    acc[1] += S;
    if (fmaps) {
      const float dmx = 2.f * my * A2 * inv - 2.f * mx * S / B1;
      const float dvx = -S / B2;
      const float dcxy = 2.f * A1 * inv;
      const int64_t p = base + (int64_t)gy * W + gx;
      fmaps[p] = dmx - 2.f * mx * dvx - my * dcxy;
      fmaps[plane + p] = dvx;
      fmaps[2 * plane + p] = dcxy;
    }
  }
  const int64_t nblk = (int64_t)gridDim.x * gridDim.y * gridDim.z;
  const int64_t blk = ((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
  block_sum_store<2>(acc, parts, nblk, blk, red);
}

// loss[0..2] = E, L1, SSIM from the per-block sums over n values (FP64,
// each thread a fixed stride of blocks, then a fixed-order tree).
__global__ void __launch_bounds__(256) k_photo_finish(const float* __restrict__ parts,
                                                      int64_t nblk, double n, float lambda,
                                                      float* __restrict__ loss) {
  __shared__ double red[2][256];
  double a = 0.0, b = 0.0;
  for (int64_t i = threadIdx.x; i < nblk; i += 256) {
    a += (double)parts[i];
    b += (double)parts[nblk + i];
  }
  red[0][threadIdx.x] = a;
  red[1][threadIdx.x] = b;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      red[0][threadIdx.x] += red[0][threadIdx.x + h];
      red[1][threadIdx.x] += red[1][threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double l1 = red[0][0] / n, s = red[1][0] / n;
    loss[0] = (float)((1.0 - lambda) * l1 + lambda * (1.0 - s));
    loss[1] = (float)l1;
    loss[2] = (float)s;
  }
}

__global__ void __launch_bounds__(256) k_photo_bwd(const float* __restrict__ img,
                                                   const float* __restrict__ tgt, int H, int W,
                                                   Window win, const float* __restrict__ fmaps,
                                                   int64_t plane, float wl1, float wssim,
                                                   float* __restrict__ grad) {
  __shared__ float pf[3][kPatch][kPatch];
  __shared__ float hs[3][kPatch][kTile];
  const int x0 = blockIdx.x * kTile, y0 = blockIdx.y * kTile;
  const int64_t base = (int64_t)blockIdx.z * H * W;
  const int tid = threadIdx.x;
  for (int k = tid; k < kPatch * kPatch; k += 256) {
    const int r = k / kPatch, c = k % kPatch;
    const int gy = y0 + r - kRad, gx = x0 + c - kRad;
    const bool in = gy >= 0 && gy < H && gx >= 0 && gx < W;
    const int64_t p = base + (int64_t)gy * W + gx;
#pragma unroll
    for (int q = 0; q < 3; ++q) pf[q][r][c] = in ? fmaps[q * plane + p] : 0.f;
  }
  __syncthreads();
  for (int k = tid; k < kPatch * kTile; k += 256) {
    const int r = k / kTile, j = k % kTile;
    float s[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < kTaps; ++t)
#pragma unroll
      for (int q = 0; q < 3; ++q) s[q] = fmaf(win.w[t], pf[q][r][j + t], s[q]);
#pragma unroll
    for (int q = 0; q < 3; ++q) hs[q][r][j] = s[q];
  }
  __syncthreads();
  const int j = tid % kTile;
  for (int i = tid / kTile; i < kTile; i += 256 / kTile) {
    const int gy = y0 + i, gx = x0 + j;
    if (gy >= H || gx >= W) continue;
    float g[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < kTaps; ++t)
#pragma unroll
      for (int q = 0; q < 3; ++q) g[q] = fmaf(win.w[t], hs[q][i + t][j], g[q]);
    const int64_t p = base + (int64_t)gy * W + gx;
    const float x = img[p], y = tgt[p];
    const float d = x - y;
    const float sgn = d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f);
    const float dssim = g[0] + 2.f * x * g[1] + y * g[2];
    grad[p] = wl1 * sgn - wssim * dssim;
  }
}

__global__ void k_prune_acc(const uint32_t* __restrict__ count, int64_t n,
                            const float* __restrict__ photo, double* __restrict__ prune,
                            uint32_t* __restrict__ split) {
  const double e = (double)photo[0];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t c = count[i];
    prune[i] += e * (double)c;
    if (split) split[i] += c;
  }
}

Window make_window() {
  Window w;
  double g[kTaps], s = 0.0;
  for (int t = 0; t < kTaps; ++t) {
    const double r = t - kRad;
    g[t] = exp(-r * r / (2.0 * 1.5 * 1.5));
    s += g[t];
  }
  for (int t = 0; t < kTaps; ++t) w.w[t] = (float)(g[t] / s);
  return w;
}

// per-block sums (2 floats per block) ahead of the SSIM partial maps
size_t parts_bytes(int32_t c, int32_t h, int32_t w) {
  const size_t nblk = (size_t)c * (size_t)div_up(h, kTile) * (size_t)div_up(w, kTile);
  return (2 * nblk * sizeof(float) + 255) / 256 * 256;
}

}  // namespace

}  // namespace gs

using namespace gs;

extern "C" gs_status gs_photo_loss_workspace(int32_t channels, int32_t height, int32_t width,
                                             size_t* bytes) {
  if (channels < 1 || height < 1 || width < 1 || !bytes) return GS_EINVAL;
  *bytes = parts_bytes(channels, height, width) +
           (size_t)3 * channels * height * width * sizeof(float);
  return GS_OK;
}

extern "C" gs_status gs_photo_loss(const float* image, const float* target, int32_t channels,
                                   int32_t height, int32_t width, float lambda, void* workspace,
                                   size_t workspace_bytes, float* loss, float* dL_dimage,
                                   void* stream) {
  if (channels < 1 || height < 1 || width < 1 || !(lambda >= 0.f && lambda <= 1.f) || !image ||
      !target || !loss || !workspace)
    return GS_EINVAL;
  const int64_t plane = (int64_t)channels * height * width;
  const size_t pb = parts_bytes(channels, height, width);
  const size_t need = pb + (dL_dimage ? (size_t)3 * plane * sizeof(float) : 0);
  if (workspace_bytes < need) return GS_ECAPACITY;
  hipStream_t st = (hipStream_t)stream;
  float* parts = (float*)workspace;
  float* fmaps = dL_dimage ? (float*)((char*)workspace + pb) : nullptr;
  const Window win = make_window();
  const dim3 grid(div_up(width, kTile), div_up(height, kTile), channels);
  const int64_t nblk = (int64_t)grid.x * grid.y * grid.z;
  GS_TIMED("photo_loss", st,
           k_photo_fwd<<<grid, 256, 0, st>>>(image, target, height, width, win, fmaps, plane,
                                             parts);
           k_photo_finish<<<1, 256, 0, st>>>(parts, nblk, (double)plane, lambda, loss);
           if (dL_dimage) k_photo_bwd<<<grid, 256, 0, st>>>(
               image, target, height, width, win, fmaps, plane,
               (float)((1.0 - lambda) / (double)plane), (float)(lambda / (double)plane),
               dL_dimage));
  GS_CHECK_LAUNCH();
  return GS_OK;
}

extern "C" gs_status gs_prune_accumulate(const uint32_t* count, int64_t n, const float* photo,
                                         double* prune_score, uint32_t* split_score,
                                         void* stream) {
  if (n < 0 || (n > 0 && (!count || !photo || !prune_score))) return GS_EINVAL;
  if (n == 0) return GS_OK;
  hipStream_t st = (hipStream_t)stream;
  const int blocks = (int)std::min<int64_t>(div_up(n, 256), 4096);
  k_prune_acc<<<blocks, 256, 0, st>>>(count, n, photo, prune_score, split_score);
  GS_CHECK_LAUNCH();
  return GS_OK;
}
