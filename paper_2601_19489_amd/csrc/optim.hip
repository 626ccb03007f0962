// L1 photometric loss with its gradient, and the fused Adam step.
#include <math.h>

#include "common.h"

namespace gs {

// loss_sum += sum |img - tgt| / n; grad = sign(img - tgt) / n.
__global__ void __launch_bounds__(256) k_l1(const float* __restrict__ img,
                                            const float* __restrict__ tgt, int64_t n, float inv_n,
                                            float* __restrict__ grad, float* __restrict__ loss) {
  __shared__ float part[256 / kWave];
  float acc = 0.f;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  // 16-byte loads and stores over the aligned whole quads, scalar for the rest
  const bool vec = (((uintptr_t)img | (uintptr_t)tgt | (uintptr_t)grad) & 15) == 0;
  const int64_t n4 = vec ? n / 4 : 0;
  const auto sg = [inv_n](float d) { return d > 0.f ? inv_n : (d < 0.f ? -inv_n : 0.f); };
  const auto quad = [&](float4 x, float4 y, int64_t i) {
    const float d0 = x.x - y.x, d1 = x.y - y.y, d2 = x.z - y.z, d3 = x.w - y.w;
    acc += (fabsf(d0) + fabsf(d1)) + (fabsf(d2) + fabsf(d3));
    reinterpret_cast<float4*>(grad)[i] = make_float4(sg(d0), sg(d1), sg(d2), sg(d3));
  };
  // four quads per thread in flight, then the rest one at a time
  constexpr int U = 4;
  int64_t i = t0;
  for (; i + (U - 1) * stride < n4; i += U * stride) {
    float4 x[U], y[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      x[u] = reinterpret_cast<const float4*>(img)[i + u * stride];
      y[u] = reinterpret_cast<const float4*>(tgt)[i + u * stride];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) quad(x[u], y[u], i + u * stride);
  }
  for (; i < n4; i += stride)
    quad(reinterpret_cast<const float4*>(img)[i], reinterpret_cast<const float4*>(tgt)[i], i);
  for (int64_t i = n4 * 4 + t0; i < n; i += stride) {
    const float d = img[i] - tgt[i];
    acc += fabsf(d);
    grad[i] = d > 0.f ? inv_n : (d < 0.f ? -inv_n : 0.f);
  }
  acc = wave_sum_to_last(acc);
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  if (lane == kWave - 1) part[w] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    float s = 0.f;
    for (int j = 0; j < 256 / kWave; ++j) s += part[j];
    unsafeAtomicAdd(loss, s * inv_n);
  }
}

// One pass over (p, g, m, v): bias-corrected Adam, FP32 state.
__global__ void __launch_bounds__(256) k_adam(float* __restrict__ p, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v,
                                              int64_t n, float b1, float b2, float eps, float ss,
                                              float rs) {
  const int64_t n4 = n / 4;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) {
    float4 P = reinterpret_cast<float4*>(p)[i];
    const float4 Gv = reinterpret_cast<const float4*>(g)[i];
    float4 M = reinterpret_cast<float4*>(m)[i];
    float4 V = reinterpret_cast<float4*>(v)[i];
    adam_update(P.x, M.x, V.x, Gv.x, b1, b2, eps, ss, rs);
    adam_update(P.y, M.y, V.y, Gv.y, b1, b2, eps, ss, rs);
    adam_update(P.z, M.z, V.z, Gv.z, b1, b2, eps, ss, rs);
    adam_update(P.w, M.w, V.w, Gv.w, b1, b2, eps, ss, rs);
    reinterpret_cast<float4*>(p)[i] = P;
    reinterpret_cast<float4*>(m)[i] = M;
    reinterpret_cast<float4*>(v)[i] = V;
  }
  for (int64_t i = n4 * 4 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    float pi = p[i], mi = m[i], vi = v[i];
    adam_update(pi, mi, vi, g[i], b1, b2, eps, ss, rs);
    p[i] = pi;
    m[i] = mi;
    v[i] = vi;
  }
}

// Eq. 3 error mask: e = (|r0-g0| + |r1-g1|) + |r2-g2| per pixel in FP32;
// minmax[0] / [1] receive min e / max e as IEEE bits (e >= 0, so the bits
// order like the values).
__global__ void k_err_init(uint32_t* minmax) {
  minmax[0] = 0x7F800000u;  // +inf
  minmax[1] = 0u;
}

__device__ __forceinline__ float pixel_err(const float* img, const float* tgt, int64_t i,
                                           int64_t hw) {
#pragma clang fp contract(off)
  return (fabsf(img[i] - tgt[i]) + fabsf(img[hw + i] - tgt[hw + i])) +
         fabsf(img[2 * hw + i] - tgt[2 * hw + i]);
}

__global__ void __launch_bounds__(256) k_err_minmax(const float* __restrict__ img,
                                                    const float* __restrict__ tgt, int64_t hw,
                                                    uint32_t* __restrict__ minmax) {
  uint32_t lo = 0x7F800000u, hi = 0u;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < hw;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t e = __float_as_uint(pixel_err(img, tgt, i, hw));
    lo = min(lo, e);
    hi = max(hi, e);
  }
  for (int d = 1; d < kWave; d <<= 1) {
    lo = min(lo, (uint32_t)__shfl_xor((int)lo, d, kWave));
    hi = max(hi, (uint32_t)__shfl_xor((int)hi, d, kWave));
  }
  // one pair of atomics per block: atomics on one address serialise in L2
  __shared__ uint32_t part[2][256 / kWave];
  const int w = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0) {
    part[0][w] = lo;
    part[1][w] = hi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < (int)blockDim.x / kWave; ++k) {
      lo = min(lo, part[0][k]);
      hi = max(hi, part[1][k]);
    }
    atomicMin(minmax, lo);
    atomicMax(minmax + 1, hi);
  }
}

__global__ void __launch_bounds__(256) k_err_mask(const float* __restrict__ img,
                                                  const float* __restrict__ tgt, int64_t hw,
                                                  float tau, const uint32_t* __restrict__ minmax,
                                                  uint8_t* __restrict__ mask) {
#pragma clang fp contract(off)
  const float mn = __uint_as_float(minmax[0]), mx = __uint_as_float(minmax[1]);
  const float thr = tau * (mx - mn);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < hw;
       i += (int64_t)gridDim.x * blockDim.x)
    mask[i] = (pixel_err(img, tgt, i, hw) - mn) > thr ? 1 : 0;
}

// Adam over up to GS_MAX_ADAM_GROUPS parameter groups in one launch, with
// the step count read from (and then advanced in) device memory, so that a
// captured graph replays correct bias corrections.
struct AdamGroups {
  float* p[GS_MAX_ADAM_GROUPS];
  const float* g[GS_MAX_ADAM_GROUPS];
  float* m[GS_MAX_ADAM_GROUPS];
  float* v[GS_MAX_ADAM_GROUPS];
  int64_t n[GS_MAX_ADAM_GROUPS];
  float lr[GS_MAX_ADAM_GROUPS];
  int blk0[GS_MAX_ADAM_GROUPS + 1];  // first block of each group
  int n_groups;
};

__global__ void __launch_bounds__(256) k_adam_grouped(AdamGroups G, float b1, float b2, float eps,
                                                      const int32_t* __restrict__ step) {
  __shared__ float sc[2];
  int k = 0;
  while (k + 1 < G.n_groups && (int)blockIdx.x >= G.blk0[k + 1]) ++k;
  if (threadIdx.x == 0) adam_scalars(*step, G.lr[k], b1, b2, sc[0], sc[1]);
  __syncthreads();
  const float ss = sc[0], rs = sc[1];
  float* __restrict__ p = G.p[k];
  const float* __restrict__ g = G.g[k];
  float* __restrict__ m = G.m[k];
  float* __restrict__ v = G.v[k];
  const int64_t n = G.n[k], n4 = n / 4;
  const int64_t nblk = G.blk0[k + 1] - G.blk0[k];
  const int64_t stride = nblk * blockDim.x;
  const int64_t first = (int64_t)(blockIdx.x - G.blk0[k]) * blockDim.x + threadIdx.x;
  for (int64_t i = first; i < n4; i += stride) {
    // streaming: every word is read and written once per step
    typedef float vf4 __attribute__((ext_vector_type(4)));
    const auto ld = [](const float* a, int64_t j) {
      const vf4 t = __builtin_nontemporal_load(reinterpret_cast<const vf4*>(a) + j);
      return make_float4(t.x, t.y, t.z, t.w);
    };
    const auto st = [](float* a, int64_t j, float4 t) {
      vf4 u = {t.x, t.y, t.z, t.w};
      __builtin_nontemporal_store(u, reinterpret_cast<vf4*>(a) + j);
    };
    float4 P = ld(p, i);
    const float4 Gv = ld(g, i);
    float4 M = ld(m, i);
    float4 V = ld(v, i);
    adam_update(P.x, M.x, V.x, Gv.x, b1, b2, eps, ss, rs);
    adam_update(P.y, M.y, V.y, Gv.y, b1, b2, eps, ss, rs);
    adam_update(P.z, M.z, V.z, Gv.z, b1, b2, eps, ss, rs);
    adam_update(P.w, M.w, V.w, Gv.w, b1, b2, eps, ss, rs);
    st(p, i, P);
    st(m, i, M);
    st(v, i, V);
  }
  for (int64_t i = n4 * 4 + first; i < n; i += stride) {
    float pi = p[i], mi = m[i], vi = v[i];
    adam_update(pi, mi, vi, g[i], b1, b2, eps, ss, rs);
    p[i] = pi;
    m[i] = mi;
    v[i] = vi;
  }
}

__global__ void k_step_advance(int32_t* step) { *step += 1; }

gs_status launch_step_advance(int32_t* step, hipStream_t st) {
  k_step_advance<<<1, 1, 0, st>>>(step);
  GS_CHECK_LAUNCH();
  return GS_OK;
}

}  // namespace gs

using namespace gs;

extern "C" gs_status gs_depth_l1_loss(const float* depth, const float* target, int64_t n,
                                      float weight, float* dL_ddepth, float* loss_sum,
                                      void* stream) {
  if (n < 0 || !(weight >= 0.f) || (n > 0 && (!depth || !target || !dL_ddepth || !loss_sum)))
    return GS_EINVAL;
  if (n == 0) return GS_OK;
  // few enough workgroups that their one atomic each on the loss does not
  // serialise into the kernel's time
  const int blocks = (int)std::min<int64_t>(div_up(n, 1024), 1024);
  GS_TIMED("l1_loss", (hipStream_t)stream,
           k_l1<<<blocks, 256, 0, (hipStream_t)stream>>>(depth, target, n, weight / (float)n,
                                                         dL_ddepth, loss_sum));
  GS_CHECK_LAUNCH();
  return GS_OK;
}

extern "C" gs_status gs_error_mask(const float* image, const float* target, int64_t n_pixels,
                                   float tau, uint8_t* mask, uint32_t* minmax, void* stream) {
  if (n_pixels < 0 || !(tau >= 0.f) ||
      (n_pixels > 0 && (!image || !target || !mask || !minmax)))
    return GS_EINVAL;
  if (n_pixels == 0) return GS_OK;
  hipStream_t st = (hipStream_t)stream;
  const int blocks = (int)std::min<int64_t>(div_up(n_pixels, 256), 1024);
  k_err_init<<<1, 1, 0, st>>>(minmax);
  GS_TIMED("error_mask", st,
           k_err_minmax<<<blocks, 256, 0, st>>>(image, target, n_pixels, minmax);
           k_err_mask<<<blocks, 256, 0, st>>>(image, target, n_pixels, tau, minmax, mask));
  GS_CHECK_LAUNCH();
  return GS_OK;
}


extern "C" gs_status gs_l1_loss(const float* image, const float* target, int64_t n,
                                float* dL_dimage, float* loss_sum, void* stream) {
  if (n < 0 || (n > 0 && (!image || !target || !dL_dimage || !loss_sum))) return GS_EINVAL;
  if (n == 0) return GS_OK;
  // few enough workgroups that their one atomic each on the loss does not
  // serialise into the kernel's time
  const int blocks = (int)std::min<int64_t>(div_up(n, 1024), 256);
  GS_TIMED("l1_loss", (hipStream_t)stream, k_l1<<<blocks, 256, 0, (hipStream_t)stream>>>(image, target, n, 1.f / (float)n, dL_dimage,
                                                loss_sum));
  GS_CHECK_LAUNCH();
  return GS_OK;
}

extern "C" gs_status gs_adam_step(float* p, const float* g, float* m, float* v, int64_t n,
                                  float lr, float beta1, float beta2, float eps, int32_t step,
                                  void* stream) {
  if (n < 0 || step < 1 || (n > 0 && (!p || !g || !m || !v))) return GS_EINVAL;
  if (n == 0) return GS_OK;
  if (!aligned16(p) || !aligned16(g) || !aligned16(m) || !aligned16(v)) return GS_EINVAL;
  float ss, rs;
  adam_scalars(step - 1, lr, beta1, beta2, ss, rs);
  const int blocks = (int)std::min<int64_t>(div_up((n + 3) / 4, 256), 8192);
  GS_TIMED("adam", (hipStream_t)stream,
           k_adam<<<blocks, 256, 0, (hipStream_t)stream>>>(p, g, m, v, n, beta1, beta2, eps, ss,
                                                            rs));
  GS_CHECK_LAUNCH();
  return GS_OK;
}

extern "C" gs_status gs_adam_step_grouped(const gs_adam_group* groups, int32_t n_groups,
                                          float beta1, float beta2, float eps, int32_t* step,
                                          void* stream) {
  if (!groups || n_groups < 1 || n_groups > GS_MAX_ADAM_GROUPS || !step) return GS_EINVAL;
  AdamGroups G;
  G.n_groups = n_groups;
  G.blk0[0] = 0;
  for (int k = 0; k < n_groups; ++k) {
    const gs_adam_group& a = groups[k];
    if (a.n < 0 || (a.n > 0 && (!a.p || !a.g || !a.m || !a.v))) return GS_EINVAL;
    if (a.n > 0 && (!aligned16(a.p) || !aligned16(a.g) || !aligned16(a.m) || !aligned16(a.v)))
      return GS_EINVAL;
    G.p[k] = a.p; G.g[k] = a.g; G.m[k] = a.m; G.v[k] = a.v; G.n[k] = a.n; G.lr[k] = a.lr;
    const int nb = a.n > 0 ? (int)std::min<int64_t>(div_up((a.n + 3) / 4, 256), 1 << 20) : 0;
    G.blk0[k + 1] = G.blk0[k] + nb;
  }
  hipStream_t st = (hipStream_t)stream;
  if (G.blk0[n_groups] > 0) {
    GS_TIMED("adam", st,
             k_adam_grouped<<<G.blk0[n_groups], 256, 0, st>>>(G, beta1, beta2, eps, step));
    GS_CHECK_LAUNCH();
  }
  k_step_advance<<<1, 1, 0, st>>>(step);
  GS_CHECK_LAUNCH();
  return GS_OK;
}
