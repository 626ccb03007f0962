// Growth step of the multi-view score-guided densification (Eq. 4): every
// Gaussian whose score reaches the threshold is cloned (largest scale at
// most split_scale) or split in two (children at mu + R S eps_k, scales
// divided by 1.6, other attributes copied). Outputs keep index order:
// Gaussian i's one or two entries follow those of i - 1.
#include <math.h>

#include "common.h"
#include "sort.h"

namespace gs {

namespace {

// kind[i]: 0 keep, 1 clone, 2 split, 3 prune; cnt[i]: output entries of i.
// With a pruning score, the min and max of its (non-negative) values are in
// mm as IEEE bit patterns, and pruning takes precedence over growth.
__global__ void k_dens_plan(const uint32_t* __restrict__ score, const float* __restrict__ ls,
                            int64_t n, uint32_t thr, double split_scale,
                            const double* __restrict__ prune, double pthr,
                            const unsigned long long* __restrict__ mm,
                            uint32_t* __restrict__ cnt, uint32_t* __restrict__ kind) {
  double lo = 0.0, span = 0.0;
  if (prune) {
    lo = __longlong_as_double((long long)mm[0]);
    span = __longlong_as_double((long long)mm[1]) - lo;
  }
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    uint32_t k = 0;
    if (prune && (prune[i] - lo) > pthr * span) {
      k = 3;
    } else if (score[i] >= thr) {
      const double m = fmax(fmax(exp((double)ls[i]), exp((double)ls[n + i])), exp((double)ls[2 * n + i]));
      k = m > split_scale ? 2u : 1u;
    }
    kind[i] = k;
    cnt[i] = k == 3 ? 0u : (k ? 2u : 1u);
  }
}

__global__ void k_mm_init(unsigned long long* mm) {
  if (threadIdx.x == 0) {
    mm[0] = ~0ull;
    mm[1] = 0ull;
  }
}

// min and max of non-negative doubles through their bit patterns (which
// order like the values)
__global__ void __launch_bounds__(256) k_mm(const double* __restrict__ v, int64_t n,
                                            unsigned long long* __restrict__ mm) {
  unsigned long long lo = ~0ull, hi = 0ull;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v[i]);
    lo = b < lo ? b : lo;
    hi = b > hi ? b : hi;
  }
  for (int d = 1; d < kWave; d <<= 1) {
    const unsigned long long ol = __shfl_xor(lo, d, kWave), oh = __shfl_xor(hi, d, kWave);
    lo = ol < lo ? ol : lo;
    hi = oh > hi ? oh : hi;
  }
  if ((threadIdx.x & (kWave - 1)) == 0) {
    atomicMin(mm, lo);
    atomicMax(mm + 1, hi);
  }
}

struct DensArrays {
  const float *means, *ls, *quats, *op, *sh;
  float *o_means, *o_ls, *o_quats, *o_op, *o_sh;
};

__global__ void __launch_bounds__(256) k_dens_apply(DensArrays a, int64_t n, int sh_rows,
                                                    const float* __restrict__ eps,
                                                    const uint32_t* __restrict__ off,
                                                    const uint32_t* __restrict__ kind,
                                                    int64_t n_out, int moments) {
#pragma clang fp contract(off)
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t kd = kind[i];
    const int64_t base = off[i];
    const int c = kd == 3 ? 0 : (kd ? 2 : 1);
    if (base + c > n_out) continue;  // only for an inconsistent n_out
    double s[3], mu[3];
    for (int d = 0; d < 3; ++d) {
      s[d] = a.ls[d * n + i];
      mu[d] = a.means[d * n + i];
    }
    const bool split = kd == 2;
    for (int k = 0; k < c; ++k) {
      const int64_t o = base + k;
      // moments of new entries (a clone's copy, both split children) start at zero
      const bool zero = moments && (k == 1 || split);
      for (int d = 0; d < 4; ++d) a.o_quats[d * n_out + o] = zero ? 0.f : a.quats[d * n + i];
      a.o_op[o] = zero ? 0.f : a.op[i];
      for (int r = 0; r < sh_rows; ++r) a.o_sh[r * n_out + o] = zero ? 0.f : a.sh[r * n + i];
      if (split && !moments) {
        double q[4];
        for (int d = 0; d < 4; ++d) q[d] = a.quats[d * n + i];
        const double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
        const double w = q[0] / qn, x = q[1] / qn, y = q[2] / qn, z = q[3] / qn;
        const double R[9] = {1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y - w * z),
                             2.0 * (x * z + w * y),       2.0 * (x * y + w * z),
                             1.0 - 2.0 * (x * x + z * z), 2.0 * (y * z - w * x),
                             2.0 * (x * z - w * y),       2.0 * (y * z + w * x),
                             1.0 - 2.0 * (x * x + y * y)};
        double l[3];
        for (int d = 0; d < 3; ++d) l[d] = exp(s[d]) * (double)eps[(k * 3 + d) * n + i];
        for (int d = 0; d < 3; ++d) {
          const double step = (R[d * 3 + 0] * l[0] + R[d * 3 + 1] * l[1]) + R[d * 3 + 2] * l[2];
          a.o_means[d * n_out + o] = (float)(mu[d] + step);
          a.o_ls[d * n_out + o] = (float)(s[d] - log(1.6));
        }
      } else {
        for (int d = 0; d < 3; ++d) {
          a.o_means[d * n_out + o] = zero ? 0.f : a.means[d * n + i];
          a.o_ls[d * n_out + o] = zero ? 0.f : a.ls[d * n + i];
        }
      }
    }
  }
}

// Growth cap: histogram of min(score, GS_SCORE_BINS - 1) (the first
// kLdsBins bins privatised in LDS: scores are mostly small counts), then one
// block finds the smallest t >= t_min whose suffix count is within the cap.
constexpr int kLdsBins = 4096;

__global__ void k_zero_u32(uint32_t* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

__global__ void __launch_bounds__(256) k_score_hist(const uint32_t* __restrict__ score, int64_t n,
                                                    uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[kLdsBins];
  for (int b = threadIdx.x; b < kLdsBins; b += blockDim.x) h[b] = 0u;
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t b = min(score[i], (uint32_t)(GS_SCORE_BINS - 1));
    if (b < (uint32_t)kLdsBins) atomicAdd(&h[b], 1u);
    else atomicAdd(&hist[b], 1u);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < kLdsBins; b += blockDim.x)
    if (h[b]) atomicAdd(&hist[b], h[b]);
}

// One block of 1024 threads; thread k owns bins [k * 64, k * 64 + 64).
// suffix(t) = sum of hist[b] for b >= t = #{i : score_i >= t} for every
// t <= GS_SCORE_BINS - 1 (the top bin holds all larger scores).
__global__ void __launch_bounds__(1024) k_score_pick(const uint32_t* __restrict__ hist,
                                                     uint32_t t_min, uint64_t cap,
                                                     uint32_t* __restrict__ out) {
  constexpr int kPer = GS_SCORE_BINS / 1024;
  __shared__ uint64_t part[1024];
  __shared__ uint32_t best;
  const int k = threadIdx.x;
  const int lo = k * kPer;
  uint64_t mine = 0;
  for (int b = lo; b < lo + kPer; ++b) mine += hist[b];
  part[k] = mine;
  if (k == 0) best = 0xFFFFFFFFu;
  __syncthreads();
  // suffix sums over the threads' chunks (Hillis-Steele from the top)
  for (int d = 1; d < 1024; d <<= 1) {
    const uint64_t add = (k + d < 1024) ? part[k + d] : 0;
    __syncthreads();
    part[k] += add;
    __syncthreads();
  }
  // suffix at the start of this chunk = part[k]; walk the chunk upwards
  uint64_t suf = part[k];
  for (int b = lo; b < lo + kPer; ++b) {
    if ((uint32_t)b >= t_min && suf <= cap) {
      atomicMin(&best, (uint32_t)b);
      break;
    }
    suf -= hist[b];
  }
  __syncthreads();
  if (k == 0) out[0] = best;  // 0xFFFFFFFF: no threshold up to the top bin qualifies
}

// workspace: offsets [n], kinds [n], scan scratch, then (8-byte aligned) the
// pruning score's min and max
int64_t dens_mm_word(int64_t n) { return (2 * n + scan_tmp_words(n) + 1 + 1) & ~(int64_t)1; }
int64_t dens_ws_words(int64_t n) { return dens_mm_word(n) + 4; }

bool gauss_ok(const gs_gaussians* g) {
  return g && g->means && g->log_scales && g->quats && g->opacity_logits && g->sh;
}

}  // namespace

}  // namespace gs

using namespace gs;

extern "C" gs_status gs_densify_workspace(int64_t n, size_t* bytes) {
  if (n < 0 || n > 0xFFFFFFFEll / 2 || !bytes) return GS_EINVAL;
  *bytes = (size_t)dens_ws_words(n) * sizeof(uint32_t);
  return GS_OK;
}

extern "C" gs_status gs_densify_plan(const uint32_t* score, const float* log_scales, int64_t n,
                                     uint32_t threshold, float split_scale, void* workspace,
                                     size_t workspace_bytes, uint32_t* n_out, void* stream) {
  if (n < 0 || n > 0xFFFFFFFEll / 2 || !n_out || threshold == 0 || !(split_scale > 0.f) ||
      (n > 0 && (!score || !log_scales)))
    return GS_EINVAL;
  if (!workspace || workspace_bytes < (size_t)dens_ws_words(n) * sizeof(uint32_t))
    return GS_ECAPACITY;
  hipStream_t st = (hipStream_t)stream;
  uint32_t* off = (uint32_t*)workspace;
  if (n > 0) {
    const int blocks = (int)std::min<int64_t>(div_up(n, 256), 4096);
    k_dens_plan<<<blocks, 256, 0, st>>>(score, log_scales, n, threshold, (double)split_scale,
                                        nullptr, 0.0, nullptr, off, off + n);
    GS_CHECK_LAUNCH();
  }
  return scan_u32(off, off, n, n_out, off + 2 * n, st);
}

extern "C" gs_status gs_densify_prune_plan(const uint32_t* score, const float* log_scales,
                                           int64_t n, uint32_t threshold, float split_scale,
                                           const double* prune_score, double prune_threshold,
                                           void* workspace, size_t workspace_bytes,
                                           uint32_t* n_out, void* stream) {
  if (n < 0 || n > 0xFFFFFFFEll / 2 || !n_out || threshold == 0 || !(split_scale > 0.f) ||
      !(prune_threshold >= 0.0) || (n > 0 && (!score || !log_scales || !prune_score)))
    return GS_EINVAL;
  if (!workspace || workspace_bytes < (size_t)dens_ws_words(n) * sizeof(uint32_t))
    return GS_ECAPACITY;
  hipStream_t st = (hipStream_t)stream;
  uint32_t* off = (uint32_t*)workspace;
  if (n > 0) {
    unsigned long long* mm = (unsigned long long*)(off + dens_mm_word(n));
    const int blocks = (int)std::min<int64_t>(div_up(n, 256), 4096);
    k_mm_init<<<1, 64, 0, st>>>(mm);
    k_mm<<<std::min(blocks, 1024), 256, 0, st>>>(prune_score, n, mm);
    k_dens_plan<<<blocks, 256, 0, st>>>(score, log_scales, n, threshold, (double)split_scale,
                                        prune_score, prune_threshold, mm, off, off + n);
    GS_CHECK_LAUNCH();
  }
  return scan_u32(off, off, n, n_out, off + 2 * n, st);
}

extern "C" gs_status gs_densify_apply(const gs_gaussians* in, int64_t n, int32_t sh_degree,
                                      const float* eps, const void* workspace, int64_t n_out,
                                      int32_t moments, gs_gaussians* out, void* stream) {
  if (n < 0 || n > 0xFFFFFFFEll / 2 || n_out < 0 || n_out > 2 * n || sh_degree < 0 ||
      sh_degree > 3 || (moments != 0 && moments != 1))
    return GS_EINVAL;
  if (n == 0 || n_out == 0) return GS_OK;  // nothing to write (everything pruned)
  if (!gauss_ok(in) || !gauss_ok(out) || !workspace || (!moments && !eps)) return GS_EINVAL;
  const int sh_rows = 3 * (sh_degree + 1) * (sh_degree + 1);
  DensArrays a;
  a.means = in->means; a.ls = in->log_scales; a.quats = in->quats; a.op = in->opacity_logits;
  a.sh = in->sh;
  a.o_means = out->means; a.o_ls = out->log_scales; a.o_quats = out->quats;
  a.o_op = out->opacity_logits; a.o_sh = out->sh;
  const uint32_t* off = (const uint32_t*)workspace;
  hipStream_t st = (hipStream_t)stream;
  const int blocks = (int)std::min<int64_t>(div_up(n, 256), 4096);
  GS_TIMED("densify", st,
           k_dens_apply<<<blocks, 256, 0, st>>>(a, n, sh_rows, eps, off, off + n, n_out,
                                                moments));
  GS_CHECK_LAUNCH();
  return GS_OK;
}

extern "C" gs_status gs_densify_threshold(const uint32_t* score, int64_t n, uint32_t min_threshold,
                                          int64_t max_selected, uint32_t* scratch,
                                          uint32_t* threshold, void* stream) {
  if (n < 0 || max_selected < 0 || min_threshold == 0 ||
      min_threshold > (uint32_t)(GS_SCORE_BINS - 1) || !scratch || !threshold ||
      (n > 0 && !score))
    return GS_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  k_zero_u32<<<div_up(GS_SCORE_BINS, 256), 256, 0, st>>>(scratch, GS_SCORE_BINS);
  GS_CHECK_LAUNCH();
  if (n > 0) {
    const int blocks = (int)std::min<int64_t>(div_up(n, 256), 1024);
    k_score_hist<<<blocks, 256, 0, st>>>(score, n, scratch);
    GS_CHECK_LAUNCH();
  }
  k_score_pick<<<1, 1024, 0, st>>>(scratch, min_threshold, (uint64_t)max_selected, threshold);
  GS_CHECK_LAUNCH();
  return GS_OK;
}
