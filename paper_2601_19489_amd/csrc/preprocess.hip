// Per-Gaussian preprocess (Sec. 2.1, first step) and its backward (Sec. 2.2,
// per-Gaussian part), FP64 inside, FP32 in memory.
//
// Forward, per Gaussian (3DGS image formation model the paper builds on):
//   S = diag(exp s), q_hat = q/|q|, R = R(q_hat), Sigma = (RS)(RS)^T,
//   o = sigmoid(omega), p = W mu + t, culled if p_z <= near,
//   J = [[fx/pz, 0, -fx x'/pz], [0, fy/pz, -fy y'/pz]] with x', y' the
//   clamped ratios p_x/p_z, p_y/p_z (|.| <= 1.3 tan(fov/2)),
//   Sigma' = J W Sigma W^T J^T + 0.3 I, conic = Sigma'^-1,
//   (u, v) = f p_xy / p_z + c, z = p_z, colour from SH at the view
//   direction, t = 2 ln(255 o) (Eq. 1), and the number of tiles of the
//   compact tile set (Eq. 2 column walk).
// Direct mode (degree GS_DIRECT, the anchor decoder's output, Sec. 2.3):
// scale, opacity and RGB are taken as given, without exp, sigmoid or SH.
#include <math.h>

#include "common.h"
#include "sh.h"

namespace gs {

bool make_cam(const gs_camera* c, CamDev* d) {
  if (!c || c->width <= 0 || c->height <= 0 || !(c->fx > 0) || !(c->fy > 0)) return false;
  if (c->tile != 8 && c->tile != 16 && c->tile != 32) return false;
  if (!(c->near_plane > 0)) return false;
  if (c->depth_mode != GS_DEPTH_Z && c->depth_mode != GS_DEPTH_INVERSE) return false;
  d->inv_depth = c->depth_mode == GS_DEPTH_INVERSE;
  d->W = c->width;
  d->H = c->height;
  d->tile = c->tile;
  d->tiles_x = (c->width + c->tile - 1) / c->tile;
  d->tiles_y = (c->height + c->tile - 1) / c->tile;
  d->fx = c->fx; d->fy = c->fy; d->cx = c->cx; d->cy = c->cy;
  for (int i = 0; i < 9; ++i) d->R[i] = c->R[i];
  for (int i = 0; i < 3; ++i) d->t[i] = c->t[i];
  // camera centre -R^T t
  for (int j = 0; j < 3; ++j)
    d->campos[j] = -(c->R[0 * 3 + j] * c->t[0] + c->R[1 * 3 + j] * c->t[1] + c->R[2 * 3 + j] * c->t[2]);
  d->near_plane = c->near_plane;
  d->limx = 1.3 * ((double)c->width / (2.0 * c->fx));
  d->limy = 1.3 * ((double)c->height / (2.0 * c->fy));
  return true;
}

struct Proj {
  double scale[3], qn[4], qnorm, R[9], Sig[6];  // Sig: 00 01 02 11 12 22
  double o, p[3], xr, yr, J00, J02, J11, J12, T0[3], T1[3];
  double A, B, C, det;
  double dir[3], dnorm;
  bool visible;
};

__device__ __forceinline__ void quat_rot(const double* q, double* R) {
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  R[0] = 1.0 - 2.0 * (y * y + z * z); R[1] = 2.0 * (x * y - w * z); R[2] = 2.0 * (x * z + w * y);
  R[3] = 2.0 * (x * y + w * z); R[4] = 1.0 - 2.0 * (x * x + z * z); R[5] = 2.0 * (y * z - w * x);
  R[6] = 2.0 * (x * z - w * y); R[7] = 2.0 * (y * z + w * x); R[8] = 1.0 - 2.0 * (x * x + y * y);
}

__device__ __forceinline__ void project(const CamDev& cam, const double* mu, const double* ls,
                                        const double* q, double omega, bool direct, Proj& P) {
  for (int j = 0; j < 3; ++j) P.scale[j] = direct ? ls[j] : exp(ls[j]);
  P.qnorm = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  for (int j = 0; j < 4; ++j) P.qn[j] = q[j] / P.qnorm;
  quat_rot(P.qn, P.R);
  double M[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) M[i * 3 + j] = P.R[i * 3 + j] * P.scale[j];
  // Sigma = M M^T
  P.Sig[0] = M[0] * M[0] + M[1] * M[1] + M[2] * M[2];
  P.Sig[1] = M[0] * M[3] + M[1] * M[4] + M[2] * M[5];
  P.Sig[2] = M[0] * M[6] + M[1] * M[7] + M[2] * M[8];
  P.Sig[3] = M[3] * M[3] + M[4] * M[4] + M[5] * M[5];
  P.Sig[4] = M[3] * M[6] + M[4] * M[7] + M[5] * M[8];
  P.Sig[5] = M[6] * M[6] + M[7] * M[7] + M[8] * M[8];
  P.o = direct ? omega : 1.0 / (1.0 + exp(-omega));
  for (int i = 0; i < 3; ++i)
    P.p[i] = cam.R[i * 3 + 0] * mu[0] + cam.R[i * 3 + 1] * mu[1] + cam.R[i * 3 + 2] * mu[2] + cam.t[i];
  P.visible = P.p[2] > cam.near_plane;
  const double pz = P.visible ? P.p[2] : 1.0;
  P.xr = P.p[0] / pz;
  P.yr = P.p[1] / pz;
  const double xc = fmin(fmax(P.xr, -cam.limx), cam.limx);
  const double yc = fmin(fmax(P.yr, -cam.limy), cam.limy);
  P.J00 = cam.fx / pz;
  P.J02 = -cam.fx * xc / pz;
  P.J11 = cam.fy / pz;
  P.J12 = -cam.fy * yc / pz;
  // T = J W: row 0 = J00 W0 + J02 W2, row 1 = J11 W1 + J12 W2
  for (int k = 0; k < 3; ++k) {
    P.T0[k] = P.J00 * cam.R[0 * 3 + k] + P.J02 * cam.R[2 * 3 + k];
    P.T1[k] = P.J11 * cam.R[1 * 3 + k] + P.J12 * cam.R[2 * 3 + k];
  }
  // Sigma T0, Sigma T1
  double s0[3], s1[3];
  s0[0] = P.Sig[0] * P.T0[0] + P.Sig[1] * P.T0[1] + P.Sig[2] * P.T0[2];
  s0[1] = P.Sig[1] * P.T0[0] + P.Sig[3] * P.T0[1] + P.Sig[4] * P.T0[2];
  s0[2] = P.Sig[2] * P.T0[0] + P.Sig[4] * P.T0[1] + P.Sig[5] * P.T0[2];
  s1[0] = P.Sig[0] * P.T1[0] + P.Sig[1] * P.T1[1] + P.Sig[2] * P.T1[2];
  s1[1] = P.Sig[1] * P.T1[0] + P.Sig[3] * P.T1[1] + P.Sig[4] * P.T1[2];
  s1[2] = P.Sig[2] * P.T1[0] + P.Sig[4] * P.T1[1] + P.Sig[5] * P.T1[2];
  P.A = P.T0[0] * s0[0] + P.T0[1] * s0[1] + P.T0[2] * s0[2] + 0.3;
  P.B = P.T0[0] * s1[0] + P.T0[1] * s1[1] + P.T0[2] * s1[2];
  P.C = P.T1[0] * s1[0] + P.T1[1] * s1[1] + P.T1[2] * s1[2] + 0.3;
  P.det = P.A * P.C - P.B * P.B;
  if (!(P.det > 0.0)) P.visible = false;
  double d[3];
  for (int j = 0; j < 3; ++j) d[j] = mu[j] - cam.campos[j];
  P.dnorm = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  for (int j = 0; j < 3; ++j) P.dir[j] = d[j] / P.dnorm;
}

// Preprocess of the 256 Gaussians of one workgroup (block index `blk`)
// for one camera; every thread of the workgroup calls it.
template <bool SEQ>
__device__ __forceinline__ void preprocess_block(
    const float* __restrict__ means, const float* __restrict__ log_scales,
    const float* __restrict__ quats, const float* __restrict__ logits,
    const float* __restrict__ sh, int64_t n, int deg, const CamDev& cam, int64_t blk,
    float* __restrict__ splats, uint32_t* __restrict__ depth_keys,
    uint32_t* __restrict__ tile_counts, SnugLds* walk, uint32_t* cnt, uint32_t* cfirst,
    uint32_t* clast) {
  const int64_t i = blk * 256 + threadIdx.x;
  Snug s;
  bool has = false;
  float zf = 0.f;
  if (i < n) {
    double mu[3], ls[3], q[4];
    for (int j = 0; j < 3; ++j) mu[j] = means[j * n + i];
    for (int j = 0; j < 3; ++j) ls[j] = log_scales[j * n + i];
    for (int j = 0; j < 4; ++j) q[j] = quats[j * n + i];
    Proj P;
    project(cam, mu, ls, q, (double)logits[i], deg == GS_DIRECT, P);
    float4* out = reinterpret_cast<float4*>(splats + i * GS_SPLAT_FLOATS);
    if (!P.visible) {
      out[0] = make_float4(0.f, 0.f, 0.f, 0.f);
      out[1] = make_float4(0.f, 0.f, 0.f, 0.f);
      out[2] = make_float4(0.f, 0.f, 0.f, 0.f);
    } else {
      const double u = cam.fx * P.xr + cam.cx;
      const double v = cam.fy * P.yr + cam.cy;
      const double a = P.C / P.det, b = -P.B / P.det, c = P.A / P.det;
      double rgb[3];
      if (deg == GS_DIRECT) {
        for (int ch = 0; ch < 3; ++ch) rgb[ch] = (double)sh[(int64_t)ch * n + i];
      } else {
        double Y[16];
        sh_basis(deg, P.dir[0], P.dir[1], P.dir[2], Y);
        const int K = (deg + 1) * (deg + 1);
        for (int ch = 0; ch < 3; ++ch) {
          double acc = 0.0;
          for (int k = 0; k < K; ++k) acc += (double)sh[((int64_t)k * 3 + ch) * n + i] * Y[k];
          rgb[ch] = fmax(acc + 0.5, 0.0);
        }
      }
      const double t = 2.0 * log(255.0 * P.o);
      const float uf = (float)u, vf = (float)v, af = (float)a, bf = (float)b, cf = (float)c;
      const float tf = (float)t;
      zf = (float)P.p[2];
      const float dval = cam.inv_depth ? (float)(1.0 / P.p[2]) : zf;  // blended depth channel
      out[0] = make_float4(uf, vf, af, bf);
      out[1] = make_float4(cf, tf, (float)P.o, dval);
      out[2] = make_float4((float)rgb[0], (float)rgb[1], (float)rgb[2], 0.f);
      has = snug_setup(uf, vf, af, bf, cf, tf, s);
    }
  }
  // compact tile count, and the first and last columns holding tiles: the
  // column walk over the SnugBox, load-balanced
  cnt[threadIdx.x] = 0;
  cfirst[threadIdx.x] = 0xFFFFFFFFu;
  clast[threadIdx.x] = 0;
  const int wbase = threadIdx.x & ~(kWave - 1);
  column_walk<SEQ>(has, s, cam.tile, cam.tiles_x, cam.tiles_y, walk + wbase,
                   [&](int owner, int tx, int ty0, int ty1) {
                     if (ty1 >= ty0) {
                       atomicAdd(&cnt[wbase + owner], (uint32_t)(ty1 - ty0 + 1));
                       atomicMin(&cfirst[wbase + owner], (uint32_t)tx);
                       atomicMax(&clast[wbase + owner], (uint32_t)tx);
                     }
                   });
  if (i < n) {
    const uint32_t c = cnt[threadIdx.x];
    tile_counts[i] = c;
    depth_keys[i] = c ? __float_as_uint(zf) : 0xFFFFFFFFu;
    const uint32_t f = cfirst[threadIdx.x], l = clast[threadIdx.x];
    splats[i * GS_SPLAT_FLOATS + 11] = __uint_as_float(c ? f | ((l - f + 1) << 16) : 0u);
  }
}

// The SH degree is a template parameter so that the coefficient loops unroll
// and their loads issue together.
template <bool SEQ, int DEG>
__global__ void __launch_bounds__(256) k_preprocess(
    const float* __restrict__ means, const float* __restrict__ log_scales,
    const float* __restrict__ quats, const float* __restrict__ logits,
    const float* __restrict__ sh, int64_t n, CamDev cam, float* __restrict__ splats,
    uint32_t* __restrict__ depth_keys, uint32_t* __restrict__ tile_counts) {
  __shared__ SnugLds walk[256];
  __shared__ uint32_t cnt[256], cfirst[256], clast[256];
  preprocess_block<SEQ>(means, log_scales, quats, logits, sh, n, DEG, cam, blockIdx.x, splats,
                        depth_keys, tile_counts, walk, cnt, cfirst, clast);
}

// All views in one launch: blockIdx.y is the view.
struct PreBatch {
  CamDev cam[GS_MAX_VIEWS];
  float* splats[GS_MAX_VIEWS];
  uint32_t* depth_keys[GS_MAX_VIEWS];
  uint32_t* tile_counts[GS_MAX_VIEWS];
};

template <bool SEQ, int DEG>
__global__ void __launch_bounds__(256) k_preprocess_batched(
    const float* __restrict__ means, const float* __restrict__ log_scales,
    const float* __restrict__ quats, const float* __restrict__ logits,
    const float* __restrict__ sh, int64_t n, PreBatch pb) {
  __shared__ SnugLds walk[256];
  __shared__ uint32_t cnt[256], cfirst[256], clast[256];
  const int v = blockIdx.y;
  preprocess_block<SEQ>(means, log_scales, quats, logits, sh, n, DEG, pb.cam[v], blockIdx.x,
                        pb.splats[v], pb.depth_keys[v], pb.tile_counts[v], walk, cnt, cfirst,
                        clast);
}

// ---------------------------------------------------------------------------
// Backward: grad2d[n][10] = dL/d(u, v, a, b, c, o, r, g, b, z) -> parameters.
// The SH degree is a template parameter so that every per-coefficient array
// has a compile-time size and stays in registers.
//
// bwd_view computes one view's terms for Gaussian i and hands them to `out`:
// the colour-coefficient terms as they are formed (out.sh), the camera-side
// terms of a visible Gaussian (out.cam: dL/dp of the camera-space mean,
// dL/d(mu - campos) through the view direction, and dL/dSigma' as (A, B, C)
// partials), the geometry terms at the end (out.geo), and out.culled() when
// the projection rejects the Gaussian. Two sinks: MemOut writes (or adds) one view's terms to the
// gradient arrays; RegOut sums the terms of several views in registers, in
// the same FP32 order as one MemOut call per view with accumulation.
// The Gaussian's 80-byte grad2d record (five 16-byte loads; zero when
// `load` is false).
__device__ __forceinline__ void load_grad2d(const double* __restrict__ grad2d, int64_t i, bool load,
                                            double* g) {
  const double2* rec = reinterpret_cast<const double2*>(grad2d + (size_t)i * GS_GRAD2D_COMPONENTS);
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const double2 q = load ? rec[k] : make_double2(0.0, 0.0);
    g[2 * k] = q.x;
    g[2 * k + 1] = q.y;
  }
}

// Colour terms: SH coefficient gradients (out.sh, zero unless `vis`) and the
// view-direction term of the mean's gradient (gmu).
template <int DEG, class Out>
__device__ __forceinline__ void bwd_colour(const float* sh, int64_t n, int64_t i,
                                           const CamDev& cam, const double* mu, const double* g,
                                           bool vis, Out& out, double* gmu) {
  constexpr int deg = DEG;
  constexpr bool direct = DEG == GS_DIRECT;
  constexpr int K = direct ? 1 : (DEG + 1) * (DEG + 1);
  gmu[0] = gmu[1] = gmu[2] = 0.0;
  if (direct) {
    for (int ch = 0; ch < 3; ++ch) {
      if constexpr (Out::kParams) {
        float c0[1] = {sh[(int64_t)ch * n + i]};
        const float gv[1] = {vis ? (float)g[6 + ch] : 0.f};
        out.template sh_row<1>(ch, gv, c0);
      } else {
        out.sh(0, ch, vis ? (float)g[6 + ch] : 0.f, 0.f);
      }
    }
  } else {
    double d[3];
    for (int j = 0; j < 3; ++j) d[j] = mu[j] - cam.campos[j];
    const double dnorm = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    const double dir[3] = {d[0] / dnorm, d[1] / dnorm, d[2] / dnorm};
    double Y[16];
    sh_basis(deg, dir[0], dir[1], dir[2], Y);
    // one channel at a time, each coefficient read once: the colour (for the
    // clamp decision), the coefficient gradients, and the weights
    // w_k = sum_ch dL/drgb_ch sh_k,ch of the basis-gradient term
    double wk[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) wk[k] = 0.0;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      float c[K];
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        c[k] = sh[((int64_t)k * 3 + ch) * n + i];
        acc += (double)c[k] * Y[k];
      }
      const double gc = (acc + 0.5 < 0.0) ? 0.0 : g[6 + ch];
      float gv[K];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        wk[k] += gc * (double)c[k];
        gv[k] = vis ? (float)(gc * Y[k]) : 0.f;
      }
      if constexpr (Out::kParams) {
        out.template sh_row<K>(ch, gv, c);  // one batch of loads and stores per channel
      } else {
#pragma unroll
        for (int k = 0; k < K; ++k) out.sh(k, ch, gv[k], c[k]);
      }
    }
    double gdx, gdy, gdz;
    sh_basis_grad_dot(deg, dir[0], dir[1], dir[2], wk, gdx, gdy, gdz);
    const double dd = gdx * dir[0] + gdy * dir[1] + gdz * dir[2];
    gmu[0] = (gdx - dir[0] * dd) / dnorm;
    gmu[1] = (gdy - dir[1] * dd) / dnorm;
    gmu[2] = (gdz - dir[2] * dd) / dnorm;
  }
}

// Geometry terms, FP64: projects the Gaussian and, when it is visible, gives
// the camera-side terms to out.cam (gdir: the view-direction term of the
// mean's gradient, for that callback only), W^T dL/dp (wgp, the rest of the
// mean's gradient), and the log-scale, quaternion and opacity-logit
// gradients; all zero when it is not. ls, q and omega receive the
// parameters as read. Returns the projection's visibility.
template <int DEG, class Out>
__device__ __forceinline__ bool bwd_geometry(const float* log_scales, const float* quats,
                                             const float* logits, int64_t n,
                                             int64_t i, const CamDev& cam, const double* mu,
                                             const double* g, const double* gdir, Out& out,
                                             double* wgp, double* gls, double* gq, double& gom,
                                             double* ls, double* q, double& omega) {
  constexpr bool direct = DEG == GS_DIRECT;
  for (int j = 0; j < 3; ++j) ls[j] = log_scales[j * n + i];
  for (int j = 0; j < 4; ++j) q[j] = quats[j * n + i];
  omega = (double)logits[i];
  Proj P;
  project(cam, mu, ls, q, omega, direct, P);
  for (int j = 0; j < 3; ++j) gls[j] = wgp[j] = 0.0;
  for (int j = 0; j < 4; ++j) gq[j] = 0.0;
  gom = 0.0;
  if (!P.visible) return false;
  const double pz = P.p[2], px = P.p[0], py = P.p[1];
  // conic (a, b, c) = (C, -B, A) / det
  const double inv = 1.0 / P.det, inv2 = inv * inv;
  const double A = P.A, B = P.B, C = P.C;
  const double gA = -g[2] * C * C * inv2 + g[3] * B * C * inv2 + g[4] * (inv - A * C * inv2);
  const double gC = g[2] * (inv - A * C * inv2) + g[3] * A * B * inv2 - g[4] * A * A * inv2;
  const double gB = 2.0 * g[2] * B * C * inv2 + g[3] * (-inv - 2.0 * B * B * inv2) +
                    2.0 * g[4] * A * B * inv2;
  // A = T0 Sig T0, B = T0 Sig T1, C = T1 Sig T1
  const double* S = P.Sig;
  double s0[3], s1[3];
  s0[0] = S[0] * P.T0[0] + S[1] * P.T0[1] + S[2] * P.T0[2];
  s0[1] = S[1] * P.T0[0] + S[3] * P.T0[1] + S[4] * P.T0[2];
  s0[2] = S[2] * P.T0[0] + S[4] * P.T0[1] + S[5] * P.T0[2];
  s1[0] = S[0] * P.T1[0] + S[1] * P.T1[1] + S[2] * P.T1[2];
  s1[1] = S[1] * P.T1[0] + S[3] * P.T1[1] + S[4] * P.T1[2];
  s1[2] = S[2] * P.T1[0] + S[4] * P.T1[1] + S[5] * P.T1[2];
  double gT0[3], gT1[3];
  for (int k = 0; k < 3; ++k) {
    gT0[k] = 2.0 * gA * s0[k] + gB * s1[k];
    gT1[k] = 2.0 * gC * s1[k] + gB * s0[k];
  }
  // T rows from J and W
  const double* W = cam.R;
  const double gJ00 = gT0[0] * W[0] + gT0[1] * W[1] + gT0[2] * W[2];
  const double gJ02 = gT0[0] * W[6] + gT0[1] * W[7] + gT0[2] * W[8];
  const double gJ11 = gT1[0] * W[3] + gT1[1] * W[4] + gT1[2] * W[5];
  const double gJ12 = gT1[0] * W[6] + gT1[1] * W[7] + gT1[2] * W[8];
  double gp[3] = {0, 0, 0};
  const double pz2 = pz * pz, pz3 = pz2 * pz;
  gp[2] += -gJ00 * cam.fx / pz2 - gJ11 * cam.fy / pz2;
  if (fabs(P.xr) <= cam.limx) {
    gp[0] += -gJ02 * cam.fx / pz2;
    gp[2] += gJ02 * 2.0 * cam.fx * px / pz3;
  } else {
    const double xc = fmin(fmax(P.xr, -cam.limx), cam.limx);
    gp[2] += gJ02 * cam.fx * xc / pz2;
  }
  if (fabs(P.yr) <= cam.limy) {
    gp[1] += -gJ12 * cam.fy / pz2;
    gp[2] += gJ12 * 2.0 * cam.fy * py / pz3;
  } else {
    const double yc = fmin(fmax(P.yr, -cam.limy), cam.limy);
    gp[2] += gJ12 * cam.fy * yc / pz2;
  }
  // centroid and depth
  gp[0] += g[0] * cam.fx / pz;
  gp[1] += g[1] * cam.fy / pz;
  // the blended depth channel carries p_z, or 1 / p_z for an inverse-depth camera
  const double dval_dpz = cam.inv_depth ? -1.0 / pz2 : 1.0;
  gp[2] += -g[0] * cam.fx * px / pz2 - g[1] * cam.fy * py / pz2 + g[9] * dval_dpz;
  out.cam(P, cam, gp, gdir, gA, gB, gC);
  for (int j = 0; j < 3; ++j)
    wgp[j] = W[0 * 3 + j] * gp[0] + W[1 * 3 + j] * gp[1] + W[2 * 3 + j] * gp[2];
  // symmetric gradient of Sigma (GS_ij = dL/dSig_ij + dL/dSig_ji) times
  // M = R diag(scale): G_M = GS M
  double M[9];
  for (int r = 0; r < 3; ++r)
    for (int cc = 0; cc < 3; ++cc) M[r * 3 + cc] = P.R[r * 3 + cc] * P.scale[cc];
  double GR[9];
  for (int cc = 0; cc < 3; ++cc) {
    double gsc = 0.0;
    for (int r = 0; r < 3; ++r) {
      double gm = 0.0;
      for (int k = 0; k < 3; ++k) {
        const double GSrk = 2.0 * gA * P.T0[r] * P.T0[k] +
                            gB * (P.T0[r] * P.T1[k] + P.T1[r] * P.T0[k]) +
                            2.0 * gC * P.T1[r] * P.T1[k];
        gm += GSrk * M[k * 3 + cc];
      }
      gsc += gm * P.R[r * 3 + cc];
      GR[r * 3 + cc] = gm * P.scale[cc];
    }
    gls[cc] = direct ? gsc : gsc * P.scale[cc];
  }
  // R(q_hat) partials
  const double w = P.qn[0], x = P.qn[1], y = P.qn[2], z = P.qn[3];
  double gqn[4];
  gqn[0] = 2.0 * (-z * GR[1] + y * GR[2] + z * GR[3] - x * GR[5] - y * GR[6] + x * GR[7]);
  gqn[1] = 2.0 * (y * GR[1] + z * GR[2] + y * GR[3] - w * GR[5] + z * GR[6] + w * GR[7]) -
           4.0 * x * (GR[4] + GR[8]);
  gqn[2] = 2.0 * (x * GR[1] + w * GR[2] + x * GR[3] + z * GR[5] - w * GR[6] + z * GR[7]) -
           4.0 * y * (GR[0] + GR[8]);
  gqn[3] = 2.0 * (-w * GR[1] + x * GR[2] + w * GR[3] + y * GR[5] + x * GR[6] + y * GR[7]) -
           4.0 * z * (GR[0] + GR[4]);
  const double dotq = gqn[0] * w + gqn[1] * x + gqn[2] * y + gqn[3] * z;
  for (int j = 0; j < 4; ++j) gq[j] = (gqn[j] - P.qn[j] * dotq) / P.qnorm;
  gom = direct ? g[5] : g[5] * P.o * (1.0 - P.o);
  return true;
}

// One view, colour terms first: they are formed before the projection state
// is built, so that the two never occupy registers together; a Gaussian the
// projection then rejects after the near-plane test passed has its colour
// terms undone (out.culled()). (det <= 0 cannot happen for finite inputs
// because of the 0.3 dilation.)
template <int DEG, class Out>
__device__ __forceinline__ void bwd_view(const float* __restrict__ means,
                                         const float* __restrict__ log_scales,
                                         const float* __restrict__ quats,
                                         const float* __restrict__ logits,
                                         const float* __restrict__ sh, int64_t n, int64_t i,
                                         const CamDev& cam, const double* __restrict__ grad2d,
                                         Out& out) {
  double mu[3];
  for (int j = 0; j < 3; ++j) mu[j] = means[j * n + i];
  const double pz_chk = cam.R[6] * mu[0] + cam.R[7] * mu[1] + cam.R[8] * mu[2] + cam.t[2];
  const bool vis_guess = pz_chk > cam.near_plane;  // refined by the projection below
  double g[10];
  load_grad2d(grad2d, i, vis_guess, g);
  double gmu[3];
  bwd_colour<DEG>(sh, n, i, cam, mu, g, vis_guess, out, gmu);
  double wgp[3], gls[3], gq[4], gom, ls[3], q[4], omega;
  if (bwd_geometry<DEG>(log_scales, quats, logits, n, i, cam, mu, g, gmu, out, wgp, gls, gq, gom,
                        ls, q, omega)) {
    for (int j = 0; j < 3; ++j) gmu[j] += wgp[j];
  } else {
    gmu[0] = gmu[1] = gmu[2] = 0.0;
    if (vis_guess) out.culled();
  }
  out.geo(gmu, gls, gq, gom);
}

// One view's terms straight to the gradient arrays (written, or added when
// `accumulate`).
template <int DEG>
struct MemOut {
  static constexpr int K = DEG == GS_DIRECT ? 1 : (DEG + 1) * (DEG + 1);
  float *g_means, *g_ls, *g_quats, *g_logits, *g_sh;
  int64_t n, i;
  int accumulate;
  static constexpr bool kParams = false;  // sh() ignores the coefficient value
  __device__ void sh(int k, int ch, float gv, float) {
    const int64_t o = ((int64_t)k * 3 + ch) * n + i;
    if (accumulate) g_sh[o] += gv; else g_sh[o] = gv;
  }
  __device__ void culled() {
    if (!accumulate)
      for (int k = 0; k < K; ++k)
        for (int ch = 0; ch < 3; ++ch) g_sh[((int64_t)k * 3 + ch) * n + i] = 0.f;
  }
  __device__ void cam(const Proj&, const CamDev&, const double*, const double*, double, double,
                      double) {}
  __device__ void geo(const double* gmu, const double* gls, const double* gq, double gom) {
    if (accumulate) {
      for (int j = 0; j < 3; ++j) g_means[j * n + i] += (float)gmu[j];
      for (int j = 0; j < 3; ++j) g_ls[j * n + i] += (float)gls[j];
      for (int j = 0; j < 4; ++j) g_quats[j * n + i] += (float)gq[j];
      g_logits[i] += (float)gom;
    } else {
      for (int j = 0; j < 3; ++j) g_means[j * n + i] = (float)gmu[j];
      for (int j = 0; j < 3; ++j) g_ls[j * n + i] = (float)gls[j];
      for (int j = 0; j < 4; ++j) g_quats[j * n + i] = (float)gq[j];
      g_logits[i] = (float)gom;
    }
  }
};

// Sums over views, kept in LDS (one column of the block's array per thread:
// conflict-free, and the registers stay free for the FP64 projection state):
// rows 0..3K-1 the colour coefficients, then means (3), log-scales (3),
// quaternion (4) and opacity logit (1). The FP32 additions happen in the same
// order as one MemOut call per view with accumulation. A Gaussian the
// projection rejects in a view has a zero image-space gradient there (the
// compositing never reads it), so its colour terms in that view are zero and
// culled() has nothing to undo.
template <int DEG>
struct SumOut {
  static constexpr int K = MemOut<DEG>::K;
  static constexpr int kBlock = 256;
  static constexpr int kRows = 3 * K + 11;
  static constexpr int kMu = 3 * K, kLs = kMu + 3, kQ = kLs + 3, kO = kQ + 4;
  float* s;  // this thread's column: row r at s[r * kBlock]
  __device__ float& at(int r) { return s[r * kBlock]; }
  static constexpr bool kParams = false;
  __device__ void sh(int k, int ch, float gv, float) { at(k * 3 + ch) += gv; }
  __device__ void culled() {}
  __device__ void cam(const Proj&, const CamDev&, const double*, const double*, double, double,
                      double) {}
  __device__ void geo(const double* gmu, const double* gls, const double* gq, double gom) {
    for (int j = 0; j < 3; ++j) at(kMu + j) += (float)gmu[j];
    for (int j = 0; j < 3; ++j) at(kLs + j) += (float)gls[j];
    for (int j = 0; j < 4; ++j) at(kQ + j) += (float)gq[j];
    at(kO) += (float)gom;
  }
};

template <int DEG>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 8))) k_preprocess_bwd(
    const float* __restrict__ means, const float* __restrict__ log_scales,
    const float* __restrict__ quats, const float* __restrict__ logits,
    const float* __restrict__ sh, int64_t n, CamDev cam,
    const double* __restrict__ grad2d, float* __restrict__ g_means, float* __restrict__ g_ls,
    float* __restrict__ g_quats, float* __restrict__ g_logits, float* __restrict__ g_sh,
    int accumulate) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  MemOut<DEG> out{g_means, g_ls, g_quats, g_logits, g_sh, n, i, accumulate};
  bwd_view<DEG>(means, log_scales, quats, logits, sh, n, i, cam, grad2d, out);
}

// The backward fused with the optimiser step (one view, gradients not
// accumulated): every parameter takes its bias-corrected Adam update as soon
// as its gradient is final, so the gradients are never written out and the
// parameters are read once. The geometry terms come first here, so that the
// visibility is known before the colour terms are formed (their Adam updates
// cannot be undone); the gradients, and so the updated p, m, v, equal those of
// bwd_view with MemOut followed by k_adam_grouped bit for bit: a Gaussian the
// projection rejects gets zero colour terms, as culled() gives there.
struct AdamArgs {
  float* p[5];  // parameters, moments: means, log_scales, quats, opacity_logits, sh
  float* m[5];
  float* v[5];
  float lr[5];
  float b1, b2, eps;
  const int32_t* step;  // steps taken before this one
};

template <int DEG>
struct AdamOut {
  static constexpr bool kParams = true;  // takes the parameter values, row by row
  const AdamArgs* a;
  const float* ss;  // per group: lr / (1 - b1^t)
  float rs;         // 1 / sqrt(1 - b2^t)
  int64_t n, i;
  // Adam on R parameters of group grp at rows o[r] of this Gaussian: every
  // moment is loaded before the first update, every result stored after the
  // last, so the loads of a row are in flight together.
  template <int R>
  __device__ void step_rows(int grp, const int64_t* o, const float* gv, const float* pv) {
    float* __restrict__ pp = a->p[grp];
    float* __restrict__ mm = a->m[grp];
    float* __restrict__ vv = a->v[grp];
    float P[R], M[R], V[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      M[r] = mm[o[r]];
      V[r] = vv[o[r]];
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      P[r] = pv[r];
      adam_update(P[r], M[r], V[r], gv[r], a->b1, a->b2, a->eps, ss[grp], rs);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      pp[o[r]] = P[r];
      mm[o[r]] = M[r];
      vv[o[r]] = V[r];
    }
  }
  template <int K>
  __device__ void sh_row(int ch, const float* gv, const float* pv) {
    int64_t o[K];
#pragma unroll
    for (int k = 0; k < K; ++k) o[k] = ((int64_t)k * 3 + ch) * n + i;
    step_rows<K>(4, o, gv, pv);
  }
  __device__ void culled() {}
  __device__ void cam(const Proj&, const CamDev&, const double*, const double*, double, double,
                      double) {}
  __device__ void shape(const double* gls, const double* gq, double gom, const double* ls,
                        const double* q, double omega) {
    int64_t o[4];
    float gv[4], pv[4];
    for (int j = 0; j < 3; ++j) {
      o[j] = j * n + i;
      gv[j] = (float)gls[j];
      pv[j] = (float)ls[j];
    }
    step_rows<3>(1, o, gv, pv);
    for (int j = 0; j < 4; ++j) {
      o[j] = j * n + i;
      gv[j] = (float)gq[j];
      pv[j] = (float)q[j];
    }
    step_rows<4>(2, o, gv, pv);
    o[0] = i;
    gv[0] = (float)gom;
    pv[0] = (float)omega;
    step_rows<1>(3, o, gv, pv);
  }
  __device__ void mean(const double* gmu, const double* mu) {
    int64_t o[3];
    float gv[3], pv[3];
    for (int j = 0; j < 3; ++j) {
      o[j] = j * n + i;
      gv[j] = (float)gmu[j];
      pv[j] = (float)mu[j];
    }
    step_rows<3>(0, o, gv, pv);
  }
};

template <int DEG>
__device__ __forceinline__ void bwd_view_adam(int64_t n, int64_t i, const CamDev& cam,
                                              const double* __restrict__ grad2d,
                                              AdamOut<DEG>& out) {
  const AdamArgs& A = *out.a;
  double mu[3];
  for (int j = 0; j < 3; ++j) mu[j] = A.p[0][j * n + i];
  const double pz_chk = cam.R[6] * mu[0] + cam.R[7] * mu[1] + cam.R[8] * mu[2] + cam.t[2];
  const bool vis_guess = pz_chk > cam.near_plane;
  double g[10];
  load_grad2d(grad2d, i, vis_guess, g);
  const double gdir[3] = {0.0, 0.0, 0.0};  // out.cam does nothing here
  double wgp[3];
  bool visible;
  {
    double gls[3], gq[4], gom, ls[3], q[4], omega;
    visible = bwd_geometry<DEG>(A.p[1], A.p[2], A.p[3], n, i, cam, mu, g, gdir, out, wgp, gls,
                                gq, gom, ls, q, omega);
    out.shape(gls, gq, gom, ls, q, omega);
  }
  double gmu[3];
  bwd_colour<DEG>(A.p[4], n, i, cam, mu, g, visible, out, gmu);
  for (int j = 0; j < 3; ++j) gmu[j] = visible ? gmu[j] + wgp[j] : 0.0;
  out.mean(gmu, mu);
}

template <int DEG>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 8)))
k_preprocess_bwd_adam(int64_t n, CamDev cam, const double* __restrict__ grad2d, AdamArgs A) {
  __shared__ float sc[6];
  if (threadIdx.x < 5) {
    float r;
    adam_scalars(*A.step, A.lr[threadIdx.x], A.b1, A.b2, sc[threadIdx.x], r);
    if (threadIdx.x == 0) sc[5] = r;
  }
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  AdamOut<DEG> out{&A, sc, sc[5], n, i};
  bwd_view_adam<DEG>(n, i, cam, grad2d, out);
}

// Several views in one pass: each thread sums its Gaussian's terms over the
// views and writes the gradients once.
struct BwdViews {
  CamDev cam[GS_MAX_VIEWS];
  const double* grad2d[GS_MAX_VIEWS];
  int n_views;
};

template <int DEG>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 8)))
k_preprocess_bwd_views(const float* __restrict__ means, const float* __restrict__ log_scales,
                       const float* __restrict__ quats, const float* __restrict__ logits,
                       const float* __restrict__ sh, int64_t n, BwdViews bv,
                       float* __restrict__ g_means, float* __restrict__ g_ls,
                       float* __restrict__ g_quats, float* __restrict__ g_logits,
                       float* __restrict__ g_sh, int accumulate) {
  using S = SumOut<DEG>;
  constexpr int K = S::K, B = S::kBlock;
  __shared__ float acc[S::kRows * B];
  const int64_t i = (int64_t)blockIdx.x * B + threadIdx.x;
  if (i >= n) return;
  S out;
  out.s = acc + threadIdx.x;
  float* const gsrc[5] = {g_sh, g_means, g_ls, g_quats, g_logits};
  const int first[5] = {0, S::kMu, S::kLs, S::kQ, S::kO};
  const int rows[5] = {3 * K, 3, 3, 4, 1};
#pragma unroll
  for (int a = 0; a < 5; ++a)
#pragma unroll
    for (int r = 0; r < rows[a]; ++r) out.at(first[a] + r) = accumulate ? gsrc[a][r * n + i] : 0.f;
#pragma unroll 1
  for (int v = 0; v < bv.n_views; ++v) {
    // Re-read the parameters in every view (they stay in cache), with their
    // addresses recomputed, rather than letting the compiler hoist either out
    // of the loop: held across views they push the projection state out of
    // registers.
    const float *pm = means, *pl = log_scales, *pq = quats, *po = logits, *ps = sh;
    int64_t nv = n;
    asm volatile("" : "+s"(pm), "+s"(pl), "+s"(pq), "+s"(po), "+s"(ps), "+s"(nv));
    bwd_view<DEG>(pm, pl, pq, po, ps, nv, i, bv.cam[v], bv.grad2d[v], out);
  }
#pragma unroll
  for (int a = 0; a < 5; ++a)
#pragma unroll
    for (int r = 0; r < rows[a]; ++r) gsrc[a][r * n + i] = out.at(first[a] + r);
}

// Camera pose gradient (global pose refinement): the correction acts on the
// world-to-camera transform from the left, p' = exp([w]x) p + d. Per visible
// Gaussian, with g_p = dL/dp, g_dir = dL/d(mu - campos) and
// G_c = J^T dL/dSigma' J:
//   dL/dd += g_p + R g_dir
//   dL/dw += p x g_p + (tr(G_c (E_k S_c - S_c E_k)))_k,  S_c = R Sigma R^T,
// E_k the cross-product matrix of the k-th axis. Only the camera-side
// callback does work; the parameter-gradient callbacks are empty.
struct PoseOut {
  double acc[6];
  static constexpr bool kParams = false;
  __device__ void sh(int, int, float, float) {}
  __device__ void culled() {}
  __device__ void geo(const double*, const double*, const double*, double) {}
  __device__ void cam(const Proj& P, const CamDev& cam, const double* gp, const double* gdir,
                      double gA, double gB, double gC) {
    const double* W = cam.R;
    for (int j = 0; j < 3; ++j)
      acc[3 + j] += gp[j] + (W[j * 3 + 0] * gdir[0] + W[j * 3 + 1] * gdir[1] +
                             W[j * 3 + 2] * gdir[2]);
    const double* p = P.p;
    acc[0] += p[1] * gp[2] - p[2] * gp[1];
    acc[1] += p[2] * gp[0] - p[0] * gp[2];
    acc[2] += p[0] * gp[1] - p[1] * gp[0];
    // G_c = J^T G J with G = [[gA, gB / 2], [gB / 2, gC]], J rows (J00, 0, J02), (0, J11, J12)
    const double J0[3] = {P.J00, 0.0, P.J02}, J1[3] = {0.0, P.J11, P.J12};
    double Gc[3][3], Sc[3][3], S3[3][3], WS[3][3];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b)
        Gc[a][b] = gA * J0[a] * J0[b] + 0.5 * gB * (J0[a] * J1[b] + J1[a] * J0[b]) +
                   gC * J1[a] * J1[b];
    const double* S = P.Sig;  // 00 01 02 11 12 22
    S3[0][0] = S[0]; S3[0][1] = S3[1][0] = S[1]; S3[0][2] = S3[2][0] = S[2];
    S3[1][1] = S[3]; S3[1][2] = S3[2][1] = S[4]; S3[2][2] = S[5];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b)
        WS[a][b] = W[a * 3 + 0] * S3[0][b] + W[a * 3 + 1] * S3[1][b] + W[a * 3 + 2] * S3[2][b];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b)
        Sc[a][b] = WS[a][0] * W[b * 3 + 0] + WS[a][1] * W[b * 3 + 1] + WS[a][2] * W[b * 3 + 2];
    // E_k v = e_k x v; M_k = E_k S_c - S_c E_k is symmetric, so
    // tr(G_c M_k) = sum_ab G_c[a][b] M_k[a][b]
    for (int k = 0; k < 3; ++k) {
      double E[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
      const int k1 = (k + 1) % 3, k2 = (k + 2) % 3;
      E[k2][k1] = 1.0;   // [e_k]x: (e_k x v)_k2 = v_k1, (e_k x v)_k1 = -v_k2
      E[k1][k2] = -1.0;
      double t = 0.0;
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
          double m = 0.0;
          for (int c = 0; c < 3; ++c) m += E[a][c] * Sc[c][b] - Sc[a][c] * E[c][b];
          t += Gc[a][b] * m;
        }
      acc[k] += t;
    }
  }
};

template <int DEG>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 8))) k_pose_grad(
    const float* __restrict__ means, const float* __restrict__ log_scales,
    const float* __restrict__ quats, const float* __restrict__ logits,
    const float* __restrict__ sh, int64_t n, CamDev cam, const double* __restrict__ grad2d,
    double* __restrict__ pose) {
  __shared__ double red[6][4];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  PoseOut out;
  for (int k = 0; k < 6; ++k) out.acc[k] = 0.0;
  if (i < n) bwd_view<DEG>(means, log_scales, quats, logits, sh, n, i, cam, grad2d, out);
  for (int k = 0; k < 6; ++k)
    for (int d = 1; d < kWave; d <<= 1) out.acc[k] += __shfl_xor(out.acc[k], d, kWave);
  const int w = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0)
    for (int k = 0; k < 6; ++k) red[k][w] = out.acc[k];
  __syncthreads();
  if (threadIdx.x < 6) {
    const int k = threadIdx.x;
    atomicAdd(pose + k, (red[k][0] + red[k][1]) + (red[k][2] + red[k][3]));
  }
}

gs_status launch_preprocess_bwd(const gs_gaussians* g, int64_t n, int deg, const CamDev& cam,
                                const double* grad2d, gs_gaussians* grads, int accumulate,
                                hipStream_t st) {
  if (n == 0) return GS_OK;
#define GS_PBWD(D)                                                                           \
  k_preprocess_bwd<D><<<div_up(n, 256), 256, 0, st>>>(                                     \
      g->means, g->log_scales, g->quats, g->opacity_logits, g->sh, n, cam, grad2d, grads->means, \
      grads->log_scales, grads->quats, grads->opacity_logits, grads->sh, accumulate)
  GS_TIMED("preprocess_bwd", st,
           switch (deg) {
             case GS_DIRECT: GS_PBWD(GS_DIRECT); break;
             case 0: GS_PBWD(0); break;
             case 1: GS_PBWD(1); break;
             case 2: GS_PBWD(2); break;
             default: GS_PBWD(3); break;
           });
#undef GS_PBWD
  GS_CHECK_LAUNCH();
  return GS_OK;
}

gs_status launch_preprocess_bwd_adam(gs_gaussians* g, int64_t n, int deg, const CamDev& cam,
                                     const double* grad2d, const gs_adam_params* adam,
                                     hipStream_t st) {
  if (n == 0) return GS_OK;
  AdamArgs A;
  float* const p[5] = {g->means, g->log_scales, g->quats, g->opacity_logits, g->sh};
  float* const m[5] = {adam->m.means, adam->m.log_scales, adam->m.quats, adam->m.opacity_logits,
                       adam->m.sh};
  float* const v[5] = {adam->v.means, adam->v.log_scales, adam->v.quats, adam->v.opacity_logits,
                       adam->v.sh};
  for (int k = 0; k < 5; ++k) {
    A.p[k] = p[k];
    A.m[k] = m[k];
    A.v[k] = v[k];
    A.lr[k] = adam->lr[k];
  }
  A.b1 = adam->beta1;
  A.b2 = adam->beta2;
  A.eps = adam->eps;
  A.step = adam->step;
#define GS_PBWDA(D) k_preprocess_bwd_adam<D><<<div_up(n, 256), 256, 0, st>>>(n, cam, grad2d, A)
  GS_TIMED("preprocess_bwd_adam", st,
           switch (deg) {
             case GS_DIRECT: GS_PBWDA(GS_DIRECT); break;
             case 0: GS_PBWDA(0); break;
             case 1: GS_PBWDA(1); break;
             case 2: GS_PBWDA(2); break;
             default: GS_PBWDA(3); break;
           });
#undef GS_PBWDA
  GS_CHECK_LAUNCH();
  return GS_OK;
}

gs_status launch_preprocess_bwd_views(const gs_gaussians* g, int64_t n, int deg,
                                      const CamDev* cams, const double* const* grad2d,
                                      int n_views, gs_gaussians* grads, int accumulate,
                                      hipStream_t st) {
  if (n == 0) return GS_OK;
  if (n_views < 1 || n_views > GS_MAX_VIEWS) return GS_EINVAL;
  BwdViews bv;
  for (int v = 0; v < n_views; ++v) {
    bv.cam[v] = cams[v];
    bv.grad2d[v] = grad2d[v];
  }
  bv.n_views = n_views;
#define GS_PBWDV(D)                                                                        \
  k_preprocess_bwd_views<D><<<div_up(n, 256), 256, 0, st>>>(                               \
      g->means, g->log_scales, g->quats, g->opacity_logits, g->sh, n, bv, grads->means,    \
      grads->log_scales, grads->quats, grads->opacity_logits, grads->sh, accumulate)
  GS_TIMED("preprocess_bwd", st,
           switch (deg) {
             case GS_DIRECT: GS_PBWDV(GS_DIRECT); break;
             case 0: GS_PBWDV(0); break;
             case 1: GS_PBWDV(1); break;
             case 2: GS_PBWDV(2); break;
             default: GS_PBWDV(3); break;
           });
#undef GS_PBWDV
  GS_CHECK_LAUNCH();
  return GS_OK;
}

}  // namespace gs

using namespace gs;

static bool gauss_ok(const gs_gaussians* g) {
  return g && g->means && g->log_scales && g->quats && g->opacity_logits && g->sh;
}

extern "C" gs_status gs_preprocess(const gs_gaussians* g, int64_t n, int32_t sh_degree,
                                   const gs_camera* cam, float* splats, uint32_t* depth_keys,
                                   uint32_t* tile_counts, void* stream) {
  CamDev cd;
  if (n < 0 || sh_degree < GS_DIRECT || sh_degree > 3 || !make_cam(cam, &cd)) return GS_EINVAL;
  if (n == 0) return GS_OK;
  if (!gauss_ok(g) || !splats || !depth_keys || !tile_counts) return GS_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const bool seq = tuning().seq_walk != 0;
#define GS_PRE(S, D)                                                                      \
  k_preprocess<S, D><<<div_up(n, 256), 256, 0, st>>>(g->means, g->log_scales, g->quats,   \
                                                     g->opacity_logits, g->sh, n, cd, splats, \
                                                     depth_keys, tile_counts)
#define GS_PRE_DEG(S)                                     \
  switch (sh_degree) {                                    \
    case GS_DIRECT: GS_PRE(S, GS_DIRECT); break;          \
    case 0: GS_PRE(S, 0); break;                          \
    case 1: GS_PRE(S, 1); break;                          \
    case 2: GS_PRE(S, 2); break;                          \
    default: GS_PRE(S, 3); break;                         \
  }
  GS_TIMED("preprocess", st, if (seq) { GS_PRE_DEG(true) } else { GS_PRE_DEG(false) });
#undef GS_PRE_DEG
#undef GS_PRE
  GS_CHECK_LAUNCH();
  return GS_OK;
}

extern "C" const char* gs_version(void) { return "libgs 0.1 gfx950"; }

extern "C" gs_status gs_preprocess_batched(const gs_gaussians* g, int64_t n, int32_t sh_degree,
                                           const gs_view* views, int32_t n_views, void* stream) {
  if (n < 0 || sh_degree < GS_DIRECT || sh_degree > 3 || !views || n_views < 1 ||
      n_views > GS_MAX_VIEWS)
    return GS_EINVAL;
  PreBatch pb;
  for (int v = 0; v < n_views; ++v) {
    if (!make_cam(&views[v].cam, &pb.cam[v])) return GS_EINVAL;
    if (n > 0 && (!views[v].splats || !views[v].depth_keys || !views[v].tile_counts))
      return GS_EINVAL;
    pb.splats[v] = views[v].splats;
    pb.depth_keys[v] = views[v].depth_keys;
    pb.tile_counts[v] = views[v].tile_counts;
  }
  if (n == 0) return GS_OK;
  if (!gauss_ok(g)) return GS_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const dim3 grid(div_up(n, 256), n_views);
  const bool seq = tuning().seq_walk != 0;
#define GS_PREB(S, D)                                                                  \
  k_preprocess_batched<S, D><<<grid, 256, 0, st>>>(g->means, g->log_scales, g->quats, \
                                                   g->opacity_logits, g->sh, n, pb)
#define GS_PREB_DEG(S)                                    \
  switch (sh_degree) {                                    \
    case GS_DIRECT: GS_PREB(S, GS_DIRECT); break;         \
    case 0: GS_PREB(S, 0); break;                         \
    case 1: GS_PREB(S, 1); break;                         \
    case 2: GS_PREB(S, 2); break;                         \
    default: GS_PREB(S, 3); break;                        \
  }
  GS_TIMED("preprocess", st, if (seq) { GS_PREB_DEG(true) } else { GS_PREB_DEG(false) });
#undef GS_PREB_DEG
#undef GS_PREB
  GS_CHECK_LAUNCH();
  return GS_OK;
}

extern "C" gs_status gs_pose_grad(const gs_gaussians* g, int64_t n, int32_t sh_degree,
                                  const gs_camera* cam, const double* grad2d, double* pose_grad,
                                  void* stream) {
  CamDev cd;
  if (n < 0 || sh_degree < GS_DIRECT || sh_degree > 3 || !make_cam(cam, &cd) || !pose_grad)
    return GS_EINVAL;
  if (n == 0) return GS_OK;
  if (!gauss_ok(g) || !grad2d || !aligned16(grad2d)) return GS_EINVAL;
  hipStream_t st = (hipStream_t)stream;
#define GS_POSE(D)                                                                              \
  k_pose_grad<D><<<div_up(n, 256), 256, 0, st>>>(g->means, g->log_scales, g->quats,            \
                                                 g->opacity_logits, g->sh, n, cd, grad2d,       \
                                                 pose_grad)
  GS_TIMED("pose_grad", st, switch (sh_degree) {
    case GS_DIRECT: GS_POSE(GS_DIRECT); break;
    case 0: GS_POSE(0); break;
    case 1: GS_POSE(1); break;
    case 2: GS_POSE(2); break;
    default: GS_POSE(3); break;
  });
#undef GS_POSE
  GS_CHECK_LAUNCH();
  return GS_OK;
}
