// Internal helpers shared by the libgs kernels (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gs.h"

#define GS_CHECK_LAUNCH()                                  \
  do {                                                     \
    if (hipGetLastError() != hipSuccess) return GS_EHIP;   \
  } while (0)

namespace gs {

constexpr int kWave = 64;

// Launch timer (see gs_timer_enable): brackets a launch with HIP events on
// its stream when timing is enabled for `name`.
void timer_begin(const char* name, hipStream_t st, hipEvent_t* a, hipEvent_t* b);
void timer_end(hipStream_t st, hipEvent_t a, hipEvent_t b);

#define GS_TIMED(NAME, ST, ...)                 \
  do {                                          \
    hipEvent_t gs_ta_, gs_tb_;                  \
    ::gs::timer_begin(NAME, ST, &gs_ta_, &gs_tb_); \
    __VA_ARGS__;                                \
    ::gs::timer_end(ST, gs_ta_, gs_tb_);        \
  } while (0)

// Camera as the kernels see it (by-value kernel argument).
struct CamDev {
  int W, H, tile, tiles_x, tiles_y;
  int inv_depth;  // the blended depth channel carries 1 / p_z
  double fx, fy, cx, cy;
  double R[9], t[3], campos[3];
  double near_plane, limx, limy;
};

// Kernel tuning of the calling host thread (gs_set_tuning).
const gs_tuning& tuning();

// Validates a host camera and converts it; false on bad input.
bool make_cam(const gs_camera* c, CamDev* out);

inline int div_up(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

inline bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

// ---------------------------------------------------------------------------
// Wavefront reductions with DPP (wave64). After wave_sum_to_last(), lane 63
// holds the sum over all 64 lanes.
// DPP controls: quad_perm(1,0,3,2) = 0xB1, quad_perm(2,3,0,1) = 0x4E,
// row_half_mirror = 0x141, row_mirror = 0x140, row_bcast:15 = 0x142,
// row_bcast:31 = 0x143.
template <int CTRL, int ROW_MASK = 0xf, int BANK_MASK = 0xf, bool BOUND = false>
__device__ __forceinline__ float dpp_mov(float old, float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v), CTRL,
                                                    ROW_MASK, BANK_MASK, BOUND));
}

// Sum over each row of 16 lanes (every lane of the row receives it).
__device__ __forceinline__ float row_sum16(float v) {
  v += dpp_mov<0xB1>(0.f, v);
  v += dpp_mov<0x4E>(0.f, v);
  v += dpp_mov<0x141>(0.f, v);
  v += dpp_mov<0x140>(0.f, v);
  return v;
}

__device__ __forceinline__ float wave_sum_to_last(float v) {
  v += dpp_mov<0xB1>(0.f, v);
  v += dpp_mov<0x4E>(0.f, v);
  v += dpp_mov<0x141>(0.f, v);
  v += dpp_mov<0x140>(0.f, v);
  v += dpp_mov<0x142, 0xa>(0.f, v);
  v += dpp_mov<0x143, 0xc>(0.f, v);
  return v;
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// ---------------------------------------------------------------------------
// One bias-corrected Adam update (Kingma and Ba) in FP32. The moments as
// written; the step as p -= s m / (sqrt(v) r + eps) with the per-step
// scalars s = lr / (1 - b1^t) and r = 1 / sqrt(1 - b2^t), which is the
// textbook lr m_hat / (sqrt(v_hat) + eps) with the bias corrections taken
// out of the per-parameter work; the square root and the reciprocal are the
// hardware's (each within 1 ulp), so a parameter costs about a dozen
// instructions instead of three correctly rounded divisions. Every kernel
// that steps parameters goes through this one function, so their results
// agree bit for bit.
__device__ __forceinline__ void adam_update(float& p, float& m, float& v, float g, float b1,
                                            float b2, float eps, float s, float r) {
#pragma clang fp contract(off)
  m = b1 * m + (1.f - b1) * g;
  v = b2 * v + (1.f - b2) * g * g;
  const float den = __builtin_amdgcn_sqrtf(v) * r + eps;
  p -= s * (m * __builtin_amdgcn_rcpf(den));
}

// The per-step scalars of adam_update for step t = steps_taken + 1:
// s = lr / (1 - b1^t) and r = 1 / sqrt(1 - b2^t), formed in FP64.
__device__ __host__ inline void adam_scalars(int32_t steps_taken, float lr, float b1, float b2,
                                             float& s, float& r) {
  const double t = (double)steps_taken + 1.0;
  s = (float)((double)lr / (1.0 - pow((double)b1, t)));
  r = (float)(1.0 / sqrt(1.0 - pow((double)b2, t)));
}

// Advances a device step count by one (one thread).
gs_status launch_step_advance(int32_t* step, hipStream_t st);

// ---------------------------------------------------------------------------
// Compact tile set of one splat (Sec. 2.1, Eq. 1-2): the SnugBox column
// range and, per column of tiles, the rows the ellipse Q = t covers over the
// column's slab. Evaluated in FP64 on the FP32-stored record, in a fixed
// order of operations (the library is compiled without FP contraction), so
// the tile set is a deterministic function of the stored record.
//
// Every quotient is the correctly rounded one the plain formula asks for,
// computed more cheaply where that is exact: a quotient by the tile size
// (8, 16 or 32, a power of two) is the product with its exact reciprocal;
// the column-independent terms c t and b hy / a are formed once per splat;
// and a quotient x / c uses rc = RN(1 / c): with q = RN(x rc), within an ulp
// of x / c, the remainder x - c q is exact as one FMA and q + (x - c q) rc
// rounded once is RN(x / c) (Markstein's theorem for round-to-nearest
// division) when nothing under- or overflows. With finite FP32 record
// fields, t > 0 and det > 0, every quantity on the way stays within
// [2^-900, 2^600] or is zero (det >= 2^-298, |dl|, |dr| <= 2^277 and,
// when nonzero, >= 2^-277, the numerators <= 2^407 and, when nonzero,
// >= 2^-504), so this holds for every column; a record with a non-finite
// field takes the divisions themselves. The one difference: a zero quotient
// can come out as +0 where the division gives -0, and it only ever enters
// v + y, whose ceiling and floor are the same for either sign.
// What the walk keeps of a splat: the centroid (u, v), conic terms b, c and
// det = a c - b^2, the half extents hx, hy, and the column-independent
// c t, b hy / a and RN(1 / c) (0: divide by c).
struct Snug {
  double u, v, b, c, det, hx, hy, ct, dxt, rc;
};

__device__ __forceinline__ bool snug_setup(float uf, float vf, float af, float bf, float cf,
                                           float tf, Snug& s) {
#pragma clang fp contract(off)
  const double a = af, t = tf;
  s.u = uf; s.v = vf; s.b = bf; s.c = cf;
  s.det = a * s.c - s.b * s.b;
  if (!(t > 0.0) || !(s.det > 0.0)) return false;
  s.hx = sqrt((t * s.c) / s.det);
  s.hy = sqrt((t * a) / s.det);
  s.ct = s.c * t;
  s.dxt = (s.b * s.hy) / a;
  const bool finite = isfinite(uf) && isfinite(vf) && isfinite(af) && isfinite(bf) &&
                      isfinite(cf) && isfinite(tf);
  s.rc = finite ? 1.0 / s.c : 0.0;  // c != 0 (det > 0)
  return true;
}

// RN(x / c) from rc = RN(1 / c), as above.
__device__ __forceinline__ double snug_div_c(double x, const Snug& s) {
  const double q = x * s.rc;
  const double r = fma(-q, s.c, x);
  return fma(r, s.rc, q);
}

// 1 / tile, exact: the tile size is a power of two (8, 16 or 32)
__device__ __forceinline__ double tile_recip(int tile) {
  return ldexp(1.0, -__builtin_ctz((unsigned)tile));
}

// Inclusive column range, clamped to the grid; empty if tx0 > tx1.
__device__ __forceinline__ void snug_columns(const Snug& s, int tile, int tiles_x, int& tx0,
                                             int& tx1) {
#pragma clang fp contract(off)
  const double rT = tile_recip(tile);
  const double lo = fmax(0.0, ceil((s.u - s.hx) * rT) - 1.0);
  const double hi = fmin((double)(tiles_x - 1), floor((s.u + s.hx) * rT));
  if (!(lo <= hi)) { tx0 = 1; tx1 = 0; return; }
  tx0 = (int)lo;
  tx1 = (int)hi;
}

// Inclusive row range of column tx; empty if ty0 > ty1.
__device__ __forceinline__ void snug_rows(const Snug& s, int tx, int tile, int tiles_y, int& ty0,
                                          int& ty1) {
#pragma clang fp contract(off)
  const double T = (double)tile;
  const double rT = tile_recip(tile);
  const double xl = T * (double)tx - s.u;
  const double xr = (T * (double)tx + T) - s.u;
  const double dl = fmax(xl, -s.hx);
  const double dr = fmin(xr, s.hx);
  if (!(dl <= dr)) { ty0 = 1; ty1 = 0; return; }
  const double sl = sqrt(fmax(s.ct - s.det * (dl * dl), 0.0));
  const double sr = sqrt(fmax(s.ct - s.det * (dr * dr), 0.0));
  const double bl = s.b * dl;
  const double br = s.b * dr;
  double lo, hi;
  if (s.rc != 0.0) {
    lo = fmin(snug_div_c(-(bl + sl), s), snug_div_c(-(br + sr), s));
    hi = fmax(snug_div_c(sl - bl, s), snug_div_c(sr - br, s));
  } else {
    lo = fmin(-(bl + sl) / s.c, -(br + sr) / s.c);
    hi = fmax((sl - bl) / s.c, (sr - br) / s.c);
  }
  const double ymin = (dl <= s.dxt && s.dxt <= dr) ? -s.hy : lo;
  const double ymax = (dl <= -s.dxt && -s.dxt <= dr) ? s.hy : hi;
  const double r0 = fmax(0.0, ceil((s.v + ymin) * rT) - 1.0);
  const double r1 = fmin((double)(tiles_y - 1), floor((s.v + ymax) * rT));
  if (!(r0 <= r1)) { ty0 = 1; ty1 = 0; return; }
  ty0 = (int)r0;
  ty1 = (int)r1;
}

// ---------------------------------------------------------------------------
// Load-balanced column walk (the load-balanced tile writing of Sec. 2.1,
// on wave64): the 64 lanes of a wavefront walk the SnugBox columns of the 64
// Gaussians they hold as one flattened list, 64 columns per round, so a
// Gaussian spanning a hundred columns does not stall the other 63 lanes.
// f(owner_lane, tx, ty0, ty1) runs once per column (ty0 > ty1: the column's
// rows fall outside the grid). Every thread of the workgroup must call it
// (it synchronises the workgroup); `lds` is 64 entries of this wavefront's
// scratch.
struct SnugLds {
  Snug s;
  int tx0;
  uint32_t excl;
};

__device__ __forceinline__ uint32_t wave_incl_scan_u32_(uint32_t v) {
  const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const uint32_t o = __shfl_up(v, d, kWave);
    if (lane >= d) v += o;
  }
  return v;
}

template <typename F>
__device__ __forceinline__ void wave_column_walk(bool valid, const Snug& s, int tile, int tiles_x,
                                                 int tiles_y, SnugLds* lds, F&& f) {
  const int lane = threadIdx.x & (kWave - 1);
  int tx0 = 0, tx1 = -1;
  if (valid) snug_columns(s, tile, tiles_x, tx0, tx1);
  const uint32_t ncols = (valid && tx1 >= tx0) ? (uint32_t)(tx1 - tx0 + 1) : 0u;
  const uint32_t incl = wave_incl_scan_u32_(ncols);
  const uint32_t total = __shfl(incl, kWave - 1, kWave);
  lds[lane].s = s;
  lds[lane].tx0 = tx0;
  lds[lane].excl = incl - ncols;
  __syncthreads();
  for (uint32_t c0 = 0; c0 < total; c0 += kWave) {
    const uint32_t c = c0 + (uint32_t)lane;
    if (c < total) {
      int lo = 0, hi = kWave - 1;  // owner: last lane whose first column is <= c
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (lds[mid].excl <= c) lo = mid; else hi = mid - 1;
      }
      const SnugLds& o = lds[lo];
      const int tx = o.tx0 + (int)(c - o.excl);
      int ty0, ty1;
      snug_rows(o.s, tx, tile, tiles_y, ty0, ty1);
      f(lo, tx, ty0, ty1);
    }
  }
  __syncthreads();
}

// The same walk with each lane visiting its own Gaussian's columns in turn
// (the wavefront runs as long as its widest Gaussian; owner = own lane).
template <typename F>
__device__ __forceinline__ void seq_column_walk(bool valid, const Snug& s, int tile, int tiles_x,
                                                int tiles_y, F&& f) {
  const int lane = threadIdx.x & (kWave - 1);
  int tx0 = 0, tx1 = -1;
  if (valid) snug_columns(s, tile, tiles_x, tx0, tx1);
  for (int tx = tx0; tx <= tx1; ++tx) {
    int ty0, ty1;
    snug_rows(s, tx, tile, tiles_y, ty0, ty1);
    f(lane, tx, ty0, ty1);
  }
}

template <bool SEQ, typename F>
__device__ __forceinline__ void column_walk(bool valid, const Snug& s, int tile, int tiles_x,
                                            int tiles_y, SnugLds* lds, F&& f) {
  if constexpr (SEQ)
    seq_column_walk(valid, s, tile, tiles_x, tiles_y, f);
  else
    wave_column_walk(valid, s, tile, tiles_x, tiles_y, lds, f);
}

// ---------------------------------------------------------------------------
// Per-pixel skip decision alpha < 1/255, taken as Q > t with Q in FP64 from
// the FP32 record in the order dx*(a*dx + 2*(b*dy)) + dy*(c*dy). The FP32
// value q32 decides directly when it is farther from t than its error bound
// (about 10 ulp of a dx^2 + c dy^2; `mag` carries that sum), else the FP64
// value is computed.
// The exact FP64 decision, out of line so that the compiler cannot
// speculate it into the compositing loops (it is needed only when the FP32
// value lies within its error bound of t, a few evaluations in a million).
__device__ __attribute__((noinline)) bool splat_skips_exact(float t, float px, float py, float u,
                                                            float v, float a, float b, float c);

__device__ __forceinline__ bool splat_skips(float q32, float mag, float t, float px, float py,
                                            float u, float v, float a, float b, float c) {
#pragma clang fp contract(off)
  const float diff = q32 - t;
  const float m = 1e-5f * mag;
  if (fabsf(diff) > m) return diff > 0.f;  // decided outside the FP32 error band
  return splat_skips_exact(t, px, py, u, v, a, b, c);
}

// The same decision with a band fixed per splat instead of per pixel. With
// dx, dy rounded once each and four more roundings, |q32 - Q| <= 5 u (a dx^2
// + 2 |b dx dy| + c dy^2) to first order (u = 2^-24). For a positive
// definite conic, with r = |b| / sqrt(ac) < 1: 2 |b dx dy| <= r (a dx^2 +
// c dy^2) and Q >= (1 - r) (a dx^2 + c dy^2), so |q32 - Q| <= eta Q with
// eta = 5 u (1 + r) / (1 - r) = 5 u (sqrt(ac) + |b|)^2 / (ac - b^2). A sign
// of q32 - t other than that of Q - t then needs |q32 - t| <= eta t: outside
// the band eta t the FP32 sign is the FP64 one, and both forms take the same
// decisions. The band uses 1e-6 in place of 5 u (about 3e-7). Infinite
// (always the FP64 value) unless a > 0, ac > b^2, ac is within 1e+-30
// (normal in FP32 below) and t > 1e-20.
__device__ __forceinline__ float skip_band(float a, float b, float c, float t) {
#pragma clang fp contract(off)
  const double ac = (double)a * (double)c;          // exact
  const double det = ac - (double)b * (double)b;    // one rounding
  if (!(a > 0.f) || !(det > 0.0) || !(t > 1e-20f) || !(ac > 1e-30) || !(ac < 1e30))
    return __builtin_huge_valf();
  // (sqrt(ac) + |b|)^2 / det in FP32: a few roundings of positive terms, far
  // inside the margin; an underflowing det gives infinity
  const float sac = sqrtf((float)ac);
  const float bb = fabsf(b);
  const float num = (sac + bb) * (sac + bb);
  return (1e-6f * (num / (float)det)) * t;
}

__device__ __forceinline__ bool splat_skips_band(float q32, float band, float t, float px,
                                                 float py, float u, float v, float a, float b,
                                                 float c) {
#pragma clang fp contract(off)
  const float diff = q32 - t;
  if (fabsf(diff) > band) return diff > 0.f;  // decided outside the splat's band
  return splat_skips_exact(t, px, py, u, v, a, b, c);
}

}  // namespace gs
