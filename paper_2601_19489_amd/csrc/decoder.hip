// Anchor (neural-Gaussian) decoder of Sec. 2.3 on BF16 matrix cores
// (v_mfma_f32_16x16x32_bf16), FP32 accumulation.
//
// Per anchor i and camera centre c: x = [feat_i (32), unit(c - pos_i) (3)]
// rounded to BF16. Three heads h (opacity, colour, covariance), each
// z_h = W1_h x + b1_h, h_h = bf16(max(z_h, 0)), y_h = W2_h h_h + b2_h.
// Child j of anchor i (Gaussian j A + i): opacity max(0, tanh y_op[j]),
// rgb sigmoid(y_col[3j ..]), scale scaling[3 ..] sigmoid(y_cov[7j ..]),
// quaternion y_cov[7j+3 .. 7j+6] normalised, mean pos + offsets[3j ..]
// scaling[0 ..].
//
// Backward: BF16 rounding is taken as the identity (straight-through) and
// the rounded operands of the forward are reused. The gradient operand of
// every backward product (dL/dy, dL/dz, FP32) enters the BF16 matrix core
// as two terms hi + lo with hi = bf16(v), lo = bf16(v - hi), which keeps
// about 16 bits of it.
//
// Matrix-core operand layout (16x16x32, wave64; lane l, m = l % 16,
// kq = l / 16): A (16 x 32) lane holds A[m][8 kq .. 8 kq + 7]; B (32 x 16)
// lane holds B[8 kq .. 8 kq + 7][m]; D (16 x 16) lane holds
// D[4 kq .. 4 kq + 3][m].
#include <math.h>

#include <mutex>

#include "common.h"

namespace gs {

namespace {

constexpr int kKids = GS_ANCHOR_CHILDREN;  // 10
constexpr int kFeat = GS_ANCHOR_FEAT;      // 32
constexpr int kIn = kFeat + 3;             // 35 inputs
constexpr int kHid = 32;                   // hidden units per head
constexpr int kHidAll = 3 * kHid;          // 96
constexpr int kOut = 110;                  // 10 + 30 + 70 outputs
constexpr int kTile = 64;                  // anchors per workgroup iteration
constexpr int kThreads = 256;
// LDS row strides (elements): BF16 inputs and hidden units, FP32 outputs
constexpr int kXS = 72, kHS = 104, kYS = 161, kZS = 97, kDS = 65;
// Padded output columns: head h occupies columns 32 h .. 32 h + 31 (op,
// colour) and 64 .. 159 (covariance); the forward computes 16, 32 and 80 of
// them, the backward reads 32, 32 and 96.
__host__ __device__ constexpr int head_base(int h) { return 32 * h; }
__host__ __device__ constexpr int head_row(int h) {
  return h == 0 ? 0 : h == 1 ? 10 : h == 2 ? 40 : 110;
}
__host__ __device__ constexpr int head_len(int h) { return head_row(h + 1) - head_row(h); }
__host__ __device__ constexpr int head_fwd_tiles(int h) { return h == 0 ? 1 : h == 1 ? 2 : 5; }
__host__ __device__ constexpr int head_k_steps(int h) { return h == 2 ? 3 : 1; }
// Per-workgroup partial sums in the workspace: dW1 [96][48], dW2 [160][32]
// (padded rows), db1 [96], db2 [160].
constexpr int kWsW1 = 0, kWsW2 = kWsW1 + kHidAll * 48, kWsB1 = kWsW2 + 160 * kHid,
              kWsB2 = kWsB1 + kHidAll, kWsFloats = kWsB2 + 160;
constexpr int kMaxBlocks = 256;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f) {  // round to nearest even
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ bf16x8 pack8(const uint16_t (&h)[8]) {
  union {
    uint16_t s[8];
    bf16x8 v;
  } u;
#pragma unroll
  for (int e = 0; e < 8; ++e) u.s[e] = h[e];
  return u.v;
}

__device__ __forceinline__ bf16x8 lds8(const uint16_t* p) {  // 16-byte aligned
  union {
    uint4 q;
    bf16x8 v;
  } u;
  u.q = *reinterpret_cast<const uint4*>(p);
  return u.v;
}

// 8 FP32 values at p[0], p[stride], ... split into BF16 hi and lo terms.
__device__ __forceinline__ void split8(const float* p, int stride, bf16x8& hi, bf16x8& lo) {
  uint16_t h[8], l[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const float v = p[e * stride];
    h[e] = f2bf(v);
    l[e] = f2bf(v - __uint_as_float((uint32_t)h[e] << 16));
  }
  hi = pack8(h);
  lo = pack8(l);
}

__device__ __forceinline__ bf16x8 gather8(const uint16_t* p, int stride) {
  uint16_t h[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) h[e] = p[e * stride];
  return pack8(h);
}

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ float sigm(float x) { return 1.f / (1.f + expf(-x)); }

// BF16 copies of the weights, staged once per workgroup in LDS (in the
// space the tile loop uses later): W1 padded to 64 inputs [96][64] at s,
// W2 in padded rows [160][32] at s + 96 * 64. Ends with a barrier.
constexpr int kStageW2 = kHidAll * 64;
__device__ void stage_weights(const float* __restrict__ w1, const float* __restrict__ w2,
                              uint16_t* s) {
  for (int e = threadIdx.x; e < kHidAll * 64; e += (int)blockDim.x) {
    const int r = e / 64, c = e % 64;
    s[e] = c < kIn ? f2bf(w1[r * kIn + c]) : (uint16_t)0;
  }
  for (int e = threadIdx.x; e < 160 * kHid; e += (int)blockDim.x) {
    const int pr = e / kHid, c = e % kHid;
    const int hd = pr < 32 ? 0 : pr < 64 ? 1 : 2;
    const int local = pr - head_base(hd);
    s[kStageW2 + e] =
        local < head_len(hd) ? f2bf(w2[(head_row(hd) + local) * kHid + c]) : (uint16_t)0;
  }
  __syncthreads();
}

// Forward weight operands of one lane (B operands, constant per launch).
struct FwdW {
  bf16x8 w1[6][2];  // layer 1: N-tile (hidden 16 nt ..), K-step (inputs 32 s ..)
  bf16x8 w2[8];     // layer 2: op 1, colour 2, covariance 5 N-tiles
};

__device__ void load_fwd_weights(const uint16_t* s, FwdW& W) {
  const int l = threadIdx.x & 63, m = l & 15, kq = l >> 4;
#pragma unroll
  for (int nt = 0; nt < 6; ++nt)
#pragma unroll
    for (int k = 0; k < 2; ++k) W.w1[nt][k] = lds8(s + (16 * nt + m) * 64 + 32 * k + 8 * kq);
  int t = 0;
#pragma unroll
  for (int hd = 0; hd < 3; ++hd)
#pragma unroll
    for (int nt = 0; nt < head_fwd_tiles(hd); ++nt)
      W.w2[t++] = lds8(s + kStageW2 + (head_base(hd) + 16 * nt + m) * kHid + 8 * kq);
}

// Backward weight operands (B operands of dL/dh = W2^T dy and dL/dx = W1^T dz).
struct BwdW {
  bf16x8 w2t[10];   // [head K-step][N-tile]: op 1x2, colour 1x2, covariance 3x2
  bf16x8 w1t[3][2]; // K-step (hidden 32 s ..), N-tile (inputs 16 nt ..)
};

__device__ void load_bwd_weights(const uint16_t* s, BwdW& W) {
  const int l = threadIdx.x & 63, m = l & 15, kq = l >> 4;
  int t = 0;
#pragma unroll
  for (int hd = 0; hd < 3; ++hd)
#pragma unroll
    for (int k = 0; k < head_k_steps(hd); ++k)
#pragma unroll
      for (int nt = 0; nt < 2; ++nt)
        W.w2t[t++] = gather8(s + kStageW2 + (head_base(hd) + 32 * k + 8 * kq) * kHid + 16 * nt + m,
                             kHid);
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int nt = 0; nt < 2; ++nt)
      W.w1t[k][nt] = gather8(s + (32 * k + 8 * kq) * 64 + 16 * nt + m, 64);
}

// The backward runs 8 wavefronts per tile: wavefront w takes rows
// 16 (w % 4) .. + 15 and half h = w / 4 of every product's N-tiles, so it
// holds half of the weight operands.
constexpr int kBwdThreads = 512;
// layer-2 output tiles in order (head, N-tile): 0: (0,0), 1-2: (1,0..1),
// 3-7: (2,0..4); half h computes tiles 4 h .. 4 h + 3
__host__ __device__ constexpr int l2_head(int t) { return t == 0 ? 0 : t < 3 ? 1 : 2; }
__host__ __device__ constexpr int l2_ntile(int t) { return t == 0 ? 0 : t < 3 ? t - 1 : t - 3; }

struct FwdWHalf {
  bf16x8 w1[3][2];  // layer 1: hidden N-tiles 3 h .. 3 h + 2, both K-steps
  bf16x8 w2[4];     // layer 2: output tiles 4 h .. 4 h + 3
};

__device__ void load_fwd_weights_half(const uint16_t* s, int h, FwdWHalf& W) {
  const int l = threadIdx.x & 63, m = l & 15, kq = l >> 4;
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int k = 0; k < 2; ++k)
      W.w1[j][k] = lds8(s + (16 * (3 * h + j) + m) * 64 + 32 * k + 8 * kq);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int t = 4 * h + j;
    W.w2[j] = lds8(s + kStageW2 + (head_base(l2_head(t)) + 16 * l2_ntile(t) + m) * kHid + 8 * kq);
  }
}

struct BwdWHalf {
  bf16x8 w2t[5];  // [head K-step], N-tile h: op 1, colour 1, covariance 3
  bf16x8 w1t[3];  // K-step (hidden 32 s ..), N-tile h (inputs 16 h ..)
};

__device__ void load_bwd_weights_half(const uint16_t* s, int h, BwdWHalf& W) {
  const int l = threadIdx.x & 63, m = l & 15, kq = l >> 4;
  int t = 0;
#pragma unroll
  for (int hd = 0; hd < 3; ++hd)
#pragma unroll
    for (int k = 0; k < head_k_steps(hd); ++k)
      W.w2t[t++] = gather8(s + kStageW2 + (head_base(hd) + 32 * k + 8 * kq) * kHid + 16 * h + m,
                           kHid);
#pragma unroll
  for (int k = 0; k < 3; ++k) W.w1t[k] = gather8(s + (32 * k + 8 * kq) * 64 + 16 * h + m, 64);
}

struct DecIn {
  const float *feat, *pos, *offsets, *scaling, *w1, *b1, *w2, *b2;
  int64_t A;
  double cx, cy, cz;  // camera centre
};

// Zero the padding columns 35 .. 71 of the input rows (never written again).
__device__ void zero_x_pad(uint16_t* sX) {
  for (int e = threadIdx.x; e < kTile * (kXS - kIn); e += (int)blockDim.x)
    sX[(e / (kXS - kIn)) * kXS + kIn + e % (kXS - kIn)] = 0;
}

// The biases, copied once per workgroup into LDS (read per N-tile in the
// tile loop: a global load there is one memory round trip per tile). Ends
// with a barrier.
struct Bias {
  float b1[kHidAll];
  float b2[kOut];
};

__device__ void stage_bias(const DecIn& in, Bias& B) {
  for (int e = threadIdx.x; e < kHidAll; e += (int)blockDim.x) B.b1[e] = in.b1[e];
  for (int e = threadIdx.x; e < kOut; e += (int)blockDim.x) B.b2[e] = in.b2[e];
  __syncthreads();
}

// Forward of one tile of anchors a0 .. a0 + 63: sX (BF16 inputs), sH (BF16
// hidden units), sY (FP32 y + b2 in padded columns). Ends with a barrier.
// BATCH: the thread's feature loads all issued before the first is used
// (faster in the backward, where the loop's loads wait one by one; slower in
// the forward, measured).
template <bool BATCH>
__device__ void tile_forward(const DecIn& in, const Bias& B, int64_t a0, const FwdW& W,
                             uint16_t* sX, uint16_t* sH, float* sY) {
  const int tid = threadIdx.x;
  const int64_t A = in.A;
  if constexpr (BATCH) {
    constexpr int kPer = kFeat * kTile / kThreads;  // 8
    static_assert(kFeat * kTile % kThreads == 0, "whole rounds");
    float fv[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int e = tid + q * kThreads, k = e / kTile, m = e % kTile;
      const int64_t ai = a0 + m;
      fv[q] = in.feat[k * A + (ai < A ? ai : a0)];  // a0 < A: a valid row
    }
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int e = tid + q * kThreads, k = e / kTile, m = e % kTile;
      sX[m * kXS + k] = a0 + m < A ? f2bf(fv[q]) : (uint16_t)0;
    }
  } else {
    for (int e = tid; e < kFeat * kTile; e += kThreads) {
      const int k = e / kTile, m = e % kTile;
      const int64_t ai = a0 + m;
      sX[m * kXS + k] = ai < A ? f2bf(in.feat[k * A + ai]) : (uint16_t)0;
    }
  }
  if (tid < kTile) {
#pragma clang fp contract(off)
    const int64_t ai = a0 + tid;
    uint16_t d3[3] = {0, 0, 0};
    if (ai < A) {
      const double d0 = in.cx - (double)in.pos[ai];
      const double d1 = in.cy - (double)in.pos[A + ai];
      const double d2 = in.cz - (double)in.pos[2 * A + ai];
      const double nrm = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
      d3[0] = f2bf((float)(d0 / nrm));
      d3[1] = f2bf((float)(d1 / nrm));
      d3[2] = f2bf((float)(d2 / nrm));
    }
    for (int j = 0; j < 3; ++j) sX[tid * kXS + kFeat + j] = d3[j];
  }
  __syncthreads();
  const int l = tid & 63, w = tid >> 6, m = l & 15, kq = l >> 4;
  const int row = 16 * w + m;
  const bf16x8 xa0 = lds8(sX + row * kXS + 8 * kq);
  const bf16x8 xa1 = lds8(sX + row * kXS + 32 + 8 * kq);
#pragma unroll
  for (int nt = 0; nt < 6; ++nt) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = mfma(xa0, W.w1[nt][0], acc);
    acc = mfma(xa1, W.w1[nt][1], acc);
    const int hid = 16 * nt + m;
    const float bb = B.b1[hid];
#pragma unroll
    for (int i = 0; i < 4; ++i)
      sH[(16 * w + 4 * kq + i) * kHS + hid] = f2bf(fmaxf(acc[i] + bb, 0.f));
  }
  __syncthreads();
  int t = 0;
#pragma unroll
  for (int hd = 0; hd < 3; ++hd) {
    const bf16x8 ha = lds8(sH + row * kHS + kHid * hd + 8 * kq);
#pragma unroll
    for (int nt = 0; nt < head_fwd_tiles(hd); ++nt) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
      acc = mfma(ha, W.w2[t++], acc);
      const int local = 16 * nt + m;
      const float bb = local < head_len(hd) ? B.b2[head_row(hd) + local] : 0.f;
#pragma unroll
      for (int i = 0; i < 4; ++i) sY[(16 * w + 4 * kq + i) * kYS + head_base(hd) + local] = acc[i] + bb;
    }
  }
  __syncthreads();
}

__global__ void __launch_bounds__(kThreads) k_decode_fwd(DecIn in, float* __restrict__ means,
                                                         float* __restrict__ scales,
                                                         float* __restrict__ quats,
                                                         float* __restrict__ opac,
                                                         float* __restrict__ rgb) {
  __shared__ __align__(16) uint16_t sX[kTile * kXS];
  __shared__ __align__(16) uint16_t sH[kTile * kHS];
  __shared__ __align__(16) float sY[kTile * kYS];
  __shared__ Bias sB;
  FwdW W;
  stage_bias(in, sB);
  stage_weights(in.w1, in.w2, reinterpret_cast<uint16_t*>(sY));
  load_fwd_weights(reinterpret_cast<const uint16_t*>(sY), W);
  zero_x_pad(sX);
  __syncthreads();
  const int64_t A = in.A, N = A * kKids;
  for (int64_t a0 = (int64_t)blockIdx.x * kTile; a0 < A; a0 += (int64_t)gridDim.x * kTile) {
    tile_forward<false>(in, sB, a0, W, sX, sH, sY);
    // the (child, anchor) items of a thread, unrolled: every anchor value is
    // loaded before the first output is stored
    constexpr int kRounds = (kKids * kTile + kThreads - 1) / kThreads;  // 3
    float av[kRounds][12];  // child scale factors 3, pos 3, offsets 3, offset scaling 3
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
      const int it = threadIdx.x + r * kThreads;
      const int j = it / kTile, m = it % kTile;
      const int64_t ai = a0 + m;
      if (it < kKids * kTile && ai < A) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          av[r][d] = in.scaling[(3 + d) * A + ai];
          av[r][3 + d] = in.pos[d * A + ai];
          av[r][6 + d] = in.offsets[(3 * j + d) * A + ai];
          av[r][9 + d] = in.scaling[d * A + ai];
        }
      }
    }
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
      const int it = threadIdx.x + r * kThreads;
      if (it >= kKids * kTile) break;
      const int j = it / kTile, m = it % kTile;
      const int64_t ai = a0 + m;
      if (ai >= A) continue;
      const float* y = sY + m * kYS;
      const int64_t g = j * A + ai;
      opac[g] = fmaxf(tanhf(y[j]), 0.f);
#pragma unroll
      for (int c = 0; c < 3; ++c) rgb[c * N + g] = sigm(y[32 + 3 * j + c]);
#pragma unroll
      for (int a = 0; a < 3; ++a) scales[a * N + g] = av[r][a] * sigm(y[64 + 7 * j + a]);
      const float q0 = y[64 + 7 * j + 3], q1 = y[64 + 7 * j + 4], q2 = y[64 + 7 * j + 5],
                  q3 = y[64 + 7 * j + 6];
      const float inv = 1.f / sqrtf(q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3);
      quats[g] = q0 * inv;
      quats[N + g] = q1 * inv;
      quats[2 * N + g] = q2 * inv;
      quats[3 * N + g] = q3 * inv;
#pragma unroll
      for (int d = 0; d < 3; ++d) means[d * N + g] = av[r][3 + d] + av[r][6 + d] * av[r][9 + d];
    }
    __syncthreads();
  }
}

struct DecGrad {
  const float *dmeans, *dscales, *dquats, *dopac, *drgb;  // child-Gaussian gradients
  float *dfeat, *doffsets, *dscaling;                     // per-anchor outputs (may be null)
  float* ws;                                              // per-workgroup partial sums
  int accumulate;
};

// tile_forward for the backward's 8 wavefronts: the same sX, sH and sY,
// with wavefront w computing rows 16 (w % 4) .. and the N-tiles of half
// h = w / 4 (hidden N-tiles 3 h .. 3 h + 2; output tiles 4 h .. 4 h + 3).
// Ends with a barrier.
__device__ void tile_forward_half(const DecIn& in, const Bias& B, int64_t a0, int h,
                                  const FwdWHalf& W, uint16_t* sX, uint16_t* sH, float* sY) {
  const int tid = threadIdx.x;
  const int64_t A = in.A;
  {
    constexpr int kPer = kFeat * kTile / kBwdThreads;  // 4
    static_assert(kFeat * kTile % kBwdThreads == 0, "whole rounds");
    float fv[kPer];  // every load issued before the first is used
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int e = tid + q * kBwdThreads, k = e / kTile, m = e % kTile;
      const int64_t ai = a0 + m;
      fv[q] = in.feat[k * A + (ai < A ? ai : a0)];  // a0 < A: a valid row
    }
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int e = tid + q * kBwdThreads, k = e / kTile, m = e % kTile;
      sX[m * kXS + k] = a0 + m < A ? f2bf(fv[q]) : (uint16_t)0;
    }
  }
  if (tid < kTile) {
#pragma clang fp contract(off)
    const int64_t ai = a0 + tid;
    uint16_t d3[3] = {0, 0, 0};
    if (ai < A) {
      const double d0 = in.cx - (double)in.pos[ai];
      const double d1 = in.cy - (double)in.pos[A + ai];
      const double d2 = in.cz - (double)in.pos[2 * A + ai];
      const double nrm = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
      d3[0] = f2bf((float)(d0 / nrm));
      d3[1] = f2bf((float)(d1 / nrm));
      d3[2] = f2bf((float)(d2 / nrm));
    }
    for (int j = 0; j < 3; ++j) sX[tid * kXS + kFeat + j] = d3[j];
  }
  __syncthreads();
  const int l = tid & 63, wr = (tid >> 6) & 3, m = l & 15, kq = l >> 4;
  const int row = 16 * wr + m;
  const bf16x8 xa0 = lds8(sX + row * kXS + 8 * kq);
  const bf16x8 xa1 = lds8(sX + row * kXS + 32 + 8 * kq);
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = mfma(xa0, W.w1[j][0], acc);
    acc = mfma(xa1, W.w1[j][1], acc);
    const int hid = 16 * (3 * h + j) + m;
    const float bb = B.b1[hid];
#pragma unroll
    for (int i = 0; i < 4; ++i)
      sH[(16 * wr + 4 * kq + i) * kHS + hid] = f2bf(fmaxf(acc[i] + bb, 0.f));
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int t = 4 * h + j, hd = l2_head(t), nt = l2_ntile(t);
    const bf16x8 ha = lds8(sH + row * kHS + kHid * hd + 8 * kq);
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = mfma(ha, W.w2[j], acc);
    const int local = 16 * nt + m;
    const float bb = local < head_len(hd) ? B.b2[head_row(hd) + local] : 0.f;
#pragma unroll
    for (int i = 0; i < 4; ++i)
      sY[(16 * wr + 4 * kq + i) * kYS + head_base(hd) + local] = acc[i] + bb;
  }
  __syncthreads();
}

__device__ __forceinline__ void put(float* p, float v, int accumulate) {
  if (accumulate) *p += v; else *p = v;
}

__global__ void __launch_bounds__(kBwdThreads) k_decode_bwd(DecIn in, DecGrad gr) {
  __shared__ __align__(16) uint16_t sX[kTile * kXS];
  __shared__ __align__(16) uint16_t sH[kTile * kHS];
  __shared__ __align__(16) float sY[kTile * kYS];   // y, then dL/dy in place
  __shared__ float sZ[kTile * kZS];   // dL/dz
  __shared__ float sD[kFeat * kDS];   // dL/dfeat, transposed for coalesced writes
  __shared__ Bias sB;
  const int tid = threadIdx.x, l = tid & 63, w = tid >> 6, m = l & 15, kq = l >> 4;
  const int wr = w & 3, h = w >> 2;  // row block and N-tile half of this wavefront
  FwdWHalf Wf;
  BwdWHalf Wb;
  stage_bias(in, sB);
  stage_weights(in.w1, in.w2, reinterpret_cast<uint16_t*>(sY));
  load_fwd_weights_half(reinterpret_cast<const uint16_t*>(sY), h, Wf);
  load_bwd_weights_half(reinterpret_cast<const uint16_t*>(sY), h, Wb);
  zero_x_pad(sX);
  __syncthreads();
  const int64_t A = in.A, N = A * kKids;
  // weight-gradient tiles of this wavefront: W2 (8 x 2 tiles) 2 w, 2 w + 1;
  // W1 (6 x 3 tiles) w, w + 8, w + 16 (below 18)
  f32x4 accW2[2], accW1[3];
#pragma unroll
  for (int q = 0; q < 2; ++q) accW2[q] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int q = 0; q < 3; ++q) accW1[q] = f32x4{0.f, 0.f, 0.f, 0.f};
  float dbias = 0.f;  // threads 0..159: b2 padded column; 160..255: b1 unit
  for (int64_t a0 = (int64_t)blockIdx.x * kTile; a0 < A; a0 += (int64_t)gridDim.x * kTile) {
    tile_forward_half(in, sB, a0, h, Wf, sX, sH, sY);
    // offsets and scaling gradients, one thread per (anchor, axis d), the
    // children in two groups of five whose values are loaded together
    if (tid < 3 * kTile && a0 + tid % kTile < A) {
      const int mm = tid % kTile, d = tid / kTile;
      const int64_t ai = a0 + mm;
      const float* y = sY + mm * kYS;
      const float sc = in.scaling[d * A + ai];
      float g_off = 0.f, g_sc = 0.f;
      constexpr int kHalf = kKids / 2;
#pragma unroll
      for (int j0 = 0; j0 < kKids; j0 += kHalf) {
        float dm[kHalf], off[kHalf], dsc[kHalf];
#pragma unroll
        for (int j = 0; j < kHalf; ++j) {
          const int64_t g = (j0 + j) * A + ai;
          dm[j] = gr.dmeans[d * N + g];
          off[j] = in.offsets[(3 * (j0 + j) + d) * A + ai];
          dsc[j] = gr.dscales[d * N + g];
        }
#pragma unroll
        for (int j = 0; j < kHalf; ++j) {
          g_off += dm[j] * off[j];
          g_sc += dsc[j] * sigm(y[64 + 7 * (j0 + j) + d]);
        }
        if (gr.doffsets)
#pragma unroll
          for (int j = 0; j < kHalf; ++j)
            put(gr.doffsets + (3 * (j0 + j) + d) * A + ai, dm[j] * sc, gr.accumulate);
      }
      if (gr.dscaling) {
        put(gr.dscaling + d * A + ai, g_off, gr.accumulate);
        put(gr.dscaling + (3 + d) * A + ai, g_sc, gr.accumulate);
      }
    }
    __syncthreads();
    // dL/dy in place of y; absent anchors and padded columns get zero (one
    // (child, anchor) item per thread and round).
    constexpr int kRounds = (kKids * kTile + kBwdThreads - 1) / kBwdThreads;  // 2
#pragma unroll 1
    for (int r = 0; r < kRounds; ++r) {
      const int it = tid + r * kBwdThreads;
      if (it >= kKids * kTile) break;
      const int j = it / kTile, mm = it % kTile;
      const int64_t ai = a0 + mm;
      float* y = sY + mm * kYS;
      float* yc = y + 32 + 3 * j;
      float* yv = y + 64 + 7 * j;
      if (ai >= A) {
        y[j] = 0.f;
        for (int c = 0; c < 3; ++c) yc[c] = 0.f;
        for (int c = 0; c < 7; ++c) yv[c] = 0.f;
        continue;
      }
      // the item's gradient loads, all issued before the first is used
      float q[14];
      const int64_t g = j * A + ai;
      q[0] = gr.dopac[g];
#pragma unroll
      for (int c = 0; c < 3; ++c) q[1 + c] = gr.drgb[c * N + g];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        q[4 + a] = gr.dscales[a * N + g];
        q[7 + a] = in.scaling[(3 + a) * A + ai];
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) q[10 + c] = gr.dquats[c * N + g];
      const float th = tanhf(y[j]);
      y[j] = th > 0.f ? q[0] * (1.f - th * th) : 0.f;
      for (int c = 0; c < 3; ++c) {
        const float s = sigm(yc[c]);
        yc[c] = q[1 + c] * s * (1.f - s);
      }
      for (int a = 0; a < 3; ++a) {
        const float s = sigm(yv[a]);
        yv[a] = q[4 + a] * q[7 + a] * s * (1.f - s);
      }
      const float q0 = yv[3], q1 = yv[4], q2 = yv[5], q3 = yv[6];
      const float nrm = sqrtf(q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3);
      const float n0 = q0 / nrm, n1 = q1 / nrm, n2 = q2 / nrm, n3 = q3 / nrm;
      const float d0 = q[10], d1 = q[11], d2 = q[12], d3 = q[13];
      const float dot = n0 * d0 + n1 * d1 + n2 * d2 + n3 * d3;
      yv[3] = (d0 - n0 * dot) / nrm;
      yv[4] = (d1 - n1 * dot) / nrm;
      yv[5] = (d2 - n2 * dot) / nrm;
      yv[6] = (d3 - n3 * dot) / nrm;
    }
    // padded columns 10..31, 62..63, 134..159 (50 per row)
    for (int it = tid; it < kTile * 50; it += kBwdThreads) {
      const int mm = it / 50, p = it % 50;
      const int col = p < 22 ? 10 + p : p < 24 ? 62 + (p - 22) : 134 + (p - 24);
      sY[mm * kYS + col] = 0.f;
    }
    __syncthreads();
    const int row = 16 * wr + m;
    // dL/dh = W2^T dy per head (this wavefront's N-tile h of its 32 hidden
    // units), through the ReLU into dL/dz
    {
      int t = 0;
#pragma unroll
      for (int hd = 0; hd < 3; ++hd) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < head_k_steps(hd); ++s) {
          bf16x8 hi, lo;
          split8(sY + row * kYS + head_base(hd) + 32 * s + 8 * kq, 1, hi, lo);
          acc = mfma(hi, Wb.w2t[t], acc);
          acc = mfma(lo, Wb.w2t[t], acc);
          ++t;
        }
        const int hid = kHid * hd + 16 * h + m;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int r = 16 * wr + 4 * kq + i;
          sZ[r * kZS + hid] = sH[r * kHS + hid] != 0 ? acc[i] : 0.f;
        }
      }
    }
    __syncthreads();
    // dL/dfeat = (W1^T dz)[0..31], inputs 16 h .. 16 h + 15
    {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < 3; ++s) {
        bf16x8 hi, lo;
        split8(sZ + row * kZS + 32 * s + 8 * kq, 1, hi, lo);
        acc = mfma(hi, Wb.w1t[s], acc);
        acc = mfma(lo, Wb.w1t[s], acc);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) sD[(16 * h + m) * kDS + 16 * wr + 4 * kq + i] = acc[i];
    }
    // weight gradients over this tile (K = anchors, two 32-anchor steps)
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int idx = 2 * w + q, mt = idx >> 1, nt = idx & 1;
      const int hd = mt == 0 ? 0 : mt < 3 ? 1 : 2;
      const int lt = mt == 0 ? 0 : mt < 3 ? mt - 1 : mt - 3;
      const int colb = head_base(hd) + 16 * lt;
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const int k0 = 32 * s + 8 * kq;
        bf16x8 hi, lo;
        split8(sY + k0 * kYS + colb + m, kYS, hi, lo);
        const bf16x8 b = gather8(sH + k0 * kHS + kHid * hd + 16 * nt + m, kHS);
        accW2[q] = mfma(hi, b, accW2[q]);
        accW2[q] = mfma(lo, b, accW2[q]);
      }
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const int idx = w + 8 * q;
      if (idx < 18) {
        const int mt = idx / 3, nt = idx % 3;
#pragma unroll
        for (int s = 0; s < 2; ++s) {
          const int k0 = 32 * s + 8 * kq;
          bf16x8 hi, lo;
          split8(sZ + k0 * kZS + 16 * mt + m, kZS, hi, lo);
          const bf16x8 b = gather8(sX + k0 * kXS + 16 * nt + m, kXS);
          accW1[q] = mfma(hi, b, accW1[q]);
          accW1[q] = mfma(lo, b, accW1[q]);
        }
      }
    }
    if (tid < 160) {
      for (int r = 0; r < kTile; ++r) dbias += sY[r * kYS + tid];
    } else if (tid < 160 + kHidAll) {
      for (int r = 0; r < kTile; ++r) dbias += sZ[r * kZS + tid - 160];
    }
    __syncthreads();
    if (gr.dfeat)
      for (int e = tid; e < kFeat * kTile; e += kBwdThreads) {
        const int k = e / kTile, mm = e % kTile;
        const int64_t ai = a0 + mm;
        if (ai < A) put(gr.dfeat + k * A + ai, sD[k * kDS + mm], gr.accumulate);
      }
    __syncthreads();
  }
  // partial sums of this workgroup
  float* ws = gr.ws + (int64_t)blockIdx.x * kWsFloats;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int idx = 2 * w + q, mt = idx >> 1, nt = idx & 1;
    const int hd = mt == 0 ? 0 : mt < 3 ? 1 : 2;
    const int lt = mt == 0 ? 0 : mt < 3 ? mt - 1 : mt - 3;
    const int colb = head_base(hd) + 16 * lt;
#pragma unroll
    for (int i = 0; i < 4; ++i) ws[kWsW2 + (colb + 4 * kq + i) * kHid + 16 * nt + m] = accW2[q][i];
  }
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const int idx = w + 8 * q;
    if (idx < 18) {
      const int mt = idx / 3, nt = idx % 3;
#pragma unroll
      for (int i = 0; i < 4; ++i) ws[kWsW1 + (16 * mt + 4 * kq + i) * 48 + 16 * nt + m] = accW1[q][i];
    }
  }
  if (tid < 160) ws[kWsB2 + tid] = dbias;
  else if (tid < 160 + kHidAll) ws[kWsB1 + tid - 160] = dbias;
}

// Sum of the per-workgroup partials (deterministic): a block takes 32
// parameters; thread group g (of 8) sums the partials of workgroups g, g + 8,
// ... in order, then the 8 group sums are added in group order.
constexpr int kRedParams = 32, kRedGroups = 8;
__global__ void __launch_bounds__(kRedParams* kRedGroups) k_decode_reduce(
    const float* __restrict__ ws, int nblk, float* __restrict__ dw1, float* __restrict__ db1,
    float* __restrict__ dw2, float* __restrict__ db2, int accumulate) {
  __shared__ float part[kRedGroups][kRedParams];
  const int lp = threadIdx.x % kRedParams, grp = threadIdx.x / kRedParams;
  const int t = blockIdx.x * kRedParams + lp;
  int src = -1;
  float* dst = nullptr;
  if (t < kHidAll * kIn) {
    src = kWsW1 + (t / kIn) * 48 + t % kIn;
    dst = dw1 + t;
  } else if (t < kHidAll * kIn + kHidAll) {
    const int h = t - kHidAll * kIn;
    src = kWsB1 + h;
    dst = db1 + h;
  } else if (t < kHidAll * kIn + kHidAll + kOut * kHid) {
    const int u = t - kHidAll * kIn - kHidAll, r = u / kHid, c = u % kHid;
    const int hd = r < 10 ? 0 : r < 40 ? 1 : 2;
    src = kWsW2 + (head_base(hd) + r - head_row(hd)) * kHid + c;
    dst = dw2 + u;
  } else if (t < kHidAll * kIn + kHidAll + kOut * kHid + kOut) {
    const int r = t - kHidAll * kIn - kHidAll - kOut * kHid;
    const int hd = r < 10 ? 0 : r < 40 ? 1 : 2;
    src = kWsB2 + head_base(hd) + r - head_row(hd);
    dst = db2 + r;
  }
  float s = 0.f;
  if (src >= 0) {
#pragma unroll 4
    for (int b = grp; b < nblk; b += kRedGroups) s += ws[(int64_t)b * kWsFloats + src];
  }
  part[grp][lp] = s;
  __syncthreads();
  if (grp == 0 && src >= 0) {
    float tot = 0.f;
#pragma unroll
    for (int k = 0; k < kRedGroups; ++k) tot += part[k][lp];
    put(dst, tot, accumulate);
  }
}

constexpr int kParamCount = kHidAll * kIn + kHidAll + kOut * kHid + kOut;

int decode_blocks(int64_t A) {
  const int64_t tiles = (A + kTile - 1) / kTile;
  return (int)(tiles < kMaxBlocks ? tiles : kMaxBlocks);
}

bool anchors_ok(const gs_anchors* a) {
  return a && a->feat && a->pos && a->offsets && a->scaling;
}
bool mlp_ok(const gs_mlp* p) { return p && p->w1 && p->b1 && p->w2 && p->b2; }

DecIn make_in(const gs_anchors* a, int64_t A, const gs_mlp* p, const CamDev& cd) {
  DecIn in;
  in.feat = a->feat; in.pos = a->pos; in.offsets = a->offsets; in.scaling = a->scaling;
  in.w1 = p->w1; in.b1 = p->b1; in.w2 = p->w2; in.b2 = p->b2;
  in.A = A;
  in.cx = cd.campos[0]; in.cy = cd.campos[1]; in.cz = cd.campos[2];
  return in;
}

}  // namespace

}  // namespace gs

using namespace gs;

extern "C" gs_status gs_anchor_decode_fwd(const gs_anchors* anchors, int64_t n_anchors,
                                          const gs_mlp* mlp, const gs_camera* cam,
                                          gs_gaussians* out, void* stream) {
  CamDev cd;
  if (n_anchors < 0 || n_anchors > ((int64_t)1 << 28) || !make_cam(cam, &cd)) return GS_EINVAL;
  if (n_anchors == 0) return GS_OK;
  if (!anchors_ok(anchors) || !mlp_ok(mlp) || !out || !out->means || !out->log_scales ||
      !out->quats || !out->opacity_logits || !out->sh)
    return GS_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const DecIn in = make_in(anchors, n_anchors, mlp, cd);
  const int64_t tiles = (n_anchors + kTile - 1) / kTile;
  const int nb = (int)(tiles < 512 ? tiles : 512);
  GS_TIMED("decode_fwd", st,
           k_decode_fwd<<<nb, kThreads, 0, st>>>(in, out->means, out->log_scales, out->quats,
                                                 out->opacity_logits, out->sh));
  GS_CHECK_LAUNCH();
  return GS_OK;
}

extern "C" gs_status gs_anchor_decode_workspace(int64_t n_anchors, size_t* bytes) {
  if (n_anchors < 0 || !bytes) return GS_EINVAL;
  *bytes = (size_t)decode_blocks(n_anchors) * kWsFloats * sizeof(float);
  return GS_OK;
}

namespace gs {
namespace {

// The backward's two launches on a caller-given partial-sum buffer `ws` of
// decode_blocks(A) * kWsFloats floats (every launched workgroup writes all of
// its partials, so the buffer needs no clearing). `timed`: bracket the
// launches with the launch timer (which creates events; the allocation-free
// entry point passes false).
gs_status decode_bwd_launch(const gs_anchors* anchors, int64_t n_anchors, const gs_mlp* mlp,
                            const CamDev& cd, const gs_gaussians* dchild, gs_anchors* danchors,
                            gs_mlp* dmlp, float* ws, int32_t accumulate, hipStream_t st,
                            bool timed) {
  const int nb = decode_blocks(n_anchors);
  if (n_anchors > 0) {
    const DecIn in = make_in(anchors, n_anchors, mlp, cd);
    DecGrad gr;
    gr.dmeans = dchild->means; gr.dscales = dchild->log_scales; gr.dquats = dchild->quats;
    gr.dopac = dchild->opacity_logits; gr.drgb = dchild->sh;
    gr.dfeat = danchors->feat; gr.doffsets = danchors->offsets; gr.dscaling = danchors->scaling;
    gr.ws = ws;
    gr.accumulate = accumulate;
    if (timed)
      GS_TIMED("decode_bwd", st, k_decode_bwd<<<nb, kBwdThreads, 0, st>>>(in, gr));
    else
      k_decode_bwd<<<nb, kBwdThreads, 0, st>>>(in, gr);
    GS_CHECK_LAUNCH();
  }
  const int rb = div_up(kParamCount, kRedParams);
  const int rnb = n_anchors > 0 ? nb : 0;
  if (timed)
    GS_TIMED("decode_reduce", st,
             k_decode_reduce<<<rb, kRedParams * kRedGroups, 0, st>>>(
                 ws, rnb, dmlp->w1, dmlp->b1, dmlp->w2, dmlp->b2, accumulate));
  else
    k_decode_reduce<<<rb, kRedParams * kRedGroups, 0, st>>>(ws, rnb, dmlp->w1, dmlp->b1,
                                                            dmlp->w2, dmlp->b2, accumulate);
  GS_CHECK_LAUNCH();
  return GS_OK;
}

// Arguments shared by both backward entry points: GS_EINVAL checks.
bool decode_bwd_args_ok(const gs_anchors* anchors, int64_t n_anchors, const gs_mlp* mlp,
                        const gs_camera* cam, const gs_gaussians* dchild,
                        const gs_anchors* danchors, const gs_mlp* dmlp, int32_t accumulate,
                        CamDev* cd) {
  if (n_anchors < 0 || n_anchors > ((int64_t)1 << 28) || !make_cam(cam, cd) ||
      (accumulate != 0 && accumulate != 1) || !mlp_ok(dmlp))
    return false;
  if (n_anchors > 0 &&
      (!anchors_ok(anchors) || !mlp_ok(mlp) || !dchild || !dchild->means ||
       !dchild->log_scales || !dchild->quats || !dchild->opacity_logits || !dchild->sh ||
       !danchors))
    return false;
  return true;
}

}  // namespace
}  // namespace gs

extern "C" gs_status gs_anchor_decode_bwd(const gs_anchors* anchors, int64_t n_anchors,
                                          const gs_mlp* mlp, const gs_camera* cam,
                                          const gs_gaussians* dchild, gs_anchors* danchors,
                                          gs_mlp* dmlp, void* workspace, size_t workspace_bytes,
                                          int32_t accumulate, void* stream) {
  CamDev cd;
  if (!decode_bwd_args_ok(anchors, n_anchors, mlp, cam, dchild, danchors, dmlp, accumulate, &cd))
    return GS_EINVAL;
  const int nb = decode_blocks(n_anchors);
  if (n_anchors > 0 &&
      (!workspace || workspace_bytes < (size_t)nb * kWsFloats * sizeof(float)))
    return GS_ECAPACITY;
  return decode_bwd_launch(anchors, n_anchors, mlp, cd, dchild, danchors, dmlp,
                           (float*)workspace, accumulate, (hipStream_t)stream, true);
}

// ---------------------------------------------------------------------------
// Allocation-free backward: the per-workgroup partials live in a fixed
// device array of the library instead of a caller workspace. The array is
// sized for the largest grid the backward launches (kMaxBlocks workgroups,
// whatever the anchor count), so every A the backward accepts fits.
static __device__ __align__(256) float scratch[kMaxBlocks * kWsFloats];
static_assert(sizeof(scratch) == GS_DECODE_SCRATCH_BYTES, "header states the scratch size");

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch[kMaxDevices] = {};  // device address of `scratch`, per device

// The address of the current device's copy of `scratch`, looked up once per
// device (with that device current) and kept; never the array's host-side
// name, which is no device address.
gs_status scratch_on_current_device(float** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return GS_EHIP;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return GS_EHIP;
    g_scratch[dev] = static_cast<float*>(p);
  }
  *out = g_scratch[dev];
  return GS_OK;
}
}  // namespace

extern "C" gs_status gs_anchor_decode_bwd_noalloc(const gs_anchors* anchors, int64_t n_anchors,
                                                  const gs_mlp* mlp, const gs_camera* cam,
                                                  const gs_gaussians* dchild,
                                                  gs_anchors* danchors, gs_mlp* dmlp,
                                                  int32_t accumulate, void* stream) {
  CamDev cd;
  if (!decode_bwd_args_ok(anchors, n_anchors, mlp, cam, dchild, danchors, dmlp, accumulate, &cd))
    return GS_EINVAL;
  if ((size_t)decode_blocks(n_anchors) * kWsFloats > sizeof(scratch) / sizeof(float))
    return GS_ECAPACITY;
  float* ws = nullptr;
  const gs_status st = scratch_on_current_device(&ws);
  if (st != GS_OK) return st;
  return decode_bwd_launch(anchors, n_anchors, mlp, cd, dchild, danchors, dmlp, ws, accumulate,
                           (hipStream_t)stream, false);
}
