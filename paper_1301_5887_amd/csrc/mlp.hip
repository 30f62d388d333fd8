// The control-variate network on the matrix cores: forward, backward and
// Adam for a 4 -> 64 -> 64 -> 1 perceptron (GELU, sigmoid) with BF16 weights
// and FP32 accumulation, on v_mfma_f32_16x16x16_bf16.
//
// Layout.  One wave carries 16 samples through the network as the columns
// of 16x16 tiles.  Layers are computed transposed, H^T = W X^T, so the
// output tile of one product (lane l holds rows 4*(l/16)..+3 of column
// l%16) is exactly the B operand of the next: activations never leave
// registers on the forward pass.  The weight-gradient products, whose inner
// dimension is the sample, take their operands through LDS (one 64x16 BF16
// tile each).  The first layer's inner dimension of 4 features is padded to
// 16 with zeros; the 64 -> 1 output is a dot product on the vector unit.
#include <math.h>

#include "common.hpp"
#include "rng.hpp"

namespace wedge {

constexpr int kH = 64;
constexpr int OFF_W1 = 0, OFF_B1 = 256, OFF_W2 = 320, OFF_B2 = 4416, OFF_W3 = 4480,
              OFF_B3 = 4544, NPARAM = 4545, kPad = 4608;
constexpr uint64_t kDomainInit = 5;

struct MlpState {
  float master[kPad];
  uint16_t bf[kPad];
  float m[kPad];
  float v[kPad];
  uint16_t w2t[kH * kH];  // BF16 W2^T in MFMA A-operand order [m][kk][lane][j]
  uint16_t w2a[kH * kH];  // BF16 W2 in MFMA A-operand order [m][kk][lane][j]
};

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ inline f4 mfma16(s4 a, s4 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// float -> bfloat16, round to nearest even
__device__ inline uint16_t f2bf(float x) {
  uint32_t b = __float_as_uint(x);
  b += 0x7FFFu + ((b >> 16) & 1u);
  return (uint16_t)(b >> 16);
}
__device__ inline float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ inline s4 pack4(uint16_t a, uint16_t b, uint16_t c, uint16_t d) {
  s4 r;
  r[0] = (short)a;
  r[1] = (short)b;
  r[2] = (short)c;
  r[3] = (short)d;
  return r;
}


// Writes parameter p: FP32 master, BF16 copy and, for W2, its place in the
// transposed operand tiles (W2[o][i] is element j = o % 4 of lane
// 16 ((o % 16) / 4) + i % 16 of tile (m, kk) = (i / 16, o / 16)).
__device__ inline void store_param(MlpState* S, int p, float w) {
  S->master[p] = w;
  const uint16_t b = f2bf(w);
  S->bf[p] = b;
  if (p >= OFF_W2 && p < OFF_W2 + kH * kH) {
    const int o = (p - OFF_W2) / kH, i = (p - OFF_W2) % kH;
    const int lane_t = 16 * ((o % 16) / 4) + i % 16;
    S->w2t[(((i / 16) * 4 + o / 16) * 64 + lane_t) * 4 + o % 4] = b;
    // W2[o][i] is element j = i % 4 of lane 16 ((i % 16) / 4) + o % 16 of
    // tile (m, kk) = (o / 16, i / 16) of the forward product
    const int lane_a = 16 * ((i % 16) / 4) + o % 16;
    S->w2a[(((o / 16) * 4 + i / 16) * 64 + lane_a) * 4 + i % 4] = b;
  }
}

// GELU(a) = a Phi(a) with Phi the standard normal CDF; its derivative is
// Phi(a) + a phi(a).  The forward pass keeps Phi for the backward pass.
// erf is the branch-free rational approximation 7.1.26 of Abramowitz and
// Stegun (Handbook of Mathematical Functions, 1964): for x >= 0,
// erf x = 1 - (a1 t + ... + a5 t^5) exp(-x^2), t = 1 / (1 + p x), with
// absolute error below 1.5e-7, far inside the BF16 rounding of the network.
__device__ inline float norm_cdf(float a) {
  const float x = fabsf(a) * 0.70710678118654752f;
  const float t = 1.0f / (1.0f + 0.3275911f * x);
  const float poly =
      t * (0.254829592f +
           t * (-0.284496736f + t * (1.421413741f + t * (-1.453152027f + t * 1.061405429f))));
  const float erf_x = 1.0f - poly * __expf(-x * x);
  return 0.5f + 0.5f * (a < 0.f ? -erf_x : erf_x);
}
__device__ inline float gelu_grad_from(float a, float cdf) {
  return cdf + a * (__expf(-0.5f * a * a) * 0.39894228040143268f);
}

// Log-degree bucket K(d) = floor(8 L(d)), L Mitchell's log2, in integers.
__device__ inline uint32_t log_bucket(uint32_t d) {
  if (d == 0) return 0;
  const uint32_t e = 31 - __clz(d);
  return 8 * e + (uint32_t)((((uint64_t)d - (1ULL << e)) * 8) >> e);
}

// x = (K(d_v), K(d_lo), K(d_hi)) / 256 and bin / 32: every value is exact in
// BF16, so the network is a function of (bin, bucket, bucket, bucket).
__device__ inline void features(const wedge_feature_rec& r, float x[4]) {
  x[0] = (float)log_bucket(r.dv) * 0.00390625f;
  x[1] = (float)log_bucket(r.dlo) * 0.00390625f;
  x[2] = (float)log_bucket(r.dhi) * 0.00390625f;
  x[3] = (float)r.bin * 0.03125f;
}

// Weights of one wave in operand layout (sl = lane % 16, kb = lane / 16).
struct WaveWeights {
  s4 w1[4];       // layer-1 A tiles: W1[16m+sl][4kb+j] (zero for kb > 0)
  s4 w2[4][4];    // layer-2 A tiles [m][kk]: W2[16m+sl][16kk+4kb+j]
  float b1[4][4]; // b1[16m+4kb+t]
  float b2[4][4];
  float w3[4][4]; // BF16 W3[16m+4kb+t]
  float b3;
};

__device__ inline void load_weights(const MlpState* __restrict__ S, WaveWeights& W, int sl,
                                    int kb) {
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int r = 16 * m + sl;
    if (kb == 0)
      W.w1[m] = pack4(S->bf[OFF_W1 + r * 4 + 0], S->bf[OFF_W1 + r * 4 + 1],
                      S->bf[OFF_W1 + r * 4 + 2], S->bf[OFF_W1 + r * 4 + 3]);
    else
      W.w1[m] = pack4(0, 0, 0, 0);
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int c = OFF_W2 + r * kH + 16 * kk + 4 * kb;
      W.w2[m][kk] = pack4(S->bf[c], S->bf[c + 1], S->bf[c + 2], S->bf[c + 3]);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int h = 16 * m + 4 * kb + t;
      W.b1[m][t] = S->master[OFF_B1 + h];
      W.b2[m][t] = S->master[OFF_B2 + h];
      W.w3[m][t] = bf2f(S->bf[OFF_W3 + h]);
    }
  }
  W.b3 = S->master[OFF_B3];
}

struct TileAct {
  float a1[4][4];  // pre-activations A1^T[16m+4kb+t][sl]
  float c1[4][4];  // Phi(a1)
  s4 h1[4];        // BF16 H1^T tiles (B operands of layer 2)
  float a2[4][4];
  float c2[4][4];  // Phi(a2); H2 = a2 * c2
  float z;         // logit of sample sl (same in the 4 lanes of the column)
};

// Biases and output weights held in registers (forward kernel).
struct RegBias {
  const WaveWeights& W;
  __device__ float b1(int m, int t) const { return W.b1[m][t]; }
  __device__ float b2(int m, int t) const { return W.b2[m][t]; }
  __device__ float w3(int m, int t) const { return W.w3[m][t]; }
  __device__ float b3() const { return W.b3; }
};

// Layer-2 A operands held in registers (forward kernel) or read from LDS.
struct RegW2 {
  const s4 (&w)[4][4];
  __device__ s4 operator()(int m, int kk) const { return w[m][kk]; }
};
struct LdsW2 {
  const s4 (*w)[4][64];
  int lane;
  __device__ s4 operator()(int m, int kk) const { return w[m][kk][lane]; }
};

template <class Bias, class W2>
__device__ inline void forward_tile(const s4 (&w1)[4], const W2& w2, const Bias& Bs,
                                    const float x[4], int kb, TileAct& T) {
  const s4 xb = kb == 0 ? pack4(f2bf(x[0]), f2bf(x[1]), f2bf(x[2]), f2bf(x[3])) : pack4(0, 0, 0, 0);
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    f4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = mfma16(w1[m], xb, acc);
    uint16_t hb[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const float a = acc[t] + Bs.b1(m, t);
      const float c = norm_cdf(a);
      T.a1[m][t] = a;
      T.c1[m][t] = c;
      hb[t] = f2bf(a * c);
    }
    T.h1[m] = pack4(hb[0], hb[1], hb[2], hb[3]);
  }
  float part = 0.f;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) acc = mfma16(w2(m, kk), T.h1[kk], acc);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const float a = acc[t] + Bs.b2(m, t);
      const float c = norm_cdf(a);
      T.a2[m][t] = a;
      T.c2[m][t] = c;
      part += Bs.w3(m, t) * (a * c);
    }
  }
  part += __shfl_xor(part, 16, 64);
  part += __shfl_xor(part, 32, 64);
  T.z = part + Bs.b3();
}

__global__ __launch_bounds__(256) void k_mlp_forward(const MlpState* __restrict__ S,
                                                     const wedge_feature_rec* __restrict__ x,
                                                     uint64_t n, float* __restrict__ g) {
  const int lane = threadIdx.x & 63, sl = lane & 15, kb = lane >> 4;
  const uint64_t wave = (uint64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  const uint64_t nwaves = (uint64_t)gridDim.x * (blockDim.x / 64);
  WaveWeights W;
  load_weights(S, W, sl, kb);
  for (uint64_t tile = wave; tile * 16 < n; tile += nwaves) {
    const uint64_t i = tile * 16 + sl;
    const bool valid = i < n;
    float xf[4] = {0.f, 0.f, 0.f, 0.f};
    if (valid) features(x[i], xf);
    TileAct T;
    forward_tile(W.w1, RegW2{W.w2}, RegBias{W}, xf, kb, T);
    if (kb == 0 && valid) g[i] = 1.0f / (1.0f + expf(-T.z));
  }
}

// Record i of a minibatch made of `per` consecutive records from each of the
// rows of a [rows][stride] block, starting at column j0 of every row.
struct RowView {
  const wedge_feature_rec* x;
  uint64_t stride, j0, per;
  __device__ const wedge_feature_rec& operator[](uint64_t i) const {
    return x[(i / per) * stride + j0 + (i % per)];
  }
};

constexpr int kGradWaves = 4;
constexpr int kGradTilesPerWave = 4;
constexpr uint64_t kGradChunk = 16ULL * kGradWaves * kGradTilesPerWave;  // records per WG

// LDS operand tiles of one wave (transposes for the weight-gradient products).
// Rows hold 16 values padded to 20 (40 bytes): 8-byte reads stay aligned and
// the rows a wave touches at once fall in different banks.
constexpr int kGradRow = 20;
struct GradSmem {
  uint16_t da2[kH][kGradRow];  // dA2^T [o][s]
  uint16_t h1[kH][kGradRow];   // H1^T  [i][s]
  uint16_t da1[kH][kGradRow];  // dA1^T [i][s]
  uint16_t x[16][kGradRow];    // X     [s][f], f >= 4 zero
};

// Biases and output weights read from LDS (gradient kernel).
struct LdsBias {
  const float* pb1;
  const float* pb2;
  const float* pw3;
  float pb3;
  int kb;
  __device__ float b1(int m, int t) const { return pb1[16 * m + 4 * kb + t]; }
  __device__ float b2(int m, int t) const { return pb2[16 * m + 4 * kb + t]; }
  __device__ float w3(int m, int t) const { return pw3[16 * m + 4 * kb + t]; }
  __device__ float b3() const { return pb3; }
};

// Gradient of the mean BCE over minibatch records [kGradChunk*wg, +kGradChunk)
// into partial[wg][kPad] (entry NPARAM holds the loss sum).  Four waves per
// workgroup work in rounds: each wave carries its own 16-record tile through
// the network and leaves dA2^T, H1^T, dA1^T and X in LDS; then wave w forms
// rows 16w .. 16w+15 of dW2 and dW1 from all four tiles, so every weight
// gradient has one owner and no cross-wave sum.  The bias and W3 sums are
// added up at the end in a fixed order (waves, then sample columns), so the
// result does not depend on scheduling.
__global__ __launch_bounds__(64 * kGradWaves, 2) void k_mlp_grad(const MlpState* __restrict__ S,
                                                                 RowView x, uint64_t n,
                                                                 float inv_n,
                                                                 float* __restrict__ partial) {
  struct LoopSmem {
    GradSmem w[kGradWaves];
    float b1[kH], b2[kH], w3[kH], b3;
    s4 w2t[4][4][64];  // A tiles of W2^T [m][kk][lane]
    s4 w2[4][4][64];   // A tiles of W2 [m][kk][lane]
  };
  struct EndSmem {
    float col[kGradWaves][3][kH][16];  // W3, b2, b1 sums per sample column
    float sc[kGradWaves][2][64];       // b3 and loss per lane
  };
  __shared__ union {
    LoopSmem loop;
    EndSmem end;
  } u;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int sl = lane & 15, kb = lane >> 4;
  GradSmem& sm = u.loop.w[wave];
  s4 w1[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int r = 16 * m + sl;
    w1[m] = kb == 0 ? pack4(S->bf[OFF_W1 + r * 4 + 0], S->bf[OFF_W1 + r * 4 + 1],
                            S->bf[OFF_W1 + r * 4 + 2], S->bf[OFF_W1 + r * 4 + 3])
                    : pack4(0, 0, 0, 0);
  }
  if (tid < kH) {
    u.loop.b1[tid] = S->master[OFF_B1 + tid];
    u.loop.b2[tid] = S->master[OFF_B2 + tid];
    u.loop.w3[tid] = bf2f(S->bf[OFF_W3 + tid]);
    if (tid == 0) u.loop.b3 = S->master[OFF_B3];
  }
  for (int e = tid; e < 16 * 64; e += 64 * kGradWaves) {
    (&u.loop.w2t[0][0][0])[e] = reinterpret_cast<const s4*>(S->w2t)[e];
    (&u.loop.w2[0][0][0])[e] = reinterpret_cast<const s4*>(S->w2a)[e];
  }
  __syncthreads();
  const LdsBias Bs{u.loop.b1, u.loop.b2, u.loop.w3, u.loop.b3, kb};
  const LdsW2 W2{u.loop.w2, lane};
  f4 dW2[4], dW1 = {0.f, 0.f, 0.f, 0.f};  // rows 16 wave + 4 kb + t of the products
#pragma unroll
  for (int nn = 0; nn < 4; ++nn) dW2[nn] = f4{0.f, 0.f, 0.f, 0.f};
  float gW3[4][4], gb2[4][4], gb1[4][4];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int t = 0; t < 4; ++t) gW3[m][t] = gb2[m][t] = gb1[m][t] = 0.f;
  float gb3 = 0.f, lsum = 0.f;

  const uint64_t begin = (uint64_t)blockIdx.x * kGradChunk;
  const uint64_t end = min(begin + kGradChunk, n);
  // the next round's record is loaded while the current tile is computed
  wedge_feature_rec next{};
  {
    const uint64_t i0 = begin + 16 * (uint64_t)wave + sl;
    if (i0 < end) next = x[i0];
  }
  for (int round = 0; round < kGradTilesPerWave; ++round) {
    const uint64_t i = begin + 16 * ((uint64_t)round * kGradWaves + wave) + sl;
    const bool valid = i < end;
    const wedge_feature_rec r = next;
    {
      const uint64_t i2 = i + 16 * kGradWaves;
      if (round + 1 < kGradTilesPerWave && i2 < end) next = x[i2];
    }
    float xf[4] = {0.f, 0.f, 0.f, 0.f};
    float y = 0.f;
    if (valid) {
      features(r, xf);
      y = r.closed ? 1.f : 0.f;
    }
    TileAct T;
    forward_tile(w1, W2, Bs, xf, kb, T);
    const float gz = 1.0f / (1.0f + expf(-T.z));
    const float dz = valid ? (gz - y) * inv_n : 0.f;
    if (kb == 0) {
      gb3 += dz;
      if (valid) lsum += fmaxf(T.z, 0.f) + log1pf(expf(-fabsf(T.z))) - y * T.z;
    }
    float da2[4][4];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int h = 16 * m + 4 * kb + t;
        gW3[m][t] += dz * (T.a2[m][t] * T.c2[m][t]);
        da2[m][t] = dz * Bs.w3(m, t) * gelu_grad_from(T.a2[m][t], T.c2[m][t]);
        gb2[m][t] += da2[m][t];
        sm.da2[h][sl] = f2bf(da2[m][t]);
        sm.h1[h][sl] = (uint16_t)T.h1[m][t];
      }
#pragma unroll
    for (int j = 0; j < 4; ++j) sm.x[sl][4 * kb + j] = kb == 0 ? f2bf(xf[j]) : (uint16_t)0;
    // dH1^T = W2^T dA2^T; dA1^T = dH1^T * GELU'(A1^T)
    s4 bda2[4];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk)
      bda2[kk] = pack4(f2bf(da2[kk][0]), f2bf(da2[kk][1]), f2bf(da2[kk][2]), f2bf(da2[kk][3]));
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) acc = mfma16(u.loop.w2t[m][kk][lane], bda2[kk], acc);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const float da1 = acc[t] * gelu_grad_from(T.a1[m][t], T.c1[m][t]);
        gb1[m][t] += da1;
        sm.da1[16 * m + 4 * kb + t][sl] = f2bf(da1);
      }
    }
    __syncthreads();
    // rows 16 wave .. +15 of dW2[o][i] += sum_s dA2^T[o][s] H1^T[i][s] and of
    // dW1[i][f] += sum_s dA1^T[i][s] X[s][f], over the four tiles
#pragma unroll
    for (int j = 0; j < kGradWaves; ++j) {
      const GradSmem& tj = u.loop.w[j];
      const s4 a2 = *reinterpret_cast<const s4*>(&tj.da2[16 * wave + sl][4 * kb]);
#pragma unroll
      for (int nn = 0; nn < 4; ++nn) {
        const s4 b = *reinterpret_cast<const s4*>(&tj.h1[16 * nn + sl][4 * kb]);
        dW2[nn] = mfma16(a2, b, dW2[nn]);
      }
      const s4 a1 = *reinterpret_cast<const s4*>(&tj.da1[16 * wave + sl][4 * kb]);
      const s4 bx = pack4(tj.x[4 * kb + 0][sl], tj.x[4 * kb + 1][sl], tj.x[4 * kb + 2][sl],
                          tj.x[4 * kb + 3][sl]);
      dW1 = mfma16(a1, bx, dW1);
    }
    __syncthreads();
  }
  float* P = partial + (uint64_t)blockIdx.x * kPad;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int o = 16 * wave + 4 * kb + t;
#pragma unroll
    for (int nn = 0; nn < 4; ++nn) P[OFF_W2 + o * kH + 16 * nn + sl] = dW2[nn][t];
    if (sl < 4) P[OFF_W1 + o * 4 + sl] = dW1[t];
  }
  EndSmem& E = u.end;  // the loop's LDS is free after the last barrier
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int h = 16 * m + 4 * kb + t;
      E.col[wave][0][h][sl] = gW3[m][t];
      E.col[wave][1][h][sl] = gb2[m][t];
      E.col[wave][2][h][sl] = gb1[m][t];
    }
  E.sc[wave][0][lane] = kb == 0 ? gb3 : 0.f;
  E.sc[wave][1][lane] = kb == 0 ? lsum : 0.f;
  __syncthreads();
  // b1, b2, W3 (64 each), b3 and the loss sum: added in a fixed order
  for (int q = tid; q < 3 * kH + 2; q += 64 * kGradWaves) {
    float v = 0.f;
    int p;
    if (q < 3 * kH) {
      const int which = q / kH, h = q % kH;  // 0: W3, 1: b2, 2: b1
      for (int w = 0; w < kGradWaves; ++w)
        for (int c = 0; c < 16; ++c) v += E.col[w][which][h][c];
      p = (which == 0 ? OFF_W3 : which == 1 ? OFF_B2 : OFF_B1) + h;
    } else {
      const int j = q - 3 * kH;  // 0: b3, 1: loss (kept in the padding entry NPARAM)
      for (int w = 0; w < kGradWaves; ++w)
        for (int l = 0; l < 64; ++l) v += E.sc[w][j][l];
      p = OFF_B3 + j;
    }
    P[p] = v;
  }
}

// Sum of the partial gradients (deterministic: wave q of a block sums the
// workgroups w = q mod 16 in order, and the 16 sums are added in q order);
// the padding entry NPARAM carries the loss sum.
constexpr int kRedSplit = 16;
__device__ inline float reduce_param(const float* __restrict__ partial, uint32_t nwg, int p,
                                     float (*s_q)[64], int lane, int q) {
  float s = 0.f;
  if (p <= NPARAM) {
#pragma unroll 4
    for (uint32_t w = q; w < nwg; w += kRedSplit) s += partial[(uint64_t)w * kPad + p];
  }
  s_q[q][lane] = s;
  __syncthreads();
  float t = 0.f;
  if (q == 0)
    for (int j = 0; j < kRedSplit; ++j) t += s_q[j][lane];
  return t;
}

__global__ __launch_bounds__(64 * kRedSplit) void k_mlp_reduce(const float* __restrict__ partial,
                                                               uint32_t nwg,
                                                               float* __restrict__ grad,
                                                               float inv_n,
                                                               float* __restrict__ loss) {
  __shared__ float s_q[kRedSplit][64];
  const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
  const int p = blockIdx.x * 64 + lane;
  const float t = reduce_param(partial, nwg, p, s_q, lane, q);
  if (q == 0 && p <= NPARAM) {
    if (p < NPARAM)
      grad[p] = t;
    else if (loss)
      *loss = t * inv_n;
  }
}

__device__ inline void adam_update(MlpState* S, int p, float g, float lr, float b1, float b2,
                                   float eps, float c1, float c2) {
  const float m = b1 * S->m[p] + (1.f - b1) * g;
  const float v = b2 * S->v[p] + (1.f - b2) * g * g;
  S->m[p] = m;
  S->v[p] = v;
  const float mh = m / c1, vh = v / c2;
  store_param(S, p, S->master[p] - lr * mh / (sqrtf(vh) + eps));
}

// The reduction above followed by the Adam step of each parameter.
__global__ __launch_bounds__(64 * kRedSplit) void k_mlp_reduce_adam(
    const float* __restrict__ partial, uint32_t nwg, MlpState* __restrict__ S, float inv_n,
    float* __restrict__ loss, float lr, float b1, float b2, float eps, float c1, float c2) {
  __shared__ float s_q[kRedSplit][64];
  const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
  const int p = blockIdx.x * 64 + lane;
  const float t = reduce_param(partial, nwg, p, s_q, lane, q);
  if (q == 0 && p <= NPARAM) {
    if (p < NPARAM)
      adam_update(S, p, t, lr, b1, b2, eps, c1, c2);
    else if (loss)
      *loss = t * inv_n;
  }
}

__global__ void k_mlp_adam(MlpState* __restrict__ S, const float* __restrict__ grad, float lr,
                           float b1, float b2, float eps, float c1, float c2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NPARAM) return;
  adam_update(S, p, grad[p], lr, b1, b2, eps, c1, c2);
}

__global__ void k_mlp_set(MlpState* __restrict__ S, const float* __restrict__ params) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kPad) return;
  store_param(S, p, p < NPARAM ? params[p] : 0.f);
  S->m[p] = 0.f;
  S->v[p] = 0.f;
}

__global__ void k_mlp_get(const MlpState* __restrict__ S, float* __restrict__ params) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < NPARAM) params[p] = S->master[p];
}

__global__ void k_mlp_init(MlpState* __restrict__ S, uint64_t seed) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kPad) return;
  float w = 0.f;
  if (p < NPARAM) {
    const float fan = (p < OFF_W2) ? 4.f : 64.f;  // W1, b1 see 4 inputs; the rest 64
    const U64x4 o = philox4x64_10((uint64_t)p, 0, 0, 0, seed, kDomainInit);
    const double u = (double)(o.w[0] >> 11) * (1.0 / 9007199254740992.0);
    w = (float)((2.0 * u - 1.0) / sqrt((double)fan));
  }
  store_param(S, p, w);
  S->m[p] = 0.f;
  S->v[p] = 0.f;
}

constexpr int kMomRows = 64;  // rows per launch
struct RowCounts {
  uint64_t n[kMomRows];
};

// Rows row0 + blockIdx.y; row r uses its first counts.n[blockIdx.y] records.
__global__ __launch_bounds__(256) void k_cv_moments(const wedge_feature_rec* __restrict__ x,
                                                    const float* __restrict__ g, uint64_t stride,
                                                    uint32_t row0, RowCounts counts,
                                                    long long* __restrict__ mom) {
  __shared__ long long s_m[4][5];
  const uint64_t row = row0 + blockIdx.y;
  const uint64_t npr = counts.n[blockIdx.y];
  long long c = 0, sx = 0, sg = 0, sg2 = 0, sxg = 0;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < npr;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t at = row * stride + i;
    const double gv = (double)g[at];
    const long long gq = llrint(gv * 4294967296.0);
    const long long g2q = llrint(gv * gv * 4294967296.0);
    const int X = (x && x[at].closed) ? 1 : 0;
    c += 1;
    sx += X;
    sg += gq;
    sg2 += g2q;
    sxg += X ? gq : 0;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    c += __shfl_xor(c, off, 64);
    sx += __shfl_xor(sx, off, 64);
    sg += __shfl_xor(sg, off, 64);
    sg2 += __shfl_xor(sg2, off, 64);
    sxg += __shfl_xor(sxg, off, 64);
  }
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    s_m[wave][0] = c;
    s_m[wave][1] = sx;
    s_m[wave][2] = sg;
    s_m[wave][3] = sg2;
    s_m[wave][4] = sxg;
  }
  __syncthreads();
  if (threadIdx.x < 5) {  // integer sums: the order of the atomics does not matter
    const long long t = s_m[0][threadIdx.x] + s_m[1][threadIdx.x] + s_m[2][threadIdx.x] +
                        s_m[3][threadIdx.x];
    atomicAdd((unsigned long long*)(mom + row * 5 + threadIdx.x), (unsigned long long)t);
  }
}

static uint32_t grad_groups(uint64_t n) { return (uint32_t)ceil_div(n, kGradChunk); }

// One minibatch: gradient into d_grad (and the mean loss into d_loss).
static int grad_impl(const MlpState* S, const wedge_feature_rec* d_x, uint64_t stride,
                     uint64_t j0, uint64_t per_row, uint64_t n, float* d_grad, float* d_loss,
                     float* partial, hipStream_t st) {
  const uint32_t nwg = grad_groups(n);
  const float inv_n = 1.0f / (float)n;
  RowView view{d_x, stride, j0, per_row};
  k_mlp_grad<<<nwg, 64 * kGradWaves, 0, st>>>(S, view, n, inv_n, partial);
  WEDGE_LAUNCH_CHECK("k_mlp_grad");
  k_mlp_reduce<<<(NPARAM + 1 + 63) / 64, 64 * kRedSplit, 0, st>>>(partial, nwg, d_grad, inv_n,
                                                                  d_loss);
  WEDGE_LAUNCH_CHECK("k_mlp_reduce");
  return WEDGE_OK;
}

static void adam_consts(uint32_t t, float b1, float b2, float* c1, float* c2) {
  *c1 = (float)(1.0 - pow((double)b1, (double)t));
  *c2 = (float)(1.0 - pow((double)b2, (double)t));
}

}  // namespace wedge

using namespace wedge;

extern "C" size_t wedge_mlp_state_bytes(void) { return round_up(sizeof(MlpState), 256); }

extern "C" int wedge_mlp_set(void* d_state, const float* d_params, void* stream) {
  clear_error();
  if (!d_state || !d_params) return set_error(WEDGE_EINVAL, "wedge_mlp_set: null pointer");
  if (!aligned(d_state, 256) || !aligned(d_params, 4))
    return set_error(WEDGE_EINVAL, "wedge_mlp_set: misaligned pointer");
  k_mlp_set<<<(kPad + 255) / 256, 256, 0, (hipStream_t)stream>>>((MlpState*)d_state, d_params);
  WEDGE_LAUNCH_CHECK("k_mlp_set");
  return WEDGE_OK;
}

extern "C" int wedge_mlp_get(const void* d_state, float* d_params, void* stream) {
  clear_error();
  if (!d_state || !d_params) return set_error(WEDGE_EINVAL, "wedge_mlp_get: null pointer");
  k_mlp_get<<<(kPad + 255) / 256, 256, 0, (hipStream_t)stream>>>((const MlpState*)d_state,
                                                                  d_params);
  WEDGE_LAUNCH_CHECK("k_mlp_get");
  return WEDGE_OK;
}

extern "C" int wedge_mlp_init(void* d_state, uint64_t seed, void* stream) {
  clear_error();
  if (!d_state || !aligned(d_state, 256))
    return set_error(WEDGE_EINVAL, "wedge_mlp_init: null or misaligned state");
  k_mlp_init<<<(kPad + 255) / 256, 256, 0, (hipStream_t)stream>>>((MlpState*)d_state, seed);
  WEDGE_LAUNCH_CHECK("k_mlp_init");
  return WEDGE_OK;
}

namespace wedge {
int mlp_forward_impl(const void* d_state, const wedge_feature_rec* d_x, uint64_t n, float* d_g,
                     hipStream_t st) {
  if (n == 0) return WEDGE_OK;
  uint64_t tiles = (n + 15) / 16;
  uint64_t blocks = (tiles + 3) / 4;
  if (blocks > 4096) blocks = 4096;
  k_mlp_forward<<<(unsigned)blocks, 256, 0, st>>>((const MlpState*)d_state, d_x, n, d_g);
  WEDGE_LAUNCH_CHECK("k_mlp_forward");
  return WEDGE_OK;
}
}  // namespace wedge

extern "C" int wedge_mlp_forward(const void* d_state, const wedge_feature_rec* d_x, uint64_t n,
                                 float* d_g, void* stream) {
  clear_error();
  if (n == 0) return WEDGE_OK;
  if (!d_state || !d_x || !d_g) return set_error(WEDGE_EINVAL, "wedge_mlp_forward: null pointer");
  if (!aligned(d_state, 256) || !aligned(d_x, 16) || !aligned(d_g, 4))
    return set_error(WEDGE_EINVAL, "wedge_mlp_forward: misaligned pointer");
  return mlp_forward_impl(d_state, d_x, n, d_g, (hipStream_t)stream);
}

extern "C" size_t wedge_mlp_grad_workspace(uint64_t n) {
  return round_up((size_t)grad_groups(n ? n : 1) * kPad * 4, 256);
}

extern "C" int wedge_mlp_grad(const void* d_state, const wedge_feature_rec* d_x, uint32_t rows,
                              uint64_t stride, uint64_t j0, uint64_t per_row, float* d_grad,
                              float* d_loss, void* d_workspace, size_t workspace_bytes,
                              void* stream) {
  clear_error();
  const uint64_t n = (uint64_t)rows * per_row;
  if (n == 0) return set_error(WEDGE_ERANGE, "wedge_mlp_grad: empty minibatch");
  if (j0 + per_row > stride) return set_error(WEDGE_ERANGE, "wedge_mlp_grad: j0 + per_row > stride");
  if (!d_state || !d_x || !d_grad || !d_workspace)
    return set_error(WEDGE_EINVAL, "wedge_mlp_grad: null pointer");
  if (!aligned(d_state, 256) || !aligned(d_x, 16) || !aligned(d_grad, 4) ||
      !aligned(d_workspace, 256))
    return set_error(WEDGE_EINVAL, "wedge_mlp_grad: misaligned pointer");
  if (workspace_bytes < wedge_mlp_grad_workspace(n))
    return set_error(WEDGE_EWORKSPACE, "wedge_mlp_grad: workspace too small");
  return grad_impl((const MlpState*)d_state, d_x, stride, j0, per_row, n, d_grad, d_loss,
                   (float*)d_workspace, (hipStream_t)stream);
}

extern "C" int wedge_mlp_adam(void* d_state, const float* d_grad, uint32_t t, float lr,
                              float beta1, float beta2, float eps, void* stream) {
  clear_error();
  if (!d_state || !d_grad) return set_error(WEDGE_EINVAL, "wedge_mlp_adam: null pointer");
  if (t == 0) return set_error(WEDGE_ERANGE, "wedge_mlp_adam: step t must be >= 1");
  float c1, c2;
  adam_consts(t, beta1, beta2, &c1, &c2);
  k_mlp_adam<<<(NPARAM + 255) / 256, 256, 0, (hipStream_t)stream>>>(
      (MlpState*)d_state, d_grad, lr, beta1, beta2, eps, c1, c2);
  WEDGE_LAUNCH_CHECK("k_mlp_adam");
  return WEDGE_OK;
}

extern "C" size_t wedge_mlp_train_workspace(uint32_t rows, uint64_t per_row_batch) {
  return wedge_mlp_grad_workspace((uint64_t)rows * per_row_batch) + round_up(kPad * 4, 256);
}

extern "C" int wedge_mlp_train(void* d_state, const wedge_feature_rec* d_x, uint32_t rows,
                               uint64_t stride, uint64_t n_fit, uint64_t per_row_batch,
                               uint32_t epochs, uint32_t t0, float lr, float beta1, float beta2,
                               float eps, float* d_loss, void* d_workspace,
                               size_t workspace_bytes, void* stream) {
  clear_error();
  if (rows == 0 || per_row_batch == 0 || n_fit == 0 || epochs == 0)
    return set_error(WEDGE_ERANGE, "wedge_mlp_train: empty schedule");
  if (n_fit % per_row_batch != 0 || n_fit > stride)
    return set_error(WEDGE_ERANGE,
                     "wedge_mlp_train: n_fit must be a multiple of per_row_batch and <= stride");
  if (!d_state || !d_x || !d_workspace)
    return set_error(WEDGE_EINVAL, "wedge_mlp_train: null pointer");
  if (!aligned(d_state, 256) || !aligned(d_x, 16) || !aligned(d_workspace, 256))
    return set_error(WEDGE_EINVAL, "wedge_mlp_train: misaligned pointer");
  if (workspace_bytes < wedge_mlp_train_workspace(rows, per_row_batch))
    return set_error(WEDGE_EWORKSPACE, "wedge_mlp_train: workspace too small");
  hipStream_t st = (hipStream_t)stream;
  MlpState* S = (MlpState*)d_state;
  const uint64_t n = (uint64_t)rows * per_row_batch;
  float* partial = (float*)d_workspace;
  uint32_t t = t0;
  for (uint32_t ep = 0; ep < epochs; ++ep) {
    for (uint64_t j0 = 0; j0 < n_fit; j0 += per_row_batch) {
      const bool last = ep + 1 == epochs && j0 + per_row_batch == n_fit;
      const uint32_t nwg = grad_groups(n);
      const float inv_n = 1.0f / (float)n;
      RowView view{d_x, stride, j0, per_row_batch};
      k_mlp_grad<<<nwg, 64 * kGradWaves, 0, st>>>(S, view, n, inv_n, partial);
      WEDGE_LAUNCH_CHECK("k_mlp_grad");
      float c1, c2;
      adam_consts(++t, beta1, beta2, &c1, &c2);
      k_mlp_reduce_adam<<<(NPARAM + 1 + 63) / 64, 64 * kRedSplit, 0, st>>>(
          partial, nwg, S, inv_n, last ? d_loss : nullptr, lr, beta1, beta2, eps, c1, c2);
      WEDGE_LAUNCH_CHECK("k_mlp_reduce_adam");
    }
  }
  return WEDGE_OK;
}

extern "C" int wedge_cv_moments(const wedge_feature_rec* d_x, const float* d_g, uint32_t rows,
                                uint64_t stride, uint64_t n_per_row, const uint64_t* h_counts,
                                int64_t* d_mom, void* stream) {
  clear_error();
  if (rows == 0) return WEDGE_OK;
  if (!d_g || !d_mom) return set_error(WEDGE_EINVAL, "wedge_cv_moments: null pointer");
  uint64_t most = 0;
  for (uint32_t r = 0; r < rows; ++r) {
    const uint64_t c = h_counts ? h_counts[r] : n_per_row;
    if (c > stride) return set_error(WEDGE_ERANGE, "wedge_cv_moments: count of row %u > stride", r);
    most = c > most ? c : most;
  }
  if (most == 0) return WEDGE_OK;
  uint64_t bx = (most + 4095) / 4096;  // about 16 records per thread
  if (bx > 512) bx = 512;
  for (uint32_t r0 = 0; r0 < rows; r0 += kMomRows) {
    const uint32_t nr = rows - r0 < (uint32_t)kMomRows ? rows - r0 : (uint32_t)kMomRows;
    RowCounts rc;
    for (int j = 0; j < kMomRows; ++j)
      rc.n[j] = j < (int)nr ? (h_counts ? h_counts[r0 + j] : n_per_row) : 0;
    dim3 grid((unsigned)bx, nr);
    k_cv_moments<<<grid, 256, 0, (hipStream_t)stream>>>(d_x, d_g, stride, r0, rc,
                                                       (long long*)d_mom);
    WEDGE_LAUNCH_CHECK("k_cv_moments");
  }
  return WEDGE_OK;
}
