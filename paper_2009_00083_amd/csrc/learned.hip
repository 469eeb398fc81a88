// Learned refinement order (gfx950): a small MLP scores the coarse vertices
// of a level by the density of critical points of the exact (full-resolution)
// classification in their cells; regions are refined in the order of their
// summed scores.  The classification itself never depends on it: every
// vertex of every level is still classified by the classification kernels,
// so the final result is the same whatever the order.
//
// Network: 32 inputs (the 27 samples of the 3x3x3 neighbourhood at the coarse
// stride, relative to the centre and scaled by their largest magnitude, the
// coarse resolution, four zeros) -> 64 GELU -> 64 GELU -> 1 logit.  Weights
// are kept in FP32 and rounded to BF16 when a kernel loads them; the hidden
// products run on the matrix cores (v_mfma_f32_16x16x32_bf16) with FP32
// accumulation; biases, GELU and the output layer are FP32.
//
// Layouts of the 16x16x32 BF16 MFMA (one wave): A (16 x 32) -- lane l holds
// row l % 16, columns 8 (l / 16) .. +7; B (32 x 16) -- lane l holds column
// l % 16, rows 8 (l / 16) .. +7; D (16 x 16) -- lane l holds column l % 16,
// rows 4 (l / 16) .. +3.  The kernels keep samples in the N dimension, so the
// activations of a sample stay in the four lanes of its column: lane (j, g)
// (sample j = l % 16, group g = l / 16) holds hidden units 16 m + 4 g + r
// (m, r = 0..3) after a layer.  The next layer's K positions are numbered so
// that these are exactly its B operand (position 32 kk + 8 g + t is unit
// 16 (2 kk + t / 4) + 4 g + t % 4), and the weights are read in that order.
#include <math.h>

#include <algorithm>

#include "device_util.h"
#include "pcrit_internal.h"

namespace pcrit {
namespace {

using namespace dev;

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;

__device__ __forceinline__ f32x4 mfma(const bf16x8 &a, const bf16x8 &b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// K position p (0..63) of a layer whose input is the previous layer's output
// -> hidden unit of that output
__device__ __forceinline__ int unit_of_pos(int p) {
  const int kk = p >> 5, g = (p >> 3) & 3, t = p & 7;
  return 16 * (2 * kk + (t >> 2)) + 4 * g + (t & 3);
}

// Standard normal CDF Phi(u) = (1 + erf(u / sqrt 2)) / 2, with erf from
// Abramowitz and Stegun 7.1.26 (|error| <= 1.5e-7 on erf): for x >= 0,
// 1 - erf(x) = t (a1 + t (a2 + t (a3 + t (a4 + t a5)))) exp(-x^2),
// t = 1 / (1 + p x).  Branch free: the tail q = 1 - erf(|u| / sqrt 2) gives
// Phi = q / 2 for u < 0 and 1 - q / 2 otherwise, without cancellation in
// the lower tail.  *e receives exp(-u^2 / 2), which the derivative reuses.
__device__ __forceinline__ float normal_cdf(float u, float *e) {
  const float x = fabsf(u) * 0.70710678118654752f;
  const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, x, 1.0f));
  float poly = fmaf(t, 1.061405429f, -1.453152027f);
  poly = fmaf(t, poly, 1.421413741f);
  poly = fmaf(t, poly, -0.284496736f);
  poly = fmaf(t, poly, 0.254829592f);
  *e = __builtin_amdgcn_exp2f(-x * x * 1.4426950408889634f);
  const float hq = 0.5f * t * poly * *e;
  return u < 0.f ? hq : 1.0f - hq;
}
__device__ __forceinline__ float gelu(float x) {
  float e;
  return x * normal_cdf(x, &e);
}
__device__ __forceinline__ float gelu_grad(float x) {
  float e;
  const float cdf = normal_cdf(x, &e);
  return cdf + x * 0.39894228040143268f * e;
}

// Weight fragments of one wave (A operands) and the per-lane biases.
struct MlpWeights {
  bf16x8 w1[4];      // W1^T, M-block m (hidden units 16 m ..), the one K step
  bf16x8 w2[4][2];   // W2^T, M-block m, K step kk (positions of layer-1 units)
  float b1[4][4], b2[4][4], w3[4][4];  // unit 16 m + 4 g + r of this lane
  float b3;
};

__device__ __forceinline__ void load_weights(const float *p, int lane, MlpWeights &W) {
  const int i = lane & 15, g = lane >> 4;
#pragma unroll
  for (int m = 0; m < 4; m++) {
#pragma unroll
    for (int t = 0; t < 8; t++) W.w1[m][t] = (__bf16)p[kMlpOffW1 + (8 * g + t) * kMlpHidden + 16 * m + i];
#pragma unroll
    for (int kk = 0; kk < 2; kk++)
#pragma unroll
      for (int t = 0; t < 8; t++)
        W.w2[m][kk][t] =
            (__bf16)p[kMlpOffW2 + unit_of_pos(32 * kk + 8 * g + t) * kMlpHidden + 16 * m + i];
#pragma unroll
    for (int r = 0; r < 4; r++) {
      const int u = 16 * m + 4 * g + r;
      W.b1[m][r] = p[kMlpOffB1 + u];
      W.b2[m][r] = p[kMlpOffB2 + u];
      W.w3[m][r] = (float)(__bf16)p[kMlpOffW3 + u];
    }
  }
  W.b3 = p[kMlpOffB3];
}

// Forward pass of the 16 samples whose inputs are xb (this lane's B
// fragment: sample lane % 16, inputs 8 g .. +7).  Keeps the pre-activations
// and the activations for the backward pass; returns this lane's part of the
// logit (the sum over its 16 units of layer 2).
struct MlpActs {
  float a1[4][4], a2[4][4];  // pre-activations, unit 16 m + 4 g + r
  bf16x8 h1b[2];             // GELU(a1) in BF16: B operand of layer 2, K step kk
  float h2[4][4];            // GELU(a2)
};

__device__ __forceinline__ float forward16(const MlpWeights &W, const bf16x8 &xb, MlpActs &A) {
#pragma unroll
  for (int m = 0; m < 4; m++) {
    const f32x4 d = mfma(W.w1[m], xb, f32x4{0.f, 0.f, 0.f, 0.f});
#pragma unroll
    for (int r = 0; r < 4; r++) A.a1[m][r] = d[r] + W.b1[m][r];
  }
#pragma unroll
  for (int kk = 0; kk < 2; kk++)
#pragma unroll
    for (int t = 0; t < 8; t++) A.h1b[kk][t] = (__bf16)gelu(A.a1[2 * kk + (t >> 2)][t & 3]);
  float part = 0.f;
#pragma unroll
  for (int m = 0; m < 4; m++) {
    f32x4 d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kk = 0; kk < 2; kk++) d = mfma(W.w2[m][kk], A.h1b[kk], d);
#pragma unroll
    for (int r = 0; r < 4; r++) {
      A.a2[m][r] = d[r] + W.b2[m][r];
      A.h2[m][r] = gelu(A.a2[m][r]);
      part += A.h2[m][r] * W.w3[m][r];
    }
  }
  return part;
}

// sum over the four lanes of a sample's column (lanes j, j+16, j+32, j+48)
__device__ __forceinline__ float column_sum(float v) {
  v += __shfl_xor(v, 16);
  v += __shfl_xor(v, 32);
  return v;
}

__device__ __forceinline__ bf16x8 load_x(const uint16_t *X, int64_t sample, int g, bool ok) {
  bf16x8 x;
  if (ok) {
    const uint4 q = *reinterpret_cast<const uint4 *>(X + sample * kMlpIn + 8 * g);
    x = __builtin_bit_cast(bf16x8, q);
  } else {
    x = __builtin_bit_cast(bf16x8, uint4{0u, 0u, 0u, 0u});
  }
  return x;
}

// Logits of n samples (X: n x 32 BF16, row-major).  One wave: 16 samples at
// a time.
__global__ __launch_bounds__(256) void mlp_forward_kernel(const float *params,
                                                          const uint16_t *X, int64_t n,
                                                          float *logits) {
  const int lane = threadIdx.x & 63, g = lane >> 4, j = lane & 15;
  MlpWeights W;
  load_weights(params, lane, W);
  const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t grp = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
       grp * 16 < n; grp += nw) {
    const int64_t s = grp * 16 + j;
    MlpActs A;
    const float z = column_sum(forward16(W, load_x(X, s, g, s < n), A)) + W.b3;
    if (g == 0 && s < n) logits[s] = z;
  }
}

// Gradient of the mean binary cross-entropy (with logits) of n samples
// against the targets y / 255 (bytes), added to grad (kMlpParams floats, FP32,
// zeroed by the caller); the loss sum is added to loss_acc[0].  One wave
// handles 32 samples at a time (two groups of 16): the K dimension of the
// weight-gradient products is the sample.  LDS holds the wave's activations
// transposed (unit x sample) for those products.
__global__ __launch_bounds__(256) void mlp_backward_kernel(const float *params,
                                                           const uint16_t *X,
                                                           const uint8_t *y, int64_t n,
                                                           float *grad, float *loss_acc) {
  constexpr int NW = 4;
  __shared__ __attribute__((aligned(16))) __bf16 s_xT[NW][32][32];   // input x sample
  __shared__ __attribute__((aligned(16))) __bf16 s_h1T[NW][64][32];  // layer-1 unit x sample
  __shared__ __attribute__((aligned(16))) __bf16 s_d2T[NW][64][32];  // dA2: layer-2 unit x sample
  __shared__ __attribute__((aligned(16))) __bf16 s_d1T[NW][64][32];  // dA1
  __shared__ __attribute__((aligned(16))) __bf16 s_h2T[NW][64][32];  // GELU(a2)
  __shared__ __attribute__((aligned(16))) __bf16 s_dz[NW][32];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, g = lane >> 4, j = lane & 15;
  MlpWeights W;
  load_weights(params, lane, W);
  // W2 fragments for dH1 = dA2 W2^T: A[i][p] = W2[16 m + i][unit_of_pos(p)]
  bf16x8 w2b[4][2];
#pragma unroll
  for (int m = 0; m < 4; m++)
#pragma unroll
    for (int kk = 0; kk < 2; kk++)
#pragma unroll
      for (int t = 0; t < 8; t++)
        w2b[m][kk][t] = (__bf16)params[kMlpOffW2 + (16 * m + j) * kMlpHidden +
                                       unit_of_pos(32 * kk + 8 * g + t)];
  const float inv_n = 1.0f / (float)n;
  // gradient accumulators (D fragments)
  f32x4 gW2[4][4], gW1[2][4], gB1[4], gB2[4], gW3[4];
  const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int a = 0; a < 4; a++) {
    gB1[a] = zero;
    gB2[a] = zero;
    gW3[a] = zero;
#pragma unroll
    for (int b = 0; b < 4; b++) gW2[a][b] = zero;
  }
#pragma unroll
  for (int a = 0; a < 2; a++)
#pragma unroll
    for (int b = 0; b < 4; b++) gW1[a][b] = zero;
  float gb3 = 0.f, loss = 0.f;
  bf16x8 ones;
#pragma unroll
  for (int t = 0; t < 8; t++) ones[t] = (__bf16)1.0f;

  const int64_t nw = (int64_t)gridDim.x * NW;
  for (int64_t pair = (int64_t)blockIdx.x * NW + w; pair * 32 < n; pair += nw) {
#pragma unroll
    for (int half = 0; half < 2; half++) {
      const int64_t s = pair * 32 + 16 * half + j;
      const bool ok = s < n;
      const bf16x8 xb = load_x(X, s, g, ok);
      MlpActs A;
      const float z = column_sum(forward16(W, xb, A)) + W.b3;
      // d loss / d z for this sample (0 for padding samples)
      const float yv = ok ? (float)y[s] * (1.0f / 255.0f) : 0.f;
      const float sig = 1.0f / (1.0f + __expf(-z));
      const float dz = ok ? (sig - yv) * inv_n : 0.f;
      if (g == 0 && ok) {
        // softplus(z) - y z, computed stably
        loss += fmaxf(z, 0.f) - z * yv + log1pf(__expf(-fabsf(z)));
        gb3 += dz;
      }
      const int col = 16 * half + j;  // sample column in this wave's 32
      // dA2 = dz w3 GELU'(a2)
      float d2[4][4];
#pragma unroll
      for (int m = 0; m < 4; m++)
#pragma unroll
        for (int r = 0; r < 4; r++) d2[m][r] = dz * W.w3[m][r] * gelu_grad(A.a2[m][r]);
      // dH1 = dA2 W2^T (layer-1 units in M, samples in N)
      bf16x8 d2b[2];
#pragma unroll
      for (int kk = 0; kk < 2; kk++)
#pragma unroll
        for (int t = 0; t < 8; t++) d2b[kk][t] = (__bf16)d2[2 * kk + (t >> 2)][t & 3];
      float d1[4][4];
#pragma unroll
      for (int m = 0; m < 4; m++) {
        f32x4 d = zero;
#pragma unroll
        for (int kk = 0; kk < 2; kk++) d = mfma(w2b[m][kk], d2b[kk], d);
#pragma unroll
        for (int r = 0; r < 4; r++) d1[m][r] = d[r] * gelu_grad(A.a1[m][r]);
      }
      // transposed copies for the weight-gradient products
#pragma unroll
      for (int t = 0; t < 8; t++) s_xT[w][8 * g + t][col] = xb[t];
#pragma unroll
      for (int m = 0; m < 4; m++)
#pragma unroll
        for (int r = 0; r < 4; r++) {
          const int u = 16 * m + 4 * g + r;
          s_h1T[w][u][col] = (__bf16)gelu(A.a1[m][r]);
          s_h2T[w][u][col] = (__bf16)A.h2[m][r];
          s_d2T[w][u][col] = (__bf16)d2[m][r];
          s_d1T[w][u][col] = (__bf16)d1[m][r];
        }
      if (g == 0) s_dz[w][col] = (__bf16)dz;
    }
    wave_lds_sync();
    // A fragment of a transposed matrix: row 16 m + i, samples 8 g .. +7
    auto frag = [&](const __bf16 (*T)[32], int row) {
      return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(&T[row][8 * g]));
    };
    // dW2[k][u] = sum_s h1[s][k] dA2[s][u]: M = k (layer-1 unit), N = u
#pragma unroll
    for (int m = 0; m < 4; m++) {
      const bf16x8 a = frag(s_h1T[w], 16 * m + j);
#pragma unroll
      for (int nb = 0; nb < 4; nb++) gW2[m][nb] = mfma(a, frag(s_d2T[w], 16 * nb + j), gW2[m][nb]);
    }
    // dW1[i][k] = sum_s x[s][i] dA1[s][k]: M = input, N = layer-1 unit
#pragma unroll
    for (int m = 0; m < 2; m++) {
      const bf16x8 a = frag(s_xT[w], 16 * m + j);
#pragma unroll
      for (int nb = 0; nb < 4; nb++) gW1[m][nb] = mfma(a, frag(s_d1T[w], 16 * nb + j), gW1[m][nb]);
    }
    // bias gradients (an all-ones A operand sums over samples) and
    // dw3[u] = sum_s dz[s] h2[s][u] (A rows all dz)
    bf16x8 dza;
#pragma unroll
    for (int t = 0; t < 8; t++) dza[t] = s_dz[w][8 * g + t];
#pragma unroll
    for (int nb = 0; nb < 4; nb++) {
      gB1[nb] = mfma(ones, frag(s_d1T[w], 16 * nb + j), gB1[nb]);
      gB2[nb] = mfma(ones, frag(s_d2T[w], 16 * nb + j), gB2[nb]);
      gW3[nb] = mfma(dza, frag(s_h2T[w], 16 * nb + j), gW3[nb]);
    }
    wave_lds_sync();  // the next pair overwrites the staging
  }
  // D fragment element (row 4 g + r, column j) of block (m, nb)
#pragma unroll
  for (int m = 0; m < 4; m++)
#pragma unroll
    for (int nb = 0; nb < 4; nb++)
#pragma unroll
      for (int r = 0; r < 4; r++)
        atomicAdd(&grad[kMlpOffW2 + (16 * m + 4 * g + r) * kMlpHidden + 16 * nb + j], gW2[m][nb][r]);
#pragma unroll
  for (int m = 0; m < 2; m++)
#pragma unroll
    for (int nb = 0; nb < 4; nb++)
#pragma unroll
      for (int r = 0; r < 4; r++)
        atomicAdd(&grad[kMlpOffW1 + (16 * m + 4 * g + r) * kMlpHidden + 16 * nb + j], gW1[m][nb][r]);
  // every row of the ones / dz products holds the same sums: row 0 only
  if (g == 0) {
#pragma unroll
    for (int nb = 0; nb < 4; nb++) {
      atomicAdd(&grad[kMlpOffB1 + 16 * nb + j], gB1[nb][0]);
      atomicAdd(&grad[kMlpOffB2 + 16 * nb + j], gB2[nb][0]);
      atomicAdd(&grad[kMlpOffW3 + 16 * nb + j], gW3[nb][0]);
    }
  }
  gb3 = column_sum(gb3);
  loss = column_sum(loss);
#pragma unroll
  for (int d = 8; d >= 1; d >>= 1) {
    gb3 += __shfl_xor(gb3, d);
    loss += __shfl_xor(loss, d);
  }
  if (lane == 0) {
    atomicAdd(&grad[kMlpOffB3], gb3);
    atomicAdd(loss_acc, loss);
  }
}

// Adam step on the FP32 parameters (moments m, v; step number t >= 1).
__global__ void mlp_adam_kernel(float *p, const float *grad, float *m, float *v, int n,
                                float lr, float b1, float b2, float eps, int t) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = grad[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / (1.f - powf(b1, (float)t));
  const float vh = vi / (1.f - powf(b2, (float)t));
  p[i] -= lr * mh / (sqrtf(vh) + eps);
}

__global__ void fill_kernel(float *p, int n, float v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void zero_i64_kernel(int64_t *p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// Inputs of the coarse vertices of level `level` (stride s): vertex q
// (level-local index) gets the 27 samples f(v + s d), d in {-1,0,1}^3
// (clamped to the grid), as (f(v + s d) - f(v)) / max |f(v + s d) - f(v)|
// (0 when all are equal), then `res` (the coarse resolution feature), then
// zeros; BF16.  Order of the 27: d_z slowest, d_x fastest.
__global__ void mlp_features_kernel(const float *f, int64_t nx, int64_t ny, int64_t nz,
                                    int s, int mx, int my, int mz, float res, uint16_t *X) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nq = (int64_t)mx * my * mz;
  if (q >= nq) return;
  const int x = (int)(q % mx), y = (int)((q / mx) % my), z = (int)(q / ((int64_t)mx * my));
  const float c = f[((int64_t)z * s * ny + (int64_t)y * s) * nx + (int64_t)x * s];
  float v[27];
  float mag = 0.f;
#pragma unroll
  for (int k = 0; k < 27; k++) {
    const int dx = k % 3 - 1, dy = (k / 3) % 3 - 1, dz = k / 9 - 1;
    const int xx = min(max(x + dx, 0), mx - 1), yy = min(max(y + dy, 0), my - 1),
              zz = min(max(z + dz, 0), mz - 1);
    v[k] = f[((int64_t)zz * s * ny + (int64_t)yy * s) * nx + (int64_t)xx * s] - c;
    mag = fmaxf(mag, fabsf(v[k]));
  }
  const float inv = mag > 0.f ? 1.f / mag : 0.f;
  __bf16 out[32];
#pragma unroll
  for (int k = 0; k < 27; k++) out[k] = (__bf16)(v[k] * inv);
  out[27] = (__bf16)res;
#pragma unroll
  for (int k = 28; k < 32; k++) out[k] = (__bf16)0.f;
  uint4 *dst = reinterpret_cast<uint4 *>(X + q * kMlpIn);
#pragma unroll
  for (int k = 0; k < 4; k++) dst[k] = __builtin_bit_cast(uint4, *reinterpret_cast<bf16x8 *>(&out[8 * k]));
}

// Target of coarse vertex q of level `level` (stride s): the fraction of
// critical vertices (full-resolution codes of level 0) among the vertices of
// the full-resolution grid within [v - s/2, v + s/2) on every axis (its
// cell, clipped to the grid), as ceil(255 * count / volume): 0 only for no
// critical vertex, 255 only when all are.
__global__ void mlp_labels_kernel(const uint8_t *codes, int64_t nx, int64_t ny, int64_t nz,
                                  int s, int mx, int my, int mz, uint8_t *label) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nq = (int64_t)mx * my * mz;
  if (q >= nq) return;
  const int x = (int)(q % mx), y = (int)((q / mx) % my), z = (int)(q / ((int64_t)mx * my));
  const int h = s / 2;
  const int x0 = max(x * s - h, 0), x1 = min(x * s + s - h, (int)nx);
  const int y0 = max(y * s - h, 0), y1 = min(y * s + s - h, (int)ny);
  const int z0 = max(z * s - h, 0), z1 = min(z * s + s - h, (int)nz);
  unsigned cnt = 0;
  for (int zz = z0; zz < z1; zz++)
    for (int yy = y0; yy < y1; yy++) {
      const uint8_t *row = codes + ((int64_t)zz * ny + yy) * nx;
      for (int xx = x0; xx < x1; xx++) cnt += (row[xx] & 0xBFu) != 0x09u;
    }
  const uint64_t vol = (uint64_t)(x1 - x0) * (y1 - y0) * (z1 - z0);
  label[q] = (uint8_t)((255u * (uint64_t)cnt + vol - 1) / vol);
}

// Region scores straight from the field: the inputs of each coarse vertex
// (as mlp_features_kernel, the four lanes of a sample computing eight of
// them each), the network (forward16), the sigmoid, summed per region.
// Every wave takes a contiguous run of 16-sample groups, so a lane's
// samples stay in one region for many groups; each lane flushes its running
// sum with one atomic add when its region changes (scores spaced
// kCounterStride floats apart, zeroed by the caller).
__global__ __launch_bounds__(256) void mlp_region_scores_kernel(
    const float *params, const float *f, int64_t nx, int64_t ny, int s, int mx, int my, int mz,
    float res, int E, int nry, float *scores) {
  const int lane = threadIdx.x & 63, g = lane >> 4, j = lane & 15;
  MlpWeights W;
  load_weights(params, lane, W);
  const int64_t n = (int64_t)mx * my * mz, groups = (n + 15) / 16;
  const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
  const int64_t wv = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int64_t g0 = groups * wv / nw, g1 = groups * (wv + 1) / nw;
  float acc = 0.f;
  int cur = -1;
  // this lane's samples of group grp: centre and its eight neighbour
  // differences, loaded one group ahead of the network
  struct Sample {
    float c, v[8];
    int r;
    bool ok;
  };
  // level vertex counts fit in 32 bits (the grid has at most 2^32
  // vertices and the level at least stride 2), so the index arithmetic is
  // 32-bit; addresses step by the level's strides
  const int64_t sy = (int64_t)s * nx, sz = (int64_t)s * nx * ny;
  auto fetch = [&](int64_t grp, Sample &S) {
    const int64_t q = grp * 16 + j;
    S.ok = q < n;
    const uint32_t qq = (uint32_t)(S.ok ? q : n - 1);
    const uint32_t row = qq / (uint32_t)mx;
    const int x = (int)(qq - row * (uint32_t)mx);
    const int z = (int)(row / (uint32_t)my), y = (int)(row - (uint32_t)z * (uint32_t)my);
    S.r = ((z * s) / E) * nry + (y * s) / E;
    const float *cp = f + z * sz + y * sy + (int64_t)x * s;
    S.c = *cp;
#pragma unroll
    for (int t = 0; t < 8; t++) {
      const int k = 8 * g + t;
      S.v[t] = S.c;
      if (k < 27) {
        const int dx = k % 3 - 1, dy = (k / 3) % 3 - 1, dz = k / 9 - 1;
        const int ex = min(max(x + dx, 0), mx - 1) - x, ey = min(max(y + dy, 0), my - 1) - y,
                  ez = min(max(z + dz, 0), mz - 1) - z;
        S.v[t] = cp[ez * sz + ey * sy + ex * s];
      }
    }
  };
  Sample S;
  if (g0 < g1) fetch(g0, S);
  for (int64_t grp = g0; grp < g1; grp++) {
    const Sample C = S;
    if (grp + 1 < g1) fetch(grp + 1, S);
    float v[8];
    float mag = 0.f;
#pragma unroll
    for (int t = 0; t < 8; t++) {
      v[t] = C.v[t] - C.c;
      mag = fmaxf(mag, fabsf(v[t]));
    }
    mag = fmaxf(mag, __shfl_xor(mag, 16));
    mag = fmaxf(mag, __shfl_xor(mag, 32));
    const float inv = mag > 0.f ? 1.f / mag : 0.f;
    bf16x8 xb;
#pragma unroll
    for (int t = 0; t < 8; t++) {
      const int k = 8 * g + t;
      xb[t] = (__bf16)(k < 27 ? v[t] * inv : (k == 27 ? res : 0.f));
    }
    MlpActs A;
    const float zl = column_sum(forward16(W, xb, A)) + W.b3;
    if (g == 0 && C.ok) {
      if (C.r != cur) {
        if (cur >= 0) atomicAdd(&scores[kCounterStride * cur], acc);
        cur = C.r;
        acc = 0.f;
      }
      acc += 1.f / (1.f + __expf(-zl));
    }
  }
  if (g == 0 && cur >= 0) atomicAdd(&scores[kCounterStride * cur], acc);
}

// Rank of each region: number of regions with a higher score, or an equal
// score and a smaller id (one block, nregions <= kMaxRegions).
__global__ __launch_bounds__(1024) void region_rank_kernel(const float *scores, int stride,
                                                           int nregions, int *rank) {
  __shared__ float s_sc[kMaxRegions];
  for (int i = threadIdx.x; i < nregions; i += blockDim.x) s_sc[i] = scores[(int64_t)stride * i];
  __syncthreads();
  for (int r = threadIdx.x; r < nregions; r += blockDim.x) {
    const float v = s_sc[r];
    int k = 0;
    for (int q = 0; q < nregions; q++) k += (s_sc[q] > v) || (s_sc[q] == v && q < r);
    rank[r] = k;
  }
}

// Tile rows / z-chunks of region (ry, rz) at a quad level: [a, b) ranges.
struct RegionTiles {
  int ty0, ty1, zc0, zc1;
};
__device__ __forceinline__ RegionTiles region_tiles(const LevelDesc &l, int R, int s, int E,
                                                    int ry, int rz) {
  const int ey = E / (s * R), ez = E / (s * l.zchunk);  // tile rows / chunks per region
  const int nzc = (l.mz + l.zchunk - 1) / l.zchunk;
  return {min(ry * ey, l.nty), min((ry + 1) * ey, l.nty), min(rz * ez, nzc),
          min((rz + 1) * ez, nzc)};
}

// Tile lists of a level in region order, first step (one block): region
// tile counts, where part x of the region at each rank starts in list x
// (regions in rank order; region_part_start), the start of every list
// (xcd_off, kXcds + 1 entries) and zero queue counters.
__global__ __launch_bounds__(1024) void region_parts_kernel(LevelDesc l, int R, int s, int E,
                                                            int nry, int nregions,
                                                            const int *rank,
                                                            unsigned *region_left,
                                                            int *scratch) {
  __shared__ int s_cnt[kMaxRegions];                // tile count of the region at each rank
  __shared__ int s_pre[kXcds][kMaxRegions + 1];     // part-x tiles of the ranks before
  for (int r = threadIdx.x; r < nregions; r += blockDim.x) {
    const RegionTiles t = region_tiles(l, R, s, E, r % nry, r / nry);
    const int c = l.ntx * max(t.ty1 - t.ty0, 0) * max(t.zc1 - t.zc0, 0);
    region_left[kCounterStride * r] = (unsigned)c;
    s_cnt[rank[r]] = c;
  }
  __syncthreads();
  if (threadIdx.x < kXcds) {
    const int x = threadIdx.x;
    int acc = 0;
    for (int k = 0; k < nregions; k++) {
      s_pre[x][k] = acc;
      const int64_t c = s_cnt[k];
      acc += (int)(c * (x + 1) / kXcds - c * x / kXcds);
    }
    s_pre[x][nregions] = acc;
  }
  __syncthreads();
  __shared__ int s_off[kXcds];
  if (threadIdx.x == 0) {
    int *xcd_off = region_xcd_off(scratch, nregions);
    int acc = 0;
    for (int x = 0; x < kXcds; x++) {
      s_off[x] = acc;
      xcd_off[x] = acc;
      acc += s_pre[x][nregions];
    }
    xcd_off[kXcds] = acc;
    int *queue = region_queue(scratch, nregions);
    for (int x = 0; x < kXcds; x++) queue[kCounterStride * x] = 0;
  }
  __syncthreads();
  int *start = region_part_start(scratch, nregions);
  for (int i = threadIdx.x; i < kXcds * nregions; i += blockDim.x) {
    const int k = i / kXcds, x = i % kXcds;
    start[i] = s_off[x] + s_pre[x][k];
  }
}

// Second step: every tile placed; tile i of its region (x fastest, then
// rows, then chunks) falls in part x, the one of the kXcds contiguous parts
// that holds i.
__global__ void region_place_kernel(LevelDesc l, int R, int s, int E, int nry, int nregions,
                                    const int *rank, const int *scratch, int *tile_list) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= l.ntiles) return;
  const TilePos p = tile_pos(l, t);
  const int ry = (p.ty * R * s) / E, rz = (p.zc * l.zchunk * s) / E;
  const RegionTiles rt = region_tiles(l, R, s, E, ry, rz);
  const int local = p.tx + l.ntx * ((p.ty - rt.ty0) + (rt.ty1 - rt.ty0) * (p.zc - rt.zc0));
  const int64_t c = (int64_t)l.ntx * (rt.ty1 - rt.ty0) * (rt.zc1 - rt.zc0);
  int x = kXcds - 1;
  while (x > 0 && c * x / kXcds > local) x--;
  const int *start = region_part_start(const_cast<int *>(scratch), nregions);
  tile_list[start[kXcds * rank[rz * nry + ry] + x] + local - (int)(c * x / kXcds)] = t;
}

__global__ void stamp_kernel(uint64_t *out) {
  if (threadIdx.x == 0) *out = __builtin_amdgcn_s_memrealtime();
}

// Waits `ticks` of the 100 MHz clock (at most 2^20 short sleeps), then
// stores the clock in *out (if out is not null).
__global__ void wait_stamp_kernel(uint64_t *out, uint64_t ticks) {
  if (threadIdx.x == 0) {
    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
    for (int i = 0; i < (1 << 20); i++) {
      if (__builtin_amdgcn_s_memrealtime() - t0 >= ticks) break;
      __builtin_amdgcn_s_sleep(8);
    }
    if (out) *out = __builtin_amdgcn_s_memrealtime();
  }
}

}  // namespace

hipError_t launch_region_rank(const float *scores, int stride, int nregions, int *rank,
                              hipStream_t st) {
  if (nregions < 1 || nregions > kMaxRegions) return hipErrorInvalidValue;
  hipLaunchKernelGGL(region_rank_kernel, dim3(1), dim3(1024), 0, st, scores, stride, nregions,
                     rank);
  return hipGetLastError();
}

hipError_t launch_region_tiles(const LevelDesc &l, int R, int s, int E, int nry, int nregions,
                               const int *rank, int *tile_list, unsigned *region_left,
                               int *scratch, hipStream_t st) {
  if (nregions < 1 || nregions > kMaxRegions) return hipErrorInvalidValue;
  hipLaunchKernelGGL(region_parts_kernel, dim3(1), dim3(1024), 0, st, l, R, s, E, nry, nregions,
                     rank, region_left, scratch);
  hipLaunchKernelGGL(region_place_kernel, dim3((l.ntiles + 255) / 256), dim3(256), 0, st, l, R, s,
                     E, nry, nregions, rank, scratch, tile_list);
  return hipGetLastError();
}

hipError_t launch_wait_stamp(uint64_t *out, double us, hipStream_t st) {
  hipLaunchKernelGGL(wait_stamp_kernel, dim3(1), dim3(64), 0, st, out, (uint64_t)(us * 100.0));
  return hipGetLastError();
}

hipError_t launch_zero_i64(int64_t *p, int n, hipStream_t st) {
  hipLaunchKernelGGL(zero_i64_kernel, dim3((n + 255) / 256), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

hipError_t launch_stamp(uint64_t *out, hipStream_t st) {
  hipLaunchKernelGGL(stamp_kernel, dim3(1), dim3(64), 0, st, out);
  return hipGetLastError();
}

hipError_t launch_mlp_forward(const float *params, const uint16_t *X, int64_t n, float *logits,
                              hipStream_t st) {
  const int64_t groups = (n + 15) / 16;
  // each wave loads the weights once and then takes groups of 16 samples
  const int blocks = (int)std::min<int64_t>((groups + 3) / 4, 1024);
  hipLaunchKernelGGL(mlp_forward_kernel, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, st, params, X,
                     n, logits);
  return hipGetLastError();
}

hipError_t launch_mlp_backward(const float *params, const uint16_t *X, const uint8_t *y,
                               int64_t n, float *grad, float *loss, hipStream_t st) {
  const int64_t pairs = (n + 31) / 32;
  const int blocks = (int)std::min<int64_t>((pairs + 3) / 4, 1024);
  hipLaunchKernelGGL(fill_kernel, dim3((kMlpParams + 255) / 256), dim3(256), 0, st, grad,
                     kMlpParams, 0.f);
  hipLaunchKernelGGL(fill_kernel, dim3(1), dim3(64), 0, st, loss, 1, 0.f);
  hipLaunchKernelGGL(mlp_backward_kernel, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, st,
                     params, X, y, n, grad, loss);
  return hipGetLastError();
}

hipError_t launch_mlp_adam(float *params, const float *grad, float *m, float *v, float lr,
                           int t, hipStream_t st) {
  hipLaunchKernelGGL(mlp_adam_kernel, dim3((kMlpParams + 255) / 256), dim3(256), 0, st, params,
                     grad, m, v, kMlpParams, lr, 0.9f, 0.999f, 1e-8f, t);
  return hipGetLastError();
}

hipError_t launch_mlp_features(const float *f, int64_t nx, int64_t ny, int64_t nz, int s,
                               int mx, int my, int mz, float res, uint16_t *X, hipStream_t st) {
  const int64_t nq = (int64_t)mx * my * mz;
  hipLaunchKernelGGL(mlp_features_kernel, dim3((unsigned)((nq + 255) / 256)), dim3(256), 0, st, f,
                     nx, ny, nz, s, mx, my, mz, res, X);
  return hipGetLastError();
}

hipError_t launch_mlp_labels(const uint8_t *codes, int64_t nx, int64_t ny, int64_t nz, int s,
                             int mx, int my, int mz, uint8_t *label, hipStream_t st) {
  const int64_t nq = (int64_t)mx * my * mz;
  hipLaunchKernelGGL(mlp_labels_kernel, dim3((unsigned)((nq + 255) / 256)), dim3(256), 0, st,
                     codes, nx, ny, nz, s, mx, my, mz, label);
  return hipGetLastError();
}

hipError_t launch_mlp_region_scores(const float *params, const float *f, int64_t nx, int64_t ny,
                                    int s, int mx, int my, int mz, float res, int E, int nry,
                                    int nregions, float *scores, hipStream_t st) {
  const int n = kCounterStride * nregions;
  hipLaunchKernelGGL(fill_kernel, dim3((n + 255) / 256), dim3(256), 0, st, scores, n, 0.f);
  // two waves per SIMD (the weights live in registers); each wave loads
  // them once and then takes a run of sample groups
  hipLaunchKernelGGL(mlp_region_scores_kernel, dim3(512), dim3(256), 0, st, params, f, nx, ny, s,
                     mx, my, mz, res, E, nry, scores);
  return hipGetLastError();
}


}  // namespace pcrit
