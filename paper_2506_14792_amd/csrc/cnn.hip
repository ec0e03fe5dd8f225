// Closure network for a coarse periodic 2D field: three periodic 3x3 convolutions
// 1 -> 32 -> 32 -> 1 channels with GELU between them (exact erf form).  Weights and
// activations are stored in bfloat16 and products accumulated in FP32; the 32 -> 32 layer
// runs on MFMA (bf16 x bf16 -> f32 forward; f32 x f32 -> f32 for its input cotangent and
// weight gradient).  The network is not part of the paper's method: its output is added to
// the explicit term F of the coarse problem, and its parameters receive gradients through
// the discrete adjoint like any parameter of F (equ:efficient_gradient).
//
// Layouts: images [B][H][W] (FP64 in and out); activations NHWC [B][H*W][32]; parameters as
// one FP64 vector in the order w1 (32x1x3x3), b1 (32), w2 (32x32x3x3), b2 (32), w3 (1x32x3x3),
// b3 (1), w[o][c][dy+1][dx+1] multiplying the input at (y + dy, x + dx) (periodic).
#include <hip/hip_runtime.h>
#include <math.h>

#include <vector>

#include "cnn.h"
#include "sps_internal.h"

namespace sps {
namespace {

constexpr int CH = 32;                  // hidden channels
constexpr int NP1 = CH * 9, NP2 = CH * CH * 9, NP3 = CH * 9;
constexpr int OFF_W1 = 0, OFF_B1 = NP1, OFF_W2 = OFF_B1 + CH, OFF_B2 = OFF_W2 + NP2, OFF_W3 = OFF_B2 + CH,
              OFF_B3 = OFF_W3 + NP3, NPARAM = OFF_B3 + 1;
constexpr int NTC = 256;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

struct CnnDev {
  int B, H, W;
  const float* w1;     // [32][9]   bf16-rounded
  const float* b1;     // [32]
  const __bf16* w2r;   // [9][32 co][32 ci] bf16 (forward MFMA operand)
  const float* w2f;    // [9][32 co][32 ci] the same values in FP32
  const float* b2;     // [32]
  const float* w3;     // [32][9]   bf16-rounded
  const float* b3;     // [1]
  __bf16 *a0, *a1, *a2;   // a0: [B][HW]; a1, a2: [B][HW][32]
  float *z1, *z2;         // pre-activations [B][HW][32]
  float *g1, *g2;         // cotangents of z1, z2
};

__device__ __forceinline__ int nb(int p, int t, int H, int W) {
  // pixel index of the neighbour (y + dy, x + dx) of pixel p for tap t = (dy+1)*3 + (dx+1)
  const int y = p / W, x = p - y * W;
  const int dy = t / 3 - 1, dx = t % 3 - 1;
  int yy = y + dy, xx = x + dx;
  yy += (yy < 0) ? H : (yy >= H ? -H : 0);
  xx += (xx < 0) ? W : (xx >= W ? -W : 0);
  return yy * W + xx;
}
__device__ __forceinline__ int nb_t(int p, int t, int H, int W) { return nb(p, 8 - t, H, W); }   // (y - dy, x - dx)
// neighbour (y + dy, x + dx) of the pixel at row y, column x (periodic)
__device__ __forceinline__ int nb_yx(int y, int x, int dy, int dx, int H, int W) {
  int yy = y + dy, xx = x + dx;
  yy += (yy < 0) ? H : (yy >= H ? -H : 0);
  xx += (xx < 0) ? W : (xx >= W ? -W : 0);
  return yy * W + xx;
}
__device__ __forceinline__ float gelu_f(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_df(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

// parameters (FP64) -> stored tables
__global__ void cnn_prepare(const double* th, float* w1, float* b1, __bf16* w2r, float* w2f, float* b2, float* w3,
                            float* b3) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  auto r16 = [](double v) { return (float)(__bf16)(float)v; };
  if (i < NP1) w1[i] = r16(th[OFF_W1 + i]);
  if (i < CH) {
    b1[i] = (float)th[OFF_B1 + i];
    b2[i] = (float)th[OFF_B2 + i];
  }
  if (i < NP2) {   // i = (co * 32 + ci) * 9 + t
    const int t = i % 9, ci = (i / 9) % CH, co = i / (9 * CH);
    const float v = r16(th[OFF_W2 + i]);
    w2r[(t * CH + co) * CH + ci] = (__bf16)v;
    w2f[(t * CH + co) * CH + ci] = v;
  }
  if (i < NP3) w3[i] = r16(th[OFF_W3 + i]);
  if (i == 0) b3[0] = (float)th[OFF_B3];
}

// ---------------------------------------------------------------------------- forward
// layer 1 (1 -> 32) and GELU: one thread per pixel
__global__ void __launch_bounds__(NTC) cnn_l1(CnnDev d, const double* x) {
  const int HW = d.H * d.W;
  const int g = blockIdx.x * NTC + threadIdx.x;
  if (g >= d.B * HW) return;
  const int b = g / HW, p = g - b * HW;
  float v[9];
#pragma unroll
  for (int t = 0; t < 9; ++t) v[t] = (float)(__bf16)(float)x[(long long)b * HW + nb(p, t, d.H, d.W)];
  d.a0[g] = (__bf16)v[4];
  // a pixel's 32 channels are contiguous: 16-byte stores
  float4* zo = reinterpret_cast<float4*>(d.z1 + (long long)g * CH);
  bf16x8* ao = reinterpret_cast<bf16x8*>(d.a1 + (long long)g * CH);
#pragma unroll
  for (int c8 = 0; c8 < CH; c8 += 8) {
    float z[8];
    bf16x8 a;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int c = c8 + j;
      float acc = d.b1[c];
#pragma unroll
      for (int t = 0; t < 9; ++t) acc = fmaf(d.w1[c * 9 + t], v[t], acc);
      z[j] = acc;
      a[j] = (__bf16)gelu_f(acc);
    }
    zo[c8 / 4] = make_float4(z[0], z[1], z[2], z[3]);
    zo[c8 / 4 + 1] = make_float4(z[4], z[5], z[6], z[7]);
    ao[c8 / 8] = a;
  }
}

// layer 2 (32 -> 32) and GELU on MFMA: each wave computes 32 pixels (a row segment) x 32
// output channels; K = 9 taps x 32 input channels in 18 steps of 16.  LDS: w2r.
__global__ void __launch_bounds__(NTC) cnn_l2(CnnDev d) {
  __shared__ __bf16 w[9 * CH * CH];
  for (int e = threadIdx.x; e < 9 * CH * CH; e += NTC) w[e] = d.w2r[e];
  __syncthreads();
  const int HW = d.H * d.W, lane = threadIdx.x & 63;
  const int tile = blockIdx.x * (NTC / 64) + (threadIdx.x >> 6);   // 32-pixel tiles
  const int tiles_per_img = HW / 32;
  if (tile >= d.B * tiles_per_img) return;
  const int b = tile / tiles_per_img, p0 = (tile - b * tiles_per_img) * 32;
  const int row = lane & 31, half = lane >> 5;
  const int p = p0 + row;
  const __bf16* A = d.a1 + (long long)b * HW * CH;
  f32x16 acc = {};
#pragma unroll
  for (int s = 0; s < 18; ++s) {
    const int t = s >> 1, ci0 = (s & 1) * 16 + half * 8;
    const bf16x8 av = *reinterpret_cast<const bf16x8*>(A + (long long)nb(p, t, d.H, d.W) * CH + ci0);
    const bf16x8 bv = *reinterpret_cast<const bf16x8*>(w + (t * CH + row) * CH + ci0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
  }
  // acc[r]: pixel p0 + 8 (r / 4) + 4 half + r % 4, channel `row`
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int pi = p0 + 8 * (r >> 2) + 4 * half + (r & 3);
    const float z = acc[r] + d.b2[row];
    const long long o = ((long long)b * HW + pi) * CH + row;
    d.z2[o] = z;
    d.a2[o] = (__bf16)gelu_f(z);
  }
}

// layer 3 (32 -> 1): one thread per pixel; y (FP64) = scale * output (+= when accumulate)
__global__ void __launch_bounds__(NTC) cnn_l3(CnnDev d, double* y, double scale, int accumulate) {
  const int HW = d.H * d.W;
  const int g = blockIdx.x * NTC + threadIdx.x;
  if (g >= d.B * HW) return;
  const int b = g / HW, p = g - b * HW;
  float s = d.b3[0];
  for (int t = 0; t < 9; ++t) {
    const bf16x8* a8 = reinterpret_cast<const bf16x8*>(d.a2 + ((long long)b * HW + nb(p, t, d.H, d.W)) * CH);
#pragma unroll
    for (int c8 = 0; c8 < CH / 8; ++c8) {
      const bf16x8 a = a8[c8];
#pragma unroll
      for (int j = 0; j < 8; ++j) s = fmaf(d.w3[(c8 * 8 + j) * 9 + t], (float)a[j], s);
    }
  }
  const double v = scale * (double)s;
  y[g] = accumulate ? y[g] + v : v;
}

// ---------------------------------------------------------------------------- backward
// layer 3: g2 = (w3 conv^T ybar) * gelu'(z2); one thread per pixel
__global__ void __launch_bounds__(NTC) cnn_l3_back(CnnDev d, const double* yb) {
  const int HW = d.H * d.W;
  const int g = blockIdx.x * NTC + threadIdx.x;
  if (g >= d.B * HW) return;
  const int b = g / HW, p = g - b * HW;
  float ys[9];
#pragma unroll
  for (int t = 0; t < 9; ++t) ys[t] = (float)yb[(long long)b * HW + nb_t(p, t, d.H, d.W)];
  const float4* zi = reinterpret_cast<const float4*>(d.z2 + (long long)g * CH);
  float4* go = reinterpret_cast<float4*>(d.g2 + (long long)g * CH);
#pragma unroll
  for (int c4 = 0; c4 < CH / 4; ++c4) {
    const float4 z = zi[c4];
    const float zz[4] = {z.x, z.y, z.z, z.w};
    float r[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = 4 * c4 + j;
      float s = 0.f;
#pragma unroll
      for (int t = 0; t < 9; ++t) s = fmaf(d.w3[c * 9 + t], ys[t], s);
      r[j] = s * gelu_df(zz[j]);
    }
    go[c4] = make_float4(r[0], r[1], r[2], r[3]);
  }
}

// layer 2 input cotangent on MFMA f32: g1[p][ci] = gelu'(z1) sum_{t, co} w2[co][ci][t] g2[p - d_t][co];
// each wave 32 pixels x 32 input channels, K = 9 x 32 in 144 steps of 2.
__global__ void __launch_bounds__(NTC) cnn_l2_back_input(CnnDev d) {
  __shared__ float w[9 * CH * CH];
  for (int e = threadIdx.x; e < 9 * CH * CH; e += NTC) w[e] = d.w2f[e];
  __syncthreads();
  const int HW = d.H * d.W, lane = threadIdx.x & 63;
  const int tile = blockIdx.x * (NTC / 64) + (threadIdx.x >> 6);
  const int tiles_per_img = HW / 32;
  if (tile >= d.B * tiles_per_img) return;
  const int b = tile / tiles_per_img, p0 = (tile - b * tiles_per_img) * 32;
  const int row = lane & 31, half = lane >> 5;
  const float* G = d.g2 + (long long)b * HW * CH;
  f32x16 acc = {};
  for (int t = 0; t < 9; ++t) {
    // 16-byte loads: lane (pixel row, half) holds channels 8j + 4 half .. 8j + 4 half + 3, and
    // each of the four MFMAs pairs channel 8j + m (half 0) with 8j + 4 + m (half 1)
    const float4* Gt = reinterpret_cast<const float4*>(G + (long long)nb_t(p0 + row, t, d.H, d.W) * CH);
#pragma unroll
    for (int j = 0; j < CH / 8; ++j) {
      const float4 q = Gt[2 * j + half];
      const float qa[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int co = 8 * j + 4 * half + m;
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(qa[m], w[(t * CH + co) * CH + row], acc, 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int pi = p0 + 8 * (r >> 2) + 4 * half + (r & 3);
    const long long o = ((long long)b * HW + pi) * CH + row;
    d.g1[o] = acc[r] * gelu_df(d.z1[o]);
  }
}

// layer 2 weight gradient on MFMA f32: dw2[co][ci][t] = sum_q g2[q][co] a1[q + d_t][ci].  One
// block per (tap, chunk of W2_CHUNK pixels), its four waves on a quarter of the chunk each,
// summed in a fixed order; the chunk's partial is written to (add == 0) or added to the FP64
// accumulator acc2[chunk][t][co][ci] (each slot has one owner: deterministic).
constexpr int W2_CHUNK = 512;
__global__ void __launch_bounds__(256) cnn_l2_back_weight(CnnDev d, double* acc2, int add) {
  __shared__ float red[3][16][64];
  const int HW = d.H * d.W, lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int t = blockIdx.x % 9, chunk = blockIdx.x / 9;
  const int q0 = chunk * W2_CHUNK + wv * (W2_CHUNK / 4);
  const int total = d.B * HW;
  const int row = lane & 31, half = lane >> 5;
  f32x16 acc = {};
  // this lane's pixel q = q0 + k + half, tracked as (image, row, column) without divisions
  const int dy = t / 3 - 1, dx = t % 3 - 1;
  int qi = min(q0 + half, total - 1);
  int bq = qi / HW, yq = (qi - bq * HW) / d.W, xq = qi - bq * HW - yq * d.W;
#pragma unroll 8
  for (int k = 0; k < W2_CHUNK / 4; k += 2) {
    const int q = q0 + k + half;
    float av = 0.f, bv = 0.f;
    if (q < total) {
      av = d.g2[(long long)q * CH + row];
      bv = (float)d.a1[((long long)bq * HW + nb_yx(yq, xq, dy, dx, d.H, d.W)) * CH + row];
    }
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, acc, 0, 0, 0);
    xq += 2;
    if (xq >= d.W) {
      xq -= d.W;
      if (++yq == d.H) {
        yq = 0;
        ++bq;
      }
    }
  }
  if (wv > 0) {
#pragma unroll
    for (int r = 0; r < 16; ++r) red[wv - 1][r][lane] = acc[r];
  }
  __syncthreads();
  if (wv != 0) return;
  // acc[r]: co = 8 (r / 4) + 4 half + r % 4, ci = row
  double* o = acc2 + ((long long)chunk * 9 + t) * CH * CH;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const float v = ((acc[r] + red[0][r][lane]) + red[1][r][lane]) + red[2][r][lane];
    double* slot = o + (8 * (r >> 2) + 4 * half + (r & 3)) * CH + row;
    *slot = add ? *slot + (double)v : (double)v;
  }
}

// layer 1 input cotangent, one thread per pixel: xb = xscale sum_{t, c} w1[c][t] g1[p - d_t][c]
__global__ void __launch_bounds__(NTC) cnn_l1_back_input(CnnDev d, double* xb, double xscale, int accumulate) {
  const int HW = d.H * d.W;
  const int g = blockIdx.x * NTC + threadIdx.x;
  if (g >= d.B * HW) return;
  const int b = g / HW, p = g - b * HW;
  float s = 0.f;
  for (int t = 0; t < 9; ++t) {
    const float4* G = reinterpret_cast<const float4*>(d.g1 + ((long long)b * HW + nb_t(p, t, d.H, d.W)) * CH);
#pragma unroll
    for (int c4 = 0; c4 < CH / 4; ++c4) {
      const float4 q = G[c4];
      s = fmaf(d.w1[(4 * c4 + 0) * 9 + t], q.x, s);
      s = fmaf(d.w1[(4 * c4 + 1) * 9 + t], q.y, s);
      s = fmaf(d.w1[(4 * c4 + 2) * 9 + t], q.z, s);
      s = fmaf(d.w1[(4 * c4 + 3) * 9 + t], q.w, s);
    }
  }
  const double v = xscale * (double)s;
  xb[g] = accumulate ? xb[g] + v : v;
}

// the small parameter gradients (dw1, db1, dw3, db3, db2) of one chunk of SW_CHUNK pixels: a
// thread per (4 channels, tap) or per 4 channels (biases) sums over the chunk's pixels in order
// with 16-byte loads of the channel vectors; written to (add == 0) or added to the FP64
// accumulator acc1[chunk][SMALL] (one owner per slot).  SMALL layout: dw1 [c][t], db1 [c],
// dw3 [c][t], db3, db2 [c].
constexpr int SMALL = NP1 + CH + NP3 + 1 + CH;
constexpr int SW_CHUNK = 64;
constexpr int SW_THREADS = 128;   // 72 weight threads, 8 bias threads
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void acc_store(double* slot, float v, int add) { *slot = add ? *slot + (double)v : (double)v; }
__global__ void __launch_bounds__(SW_THREADS) cnn_small_weight(CnnDev d, const double* yb, double* acc1, int add) {
  const int HW = d.H * d.W, total = d.B * HW, tid = threadIdx.x;
  const int q0 = blockIdx.x * SW_CHUNK, q1 = min(q0 + SW_CHUNK, total);
  double* o = acc1 + (long long)blockIdx.x * SMALL;
  int b = q0 / HW, y = (q0 - b * HW) / d.W, x = q0 - b * HW - y * d.W;
  if (tid < 72) {
    const int c4 = tid & 7, t = tid >> 3, dy = t / 3 - 1, dx = t % 3 - 1;
    float s1[4] = {0.f, 0.f, 0.f, 0.f}, s3[4] = {0.f, 0.f, 0.f, 0.f};
    for (int q = q0; q < q1; ++q) {
      const long long nq = (long long)b * HW + nb_yx(y, x, dy, dx, d.H, d.W);
      const float4 g = *reinterpret_cast<const float4*>(d.g1 + (long long)q * CH + 4 * c4);
      const bf16x4 a2 = *reinterpret_cast<const bf16x4*>(d.a2 + nq * CH + 4 * c4);
      const float a0 = (float)d.a0[nq], yv = (float)yb[q];
      s1[0] = fmaf(g.x, a0, s1[0]);
      s1[1] = fmaf(g.y, a0, s1[1]);
      s1[2] = fmaf(g.z, a0, s1[2]);
      s1[3] = fmaf(g.w, a0, s1[3]);
#pragma unroll
      for (int j = 0; j < 4; ++j) s3[j] = fmaf(yv, (float)a2[j], s3[j]);
      if (++x == d.W) {
        x = 0;
        if (++y == d.H) {
          y = 0;
          ++b;
        }
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = 4 * c4 + j;
      acc_store(o + c * 9 + t, s1[j], add);
      acc_store(o + NP1 + CH + c * 9 + t, s3[j], add);
    }
  } else if (tid < 80) {
    const int c4 = tid - 72;
    float sb1[4] = {0.f, 0.f, 0.f, 0.f}, sb2[4] = {0.f, 0.f, 0.f, 0.f}, sb3 = 0.f;
    for (int q = q0; q < q1; ++q) {
      const float4 g1 = *reinterpret_cast<const float4*>(d.g1 + (long long)q * CH + 4 * c4);
      const float4 g2 = *reinterpret_cast<const float4*>(d.g2 + (long long)q * CH + 4 * c4);
      sb1[0] += g1.x;
      sb1[1] += g1.y;
      sb1[2] += g1.z;
      sb1[3] += g1.w;
      sb2[0] += g2.x;
      sb2[1] += g2.y;
      sb2[2] += g2.z;
      sb2[3] += g2.w;
      if (c4 == 0) sb3 += (float)yb[q];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      acc_store(o + NP1 + 4 * c4 + j, sb1[j], add);
      acc_store(o + NP1 + CH + NP3 + 1 + 4 * c4 + j, sb2[j], add);
    }
    if (c4 == 0) acc_store(o + NP1 + CH + NP3, sb3, add);
  }
}

// sum the FP64 partials over chunks in a fixed order and add to the parameter gradient
__global__ void cnn_reduce(const double* acc1, int n1, const double* acc2, int n2, double* th_bar) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < NP1 + CH) {   // w1, b1
    double s = 0.0;
    for (int k = 0; k < n1; ++k) s += acc1[(long long)k * SMALL + i];
    th_bar[OFF_W1 + i] += s;
  } else if (i < NP1 + CH + NP2) {   // w2: i - (NP1 + CH) = (co * 32 + ci) * 9 + t
    const int j = i - NP1 - CH, t = j % 9, ci = (j / 9) % CH, co = j / (9 * CH);
    double s = 0.0;
    for (int k = 0; k < n2; ++k) s += acc2[(((long long)k * 9 + t) * CH + co) * CH + ci];
    th_bar[OFF_W2 + j] += s;
  } else if (i < NP1 + CH + NP2 + CH) {   // b2
    const int c = i - (NP1 + CH + NP2);
    double s = 0.0;
    for (int k = 0; k < n1; ++k) s += acc1[(long long)k * SMALL + NP1 + CH + NP3 + 1 + c];
    th_bar[OFF_B2 + c] += s;
  } else if (i < NPARAM) {   // w3, b3
    const int j = i - (NP1 + CH + NP2 + CH);
    double s = 0.0;
    for (int k = 0; k < n1; ++k) s += acc1[(long long)k * SMALL + NP1 + CH + j];
    th_bar[OFF_W3 + j] += s;
  }
}

__global__ void cnn_zero(double* p, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

}  // namespace

// ---------------------------------------------------------------------------- host
struct Cnn::Impl {
  int B, H, W;
  hipStream_t s;
  DevArena arena;
  CnnDev d{};
  float *w1, *b1, *w2f, *b2, *w3, *b3;
  double *acc1, *acc2;
  __bf16* w2r;
  int n1, n2;   // chunks of the small and the layer-2 weight gradients
};

Cnn::Cnn(int batch, int H, int W, hipStream_t s) : p_(new Impl) {
  SPS_REQUIRE(batch >= 1 && H >= 3 && W >= 32 && W % 32 == 0, "closure images need W a multiple of 32");
  Impl& m = *p_;
  m.B = batch;
  m.H = H;
  m.W = W;
  m.s = s;
  const long long HW = (long long)H * W, n = batch * HW;
  m.w1 = m.arena.alloc<float>(NP1);
  m.b1 = m.arena.alloc<float>(CH);
  m.w2r = m.arena.alloc<__bf16>(NP2);
  m.w2f = m.arena.alloc<float>(NP2);
  m.b2 = m.arena.alloc<float>(CH);
  m.w3 = m.arena.alloc<float>(NP3);
  m.b3 = m.arena.alloc<float>(1);
  m.n1 = (int)((n + SW_CHUNK - 1) / SW_CHUNK);
  m.n2 = (int)((n + W2_CHUNK - 1) / W2_CHUNK);
  m.acc1 = m.arena.alloc<double>((size_t)m.n1 * SMALL);
  m.acc2 = m.arena.alloc<double>((size_t)m.n2 * 9 * CH * CH);
  CnnDev& d = m.d;
  d.B = batch;
  d.H = H;
  d.W = W;
  d.w1 = m.w1;
  d.b1 = m.b1;
  d.w2r = m.w2r;
  d.w2f = m.w2f;
  d.b2 = m.b2;
  d.w3 = m.w3;
  d.b3 = m.b3;
  d.a0 = m.arena.alloc<__bf16>(n);
  d.a1 = m.arena.alloc<__bf16>(n * CH);
  d.a2 = m.arena.alloc<__bf16>(n * CH);
  d.z1 = m.arena.alloc<float>(n * CH);
  d.z2 = m.arena.alloc<float>(n * CH);
  d.g1 = m.arena.alloc<float>(n * CH);
  d.g2 = m.arena.alloc<float>(n * CH);
}
Cnn::~Cnn() = default;

int Cnn::nparam() { return NPARAM; }

void Cnn::set_params(const double* theta_dev) {
  Impl& m = *p_;
  hipLaunchKernelGGL(cnn_prepare, dim3((NP2 + 255) / 256), dim3(256), 0, m.s, theta_dev, m.w1, m.b1, m.w2r, m.w2f,
                     m.b2, m.w3, m.b3);
  SPS_CHECK_LAUNCH();
}

void Cnn::forward(const double* x, double* y, double scale, bool accumulate) {
  Impl& m = *p_;
  const long long n = (long long)m.B * m.H * m.W;
  const int g1 = (int)((n + NTC - 1) / NTC), g2 = (int)((n / 32 + 3) / 4);
  hipLaunchKernelGGL(cnn_l1, dim3(g1), dim3(NTC), 0, m.s, m.d, x);
  SPS_CHECK_LAUNCH();
  hipLaunchKernelGGL(cnn_l2, dim3(g2), dim3(NTC), 0, m.s, m.d);
  SPS_CHECK_LAUNCH();
  hipLaunchKernelGGL(cnn_l3, dim3(g1), dim3(NTC), 0, m.s, m.d, y, scale, (int)accumulate);
  SPS_CHECK_LAUNCH();
}

void Cnn::backward(const double* x, const double* yb, double* xb, double xscale, bool accumulate, bool add) {
  Impl& m = *p_;
  const long long n = (long long)m.B * m.H * m.W;
  const int g1 = (int)((n + NTC - 1) / NTC), g2 = (int)((n / 32 + 3) / 4);
  // the forward activations of this input (recomputed: the adjoint sweep revisits states)
  hipLaunchKernelGGL(cnn_l1, dim3(g1), dim3(NTC), 0, m.s, m.d, x);
  SPS_CHECK_LAUNCH();
  hipLaunchKernelGGL(cnn_l2, dim3(g2), dim3(NTC), 0, m.s, m.d);
  SPS_CHECK_LAUNCH();
  hipLaunchKernelGGL(cnn_l3_back, dim3(g1), dim3(NTC), 0, m.s, m.d, yb);
  SPS_CHECK_LAUNCH();
  hipLaunchKernelGGL(cnn_l2_back_input, dim3(g2), dim3(NTC), 0, m.s, m.d);
  SPS_CHECK_LAUNCH();
  hipLaunchKernelGGL(cnn_l2_back_weight, dim3(9 * m.n2), dim3(256), 0, m.s, m.d, m.acc2, (int)add);
  SPS_CHECK_LAUNCH();
  hipLaunchKernelGGL(cnn_small_weight, dim3(m.n1), dim3(SW_THREADS), 0, m.s, m.d, yb, m.acc1, (int)add);
  SPS_CHECK_LAUNCH();
  hipLaunchKernelGGL(cnn_l1_back_input, dim3(g1), dim3(NTC), 0, m.s, m.d, xb, xscale, (int)accumulate);
  SPS_CHECK_LAUNCH();
}

void Cnn::vjp(const double* x, const double* yb, double* xb, double xscale, bool accumulate, double* th_bar) {
  backward(x, yb, xb, xscale, accumulate, false);
  if (th_bar) grad_flush(th_bar);
}

void Cnn::vjp_accumulate(const double* x, const double* yb, double* xb, double xscale, bool accumulate) {
  backward(x, yb, xb, xscale, accumulate, true);
}

void Cnn::grad_reset() {
  Impl& m = *p_;
  const long long n1 = (long long)m.n1 * SMALL, n2 = (long long)m.n2 * 9 * CH * CH;
  hipLaunchKernelGGL(cnn_zero, dim3((unsigned)((n1 + 255) / 256)), dim3(256), 0, m.s, m.acc1, n1);
  SPS_CHECK_LAUNCH();
  hipLaunchKernelGGL(cnn_zero, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, m.s, m.acc2, n2);
  SPS_CHECK_LAUNCH();
}

void Cnn::grad_flush(double* th_bar) {
  Impl& m = *p_;
  hipLaunchKernelGGL(cnn_reduce, dim3((NPARAM + 255) / 256), dim3(256), 0, m.s, m.acc1, m.n1, m.acc2, m.n2, th_bar);
  SPS_CHECK_LAUNCH();
}

}  // namespace sps
