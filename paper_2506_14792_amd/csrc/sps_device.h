// Device helpers shared by the gfx950 kernels: complex FP64 arithmetic, a batched
// mixed-radix (2/3/4/6/8) Stockham FFT staged through LDS, and wave64 lane utilities.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define SPS_WAVE 64

typedef double2 cplx;

__device__ __forceinline__ cplx cmk(double r, double i) { return make_double2(r, i); }
__device__ __forceinline__ cplx cadd(cplx a, cplx b) { return cmk(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ cplx csub(cplx a, cplx b) { return cmk(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ cplx cscale(cplx a, double s) { return cmk(a.x * s, a.y * s); }
__device__ __forceinline__ cplx cmul(cplx a, cplx b) {
  return cmk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ cplx cconj(cplx a) { return cmk(a.x, -a.y); }
__device__ __forceinline__ cplx cmul_i(cplx a) { return cmk(-a.y, a.x); }      // i * a
__device__ __forceinline__ cplx cmul_mi(cplx a) { return cmk(a.y, -a.x); }     // -i * a
__device__ __forceinline__ cplx czero() { return cmk(0.0, 0.0); }

// ---------------------------------------------------------------------------- FFT plan
// n = product of radices; every radix is 2, 3, 4, 6 or 8.  Twiddles tw[t] = exp(-2 pi i t / n).
#include "fft_plan.h"

// Radix-R DFT in registers: v_k <- sum_r v_r w^(r k), w = exp(sign 2 pi i / R)
// (sign = -1 forward, +1 inverse, unnormalized).
template <int R>
__device__ __forceinline__ void dft_small(cplx* v, int sign);

template <>
__device__ __forceinline__ void dft_small<2>(cplx* v, int) {
  cplx a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

template <>
__device__ __forceinline__ void dft_small<3>(cplx* v, int sign) {
  const double h = 0.86602540378443864676;  // sqrt(3)/2
  cplx a = v[0], b = v[1], c = v[2];
  cplx s = cadd(b, c);
  cplx d = csub(b, c);
  cplx m = cmk(a.x - 0.5 * s.x, a.y - 0.5 * s.y);
  // w = -1/2 + sign i sqrt(3)/2: y1 = m + sign i h d, y2 = m - sign i h d
  cplx t = cscale(cmul_i(d), h * (double)sign);
  v[0] = cadd(a, s);
  v[1] = cadd(m, t);
  v[2] = csub(m, t);
}

template <>
__device__ __forceinline__ void dft_small<4>(cplx* v, int sign) {
  cplx a = v[0], b = v[1], c = v[2], d = v[3];
  cplx s0 = cadd(a, c), s1 = csub(a, c);
  cplx s2 = cadd(b, d), s3 = csub(b, d);
  // w = sign i: y1 = s1 + sign i s3, y3 = s1 - sign i s3
  cplx t = (sign < 0) ? cmul_mi(s3) : cmul_i(s3);
  v[0] = cadd(s0, s2);
  v[1] = cadd(s1, t);
  v[2] = csub(s0, s2);
  v[3] = csub(s1, t);
}

// Radix 6 = two radix-3 DFTs (even and odd inputs) joined by w6^k:
// y_k = E_k + w6^k O_k, y_(k+3) = E_k - w6^k O_k.
template <>
__device__ __forceinline__ void dft_small<6>(cplx* v, int sign) {
  const double h = 0.86602540378443864676;  // sqrt(3)/2
  cplx e[3] = {v[0], v[2], v[4]};
  cplx o[3] = {v[1], v[3], v[5]};
  dft_small<3>(e, sign);
  dft_small<3>(o, sign);
  const double sh = h * (double)sign;
  // w6 = 1/2 + sign i h, w6^2 = -1/2 + sign i h
  const cplx o1 = cmk(0.5 * o[1].x - sh * o[1].y, 0.5 * o[1].y + sh * o[1].x);
  const cplx o2 = cmk(-0.5 * o[2].x - sh * o[2].y, -0.5 * o[2].y + sh * o[2].x);
  v[0] = cadd(e[0], o[0]);
  v[3] = csub(e[0], o[0]);
  v[1] = cadd(e[1], o1);
  v[4] = csub(e[1], o1);
  v[2] = cadd(e[2], o2);
  v[5] = csub(e[2], o2);
}

// Radix 8 = two radix-4 DFTs joined by w8^k: w8 = (1 + sign i)/sqrt(2), w8^2 = sign i,
// w8^3 = (-1 + sign i)/sqrt(2).
template <>
__device__ __forceinline__ void dft_small<8>(cplx* v, int sign) {
  const double c = 0.70710678118654752440;  // 1/sqrt(2)
  cplx e[4] = {v[0], v[2], v[4], v[6]};
  cplx o[4] = {v[1], v[3], v[5], v[7]};
  dft_small<4>(e, sign);
  dft_small<4>(o, sign);
  const double sg = (double)sign;
  const cplx o1 = cmk(c * (o[1].x - sg * o[1].y), c * (o[1].y + sg * o[1].x));
  const cplx o2 = cmk(-sg * o[2].y, sg * o[2].x);
  const cplx o3 = cmk(c * (-o[3].x - sg * o[3].y), c * (-o[3].y + sg * o[3].x));
  v[0] = cadd(e[0], o[0]);
  v[4] = csub(e[0], o[0]);
  v[1] = cadd(e[1], o1);
  v[5] = csub(e[1], o1);
  v[2] = cadd(e[2], o2);
  v[6] = csub(e[2], o2);
  v[3] = cadd(e[3], o3);
  v[7] = csub(e[3], o3);
}

__device__ __forceinline__ int fdiv(int x, unsigned mag) { return mag ? (int)__umulhi((unsigned)x, mag) : x; }

// One Stockham pass of radix R over nbatch sequences (batch q at q * bstride, padded).
// tw[m] = exp(-2 pi i m / n); the inverse direction uses its conjugate.
template <int R>
__device__ __forceinline__ void stockham_pass(const cplx* __restrict__ src, cplx* __restrict__ dst,
                                              const FftPlan& p, int s, const cplx* __restrict__ tw, int sign,
                                              int nbatch, int bstride, int tid, int nthreads) {
  const int nR = p.n / R, Ns = p.ns[s], tst = p.tst[s];
  const unsigned mnr = p.mag_nr[s], mns = p.mag_ns[s];
  const int total = nbatch * nR;
  for (int it = tid; it < total; it += nthreads) {
    const int q = fdiv(it, mnr);
    const int j = it - q * nR;
    const int jh = fdiv(j, mns);
    const int k = j - jh * Ns;
    const int t = k * tst;   // r t < n for r < R
    const int base = q * bstride;
    cplx v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      cplx x = src[fpad(base + j + r * nR)];
      if (r > 0) {
        cplx w = tw[r * t];
        if (sign > 0) w = cconj(w);
        x = cmul(x, w);
      }
      v[r] = x;
    }
    dft_small<R>(v, sign);
    const int idxD = base + jh * Ns * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) dst[fpad(idxD + r * Ns)] = v[r];
  }
}

// Batched in-LDS FFT of nbatch sequences (stride bstride, indices padded by fpad) held in
// buf0; buf1 is scratch of the same size.  Returns the buffer holding the result.  Contains
// __syncthreads(); must be called by every thread of the block.
__device__ __forceinline__ cplx* lds_fft_inline(cplx* buf0, cplx* buf1, const FftPlan& p, const cplx* tw, int sign,
                                                int nbatch, int bstride, int tid, int nthreads) {
  cplx* src = buf0;
  cplx* dst = buf1;
  for (int s = 0; s < p.nst; ++s) {
    switch (p.radix[s]) {
      case 8: stockham_pass<8>(src, dst, p, s, tw, sign, nbatch, bstride, tid, nthreads); break;
      case 6: stockham_pass<6>(src, dst, p, s, tw, sign, nbatch, bstride, tid, nthreads); break;
      case 4: stockham_pass<4>(src, dst, p, s, tw, sign, nbatch, bstride, tid, nthreads); break;
      case 3: stockham_pass<3>(src, dst, p, s, tw, sign, nbatch, bstride, tid, nthreads); break;
      default: stockham_pass<2>(src, dst, p, s, tw, sign, nbatch, bstride, tid, nthreads); break;
    }
    __syncthreads();
    cplx* t = src;
    src = dst;
    dst = t;
  }
  return src;
}

// The same FFT as an ordinary (inlining left to the compiler) function: kernels with several
// FFT call sites may keep one out-of-line copy; lds_fft_inline forces a copy per call site,
// which lets register allocation see each call's radix mix.
__device__ inline cplx* lds_fft(cplx* buf0, cplx* buf1, const FftPlan& p, const cplx* tw, int sign, int nbatch,
                                int bstride, int tid, int nthreads) {
  return lds_fft_inline(buf0, buf1, p, tw, sign, nbatch, bstride, tid, nthreads);
}

// ---------------------------------------------------------------------------- lanes
__device__ __forceinline__ int lane_id() { return threadIdx.x & (SPS_WAVE - 1); }
// Lane exchanges of a double inside groups of 4 or 8 lanes (DPP, no LDS traffic):
// xor1 / xor2 swap with lane i^1 / i^2 of the quad; mirror8 takes lane 7-i of the group of 8.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const int64_t b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffff), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((int64_t)(uint32_t)lo) | ((int64_t)hi << 32));
}
__device__ __forceinline__ double dpp_xor1(double v) { return dpp_d<0xB1>(v); }     // quad_perm [1,0,3,2]
__device__ __forceinline__ double dpp_xor2(double v) { return dpp_d<0x4E>(v); }     // quad_perm [2,3,0,1]
__device__ __forceinline__ double dpp_mirror8(double v) { return dpp_d<0x141>(v); } // row_half_mirror
// sum over aligned groups of G lanes (G = 1, 2, 4 or 8); every lane of the group gets the sum
template <int G>
__device__ __forceinline__ double group_sum(double v) {
  if (G >= 2) v += dpp_xor1(v);
  if (G >= 4) v += dpp_xor2(v);
  if (G >= 8) v += dpp_mirror8(v);
  return v;
}
template <int G>
__device__ __forceinline__ cplx group_sum(cplx v) {
  return make_double2(group_sum<G>(v.x), group_sum<G>(v.y));
}


// Value of v held by lane `src` (uniform across the wave).
__device__ __forceinline__ double readlane_d(double v, int src) {
  int64_t b = __double_as_longlong(v);
  int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), src);
  int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __longlong_as_double(((int64_t)(uint32_t)lo) | ((int64_t)hi << 32));
}
