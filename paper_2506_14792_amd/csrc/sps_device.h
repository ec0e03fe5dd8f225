// Device helpers shared by the gfx950 kernels: complex FP64 arithmetic, a batched
// mixed-radix (2/3/4) Stockham FFT staged through LDS, and wave64 lane utilities.
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
// n = product of radices; every radix is 2, 3 or 4.  Twiddles tw[t] = exp(-2 pi i t / n).
struct FftPlan {
  int n;
  int nst;
  int radix[12];
};

// Radix-R DFT in registers, sign = -1 forward, +1 inverse (unnormalized).
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
  // forward: y1 = m - i h d, y2 = m + i h d ; inverse swaps the sign of i
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
  // forward (w = -i): y1 = s1 - i s3, y3 = s1 + i s3
  cplx t = (sign < 0) ? cmul_mi(s3) : cmul_i(s3);
  v[0] = cadd(s0, s2);
  v[1] = cadd(s1, t);
  v[2] = csub(s0, s2);
  v[3] = csub(s1, t);
}

template <int R>
__device__ __forceinline__ void stockham_pass(const cplx* __restrict__ src, cplx* __restrict__ dst,
                                              int n, int Ns, const cplx* __restrict__ tw, int sign,
                                              int nbatch, int bstride, int tid, int nthreads) {
  const int nR = n / R;
  const int tstride = n / (Ns * R);
  const int total = nbatch * nR;
  for (int it = tid; it < total; it += nthreads) {
    const int q = it / nR;
    const int j = it - q * nR;
    const cplx* a = src + q * bstride;
    cplx* b = dst + q * bstride;
    const int k = j % Ns;
    const int t = k * tstride;
    cplx v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      cplx x = a[j + r * nR];
      if (r > 0 && t != 0) {
        cplx w = tw[(r * t) % n];
        if (sign > 0) w = cconj(w);
        x = cmul(x, w);
      }
      v[r] = x;
    }
    dft_small<R>(v, sign);
    const int idxD = (j / Ns) * Ns * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) b[idxD + r * Ns] = v[r];
  }
}

// Batched in-LDS FFT of nbatch sequences (stride bstride) held in buf0; buf1 is scratch
// of the same size.  Returns the buffer holding the result.  Contains __syncthreads();
// must be called by every thread of the block.
__device__ inline cplx* lds_fft(cplx* buf0, cplx* buf1, const FftPlan& p, const cplx* tw, int sign,
                                int nbatch, int bstride, int tid, int nthreads) {
  cplx* src = buf0;
  cplx* dst = buf1;
  int Ns = 1;
  for (int s = 0; s < p.nst; ++s) {
    const int R = p.radix[s];
    if (R == 4)
      stockham_pass<4>(src, dst, p.n, Ns, tw, sign, nbatch, bstride, tid, nthreads);
    else if (R == 3)
      stockham_pass<3>(src, dst, p.n, Ns, tw, sign, nbatch, bstride, tid, nthreads);
    else
      stockham_pass<2>(src, dst, p.n, Ns, tw, sign, nbatch, bstride, tid, nthreads);
    __syncthreads();
    cplx* t = src;
    src = dst;
    dst = t;
    Ns *= R;
  }
  return src;
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
