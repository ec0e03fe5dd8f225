// One wavefront's complex FFT of length N = 64 R1 (R1 = 2, 3, 4 or 6), the data spread over
// the 64 lanes in registers, with two LDS exchanges inside the wave and no block barrier, so
// every wave of a block transforms its own sequence at its own pace.  All index arithmetic is
// compile-time except the lane number.
//
// Factorization N = R1 x 8 x 8 (four-step in each factor).  Two register layouts:
//   natural A: lane l (all 64) holds x[l + 64 q], q < R1, in a[q];
//   permuted P: lane L < 8 R1, with k1 = L >> 3 and k1' = L & 7, holds
//               x[k1 + R1 k1' + 8 R1 m], m < 8, in p[m].
// wfft_a_to_p maps natural-order input to the DFT in the permuted layout; wfft_p_to_a maps
// permuted-layout input to the DFT in natural order (the transposed factorization: the same
// stages in reverse order).  A pointwise operation between the two can work in the permuted
// layout directly, as long as every operand is in it.
//   SIGN = -1: X_k = sum_n x_n exp(-2 pi i n k / N); SIGN = +1: the conjugate kernel
//   (unnormalized inverse).
//   tw[t] = exp(-2 pi i t / N), t < N (LDS or global); sc: this wave's scratch of
//   fpad_size(N) complex entries in LDS.
#pragma once
#include "sps_device.h"

// Compiler-only barrier between LDS accesses of one wave (the LDS executes a wave's
// instructions in order, so a lane reads what another lane of the same wave wrote before).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

template <int SIGN>
__device__ __forceinline__ cplx wtw(const cplx* tw, int e) {
  const cplx w = tw[e];
  return SIGN < 0 ? w : cconj(w);
}

template <int R1, int SIGN>
__device__ __forceinline__ void wfft_a_to_p(cplx (&a)[R1], cplx (&p)[8], cplx* sc, const cplx* tw) {
  const int l = lane_id();
  // DFT over q (stride 64), twiddle exp(SIGN 2 pi i l k1 / N)
  dft_small<R1>(a, SIGN);
#pragma unroll
  for (int k1 = 1; k1 < R1; ++k1) a[k1] = cmul(a[k1], wtw<SIGN>(tw, l * k1));
#pragma unroll
  for (int k1 = 0; k1 < R1; ++k1) sc[fpad(k1 * 64 + l)] = a[k1];
  wave_lds_sync();
  // 64-point DFT of each k1 row: 8 x 8, lane L = 8 k1 + n2' (low digit n2')
  const int k1 = l >> 3, lo = l & 7;
  const bool act = l < 8 * R1;
  cplx b[8];
  if (act) {
#pragma unroll
    for (int h = 0; h < 8; ++h) b[h] = sc[fpad(k1 * 64 + 8 * h + lo)];
  }
  wave_lds_sync();
  if (act) {
    dft_small<8>(b, SIGN);
#pragma unroll
    for (int h = 1; h < 8; ++h) b[h] = cmul(b[h], wtw<SIGN>(tw, R1 * lo * h));   // exp(SIGN 2 pi i n2' k1' / 64)
#pragma unroll
    for (int h = 0; h < 8; ++h) sc[fpad(k1 * 64 + 8 * h + lo)] = b[h];   // [k1][k1'][n2']
  }
  wave_lds_sync();
  if (act) {
#pragma unroll
    for (int h = 0; h < 8; ++h) p[h] = sc[fpad(k1 * 64 + 8 * lo + h)];   // lane L = 8 k1 + k1'
    dft_small<8>(p, SIGN);
  }
  wave_lds_sync();
}

template <int R1, int SIGN>
__device__ __forceinline__ void wfft_p_to_a(cplx (&p)[8], cplx (&a)[R1], cplx* sc, const cplx* tw) {
  const int l = lane_id();
  const int k1 = l >> 3, lo = l & 7;
  const bool act = l < 8 * R1;
  if (act) {
    // DFT over m (high digit), twiddle exp(SIGN 2 pi i k1' a / 64), to [k1][a][k1']
    dft_small<8>(p, SIGN);
#pragma unroll
    for (int h = 1; h < 8; ++h) p[h] = cmul(p[h], wtw<SIGN>(tw, R1 * lo * h));
#pragma unroll
    for (int h = 0; h < 8; ++h) sc[fpad(k1 * 64 + 8 * h + lo)] = p[h];
  }
  wave_lds_sync();
  cplx e[8];
  if (act) {
#pragma unroll
    for (int h = 0; h < 8; ++h) e[h] = sc[fpad(k1 * 64 + 8 * lo + h)];   // lane 8 k1 + a, over k1'
  }
  wave_lds_sync();
  if (act) {
    dft_small<8>(e, SIGN);
#pragma unroll
    for (int h = 0; h < 8; ++h) {
      const int n2 = lo + 8 * h;
      sc[fpad(k1 * 64 + n2)] = cmul(e[h], wtw<SIGN>(tw, k1 * n2));   // exp(SIGN 2 pi i k1 n2 / N)
    }
  }
  wave_lds_sync();
#pragma unroll
  for (int q = 0; q < R1; ++q) a[q] = sc[fpad(q * 64 + l)];
  dft_small<R1>(a, SIGN);
  wave_lds_sync();
}
