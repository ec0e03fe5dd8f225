// Batched banded LU with partial pivoting (one real system per wavenumber) and its
// forward and transposed solves, executed by one wave64 per right-hand side pair
// (the real and imaginary parts share the real factors).
//
// Factor storage of one system (n rows, kl sub-diagonals, ku super-diagonals of the
// unfactored matrix, uw = kl + ku + 1 entries per row of U after pivoting fill):
//   Lc[j*kl + i]  multiplier of row j+1+i in column j (i < kl)
//   Uc[j*uw + t]  t = 0: 1/U[j][j];  t >= 1: U[j-t][j]   (column j of U, upward)
//   Ur[j*uw + t]  t = 0: 1/U[j][j];  t >= 1: U[j][j+t]   (row j of U, rightward)
//   piv[j]        row exchanged with row j at elimination step j (>= j)
// Column-wise L and U serve the forward solve, row-wise U and column-wise L the
// transposed solve, so both sweeps are axpy-shaped except the final L^T sweep.
#pragma once
#include "sps_device.h"

struct BandFactors {
  const double* Lc;
  const double* Uc;
  const double* Ur;
  const int* piv;
};

// Shift a wave-resident window toward lower lanes: lane l receives lane l+1.
__device__ __forceinline__ cplx wave_shift_down(cplx w) {
  return cmk(__shfl_down(w.x, 1), __shfl_down(w.y, 1));
}
__device__ __forceinline__ cplx wave_shift_up(cplx w) {
  return cmk(__shfl_up(w.x, 1), __shfl_up(w.y, 1));
}

// x = A^{-1} b for one system; b (LDS, n complex) is overwritten by x.
// Must be executed by all 64 lanes of one wave, with nothing else writing b.
__device__ inline void band_solve_wave(const BandFactors f, int n, int kl, int uw, cplx* b) {
  const int lane = lane_id();
  // ---- forward sweep: row exchanges and unit-lower L, window lane l = b[j + l]
  cplx w = (lane < n) ? b[lane] : czero();
  double lnext = (lane >= 1 && lane <= kl) ? f.Lc[lane - 1] : 0.0;
  int pnext = f.piv[0];
  for (int j = 0; j < n; ++j) {
    const double lj = lnext;
    const int p = pnext - j;
    if (j + 1 < n) {
      lnext = (lane >= 1 && lane <= kl) ? f.Lc[(j + 1) * kl + lane - 1] : 0.0;
      pnext = f.piv[j + 1];
    }
    const double vr = readlane_d(w.x, p), vi = readlane_d(w.y, p);
    const double ur = readlane_d(w.x, 0), ui = readlane_d(w.y, 0);
    if (lane == p) w = cmk(ur, ui);
    w.x -= lj * vr;
    w.y -= lj * vi;
    if (lane == 0) b[j] = cmk(vr, vi);
    w = wave_shift_down(w);
    if (lane == SPS_WAVE - 1) w = (j + SPS_WAVE < n) ? b[j + SPS_WAVE] : czero();
  }
  // ---- back substitution with column-wise U, window lane l = b[j - l]
  w = (n - 1 - lane >= 0) ? b[n - 1 - lane] : czero();
  double unext = (lane < uw) ? f.Uc[(n - 1) * uw + lane] : 0.0;
  for (int j = n - 1; j >= 0; --j) {
    const double uj = unext;
    if (j > 0) unext = (lane < uw) ? f.Uc[(j - 1) * uw + lane] : 0.0;
    const double inv = readlane_d(uj, 0);
    const double xr = readlane_d(w.x, 0) * inv, xi = readlane_d(w.y, 0) * inv;
    if (lane >= 1) {
      w.x -= uj * xr;
      w.y -= uj * xi;
    }
    if (lane == 0) b[j] = cmk(xr, xi);
    w = wave_shift_down(w);
    if (lane == SPS_WAVE - 1) w = (j - SPS_WAVE >= 0) ? b[j - SPS_WAVE] : czero();
  }
}

// x = A^{-T} b (the real factors transposed; complex b handled part by part).
__device__ inline void band_solve_t_wave(const BandFactors f, int n, int kl, int uw, cplx* b) {
  const int lane = lane_id();
  // ---- U^T z = b, forward, row-wise U, window lane l = b[j + l]
  cplx w = (lane < n) ? b[lane] : czero();
  double unext = (lane < uw) ? f.Ur[lane] : 0.0;
  for (int j = 0; j < n; ++j) {
    const double uj = unext;
    if (j + 1 < n) unext = (lane < uw) ? f.Ur[(j + 1) * uw + lane] : 0.0;
    const double inv = readlane_d(uj, 0);
    const double zr = readlane_d(w.x, 0) * inv, zi = readlane_d(w.y, 0) * inv;
    if (lane >= 1) {
      w.x -= uj * zr;
      w.y -= uj * zi;
    }
    if (lane == 0) b[j] = cmk(zr, zi);
    w = wave_shift_down(w);
    if (lane == SPS_WAVE - 1) w = (j + SPS_WAVE < n) ? b[j + SPS_WAVE] : czero();
  }
  // ---- L^T and the exchanges in reverse order; window lane l = b[j + l]
  w = (lane == 0) ? b[n - 1] : czero();
  double lnext = (lane >= 1 && lane <= kl) ? f.Lc[(n - 1) * kl + lane - 1] : 0.0;
  int pnext = f.piv[n - 1];
  for (int j = n - 1; j >= 0; --j) {
    const double lj = lnext;
    const int p = pnext - j;
    if (j > 0) {
      lnext = (lane >= 1 && lane <= kl) ? f.Lc[(j - 1) * kl + lane - 1] : 0.0;
      pnext = f.piv[j - 1];
    }
    double sr = lj * w.x, si = lj * w.y;   // lanes 1..kl hold b[j+1..j+kl]
    sr += __shfl_xor(sr, 1); si += __shfl_xor(si, 1);
    sr += __shfl_xor(sr, 2); si += __shfl_xor(si, 2);
    sr += __shfl_xor(sr, 4); si += __shfl_xor(si, 4);
    if (lane == 0) { w.x -= sr; w.y -= si; }
    const double vr = readlane_d(w.x, p), vi = readlane_d(w.y, p);
    const double ur = readlane_d(w.x, 0), ui = readlane_d(w.y, 0);
    if (lane == p) w = cmk(ur, ui);
    if (lane == 0) w = cmk(vr, vi);
    // position j + 63 can no longer be reached by an exchange: it is final
    if (lane == SPS_WAVE - 1 && j + SPS_WAVE - 1 < n) b[j + SPS_WAVE - 1] = w;
    if (j > 0) {
      w = wave_shift_up(w);
      if (lane == 0) w = b[j - 1];
    }
  }
  if (lane < SPS_WAVE - 1 && lane < n) b[lane] = w;
}

// ---------------------------------------------------------------------------- factor
// One block (>= 64 threads) per system.  AB: row-band input for this system,
// band[i*(kl+ku+1) + (c - i + kl)] = A[i][c], combined as a*BM + b*BL.
// LDS layout (LAPACK band with fill rows): ab[c*ldab + (kv + i - c)] = A[i][c],
// ldab = 2kl + ku + 1, kv = kl + ku.
__device__ inline void band_factor_block(const double* __restrict__ BM, const double* __restrict__ BL,
                                         double a, double bcoef, int n, int kl, int ku, double* ab,
                                         int* sh, double* Lc, double* Uc, double* Ur, int* piv,
                                         int* err) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int ldab = 2 * kl + ku + 1, kv = kl + ku, bw = kl + ku + 1, uw = kl + ku + 1;
  for (int e = tid; e < n * ldab; e += nt) ab[e] = 0.0;
  __syncthreads();
  for (int e = tid; e < n * bw; e += nt) {
    const int i = e / bw, d = e - i * bw;
    const int c = i + d - kl;
    if (c >= 0 && c < n) ab[c * ldab + (kv + i - c)] = a * BM[e] + bcoef * BL[e];
  }
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    const int km = min(kl, n - 1 - j);
    const int wd = min(kv, n - 1 - j);  // columns right of j that can hold fill
    if (tid == 0) {
      int jp = 0;
      double best = fabs(ab[j * ldab + kv]);
      for (int i = 1; i <= km; ++i) {
        const double v = fabs(ab[j * ldab + kv + i]);
        if (v > best) { best = v; jp = i; }
      }
      sh[0] = jp;
      piv[j] = j + jp;
      if (!(best > 0.0) || !isfinite(best)) atomicOr(err, 1);
    }
    __syncthreads();
    const int jp = sh[0];
    if (jp != 0) {
      for (int c = j + tid; c <= j + wd; c += nt) {
        double* p0 = &ab[c * ldab + kv + j - c];
        double* p1 = &ab[c * ldab + kv + j + jp - c];
        const double t = *p0; *p0 = *p1; *p1 = t;
      }
    }
    __syncthreads();
    const double piv_v = ab[j * ldab + kv];
    const double rinv = 1.0 / piv_v;
    for (int i = 1 + tid; i <= km; i += nt) ab[j * ldab + kv + i] *= rinv;
    __syncthreads();
    for (int e = tid; e < km * wd; e += nt) {
      const int i = 1 + e % km;          // row j+i
      const int c = j + 1 + e / km;      // column c
      ab[c * ldab + kv + j + i - c] -= ab[j * ldab + kv + i] * ab[c * ldab + kv + j - c];
    }
    __syncthreads();
  }
  // export
  for (int e = tid; e < n * kl; e += nt) {
    const int j = e / kl, i = e - j * kl;
    Lc[e] = (i + 1 <= n - 1 - j) ? ab[j * ldab + kv + 1 + i] : 0.0;
  }
  for (int e = tid; e < n * uw; e += nt) {
    const int j = e / uw, t = e - j * uw;
    double vc, vr;
    if (t == 0) {
      vc = vr = 1.0 / ab[j * ldab + kv];
    } else {
      vc = (j - t >= 0) ? ab[j * ldab + kv - t] : 0.0;                 // U[j-t][j]
      vr = (j + t < n) ? ab[(j + t) * ldab + kv - t] : 0.0;            // U[j][j+t]
    }
    Uc[e] = vc;
    Ur[e] = vr;
  }
}
