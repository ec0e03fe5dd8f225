// Linear stability of plane Poiseuille flow on gfx950: the eigenvalue problem of the paper's
// neutral-curve example (Results, "Parametric sensitivity and numerical continuation";
// Supplementary, "Eigenvalue problems"), its adjoint eigenvectors, the eigenvalue
// sensitivities of equ:eigenvalue_sens and Newton's method on the growth rate, every system
// (one streamwise wavenumber alpha at one Reynolds number Re) in one thread block.
//
// Flow between walls y = 0 and y = 2, base flow U = y (2 - y).  Two-dimensional perturbations
// (u, v, p) ~ exp(i alpha x + lambda t) satisfy, with nu = 1/Re, x = y - 1 in [-1, 1], D = d/dx,
// U = 1 - x^2, U' = -2x:
//   lambda u + i alpha U u + U' v + i alpha p - nu (D^2 - alpha^2) u = 0
//   lambda v + i alpha U v + D p - nu (D^2 - alpha^2) v = 0
//   i alpha u + D v = 0,      u = v = 0 at x = -1, 1,
// i.e. (lambda M + L) X = 0.  The discretization is the 2D problem's ultraspherical one (paper:
// Sparse spectral methods): Chebyshev-T unknowns, momentum rows in C2 coefficients, continuity
// in C1, first-order lifted taus, four boundary rows and the row tau_p = 0; a base-flow product
// row holds the first N C2 coefficients of the exact product series.  Slots (S = 3N + 5):
// u[0:N], v[N:2N], p[2N:3N], tau_u1, tau_v1, tau_u2, tau_v2, tau_p.
//
// L = L0 + alpha La + nu Ln + nu alpha^2 Lq, so the host assembles the five parts (with M) once;
// a system's matrix A = sigma M + L(alpha, nu) is formed on the device.  The advection term
// i alpha U is imaginary in the rows where the pressure gradient i alpha p is too, so no
// diagonal phases make A real (unlike the 2D convection problem): A is factored by a complex
// banded LU with partial pivoting.  Rows and columns are interleaved by mode and the u and v
// columns recombined (T_n - T_{n-2}, Dirichlet) so that the boundary rows are short and A is
// banded (kl = 11, ku = 19 at every N).
//
// One block per system runs, for every Newton iteration: assembly, the LU factorization, the
// right eigenvector by inverse iteration y <- A^{-1} M y (wave 0) and at the same time the left
// eigenvector by w <- A^{-H} M^H w (wave 1) through the same factors, then the sensitivities
// d lambda/dRe = -<w, dL/dRe y> / <w, M y>, d lambda/dalpha likewise, and the Newton update of Re
// (or alpha) on the growth rate Re(lambda) with the next shift at the new eigenvalue.  A
// continuation step (the paper's tracing of the neutral curve) first moves along the curve's
// tangent, the gradient of the growth rate turned by a right angle, then corrects by Newton steps
// along the gradient (the smallest change of the parameters that zeroes the linearized growth
// rate), which also passes the curve's turning points.  All
// vectors stay in the permuted, recombined coordinates of A's band (the eigenvalues and the
// inner products are the same); the eigenvectors are converted to the state layout at the end.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "sps_device.h"
#include "sps_internal.h"
#include "ultra_ops.h"

namespace sps {
namespace {

constexpr int PT = 256;   // threads per system block (wave 0: right iteration, wave 1: left)

__device__ __forceinline__ double cabs1(cplx a) { return fabs(a.x) + fabs(a.y); }
__device__ __forceinline__ cplx cmulc(cplx a, cplx b) {   // conj(a) b
  return cmk(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ cplx crecip(cplx a) {
  const double s = 1.0 / (a.x * a.x + a.y * a.y);
  return cmk(a.x * s, -a.y * s);
}
// LDS vectors are read and written through volatile pointers: within one wave LDS accesses
// execute in program order, so a value one lane writes is seen by the next access of every
// lane, and the compiler keeps them in that order without a fence (a fence would also wait for
// the global loads issued ahead).
__device__ __forceinline__ cplx vld(const volatile double* v, int i) { return cmk(v[2 * i], v[2 * i + 1]); }
__device__ __forceinline__ void vst(volatile double* v, int i, cplx a) {
  v[2 * i] = a.x;
  v[2 * i + 1] = a.y;
}
__device__ __forceinline__ cplx wave_csum(cplx a) {
  for (int o = 32; o >= 1; o >>= 1) {
    a.x += __shfl_xor(a.x, o);
    a.y += __shfl_xor(a.y, o);
  }
  return a;
}

struct PoisDev {
  int N, S, kl, ku, bw, ldw;     // bw = kl + ku + 1 (the operators), ldw = 2 kl + ku + 1 (LU with fill)
  const cplx* bM;                // [S][bw] row bands of the permuted, recombined M
  const cplx* bL0;               // parts of L: L0 + alpha La + nu Ln + nu alpha^2 Lq
  const cplx* bLa;
  const cplx* bLn;
  const cplx* bLq;
  const int* rowmap;             // band row i <- state row rowmap[i]
  const int* colinv;             // state column c -> band column colinv[c]
  const double* rho;             // recombination: x[c] = y'[c] + rho[c] y'[c + 2]
  cplx* W;                       // [sys][S][ldw] LU factors, column-major (element (i, j) at j ldw + kl + ku + i - j)
  cplx* dinv;                    // [sys][S] reciprocals of U's diagonal
  int* piv;                      // [sys][S] row interchanges
  int* err;
};

struct PoisArgs {
  const double* params;          // [sys][5] alpha, Re, sigma (re, im), continuation step ds
  int iters, mode, maxit;        // inverse iterations per solve; 0: eigenpair only, 1: Newton in Re, 2: in
                                 // alpha, 3: continuation step
  double tol;                    // Newton stops when |Re(lambda)| <= tol
  cplx* lam;                     // [sys]
  cplx* dlam;                    // [sys][2]: d lambda/dRe, d lambda/dalpha
  double* info;                  // [sys][3]: alpha, Re at the end, eigenvalue solves
  cplx* X;                       // [sys][S] right eigenvector, state layout, unit norm (nullable)
  cplx* Y;                       // [sys][S] left eigenvector (nullable)
};

// y = B x (op band [S][bw]) for rows i = lane, lane + 64, ...; one wave; x, y in LDS
__device__ void wave_band_mv(const PoisDev& d, const cplx* B, const volatile double* x, volatile double* y) {
  const int lane = threadIdx.x & 63, n = d.S;
  for (int i = lane; i < n; i += 64) {
    cplx s = czero();
    const int d0 = max(0, d.kl - i), d1 = min(d.bw - 1, n - 1 - i + d.kl);
    for (int q = d0; q <= d1; ++q) s = cadd(s, cmul(B[(size_t)i * d.bw + q], vld(x, i + q - d.kl)));
    vst(y, i, s);
  }
}
// y = B^H x
__device__ void wave_band_mvh(const PoisDev& d, const cplx* B, const volatile double* x, volatile double* y) {
  const int lane = threadIdx.x & 63, n = d.S;
  for (int j = lane; j < n; j += 64) {
    cplx s = czero();
    const int i0 = max(0, j - d.ku), i1 = min(n - 1, j + d.kl);
    for (int i = i0; i <= i1; ++i) s = cadd(s, cmulc(B[(size_t)i * d.bw + (j - i + d.kl)], vld(x, i)));
    vst(y, j, s);
  }
}

// b <- A^{-1} b through the factors (row interchanges and L, then U); one wave.  The factor
// entries of the next D columns are loaded ahead into a register ring.
constexpr int PD = 8;
__device__ void wave_lu_solve(const PoisDev& d, const cplx* W, const cplx* dinv, const int* piv,
                              volatile double* b) {
  const int lane = threadIdx.x & 63, n = d.S, kl = d.kl, kv = d.kl + d.ku, ldw = d.ldw;
  auto lload = [&](int j) {
    return (j < n - 1 && lane >= 1 && lane <= min(kl, n - 1 - j)) ? W[(size_t)j * ldw + kv + lane] : czero();
  };
  cplx ring[PD];
  int pr[PD];
#pragma unroll
  for (int k = 0; k < PD; ++k) {
    ring[k] = lload(k);
    pr[k] = (k < n) ? piv[k] : k;
  }
  for (int j0 = 0; j0 < n - 1; j0 += PD) {
#pragma unroll
    for (int k = 0; k < PD; ++k) {
      const int j = j0 + k;
      if (j < n - 1) {
        const cplx l = ring[k];
        const int p = pr[k];
        ring[k] = lload(j + PD);
        pr[k] = (j + PD < n) ? piv[j + PD] : j + PD;
        if (p != j && lane == 0) {
          const cplx t = vld(b, j);
          vst(b, j, vld(b, p));
          vst(b, p, t);
        }
        const cplx bj = vld(b, j);
        if (lane >= 1 && lane <= min(kl, n - 1 - j)) vst(b, j + lane, csub(vld(b, j + lane), cmul(l, bj)));
      }
    }
  }
  auto uload = [&](int j) {
    return (j >= 0 && lane >= 1 && lane <= min(kv, j)) ? W[(size_t)j * ldw + kv - lane] : czero();
  };
#pragma unroll
  for (int k = 0; k < PD; ++k) {
    ring[k] = uload(n - 1 - k);
  }
  cplx dr[PD];
#pragma unroll
  for (int k = 0; k < PD; ++k) dr[k] = (n - 1 - k >= 0) ? dinv[n - 1 - k] : czero();
  for (int j0 = n - 1; j0 >= 0; j0 -= PD) {
#pragma unroll
    for (int k = 0; k < PD; ++k) {
      const int j = j0 - k;
      if (j >= 0) {
        const cplx u = ring[k], di = dr[k];
        ring[k] = uload(j - PD);
        dr[k] = (j - PD >= 0) ? dinv[j - PD] : czero();
        const cplx bj = cmul(vld(b, j), di);
        if (lane == 0) vst(b, j, bj);
        if (lane >= 1 && lane <= min(kv, j)) vst(b, j - lane, csub(vld(b, j - lane), cmul(u, bj)));
      }
    }
  }
}

// b <- A^{-H} b: U^H forward (row sums), then L^H backward with the row interchanges in reverse;
// one wave.
__device__ void wave_lu_solve_h(const PoisDev& d, const cplx* W, const cplx* dinv, const int* piv,
                                volatile double* b) {
  const int lane = threadIdx.x & 63, n = d.S, kl = d.kl, kv = d.kl + d.ku, ldw = d.ldw;
  auto uload = [&](int j) {
    return (j < n && lane >= 1 && lane <= min(kv, j)) ? W[(size_t)j * ldw + kv - lane] : czero();
  };
  cplx ring[PD], dr[PD];
#pragma unroll
  for (int k = 0; k < PD; ++k) {
    ring[k] = uload(k);
    dr[k] = (k < n) ? dinv[k] : czero();
  }
  for (int j0 = 0; j0 < n; j0 += PD) {
#pragma unroll
    for (int k = 0; k < PD; ++k) {
      const int j = j0 + k;
      if (j < n) {
        const cplx u = ring[k], di = dr[k];
        ring[k] = uload(j + PD);
        dr[k] = (j + PD < n) ? dinv[j + PD] : czero();
        cplx t = (lane >= 1 && lane <= min(kv, j)) ? cmulc(u, vld(b, j - lane)) : czero();
        t = wave_csum(t);
        if (lane == 0) vst(b, j, cmulc(di, csub(vld(b, j), t)));   // (b_j - sum) / conj(u_jj)
      }
    }
  }
  auto lload = [&](int j) {
    return (j >= 0 && j < n - 1 && lane >= 1 && lane <= min(kl, n - 1 - j)) ? W[(size_t)j * ldw + kv + lane]
                                                                             : czero();
  };
  int pr[PD];
#pragma unroll
  for (int k = 0; k < PD; ++k) {
    ring[k] = lload(n - 2 - k);
    pr[k] = (n - 2 - k >= 0) ? piv[n - 2 - k] : 0;
  }
  for (int j0 = n - 2; j0 >= 0; j0 -= PD) {
#pragma unroll
    for (int k = 0; k < PD; ++k) {
      const int j = j0 - k;
      if (j >= 0) {
        const cplx l = ring[k];
        const int p = pr[k];
        ring[k] = lload(j - PD);
        pr[k] = (j - PD >= 0) ? piv[j - PD] : 0;
        cplx t = (lane >= 1 && lane <= min(kl, n - 1 - j)) ? cmulc(l, vld(b, j + lane)) : czero();
        t = wave_csum(t);
        if (lane == 0) {
          const cplx bj = csub(vld(b, j), t);
          if (p != j) {
            vst(b, j, vld(b, p));
            vst(b, p, bj);
          } else {
            vst(b, j, bj);
          }
        }
      }
    }
  }
}

// Normalizes x (one wave) and returns <prev, x> / |x| before normalization's scale applied, i.e.
// mu = conj(prev) . x with prev of unit norm (the inverse-iteration Rayleigh estimate).
__device__ cplx wave_normalize(const PoisDev& d, const volatile double* prev, volatile double* x) {
  const int lane = threadIdx.x & 63;
  cplx mu = czero();
  double nn = 0.0;
  for (int i = lane; i < d.S; i += 64) {
    const cplx a = vld(prev, i), b = vld(x, i);
    mu = cadd(mu, cmulc(a, b));
    nn += b.x * b.x + b.y * b.y;
  }
  mu = wave_csum(mu);
  for (int o = 32; o >= 1; o >>= 1) nn += __shfl_xor(nn, o);
  const double inv = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
  for (int i = lane; i < d.S; i += 64) vst(x, i, cscale(vld(x, i), inv));
  return mu;
}

template <int NV>
__device__ void block_csums(cplx* v, double* red) {
  const int tid = threadIdx.x, w = tid >> 6;
  for (int q = 0; q < NV; ++q) v[q] = wave_csum(v[q]);
  __syncthreads();
  if ((tid & 63) == 0)
    for (int q = 0; q < NV; ++q) {
      red[(w * NV + q) * 2] = v[q].x;
      red[(w * NV + q) * 2 + 1] = v[q].y;
    }
  __syncthreads();
  for (int q = 0; q < NV; ++q) {
    cplx s = czero();
    for (int ww = 0; ww < PT / 64; ++ww) s = cadd(s, cmk(red[(ww * NV + q) * 2], red[(ww * NV + q) * 2 + 1]));
    v[q] = s;
  }
  __syncthreads();
}

// LDS: y, w (right and left vectors), t0, t1 (their matrix products), S complex each; then
// reduction and pivot scratch.
__global__ void __launch_bounds__(PT) pois_evp(PoisDev d, PoisArgs a) {
  extern __shared__ double sm[];
  volatile double* y = sm;
  volatile double* w = y + 2 * d.S;
  volatile double* t0 = w + 2 * d.S;
  volatile double* t1 = t0 + 2 * d.S;
  cplx* lm = reinterpret_cast<cplx*>(sm + 8 * d.S);   // kl + 1 multipliers of the current column
  double* red = reinterpret_cast<double*>(lm + 32);   // 2 * 3 * PT / 64 doubles
  __shared__ int s_p, s_ju, s_stop;
  __shared__ double s_par[2];     // alpha, Re
  __shared__ cplx s_sig, s_lam;
  const int sys = blockIdx.x, tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int n = d.S, kl = d.kl, ku = d.ku, kv = kl + ku, ldw = d.ldw, bw = d.bw;
  cplx* W = d.W + (size_t)sys * n * ldw;
  cplx* dinv = d.dinv + (size_t)sys * n;
  int* piv = d.piv + (size_t)sys * n;
  if (tid == 0) {
    s_par[0] = a.params[5 * sys];
    s_par[1] = a.params[5 * sys + 1];
    s_sig = cmk(a.params[5 * sys + 2], a.params[5 * sys + 3]);
    s_stop = 0;
  }
  // start vectors (the same for every system), unit norm
  for (int i = tid; i < n; i += PT) {
    const cplx s0 = cmk(1.0 / (1 + i % 7), 0.5 / (1 + i % 5));
    vst(t0, i, s0);
    vst(y, i, s0);
    vst(w, i, s0);
  }
  __syncthreads();
  if (wave == 0) (void)wave_normalize(d, t0, y);
  else if (wave == 1) (void)wave_normalize(d, t0, w);
  __syncthreads();
  int solves = 0;
  cplx dl0 = czero(), dl1 = czero();
  for (int it = 0; it < max(1, a.maxit); ++it) {
    const double alpha = s_par[0], Re = s_par[1], nu = 1.0 / Re, q2 = nu * alpha * alpha;
    const cplx sig = s_sig;
    // ---- assembly of A = sigma M + L0 + alpha La + nu Ln + nu alpha^2 Lq (fill rows zero)
    for (size_t e = tid; e < (size_t)n * ldw; e += PT) W[e] = czero();
    __syncthreads();
    for (size_t e = tid; e < (size_t)n * bw; e += PT) {
      const int i = (int)(e / bw), q = (int)(e - (size_t)i * bw), j = i + q - kl;
      if (j < 0 || j >= n) continue;
      cplx v = cadd(cmul(sig, d.bM[e]), d.bL0[e]);
      v = cadd(v, cscale(d.bLa[e], alpha));
      v = cadd(v, cscale(d.bLn[e], nu));
      v = cadd(v, cscale(d.bLq[e], q2));
      W[(size_t)j * ldw + kv + i - j] = v;
    }
    if (tid == 0) s_ju = 0;
    __syncthreads();
    // ---- banded LU with partial pivoting (row interchanges applied up to the fill column)
    for (int j = 0; j < n; ++j) {
      const int km = min(kl, n - 1 - j);
      if (wave == 0) {
        const cplx v = (lane <= km) ? W[(size_t)j * ldw + kv + lane] : czero();
        double m = (lane <= km) ? cabs1(v) : -1.0;
        int idx = lane;
        for (int o = 32; o >= 1; o >>= 1) {
          const double mo = __shfl_xor(m, o);
          const int io = __shfl_xor(idx, o);
          if (mo > m || (mo == m && io < idx)) {
            m = mo;
            idx = io;
          }
        }
        if (lane == 0) {
          s_p = idx;
          s_ju = max(s_ju, min(j + ku + idx, n - 1));
          piv[j] = j + idx;
          if (!(m > 0.0)) atomicOr(d.err, 1);
        }
      }
      __syncthreads();
      const int p = s_p, ju = s_ju;
      if (p != 0)
        for (int c = j + tid; c <= ju; c += PT) {
          cplx* r0 = W + (size_t)c * ldw + kv + j - c;
          cplx* r1 = r0 + p;
          const cplx t = *r0;
          *r0 = *r1;
          *r1 = t;
        }
      __syncthreads();
      const cplx pv = W[(size_t)j * ldw + kv];
      const cplx pinv = (pv.x != 0.0 || pv.y != 0.0) ? crecip(pv) : czero();
      if (tid == 0) dinv[j] = pinv;
      if (tid >= 1 && tid <= km) {
        const cplx l = cmul(W[(size_t)j * ldw + kv + tid], pinv);
        W[(size_t)j * ldw + kv + tid] = l;
        lm[tid] = l;
      }
      __syncthreads();
      const int nc = ju - j;
      for (int e = tid; e < km * nc; e += PT) {
        const int r = 1 + e / nc, c = j + 1 + e % nc;
        cplx* t = W + (size_t)c * ldw + kv + j + r - c;
        *t = csub(*t, cmul(lm[r], W[(size_t)c * ldw + kv + j - c]));
      }
      __syncthreads();
    }
    // ---- right (wave 0) and left (wave 1) inverse iterations through the factors
    if (wave == 0) {
      cplx mu = czero();
      for (int k = 0; k < a.iters; ++k) {
        wave_band_mv(d, d.bM, y, t0);
        wave_lu_solve(d, W, dinv, piv, t0);
        mu = wave_normalize(d, y, t0);
        for (int i = lane; i < n; i += 64) vst(y, i, vld(t0, i));
      }
      if (lane == 0) {
        const double m2 = mu.x * mu.x + mu.y * mu.y;
        s_lam = cmk(sig.x - mu.x / m2, sig.y + mu.y / m2);   // sigma - 1/mu
      }
    } else if (wave == 1) {
      for (int k = 0; k < a.iters; ++k) {
        wave_band_mvh(d, d.bM, w, t1);
        wave_lu_solve_h(d, W, dinv, piv, t1);
        (void)wave_normalize(d, w, t1);
        for (int i = lane; i < n; i += 64) vst(w, i, vld(t1, i));
      }
    }
    __syncthreads();
    ++solves;
    // ---- sensitivities: <w, M y>, <w, dL/dRe y>, <w, dL/dalpha y>
    cplx acc[3] = {czero(), czero(), czero()};
    for (int i = tid; i < n; i += PT) {
      cplx my = czero(), dr = czero(), da = czero();
      const int q0 = max(0, kl - i), q1 = min(bw - 1, n - 1 - i + kl);
      for (int q = q0; q <= q1; ++q) {
        const size_t e = (size_t)i * bw + q;
        const cplx yv = vld(y, i + q - kl);
        my = cadd(my, cmul(d.bM[e], yv));
        // dL/dRe = -nu^2 (Ln + alpha^2 Lq), dL/dalpha = La + 2 nu alpha Lq
        dr = cadd(dr, cmul(cadd(d.bLn[e], cscale(d.bLq[e], alpha * alpha)), yv));
        da = cadd(da, cmul(cadd(d.bLa[e], cscale(d.bLq[e], 2.0 * nu * alpha)), yv));
      }
      const cplx wv = vld(w, i);
      acc[0] = cadd(acc[0], cmulc(wv, my));
      acc[1] = cadd(acc[1], cmulc(wv, dr));
      acc[2] = cadd(acc[2], cmulc(wv, da));
    }
    block_csums<3>(acc, red);
    {
      const cplx den = acc[0];
      const double dd = den.x * den.x + den.y * den.y;
      auto qdiv = [&](cplx num) { return cscale(cmulc(den, num), -1.0 / dd); };   // -num / den
      dl0 = cscale(qdiv(acc[1]), -nu * nu);
      dl1 = qdiv(acc[2]);
    }
    if (tid == 0) {
      const cplx lam = s_lam;
      const double g = lam.x;
      // gradient of the growth rate in (alpha, ln Re)
      const double ga = dl1.x, gr = Re * dl0.x, g2 = ga * ga + gr * gr;
      if (a.mode == 3 && it == 0) {
        // predictor: a step ds along the tangent of the level curve, the gradient turned by a
        // right angle (the unstable side stays on the same hand)
        const double gn = sqrt(g2), ds = a.params[5 * sys + 4];
        s_par[0] = alpha - ds * gr / gn;
        s_par[1] = Re * exp(ds * ga / gn);
        s_sig = lam;
      } else if (a.mode == 0 || fabs(g) <= a.tol || it + 1 >= max(1, a.maxit)) {
        s_stop = 1;
        if (a.mode != 0 && fabs(g) > a.tol) atomicOr(d.err, 4);
      } else if (a.mode == 3) {
        // corrector: the minimum-norm Newton step in (alpha, ln Re)
        s_par[0] = alpha - g * ga / g2;
        s_par[1] = Re * exp(-g * gr / g2);
        s_sig = lam;
      } else if (a.mode == 1) {
        s_par[1] = Re - g / dl0.x;
        s_sig = lam;
      } else {
        s_par[0] = alpha - g / dl1.x;
        s_sig = lam;
      }
    }
    __syncthreads();
    if (s_stop) break;
  }
  // ---- outputs
  if (tid == 0) {
    a.lam[sys] = s_lam;
    a.dlam[2 * sys] = dl0;
    a.dlam[2 * sys + 1] = dl1;
    a.info[3 * sys] = s_par[0];
    a.info[3 * sys + 1] = s_par[1];
    a.info[3 * sys + 2] = solves;
  }
  if (a.X) {
    // X = R P_c y in the state layout, then unit norm
    cplx* X = a.X + (size_t)sys * n;
    double nn = 0.0;
    for (int c = tid; c < n; c += PT) {
      cplx v = vld(y, d.colinv[c]);
      if (d.rho[c] != 0.0) v = cadd(v, cscale(vld(y, d.colinv[c + 2]), d.rho[c]));
      vst(t0, c, v);
      nn += v.x * v.x + v.y * v.y;
    }
    cplx s[1] = {cmk(nn, 0.0)};
    block_csums<1>(s, red);
    const double inv = 1.0 / sqrt(s[0].x);
    for (int c = tid; c < n; c += PT) X[c] = cscale(vld(t0, c), inv);
  }
  if (a.Y) {
    cplx* Y = a.Y + (size_t)sys * n;
    double nn = 0.0;
    for (int i = tid; i < n; i += PT) {
      const cplx v = vld(w, i);
      nn += v.x * v.x + v.y * v.y;
    }
    cplx s[1] = {cmk(nn, 0.0)};
    block_csums<1>(s, red);
    const double inv = 1.0 / sqrt(s[0].x);
    for (int i = tid; i < n; i += PT) Y[d.rowmap[i]] = cscale(vld(w, i), inv);
  }
}

// ---------------------------------------------------------------------------- host assembly
// Dense parts (state slot order) of the operator, written from the formulation above.
struct PoisParts {
  Cmat M, L0, La, Ln, Lq;
  explicit PoisParts(int S) : M(S), L0(S), La(S), Ln(S), Lq(S) {}
};

// rectangular (r x c) row-major products and the exact product operators
static std::vector<double> rmat(const std::vector<double>& A, int ar, int ac, const std::vector<double>& B, int bc) {
  std::vector<double> C((size_t)ar * bc, 0.0);
  for (int i = 0; i < ar; ++i)
    for (int k = 0; k < ac; ++k) {
      const double v = A[(size_t)i * ac + k];
      if (v == 0.0) continue;
      for (int j = 0; j < bc; ++j) C[(size_t)i * bc + j] += v * B[(size_t)k * bc + j];
    }
  return C;
}
// multiplication by x of a T series of m terms: (m + 1) x m
static std::vector<double> mult_x(int m) {
  std::vector<double> A((size_t)(m + 1) * m, 0.0);
  A[(size_t)1 * m + 0] = 1.0;
  for (int k = 1; k < m; ++k) {
    A[(size_t)(k + 1) * m + k] += 0.5;
    A[(size_t)(k - 1) * m + k] += 0.5;
  }
  return A;
}
// first N C2 coefficients (N x N) of the product of a T series of N terms with a polynomial of
// degree deg, given its exact product operator P ((N + deg) x N)
static std::vector<double> c2_rows(const std::vector<double>& P, int N, int deg) {
  const int m = N + deg;
  const std::vector<double> S10 = matmul(op_S1(m), op_S0(m), m);
  const std::vector<double> full = rmat(S10, m, m, P, N);
  return std::vector<double>(full.begin(), full.begin() + (size_t)N * N);
}

static void pois_assemble(int N, PoisParts& P) {
  const int U = 0, V = N, Pp = 2 * N, T = 3 * N;
  const std::vector<double> S0 = op_S0(N), S1 = op_S1(N);
  const std::vector<double> S10 = matmul(S1, S0, N);
  const std::vector<double> D0 = op_D(N, 1.0, true), D1 = op_D(N, 2.0, false);
  const std::vector<double> DZZ = matmul(D1, D0, N), SD = matmul(S1, D0, N);
  const std::vector<double> X1 = mult_x(N);                                   // (N+1) x N
  const std::vector<double> X2 = rmat(mult_x(N + 1), N + 2, N + 1, X1, N);    // (N+2) x N: x^2
  std::vector<double> Uop(X2.size());
  for (int i = 0; i < N + 2; ++i)
    for (int j = 0; j < N; ++j) Uop[(size_t)i * N + j] = (i == j ? 1.0 : 0.0) - X2[(size_t)i * N + j];
  std::vector<double> dU(X1.size());
  for (size_t e = 0; e < X1.size(); ++e) dU[e] = -2.0 * X1[e];
  const std::vector<double> SU = c2_rows(Uop, N, 2), SdU = c2_rows(dU, N, 1);
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      const size_t e = (size_t)i * N + j;
      for (int f = 0; f < 2; ++f) {
        const int r = f * N + i, c = f * N + j;
        if (S10[e] != 0.0) {
          P.M.add(r, c, S10[e]);
          P.Lq.add(r, c, S10[e]);        // + nu alpha^2 S10
        }
        if (DZZ[e] != 0.0) P.Ln.add(r, c, -DZZ[e]);
        if (SU[e] != 0.0) P.La.add(r, c, 0.0, SU[e]);   // i alpha U
      }
      if (SdU[e] != 0.0) P.L0.add(U + i, V + j, SdU[e]);           // U' v
      if (S10[e] != 0.0) P.La.add(U + i, Pp + j, 0.0, S10[e]);     // i alpha p
      if (SD[e] != 0.0) P.L0.add(V + i, Pp + j, SD[e]);            // dp/dx
      if (S0[e] != 0.0) P.La.add(Pp + i, U + j, 0.0, S0[e]);       // continuity i alpha u
      if (D0[e] != 0.0) P.L0.add(Pp + i, V + j, D0[e]);            // continuity dv/dx
    }
  // lifted taus: -nu 2 C2_{N-2} tau_1 and C2_{N-1} tau_2 in the momentum rows, C1_{N-1} tau_v1 in
  // continuity (d/dx U_{N-1} = 2 C2_{N-2})
  P.Ln.add(U + N - 2, T + 0, -2.0);
  P.Ln.add(V + N - 2, T + 1, -2.0);
  P.L0.add(U + N - 1, T + 2, 1.0);
  P.L0.add(V + N - 1, T + 3, 1.0);
  P.L0.add(Pp + N - 1, T + 1, 1.0);
  // boundary rows u(-1), u(1), v(-1), v(1) and tau_p = 0
  for (int m = 0; m < N; ++m) {
    P.L0.add(T + 0, U + m, (m & 1) ? -1.0 : 1.0);
    P.L0.add(T + 1, U + m, 1.0);
    P.L0.add(T + 2, V + m, (m & 1) ? -1.0 : 1.0);
    P.L0.add(T + 3, V + m, 1.0);
  }
  P.L0.add(T + 4, T + 4, 1.0);
}

struct PoisBands {
  int S = 0, kl = 0, ku = 0;
  std::vector<std::vector<double2>> parts;   // M, L0, La, Ln, Lq: [S][kl+ku+1]
  std::vector<int> rowmap, colmap;
  std::vector<double> rho;
};

static void pois_bands(int N, PoisBands& hb) {
  const int S = 3 * N + 5;
  PoisParts P(S);
  pois_assemble(N, P);
  std::vector<double> rho(S, 0.0);
  for (int f = 0; f < 2; ++f)
    for (int m = 0; m + 2 < N; ++m) rho[f * N + m] = -1.0;
  std::vector<int> rowmap, colmap;
  rowmap.push_back(3 * N + 4);
  for (int q = 0; q < 4; ++q) rowmap.push_back(3 * N + q);
  for (int m = 0; m < N; ++m) {
    rowmap.push_back(2 * N + m);
    rowmap.push_back(m);
    rowmap.push_back(N + m);
  }
  colmap.push_back(3 * N + 4);
  for (int m = 0; m < N; ++m)
    for (int f = 0; f < 3; ++f) colmap.push_back(f * N + m);
  for (int q = 0; q < 4; ++q) colmap.push_back(3 * N + q);
  Cmat* mats[5] = {&P.M, &P.L0, &P.La, &P.Ln, &P.Lq};
  std::vector<std::vector<double2>> dense(5);
  int kl = 0, ku = 0;
  for (int t = 0; t < 5; ++t) {
    Cmat& A = *mats[t];
    dense[t].assign((size_t)S * S, make_double2(0.0, 0.0));
    for (int i = 0; i < S; ++i) {
      const int r = rowmap[i];
      double rowmax = 0.0;
      std::vector<double2> row(S);
      for (int j = 0; j < S; ++j) {
        const int c = colmap[j];
        double2 v = A.at(r, c);
        if (c >= 2 && rho[c - 2] != 0.0) {
          v.x += A.at(r, c - 2).x * rho[c - 2];
          v.y += A.at(r, c - 2).y * rho[c - 2];
        }
        row[j] = v;
        rowmax = std::max(rowmax, std::hypot(v.x, v.y));
      }
      for (int j = 0; j < S; ++j) {
        const double2 v = row[j];
        if (std::hypot(v.x, v.y) <= 1e-14 * rowmax) continue;   // exact cancellations of the recombination
        dense[t][(size_t)i * S + j] = v;
        kl = std::max(kl, i - j);
        ku = std::max(ku, j - i);
      }
    }
  }
  const int bw = kl + ku + 1;
  hb.S = S;
  hb.kl = kl;
  hb.ku = ku;
  hb.parts.assign(5, std::vector<double2>((size_t)S * bw, make_double2(0.0, 0.0)));
  for (int t = 0; t < 5; ++t)
    for (int i = 0; i < S; ++i)
      for (int j = std::max(0, i - kl); j <= std::min(S - 1, i + ku); ++j)
        hb.parts[t][(size_t)i * bw + (j - i + kl)] = dense[t][(size_t)i * S + j];
  hb.rowmap = rowmap;
  hb.colmap = colmap;
  hb.rho = rho;
}

class PoisProblem : public ProblemImpl {
 public:
  PoisProblem(int N, int max_systems, hipStream_t s) {
    stream = s;
    SPS_REQUIRE(N >= 8 && N <= 256, "nz must be in [8, 256]");
    SPS_REQUIRE(max_systems >= 1 && max_systems <= 4096, "max_systems must be in [1, 4096]");
    PoisBands hb;
    pois_bands(N, hb);
    maxsys_ = max_systems;
    dv_.N = N;
    dv_.S = hb.S;
    dv_.kl = hb.kl;
    dv_.ku = hb.ku;
    dv_.bw = hb.kl + hb.ku + 1;
    dv_.ldw = 2 * hb.kl + hb.ku + 1;
    SPS_REQUIRE(hb.kl + 1 <= 32 && hb.kl + hb.ku < 64, "band too wide for the one-wave solves");
    const cplx** dst[5] = {&dv_.bM, &dv_.bL0, &dv_.bLa, &dv_.bLn, &dv_.bLq};
    for (int t = 0; t < 5; ++t) *dst[t] = arena_.upload(hb.parts[t], stream);
    std::vector<int> colinv(hb.S);
    for (int j = 0; j < hb.S; ++j) colinv[hb.colmap[j]] = j;
    dv_.rowmap = arena_.upload(hb.rowmap, stream);
    dv_.colinv = arena_.upload(colinv, stream);
    dv_.rho = arena_.upload(hb.rho, stream);
    dv_.W = arena_.alloc<cplx>((size_t)maxsys_ * hb.S * dv_.ldw);
    dv_.dinv = arena_.alloc<cplx>((size_t)maxsys_ * hb.S);
    dv_.piv = arena_.alloc<int>((size_t)maxsys_ * hb.S);
    dv_.err = arena_.alloc<int>(1);
    params_ = arena_.alloc<double>((size_t)5 * maxsys_);
    SPS_HIP(hipMemsetAsync(dv_.err, 0, sizeof(int), stream));
    const size_t lds = lds_bytes();
    SPS_REQUIRE(lds <= 160 * 1024, "problem too large for LDS");
    SPS_HIP(hipFuncSetAttribute((const void*)pois_evp, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    SPS_HIP(hipStreamSynchronize(stream));
  }
  size_t lds_bytes() const {
    return sizeof(double) * 8 * (size_t)dv_.S + sizeof(cplx) * 32 + sizeof(double) * 2 * 3 * (PT / 64);
  }

  void run(int nsys, const double* params, int iters, int mode, double tol, int maxit, double* lam, double* dlam,
           double* info, double* X, double* Y) {
    SPS_REQUIRE(nsys >= 1 && nsys <= maxsys_, "nsys must be in [1, max_systems]");
    SPS_REQUIRE(params && lam && dlam && info, "null argument");
    SPS_REQUIRE(iters >= 1 && iters <= 10000, "iters must be in [1, 10000]");
    SPS_REQUIRE(mode >= 0 && mode <= 3, "mode must be 0, 1, 2 or 3");
    SPS_REQUIRE(maxit >= 1 && maxit <= 1000, "maxit must be in [1, 1000]");
    SPS_REQUIRE(std::isfinite(tol) && tol >= 0.0, "tol must be finite and >= 0");
    for (int s = 0; s < nsys; ++s) {
      const double* p = params + 5 * s;
      SPS_REQUIRE(std::isfinite(p[0]) && p[0] > 0.0, "alpha must be positive");
      SPS_REQUIRE(std::isfinite(p[1]) && p[1] > 0.0, "Re must be positive");
      SPS_REQUIRE(std::isfinite(p[2]) && std::isfinite(p[3]), "the shift must be finite");
      SPS_REQUIRE(std::isfinite(p[4]), "the continuation step must be finite");
    }
    SPS_HIP(hipMemcpyAsync(params_, params, sizeof(double) * 5 * nsys, hipMemcpyHostToDevice, stream));
    PoisArgs a{params_, iters, mode, maxit, tol, reinterpret_cast<cplx*>(lam), reinterpret_cast<cplx*>(dlam), info,
               reinterpret_cast<cplx*>(X), reinterpret_cast<cplx*>(Y)};
    hipLaunchKernelGGL(pois_evp, dim3(nsys), dim3(PT), lds_bytes(), stream, dv_, a);
    SPS_CHECK_LAUNCH();
    // the host parameters are copied before the call returns
    SPS_HIP(hipStreamSynchronize(stream));
  }

  long long state_size() const override { return 2LL * dv_.S; }
  void factor() override {}
  void step(double*, int) override { unsupported(); }
  void adjoint_step(double*, int) override { unsupported(); }
  void cost(const double*, double*, double*) override { unsupported(); }
  void gradient(const double*, int, const double*, double*, double*, double*, double*) override { unsupported(); }
  void initial_state(const double*, double*) override { unsupported(); }
  void initial_state_adjoint(const double*, double*) override { unsupported(); }
  void eval_F(const double*, double*) override { unsupported(); }
  void eval_F_vjp(const double*, const double*, double*) override { unsupported(); }
  void solve(const double*, double*, int) override { unsupported(); }
  void timer_enable(int, bool) override {}
  void timer_read(long long* l, double* ms) override {
    *l = 0;
    *ms = 0.0;
  }
  int device_error() override {
    int h = 0;
    SPS_HIP(hipMemcpyAsync(&h, dv_.err, sizeof(int), hipMemcpyDeviceToHost, stream));
    SPS_HIP(hipStreamSynchronize(stream));
    if (h) SPS_HIP(hipMemsetAsync(dv_.err, 0, sizeof(int), stream));
    return h;
  }

 private:
  [[noreturn]] static void unsupported() {
    throw Error(SPS_E_UNSUPPORTED, "the plane Poiseuille handle runs the stability problem only");
  }
  DevArena arena_;
  PoisDev dv_{};
  double* params_ = nullptr;
  int maxsys_ = 1;
};

}  // namespace

ProblemImpl* make_poiseuille(int nz, int max_systems, hipStream_t s) { return new PoisProblem(nz, max_systems, s); }

void poiseuille_run(ProblemImpl* p, int nsys, const double* params, int iters, int mode, double tol, int maxit,
                    double* lam, double* dlam, double* info, double* X, double* Y) {
  auto* q = dynamic_cast<PoisProblem*>(p);
  if (!q) throw Error(SPS_E_ARG, "not a plane Poiseuille handle");
  q->run(nsys, params, iters, mode, tol, maxit, lam, dlam, info, X, Y);
}

void poiseuille_host_band(int nz, double alpha, double re, double sig_re, double sig_im, int* S, int* kl, int* ku,
                          double* band, int* rowmap, int* colmap, double* rho) {
  SPS_REQUIRE(nz >= 8 && nz <= 256, "nz must be in [8, 256]");
  PoisBands hb;
  pois_bands(nz, hb);
  *S = hb.S;
  *kl = hb.kl;
  *ku = hb.ku;
  const double nu = 1.0 / re, q2 = nu * alpha * alpha;
  if (band) {
    const size_t cnt = (size_t)hb.S * (hb.kl + hb.ku + 1);
    for (size_t e = 0; e < cnt; ++e) {
      const double2 m = hb.parts[0][e], l0 = hb.parts[1][e], la = hb.parts[2][e], ln = hb.parts[3][e],
                    lq = hb.parts[4][e];
      band[2 * e] = sig_re * m.x - sig_im * m.y + l0.x + alpha * la.x + nu * ln.x + q2 * lq.x;
      band[2 * e + 1] = sig_re * m.y + sig_im * m.x + l0.y + alpha * la.y + nu * ln.y + q2 * lq.y;
    }
  }
  if (rowmap) std::copy(hb.rowmap.begin(), hb.rowmap.end(), rowmap);
  if (colmap) std::copy(hb.colmap.begin(), hb.colmap.end(), colmap);
  if (rho) std::copy(hb.rho.begin(), hb.rho.end(), rho);
}

}  // namespace sps
