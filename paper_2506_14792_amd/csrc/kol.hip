// 2D Kolmogorov flow in vorticity form on the periodic square [0, 2 pi)^2, a batch of
// independent runs of one size, optionally with a learned closure in the explicit term:
//   omega_t + u . grad omega = nu Laplacian omega - drag omega + f (+ C_theta(omega)),
//   u = (d_y psi, -d_x psi), Laplacian psi = -omega, nu = 1/Re, f = -4 cos 4y.
// IVP form (Supplementary, "Initial value problems"): M = 1, L_k = nu |k|^2 + drag, F = -u.grad omega
// + f (+ closure), the advection formed on the 3/2-padded grid; SBDF2 with an SBDF1 first step
// (equ:imex) and the multistep adjoint recurrence (equ:IMEX_adjoint) with injected cotangents
// of a rollout loss and the closure-parameter gradient (equ:efficient_gradient).
//
// Modes and layouts as the Swift-Hohenberg problem: per instance X[m][iy] (m < N/2 the k_x
// index, iy < N the k_y index in FFT order, iy = N/2 unused), k = integer indices on 2 pi.
// A step is a sequence of launches: column inverse y-FFTs of the fields an evaluation needs
// (u, v, omega_x, omega_y on the 3/2 grid; omega on the N grid for the closure), row x-FFTs
// with the product (or its VJP), the closure network on the N x N vorticity, and a column
// pass with the forward y-FFTs, F and the diagonal solve (or the adjoint combination).
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <memory>
#include <vector>

#include "cnn.h"
#include "sps_device.h"
#include "sps_internal.h"

namespace sps {
namespace {

constexpr int NTK = 256;
constexpr size_t kLdsMax = 160 * 1024;
constexpr size_t kLdsBudget = 80 * 1024;

struct KolDev {
  int B, N, Nh, Ng;
  double nu, drag, dt;
  int pN, pNg;              // FFT plans of lengths N and Ng
  const FftPlan* plans;
  const cplx* tw;
  const int* twoff;
};

__device__ __forceinline__ int kol_pad_row(int iy, int N, int G) {
  if (iy < N / 2) return iy;
  if (iy == N / 2) return -1;
  return iy - N + G;
}
__device__ __forceinline__ double kol_ky(int iy, int N) { return (iy < N / 2) ? (double)iy : (double)(iy - N); }

struct SbdfC {
  double a0, a1, a2, c1, c2;
};
__device__ __forceinline__ SbdfC sbdf_c(int n, double dt) {
  if (n == 1) return {1.0 / dt, -1.0 / dt, 0.0, 1.0, 0.0};
  return {1.5 / dt, -2.0 / dt, 0.5 / dt, 2.0, -1.0};
}

// spectral factor of derived field f of the vorticity at mode (m, iy): 0 u = i ky/|k|^2,
// 1 v = -i kx/|k|^2, 2 omega_x = i kx, 3 omega_y = i ky; ONE = 1
enum FieldSet { FS_PRIMAL4 = 0, FS_ONE = 1 };
__device__ __forceinline__ cplx field_factor(int f, int m, int iy, int N) {
  const double kx = m, ky = kol_ky(iy, N), k2 = kx * kx + ky * ky;
  const double ik2 = (k2 > 0.0) ? 1.0 / k2 : 0.0;
  switch (f) {
    case 0: return cmk(0.0, ky * ik2);
    case 1: return cmk(0.0, -kx * ik2);
    case 2: return cmk(0.0, kx);
    default: return cmk(0.0, ky);
  }
}

// ---------------------------------------------------------------------------- column inverse
// Z[b][f][y][m] = sum_iy factor_f X[b][m][iy] e^{i k_y y} on a G-point grid, for the tile's
// columns m = c0 .. c0 + tc - 1 and field f = blockIdx.y (of gridDim.y fields).
// Grid (column tiles, fields, instances); LDS twiddles(G) + 2 fpad_size(tc G).
__global__ void __launch_bounds__(NTK) kol_cols_inv(KolDev d, const cplx* X, int set, int G, int plan, int tc,
                                                     cplx* Z) {
  extern __shared__ double smem_d[];
  const int b = blockIdx.z, f = blockIdx.y, nf = gridDim.y, c0 = blockIdx.x * tc, N = d.N, Nh = d.Nh;
  const int tid = threadIdx.x;
  if (c0 >= Nh) return;
  const int tcn = min(tc, Nh - c0);
  cplx* tw = reinterpret_cast<cplx*>(smem_d);
  cplx* b0 = tw + G;
  cplx* b1 = b0 + fpad_size(tc * G);
  const cplx* g = d.tw + d.twoff[plan];
  for (int e = tid; e < G; e += NTK) tw[e] = g[e];
  for (int e = tid; e < tcn * G; e += NTK) b0[fpad(e)] = czero();
  __syncthreads();
  const cplx* Xb = X + (long long)b * Nh * N;
  for (int e = tid; e < tcn * N; e += NTK) {
    const int j = e / N, iy = e - j * N, m = c0 + j;
    const int row = kol_pad_row(iy, N, G);
    if (row < 0) continue;
    cplx v = Xb[(long long)m * N + iy];
    if (set == FS_PRIMAL4) v = cmul(v, field_factor(f, m, iy, N));
    b0[fpad(j * G + row)] = v;
  }
  __syncthreads();
  const cplx* o = lds_fft_inline(b0, b1, d.plans[plan], tw, +1, tcn, G, tid, NTK);
  cplx* Zb = Z + ((long long)b * nf + f) * G * Nh + c0;
  for (int e = tid; e < tcn * G; e += NTK) {
    const int y = e / tcn, j = e - y * tcn;
    Zb[(long long)y * Nh + j] = o[fpad(j * G + y)];
  }
}

// ---------------------------------------------------------------------------- rows
// Hermitian packing of two half spectra (rows y, y+1 of one field) into one length-G spectrum
// whose inverse DFT is row_y + i row_(y+1); modes m >= 1 scaled by `scale`.
__device__ __forceinline__ cplx kol_pack(const cplx* U, const cplx* V, int x, int G, int K, double scale) {
  if (x == 0) return cmk(U[0].x, V[0].x);
  if (x < K) return cscale(cmk(U[x].x - V[x].y, U[x].y + V[x].x), scale);
  if (x > G - K) {
    const int q = G - x;
    return cscale(cmk(U[q].x + V[q].y, V[q].x - U[q].y), scale);
  }
  return czero();
}
enum RowMode { R_ADV, R_ADV_VJP, R_GRID, R_FWD_GRID };

// One block per row pair (y, y + 1) of one instance on a G-point grid; y-major field layouts
// Z[b][f][y][m] in and W[b][f][y][m] out.
//  R_ADV:      Z4 (u, v, omega_x, omega_y) -> W = r2c(-(u omega_x + v omega_y))
//  R_ADV_VJP:  Z4 and Zg (the F cotangent, weight-1 modes) -> W4 = r2c of
//              (-qb omega_x, -qb omega_y, -qb u, -qb v), qb = grid cotangent / G^2
//  R_GRID:     Z (one field, modes m >= 1 scaled by `wscale`) -> grid[b][y][x] * gscale
//  R_FWD_GRID: grid[b][y][x] -> W = r2c(grid)
// LDS twiddles(G) + 2 cap, cap >= fpad_size(5 G) when R_ADV_VJP runs, else fpad_size(4 G).
template <int NT>
__global__ void __launch_bounds__(NT) kol_rows(KolDev d, int mode, int G, int plan, int cap, const cplx* Z4,
                                                 const cplx* Zg, double* grid, const double* gin, cplx* W,
                                                 double wscale, double gscale) {
  extern __shared__ double smem_d[];
  const int b = blockIdx.y, y0 = 2 * blockIdx.x, Nh = d.Nh, tid = threadIdx.x;
  const int nin = (mode == R_ADV) ? 4 : (mode == R_ADV_VJP ? 5 : 1);
  const int nout = (mode == R_ADV_VJP) ? 4 : 1;
  cplx* tw = reinterpret_cast<cplx*>(smem_d);
  cplx* b0 = tw + G;
  cplx* b1 = b0 + cap;
  const cplx* g = d.tw + d.twoff[plan];
  for (int e = tid; e < G; e += NT) tw[e] = g[e];
  if (mode == R_FWD_GRID) {
    const double* r0 = gin + ((long long)b * G + y0) * G;
    for (int x = tid; x < G; x += NT) b0[fpad(x)] = cmk(r0[x], r0[G + x]);
  } else {
    const int nz = (mode == R_GRID) ? 1 : 4;
    for (int e = tid; e < nin * G; e += NT) {
      const int f = e / G, x = e - f * G;
      const cplx* U = (f == 4) ? Zg + ((long long)b * G + y0) * Nh : Z4 + (((long long)b * nz + f) * G + y0) * Nh;
      const double sc = (mode == R_GRID) ? wscale : (f == 4 ? 0.5 : 1.0);
      b0[fpad(e)] = kol_pack(U, U + Nh, x, G, Nh, sc);
    }
  }
  __syncthreads();
  const FftPlan& P = d.plans[plan];
  cplx* h = (mode == R_FWD_GRID) ? b0 : lds_fft_inline(b0, b1, P, tw, +1, nin, G, tid, NT);
  if (mode == R_GRID) {
    double* r0 = grid + ((long long)b * G + y0) * G;
    for (int x = tid; x < G; x += NT) {
      const cplx v = h[fpad(x)];
      r0[x] = v.x * gscale;
      r0[G + x] = v.y * gscale;
    }
    return;
  }
  cplx* o = h;
  if (mode != R_FWD_GRID) {
    o = (h == b0) ? b1 : b0;
    const double inv2 = 1.0 / ((double)G * G);
    for (int x = tid; x < G; x += NT) {
      const cplx u = h[fpad(x)], v = h[fpad(G + x)], wx = h[fpad(2 * G + x)], wy = h[fpad(3 * G + x)];
      if (mode == R_ADV) {
        o[fpad(x)] = cmk(-(u.x * wx.x + v.x * wy.x), -(u.y * wx.y + v.y * wy.y));
      } else {
        const cplx q = h[fpad(4 * G + x)];
        const double qa = -q.x * inv2, qb = -q.y * inv2;
        o[fpad(x)] = cmk(qa * wx.x, qb * wx.y);           // u bar
        o[fpad(G + x)] = cmk(qa * wy.x, qb * wy.y);       // v bar
        o[fpad(2 * G + x)] = cmk(qa * u.x, qb * u.y);     // omega_x bar
        o[fpad(3 * G + x)] = cmk(qa * v.x, qb * v.y);     // omega_y bar
      }
    }
    __syncthreads();
  }
  cplx* o2 = (o == b0) ? b1 : b0;
  const cplx* r = lds_fft_inline(o, o2, P, tw, -1, nout, G, tid, NT);
  // unpack the two real rows' half spectra: Y_y = (Z_m + conj Z_-m) / 2, Y_y+1 = (Z_m - conj Z_-m) / 2i
  for (int e = tid; e < nout * 2 * Nh; e += NT) {
    const int f = e / (2 * Nh), rr = e - f * 2 * Nh, yy = rr / Nh, m = rr - yy * Nh;
    const cplx zm = r[fpad(f * G + m)], zq = r[fpad(f * G + (m == 0 ? 0 : G - m))];
    const cplx v = yy ? cmk(0.5 * (zm.y + zq.y), -0.5 * (zm.x - zq.x)) : cmk(0.5 * (zm.x + zq.x), 0.5 * (zm.y - zq.y));
    W[(((long long)b * nout + f) * G + y0 + yy) * Nh + m] = v;
  }
}

// The advection product of one row pair in two passes of two fields each (u, omega_x, then
// v, omega_y), so that long rows fit two blocks per CU: LDS twiddles(G) + 2 fpad_size(2 G) +
// fpad_size(G).  Same result as kol_rows in mode R_ADV up to the order of the two products.
template <int NT>
__global__ void __launch_bounds__(NT) kol_rows_adv2(KolDev d, int G, int plan, const cplx* Z4, cplx* W) {
  extern __shared__ double smem_d[];
  const int b = blockIdx.y, y0 = 2 * blockIdx.x, Nh = d.Nh, tid = threadIdx.x;
  cplx* tw = reinterpret_cast<cplx*>(smem_d);
  cplx* b0 = tw + G;
  cplx* b1 = b0 + fpad_size(2 * G);
  cplx* pr = b1 + fpad_size(2 * G);
  const cplx* g = d.tw + d.twoff[plan];
  for (int e = tid; e < G; e += NT) tw[e] = g[e];
  const FftPlan& P = d.plans[plan];
  for (int pass = 0; pass < 2; ++pass) {
    // pass 0: fields 0 (u) and 2 (omega_x); pass 1: fields 1 (v) and 3 (omega_y)
    for (int e = tid; e < 2 * G; e += NT) {
      const int q = e / G, x = e - q * G, f = pass + 2 * q;
      const cplx* U = Z4 + (((long long)b * 4 + f) * G + y0) * Nh;
      b0[fpad(e)] = kol_pack(U, U + Nh, x, G, Nh, 1.0);
    }
    __syncthreads();
    const cplx* h = lds_fft_inline(b0, b1, P, tw, +1, 2, G, tid, NT);
    for (int x = tid; x < G; x += NT) {
      const cplx a = h[fpad(x)], c = h[fpad(G + x)];
      const cplx p = cmk(-(a.x * c.x), -(a.y * c.y));
      pr[fpad(x)] = pass ? cmk(pr[fpad(x)].x + p.x, pr[fpad(x)].y + p.y) : p;
    }
    __syncthreads();
  }
  const cplx* r = lds_fft_inline(pr, b0, P, tw, -1, 1, G, tid, NT);
  for (int e = tid; e < 2 * Nh; e += NT) {
    const int yy = e / Nh, m = e - yy * Nh;
    const cplx zm = r[fpad(m)], zq = r[fpad(m == 0 ? 0 : G - m)];
    const cplx v = yy ? cmk(0.5 * (zm.y + zq.y), -0.5 * (zm.x - zq.x)) : cmk(0.5 * (zm.x + zq.x), 0.5 * (zm.y - zq.y));
    W[((long long)b * G + y0 + yy) * Nh + m] = v;
  }
}

// ---------------------------------------------------------------------------- column pass
enum ColMode { K_STEP, K_EVALF, K_ADJ, K_ADJ_INIT, K_VJP };
struct KolCol {
  int mode, n, nsteps, closure;
  const cplx* W;     // [B][nW][Nh][Ng] products' x-spectra (1 field, or 4 for the VJP)
  const cplx* Wc;    // [B][Nh][N] closure x-spectra (nullable)
  cplx* H;           // history [nh][B][Nh][N]
  int hring;         // 0: full history; else ring of hring states
  cplx* Fr;          // F ring [2][B][Nh][N]
  cplx* Yn;          // Y_(k+1) [B][Nh][N]
  cplx* Ln;          // linear part
  cplx* Gk;          // F cotangent for the next VJP
  const cplx* targ;  // rollout targets [nsteps][B][Nh][N] (nullable)
  const cplx* xin;   // K_ADJ_INIT: external dJ/dX_N (nullable)
  cplx* out;         // K_EVALF: F; K_VJP: Xbar; K_ADJ (k = 0): dJ/dX_0; K_STEP (n = nsteps): X_N (nullable)
  cplx* snap;        // K_STEP: filtered snapshots (nullable)
  int snap_every, Nc;
  int* err;          // sticky flags: bit 1 non-finite state
};

__device__ __forceinline__ long long hidx(const KolCol& a, int k, long long st) {
  return (long long)(a.hring ? (k % a.hring) : k) * st;
}

// Grid (column tiles, instances).  LDS twiddles(Ng) + twiddles(N) + 2 wcap (wcap >=
// fpad_size(nW tc Ng)) + 2 fpad_size(tc N) when the closure runs.
__global__ void __launch_bounds__(NTK) kol_cols_fwd(KolDev d, KolCol a, int tc, int wcap) {
  extern __shared__ double smem_d[];
  const int b = blockIdx.y, c0 = blockIdx.x * tc, N = d.N, Nh = d.Nh, Ng = d.Ng, tid = threadIdx.x;
  if (c0 >= Nh) return;
  const int tcn = min(tc, Nh - c0);
  const bool adj = (a.mode == K_ADJ || a.mode == K_VJP);
  const int nW = (a.mode == K_ADJ_INIT) ? 0 : (adj ? 4 : 1);
  const bool clo = a.closure && a.mode != K_ADJ_INIT;
  cplx* twg = reinterpret_cast<cplx*>(smem_d);
  cplx* twn = twg + Ng;
  cplx* b0 = twn + N;
  cplx* b1 = b0 + wcap;
  cplx* c0b = b1 + wcap;
  cplx* c1b = c0b + fpad_size(tc * N);
  for (int e = tid; e < Ng; e += NTK) twg[e] = d.tw[d.twoff[d.pNg] + e];
  for (int e = tid; e < N; e += NTK) twn[e] = d.tw[d.twoff[d.pN] + e];
  for (int e = tid; e < nW * Ng * tcn; e += NTK) {
    const int f = e / (Ng * tcn), r = e - f * Ng * tcn, y = r / tcn, j = r - y * tcn;
    b0[fpad((f * tcn + j) * Ng + y)] = a.W[(((long long)b * nW + f) * Ng + y) * Nh + c0 + j];
  }
  if (clo)
    for (int e = tid; e < N * tcn; e += NTK) {
      const int y = e / tcn, j = e - y * tcn;
      c0b[fpad(j * N + y)] = a.Wc[((long long)b * N + y) * Nh + c0 + j];
    }
  __syncthreads();
  const cplx* res = (nW > 0) ? lds_fft_inline(b0, b1, d.plans[d.pNg], twg, -1, nW * tcn, Ng, tid, NTK) : nullptr;
  const cplx* rc = clo ? lds_fft_inline(c0b, c1b, d.plans[d.pN], twn, -1, tcn, N, tid, NTK) : nullptr;
  const long long st = (long long)d.B * Nh * N, io = (long long)b * Nh * N;
  const double ng2 = 1.0 / ((double)Ng * Ng), n2 = 1.0 / ((double)N * N);
  for (int e = tid; e < tcn * N; e += NTK) {
    const int j = e / N, iy = e - j * N, m = c0 + j;
    const long long si = io + (long long)m * N + iy;
    const int row = kol_pad_row(iy, N, Ng), rowc = kol_pad_row(iy, N, N);
    const double k2 = (double)m * m + kol_ky(iy, N) * kol_ky(iy, N);
    const double lin = d.nu * k2 + d.drag, wm = (m == 0) ? 1.0 : 2.0;
    if (a.mode == K_STEP || a.mode == K_EVALF) {
      cplx F = czero();
      if (row >= 0) {
        F = cscale(res[fpad(j * Ng + row)], ng2);
        if (m == 0 && N > 8 && (iy == 4 || iy == N - 4)) F = cadd(F, cmk(-2.0, 0.0));   // -4 cos 4y
        if (clo) F = cadd(F, cscale(rc[fpad(j * N + rowc)], n2));
      }
      if (a.mode == K_EVALF) {
        a.out[si] = F;
        continue;
      }
      const int n = a.n;
      const SbdfC q = sbdf_c(n, d.dt);
      const cplx f2 = (n >= 2) ? a.Fr[(n & 1) * st + si] : czero();
      const cplx x1 = a.H[hidx(a, n - 1, st) + si];
      const cplx x2 = (n >= 2) ? a.H[hidx(a, n - 2, st) + si] : czero();
      cplx xn = czero();
      if (row >= 0) {
        cplx rhs = cadd(cscale(F, q.c1), cscale(f2, q.c2));
        rhs = csub(rhs, cadd(cscale(x1, q.a1), cscale(x2, q.a2)));
        xn = cscale(rhs, 1.0 / (q.a0 + lin));
      }
      a.Fr[((n - 1) & 1) * st + si] = F;
      a.H[hidx(a, n, st) + si] = xn;
      if (!(isfinite(xn.x) && isfinite(xn.y))) atomicOr(a.err, 2);
      if (n == a.nsteps && a.out) a.out[si] = xn;
      if (a.snap && n % a.snap_every == 0) {
        // spectral truncation to the Nc x Nc modes of the coarse grid
        const int Nch = a.Nc / 2;
        const int sy = (iy < N / 2) ? iy : iy - N;
        if (m < Nch && sy >= -Nch && sy < Nch) {   // sy = -Nch: the coarse Nyquist row, kept zero
          const int ic = (sy >= 0) ? sy : sy + a.Nc;
          a.snap[((long long)(n / a.snap_every - 1) * d.B + b) * Nch * a.Nc + (long long)m * a.Nc + ic] =
              (sy == -Nch) ? czero() : xn;
        }
      }
      continue;
    }
    // reverse sweep: xb of state k (K_ADJ: k = n - 1 from the VJP; K_ADJ_INIT: k = nsteps)
    cplx xb = czero();
    if (a.mode == K_ADJ || a.mode == K_VJP) {
      if (row >= 0) {
        for (int f = 0; f < 4; ++f) {
          const cplx t = cscale(res[fpad((f * tcn + j) * Ng + row)], wm);
          const cplx fac = field_factor(f, m, iy, N);
          xb = cadd(xb, cmul(cconj(fac), t));
        }
        if (clo) xb = cadd(xb, cscale(rc[fpad(j * N + rowc)], wm));
      }
      if (a.mode == K_VJP) {
        a.out[si] = xb;
        continue;
      }
      xb = csub(xb, a.Ln[si]);
    } else if (a.xin && row >= 0) {
      xb = a.xin[si];
    }
    const int k = (a.mode == K_ADJ) ? a.n - 1 : a.nsteps;
    if (a.targ && k >= 1 && row >= 0) {
      // d/dX_k of (1/nsteps) mean over the N x N grid of (omega_k - target_k)^2
      const cplx* T = a.targ + (long long)(k - 1) * st;
      cplx e1 = csub(a.H[hidx(a, k, st) + si], T[si]);
      if (m == 0) {
        const long long sm = io + (long long)((N - iy) % N);
        const cplx e2 = csub(a.H[hidx(a, k, st) + sm], T[sm]);
        e1 = cmk(0.5 * (e1.x + e2.x), 0.5 * (e1.y - e2.y));
      }
      xb = cadd(xb, cscale(e1, 2.0 * wm / a.nsteps));
    }
    if (k == 0) {
      a.out[si] = xb;
      continue;
    }
    cplx y = czero(), g = czero(), l = czero();
    if (row >= 0) {
      const SbdfC q = sbdf_c(k, d.dt);
      y = cscale(xb, 1.0 / (q.a0 + lin));
      g = cscale(y, q.c1);
      l = cscale(y, q.a1);
      if (k + 1 <= a.nsteps) {
        const SbdfC qn = sbdf_c(k + 1, d.dt);
        g = cadd(g, cscale(a.Yn[si], qn.c2));
        l = cadd(l, cscale(a.Yn[si], qn.a2));
      }
    }
    a.Yn[si] = y;
    a.Ln[si] = l;
    a.Gk[si] = g;
  }
}

// rollout loss per instance: (1/nsteps) sum_k sum_modes w |canon(X_k - T_k)|^2 (= mean over the
// N x N grid of the squared difference); one block per instance
__global__ void __launch_bounds__(NTK) kol_loss(KolDev d, const cplx* H, const cplx* T, int nsteps, double* J) {
  __shared__ double red[NTK];
  const int b = blockIdx.x, N = d.N, Nh = d.Nh, tid = threadIdx.x;
  const long long st = (long long)d.B * Nh * N, io = (long long)b * Nh * N;
  double s = 0.0;
  for (int k = 1; k <= nsteps; ++k)
    for (int e = tid; e < Nh * N; e += NTK) {
      const int m = e / N, iy = e - m * N;
      if (iy == N / 2) continue;
      cplx c = csub(H[(long long)k * st + io + e], T[(long long)(k - 1) * st + io + e]);
      if (m == 0) {
        const long long sm = io + (N - iy) % N;
        const cplx c2 = csub(H[(long long)k * st + sm], T[(long long)(k - 1) * st + sm]);
        c = cmk(0.5 * (c.x + c2.x), 0.5 * (c.y - c2.y));
      }
      s += ((m == 0) ? 1.0 : 2.0) * (c.x * c.x + c.y * c.y);
    }
  red[tid] = s;
  __syncthreads();
  for (int w = NTK / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  if (tid == 0) J[b] = red[0] / nsteps;
}

// Adam update of the closure parameters (theta, first and second moments in FP64)
__global__ void kol_adam(int n, double* th, const double* g, double* m1, double* m2, double lr, double b1, double b2,
                         double eps, int t) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  m1[i] = b1 * m1[i] + (1.0 - b1) * g[i];
  m2[i] = b2 * m2[i] + (1.0 - b2) * g[i] * g[i];
  const double mh = m1[i] / (1.0 - pow(b1, t)), vh = m2[i] / (1.0 - pow(b2, t));
  th[i] -= lr * mh / (sqrt(vh) + eps);
}

// ---------------------------------------------------------------------------- host
class KolProblem : public ProblemImpl {
 public:
  KolProblem(int batch, int N, double Re, double drag, double dt, int max_steps, int closure, int keep_history,
             hipStream_t s) {
    stream = s;
    SPS_REQUIRE(batch >= 1 && N >= 8 && N % 4 == 0 && N <= 1024, "need batch >= 1 and N a multiple of 4 in [8, 1024]");
    SPS_REQUIRE(Re > 0 && drag >= 0 && dt > 0 && max_steps >= 1, "bad Re / drag / dt / max_steps");
    SPS_REQUIRE(!closure || N % 32 == 0, "the closure needs N a multiple of 32");
    B_ = batch;
    N_ = N;
    Nh_ = N / 2;
    Ng_ = 3 * N / 2;
    max_steps_ = max_steps;
    closure_ = closure;
    hring_ = keep_history ? 0 : 3;
    FftPlan pn{}, png{};
    SPS_REQUIRE(fft_plan(N, &pn) && fft_plan(Ng_, &png), "N and 3N/2 must factor into 2 and 3");
    std::vector<FftPlan> plans = {pn, png};
    std::vector<double2> tw = twiddles(N);
    const auto tg = twiddles(Ng_);
    std::vector<int> off = {0, (int)tw.size()};
    tw.insert(tw.end(), tg.begin(), tg.end());
    d_.B = B_;
    d_.N = N;
    d_.Nh = Nh_;
    d_.Ng = Ng_;
    d_.nu = 1.0 / Re;
    d_.drag = drag;
    d_.dt = dt;
    d_.pN = 0;
    d_.pNg = 1;
    d_.plans = arena_.upload(plans, stream);
    d_.tw = arena_.upload(tw, stream);
    d_.twoff = arena_.upload(off, stream);
    st_ = (long long)B_ * Nh_ * N_;
    err_ = arena_.alloc<int>(1);
    SPS_HIP(hipMemsetAsync(err_, 0, sizeof(int), stream));
    const int nh = keep_history ? max_steps + 1 : 3;
    H_ = arena_.alloc<cplx>((size_t)nh * st_);
    Fr_ = arena_.alloc<cplx>(2 * st_);
    Yn_ = arena_.alloc<cplx>(st_);
    Ln_ = arena_.alloc<cplx>(st_);
    Gk_ = arena_.alloc<cplx>(st_);
    Xw_ = arena_.alloc<cplx>(st_);
    Z4_ = arena_.alloc<cplx>((size_t)B_ * 4 * Nh_ * Ng_);
    Zg_ = arena_.alloc<cplx>((size_t)B_ * Nh_ * Ng_);
    W_ = arena_.alloc<cplx>((size_t)B_ * 4 * Nh_ * Ng_);
    if (closure_) {
      net_.reset(new Cnn(B_, N_, N_, stream));
      Zc_ = arena_.alloc<cplx>(st_);
      Zgc_ = arena_.alloc<cplx>(st_);
      Wc_ = arena_.alloc<cplx>(st_);
      og_ = arena_.alloc<double>((size_t)B_ * N_ * N_);
      yg_ = arena_.alloc<double>((size_t)B_ * N_ * N_);
      xg_ = arena_.alloc<double>((size_t)B_ * N_ * N_);
      theta_ = arena_.alloc<double>(Cnn::nparam());
      SPS_HIP(hipMemsetAsync(theta_, 0, sizeof(double) * Cnn::nparam(), stream));
      net_->set_params(theta_);
    }
    // tiles: the widest (up to 8 columns) whose LDS stays within kLdsBudget, so that two
    // blocks fit on a CU; row buffers sized for the widest row mode this problem runs
    nwmax_ = keep_history ? 4 : 1;
    tc_ig_ = pick_tile([&](int tc) { return inv_lds(Ng_, tc); });
    tc_in_ = pick_tile([&](int tc) { return inv_lds(N_, tc); });
    tc_f_ = pick_tile([&](int tc) { return fwd_lds(tc); });
    rcap_ = fpad_size((keep_history ? 5 : 4) * Ng_);
    const size_t rl = sizeof(cplx) * (Ng_ + 2 * (size_t)rcap_);
    const size_t il = std::max(inv_lds(Ng_, tc_ig_), inv_lds(N_, tc_in_));
    SPS_REQUIRE(rl <= kLdsMax && il <= kLdsMax && fwd_lds(tc_f_) <= kLdsMax, "size too large for the Kolmogorov kernels");
    for (const void* k : {(const void*)kol_cols_inv, (const void*)kol_rows<256>, (const void*)kol_rows<512>,
                          (const void*)kol_rows_adv2<512>, (const void*)kol_cols_fwd})
      SPS_HIP(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsMax));
    SPS_HIP(hipStreamSynchronize(stream));
  }

  long long state_size() const override { return 2 * st_; }
  // a new step for the following runs: the SBDF2 coefficients take it (diagonal implicit
  // operator); drops the recorded run
  void set_dt(double dt) override {
    SPS_REQUIRE(std::isfinite(dt) && dt > 0.0, "dt must be positive");
    d_.dt = dt;
    tape_ = -1;
  }
  void factor() override {}

  void set_params(const double* theta) {
    SPS_REQUIRE(closure_, "this problem has no closure");
    SPS_HIP(hipMemcpyAsync(theta_, theta, sizeof(double) * Cnn::nparam(), hipMemcpyDeviceToDevice, stream));
    net_->set_params(theta_);
  }

  // forward sweep from X0 (state layout); XN (nullable); snapshots of the run truncated to
  // Nc x Nc modes every `every` steps (nullable)
  void forward(const cplx* X0, int nsteps, cplx* XN, cplx* snap, int every, int Nc) {
    SPS_REQUIRE(X0 && nsteps >= 1, "forward: null state or nsteps < 1");
    SPS_REQUIRE(hring_ || nsteps <= max_steps_, "forward: nsteps exceeds the history the problem was built for");
    SPS_REQUIRE(!snap || (every >= 1 && Nc >= 4 && Nc % 2 == 0 && Nc <= N_), "forward: bad snapshot arguments");
    if (!snap) every = 1;
    SPS_HIP(hipMemcpyAsync(H_, X0, sizeof(cplx) * st_, hipMemcpyDeviceToDevice, stream));
    for (int n = 1; n <= nsteps; ++n) {
      const cplx* Xp = H_ + hslot(n - 1) * st_;
      eval_products(Xp);
      KolCol a = col_args(K_STEP, n, nsteps);
      a.out = XN;
      a.snap = snap;
      a.snap_every = every;
      a.Nc = Nc;
      launch_cols(a);
    }
    tape_ = nsteps;
  }

  // reverse sweep: dJ/dX_0 of the rollout loss against targets (nullable) plus an external
  // dJ/dX_N (nullable); closure-parameter gradient added to th_bar (nullable)
  void reverse(const cplx* targets, const cplx* xbN, int nsteps, cplx* xb0, double* th_bar) {
    SPS_REQUIRE(hring_ == 0, "the reverse sweep needs the full history");
    SPS_REQUIRE(tape_ == nsteps, "reverse: nsteps does not match the recorded forward run");
    KolCol a = col_args(K_ADJ_INIT, nsteps, nsteps);
    a.targ = targets;
    a.xin = xbN;
    a.out = xb0;
    launch_cols(a);
    // the closure-parameter cotangent of every step is summed in the network's accumulators
    // and added to th_bar once at the end of the sweep
    const bool acc = closure_ && th_bar;
    if (acc) net_->grad_reset();
    for (int n = nsteps; n >= 1; --n) {
      const cplx* Xp = H_ + (long long)(n - 1) * st_;
      eval_vjp(Xp, Gk_, acc ? ACC_THETA : NO_THETA, nullptr);
      KolCol c = col_args(K_ADJ, n, nsteps);
      c.targ = targets;
      c.out = xb0;
      launch_cols(c);
    }
    if (acc) net_->grad_flush(th_bar);
  }

  // forward run from X0, the rollout loss J[b] against targets and its gradients: dJdX0
  // (state layout, nullable) and dJdtheta = sum over instances of dJ[b]/dtheta (nullable;
  // needs the closure)
  void rollout(const cplx* X0, const cplx* targets, int nsteps, cplx* XN, double* J, cplx* dJdX0, double* dJdtheta) {
    SPS_REQUIRE(targets, "rollout: targets are required");
    SPS_REQUIRE(!dJdtheta || closure_, "rollout: dJdtheta needs the closure");
    SPS_REQUIRE(!(dJdX0 || dJdtheta) || hring_ == 0, "rollout gradients need a problem built with keep_history");
    forward(X0, nsteps, XN, nullptr, 1, 0);
    if (J) loss(targets, nsteps, J);
    if (dJdX0 || dJdtheta) {
      if (dJdtheta) SPS_HIP(hipMemsetAsync(dJdtheta, 0, sizeof(double) * Cnn::nparam(), stream));
      reverse(targets, nullptr, nsteps, dJdX0 ? dJdX0 : Xw_, dJdtheta);
    }
  }

  void loss(const cplx* targets, int nsteps, double* J) {
    SPS_REQUIRE(hring_ == 0 && tape_ == nsteps, "loss: needs the full history of the last forward run");
    hipLaunchKernelGGL(kol_loss, dim3(B_), dim3(NTK), 0, stream, d_, H_, targets, nsteps, J);
    SPS_CHECK_LAUNCH();
  }

  // Adam update of the caller's parameter vector theta, which then becomes the problem's
  void adam(double* theta, const double* grad, double* m1, double* m2, double lr, int t) {
    SPS_REQUIRE(closure_, "this problem has no closure");
    const int n = Cnn::nparam();
    hipLaunchKernelGGL(kol_adam, dim3((n + 255) / 256), dim3(256), 0, stream, n, theta, grad, m1, m2, lr, 0.9, 0.999,
                       1e-8, t);
    SPS_CHECK_LAUNCH();
    set_params(theta);
  }

  // ProblemImpl
  void step(double* X, int nsteps) override {
    SPS_REQUIRE(X && nsteps >= 1 && nsteps <= max_steps_, "bad step arguments");
    forward(reinterpret_cast<const cplx*>(X), nsteps, reinterpret_cast<cplx*>(X), nullptr, 1, 0);
  }
  void adjoint_step(double* Xbar, int nsteps) override {
    SPS_REQUIRE(Xbar, "Xbar is null");
    if (tape_ != nsteps) throw Error(SPS_E_STATE, "adjoint_step: nsteps does not match the recorded forward run");
    SPS_HIP(hipMemcpyAsync(Xw_, Xbar, sizeof(cplx) * st_, hipMemcpyDeviceToDevice, stream));
    reverse(nullptr, Xw_, nsteps, reinterpret_cast<cplx*>(Xbar), nullptr);
  }
  void cost(const double*, double*, double*) override {
    throw Error(SPS_E_UNSUPPORTED, "the Kolmogorov problem's objective is the rollout loss");
  }
  void gradient(const double*, int, const double*, double*, double*, double*, double*) override {
    throw Error(SPS_E_UNSUPPORTED, "use the rollout call of the Kolmogorov problem");
  }
  void initial_state(const double*, double*) override {
    throw Error(SPS_E_UNSUPPORTED, "Kolmogorov states are given as coefficients");
  }
  void initial_state_adjoint(const double*, double*) override {
    throw Error(SPS_E_UNSUPPORTED, "Kolmogorov states are given as coefficients");
  }
  void eval_F(const double* X, double* F) override {
    eval_products(reinterpret_cast<const cplx*>(X));
    KolCol a = col_args(K_EVALF, 0, 0);
    a.out = reinterpret_cast<cplx*>(F);
    launch_cols(a);
  }
  void eval_F_vjp(const double* X, const double* Fbar, double* Xbar) override {
    eval_vjp(reinterpret_cast<const cplx*>(X), reinterpret_cast<const cplx*>(Fbar), NO_THETA, nullptr);
    KolCol a = col_args(K_VJP, 0, 0);
    a.out = reinterpret_cast<cplx*>(Xbar);
    launch_cols(a);
  }
  void param_vjp(const double* X, const double* Fbar, double* th_bar) {
    SPS_REQUIRE(closure_, "this problem has no closure");
    eval_vjp(reinterpret_cast<const cplx*>(X), reinterpret_cast<const cplx*>(Fbar), ADD_THETA, th_bar);
  }
  void solve(const double*, double*, int) override {
    throw Error(SPS_E_UNSUPPORTED, "the Kolmogorov solve is internal to its steps");
  }
  void timer_enable(int, bool) override {}
  void timer_read(long long* l, double* ms) override {
    *l = 0;
    *ms = 0;
  }
  int device_error() override {
    int h = 0;
    SPS_HIP(hipMemcpyAsync(&h, err_, sizeof(int), hipMemcpyDeviceToHost, stream));
    SPS_HIP(hipStreamSynchronize(stream));
    if (h) SPS_HIP(hipMemsetAsync(err_, 0, sizeof(int), stream));
    return h;
  }

 private:
  long long hslot(int k) const { return hring_ ? k % hring_ : k; }
  size_t inv_lds(int G, int tc) const { return sizeof(cplx) * (G + 2 * (size_t)fpad_size(tc * G)); }
  int wcap(int tc) const { return fpad_size(nwmax_ * tc * Ng_); }
  size_t fwd_lds(int tc) const {
    return sizeof(cplx) * (Ng_ + N_ + 2 * (size_t)wcap(tc) + (closure_ ? 2 * (size_t)fpad_size(tc * N_) : 0));
  }
  template <typename F>
  int pick_tile(F lds) const {
    int tc = 8;
    while (tc > 1 && lds(tc) > kLdsBudget) --tc;
    return tc;
  }
  KolCol col_args(int mode, int n, int nsteps) {
    KolCol a{};
    a.mode = mode;
    a.n = n;
    a.nsteps = nsteps;
    a.closure = closure_;
    a.W = W_;
    a.Wc = Wc_;
    a.H = H_;
    a.hring = hring_;
    a.Fr = Fr_;
    a.Yn = Yn_;
    a.Ln = Ln_;
    a.Gk = Gk_;
    a.err = err_;
    return a;
  }
  void launch_cols(const KolCol& a) {
    hipLaunchKernelGGL(kol_cols_fwd, dim3((Nh_ + tc_f_ - 1) / tc_f_, B_), dim3(NTK), fwd_lds(tc_f_), stream, d_, a,
                       tc_f_, wcap(tc_f_));
    SPS_CHECK_LAUNCH();
  }
  void cols_inv(const cplx* X, int set, int G, int plan, cplx* Z) {
    const int tc = (G == Ng_) ? tc_ig_ : tc_in_;
    const int nf = (set == FS_PRIMAL4) ? 4 : 1;
    hipLaunchKernelGGL(kol_cols_inv, dim3((Nh_ + tc - 1) / tc, nf, B_), dim3(NTK), inv_lds(G, tc), stream, d_, X,
                       set, G, plan, tc, Z);
    SPS_CHECK_LAUNCH();
  }
  void rows(int mode, int G, int plan, const cplx* Z4, const cplx* Zg, double* grid, const double* gin, cplx* W,
            double wscale, double gscale) {
    if (mode == R_ADV && G >= 384) {
      const size_t l2 = sizeof(cplx) * (G + 2 * (size_t)fpad_size(2 * G) + fpad_size(G));
      hipLaunchKernelGGL(kol_rows_adv2<512>, dim3(G / 2, B_), dim3(512), l2, stream, d_, G, plan, Z4, W);
      SPS_CHECK_LAUNCH();
      return;
    }
    // rows of 384 points or more: 512 threads, so that a CU holding one block (LDS) still has
    // eight waves
    const size_t lds = sizeof(cplx) * (G + 2 * (size_t)rcap_);
    if (G >= 384)
      hipLaunchKernelGGL(kol_rows<512>, dim3(G / 2, B_), dim3(512), lds, stream, d_, mode, G, plan, rcap_, Z4, Zg, grid,
                         gin, W, wscale, gscale);
    else
      hipLaunchKernelGGL(kol_rows<256>, dim3(G / 2, B_), dim3(256), lds, stream, d_, mode, G, plan, rcap_, Z4, Zg, grid,
                         gin, W, wscale, gscale);
    SPS_CHECK_LAUNCH();
  }
  // x-spectra of the products of F at X (W) and of the closure output (Wc)
  void eval_products(const cplx* X) {
    cols_inv(X, FS_PRIMAL4, Ng_, d_.pNg, Z4_);
    rows(R_ADV, Ng_, d_.pNg, Z4_, nullptr, nullptr, nullptr, W_, 1.0, 1.0);
    if (closure_) {
      cols_inv(X, FS_ONE, N_, d_.pN, Zc_);
      rows(R_GRID, N_, d_.pN, Zc_, nullptr, og_, nullptr, nullptr, 1.0, 1.0);
      net_->forward(og_, yg_, 1.0, false);
      rows(R_FWD_GRID, N_, d_.pN, nullptr, nullptr, nullptr, yg_, Wc_, 1.0, 1.0);
    }
  }
  // x-spectra of the VJP of F at X with cotangent G (W: 4 fields; Wc).  The closure's parameter
  // cotangent: dropped (NO_THETA), added to th_bar (ADD_THETA) or to the network's accumulators
  // (ACC_THETA).
  enum ThetaMode { NO_THETA, ADD_THETA, ACC_THETA };
  void eval_vjp(const cplx* X, const cplx* G, ThetaMode tm, double* th_bar) {
    SPS_REQUIRE(nwmax_ == 4, "VJPs need a problem built with keep_history");
    cols_inv(X, FS_PRIMAL4, Ng_, d_.pNg, Z4_);
    cols_inv(G, FS_ONE, Ng_, d_.pNg, Zg_);
    rows(R_ADV_VJP, Ng_, d_.pNg, Z4_, Zg_, nullptr, nullptr, W_, 1.0, 1.0);
    if (closure_) {
      cols_inv(X, FS_ONE, N_, d_.pN, Zc_);
      rows(R_GRID, N_, d_.pN, Zc_, nullptr, og_, nullptr, nullptr, 1.0, 1.0);
      cols_inv(G, FS_ONE, N_, d_.pN, Zgc_);
      rows(R_GRID, N_, d_.pN, Zgc_, nullptr, yg_, nullptr, nullptr, 0.5, 1.0 / ((double)N_ * N_));
      if (tm == ACC_THETA)
        net_->vjp_accumulate(og_, yg_, xg_, 1.0, false);
      else
        net_->vjp(og_, yg_, xg_, 1.0, false, tm == ADD_THETA ? th_bar : nullptr);
      rows(R_FWD_GRID, N_, d_.pN, nullptr, nullptr, nullptr, xg_, Wc_, 1.0, 1.0);
    }
  }

  int B_, N_, Nh_, Ng_, max_steps_, closure_, hring_, nwmax_ = 4, tc_ig_ = 1, tc_in_ = 1, tc_f_ = 1, rcap_ = 0;
  int tape_ = -1;
  long long st_ = 0;
  KolDev d_{};
  DevArena arena_;
  std::unique_ptr<Cnn> net_;
  int* err_ = nullptr;
  cplx *H_, *Fr_, *Yn_, *Ln_, *Gk_, *Xw_, *Z4_, *Zg_, *W_, *Zc_ = nullptr, *Zgc_ = nullptr, *Wc_ = nullptr;
  double *og_ = nullptr, *yg_ = nullptr, *xg_ = nullptr, *theta_ = nullptr;
};

}  // namespace

ProblemImpl* make_kolmo(int batch, int N, double Re, double drag, double dt, int max_steps, int closure,
                        int keep_history, hipStream_t s) {
  return new KolProblem(batch, N, Re, drag, dt, max_steps, closure, keep_history, s);
}
void kolmo_set_params(ProblemImpl* p, const double* theta) {
  auto* k = dynamic_cast<KolProblem*>(p);
  if (!k) throw Error(SPS_E_ARG, "not a Kolmogorov problem");
  k->set_params(theta);
}
void kolmo_forward(ProblemImpl* p, const double* X0, int nsteps, double* XN, double* snap, int every, int Nc) {
  auto* k = dynamic_cast<KolProblem*>(p);
  if (!k) throw Error(SPS_E_ARG, "not a Kolmogorov problem");
  k->forward(reinterpret_cast<const cplx*>(X0), nsteps, reinterpret_cast<cplx*>(XN), reinterpret_cast<cplx*>(snap),
             every, Nc);
}
void kolmo_rollout(ProblemImpl* p, const double* X0, const double* targets, int nsteps, double* XN, double* J,
                   double* dJdX0, double* dJdtheta) {
  auto* k = dynamic_cast<KolProblem*>(p);
  if (!k) throw Error(SPS_E_ARG, "not a Kolmogorov problem");
  k->rollout(reinterpret_cast<const cplx*>(X0), reinterpret_cast<const cplx*>(targets), nsteps,
             reinterpret_cast<cplx*>(XN), J, reinterpret_cast<cplx*>(dJdX0), dJdtheta);
}
void kolmo_param_vjp(ProblemImpl* p, const double* X, const double* Fbar, double* th_bar) {
  auto* k = dynamic_cast<KolProblem*>(p);
  if (!k) throw Error(SPS_E_ARG, "not a Kolmogorov problem");
  k->param_vjp(X, Fbar, th_bar);
}
void kolmo_adam(ProblemImpl* p, double* theta, const double* grad, double* m1, double* m2, double lr, int t) {
  auto* k = dynamic_cast<KolProblem*>(p);
  if (!k) throw Error(SPS_E_ARG, "not a Kolmogorov problem");
  k->adam(theta, grad, m1, m2, lr, t);
}

}  // namespace sps
