// 3D plane Couette flow: the (x, z) plane transforms and products of the explicit term, and their
// vector-Jacobian product.  The per-mode Stokes systems (time derivative, viscous term, pressure,
// continuity, walls) are the per-wavenumber systems of rbc.hip with the buoyancy coupling off:
// for a Fourier mode (kx, kz) with kh = |(kx, kz)| > 0 the horizontal velocity is written in the
// frame of the wave vector, u_par = (kx u + kz w)/kh, u_perp = (-kz u + kx w)/kh, so that the
// pressure acts on u_par alone (i kh p) and continuity reads i kh u_par + v' = 0; u_perp obeys
// the diffusion equation of the buoyancy slot.  At kh = 0, u_par = u and u_perp = w.
//
// The kernels work in the frame scaled to unit wall distance (y' = (y + 1)/2 in [0, 1],
// x' = x/2, z' = z/2, t' = t/2, same velocity and pressure), where the explicit term is
//   N = -(u.grad) u - U u_x - v U' e_x,   U = 2 y' - 1 (the wall-moving laminar profile), U' = 2,
// on the 3/2 padded grid (Supplementary, "Initial value problems": F(X) of the IVP form).
//
// Layouts (complex128): z-grid fields of the per-mode kernels [f][Ngy][K], mode k = m Nz + n
// (m < Kx half-spectrum x modes, n < Nz z modes in FFT order, the z Nyquist n = Nz/2 unforced);
// plane intermediates [f][Ngy][Ngz][Kx] (x modes contiguous).  Steps:
//   A  per (y, tile of x modes, velocity component): the component, its y-derivative and its
//      x- and z-derivatives (i kx, i kz), inverse z-FFT onto the padded z grid;
//   B  per (y, pair of z rows): packed real inverse x-FFTs of the 12 fields, the products, forward
//      real x-FFTs of the 3 densities;
//   C  per (y, tile of x modes): forward z-FFTs, truncation, 1/(Ngx Ngz), rotation to
//      (par, v, perp).
// The VJP runs the transposes in reverse order (C', B' with the primal fields of A, A').
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <vector>

#include "cou.h"
#include "sps_device.h"
#include "sps_internal.h"

namespace sps {
namespace {

constexpr size_t kCouLdsMax = 160 * 1024;
constexpr size_t kCouLdsBudget = 40 * 1024;

struct CouDev {
  int Kx, Nz, K, Ngx, Ngz, Ngy;
  double lx, lz, du;
  const double* unode;   // [Ngy] base-flow velocity at the y nodes
  FftPlan px, pz;
  const cplx* twx;       // [Ngx]
  const cplx* twz;       // [Ngz]
};

__device__ __forceinline__ int cou_zrow(int n, int Nz, int G) {
  if (n < Nz / 2) return n;
  if (n == Nz / 2) return -1;
  return n - Nz + G;
}

struct Wave {
  double kx, kz, ex, ez;
};
__device__ __forceinline__ Wave cou_wave(const CouDev& d, int m, int n) {
  const int ns = (n < d.Nz / 2) ? n : n - d.Nz;
  Wave w;
  w.kx = 2.0 * M_PI * m / d.lx;
  w.kz = 2.0 * M_PI * ns / d.lz;
  const double kh = sqrt(w.kx * w.kx + w.kz * w.kz);
  if (kh > 0.0) {
    w.ex = w.kx / kh;
    w.ez = w.kz / kh;
  } else {
    w.ex = 1.0;
    w.ez = 0.0;
  }
  return w;
}

__device__ __forceinline__ cplx lin2(double a, cplx p, double b, cplx q) {
  return cmk(a * p.x + b * q.x, a * p.y + b * q.y);
}

// Hermitian packing of two half spectra (z rows z0, z0 + 1 of one field) into one length-G
// spectrum whose inverse DFT is row_z0 + i row_(z0+1); modes m >= 1 scaled by `scale`.
__device__ __forceinline__ cplx cou_pack(const cplx* U, const cplx* V, int x, int G, int K, double scale) {
  if (x == 0) return cmk(U[0].x, V[0].x);
  if (x < K) return cscale(cmk(U[x].x - V[x].y, U[x].y + V[x].x), scale);
  if (x > G - K) {
    const int q = G - x;
    return cscale(cmk(U[q].x + V[q].y, V[q].x - U[q].y), scale);
  }
  return czero();
}
// ---------------------------------------------------------------------------- in-place FFT
// The plane kernels run the mixed-radix Stockham passes in place in one LDS buffer: a thread
// loads and transforms all of its butterflies of a pass into registers, the block
// synchronizes, and the results go to their Stockham positions.  One buffer instead of a
// ping-pong pair lets two or three blocks share a CU.  A pass of radix R holds up to MB
// butterflies per thread, so a block of nt threads transforms up to 6 nt points
// (nbatch * n <= 6 nt, checked on the host).
// HALF: tw holds only the first n/2 twiddles (w^(m + n/2) = -w^m for even n).
template <int R, int MB, bool HALF>
__device__ __forceinline__ void ip_pass(cplx* buf, const FftPlan& p, int s, const cplx* __restrict__ tw, int sign,
                                        int nbatch, int bstride, int tid, int nt) {
  const int nR = p.n / R, Ns = p.ns[s], tst = p.tst[s];
  const unsigned mnr = p.mag_nr[s], mns = p.mag_ns[s];
  const int total = nbatch * nR;
  cplx v[MB][R];
  int dst[MB];
#pragma unroll
  for (int b = 0; b < MB; ++b) {
    const int it = tid + b * nt;
    dst[b] = -1;
    if (it < total) {
      const int q = fdiv(it, mnr);
      const int j = it - q * nR;
      const int jh = fdiv(j, mns);
      const int k = j - jh * Ns;
      const int t = k * tst;
      const int base = q * bstride;
      // all LDS reads of the butterfly first (one wait), then the twiddle products
      cplx w[R];
#pragma unroll
      for (int r = 0; r < R; ++r) v[b][r] = buf[fpad(base + j + r * nR)];
#pragma unroll
      for (int r = 1; r < R; ++r) {
        const int ti = r * t;
        if (HALF) {
          const int hn = p.n >> 1;
          const cplx u = tw[ti < hn ? ti : ti - hn];
          w[r] = (ti < hn) ? u : cmk(-u.x, -u.y);
        } else {
          w[r] = tw[ti];
        }
      }
#pragma unroll
      for (int r = 1; r < R; ++r) v[b][r] = cmul(v[b][r], sign > 0 ? cconj(w[r]) : w[r]);
      dft_small<R>(v[b], sign);
      dst[b] = base + jh * Ns * R + k;
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < MB; ++b)
    if (dst[b] >= 0) {
#pragma unroll
      for (int r = 0; r < R; ++r) buf[fpad(dst[b] + r * Ns)] = v[b][r];
    }
  __syncthreads();
}

// nbatch sequences of length p.n at buf + q * bstride (padded indices), transformed in place;
// ends synchronized.  Every thread of the block calls it.
template <bool HALF = false>
__device__ __forceinline__ void ip_fft(cplx* buf, const FftPlan& p, const cplx* tw, int sign, int nbatch, int bstride,
                                       int tid, int nt) {
  for (int s = 0; s < p.nst; ++s) {
    switch (p.radix[s]) {
      case 8: ip_pass<8, 1, HALF>(buf, p, s, tw, sign, nbatch, bstride, tid, nt); break;
      case 6: ip_pass<6, 1, HALF>(buf, p, s, tw, sign, nbatch, bstride, tid, nt); break;
      case 4: ip_pass<4, 2, HALF>(buf, p, s, tw, sign, nbatch, bstride, tid, nt); break;
      case 3: ip_pass<3, 2, HALF>(buf, p, s, tw, sign, nbatch, bstride, tid, nt); break;
      default: ip_pass<2, 3, HALF>(buf, p, s, tw, sign, nbatch, bstride, tid, nt); break;
    }
  }
}

// half spectrum of row yy (0 or 1) of a packed forward DFT r of two real rows
__device__ __forceinline__ cplx cou_unpack(const cplx* r, int base, int m, int G, int yy) {
  const cplx zm = r[fpad(base + m)], zq = r[fpad(base + (m == 0 ? 0 : G - m))];
  return yy ? cmk(0.5 * (zm.y + zq.y), -0.5 * (zm.x - zq.x)) : cmk(0.5 * (zm.x + zq.x), 0.5 * (zm.y - zq.y));
}

// ---------------------------------------------------------------------------- A: z inverse
// Grid (x-mode tiles, 3 components, Ngy).  Component g (u, v, w) writes fields g, 3 + g,
// 6 + 2g, 7 + 2g of Z: the component, its y-derivative, i kx times it, i kz times it.
template <int NT>
__global__ void __launch_bounds__(NT) cou_zinv(CouDev d, const cplx* zg, int tc, cplx* Z) {
  extern __shared__ double smem_d[];
  const int g = blockIdx.y, y = blockIdx.z, m0 = blockIdx.x * tc, tid = threadIdx.x;
  const int Nz = d.Nz, G = d.Ngz, K = d.K, Kx = d.Kx, Ngy = d.Ngy;
  if (m0 >= Kx) return;
  const int tcn = min(tc, Kx - m0);
  cplx* tw = reinterpret_cast<cplx*>(smem_d);
  cplx* b0 = tw + G;
  for (int e = tid; e < G; e += NT) tw[e] = d.twz[e];
  for (int e = tid; e < 4 * tcn * G; e += NT) b0[fpad(e)] = czero();
  __syncthreads();
  for (int e = tid; e < tcn * Nz; e += NT) {
    const int j = e / Nz, n = e - j * Nz, m = m0 + j;
    const int row = cou_zrow(n, Nz, G);
    if (row < 0) continue;
    const long long k = (long long)m * Nz + n;
    const Wave w = cou_wave(d, m, n);
    cplx val, dy;
    if (g == 1) {
      val = zg[(1LL * Ngy + y) * K + k];
      dy = zg[(4LL * Ngy + y) * K + k];
    } else {
      const cplx a = zg[(0LL * Ngy + y) * K + k], c = zg[(2LL * Ngy + y) * K + k];
      const cplx da = zg[(3LL * Ngy + y) * K + k], dc = zg[(5LL * Ngy + y) * K + k];
      if (g == 0) {   // u = ex u_par - ez u_perp
        val = lin2(w.ex, a, -w.ez, c);
        dy = lin2(w.ex, da, -w.ez, dc);
      } else {        // w = ez u_par + ex u_perp
        val = lin2(w.ez, a, w.ex, c);
        dy = lin2(w.ez, da, w.ex, dc);
      }
    }
    b0[fpad((0 * tcn + j) * G + row)] = val;
    b0[fpad((1 * tcn + j) * G + row)] = dy;
    b0[fpad((2 * tcn + j) * G + row)] = cscale(cmul_i(val), w.kx);
    b0[fpad((3 * tcn + j) * G + row)] = cscale(cmul_i(val), w.kz);
  }
  __syncthreads();
  ip_fft(b0, d.pz, tw, +1, 4 * tcn, G, tid, NT);
  const cplx* o = b0;
  const int fid[4] = {g, 3 + g, 6 + 2 * g, 7 + 2 * g};
  for (int e = tid; e < 4 * G * tcn; e += NT) {
    const int q = e / (G * tcn), r = e - q * G * tcn, z = r / tcn, j = r - z * tcn;
    Z[(((long long)fid[q] * Ngy + y) * G + z) * Kx + m0 + j] = o[fpad((q * tcn + j) * G + z)];
  }
}

// ---------------------------------------------------------------------------- B: x rows
// densities of one grid point from the 12 fields (one real row of each)
struct Dens {
  double nu, nv, nw;
};
__device__ __forceinline__ Dens cou_dens(const double* f, double U, double dU) {
  // f: u v w uy vy wy ux uz vx vz wx wz
  Dens r;
  r.nu = -(f[0] * f[6] + f[1] * f[3] + f[2] * f[7]) - U * f[6] - dU * f[1];
  r.nv = -(f[0] * f[8] + f[1] * f[4] + f[2] * f[9]) - U * f[8];
  r.nw = -(f[0] * f[10] + f[1] * f[5] + f[2] * f[11]) - U * f[10];
  return r;
}

// Grid (Ngz / 2, Ngy), 12 Ngx <= 6 NT.  LDS twiddles(Ngx) + fpad_size(12 Ngx).  The densities
// of a grid point overwrite its u, v, w slots (one thread reads and writes each x).
template <int NT>
__global__ void __launch_bounds__(NT) cou_xrow(CouDev d, const cplx* __restrict__ Z, cplx* __restrict__ W) {
  extern __shared__ double smem_d[];
  const int y = blockIdx.y, z0 = 2 * blockIdx.x, tid = threadIdx.x, G = d.Ngx, Kx = d.Kx, Ngy = d.Ngy, Gz = d.Ngz;
  cplx* tw = reinterpret_cast<cplx*>(smem_d);
  cplx* h = tw + G;
  for (int e = tid; e < G; e += NT) tw[e] = d.twx[e];
  for (int e = tid; e < 12 * G; e += NT) {
    const int f = e / G, x = e - f * G;
    const cplx* U = Z + (((long long)f * Ngy + y) * Gz + z0) * Kx;
    h[fpad(e)] = cou_pack(U, U + Kx, x, G, Kx, 1.0);
  }
  __syncthreads();
  ip_fft(h, d.px, tw, +1, 12, G, tid, NT);
  const double Uy = d.unode[y], dU = d.du;
  for (int x = tid; x < G; x += NT) {
    double fa[12], fb[12];
#pragma unroll
    for (int i = 0; i < 12; ++i) {
      const cplx v = h[fpad(i * G + x)];
      fa[i] = v.x;
      fb[i] = v.y;
    }
    const Dens a = cou_dens(fa, Uy, dU), b = cou_dens(fb, Uy, dU);
    h[fpad(x)] = cmk(a.nu, b.nu);
    h[fpad(G + x)] = cmk(a.nv, b.nv);
    h[fpad(2 * G + x)] = cmk(a.nw, b.nw);
  }
  __syncthreads();
  ip_fft(h, d.px, tw, -1, 3, G, tid, NT);
  const cplx* r = h;
  for (int e = tid; e < 3 * 2 * Kx; e += NT) {
    const int f = e / (2 * Kx), rr = e - f * 2 * Kx, yy = rr / Kx, m = rr - yy * Kx;
    W[(((long long)f * Ngy + y) * Gz + z0 + yy) * Kx + m] = cou_unpack(r, f * G, m, G, yy);
  }
}

// ---------------------------------------------------------------------------- C: z forward
// Grid (x-mode tiles, Ngy).
template <int NT>
__global__ void __launch_bounds__(NT) cou_zfwd(CouDev d, const cplx* W, int tc, cplx* nl) {
  extern __shared__ double smem_d[];
  const int y = blockIdx.y, m0 = blockIdx.x * tc, tid = threadIdx.x;
  const int Nz = d.Nz, G = d.Ngz, K = d.K, Kx = d.Kx, Ngy = d.Ngy;
  if (m0 >= Kx) return;
  const int tcn = min(tc, Kx - m0);
  cplx* tw = reinterpret_cast<cplx*>(smem_d);
  cplx* b0 = tw + G;
  for (int e = tid; e < G; e += NT) tw[e] = d.twz[e];
  for (int e = tid; e < 3 * G * tcn; e += NT) {
    const int f = e / (G * tcn), r = e - f * G * tcn, z = r / tcn, j = r - z * tcn;
    b0[fpad((f * tcn + j) * G + z)] = W[(((long long)f * Ngy + y) * G + z) * Kx + m0 + j];
  }
  __syncthreads();
  ip_fft(b0, d.pz, tw, -1, 3 * tcn, G, tid, NT);
  const cplx* res = b0;
  const double s = 1.0 / ((double)d.Ngx * G);
  for (int e = tid; e < tcn * Nz; e += NT) {
    const int j = e / Nz, n = e - j * Nz, m = m0 + j;
    const long long k = (long long)m * Nz + n;
    const int row = cou_zrow(n, Nz, G);
    cplx a = czero(), b = czero(), c = czero();
    if (row >= 0) {
      const Wave w = cou_wave(d, m, n);
      const cplx nu = cscale(res[fpad((0 * tcn + j) * G + row)], s);
      const cplx nv = cscale(res[fpad((1 * tcn + j) * G + row)], s);
      const cplx nw = cscale(res[fpad((2 * tcn + j) * G + row)], s);
      a = lin2(w.ex, nu, w.ez, nw);
      b = nv;
      c = lin2(-w.ez, nu, w.ex, nw);
    }
    nl[(0LL * Ngy + y) * K + k] = a;
    nl[(1LL * Ngy + y) * K + k] = b;
    nl[(2LL * Ngy + y) * K + k] = c;
  }
}

// ---------------------------------------------------------------------------- C': transpose of C
template <int NT>
__global__ void __launch_bounds__(NT) cou_zfwd_adj(CouDev d, const cplx* nlbar, int tc, cplx* Wb) {
  extern __shared__ double smem_d[];
  const int y = blockIdx.y, m0 = blockIdx.x * tc, tid = threadIdx.x;
  const int Nz = d.Nz, G = d.Ngz, K = d.K, Kx = d.Kx, Ngy = d.Ngy;
  if (m0 >= Kx) return;
  const int tcn = min(tc, Kx - m0);
  cplx* tw = reinterpret_cast<cplx*>(smem_d);
  cplx* b0 = tw + G;
  for (int e = tid; e < G; e += NT) tw[e] = d.twz[e];
  for (int e = tid; e < 3 * tcn * G; e += NT) b0[fpad(e)] = czero();
  __syncthreads();
  const double s = 1.0 / ((double)d.Ngx * G);
  for (int e = tid; e < tcn * Nz; e += NT) {
    const int j = e / Nz, n = e - j * Nz, m = m0 + j;
    const int row = cou_zrow(n, Nz, G);
    if (row < 0) continue;
    const long long k = (long long)m * Nz + n;
    const Wave w = cou_wave(d, m, n);
    const cplx a = nlbar[(0LL * Ngy + y) * K + k], b = nlbar[(1LL * Ngy + y) * K + k];
    const cplx c = nlbar[(2LL * Ngy + y) * K + k];
    b0[fpad((0 * tcn + j) * G + row)] = cscale(lin2(w.ex, a, -w.ez, c), s);
    b0[fpad((1 * tcn + j) * G + row)] = cscale(b, s);
    b0[fpad((2 * tcn + j) * G + row)] = cscale(lin2(w.ez, a, w.ex, c), s);
  }
  __syncthreads();
  ip_fft(b0, d.pz, tw, +1, 3 * tcn, G, tid, NT);
  const cplx* o = b0;
  for (int e = tid; e < 3 * G * tcn; e += NT) {
    const int f = e / (G * tcn), r = e - f * G * tcn, z = r / tcn, j = r - z * tcn;
    Wb[(((long long)f * Ngy + y) * G + z) * Kx + m0 + j] = o[fpad((f * tcn + j) * G + z)];
  }
}

// ---------------------------------------------------------------------------- B': transpose of B
// Grid (Ngz / 2, Ngy), 15 Ngx <= 6 NT.  LDS twiddles(Ngx / 2) + fpad_size(15 Ngx): three
// 512-thread blocks share a CU at Ngx = 192.  The primal fields Zp (12) and
// the density cotangents Wb (3, weight-1 modes) in; the 12 field cotangents out, as x half
// spectra times w_m (the transpose of the inverse transform).  The cotangents of a grid point
// overwrite its first 12 slots (one thread reads and writes each x).
template <int NT>
__global__ void __launch_bounds__(NT)
cou_xrow_adj(CouDev d, const cplx* __restrict__ Zp, const cplx* __restrict__ Wb, cplx* __restrict__ Gb) {
  extern __shared__ double smem_d[];
  const int y = blockIdx.y, z0 = 2 * blockIdx.x, tid = threadIdx.x, G = d.Ngx, Kx = d.Kx, Ngy = d.Ngy, Gz = d.Ngz;
  cplx* tw = reinterpret_cast<cplx*>(smem_d);
  cplx* h = tw + G / 2;
  cplx* o = h;
  for (int e = tid; e < G / 2; e += NT) tw[e] = d.twx[e];
  for (int e = tid; e < 15 * G; e += NT) {
    const int f = e / G, x = e - f * G;
    const cplx* U = (f < 12) ? Zp + (((long long)f * Ngy + y) * Gz + z0) * Kx
                             : Wb + (((long long)(f - 12) * Ngy + y) * Gz + z0) * Kx;
    h[fpad(e)] = cou_pack(U, U + Kx, x, G, Kx, f < 12 ? 1.0 : 0.5);
  }
  __syncthreads();
  ip_fft<true>(h, d.px, tw, +1, 15, G, tid, NT);
  const double Uy = d.unode[y], dU = d.du;
  for (int x = tid; x < G; x += NT) {
    // the two packed rows (real and imaginary parts) one after the other, as doubles
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      double* hd = reinterpret_cast<double*>(h) + r;
      double a[12];
#pragma unroll
      for (int i = 0; i < 12; ++i) a[i] = hd[2 * fpad(i * G + x)];
      const double nu = hd[2 * fpad(12 * G + x)], nv = hd[2 * fpad(13 * G + x)], nw = hd[2 * fpad(14 * G + x)];
      const double adv = a[0] + Uy;
      double out[12];
      out[0] = -(nu * a[6] + nv * a[8] + nw * a[10]);
      out[1] = -(nu * a[3] + nv * a[4] + nw * a[5]) - dU * nu;
      out[2] = -(nu * a[7] + nv * a[9] + nw * a[11]);
      out[3] = -nu * a[1];
      out[4] = -nv * a[1];
      out[5] = -nw * a[1];
      out[6] = -nu * adv;
      out[7] = -nu * a[2];
      out[8] = -nv * adv;
      out[9] = -nv * a[2];
      out[10] = -nw * adv;
      out[11] = -nw * a[2];
#pragma unroll
      for (int i = 0; i < 12; ++i) hd[2 * fpad(i * G + x)] = out[i];
    }
  }
  __syncthreads();
  ip_fft<true>(o, d.px, tw, -1, 12, G, tid, NT);
  const cplx* r = o;
  for (int e = tid; e < 12 * 2 * Kx; e += NT) {
    const int f = e / (2 * Kx), rr = e - f * 2 * Kx, yy = rr / Kx, m = rr - yy * Kx;
    const cplx v = cou_unpack(r, f * G, m, G, yy);
    Gb[(((long long)f * Ngy + y) * Gz + z0 + yy) * Kx + m] = (m == 0) ? v : cscale(v, 2.0);
  }
}

// ---------------------------------------------------------------------------- A': transpose of A
// Grid (x-mode tiles, 2 groups, Ngy): group 0 the u and w fields (8: they mix in the rotation),
// group 1 the v fields (4).  Forward z-FFTs of the field cotangents, the transposes of the
// derivative factors and of the rotation, into zbar[6][Ngy][K].
template <int NT>
__global__ void __launch_bounds__(NT) cou_zinv_adj(CouDev d, const cplx* Gb, int tc, cplx* zbar) {
  extern __shared__ double smem_d[];
  const int grp = blockIdx.y, y = blockIdx.z, m0 = blockIdx.x * tc, tid = threadIdx.x;
  const int Nz = d.Nz, G = d.Ngz, K = d.K, Kx = d.Kx, Ngy = d.Ngy;
  if (m0 >= Kx) return;
  const int tcn = min(tc, Kx - m0);
  const int nf = grp == 0 ? 8 : 4;
  // local slot -> field of Gb: group 0: u, uy, ux, uz, w, wy, wx, wz; group 1: v, vy, vx, vz
  const int fid0[8] = {0, 3, 6, 7, 2, 5, 10, 11};
  const int fid1[4] = {1, 4, 8, 9};
  cplx* tw = reinterpret_cast<cplx*>(smem_d);
  cplx* b0 = tw + G;
  for (int e = tid; e < G; e += NT) tw[e] = d.twz[e];
  for (int e = tid; e < nf * G * tcn; e += NT) {
    const int q = e / (G * tcn), r = e - q * G * tcn, z = r / tcn, j = r - z * tcn;
    const int f = grp == 0 ? fid0[q] : fid1[q];
    b0[fpad((q * tcn + j) * G + z)] = Gb[(((long long)f * Ngy + y) * G + z) * Kx + m0 + j];
  }
  __syncthreads();
  ip_fft(b0, d.pz, tw, -1, nf * tcn, G, tid, NT);
  const cplx* res = b0;
  for (int e = tid; e < tcn * Nz; e += NT) {
    const int j = e / Nz, n = e - j * Nz, m = m0 + j;
    const long long k = (long long)m * Nz + n;
    const int row = cou_zrow(n, Nz, G);
    const Wave w = cou_wave(d, m, n);
    auto at = [&](int q) { return row < 0 ? czero() : res[fpad((q * tcn + j) * G + row)]; };
    // total cotangent of a component: value + conj(i kx) d/dx part + conj(i kz) d/dz part
    auto total = [&](int qv, int qx, int qz) {
      return cadd(at(qv), cadd(cscale(cmul_mi(at(qx)), w.kx), cscale(cmul_mi(at(qz)), w.kz)));
    };
    if (grp == 0) {
      const cplx ut = total(0, 2, 3), wt = total(4, 6, 7);
      const cplx uy = at(1), wy = at(5);
      zbar[(0LL * Ngy + y) * K + k] = lin2(w.ex, ut, w.ez, wt);
      zbar[(2LL * Ngy + y) * K + k] = lin2(-w.ez, ut, w.ex, wt);
      zbar[(3LL * Ngy + y) * K + k] = lin2(w.ex, uy, w.ez, wy);
      zbar[(5LL * Ngy + y) * K + k] = lin2(-w.ez, uy, w.ex, wy);
    } else {
      zbar[(1LL * Ngy + y) * K + k] = total(0, 2, 3);
      zbar[(4LL * Ngy + y) * K + k] = at(1);
    }
  }
}

// Launch shapes.  A block transforms in place at most 6 NT points (ip_fft); the column kernels
// take x-mode tiles of tc columns of nf fields.  Blocks of 256 threads with at most kCouLdsBudget
// bytes of LDS, so that several share a CU; 1024 threads where one column of nf fields needs
// more.
constexpr int kColSmall = 256, kColLarge = 1024;
size_t lds_bytes(int G, int points) { return sizeof(cplx) * (G + (size_t)fpad_size(points)); }
int pick_nt(int points) { return points <= 6 * 256 ? 256 : (points <= 6 * 512 ? 512 : 1024); }

struct ColShape {
  int nt = kColSmall, tc = 1;
  size_t lds = 0;
};
ColShape col_shape(int G, int nf, int Kx) {
  ColShape c;
  c.nt = (nf * G <= 6 * kColSmall) ? kColSmall : kColLarge;
  SPS_REQUIRE(nf * G <= 6 * c.nt, "padded z grid too large for the plane kernels");
  int tc = std::min(8, Kx);
  while (tc > 1 && (nf * tc * G > 6 * c.nt || lds_bytes(G, nf * tc * G) > kCouLdsBudget)) --tc;
  c.tc = tc;
  c.lds = lds_bytes(G, nf * tc * G);
  SPS_REQUIRE(c.lds <= kCouLdsMax, "padded z grid too large for LDS");
  return c;
}

template <typename F1, typename F2>
void launch_col(const ColShape& c, F1 small, F2 large, dim3 grid, hipStream_t s) {
  if (c.nt == kColSmall) small(grid, s);
  else large(grid, s);
  SPS_CHECK_LAUNCH();
}

}  // namespace

struct CouettePlanes::Impl {
  CouDev d{};
  DevArena arena;
  ColShape A, C, A2;
  int ntB = 256, ntB2 = 256;
  size_t ldsB = 0, ldsB2 = 0;
  cplx *Zf = nullptr, *Wf = nullptr, *Zv = nullptr, *Wbv = nullptr, *Gv = nullptr;
};

CouettePlanes::CouettePlanes(const CouetteGeom& g, hipStream_t s) : p_(new Impl) {
  Impl& m = *p_;
  CouDev& d = m.d;
  SPS_REQUIRE(g.Kx >= 1 && g.Nz >= 2 && g.Nz % 2 == 0 && g.Ngx % 2 == 0 && g.Ngz % 2 == 0, "bad plane sizes");
  SPS_REQUIRE(g.Ngx >= 2 * g.Kx && g.Ngz >= g.Nz, "padded plane grid smaller than the modes");
  d.Kx = g.Kx;
  d.Nz = g.Nz;
  d.K = g.Kx * g.Nz;
  d.Ngx = g.Ngx;
  d.Ngz = g.Ngz;
  d.Ngy = g.Ngy;
  d.lx = g.lx;
  d.lz = g.lz;
  d.du = g.dunode;
  SPS_REQUIRE(fft_plan(g.Ngx, &d.px) && fft_plan(g.Ngz, &d.pz), "padded plane sizes must factor into 2 and 3");
  SPS_REQUIRE(15 * g.Ngx <= 6 * 1024, "padded x grid too large for the plane kernels");
  d.unode = m.arena.upload(std::vector<double>(g.unode, g.unode + g.Ngy), s);
  d.twx = m.arena.upload(twiddles(g.Ngx), s);
  d.twz = m.arena.upload(twiddles(g.Ngz), s);
  m.A = col_shape(g.Ngz, 4, g.Kx);
  m.C = col_shape(g.Ngz, 3, g.Kx);
  m.A2 = col_shape(g.Ngz, 8, g.Kx);
  m.ntB = pick_nt(12 * g.Ngx);
  m.ntB2 = pick_nt(15 * g.Ngx);
  m.ldsB = lds_bytes(g.Ngx, 12 * g.Ngx);
  m.ldsB2 = lds_bytes(g.Ngx / 2, 15 * g.Ngx);
  SPS_REQUIRE(m.ldsB2 <= kCouLdsMax, "padded x grid too large for LDS");
  for (const void* k :
       {(const void*)cou_zinv<kColSmall>, (const void*)cou_zinv<kColLarge>, (const void*)cou_zfwd<kColSmall>,
        (const void*)cou_zfwd<kColLarge>, (const void*)cou_zfwd_adj<kColSmall>, (const void*)cou_zfwd_adj<kColLarge>,
        (const void*)cou_zinv_adj<kColSmall>, (const void*)cou_zinv_adj<kColLarge>, (const void*)cou_xrow<256>,
        (const void*)cou_xrow<512>, (const void*)cou_xrow<1024>, (const void*)cou_xrow_adj<256>,
        (const void*)cou_xrow_adj<512>, (const void*)cou_xrow_adj<1024>})
    SPS_HIP(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kCouLdsMax));
  const size_t plane = (size_t)g.Ngy * g.Ngz * g.Kx;
  m.Zf = m.arena.alloc<cplx>(12 * plane);
  m.Wf = m.arena.alloc<cplx>(3 * plane);
  m.Zv = m.arena.alloc<cplx>(12 * plane);
  m.Wbv = m.arena.alloc<cplx>(3 * plane);
  m.Gv = m.arena.alloc<cplx>(12 * plane);
}
CouettePlanes::~CouettePlanes() = default;

namespace {
// (x-mode tiles, groups, Ngy) for the kernels that read y from blockIdx.z (A, A'); (x-mode
// tiles, Ngy) for C and C', which read it from blockIdx.y.
dim3 col_grid(const CouDev& d, const ColShape& c, int groups) { return dim3((d.Kx + c.tc - 1) / c.tc, groups, d.Ngy); }
dim3 col_grid_y(const CouDev& d, const ColShape& c) { return dim3((d.Kx + c.tc - 1) / c.tc, d.Ngy); }

void launch_zinv(const CouDev& d, const ColShape& c, const cplx* zg, cplx* Z, hipStream_t s) {
  launch_col(
      c, [&](dim3 g, hipStream_t st) { hipLaunchKernelGGL(cou_zinv<kColSmall>, g, dim3(kColSmall), c.lds, st, d, zg, c.tc, Z); },
      [&](dim3 g, hipStream_t st) { hipLaunchKernelGGL(cou_zinv<kColLarge>, g, dim3(kColLarge), c.lds, st, d, zg, c.tc, Z); },
      col_grid(d, c, 3), s);
}

}  // namespace

void CouettePlanes::forward(const double2* zg, double2* nl, hipStream_t s) {
  Impl& m = *p_;
  const CouDev& d = m.d;
  launch_zinv(d, m.A, zg, m.Zf, s);
  const dim3 gb(d.Ngz / 2, d.Ngy);
  if (m.ntB == 256)
    hipLaunchKernelGGL(cou_xrow<256>, gb, dim3(256), m.ldsB, s, d, m.Zf, m.Wf);
  else if (m.ntB == 512)
    hipLaunchKernelGGL(cou_xrow<512>, gb, dim3(512), m.ldsB, s, d, m.Zf, m.Wf);
  else
    hipLaunchKernelGGL(cou_xrow<1024>, gb, dim3(1024), m.ldsB, s, d, m.Zf, m.Wf);
  SPS_CHECK_LAUNCH();
  const ColShape& c = m.C;
  launch_col(
      c, [&](dim3 g, hipStream_t st) { hipLaunchKernelGGL(cou_zfwd<kColSmall>, g, dim3(kColSmall), c.lds, st, d, m.Wf, c.tc, nl); },
      [&](dim3 g, hipStream_t st) { hipLaunchKernelGGL(cou_zfwd<kColLarge>, g, dim3(kColLarge), c.lds, st, d, m.Wf, c.tc, nl); },
      col_grid_y(d, c), s);
}

void CouettePlanes::vjp(const double2* nlbar, const double2* zg, double2* zbar, hipStream_t s) {
  Impl& m = *p_;
  const CouDev& d = m.d;
  launch_zinv(d, m.A, zg, m.Zv, s);
  const ColShape& c = m.C;
  launch_col(
      c,
      [&](dim3 g, hipStream_t st) {
        hipLaunchKernelGGL(cou_zfwd_adj<kColSmall>, g, dim3(kColSmall), c.lds, st, d, nlbar, c.tc, m.Wbv);
      },
      [&](dim3 g, hipStream_t st) {
        hipLaunchKernelGGL(cou_zfwd_adj<kColLarge>, g, dim3(kColLarge), c.lds, st, d, nlbar, c.tc, m.Wbv);
      },
      col_grid_y(d, c), s);
  const dim3 gb(d.Ngz / 2, d.Ngy);
  if (m.ntB2 == 256)
    hipLaunchKernelGGL(cou_xrow_adj<256>, gb, dim3(256), m.ldsB2, s, d, m.Zv, m.Wbv, m.Gv);
  else if (m.ntB2 == 512)
    hipLaunchKernelGGL(cou_xrow_adj<512>, gb, dim3(512), m.ldsB2, s, d, m.Zv, m.Wbv, m.Gv);
  else
    hipLaunchKernelGGL(cou_xrow_adj<1024>, gb, dim3(1024), m.ldsB2, s, d, m.Zv, m.Wbv, m.Gv);
  SPS_CHECK_LAUNCH();
  const ColShape& a2 = m.A2;
  launch_col(
      a2,
      [&](dim3 g, hipStream_t st) {
        hipLaunchKernelGGL(cou_zinv_adj<kColSmall>, g, dim3(kColSmall), a2.lds, st, d, m.Gv, a2.tc, zbar);
      },
      [&](dim3 g, hipStream_t st) {
        hipLaunchKernelGGL(cou_zinv_adj<kColLarge>, g, dim3(kColLarge), a2.lds, st, d, m.Gv, a2.tc, zbar);
      },
      col_grid(d, a2, 2), s);
}

}  // namespace sps
