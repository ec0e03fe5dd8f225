// Batched 2D Swift-Hohenberg equation u_t = r u - (1 + Laplacian)^2 u - u^3 on doubly
// periodic squares [0, L)^2, many independent instances of different sizes in one
// persistent launch.  IVP form M dX/dt + L X = F(X) (Supplementary, "Initial value
// problems") with one unknown per Fourier mode: M = 1, L_k = -r + (1 - |k|^2)^2, F = -u^3
// with the cube formed on a grid padded by 2 in each direction.  SBDF2 with an SBDF1 first
// step (equ:imex); the reverse sweep is the multistep adjoint recurrence (equ:IMEX_adjoint).
//
// Instance i has N_i x N_i modes: k_x index m < N/2 (half spectrum, Nyquist dropped), k_y
// index iy < N in FFT order (iy = N/2, the Nyquist row, unused and zero).  States are
// column-major per instance, X[m][iy] (m-major), instances concatenated; grid fields are
// row-major [y][x] per instance, instances concatenated.  The real field is
// u = Re sum w_m X[m][iy] e^{i (k_x x + k_y y)}, w_0 = 1, w_m = 2.
//
// One step is two phases separated by a grid barrier:
//   column phase, per tile of k_x columns: forward y-FFT of the products' x-spectra, F,
//     the diagonal SBDF2 solve, and the inverse y-FFT of the new state (all column-local, so
//     a tile keeps its columns, and its block, for the whole sweep);
//   row phase, per tile of grid-row pairs: inverse real x-FFT (two rows per complex FFT),
//     the cube (or, in the reverse sweep, the product VJP 3 u^2 q), forward real x-FFT.
// Padded intermediate grids are [N/2][Ng] (column-major) so the column phase streams whole
// columns and the row phase reads row-tile segments.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <memory>
#include <vector>

#include "sps_device.h"
#include "sps_internal.h"

namespace sps {
namespace {

constexpr int NTB = 256;                  // threads of the initial-transform and solve blocks
constexpr unsigned kSpinLimit = 1u << 22; // bounded wait of a grid barrier (then abort)

struct ShInst {
  int N, Nh, Ng;
  int pn, png;        // FFT plans (index into the plan table) of lengths N and Ng
  int tc, trp;        // column tile (columns) and row tile (row pairs)
  double r;
  long long so;       // offset (complex) of the instance in state arrays: [Nh][N]
  long long go;       // offset (double) of the instance in grid arrays: [N][N]
  long long xo;       // history X_0 .. X_nmax, each [Nh][N]
  long long fo;       // F ring [2][Nh][N]
  long long yo, lo;   // reverse sweep: Y_(n+1) and the linear part, [Nh][N] each
  long long bo;       // dJ/dX_N from the cost phase, [Nh][N]
  long long zo, z2o, wo;   // padded x-spectra [Nh][Ng]
};

struct ShDev {
  int batch, nplan;
  double lx, dt;
  const ShInst* inst;
  const FftPlan* plans;
  const cplx* tw;       // twiddles of every plan, concatenated
  const int* twoff;     // offset of plan p's twiddles
  cplx* work;
  const int* cptr;      // column items of block b: citem[cptr[b] .. cptr[b+1])
  const int2* citem;    // (instance, first column)
  const int* rptr;
  const int2* ritem;    // (instance, first row pair)
  const int* jptr;
  const int* jitem;     // cost items: instance
  unsigned* bar;
  int* err;             // bit 1: non-finite state, bit 2: barrier timed out
};

enum RunMode { RUN_FWD = 1, RUN_COST = 2, RUN_ADJ = 4, RUN_EVALF = 8, RUN_VJP = 16 };

struct ShRun {
  int mode, nsteps;
  const cplx* xin;   // FWD: X_0; EVALF / VJP: X
  cplx* xout;        // FWD: X_N (nullable); EVALF: F; VJP: Xbar
  const cplx* gin;   // ADJ without COST: dJ/dX_N; VJP: Fbar
  cplx* gout;        // ADJ: dJ/dX_0
  double* J;         // COST: one per instance (nullable)
  cplx* dJ;          // COST: dJ/dX_N in the state layout (nullable)
};

struct SbdfCoef {
  double a0, a1, a2, c1, c2;
};
__device__ __forceinline__ SbdfCoef sbdf_coef(int n, double dt) {
  if (n == 1) return {1.0 / dt, -1.0 / dt, 0.0, 1.0, 0.0};
  return {1.5 / dt, -2.0 / dt, 0.5 / dt, 2.0, -1.0};
}

// padded FFT row of mode index iy (FFT order, N modes) in a length-Ng transform; -1 for the
// unused Nyquist row
__device__ __forceinline__ int pad_row(int iy, int N, int Ng) {
  if (iy < N / 2) return iy;
  if (iy == N / 2) return -1;
  return iy - N + Ng;
}
__device__ __forceinline__ double sh_lin(const ShDev& d, const ShInst& I, int m, int iy) {
  const double s = (iy < I.N / 2) ? (double)iy : (double)(iy - I.N);
  const double kx = 2.0 * M_PI * m / d.lx, ky = 2.0 * M_PI * s / d.lx;
  const double q = 1.0 - (kx * kx + ky * ky);
  return -I.r + q * q;
}

// Hermitian packing of two half spectra U, V (K modes, stride 1) into one length-n spectrum
// whose inverse DFT is u + i v; modes m >= 1 are scaled by `scale`.
__device__ __forceinline__ cplx pack2(const cplx* U, const cplx* V, int m, int n, int K, double scale) {
  if (m == 0) return cmk(U[0].x, V[0].x);
  if (m < K) {
    const cplx u = U[m], v = V[m];
    return cscale(cmk(u.x - v.y, u.y + v.x), scale);
  }
  if (m > n - K) {
    const cplx u = U[n - m], v = V[n - m];
    return cscale(cmk(u.x + v.y, v.x - u.y), scale);
  }
  return czero();
}

__device__ __forceinline__ void stage_tw(const ShDev& d, int plan, int n, cplx* tw) {
  const cplx* g = d.tw + d.twoff[plan];
  for (int e = threadIdx.x; e < n; e += blockDim.x) tw[e] = g[e];
}

// ---------------------------------------------------------------------------- grid barrier
// All blocks of the (cooperative) launch.  Thread 0 arrives with a release and waits with
// acquire loads; a wait longer than kSpinLimit polls, or another block's timeout, aborts:
// the block sets err bit 2 and returns false, and the caller leaves the kernel.
__device__ bool grid_sync(const ShDev& d, unsigned& epoch, int* sh_ok) {
  __syncthreads();
  if (threadIdx.x == 0) {
    epoch += 1;
    const unsigned target = epoch * gridDim.x;
    __atomic_thread_fence(__ATOMIC_RELEASE);
    __hip_atomic_fetch_add(d.bar, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    int ok = 1;
    unsigned it = 0;
    while (__hip_atomic_load(d.bar, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (++it > kSpinLimit || (__hip_atomic_load(d.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 4)) {
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    if (!ok) __hip_atomic_fetch_or(d.err, 4, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __atomic_thread_fence(__ATOMIC_ACQUIRE);
    *sh_ok = ok;
  }
  __syncthreads();
  return *sh_ok != 0;
}

// ---------------------------------------------------------------------------- column phase
enum ColKind { C_FWD_INIT, C_FWD_STEP, C_EVAL_INIT, C_EVAL_F, C_ADJ_INIT, C_ADJ_STEP, C_VJP_INIT, C_VJP_OUT };

// LDS of a column item: twiddles (Ng), two FFT buffers of 2 tc Ng (padded)
template <int NT>
__device__ void col_item(const ShDev& d, const ShRun& a, int2 item, int kind, int n, double* smem) {
  const ShInst I = d.inst[item.x];
  const int N = I.N, Nh = I.Nh, Ng = I.Ng, c0 = item.y;
  const int tcn = min(I.tc, Nh - c0);
  const FftPlan& P = d.plans[I.png];
  cplx* tw = reinterpret_cast<cplx*>(smem);
  cplx* b0 = tw + Ng;
  cplx* b1 = b0 + fpad_size(2 * I.tc * Ng);
  const int tid = threadIdx.x;
  cplx* W = d.work + I.wo;
  cplx* Z = d.work + I.zo;
  cplx* Z2 = d.work + I.z2o;
  cplx* H = d.work + I.xo;                  // history
  const long long nn = (long long)Nh * N;   // one state of the instance
  stage_tw(d, I.png, Ng, tw);

  // forward y-FFT of the x-spectra W for the tile's columns -> res (unnormalized)
  const cplx* res = nullptr;
  if (kind == C_FWD_STEP || kind == C_EVAL_F || kind == C_ADJ_STEP || kind == C_VJP_OUT) {
    for (int e = tid; e < tcn * Ng; e += NT) {
      const int j = e / Ng, y = e - j * Ng;
      b0[fpad(e)] = W[(long long)(c0 + j) * Ng + y];
    }
    __syncthreads();
    res = lds_fft(b0, b1, P, tw, -1, tcn, Ng, tid, NT);
  }
  cplx* ibuf = (res == b0) ? b1 : b0;   // free buffer for the inverse transforms
  // inverse y-FFTs to run per column: the new state (1), or the primal state and the
  // cotangent (2); none after the last forward step or once dJ/dX_0 is out
  const bool two = (kind == C_VJP_INIT || kind == C_ADJ_INIT || kind == C_ADJ_STEP);
  const bool inv = (kind == C_FWD_INIT || kind == C_EVAL_INIT || kind == C_VJP_INIT ||
                    (kind == C_FWD_STEP && n < a.nsteps) || (kind == C_ADJ_INIT && n >= 1) ||
                    (kind == C_ADJ_STEP && n - 1 >= 1));
  const int ninv = inv ? (two ? 2 : 1) : 0;
  const double ng2 = 1.0 / ((double)Ng * Ng);

  for (int e = tid; e < tcn * N; e += NT) {
    const int j = e / N, iy = e - j * N, m = c0 + j;
    const int row = pad_row(iy, N, Ng);
    const long long si = (long long)m * N + iy;     // index inside one [Nh][N] array
    const double wm = (m == 0) ? 1.0 : 2.0;
    cplx v1 = czero(), v2 = czero();                // values for the inverse transforms
    switch (kind) {
      case C_FWD_INIT: {
        const cplx x = (row >= 0) ? a.xin[I.so + si] : czero();
        H[si] = x;
        v1 = x;
        break;
      }
      case C_EVAL_INIT:
        v1 = (row >= 0) ? a.xin[I.so + si] : czero();
        break;
      case C_VJP_INIT:
        v1 = (row >= 0) ? a.xin[I.so + si] : czero();
        v2 = (row >= 0) ? cscale(a.gin[I.so + si], -1.0) : czero();
        break;
      case C_EVAL_F: {
        const cplx f = (row >= 0) ? cscale(res[fpad(j * Ng + row)], -ng2) : czero();
        a.xout[I.so + si] = f;
        break;
      }
      case C_VJP_OUT: {
        const cplx xb = (row >= 0) ? cscale(res[fpad(j * Ng + row)], wm) : czero();
        a.xout[I.so + si] = xb;
        break;
      }
      case C_FWD_STEP: {
        // F_(n-1) from the products, then (a0 + L) X_n = c1 F_(n-1) + c2 F_(n-2) - a1 X_(n-1) - a2 X_(n-2)
        cplx* Fr = d.work + I.fo;
        cplx xn = czero();
        if (row >= 0) {
          const SbdfCoef q = sbdf_coef(n, d.dt);
          const cplx f1 = cscale(res[fpad(j * Ng + row)], -ng2);
          const cplx f2 = (n >= 2) ? Fr[(n & 1) * nn + si] : czero();
          const cplx x1 = H[(n - 1) * nn + si];
          const cplx x2 = (n >= 2) ? H[(n - 2) * nn + si] : czero();
          cplx rhs = cadd(cscale(f1, q.c1), cscale(f2, q.c2));
          rhs = csub(rhs, cadd(cscale(x1, q.a1), cscale(x2, q.a2)));
          xn = cscale(rhs, 1.0 / (q.a0 + sh_lin(d, I, m, iy)));
          Fr[((n - 1) & 1) * nn + si] = f1;
          if (!(isfinite(xn.x) && isfinite(xn.y))) atomicOr(d.err, 2);
        }
        H[n * nn + si] = xn;
        if (n == a.nsteps && a.xout) a.xout[I.so + si] = xn;
        v1 = xn;
        break;
      }
      case C_ADJ_INIT:
      case C_ADJ_STEP: {
        // cotangent of X_n (ADJ_INIT: from the cost or the caller; ADJ_STEP: of X_(n-1) from
        // the products' VJP minus the linear part stored by the previous column phase)
        cplx* Yn = d.work + I.yo;
        cplx* Ln = d.work + I.lo;
        int k = n;                        // index of the state whose cotangent is complete
        cplx xb = czero();
        if (kind == C_ADJ_INIT) {
          if (row >= 0) xb = (a.mode & RUN_COST) ? d.work[I.bo + si] : a.gin[I.so + si];
        } else {
          k = n - 1;
          if (row >= 0) xb = csub(cscale(res[fpad(j * Ng + row)], wm), Ln[si]);
        }
        if (k == 0) {
          a.gout[I.so + si] = xb;
          break;
        }
        cplx g = czero(), lin = czero(), y = czero();
        if (row >= 0) {
          const SbdfCoef q = sbdf_coef(k, d.dt);
          y = cscale(xb, 1.0 / (q.a0 + sh_lin(d, I, m, iy)));
          g = cscale(y, q.c1);
          lin = cscale(y, q.a1);
          if (k + 1 <= a.nsteps) {
            const SbdfCoef qn = sbdf_coef(k + 1, d.dt);
            const cplx yn = Yn[si];
            g = cadd(g, cscale(yn, qn.c2));
            lin = cadd(lin, cscale(yn, qn.a2));
          }
        }
        Yn[si] = y;
        Ln[si] = lin;
        v1 = H[(k - 1) * nn + si];        // X_(k-1): primal field of the products' VJP
        v2 = cscale(g, -1.0);
        break;
      }
      default:
        break;
    }
    if (ninv > 0 && row >= 0) {
      ibuf[fpad(j * Ng + row)] = v1;
      if (ninv == 2) ibuf[fpad((tcn + j) * Ng + row)] = v2;
    }
  }
  if (ninv > 0) {
    // rows no mode maps to: N/2 .. Ng - N/2 (the Nyquist row and the padding), then the
    // inverse y-FFTs
    const int nz = Ng - N + 1;
    for (int e = tid; e < ninv * tcn * nz; e += NT) {
      const int col = e / nz, t = e - col * nz;
      ibuf[fpad(col * Ng + N / 2 + t)] = czero();
    }
    __syncthreads();
    cplx* other = (ibuf == b0) ? b1 : b0;
    const cplx* out = lds_fft(ibuf, other, P, tw, +1, ninv * tcn, Ng, tid, NT);
    for (int e = tid; e < tcn * Ng; e += NT) {
      const int j = e / Ng, y = e - j * Ng;
      Z[(long long)(c0 + j) * Ng + y] = out[fpad(e)];
      if (ninv == 2) Z2[(long long)(c0 + j) * Ng + y] = out[fpad((tcn + j) * Ng + y)];
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------- row phase
enum RowKind { R_CUBE, R_VJP };

// LDS of a row item: twiddles (Ng), spectra of the tile's rows (2 arrays x 2 trp x Nh), two
// FFT buffers of 2 trp Ng (padded)
template <int NT>
__device__ void row_item(const ShDev& d, int2 item, int kind, double* smem) {
  const ShInst I = d.inst[item.x];
  const int Nh = I.Nh, Ng = I.Ng, p0 = item.y;
  const int R = 2 * I.trp;                 // rows of a full tile
  const int y0 = 2 * p0;
  const int rn = min(R, Ng - y0);          // rows in this tile (even)
  const int pn = rn / 2;
  const FftPlan& P = d.plans[I.png];
  cplx* tw = reinterpret_cast<cplx*>(smem);
  cplx* sp = tw + Ng;                      // [2][R][Nh]: rows of Z (and Z2)
  cplx* b0 = sp + 2 * R * Nh;
  cplx* b1 = b0 + fpad_size(2 * I.trp * Ng);
  const int tid = threadIdx.x;
  const cplx* Z = d.work + I.zo;
  const cplx* Z2 = d.work + I.z2o;
  cplx* W = d.work + I.wo;
  const bool vjp = (kind == R_VJP);
  stage_tw(d, I.png, Ng, tw);
  // the tile's rows of the column-major x-spectra: rn consecutive y for each column m
  const int na = vjp ? 2 : 1;
  for (int e = tid; e < na * Nh * rn; e += NT) {
    const int arr = e / (Nh * rn), rem = e - arr * Nh * rn;
    const int m = rem / rn, yy = rem - m * rn;
    const cplx* src = arr ? Z2 : Z;
    sp[(arr * R + yy) * Nh + m] = src[(long long)m * Ng + y0 + yy];
  }
  __syncthreads();
  // pack row pairs (2q, 2q+1): batch q < pn (values u), pn + q (values q, weight-1 modes)
  for (int e = tid; e < na * pn * Ng; e += NT) {
    const int b = e / Ng, x = e - b * Ng;
    const int arr = b / pn, q = b - arr * pn;
    const cplx* U = sp + (arr * R + 2 * q) * Nh;
    b0[fpad(e)] = pack2(U, U + Nh, x, Ng, Nh, arr ? 0.5 : 1.0);
  }
  __syncthreads();
  const cplx* g = lds_fft(b0, b1, P, tw, +1, na * pn, Ng, tid, NT);
  cplx* o = (g == b0) ? b1 : b0;
  const double ng2 = 1.0 / ((double)Ng * Ng);
  for (int e = tid; e < pn * Ng; e += NT) {
    const cplx u = g[fpad(e)];
    cplx v;
    if (!vjp) {
      v = cmk(u.x * u.x * u.x, u.y * u.y * u.y);
    } else {
      const cplx qv = g[fpad(pn * Ng + e)];
      v = cmk(3.0 * u.x * u.x * qv.x * ng2, 3.0 * u.y * u.y * qv.y * ng2);
    }
    o[fpad(e)] = v;
  }
  __syncthreads();
  cplx* g2 = (o == b0) ? b1 : b0;
  const cplx* h = lds_fft(o, g2, P, tw, -1, pn, Ng, tid, NT);
  // unpack A_m = (Z_m + conj Z_-m)/2 (row 2q), B_m = (Z_m - conj Z_-m)/(2i) (row 2q+1), m < Nh
  for (int e = tid; e < Nh * rn; e += NT) {
    const int m = e / rn, yy = e - m * rn;
    const int q = yy >> 1;
    const cplx zm = h[fpad(q * Ng + m)], zq = h[fpad(q * Ng + (m == 0 ? 0 : Ng - m))];
    const cplx v = (yy & 1) ? cmk(0.5 * (zm.y + zq.y), -0.5 * (zm.x - zq.x)) : cmk(0.5 * (zm.x + zq.x), 0.5 * (zm.y - zq.y));
    W[(long long)m * Ng + y0 + yy] = v;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------- cost phase
// J = 1/2 mean over the N x N grid of u^2 = 1/2 sum w |c~|^2 with c~ the coefficients of
// the real field (the k_x = 0 column made Hermitian in k_y), dJ/dX = w c~.
template <int NT>
__device__ void cost_item(const ShDev& d, const ShRun& a, int inst, double* smem) {
  const ShInst I = d.inst[inst];
  const int N = I.N, Nh = I.Nh, tid = threadIdx.x;
  const cplx* X = d.work + I.xo + (long long)a.nsteps * Nh * N;
  double* red = smem;
  double part = 0.0;
  for (int e = tid; e < Nh * N; e += NT) {
    const int m = e / N, iy = e - m * N;
    cplx c = czero();
    if (iy != N / 2) {
      c = X[e];
      if (m == 0) {
        const int jm = (N - iy) % N;        // row of -k_y
        const cplx cm = X[jm];
        c = cmk(0.5 * (c.x + cm.x), 0.5 * (c.y - cm.y));
      }
    }
    const double w = (m == 0) ? 1.0 : 2.0;
    const cplx g = cscale(c, w);
    d.work[I.bo + e] = g;
    if (a.dJ) a.dJ[I.so + e] = g;
    part += 0.5 * w * (c.x * c.x + c.y * c.y);
  }
  red[tid] = part;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  if (tid == 0 && a.J) a.J[inst] = red[0];
  __syncthreads();
}

// ---------------------------------------------------------------------------- persistent launch
template <int NT>
__global__ void __launch_bounds__(NT) sh_persistent(ShDev d, ShRun a) {
  extern __shared__ double smem_d[];
  __shared__ int sh_ok;
  unsigned epoch = 0;
  const int b = blockIdx.x;
  auto cols = [&](int kind, int n) {
    for (int it = d.cptr[b]; it < d.cptr[b + 1]; ++it) col_item<NT>(d, a, d.citem[it], kind, n, smem_d);
  };
  auto rows = [&](int kind) {
    for (int it = d.rptr[b]; it < d.rptr[b + 1]; ++it) row_item<NT>(d, d.ritem[it], kind, smem_d);
  };
  if (a.mode & RUN_FWD) {
    cols(C_FWD_INIT, 0);
    for (int n = 1; n <= a.nsteps; ++n) {
      if (!grid_sync(d, epoch, &sh_ok)) return;
      rows(R_CUBE);
      if (!grid_sync(d, epoch, &sh_ok)) return;
      cols(C_FWD_STEP, n);
    }
  }
  if (a.mode & RUN_COST) {
    if (!grid_sync(d, epoch, &sh_ok)) return;
    for (int it = d.jptr[b]; it < d.jptr[b + 1]; ++it) cost_item<NT>(d, a, d.jitem[it], smem_d);
  }
  if (a.mode & RUN_ADJ) {
    if (!grid_sync(d, epoch, &sh_ok)) return;
    cols(C_ADJ_INIT, a.nsteps);
    for (int n = a.nsteps; n >= 1; --n) {
      if (!grid_sync(d, epoch, &sh_ok)) return;
      rows(R_VJP);
      if (!grid_sync(d, epoch, &sh_ok)) return;
      cols(C_ADJ_STEP, n);
    }
  }
  if (a.mode & RUN_EVALF) {
    cols(C_EVAL_INIT, 0);
    if (!grid_sync(d, epoch, &sh_ok)) return;
    rows(R_CUBE);
    if (!grid_sync(d, epoch, &sh_ok)) return;
    cols(C_EVAL_F, 0);
  }
  if (a.mode & RUN_VJP) {
    cols(C_VJP_INIT, 0);
    if (!grid_sync(d, epoch, &sh_ok)) return;
    rows(R_VJP);
    if (!grid_sync(d, epoch, &sh_ok)) return;
    cols(C_VJP_OUT, 0);
  }
}

// ---------------------------------------------------------------------------- initial transform
// X0 = (1/N^2) sum_grid u0 e^{-i k.x} on the N x N grid (kept modes), and its transpose
// ubar = (1/N^2) Re sum_k Xbar_k e^{i k.x} (weight 1 for every kept mode).  One block per
// instance and direction pass, in two launches each (rows, then columns).
constexpr int INIT_TILE = 8;   // row pairs or columns per block of the initial transforms

// rows: grid [y][x] -> T[m][y] (m < Nh), r2c per row pair; block (instance, tile of pairs)
__global__ void __launch_bounds__(NTB) sh_init_rows(ShDev d, const double* grid, cplx* tmp) {
  extern __shared__ double smem_d[];
  const ShInst I = d.inst[blockIdx.x];
  const int N = I.N, Nh = I.Nh, tid = threadIdx.x;
  const int p0 = blockIdx.y * INIT_TILE;
  if (p0 >= Nh) return;
  const int pn = min(INIT_TILE, Nh - p0);
  cplx* tw = reinterpret_cast<cplx*>(smem_d);
  cplx* b0 = tw + N;
  cplx* b1 = b0 + fpad_size(INIT_TILE * N);
  stage_tw(d, I.pn, N, tw);
  const double* u = grid + I.go;
  for (int e = tid; e < pn * N; e += NTB) {     // pair q: rows 2(p0+q), 2(p0+q)+1
    const int q = e / N, x = e - q * N, y = 2 * (p0 + q);
    b0[fpad(e)] = cmk(u[(long long)y * N + x], u[(long long)(y + 1) * N + x]);
  }
  __syncthreads();
  const cplx* h = lds_fft(b0, b1, d.plans[I.pn], tw, -1, pn, N, tid, NTB);
  cplx* T = tmp + I.so;   // [Nh][N] column-major like the state
  for (int e = tid; e < Nh * 2 * pn; e += NTB) {
    const int m = e / (2 * pn), yy = e - m * 2 * pn, q = yy >> 1;
    const cplx zm = h[fpad(q * N + m)], zq = h[fpad(q * N + (m == 0 ? 0 : N - m))];
    T[(long long)m * N + 2 * p0 + yy] =
        (yy & 1) ? cmk(0.5 * (zm.y + zq.y), -0.5 * (zm.x - zq.x)) : cmk(0.5 * (zm.x + zq.x), 0.5 * (zm.y - zq.y));
  }
}
// columns: T[m][y] -> X[m][iy] = FFT_y / N^2 (kept rows); block (instance, tile of columns)
__global__ void __launch_bounds__(NTB) sh_init_cols(ShDev d, const cplx* tmp, cplx* X) {
  extern __shared__ double smem_d[];
  const ShInst I = d.inst[blockIdx.x];
  const int N = I.N, Nh = I.Nh, tid = threadIdx.x;
  const int c0 = blockIdx.y * INIT_TILE;
  if (c0 >= Nh) return;
  const int cn = min(INIT_TILE, Nh - c0);
  cplx* tw = reinterpret_cast<cplx*>(smem_d);
  cplx* b0 = tw + N;
  cplx* b1 = b0 + fpad_size(INIT_TILE * N);
  stage_tw(d, I.pn, N, tw);
  for (int e = tid; e < cn * N; e += NTB) b0[fpad(e)] = tmp[I.so + (long long)c0 * N + e];
  __syncthreads();
  const cplx* h = lds_fft(b0, b1, d.plans[I.pn], tw, -1, cn, N, tid, NTB);
  const double s = 1.0 / ((double)N * N);
  for (int e = tid; e < cn * N; e += NTB) {
    const int iy = e % N;
    X[I.so + (long long)c0 * N + e] = (iy == N / 2) ? czero() : cscale(h[fpad(e)], s);
  }
}
// adjoint, columns: Xbar[m][iy] -> T[m][y] = sum_iy Xbar e^{i k_y y} (kept rows)
__global__ void __launch_bounds__(NTB) sh_init_adj_cols(ShDev d, const cplx* Xb, cplx* tmp) {
  extern __shared__ double smem_d[];
  const ShInst I = d.inst[blockIdx.x];
  const int N = I.N, Nh = I.Nh, tid = threadIdx.x;
  const int c0 = blockIdx.y * INIT_TILE;
  if (c0 >= Nh) return;
  const int cn = min(INIT_TILE, Nh - c0);
  cplx* tw = reinterpret_cast<cplx*>(smem_d);
  cplx* b0 = tw + N;
  cplx* b1 = b0 + fpad_size(INIT_TILE * N);
  stage_tw(d, I.pn, N, tw);
  for (int e = tid; e < cn * N; e += NTB) {
    const int iy = e % N;
    b0[fpad(e)] = (iy == N / 2) ? czero() : Xb[I.so + (long long)c0 * N + e];
  }
  __syncthreads();
  const cplx* h = lds_fft(b0, b1, d.plans[I.pn], tw, +1, cn, N, tid, NTB);
  for (int e = tid; e < cn * N; e += NTB) tmp[I.so + (long long)c0 * N + e] = h[fpad(e)];
}
// adjoint, rows: T[m][y] -> ubar[y][x] = (1/N^2) Re sum_m T[m][y] e^{i k_x x} (weight 1)
__global__ void __launch_bounds__(NTB) sh_init_adj_rows(ShDev d, const cplx* tmp, double* grid) {
  extern __shared__ double smem_d[];
  const ShInst I = d.inst[blockIdx.x];
  const int N = I.N, Nh = I.Nh, tid = threadIdx.x;
  const int p0 = blockIdx.y * INIT_TILE;
  if (p0 >= Nh) return;
  const int pn = min(INIT_TILE, Nh - p0);
  cplx* tw = reinterpret_cast<cplx*>(smem_d);
  cplx* sp = tw + N;                          // [2 INIT_TILE rows][Nh]
  cplx* b0 = sp + 2 * INIT_TILE * Nh;
  cplx* b1 = b0 + fpad_size(INIT_TILE * N);
  stage_tw(d, I.pn, N, tw);
  for (int e = tid; e < Nh * 2 * pn; e += NTB) {
    const int m = e / (2 * pn), yy = e - m * 2 * pn;
    sp[yy * Nh + m] = tmp[I.so + (long long)m * N + 2 * p0 + yy];
  }
  __syncthreads();
  for (int e = tid; e < pn * N; e += NTB) {   // pair q: rows 2(p0+q), 2(p0+q)+1
    const int q = e / N, x = e - q * N;
    const cplx* U = sp + (2 * q) * Nh;
    b0[fpad(e)] = pack2(U, U + Nh, x, N, Nh, 0.5);
  }
  __syncthreads();
  const cplx* h = lds_fft(b0, b1, d.plans[I.pn], tw, +1, pn, N, tid, NTB);
  const double s = 1.0 / ((double)N * N);
  double* g = grid + I.go;
  for (int e = tid; e < pn * N; e += NTB) {
    const int q = e / N, x = e - q * N, y = 2 * (p0 + q);
    const cplx v = h[fpad(e)];
    g[(long long)y * N + x] = v.x * s;
    g[(long long)(y + 1) * N + x] = v.y * s;
  }
}

// X = (1.5/dt + L)^{-1} R per mode (the SBDF2 matrix; real diagonal, equal to its adjoint)
__global__ void __launch_bounds__(NTB) sh_solve(ShDev d, const cplx* R, cplx* X) {
  const ShInst I = d.inst[blockIdx.x];
  for (int e = threadIdx.x; e < I.Nh * I.N; e += NTB) {
    const int m = e / I.N, iy = e - m * I.N;
    X[I.so + e] = (iy == I.N / 2) ? czero() : cscale(R[I.so + e], 1.0 / (1.5 / d.dt + sh_lin(d, I, m, iy)));
  }
}

// ---------------------------------------------------------------------------- host
class ShProblem : public ProblemImpl {
 public:
  ShProblem(int batch, const int* n, const double* r, double lx, double dt, int max_steps, hipStream_t s) {
    stream = s;
    SPS_REQUIRE(batch >= 1 && n && r, "bad batch");
    SPS_REQUIRE(lx > 0 && dt > 0 && max_steps >= 1, "bad lx / dt / max_steps");
    batch_ = batch;
    lx_ = lx;
    dt_ = dt;
    max_steps_ = max_steps;
    ns_.assign(n, n + batch);
    rs_.assign(r, r + batch);
    for (int i = 0; i < batch; ++i)
      SPS_REQUIRE(ns_[i] >= 8 && ns_[i] % 2 == 0 && ns_[i] <= 512, "instance sizes must be even, 8 <= N <= 512");
    hipDeviceProp_t prop;
    int dev = 0;
    SPS_HIP(hipGetDevice(&dev));
    SPS_HIP(hipGetDeviceProperties(&prop, dev));
    cus_ = prop.multiProcessorCount;
    build_plans();
    layout();
    bar_ = arena_.alloc<unsigned>(1);
    err_ = arena_.alloc<int>(1);
    SPS_HIP(hipMemsetAsync(err_, 0, sizeof(int), stream));
    const std::pair<const void*, size_t> init[] = {{(const void*)sh_init_rows, init_lds(false)},
                                                   {(const void*)sh_init_cols, init_lds(false)},
                                                   {(const void*)sh_init_adj_cols, init_lds(false)},
                                                   {(const void*)sh_init_adj_rows, init_lds(true)}};
    for (const auto& k : init) {
      SPS_REQUIRE(k.second <= 160 * 1024, "instance too large for the initial transforms");
      SPS_HIP(hipFuncSetAttribute(k.first, hipFuncAttributeMaxDynamicSharedMemorySize, (int)k.second));
    }
    tune();
  }

  long long state_size() const override { return 2 * state_cplx_; }
  // a new step for the following runs: the SBDF2 coefficients take it (the implicit operator is
  // diagonal, nothing is factored); drops the recorded run
  void set_dt(double dt) override {
    SPS_REQUIRE(std::isfinite(dt) && dt > 0.0, "dt must be positive");
    dt_ = dt;
    dv_.dt = dt;
    tape_steps_ = -1;
  }
  void factor() override {}

  void step(double* X, int nsteps) override {
    SPS_REQUIRE(X, "X is null");
    SPS_REQUIRE(nsteps >= 1 && nsteps <= max_steps_, "nsteps out of range");
    ShRun a{RUN_FWD, nsteps, reinterpret_cast<const cplx*>(X), reinterpret_cast<cplx*>(X), nullptr, nullptr, nullptr,
            nullptr};
    run(a);
    tape_steps_ = nsteps;
  }
  void adjoint_step(double* Xbar, int nsteps) override {
    SPS_REQUIRE(Xbar, "Xbar is null");
    if (tape_steps_ != nsteps) throw Error(SPS_E_STATE, "adjoint_step: nsteps does not match the recorded forward run");
    ShRun a{RUN_ADJ, nsteps, nullptr, nullptr, reinterpret_cast<const cplx*>(Xbar), reinterpret_cast<cplx*>(Xbar),
            nullptr, nullptr};
    run(a);
  }
  void cost(const double* X, double* J, double* dJdX) override {
    SPS_REQUIRE(X && dJdX, "null argument");
    // the cost phase reads history slot nsteps: X goes to the spare slot max_steps + 1,
    // leaving a recorded forward run intact
    SPS_HIP(hipMemcpyAsync(tmp_, X, sizeof(cplx) * state_cplx_, hipMemcpyDeviceToDevice, stream));
    copy_into_history(max_steps_ + 1);
    ShRun a{RUN_COST, max_steps_ + 1, nullptr, nullptr, nullptr, nullptr, J, reinterpret_cast<cplx*>(dJdX)};
    run(a);
  }
  void gradient(const double* X0, int nsteps, const double* dJdXN, double* XN, double* dJdX0, double* dJdtheta,
                double* J) override {
    SPS_REQUIRE(X0 && dJdX0, "null argument");
    SPS_REQUIRE(nsteps >= 1 && nsteps <= max_steps_, "nsteps out of range");
    if (dJdtheta) throw Error(SPS_E_UNSUPPORTED, "the Swift-Hohenberg batch has no parameter gradients");
    // an upstream cotangent replaces the cost phase: the reverse sweep starts from dJdXN
    ShRun a{dJdXN ? (RUN_FWD | RUN_ADJ) : (RUN_FWD | RUN_COST | RUN_ADJ), nsteps, reinterpret_cast<const cplx*>(X0),
            reinterpret_cast<cplx*>(XN), reinterpret_cast<const cplx*>(dJdXN), reinterpret_cast<cplx*>(dJdX0), J,
            nullptr};
    run(a);
    tape_steps_ = nsteps;
  }
  void initial_state(const double* grid, double* X) override {
    SPS_REQUIRE(grid && X, "null argument");
    hipLaunchKernelGGL(sh_init_rows, init_grid(), dim3(NTB), init_lds(false), stream, dv_, grid, tmp_);
    SPS_CHECK_LAUNCH();
    hipLaunchKernelGGL(sh_init_cols, init_grid(), dim3(NTB), init_lds(false), stream, dv_, tmp_,
                       reinterpret_cast<cplx*>(X));
    SPS_CHECK_LAUNCH();
  }
  void initial_state_adjoint(const double* Xbar, double* grid) override {
    SPS_REQUIRE(grid && Xbar, "null argument");
    hipLaunchKernelGGL(sh_init_adj_cols, init_grid(), dim3(NTB), init_lds(false), stream, dv_,
                       reinterpret_cast<const cplx*>(Xbar), tmp_);
    SPS_CHECK_LAUNCH();
    hipLaunchKernelGGL(sh_init_adj_rows, init_grid(), dim3(NTB), init_lds(true), stream, dv_, tmp_, grid);
    SPS_CHECK_LAUNCH();
  }
  void eval_F(const double* X, double* F) override {
    SPS_REQUIRE(X && F, "null argument");
    ShRun a{RUN_EVALF, 0, reinterpret_cast<const cplx*>(X), reinterpret_cast<cplx*>(F), nullptr, nullptr, nullptr,
            nullptr};
    run(a);
  }
  void eval_F_vjp(const double* X, const double* Fbar, double* Xbar) override {
    SPS_REQUIRE(X && Fbar && Xbar, "null argument");
    ShRun a{RUN_VJP, 0, reinterpret_cast<const cplx*>(X), reinterpret_cast<cplx*>(Xbar),
            reinterpret_cast<const cplx*>(Fbar), nullptr, nullptr, nullptr};
    run(a);
  }
  void solve(const double* R, double* X, int) override {
    SPS_REQUIRE(R && X, "null argument");
    hipLaunchKernelGGL(sh_solve, dim3(batch_), dim3(NTB), 0, stream, dv_, reinterpret_cast<const cplx*>(R),
                       reinterpret_cast<cplx*>(X));
    SPS_CHECK_LAUNCH();
  }
  void timer_enable(int kind, bool on) override {
    SPS_REQUIRE(kind == 0, "unknown timer kind");
    timer_.enable(on);
  }
  void timer_read(long long* launches, double* ms) override { timer_.read(launches, ms); }
  int device_error() override {
    int h = 0;
    SPS_HIP(hipMemcpyAsync(&h, err_, sizeof(int), hipMemcpyDeviceToHost, stream));
    SPS_HIP(hipStreamSynchronize(stream));
    if (h) SPS_HIP(hipMemsetAsync(err_, 0, sizeof(int), stream));
    return h;
  }
  void tuning(int* col_tile, int* row_tile, int* blocks, int* threads, double* tuned_ms) const {
    *threads = nt_;
    for (int k = 0; k < 4; ++k) {
      col_tile[k] = tc_by_size_[k];
      row_tile[k] = trp_by_size_[k];
    }
    *blocks = blocks_;
    *tuned_ms = tuned_ms_;
  }

 private:
  // ---------------------------------------------------------------- set-up
  int plan_of(int n) {
    for (size_t p = 0; p < plan_len_.size(); ++p)
      if (plan_len_[p] == n) return (int)p;
    FftPlan pl{};
    SPS_REQUIRE(fft_plan(n, &pl), "instance sizes must factor into 2 and 3");
    plan_len_.push_back(n);
    plans_h_.push_back(pl);
    return (int)plans_h_.size() - 1;
  }
  void build_plans() {
    inst_.resize(batch_);
    for (int i = 0; i < batch_; ++i) {
      inst_[i].N = ns_[i];
      inst_[i].Nh = ns_[i] / 2;
      inst_[i].Ng = 2 * ns_[i];
      inst_[i].r = rs_[i];
      inst_[i].pn = plan_of(ns_[i]);
      inst_[i].png = plan_of(2 * ns_[i]);
    }
    std::vector<double2> tw;
    std::vector<int> off;
    for (int n : plan_len_) {
      off.push_back((int)tw.size());
      const auto t = twiddles(n);
      tw.insert(tw.end(), t.begin(), t.end());
    }
    dv_.nplan = (int)plans_h_.size();
    dv_.plans = arena_.upload(plans_h_, stream);
    dv_.tw = arena_.upload(tw, stream);
    dv_.twoff = arena_.upload(off, stream);
  }
  void layout() {
    long long so = 0, go = 0, wk = 0;
    for (int i = 0; i < batch_; ++i) {
      ShInst& I = inst_[i];
      const long long st = (long long)I.Nh * I.N, pg = (long long)I.Nh * I.Ng;
      I.so = so;
      I.go = go;
      so += st;
      go += (long long)I.N * I.N;
      I.xo = wk; wk += (max_steps_ + 2) * st;   // X_0 .. X_max, plus a spare slot
      I.fo = wk; wk += 2 * st;
      I.yo = wk; wk += st;
      I.lo = wk; wk += st;
      I.bo = wk; wk += st;
      I.zo = wk; wk += pg;
      I.z2o = wk; wk += pg;
      I.wo = wk; wk += pg;
    }
    state_cplx_ = so;
    work_ = arena_.alloc<cplx>(wk);
    tmp_ = arena_.alloc<cplx>(so);
    dv_.batch = batch_;
    dv_.lx = lx_;
    dv_.dt = dt_;
    dv_.work = work_;
  }
  size_t init_lds(bool rows_adj) const {
    size_t m = 0;
    for (const auto& I : inst_) {
      size_t b = sizeof(cplx) * (I.N + 2 * fpad_size(INIT_TILE * I.N) + (rows_adj ? 2 * INIT_TILE * I.Nh : 0));
      m = std::max(m, b);
    }
    return m;
  }
  dim3 init_grid() const {
    int t = 0;
    for (const auto& I : inst_) t = std::max(t, (I.Nh + INIT_TILE - 1) / INIT_TILE);
    return dim3(batch_, t);
  }
  static size_t col_lds(const ShInst& I, int tc) { return sizeof(cplx) * (I.Ng + 2 * fpad_size(2 * tc * I.Ng)); }
  static size_t row_lds(const ShInst& I, int trp) {
    return sizeof(cplx) * (I.Ng + 2 * 2 * trp * I.Nh + 2 * fpad_size(2 * trp * I.Ng));
  }
  static int size_class(int N) { return N <= 64 ? 0 : N <= 96 ? 1 : N <= 128 ? 2 : 3; }

  // Work items for tiles (tc, trp) per size class and a block count: longest-first
  // assignment of the items of each phase to the least-loaded block (costs ~ points x log).
  static const void* kernel_of(int nt) {
    return nt == 64 ? (const void*)sh_persistent<64> : nt == 128 ? (const void*)sh_persistent<128>
                                                                  : (const void*)sh_persistent<256>;
  }
  void schedule(const int* tcs, const int* trps, int blocks, int nt) {
    nt_ = nt;
    lds_ = 0;
    for (auto& I : inst_) {
      I.tc = tcs[size_class(I.N)];
      I.trp = trps[size_class(I.N)];
      lds_ = std::max({lds_, col_lds(I, I.tc), row_lds(I, I.trp), sizeof(double) * nt});
    }
    struct It {
      double cost;
      int inst, first;
    };
    auto assign = [&](std::vector<It>& items, std::vector<int>& ptr, std::vector<int2>& list) {
      std::sort(items.begin(), items.end(), [](const It& a, const It& b) { return a.cost > b.cost; });
      std::vector<double> load(blocks, 0.0);
      std::vector<std::vector<int2>> per(blocks);
      for (const auto& it : items) {
        const int b = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        load[b] += it.cost;
        per[b].push_back(make_int2(it.inst, it.first));
      }
      ptr.assign(blocks + 1, 0);
      list.clear();
      for (int b = 0; b < blocks; ++b) {
        ptr[b + 1] = ptr[b] + (int)per[b].size();
        list.insert(list.end(), per[b].begin(), per[b].end());
      }
    };
    std::vector<It> ci, ri, ji;
    for (int i = 0; i < batch_; ++i) {
      const ShInst& I = inst_[i];
      const double lg = std::log2((double)I.Ng);
      for (int c = 0; c < I.Nh; c += I.tc) ci.push_back({std::min(I.tc, I.Nh - c) * I.Ng * lg + 2000.0, i, c});
      for (int p = 0; p < I.Ng / 2; p += I.trp) ri.push_back({std::min(I.trp, I.Ng / 2 - p) * I.Ng * lg + 2000.0, i, p});
      ji.push_back({(double)I.N * I.N, i, 0});
    }
    std::vector<int> cptr, rptr, jptr;
    std::vector<int2> cl, rl, jl;
    assign(ci, cptr, cl);
    assign(ri, rptr, rl);
    assign(ji, jptr, jl);
    std::vector<int> jlist;
    for (const auto& v : jl) jlist.push_back(v.x);
    // the previous candidate's arrays are released (hipFree waits for the device)
    sched_.reset(new Sched());
    sched_->upload(stream, inst_, cptr, cl, rptr, rl, jptr, jlist);
    dv_.inst = sched_->inst;
    dv_.cptr = sched_->cptr;
    dv_.citem = sched_->citem;
    dv_.rptr = sched_->rptr;
    dv_.ritem = sched_->ritem;
    dv_.jptr = sched_->jptr;
    dv_.jitem = sched_->jitem;
    blocks_ = blocks;
  }

  // Tuning: tile widths (columns per column item, row pairs per row item) for each size
  // class and the number of persistent blocks; each candidate that fits LDS and co-residency
  // is timed on a few forward steps of this batch and the fastest is kept.
  void tune() {
    const int cand[4] = {256, 512, 1024, 2048};   // points of one FFT batch (tile x Ng)
    const int cand_nt[3] = {64, 128, 256};
    const int Ngs[4] = {128, 192, 256, 384};
    double best = 1e30;
    int best_tc[4] = {1, 1, 1, 1}, best_trp[4] = {1, 1, 1, 1}, best_blocks = cus_, best_nt = 256;
    const int nsteps = std::min(4, max_steps_);
    // the timing events are destroyed on every exit from the tuner, also by an exception
    struct Events {
      hipEvent_t e[2] = {nullptr, nullptr};
      ~Events() {
        for (hipEvent_t x : e)
          if (x) (void)hipEventDestroy(x);
      }
    } ev;
    SPS_HIP(hipEventCreate(&ev.e[0]));
    SPS_HIP(hipEventCreate(&ev.e[1]));
    hipEvent_t e0 = ev.e[0], e1 = ev.e[1];
    for (int nt : cand_nt)
      for (int bc : cand)
        for (int br : cand)
          for (int bmul = 1; bmul <= 4; ++bmul) {
            int tcs[4], trps[4];
            for (int k = 0; k < 4; ++k) {
              tcs[k] = std::max(1, std::min(8, bc / Ngs[k]));
              trps[k] = std::max(1, std::min(8, br / Ngs[k]));
              while (tcs[k] & (tcs[k] - 1)) --tcs[k];
              while (trps[k] & (trps[k] - 1)) --trps[k];
            }
            const int blocks = bmul * cus_;
            schedule(tcs, trps, blocks, nt);
            if (lds_ > 160 * 1024 || !fits(blocks)) continue;
            ShRun a{RUN_FWD, nsteps, tmp_, nullptr, nullptr, nullptr, nullptr, nullptr};
            SPS_HIP(hipMemsetAsync(tmp_, 0, sizeof(cplx) * state_cplx_, stream));
            run(a);   // warm
            SPS_HIP(hipEventRecord(e0, stream));
            run(a);
            SPS_HIP(hipEventRecord(e1, stream));
            SPS_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            SPS_HIP(hipEventElapsedTime(&ms, e0, e1));
            if (check_error()) throw Error(SPS_E_HIP, "persistent launch aborted while tuning");
            if (ms < best) {
              best = ms;
              std::copy(tcs, tcs + 4, best_tc);
              std::copy(trps, trps + 4, best_trp);
              best_blocks = blocks;
              best_nt = nt;
            }
          }
    SPS_REQUIRE(best < 1e29, "no tile configuration fits this batch");
    schedule(best_tc, best_trp, best_blocks, best_nt);
    std::copy(best_tc, best_tc + 4, tc_by_size_);
    std::copy(best_trp, best_trp + 4, trp_by_size_);
    tuned_ms_ = best / nsteps;
  }
  bool fits(int blocks) {
    int per = 0;
    const void* k = kernel_of(nt_);
    SPS_HIP(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_));
    SPS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k, nt_, lds_));
    return per * cus_ >= blocks;
  }
  int check_error() {
    int h = 0;
    SPS_HIP(hipMemcpyAsync(&h, err_, sizeof(int), hipMemcpyDeviceToHost, stream));
    SPS_HIP(hipStreamSynchronize(stream));
    return h & 4;
  }
  void copy_into_history(int n) {
    // tmp_ (state layout) -> history slot n of every instance (used by the stand-alone cost)
    for (const auto& I : inst_)
      SPS_HIP(hipMemcpyAsync(work_ + I.xo + (long long)n * I.Nh * I.N, tmp_ + I.so, sizeof(cplx) * I.Nh * I.N,
                             hipMemcpyDeviceToDevice, stream));
  }
  void run(const ShRun& a) {
    const void* k = kernel_of(nt_);
    SPS_HIP(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_));
    SPS_HIP(hipMemsetAsync(bar_, 0, sizeof(unsigned), stream));
    dv_.bar = bar_;
    dv_.err = err_;
    ShDev d = dv_;
    ShRun r = a;
    void* args[] = {&d, &r};
    hipEvent_t e0, e1;
    const bool timed = timer_.take(&e0, &e1);
    if (timed) SPS_HIP(hipEventRecord(e0, stream));
    SPS_HIP(hipLaunchCooperativeKernel(k, dim3(blocks_), dim3(nt_), args, lds_, stream));
    if (timed) SPS_HIP(hipEventRecord(e1, stream));
  }

  // device copies of one schedule (instances with their tiles, item lists per block)
  struct Sched {
    DevArena arena;
    ShInst* inst = nullptr;
    int *cptr = nullptr, *rptr = nullptr, *jptr = nullptr, *jitem = nullptr;
    int2 *citem = nullptr, *ritem = nullptr;
    void upload(hipStream_t s, const std::vector<ShInst>& in, const std::vector<int>& cp, const std::vector<int2>& cl,
                const std::vector<int>& rp, const std::vector<int2>& rl, const std::vector<int>& jp,
                const std::vector<int>& jl) {
      inst = arena.upload(in, s);
      cptr = arena.upload(cp, s);
      citem = arena.upload(cl, s);
      rptr = arena.upload(rp, s);
      ritem = arena.upload(rl, s);
      jptr = arena.upload(jp, s);
      jitem = arena.upload(jl, s);
    }
  };

  int batch_ = 0, max_steps_ = 0, cus_ = 0, blocks_ = 0, nt_ = 256;
  double lx_ = 0, dt_ = 0, tuned_ms_ = 0;
  std::vector<int> ns_;
  std::vector<double> rs_;
  std::vector<ShInst> inst_;
  std::vector<int> plan_len_;
  std::vector<FftPlan> plans_h_;
  int tc_by_size_[4] = {0, 0, 0, 0}, trp_by_size_[4] = {0, 0, 0, 0};
  size_t lds_ = 0;
  long long state_cplx_ = 0;
  ShDev dv_{};
  DevArena arena_;
  std::unique_ptr<Sched> sched_;
  cplx *work_ = nullptr, *tmp_ = nullptr;
  unsigned* bar_ = nullptr;
  int* err_ = nullptr;
  int tape_steps_ = -1;
  KernelTimer timer_;
};

}  // namespace

ProblemImpl* make_sh_batch(int batch, const int* n, const double* r, double lx, double dt, int max_steps,
                           hipStream_t s) {
  return new ShProblem(batch, n, r, lx, dt, max_steps, s);
}

void sh_tuning(ProblemImpl* p, int* col_tile, int* row_tile, int* blocks, int* threads, double* tuned_ms) {
  auto* sh = dynamic_cast<ShProblem*>(p);
  if (!sh) throw Error(SPS_E_ARG, "not a batched Swift-Hohenberg problem");
  sh->tuning(col_tile, row_tile, blocks, threads, tuned_ms);
}

}  // namespace sps
