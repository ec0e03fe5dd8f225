// 1D Kuramoto-Sivashinsky equation u_t + u_xx + u_xxxx + u u_x = 0 on a periodic interval,
// in the IVP form M dX/dt + L X = F(X) (Supplementary, "Initial value problems") with one
// unknown per stored Fourier mode m < K = nx/2: M = 1, L_m = -k_m^2 + k_m^4,
// F = -1/2 d/dx(u^2) with the product on the 3/2 grid (Methods, dealiasing).  Timestepping is
// SBDF-k, k = 2, 3 or 4, reverting to SBDF-n on the first k - 1 steps (equ:imex), with the
// multistep adjoint recurrence (equ:IMEX_adjoint) as reverse sweep, or the IMEX Runge-Kutta
// schemes ARS(2,2,2) and ARS(4,4,3) with the RK adjoint equations (Supplementary, "Initial value
// problems").  The implicit matrices are diagonal, so a whole sweep is
// one block that loops over the steps (a persistent launch) and keeps the per-mode history
// in registers; the states of the run are stored for the reverse sweep.
#include <hip/hip_runtime.h>
#include <math.h>

#include <vector>

#include "sps_device.h"
#include "sps_internal.h"

namespace sps {
namespace {

constexpr int NTS = 256;  // threads of every KS block

struct KsDev {
  int K, Ng;
  const double* kx;   // [K] k_m = 2 pi m / L
  const double* lin;  // [K] L_m = -k_m^2 + k_m^4
  const cplx* ex;     // [Ng] exp(2 pi i t / Ng)
};

// Multistep coefficients of step n (equ:imex): (a_0 M + L) X_n = sum_i c_i F_{n-i} - a_i M X_{n-i},
// i = 1..4 (zero beyond the order): SBDF-k at a constant step (the k-step backward difference
// of M dX/dt and the k-th order extrapolation of F), SBDF-n while n < k.
constexpr int KS_MAX_ORDER = 4;
struct SbdfCoef {
  double a[KS_MAX_ORDER + 1];
  double c[KS_MAX_ORDER + 1];   // c[0] unused
};
__host__ __device__ __forceinline__ SbdfCoef sbdf_coef(int n, int order, double dt) {
  const int q = n < order ? n : order;
  SbdfCoef r;
  for (int i = 0; i <= KS_MAX_ORDER; ++i) r.a[i] = r.c[i] = 0.0;
  if (q <= 1) {
    r.a[0] = 1.0; r.a[1] = -1.0;
    r.c[1] = 1.0;
  } else if (q == 2) {
    r.a[0] = 1.5; r.a[1] = -2.0; r.a[2] = 0.5;
    r.c[1] = 2.0; r.c[2] = -1.0;
  } else if (q == 3) {
    r.a[0] = 11.0 / 6.0; r.a[1] = -3.0; r.a[2] = 1.5; r.a[3] = -1.0 / 3.0;
    r.c[1] = 3.0; r.c[2] = -3.0; r.c[3] = 1.0;
  } else {
    r.a[0] = 25.0 / 12.0; r.a[1] = -4.0; r.a[2] = 3.0; r.a[3] = -4.0 / 3.0; r.a[4] = 0.25;
    r.c[1] = 4.0; r.c[2] = -6.0; r.c[3] = 4.0; r.c[4] = -1.0;
  }
  for (int i = 0; i <= KS_MAX_ORDER; ++i) r.a[i] = r.a[i] / dt;
  return r;
}
// Row of step n for step sizes h (h[i] = t_{i+1} - t_i; step n advances from t_{n-1} by
// h[n-1]): with q = min(n, order) and the nodes tau_j = t_{n-j} - t_n, j = 0..q, a_j is the
// derivative at tau = 0 of the Lagrange basis polynomial of node j on tau_0..tau_q (the
// q-step backward difference of dX/dt at t_n) and c_i the value at 0 of the basis polynomial
// of node i on tau_1..tau_q (extrapolation of F).  Equal steps give the rows of sbdf_coef.
SbdfCoef sbdf_row_variable(const double* h, int n, int order) {
  const int q = n < order ? n : order;
  double tau[KS_MAX_ORDER + 1];
  tau[0] = 0.0;
  for (int j = 1; j <= q; ++j) tau[j] = tau[j - 1] - h[n - j];
  SbdfCoef r;
  for (int i = 0; i <= KS_MAX_ORDER; ++i) r.a[i] = r.c[i] = 0.0;
  for (int j = 0; j <= q; ++j) {
    double d = 0.0;
    for (int k = 0; k <= q; ++k) {
      if (k == j) continue;
      double p = 1.0 / (tau[j] - tau[k]);
      for (int m = 0; m <= q; ++m)
        if (m != j && m != k) p *= (0.0 - tau[m]) / (tau[j] - tau[m]);
      d += p;
    }
    r.a[j] = d;
  }
  for (int i = 1; i <= q; ++i) {
    double p = 1.0;
    for (int m = 1; m <= q; ++m)
      if (m != i) p *= (0.0 - tau[m]) / (tau[i] - tau[m]);
    r.c[i] = p;
  }
  return r;
}

// Grid values from half-spectrum coefficients (LDS), W = 2 for the real field
// u_j = Re c_0 + 2 sum_{m>=1} Re(c_m e^{2 pi i j m / Ng}), W = 1 for the transposed forward
// transform (unweighted).  Two series at once (b may be null).  Two lanes (an aligned pair,
// h = 0, 1) per grid point, lane h summing the modes m = 1 + h, 3 + h, ...; both lanes of the
// pair return the values.  Block-wide, no barrier.
__device__ __forceinline__ void ks_grid_point(const KsDev& d, const cplx* ex, const cplx* a, double Wa,
                                              const cplx* b, double Wb, int j, int h, double& ua, double& ub) {
  const int Ng = d.Ng;
  int t = (int)(((long long)(1 + h) * j) % Ng);
  const int st = (2 * j) % Ng;
  double sa = 0.0, sb = 0.0;
  for (int m = 1 + h; m < d.K; m += 2) {
    const cplx e = ex[t];
    sa = fma(a[m].x, e.x, fma(-a[m].y, e.y, sa));
    if (b) sb = fma(b[m].x, e.x, fma(-b[m].y, e.y, sb));
    t += st;
    if (t >= Ng) t -= Ng;
  }
  sa = group_sum<2>(sa);
  if (b) sb = group_sum<2>(sb);
  ua = a[0].x + Wa * sa;
  ub = b ? b[0].x + Wb * sb : 0.0;
}

// sum_j v_j e^{-2 pi i j m / Ng} over the grid, eight lanes (an aligned group, h = 0..7) per
// mode; every lane of the group returns the sum.
constexpr int KS_MG = 8;
__device__ __forceinline__ cplx ks_mode_sum(const KsDev& d, const cplx* ex, const double* v, int m, int h) {
  const int Ng = d.Ng;
  int t = (h * m) % Ng;
  const int st = (KS_MG * m) % Ng;
  double sr = 0.0, si = 0.0;
  for (int j = h; j < Ng; j += KS_MG) {
    const cplx e = ex[t];
    sr = fma(v[j], e.x, sr);
    si = fma(-v[j], e.y, si);
    t += st;
    if (t >= Ng) t -= Ng;
  }
  return group_sum<KS_MG>(cmk(sr, si));
}

// F(X) for X in LDS c; result fo[m] (LDS).  u: Ng doubles scratch.  Starts after a barrier
// that made c visible; ends with a barrier.
__device__ void ks_eval_F(const KsDev& d, const cplx* ex, const cplx* c, double* u, cplx* fo) {
  for (int e = threadIdx.x; e < 2 * d.Ng; e += NTS) {
    const int j = e >> 1;
    double v, unused;
    ks_grid_point(d, ex, c, 2.0, nullptr, 0.0, j, e & 1, v, unused);
    if ((e & 1) == 0) u[j] = v * v;
  }
  __syncthreads();
  const double inv = 1.0 / d.Ng;
  for (int e = threadIdx.x; e < KS_MG * d.K; e += NTS) {
    const int m = e / KS_MG, h = e % KS_MG;
    const cplx s = ks_mode_sum(d, ex, u, m, h);
    const double k = d.kx[m];
    // -1/2 i k (s / Ng)
    if (h == 0) fo[m] = cmk(0.5 * k * s.y * inv, -0.5 * k * s.x * inv);
  }
  __syncthreads();
}

// Vector-Jacobian product of F at X (LDS c) with cotangent G (LDS g): sqbar = (1/2) i k G,
// ubar_j = 2 u_j (1/Ng) sum_m Re(sqbar_m e^{i theta_jm}), Xbar_m = w_m sum_j ubar_j e^{-i theta_jm}
// (w_0 = 1, w_m = 2).  sb: K, u: Ng scratch; result xo[m].  Starts after a barrier that made
// c and g visible; ends with a barrier.
__device__ void ks_F_vjp(const KsDev& d, const cplx* ex, const cplx* c, const cplx* g, cplx* sb, double* u,
                         cplx* xo) {
  const int tid = threadIdx.x;
  if (tid < d.K) {
    const double k = d.kx[tid];
    sb[tid] = cmk(-0.5 * k * g[tid].y, 0.5 * k * g[tid].x);
  }
  __syncthreads();
  const double inv = 1.0 / d.Ng;
  for (int e = tid; e < 2 * d.Ng; e += NTS) {
    const int j = e >> 1;
    double uj, rj;
    ks_grid_point(d, ex, c, 2.0, sb, 1.0, j, e & 1, uj, rj);
    if ((e & 1) == 0) u[j] = 2.0 * uj * rj * inv;
  }
  __syncthreads();
  for (int e = tid; e < KS_MG * d.K; e += NTS) {
    const int m = e / KS_MG, h = e % KS_MG;
    const cplx s = ks_mode_sum(d, ex, u, m, h);
    if (h == 0) xo[m] = cscale(s, m == 0 ? 1.0 : 2.0);
  }
  __syncthreads();
}

// IMEX RK tableau with S implicit stages past the initial one: explicit part A and implicit
// part H, (S+1) x (S+1), lower triangular, row i giving stage i; X_{n+1} is stage S.
struct RkTab {
  double A[5][5];
  double H[5][5];
};

// LDS of every KS kernel: ex (Ng), c, g, sb, fo (K each), u (Ng doubles)
struct KsLds {
  cplx *ex, *c, *g, *sb, *fo;
  double* u;
};
__device__ __forceinline__ KsLds ks_lds(const KsDev& d, double* smem) {
  KsLds L;
  L.ex = reinterpret_cast<cplx*>(smem);
  L.c = L.ex + d.Ng;
  L.g = L.c + d.K;
  L.sb = L.g + d.K;
  L.fo = L.sb + d.K;
  L.u = reinterpret_cast<double*>(L.fo + d.K);
  for (int t = threadIdx.x; t < d.Ng; t += NTS) L.ex[t] = d.ex[t];
  return L;
}

// Forward sweep: X (in: X_0, out: X_N), history H[n][K] of X_0 .. X_N.  One block.
// rows[n]: the coefficients of step n (device array, rows beyond the run zero)
__global__ void __launch_bounds__(NTS) ks_forward(KsDev d, cplx* X, cplx* H, int nsteps, const SbdfCoef* rows,
                                                 int* err) {
  extern __shared__ double smem_d[];
  const KsLds L = ks_lds(d, smem_d);
  const int m = threadIdx.x, K = d.K;
  const bool own = m < K;
  const double lin = own ? d.lin[m] : 0.0;
  // x[i] = X_{n-1-i}, f[i] = F(X_{n-1-i}) of this mode (zero before X_0)
  cplx x[KS_MAX_ORDER], f[KS_MAX_ORDER];
#pragma unroll
  for (int i = 0; i < KS_MAX_ORDER; ++i) x[i] = f[i] = czero();
  x[0] = own ? X[m] : czero();
  if (own) {
    H[m] = x[0];
    L.c[m] = x[0];
  }
  __syncthreads();
  ks_eval_F(d, L.ex, L.c, L.u, L.fo);
  if (own) f[0] = L.fo[m];
  for (int n = 1; n <= nsteps; ++n) {
    const SbdfCoef q = rows[n];
    cplx fs = czero(), xs = czero();
#pragma unroll
    for (int i = 1; i <= KS_MAX_ORDER; ++i) {
      fs = cadd(fs, cscale(f[i - 1], q.c[i]));
      xs = cadd(xs, cscale(x[i - 1], q.a[i]));
    }
    const cplx xn = cscale(csub(fs, xs), 1.0 / (q.a[0] + lin));
    if (own) {
      H[(size_t)n * K + m] = xn;
      L.c[m] = xn;
    }
#pragma unroll
    for (int i = KS_MAX_ORDER - 1; i > 0; --i) {
      x[i] = x[i - 1];
      f[i] = f[i - 1];
    }
    x[0] = xn;
    if (n < nsteps) {
      __syncthreads();
      ks_eval_F(d, L.ex, L.c, L.u, L.fo);
      if (own) f[0] = L.fo[m];
    }
  }
  if (own) {
    const cplx x1 = x[0];
    X[m] = x1;
    if (__any(!(isfinite(x1.x) && isfinite(x1.y))) && lane_id() == 0) atomicOr(err, 2);
  }
}

// Reverse sweep: Xbar (in: dJ/dX_N, out: dJ/dX_0) through the history H of the forward run.
// The cotangent of X_{n-1} collects Y_{n-1+i} from steps n-1+i, i = 1..order (equ:IMEX_adjoint),
// so it is complete once Y_n is known; F's VJP, linear in its cotangent, is applied once per
// state.  Y of steps beyond nsteps are zero.
__global__ void __launch_bounds__(NTS) ks_adjoint(KsDev d, cplx* Xbar, const cplx* H, int nsteps,
                                                 const SbdfCoef* rows) {
  extern __shared__ double smem_d[];
  const KsLds L = ks_lds(d, smem_d);
  const int m = threadIdx.x, K = d.K;
  const bool own = m < K;
  const double lin = own ? d.lin[m] : 0.0;
  cplx xb = own ? Xbar[m] : czero();   // cotangent of X_n (complete)
  cplx ys[KS_MAX_ORDER - 1];           // Y_{n+1}, Y_{n+2}, Y_{n+3}
#pragma unroll
  for (int i = 0; i < KS_MAX_ORDER - 1; ++i) ys[i] = czero();
  cplx hnext = (own && nsteps >= 1) ? H[(size_t)(nsteps - 1) * K + m] : czero();
  for (int n = nsteps; n >= 1; --n) {
    const SbdfCoef q = rows[n];
    const cplx y = cscale(xb, 1.0 / (q.a[0] + lin));
    cplx g = cscale(y, q.c[1]);
    cplx lin_part = cscale(y, q.a[1]);
#pragma unroll
    for (int i = 2; i <= KS_MAX_ORDER; ++i) {
      const SbdfCoef qi = rows[n - 1 + i];   // step n-1+i, its term i
      g = cadd(g, cscale(ys[i - 2], qi.c[i]));
      lin_part = cadd(lin_part, cscale(ys[i - 2], qi.a[i]));
    }
    const cplx hcur = hnext;
    if (own && n >= 2) hnext = H[(size_t)(n - 2) * K + m];   // next iteration's state, early
    if (own) {
      L.c[m] = hcur;
      L.g[m] = g;
    }
    __syncthreads();
    ks_F_vjp(d, L.ex, L.c, L.g, L.sb, L.u, L.fo);
    xb = own ? csub(L.fo[m], lin_part) : czero();
#pragma unroll
    for (int i = KS_MAX_ORDER - 2; i > 0; --i) ys[i] = ys[i - 1];
    ys[0] = y;
  }
  if (own) Xbar[m] = xb;
}

// RK forward sweep, S stages, step dt0 or dts[n] for step n + 1 (dts: device array, nullable):
// X (in: X_0, out: X_N); the stage states X_{n,0..S-1} of step n at
// H[(n S + i) K] for the reverse sweep.  Stage i solves
// (1 + dt H_ii L_m) X_{n,i} = X_{n,0} + dt sum_{j<i} (A_ij F_{n,j} - H_ij L_m X_{n,j}) per mode
// (M = 1); F of stage S is not needed (column S of A is zero).  One block; the stage values of
// this thread's mode stay in registers.
template <int S>
__global__ void __launch_bounds__(NTS) ks_forward_rk(KsDev d, cplx* X, cplx* H, int nsteps, RkTab tab, double dt0,
                                                    const double* dts, int* err) {
  extern __shared__ double smem_d[];
  const KsLds L = ks_lds(d, smem_d);
  const int m = threadIdx.x, K = d.K;
  const bool own = m < K;
  const double lin = own ? d.lin[m] : 0.0;
  double inv[S + 1];
  cplx x0 = own ? X[m] : czero();
  for (int n = 0; n < nsteps; ++n) {
    const double dt = dts ? dts[n] : dt0;   // step n + 1 advances by dts[n]
    if (n == 0 || dts) {
#pragma unroll
      for (int i = 1; i <= S; ++i) inv[i] = 1.0 / (1.0 + dt * tab.H[i][i] * lin);
    }
    cplx xs[S + 1], fs[S];
    xs[0] = x0;
#pragma unroll
    for (int i = 0; i <= S; ++i) {
      if (i > 0) {
        cplx r = xs[0];
#pragma unroll
        for (int j = 0; j < i; ++j) {
          r = cadd(r, cscale(fs[j], dt * tab.A[i][j]));
          r = csub(r, cscale(xs[j], dt * tab.H[i][j] * lin));
        }
        xs[i] = cscale(r, inv[i]);
      }
      if (i < S) {
        if (own) {
          H[((size_t)n * S + i) * K + m] = xs[i];
          L.c[m] = xs[i];
        }
        __syncthreads();
        ks_eval_F(d, L.ex, L.c, L.u, L.fo);
        fs[i] = own ? L.fo[m] : czero();
      }
    }
    x0 = xs[S];
  }
  if (own) {
    X[m] = x0;
    if (__any(!(isfinite(x0.x) && isfinite(x0.y))) && lane_id() == 0) atomicOr(err, 2);
  }
}

// RK reverse sweep: Xbar (in: dJ/dX_N, out: dJ/dX_0) through the stage states of the forward
// run.  Per step, from the cotangent Yn of X_{n+1} (M = 1, L real diagonal, so each implicit
// matrix is its own adjoint):
//   Y_S = Yn / (1 + dt H_SS L),
//   Y_i = [dF(X_{n,i})^H (dt sum_{j>i} A_ji Y_j) - dt L sum_{j>i} H_ji Y_j] / (1 + dt H_ii L),
//   cotangent of X_n = sum_{j>=1} Y_j + dF(X_{n,0})^H (dt sum_j A_j0 Y_j) - dt L sum_j H_j0 Y_j.
template <int S>
__global__ void __launch_bounds__(NTS) ks_adjoint_rk(KsDev d, cplx* Xbar, const cplx* H, int nsteps, RkTab tab,
                                                    double dt0, const double* dts) {
  extern __shared__ double smem_d[];
  const KsLds L = ks_lds(d, smem_d);
  const int m = threadIdx.x, K = d.K;
  const bool own = m < K;
  const double lin = own ? d.lin[m] : 0.0;
  double inv[S + 1];
  cplx yn = own ? Xbar[m] : czero();
  for (int n = nsteps - 1; n >= 0; --n) {
    const double dt = dts ? dts[n] : dt0;
    if (n == nsteps - 1 || dts) {
#pragma unroll
      for (int i = 1; i <= S; ++i) inv[i] = 1.0 / (1.0 + dt * tab.H[i][i] * lin);
    }
    cplx ys[S + 1];
    ys[S] = cscale(yn, inv[S]);
#pragma unroll
    for (int i = S - 1; i >= 0; --i) {
      cplx g = czero(), lp = czero();
#pragma unroll
      for (int j = i + 1; j <= S; ++j) {
        g = cadd(g, cscale(ys[j], dt * tab.A[j][i]));
        lp = cadd(lp, cscale(ys[j], dt * tab.H[j][i] * lin));
      }
      if (own) {
        L.c[m] = H[((size_t)n * S + i) * K + m];
        L.g[m] = g;
      }
      __syncthreads();
      ks_F_vjp(d, L.ex, L.c, L.g, L.sb, L.u, L.fo);
      const cplx v = own ? L.fo[m] : czero();
      if (i > 0) {
        ys[i] = cscale(csub(v, lp), inv[i]);
      } else {
        cplx sum = czero();
#pragma unroll
        for (int j = 1; j <= S; ++j) sum = cadd(sum, ys[j]);
        yn = csub(cadd(sum, v), lp);
      }
    }
  }
  if (own) Xbar[m] = yn;
}

// F or its VJP at one state (one block).
__global__ void __launch_bounds__(NTS) ks_eval(KsDev d, const cplx* X, const cplx* G, cplx* out) {
  extern __shared__ double smem_d[];
  const KsLds L = ks_lds(d, smem_d);
  const int m = threadIdx.x;
  if (m < d.K) {
    L.c[m] = X[m];
    if (G) L.g[m] = G[m];
  }
  __syncthreads();
  if (G) ks_F_vjp(d, L.ex, L.c, L.g, L.sb, L.u, L.fo);
  else ks_eval_F(d, L.ex, L.c, L.u, L.fo);
  if (m < d.K) out[m] = L.fo[m];
}

// J = 1/2 sum_m w_m |c_m|^2 (Parseval of (1/L) int u^2 / 2, c_0 by its real part), dJ/dX = w c.
__global__ void __launch_bounds__(NTS) ks_cost(KsDev d, const cplx* X, cplx* dJ, double* J) {
  __shared__ double red[NTS];
  const int m = threadIdx.x;
  double part = 0.0;
  if (m < d.K) {
    cplx c = X[m];
    if (m == 0) c.y = 0.0;
    const double w = (m == 0) ? 1.0 : 2.0;
    dJ[m] = cscale(c, w);
    part = 0.5 * w * (c.x * c.x + c.y * c.y);
  }
  red[m] = part;
  __syncthreads();
  for (int s = NTS / 2; s > 0; s >>= 1) {
    if (m < s) red[m] += red[m + s];
    __syncthreads();
  }
  if (J && m == 0) J[0] = red[0];
}

// X = (a_0 M + b L)^{-1} R: the scheme's implicit matrix, a_0 the steady SBDF-k a_0 (3/2, 11/6
// or 25/12 over dt) with b = 1, or a_0 = 1 and b = dt gamma for the RK schemes (real diagonal,
// so equal to its adjoint).
__global__ void __launch_bounds__(NTS) ks_solve(KsDev d, const cplx* R, cplx* X, double a0, double b) {
  const int m = threadIdx.x;
  if (m < d.K) X[m] = cscale(R[m], 1.0 / (a0 + b * d.lin[m]));
}

// ARS(2,2,2) (gamma = 1 - 1/sqrt 2, delta = 1 - 1/(2 gamma)) and ARS(4,4,3) of Ascher, Ruuth &
// Spiteri (1997).
RkTab rk_tableau(int scheme, int* stages) {
  RkTab t;
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j < 5; ++j) t.A[i][j] = t.H[i][j] = 0.0;
  if (scheme == SPS_RK222) {
    const double g = 1.0 - 1.0 / std::sqrt(2.0), dl = 1.0 - 1.0 / (2.0 * g);
    t.A[1][0] = g;
    t.A[2][0] = dl; t.A[2][1] = 1.0 - dl;
    t.H[1][1] = g;
    t.H[2][1] = 1.0 - g; t.H[2][2] = g;
    *stages = 2;
  } else {
    t.A[1][0] = 0.5;
    t.A[2][0] = 11.0 / 18.0; t.A[2][1] = 1.0 / 18.0;
    t.A[3][0] = 5.0 / 6.0; t.A[3][1] = -5.0 / 6.0; t.A[3][2] = 0.5;
    t.A[4][0] = 0.25; t.A[4][1] = 1.75; t.A[4][2] = 0.75; t.A[4][3] = -1.75;
    t.H[1][1] = 0.5;
    t.H[2][1] = 1.0 / 6.0; t.H[2][2] = 0.5;
    t.H[3][1] = -0.5; t.H[3][2] = 0.5; t.H[3][3] = 0.5;
    t.H[4][1] = 1.5; t.H[4][2] = -1.5; t.H[4][3] = 0.5; t.H[4][4] = 0.5;
    *stages = 4;
  }
  return t;
}

class KsProblem : public ProblemImpl {
 public:
  KsProblem(const sps_desc& desc, hipStream_t s) : desc_(desc) {
    stream = s;
    SPS_REQUIRE(desc.scheme == SPS_SBDF2 || desc.scheme == SPS_SBDF3 || desc.scheme == SPS_SBDF4 ||
                    desc.scheme == SPS_RK222 || desc.scheme == SPS_RK443,
                "KS supports the SBDF2, SBDF3, SBDF4, RK222 and RK443 schemes");
    rk_ = desc.scheme == SPS_RK222 || desc.scheme == SPS_RK443;
    if (rk_) tab_ = rk_tableau(desc.scheme, &stages_);
    else order_ = desc.scheme - SPS_SBDF2 + 2;
    SPS_REQUIRE(desc.nx >= 4 && desc.nx % 2 == 0 && desc.nx / 2 <= NTS, "nx must be even, 4 <= nx <= 512");
    SPS_REQUIRE(desc.dealias == 1.5, "KS uses 3/2 dealiasing");
    SPS_REQUIRE(desc.lx > 0 && desc.dt > 0 && desc.max_steps >= 1, "bad lx / dt / max_steps");
    K_ = desc.nx / 2;
    Ng_ = 3 * desc.nx / 2;
    std::vector<double> kx(K_), lin(K_);
    for (int m = 0; m < K_; ++m) {
      kx[m] = 2.0 * M_PI * m / desc.lx;
      lin[m] = -kx[m] * kx[m] + kx[m] * kx[m] * kx[m] * kx[m];
    }
    std::vector<double2> ex(Ng_);
    const long double tau = 6.28318530717958647692528676655900577L;
    for (int t = 0; t < Ng_; ++t) {
      const long double a = tau * (long double)t / (long double)Ng_;
      ex[t] = make_double2((double)cosl(a), (double)sinl(a));
    }
    dv_.K = K_;
    dv_.Ng = Ng_;
    dv_.kx = arena_.upload(kx, stream);
    dv_.lin = arena_.upload(lin, stream);
    dv_.ex = arena_.upload(ex, stream);
    // history: X_0 .. X_N (SBDF) or the stage states X_{n,0..S-1} of every step (RK)
    H_ = arena_.alloc<cplx>((size_t)(rk_ ? (size_t)desc.max_steps * stages_ : desc.max_steps + 1) * K_);
    Xw_ = arena_.alloc<cplx>(K_);
    err_ = arena_.alloc<int>(1);
    nrows_ = desc.max_steps + KS_MAX_ORDER + 2;
    rows_ = arena_.alloc<SbdfCoef>(nrows_);
    SPS_HIP(hipMemsetAsync(err_, 0, sizeof(int), stream));
    upload_rows(0, nullptr);
  }

  // Rows of the run: the constant-step rows of desc.dt (dts null), or the variable-step rows of
  // the step sizes dts[0..n-1]; rows past the last step are zero (the adjoint reads up to
  // KS_MAX_ORDER - 1 of them, against zero cotangents).
  void upload_rows(int n, const double* dts) {
    hrows_.assign(nrows_, SbdfCoef{});
    for (auto& r : hrows_)
      for (int i = 0; i <= KS_MAX_ORDER; ++i) r.a[i] = r.c[i] = 0.0;
    if (!dts) {
      for (int m = 1; m <= desc_.max_steps; ++m) hrows_[m] = sbdf_coef(m, order_, desc_.dt);
    } else {
      for (int m = 1; m <= n; ++m) hrows_[m] = sbdf_row_variable(dts, m, order_);
    }
    SPS_HIP(hipMemcpyAsync(rows_, hrows_.data(), sizeof(SbdfCoef) * nrows_, hipMemcpyHostToDevice, stream));
    SPS_HIP(hipStreamSynchronize(stream));
  }
  // A new constant step: the SBDF rows of the constant step (unless variable steps are set) or
  // the RK stage coefficients take it; the recorded run is dropped.
  void set_dt(double dt) override {
    SPS_REQUIRE(std::isfinite(dt) && dt > 0.0, "dt must be positive");
    desc_.dt = dt;
    if (!rk_ && var_n_ == 0) upload_rows(0, nullptr);
    tape_steps_ = -1;
  }
  void set_timesteps(const double* dts, int n) override {
    if (rk_) {
      if (!dts || n == 0) {
        var_n_ = 0;
      } else {
        SPS_REQUIRE(n >= 1 && n <= desc_.max_steps, "the step sequence must have 1 .. max_steps entries");
        for (int i = 0; i < n; ++i) SPS_REQUIRE(std::isfinite(dts[i]) && dts[i] > 0.0, "step sizes must be positive");
        if (!dts_) dts_ = arena_.alloc<double>(desc_.max_steps);
        SPS_HIP(hipMemcpyAsync(dts_, dts, sizeof(double) * n, hipMemcpyHostToDevice, stream));
        SPS_HIP(hipStreamSynchronize(stream));
        var_n_ = n;
      }
      tape_steps_ = -1;
      return;
    }
    if (!dts || n == 0) {
      upload_rows(0, nullptr);
      var_n_ = 0;
    } else {
      SPS_REQUIRE(n >= 1 && n <= desc_.max_steps, "the step sequence must have 1 .. max_steps entries");
      for (int i = 0; i < n; ++i) SPS_REQUIRE(std::isfinite(dts[i]) && dts[i] > 0.0, "step sizes must be positive");
      upload_rows(n, dts);
      var_n_ = n;
    }
    tape_steps_ = -1;
  }

  long long state_size() const override { return 2LL * K_; }
  void factor() override {}   // diagonal: nothing to factor

  void step(double* X, int nsteps) override {
    SPS_REQUIRE(X != nullptr, "X is null");
    SPS_REQUIRE(nsteps >= 1 && nsteps <= (var_n_ ? var_n_ : desc_.max_steps), "nsteps out of range");
    forward(reinterpret_cast<cplx*>(X), nsteps);
  }
  void adjoint_step(double* Xbar, int nsteps) override {
    SPS_REQUIRE(Xbar != nullptr, "Xbar is null");
    if (tape_steps_ != nsteps) throw Error(SPS_E_STATE, "adjoint_step: nsteps does not match the recorded forward run");
    cplx* xb = reinterpret_cast<cplx*>(Xbar);
    if (!rk_)
      hipLaunchKernelGGL(ks_adjoint, dim3(1), dim3(NTS), lds(), stream, dv_, xb, H_, nsteps, rows_);
    else if (stages_ == 2)
      hipLaunchKernelGGL(ks_adjoint_rk<2>, dim3(1), dim3(NTS), lds(), stream, dv_, xb, H_, nsteps, tab_, desc_.dt,
                         rk_dts());
    else
      hipLaunchKernelGGL(ks_adjoint_rk<4>, dim3(1), dim3(NTS), lds(), stream, dv_, xb, H_, nsteps, tab_, desc_.dt,
                         rk_dts());
    SPS_CHECK_LAUNCH();
  }
  void cost(const double* X, double* J, double* dJdX) override {
    SPS_REQUIRE(X && dJdX, "null argument");
    hipLaunchKernelGGL(ks_cost, dim3(1), dim3(NTS), 0, stream, dv_, reinterpret_cast<const cplx*>(X),
                       reinterpret_cast<cplx*>(dJdX), J);
    SPS_CHECK_LAUNCH();
  }
  void gradient(const double* X0, int nsteps, const double* dJdXN, double* XN, double* dJdX0, double* dJdtheta,
                double* J) override {
    SPS_REQUIRE(X0 && dJdX0, "null argument");
    if (dJdtheta) throw Error(SPS_E_UNSUPPORTED, "the KS problem has no parameters to differentiate");
    SPS_REQUIRE(nsteps >= 1 && nsteps <= (var_n_ ? var_n_ : desc_.max_steps), "nsteps out of range");
    SPS_HIP(hipMemcpyAsync(Xw_, X0, sizeof(cplx) * K_, hipMemcpyDeviceToDevice, stream));
    forward(Xw_, nsteps);
    if (XN) SPS_HIP(hipMemcpyAsync(XN, Xw_, sizeof(cplx) * K_, hipMemcpyDeviceToDevice, stream));
    if (dJdXN) {
      if (dJdXN != dJdX0) SPS_HIP(hipMemcpyAsync(dJdX0, dJdXN, sizeof(cplx) * K_, hipMemcpyDeviceToDevice, stream));
    } else {
      cost(reinterpret_cast<const double*>(Xw_), J, dJdX0);
    }
    adjoint_step(dJdX0, nsteps);
  }
  void initial_state(const double*, double*) override {
    throw Error(SPS_E_UNSUPPORTED, "KS states are given as Fourier coefficients");
  }
  void initial_state_adjoint(const double*, double*) override {
    throw Error(SPS_E_UNSUPPORTED, "KS states are given as Fourier coefficients");
  }
  void eval_F(const double* X, double* F) override {
    SPS_REQUIRE(X && F, "null argument");
    hipLaunchKernelGGL(ks_eval, dim3(1), dim3(NTS), lds(), stream, dv_, reinterpret_cast<const cplx*>(X), nullptr,
                       reinterpret_cast<cplx*>(F));
    SPS_CHECK_LAUNCH();
  }
  void eval_F_vjp(const double* X, const double* Fbar, double* Xbar) override {
    SPS_REQUIRE(X && Fbar && Xbar, "null argument");
    hipLaunchKernelGGL(ks_eval, dim3(1), dim3(NTS), lds(), stream, dv_, reinterpret_cast<const cplx*>(X),
                       reinterpret_cast<const cplx*>(Fbar), reinterpret_cast<cplx*>(Xbar));
    SPS_CHECK_LAUNCH();
  }
  void solve(const double* R, double* X, int) override {
    SPS_REQUIRE(R && X, "null argument");
    const double a0 = rk_ ? 1.0 : sbdf_coef(order_, order_, desc_.dt).a[0];
    const double b = rk_ ? desc_.dt * tab_.H[1][1] : 1.0;
    hipLaunchKernelGGL(ks_solve, dim3(1), dim3(NTS), 0, stream, dv_, reinterpret_cast<const cplx*>(R),
                       reinterpret_cast<cplx*>(X), a0, b);
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

 private:
  size_t lds() const { return sizeof(cplx) * (Ng_ + 4 * K_) + sizeof(double) * Ng_; }
  const double* rk_dts() const { return var_n_ ? dts_ : nullptr; }
  // one-block sweep launch, bracketed by the timer's events while it records
  template <typename... P, typename... A>
  void launch_timed(void (*kern)(P...), A... args) {
    hipEvent_t e0, e1;
    if (timer_.take(&e0, &e1))
      hipExtLaunchKernelGGL(kern, dim3(1), dim3(NTS), lds(), stream, e0, e1, 0, args...);
    else
      hipLaunchKernelGGL(kern, dim3(1), dim3(NTS), lds(), stream, args...);
  }
  void forward(cplx* X, int nsteps) {
    if (!rk_) launch_timed(ks_forward, dv_, X, H_, nsteps, static_cast<const SbdfCoef*>(rows_), err_);
    else if (stages_ == 2) launch_timed(ks_forward_rk<2>, dv_, X, H_, nsteps, tab_, desc_.dt, rk_dts(), err_);
    else launch_timed(ks_forward_rk<4>, dv_, X, H_, nsteps, tab_, desc_.dt, rk_dts(), err_);
    SPS_CHECK_LAUNCH();
    tape_steps_ = nsteps;
  }

  int order_ = 2;   // SBDF order (2, 3 or 4)
  bool rk_ = false;  // an IMEX RK scheme: tab_ with stages_ stages
  int stages_ = 0;
  RkTab tab_{};
  double* dts_ = nullptr;   // RK on variable steps: the step sizes (device, max_steps entries)
  sps_desc desc_;
  int K_ = 0, Ng_ = 0;
  KsDev dv_{};
  DevArena arena_;
  cplx *H_ = nullptr, *Xw_ = nullptr;
  int* err_ = nullptr;
  SbdfCoef* rows_ = nullptr;          // [nrows_] coefficient rows of the steps (device)
  std::vector<SbdfCoef> hrows_;       // their host copy
  int nrows_ = 0, var_n_ = 0;         // var_n_ > 0: variable steps, runs of at most var_n_ steps
  int tape_steps_ = -1;
  KernelTimer timer_;
};

}  // namespace

ProblemImpl* make_ks(const sps_desc& d, hipStream_t s) { return new KsProblem(d, s); }

}  // namespace sps
