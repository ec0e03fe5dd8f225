// 2D Rayleigh-Benard convection, Fourier (x) x Chebyshev (z), IMEX Runge-Kutta (ARS(2,2,2)
// or ARS(4,4,3)), and its discrete adjoint on gfx950.
//
// Equations (paper, Supplementary: Initial value problems) in the form
// M dX/dt + L X = F(X) with the ultraspherical/tau discretization (paper: Sparse spectral
// methods).  Per wavenumber k the unknowns are u, w, b, p (Chebyshev-T coefficients,
// N each) and the tau variables tau_u1, tau_w1, tau_b1, tau_u2, tau_w2, tau_b2, tau_p
// (S = 4N + 7 slots).  Equation rows share the slot numbers: u-, w-, b-momentum in C2
// coefficients, continuity in C1, boundary rows u(0), u(1), w(0), w(1), b(0), b(1), and
// the pressure gauge int p dz = 0 (k = 0) or tau_p = 0 (k != 0).
//
// Device data flow of one Runge-Kutta stage:
//   grid-row kernel (one block per Gauss node z_j): inverse real FFTs of the 8 fields
//     (u, w, ux, uz, wx, wz, bx, bz) from their x-spectra at z_j, products
//     N = -(u.grad)(u, w, b), forward real FFTs, truncation  -> nl[3][Ngz][K]
//   per-wavenumber kernel (one block per k): Chebyshev forward transform of nl, S10
//     conversion, stage right-hand side, banded LU solve of the real-ified system,
//     Chebyshev backward transforms of the new state and its z-derivatives
//     -> state[k], zgrid[6][Ngz][K]
// The adjoint runs the transposed chain: transposed solve, S10^T, adjoint Chebyshev
// forward transform, adjoint real FFTs with the product rule, adjoint Chebyshev
// backward transform and derivative transposes (paper, Methods: Spectral transforms;
// Nonlinear operator graphs).
//
// Linear solves: per k the system A = a M + b L is made real by the diagonal phases
// D_r (u rows times -i) and D_c (u and its taus times i), its boundary rows are made
// sparse by the right preconditioner R (Dirichlet recombination T_n - T_{n-2} for u, w, b
// and an integral-free recombination for p), and rows/columns are interleaved by mode.
// B = D_r A D_c R is then a real banded matrix (kl = 7, ku = 20 at N = 64) factored by
// banded LU with partial pivoting.  A x = r is solved as B y = D_r r, x = D_c R y, and
// A^H z = g as B^T w = R^T D_c^H g, z = D_r^H w, through the same factors.
#include <fcntl.h>
#include <math.h>
#include <unistd.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "band_lu.h"
#include "ckpt.h"
#include "cou.h"
#include "sps_device.h"
#include "sps_internal.h"
#include "ultra_ops.h"
#include "wave_fft.h"

// Scratch of the allocation-free explicit-term evaluation (sps_eval_F_noalloc): the x-spectral
// z-grid fields and the nonlinear terms of one evaluation.  One copy per GPU that the library
// runs on, held until the process ends.  Host code never passes this name to a kernel (on the
// host it is a stand-in, not a device address); it uses the per-device address from
// hipGetSymbolAddress (sps::scratch_address).
constexpr size_t SPS_SCRATCH_BYTES = size_t(2) << 20;
static __device__ __align__(256) double scratch[SPS_SCRATCH_BYTES / sizeof(double)];

namespace sps {

// Device address of `scratch` on device dev, looked up once per device with that device current.
static double* scratch_address(int dev) {
  static std::mutex mu;
  static std::map<int, double*> addr;
  std::lock_guard<std::mutex> lock(mu);
  auto it = addr.find(dev);
  if (it != addr.end()) return it->second;
  int cur = -1;
  SPS_HIP(hipGetDevice(&cur));
  if (cur != dev) SPS_HIP(hipSetDevice(dev));
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (cur != dev) SPS_HIP(hipSetDevice(cur));
  if (e != hipSuccess || ptr == nullptr)
    throw Error(SPS_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  addr.emplace(dev, static_cast<double*>(ptr));
  return static_cast<double*>(ptr);
}

namespace {

constexpr int NT = 256;   // threads per block of the grid-row, factor and set-up kernels
constexpr int NTK = 512;  // threads per block of the per-wavenumber step kernels
// Partitioned solves: at most SPS_MAXPART partitions; a row's spike entries (both couplings)
// at most SPS_SPIKE_W; the coupled entries' system at most SPS_RED_MAX unknowns.
constexpr int SPS_MAXPART = 4;
constexpr int SPS_SPIKE_W = 24;
constexpr int SPS_RED_MAX = 72;
constexpr int SPS_CP_REG = 16;   // 16-byte loads per thread of the spike copy
constexpr int NTX = 512;  // threads per block of the grid-row step kernels

struct RbcDev {
  int K, N, S, Ngx, Ngz, Nx1, Nz1;
  int n, kl, ku, uw;
  double Lx, nu, ka;
  double cp, bc0;       // buoyancy coupling in the w rows (1, or 0 without buoyancy); b(0) at k = 0
  double cost_scale;    // J = cost_scale / 2 sum_k w_k Re(c^H G c)
  int Kz, ncost;        // modes per x wavenumber (cost weight of mode k: k / Kz == 0 ? 1 : 2); fields in J
  const unsigned char* ckeep;   // [K] modes counted in J (null: all)
  const double* kx;     // [K] horizontal wavenumber of each mode
  // T_n at the ascending Gauss node j of an Ng-point grid equals cos(pi M / (2 Ng)) with
  // M = n (2 (Ng - j) - 1) mod 4 Ng, so one table of 4 Ng cosines serves every (n, j).
  const double* cosz;   // [4 Ngz]
  const double* cosz1;  // [4 Nz1] (scale-1 grid)
  const cplx* twx;      // [Ngx]
  const cplx* twx1;     // [Nx1]
  FftPlan px, px1;
  const int* rowmap;    // [S] solver row i  <- ABI row slot
  const int* colmap;    // [S] solver col i  -> ABI column slot
  const signed char* rowph;  // [S] 1: row slot multiplied by -i
  const signed char* colph;  // [S] 1: column slot multiplied by +i
  const double* rho;    // [S] X[s] = y[s] + rho[s] y[s+2]
  // per-thread copies of the permutation tables (index i < S):
  const int* gmap;      // rowmap[i] | rowph(rowmap[i]) << 30
  const int* hmap;      // colmap[i] | colph(s) << 30 | colph(s-2) << 29, s = colmap[i]
  const double* hrho;   // rho[s - 2] for s = colmap[i] (0 if s < 2)
  const int* sflag;     // colph[i] (slot i)
  const double* gram;   // [N][N] int_0^1 T_m T_n dz
  const double* ops;    // [B][K][opsize] block operators of the LU factors (T blocks, then G blocks)
  int opsize;           // doubles per system (stride)
  int blksz;            // of which block operators (staged into LDS)
  int tsz;              // of which T blocks (the G blocks follow at tsz)
  // Partitioned solve (the staged path): part = P > 1 partitions of rows [ps_p, ps_{p+1}),
  // ps_0 = 0, ps_P = n, the starts multiples of 8.  Each partition has its own factors and
  // block operators (its T blocks at block ps_p / 8 of the T set, its G blocks likewise).
  // Direction dir (0 forward, 1 transposed) keeps at spk[dir] each partition's spike rows
  // [V_p | W_p] (column-major within the partition: entry c of its row t at c n_p + t, so that
  // a wave's rows load contiguously) and, at spk[dir] + rof[dir], the inverse of the coupled
  // entries' system (nrr[dir] x nrr[dir], column-major).  smap[dir * n + i] = {offset of row
  // i's first entry | n_p << 16, its widths and coupled-entry offsets} (see rbc_solve_part);
  // coupled entry z of interface q (z >= zb_q) is the entry of row z + rsh_q.  pmeta holds the
  // layout for the factor kernel.
  int part, ps1, ps2, ps3;
  int spk[2], rof[2], nrr[2], zb1[2], zb2[2], rsh0[2], rsh1[2], rsh2[2];
  const int2* smap;
  const int* pmeta;
  int* err;             // bit 0 singular pivot, bit 1 non-finite state
  // A batch of B instances of the problem (blockIdx.y = instance) that differ in their
  // Rayleigh number: per-instance nu and kappa (null for a single problem), factors and arrays
  // at instance strides.
  int B;
  const double* nub;    // [B]
  const double* kab;    // [B]
};

// The wavenumber of a per-wavenumber block.  Workgroups are dealt to the eight XCDs in turn, and
// each XCD has its own L2; the z-column arrays ([field][z][k]) hold eight wavenumbers per
// 128-byte line, so consecutive wavenumbers go to one XCD (XCD x takes a contiguous range), and
// the blocks that read or write the same lines share that XCD's L2 instead of each fetching the
// line from memory.
__device__ __forceinline__ int xcd_wavenumber(int b, int K) {
  constexpr int X = 8;
  const int per = K / X, rem = K - per * X, x = b % X;
  return x * per + min(x, rem) + b / X;
}

// Instance b's view of the problem: its diffusivities and its factors.
__device__ __forceinline__ void rbc_inst(RbcDev& d, int b) {
  if (d.nub) {
    d.nu = d.nub[b];
    d.ka = d.kab[b];
  }
  d.ops += (size_t)b * d.K * d.opsize;
}
// p + b * stride for a non-null per-instance array
template <typename T>
__device__ __forceinline__ T* inst_ptr(T* p, int b, size_t stride) {
  return p ? p + (size_t)b * stride : p;
}

// ---------------------------------------------------------------------------- operators
// Sparse ultraspherical operators on [0,1] applied to length-N coefficient arrays in LDS.
__device__ __forceinline__ double s0d(int m) { return m == 0 ? 1.0 : 0.5; }

// (S0 c)[m] = s0d(m) c[m] - c[m+2]/2 : T -> C1
__device__ __forceinline__ cplx s0_at(const cplx* c, int m, int N) {
  cplx v = cscale(c[m], s0d(m));
  if (m + 2 < N) v = csub(v, cscale(c[m + 2], 0.5));
  return v;
}
// (S10 c)[n] = (S0 c)[n]/(n+1) - (S0 c)[n+2]/(n+3) : T -> C2
__device__ __forceinline__ cplx s10_at(const cplx* c, int n, int N) {
  cplx v = cscale(s0_at(c, n, N), 1.0 / (n + 1));
  if (n + 2 < N) v = csub(v, cscale(s0_at(c, n + 2, N), 1.0 / (n + 3)));
  return v;
}
// (DZZ c)[n] = 4 (D1 D0 c)[n] = 8 (n+2) c[n+2]
__device__ __forceinline__ cplx dzz_at(const cplx* c, int n, int N) {
  return (n + 2 < N) ? cscale(c[n + 2], 8.0 * (n + 2)) : czero();
}
// (S1 DZ1 c)[n] = 2 (c[n+1] - c[n+3])
__device__ __forceinline__ cplx s1dz_at(const cplx* c, int n, int N) {
  cplx v = (n + 1 < N) ? cscale(c[n + 1], 2.0) : czero();
  if (n + 3 < N) v = csub(v, cscale(c[n + 3], 2.0));
  return v;
}
// (DZ1 c)[n] = 2 (n+1) c[n+1] : T -> C1
__device__ __forceinline__ cplx dz1_at(const cplx* c, int n, int N) {
  return (n + 1 < N) ? cscale(c[n + 1], 2.0 * (n + 1)) : czero();
}
// transposes
__device__ __forceinline__ cplx s1t_at(const cplx* y, int j, int N) {  // (S1^T y)[j]
  cplx v = cscale(y[j], 1.0 / (j + 1));
  if (j >= 2) v = csub(v, cscale(y[j - 2], 1.0 / (j + 1)));
  return v;
}
__device__ __forceinline__ cplx s0t_at(const cplx* y, int m, int N) {  // (S0^T y)[m]
  cplx v = cscale(y[m], s0d(m));
  if (m >= 2) v = csub(v, cscale(y[m - 2], 0.5));
  return v;
}
__device__ __forceinline__ cplx s10t_at(const cplx* y, int m, int N) {  // (S0^T S1^T y)[m]
  cplx v = cscale(s1t_at(y, m, N), s0d(m));
  if (m >= 2) v = csub(v, cscale(s1t_at(y, m - 2, N), 0.5));
  return v;
}
__device__ __forceinline__ cplx dzzt_at(const cplx* y, int m, int N) {
  return (m >= 2) ? cscale(y[m - 2], 8.0 * m) : czero();
}
__device__ __forceinline__ cplx s1dzt_at(const cplx* y, int m, int N) {
  cplx v = (m >= 1) ? cscale(y[m - 1], 2.0) : czero();
  if (m >= 3) v = csub(v, cscale(y[m - 3], 2.0));
  return v;
}
__device__ __forceinline__ cplx dz1t_at(const cplx* y, int m, int N) {
  return (m >= 1) ? cscale(y[m - 1], 2.0 * m) : czero();
}


// int_0^1 T_m(2z - 1) dz: 1 / (1 - m^2) for even m, zero for odd m (computed, not loaded, so
// that the stage kernels read no global memory between issuing their loads and the solve)
__device__ __forceinline__ double intw_at(int m) { return (m & 1) ? 0.0 : 1.0 / (1.0 - (double)m * m); }

// Row s < 4N of (M X) and (L X) for wavenumber k (momentum, buoyancy and continuity rows),
// kx = d.kx[k] (loaded by the caller at kernel start).  X in ABI column slots.
struct MLRow {
  cplx m, l;
};
__device__ MLRow ml_row(const RbcDev& d, int k, double kx, const cplx* X, int s) {
  const int N = d.N;
  const double k2 = kx * kx;
  const cplx* u = X;
  const cplx* w = X + N;
  const cplx* b = X + 2 * N;
  const cplx* p = X + 3 * N;
  const cplx* tau = X + 4 * N;
  MLRow r{czero(), czero()};
  if (s < 3 * N) {
    const int f = s / N, n = s - f * N;
    const cplx* c = X + f * N;
    const double dif = (f == 2) ? d.ka : d.nu;
    const cplx sc = s10_at(c, n, N);
    r.m = sc;
    cplx l = cadd(cscale(dzz_at(c, n, N), -dif), cscale(sc, dif * k2));
    if (f == 0) l = cadd(l, cmul_i(cscale(s10_at(p, n, N), kx)));
    if (f == 1) l = csub(cadd(l, s1dz_at(p, n, N)), cscale(s10_at(b, n, N), d.cp));
    if (n == N - 2) l = csub(l, cscale(tau[f], 4.0 * dif));   // lifted tau_1
    if (n == N - 1) l = cadd(l, tau[3 + f]);                  // tau_2
    r.l = l;
  } else {
    const int n = s - 3 * N;
    cplx l = cadd(cmul_i(cscale(s0_at(u, n, N), kx)), dz1_at(w, n, N));
    if (n == N - 1) l = cadd(l, tau[1]);
    if (k == 0 && n == 0) l = cadd(l, tau[6]);
    r.l = l;
  }
  return r;
}

// Rows 4N + q (q < 7) of L X, the boundary values and the gauge row, summed by an aligned quad:
// lane h takes the modes m = h, h + 4, ...  Row 4N + q, q < 6: field q/2 at z = 0 (q even,
// sum of (-1)^m c_m) or z = 1 (sum of c_m).  Row 4N + 6: the mean of p at k = 0, else tau_p.
// Every lane of the quad returns the row value.
__device__ __forceinline__ cplx l_bc_row(const RbcDev& d, int k, const cplx* X, int q, int h) {
  const int N = d.N;
  double sr = 0.0, si = 0.0;
  if (q < 6) {
    const cplx* c = X + (q / 2) * N;
    const double sg = ((q & 1) == 0 && (h & 1)) ? -1.0 : 1.0;   // m has the parity of h
    for (int m = h; m < N; m += 4) {
      sr += c[m].x;
      si += c[m].y;
    }
    sr *= sg;
    si *= sg;
  } else if (k == 0) {
    const cplx* p = X + 3 * N;
    for (int m = h; m < N; m += 4) {
      const double w = intw_at(m);
      sr = fma(w, p[m].x, sr);
      si = fma(w, p[m].y, si);
    }
  } else if (h == 0) {
    sr = X[4 * N + 6].x;
    si = X[4 * N + 6].y;
  }
  return group_sum<4>(cmk(sr, si));
}

// Column s of (M^H Y) and (L^H Y), kx = d.kx[k]; Y in ABI row slots.
__device__ MLRow mlt_col(const RbcDev& d, int k, double kx, const cplx* Y, int s) {
  const int N = d.N;
  const double k2 = kx * kx;
  const cplx* yu = Y;
  const cplx* yw = Y + N;
  const cplx* yb = Y + 2 * N;
  const cplx* yc = Y + 3 * N;
  const cplx* ybc = Y + 4 * N;
  MLRow r{czero(), czero()};
  if (s < 3 * N) {
    const int f = s / N, m = s - f * N;
    const cplx* yf = Y + f * N;
    const double dif = (f == 2) ? d.ka : d.nu;
    const cplx st = s10t_at(yf, m, N);
    r.m = st;
    cplx l = cadd(cscale(dzzt_at(yf, m, N), -dif), cscale(st, dif * k2));
    if (f == 0) l = cadd(l, cmul_mi(cscale(s0t_at(yc, m, N), kx)));   // (i kx S0)^H
    if (f == 1) l = cadd(l, dz1t_at(yc, m, N));
    if (f == 2) l = csub(l, cscale(s10t_at(yw, m, N), d.cp));          // -S10 b in w rows
    const cplx bot = ybc[2 * f], top = ybc[2 * f + 1];
    l = cadd(l, (m & 1) ? csub(top, bot) : cadd(top, bot));
    r.l = l;
  } else if (s < 4 * N) {
    const int m = s - 3 * N;
    cplx l = cadd(cmul_mi(cscale(s10t_at(yu, m, N), kx)), s1dzt_at(yw, m, N));
    if (k == 0) l = cadd(l, cscale(Y[4 * N + 6], intw_at(m)));
    r.l = l;
  } else {
    const int t = s - 4 * N;
    cplx l;
    switch (t) {
      case 0: l = cscale(yu[N - 2], -4.0 * d.nu); break;
      case 1: l = cadd(cscale(yw[N - 2], -4.0 * d.nu), yc[N - 1]); break;
      case 2: l = cscale(yb[N - 2], -4.0 * d.ka); break;
      case 3: l = yu[N - 1]; break;
      case 4: l = yw[N - 1]; break;
      case 5: l = yb[N - 1]; break;
      default: l = (k == 0) ? yc[0] : Y[4 * N + 6]; break;
    }
    r.l = l;
  }
  return r;
}

// d/dz of a T series on [0,1]: 2 x the T-basis derivative by its backward recurrence
// d[N-1] = 0, d[m] = d[m+2] + 2(m+1) c[m+1] (m >= 1), d[0] = c[1] + d[2]/2.  One thread.
__device__ void dz_series(const cplx* c, cplx* dcf, int N) {
  cplx dp2 = czero(), dp1 = czero();  // d[m+2], d[m+1]
  for (int m = N - 1; m >= 0; --m) {
    cplx dm;
    if (m == N - 1) dm = czero();
    else if (m >= 1) dm = cadd(dp2, cscale(c[m + 1], 2.0 * (m + 1)));
    else dm = cadd(c[1], cscale(dp2, 0.5));
    dcf[m] = cscale(dm, 2.0);
    dp2 = dp1;
    dp1 = dm;
  }
}
// transpose of dz_series: e = (2 D_T)^T y
__device__ void dz_series_t(const cplx* y, cplx* e, int N) {
  cplx a_nm2 = czero(), a_nm1 = czero();  // A[n-2], A[n-1]
  for (int n = 0; n < N; ++n) {
    cplx a;
    if (n == 0) a = czero();
    else if (n == 1) a = cscale(y[0], 0.5);
    else a = cadd(a_nm2, y[n - 1]);
    e[n] = cscale(a, 4.0 * n);
    a_nm2 = a_nm1;
    a_nm1 = a;
  }
}

// ---------------------------------------------------------------------------- Chebyshev sums
// Stage the cosine table of an Ng-point Gauss grid into LDS (block-wide; caller syncs).
__device__ __forceinline__ void stage_cos(const double* g, double* ct, int Ng) {
  for (int e = threadIdx.x; e < 4 * Ng; e += blockDim.x) ct[e] = g[e];
}
// sum_j T_n(x_j) v[j] over the Ng nodes (complex v in LDS), cos table ct in LDS.
__device__ __forceinline__ cplx cheb_sum_nodes(const double* ct, const cplx* v, int n, int Ng) {
  const int P = 4 * Ng, dn = (2 * n) % P;
  int M = (int)((unsigned)n * (unsigned)(2 * Ng - 1) % (unsigned)P);
  double sr = 0.0, si = 0.0;
#pragma unroll 8
  for (int j = 0; j < Ng; ++j) {
    const double t = ct[M];
    sr += t * v[j].x;
    si += t * v[j].y;
    M -= dn;
    if (M < 0) M += P;
  }
  return cmk(sr, si);
}
// sum_n T_n(x_j) c[n] over N modes at node j.
__device__ __forceinline__ cplx cheb_sum_modes(const double* ct, const cplx* c, int j, int N, int Ng) {
  const int P = 4 * Ng, dm = 2 * (Ng - j) - 1;
  int M = 0;
  double sr = 0.0, si = 0.0;
#pragma unroll 8
  for (int n = 0; n < N; ++n) {
    const double t = ct[M];
    sr += t * c[n].x;
    si += t * c[n].y;
    M += dm;
    if (M >= P) M -= P;
  }
  return cmk(sr, si);
}

// Mirror-symmetric forms.  The Gauss nodes j and j' = Ng-1-j are mirror images (x -> -x) and
// T_n(-x) = (-1)^n T_n(x).  A node sum over all Ng nodes is therefore a sum over the Hc =
// ceil(Ng/2) pairs of P_j = v_j + v_j' (n even) or Q_j = v_j - v_j' (n odd), and the mode sums
// at node j give node j' from the same even and odd parts: v_j = E + O, v_j' = E - O.
__host__ __device__ inline int half_nodes(int Ng) { return (Ng + 1) / 2; }

// P, Q of a mirror pair (the middle node of an odd grid is its own mirror: P = Q = v_j),
// stored as pq[2 i] = P, pq[2 i + 1] = Q.
__device__ __forceinline__ void store_mirror_pair(cplx vj, cplx vm, bool middle, cplx* pq2) {
  pq2[0] = middle ? vj : cadd(vj, vm);
  pq2[1] = middle ? vj : csub(vj, vm);
}

// sum_j T_n(x_j) v_f[j] for NF fields at once from their mirror sums pq (field f at
// pq + 2 f Hc).  SPL lanes (an aligned group) share one mode n; lane h takes pairs
// j = h, h + SPL, ...  Every lane of the group returns the full sums.
template <int NF, int SPL>
__device__ __forceinline__ void nodes_to_mode(const double* ct, const cplx* pq, int Hc, int Ng, int n, int h,
                                              cplx (&acc)[NF]) {
  const int P4 = 4 * Ng, par = n & 1;
  // T_n(x_j) = ct[n (2 (Ng - j) - 1) mod 4 Ng] (32-bit products: n < 64 and Ng <= 128 here; a
  // 64-bit remainder is a long instruction sequence)
  int M = (int)((unsigned)n * (unsigned)(2 * (Ng - h) - 1) % (unsigned)P4);
  const int dn = (int)((unsigned)(2 * SPL * n) % (unsigned)P4);
#pragma unroll
  for (int f = 0; f < NF; ++f) acc[f] = czero();
  for (int j = h; j < Hc; j += SPL) {
    const double t = ct[M];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      const cplx v = pq[2 * (f * Hc + j) + par];
      acc[f].x = fma(t, v.x, acc[f].x);
      acc[f].y = fma(t, v.y, acc[f].y);
    }
    M -= dn;
    if (M < 0) M += P4;
  }
#pragma unroll
  for (int f = 0; f < NF; ++f) acc[f] = group_sum<SPL>(acc[f]);
}

// Values at the mirror pair (j, j') of NF series (field f at c + f cstride, N modes).  Four
// lanes (an aligned quad) share the pair; lane h sums modes n = h, h + 4, ... (one parity).
// Returns in lane h = 0 the values at j, in lane h = 1 the values at j'.
template <int NF>
__device__ __forceinline__ void modes_to_pair(const double* ct, const cplx* c, int cstride, int N, int Ng, int j,
                                              int h, cplx (&val)[NF]) {
  const int P4 = 4 * Ng, dm = 2 * (Ng - j) - 1;
  int M = (int)((unsigned)h * (unsigned)dm % (unsigned)P4);
  const int step = (int)((unsigned)(4 * dm) % (unsigned)P4);
#pragma unroll
  for (int f = 0; f < NF; ++f) val[f] = czero();
  for (int n = h; n < N; n += 4) {
    const double t = ct[M];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      const cplx v = c[f * cstride + n];
      val[f].x = fma(t, v.x, val[f].x);
      val[f].y = fma(t, v.y, val[f].y);
    }
    M += step;
    if (M >= P4) M -= P4;
  }
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    const cplx s = make_double2(val[f].x + dpp_xor2(val[f].x), val[f].y + dpp_xor2(val[f].y));   // E (h even), O (h odd)
    const cplx o = make_double2(dpp_xor1(s.x), dpp_xor1(s.y));
    val[f] = (h & 1) ? csub(o, s) : cadd(s, o);
  }
}

// Coefficient m of d/dz of a T series on [0,1] (twice the T-basis derivative) is
// 4 sum_{p > m, p - m odd} p c_p, halved for m = 0.
// For the three fields of c at once, field f on wave f and mode p on lane p (N <= 64):
// with w_p = p c_p, coefficient m is the stride-2 suffix sum of w from p = m + 1, formed by
// shuffles (five steps instead of a serial sum per coefficient).  Called by waves 0-2.
__device__ __forceinline__ void dz_coefs_wave(const cplx* c, int N, cplx* dz) {
  const int f = threadIdx.x >> 6, p = threadIdx.x & 63;
  cplx w = (p < N) ? cscale(c[f * N + p], (double)p) : czero();
  for (int o = 2; o < 64; o <<= 1) {
    const double tx = __shfl_down(w.x, o), ty = __shfl_down(w.y, o);
    if (p + o < 64) {
      w.x += tx;
      w.y += ty;
    }
  }
  // w = sum over q >= p of the parity of p of q c_q, the sum that coefficient p - 1 needs
  if (p >= 1 && p <= N) dz[f * N + p - 1] = cscale(w, p == 1 ? 2.0 : 4.0);
  if (p == 0 && N == 64) dz[f * N + N - 1] = czero();
}
// The transpose of that map applied to y has entry n = 4 n sum_{p < n, n - p odd} y_p, with y_0
// halved (formed by prefix shuffles in zbar_to_coeffs).

// The banded solves run in solver coordinates: real-ified (phases D_r, D_c), recombined (R)
// and interleaved by mode (rowmap, colmap).
// A x = r:  vA = (D_r r)[rowmap];  B y = vA;  x = D_c R y.
// A^H z = g: vA = (R^T D_c^H g)[colmap];  B^T w = vA;  z[rowmap] = D_r^H w.

// Per-thread entries of the permutation tables for index i = tid (S <= NTK), loaded once at
// kernel start so the gathers and scatters do not wait on global memory.
struct MapRegs {
  int gm, hm, cm, sf;
  double hr, rh;
};
// (unconditional loads, clamped to the last entry: threads i >= S never use theirs, and loads
// under a branch would make the compiler wait for every load in flight at their first use)
__device__ __forceinline__ void load_maps(const RbcDev& d, MapRegs& m) {
  const int i = min((int)threadIdx.x, d.S - 1);
  m.gm = d.gmap[i];
  m.hm = d.hmap[i];
  m.cm = d.colmap[i];
  m.sf = d.sflag[i];
  m.hr = d.hrho[i];
  m.rh = d.rho[i];
}

// r (ABI row slots) -> vA (solver rows), zero tail.  Block-wide, ends with a barrier.
__device__ void rbc_gather(const RbcDev& d, const MapRegs& m, const cplx* r, cplx* vA) {
  const int i = threadIdx.x;
  if (i < d.S) {
    const int s = m.gm & 0xffff;
    const cplx v = r[s];
    vA[i] = (m.gm >> 30) ? cmul_mi(v) : v;
  } else if (i < d.S + SPS_PAD) {
    vA[i] = czero();
  }
  __syncthreads();
}
// vA (solution y, solver columns) -> x = D_c R y (ABI column slots); vB scratch.
__device__ void rbc_scatter(const RbcDev& d, const MapRegs& m, const cplx* vA, cplx* vB, cplx* x) {
  const int i = threadIdx.x;
  if (i < d.S) vB[m.cm] = vA[i];
  __syncthreads();
  if (i < d.S) {
    cplx y = vB[i];
    if (m.rh != 0.0) y = cadd(y, cscale(vB[i + 2], m.rh));
    x[i] = m.sf ? cmul_i(y) : y;
  }
  __syncthreads();
}
// g (ABI column slots) -> vA = (R^T D_c^H g)[colmap], zero tail.
__device__ void rbc_gather_h(const RbcDev& d, const MapRegs& m, const cplx* g, cplx* vA) {
  const int i = threadIdx.x;
  if (i < d.S) {
    const int s = m.hm & 0xffff;
    cplx v = g[s];
    if ((m.hm >> 30) & 1) v = cmul_mi(v);
    if (m.hr != 0.0) {
      cplx v2 = g[s - 2];
      if ((m.hm >> 29) & 1) v2 = cmul_mi(v2);
      v = cadd(v, cscale(v2, m.hr));
    }
    vA[i] = v;
  } else if (i < d.S + SPS_PAD) {
    vA[i] = czero();
  }
  __syncthreads();
}
// vA (solver rows) -> z (ABI row slots) = D_r^H w.
__device__ void rbc_scatter_h(const RbcDev& d, const MapRegs& m, const cplx* vA, cplx* z) {
  const int i = threadIdx.x;
  if (i < d.S) {
    const int s = m.gm & 0xffff;
    z[s] = (m.gm >> 30) ? cmul_i(vA[i]) : vA[i];
  }
  __syncthreads();
}
// Staged solves hold a system's block operators in LDS from o.  The set the first sweep reads
// (T for the forward solve, G for the transposed one: the early set) sits above the other (the
// late set, from o), so that it can be written while the stage kernel's phase buffers, which
// share the late set's space, are still in use; the late set is written during the first sweep.
struct StagedOps {
  double* T;
  double* G;
};
__device__ __forceinline__ StagedOps staged_ops(const RbcDev& d, double* o, bool transposed) {
  return transposed ? StagedOps{o, o + d.tsz} : StagedOps{o + (d.blksz - d.tsz), o};
}
// This thread's share of the early set into LDS (waits for those loads only, which were issued
// first).  Every thread, before the block barrier that precedes the solve.
__device__ __forceinline__ void stage_early(const RbcDev& d, const OpsRegs& r, double* o, bool transposed) {
  const StagedOps s = staged_ops(d, o, transposed);
  if (transposed) ops_store_part(r.g, d.blksz - d.tsz, s.G);
  else ops_store_part(r.t, d.tsz, s.T);
}
__device__ __forceinline__ void stage_late(const RbcDev& d, const OpsRegs& r, double* o, bool transposed) {
  const StagedOps s = staged_ops(d, o, transposed);
  if (transposed) ops_store_part(r.t, d.tsz, s.T);
  else ops_store_part(r.g, d.blksz - d.tsz, s.G);
}
// The first and second sweeps of one wave's solve of the nrow-row system whose operators
// start at T, G.
__device__ __forceinline__ void sweep_first(const double* T, const double* G, int nrow, double* b, bool transposed) {
  if (transposed) blk_Ut_range(G, 0, blk_count(nrow), b, nrow);
  else blk_L_range(T, 0, blk_count(nrow), b, nrow);
}
__device__ __forceinline__ void sweep_second(const double* T, const double* G, int nrow, double* b, bool transposed) {
  if (transposed) blk_Lt_range(T, 0, blk_count(nrow), b, nrow);
  else blk_U_range(G, 0, blk_count(nrow), b, nrow);
}

// Solve in place on vA (forward or transposed) with the early set already in LDS (stage_early
// before the last barrier); wave 0 takes the complex vector (real parts on lanes 0-31,
// imaginary on 32-63) while the other waves write the late set.  Block-wide.
__device__ void rbc_solve_staged(const RbcDev& d, const OpsRegs& regs, double* o, cplx* vA, bool transposed) {
  const StagedOps s = staged_ops(d, o, transposed);
  double* b = reinterpret_cast<double*>(vA);
  const bool solver = threadIdx.x < SPS_WAVE;
  if (solver) sweep_first(s.T, s.G, d.n, b, transposed);
  stage_late(d, regs, o, transposed);
  __syncthreads();
  if (solver) sweep_second(s.T, s.G, d.n, b, transposed);
  __syncthreads();
}

// The same solve with the block operators streamed from global memory through two LDS buffers
// of SPS_CHUNK blocks: wave 0 runs the sweeps over chunk q while the other waves copy
// chunk q + 1 (for launches with many more systems than CUs: no register prefetch and a small
// LDS footprint, so several blocks share a CU).  Block-wide; buf holds 2 * SOLVE_CHUNK_D doubles.
constexpr int SPS_CHUNK = 6;
constexpr int SOLVE_CHUNK_D = SPS_CHUNK * SPS_BLK * SPS_GS;   // >= SPS_CHUNK * SPS_TW * SPS_TS
__device__ void rbc_solve_streamed(const RbcDev& d, const double* gops, double* buf, cplx* vA, bool transposed) {
  const int nblk = blk_count(d.n), nch = (nblk + SPS_CHUNK - 1) / SPS_CHUNK, Q = 2 * nch;
  const double* Tg = gops;
  const double* Gg = gops + nblk * SPS_TW * SPS_TS;
  const int tid = threadIdx.x, wave = tid >> 6;
  // chunk q: the first sweep (L, or U^T) runs over ascending chunks, the second (U, or L^T)
  // over descending ones; the forward solve reads T then G, the transposed G then T
  auto range = [&](int q, int* t0, int* t1, bool* useT) {
    const bool first = q < nch;
    const int c = first ? q : 2 * nch - 1 - q;
    *t0 = c * SPS_CHUNK;
    *t1 = min(nblk, *t0 + SPS_CHUNK);
    *useT = (first != transposed);
  };
  auto copy = [&](int q, double* dst, int i0, int step) {
    int t0, t1;
    bool useT;
    range(q, &t0, &t1, &useT);
    const int per = useT ? SPS_TW * SPS_TS : SPS_BLK * SPS_GS;
    const double2* src = reinterpret_cast<const double2*>((useT ? Tg : Gg) + (size_t)t0 * per);
    double2* d2 = reinterpret_cast<double2*>(dst);
    const int h = (t1 - t0) * per / 2;
    for (int e = i0; e < h; e += step) d2[e] = src[e];
  };
  copy(0, buf, tid, blockDim.x);
  __syncthreads();
  for (int q = 0; q < Q; ++q) {
    double* cur = buf + (q & 1) * SOLVE_CHUNK_D;
    if (wave >= 1) {
      if (q + 1 < Q) copy(q + 1, buf + ((q + 1) & 1) * SOLVE_CHUNK_D, tid - SPS_WAVE, blockDim.x - SPS_WAVE);
    } else {
      int t0, t1;
      bool useT;
      range(q, &t0, &t1, &useT);
      double* b = reinterpret_cast<double*>(vA);
      if (!transposed) {
        if (useT) blk_L_range(cur, t0, t1, b, d.n);
        else blk_U_range(cur, t0, t1, b, d.n);
      } else {
        if (useT) blk_Lt_range(cur, t0, t1, b, d.n);
        else blk_Ut_range(cur, t0, t1, b, d.n);
      }
    }
    __syncthreads();
  }
}

// The staged solve in P = d.part partitions (a SPIKE solve): wave p < P solves partition p's
// rows in place in vA with that partition's own block operators (its sweeps never write past
// its rows, and read the next partition's live rows only through zero operator columns), so
// the P dependent chains run at the same time.  With y_p the partition solutions and V_p, W_p
// the precomputed spikes (the partition's inverse applied to the columns that couple it to the
// next and to the previous partition), the exact solution is
// x_p = y_p - V_p c_p - W_p a_{p-1}, where a_q (the last entries of partition q) and c_q (the
// first entries of partition q + 1) are the coupled entries of interface q; they solve a
// small system R z = g whose right-hand side g is y at the coupled rows and whose inverse is
// precomputed.  The transposed solve has its own spikes and system.  The early set is in LDS
// (stage_early before the last barrier); the other waves write the late set during the first
// sweeps, the solver waves theirs after them.  During the second sweeps the other waves copy
// the spikes and the inverse into the early set's space (free once every first sweep is
// done).  vB is scratch (the coupled entries).  Block-wide; vA holds the gathered right-hand
// side and gets the solution.
__device__ __forceinline__ void rbc_solve_part(const RbcDev& d, int k, const OpsRegs& regs, double* o, cplx* vA, cplx* vB,
                               bool transposed) {
  const int tid = threadIdx.x, wave = tid >> 6, n = d.n, P = d.part, dir = transposed ? 1 : 0;
  const int2 sm2 = d.smap[dir * n + min(tid, n - 1)];   // this row's spike layout (used last)
  const int sm = sm2.y, soff = sm2.x & 0xffff, sstr = sm2.x >> 16;
  // this wave's partition (sums of differences rather than selects between fields: a select
  // between two fields of the descriptor becomes a computed offset into it, which keeps a copy
  // of the whole descriptor in scratch memory)
  const int ps1 = d.ps1, ps2 = d.ps2, ps3 = d.ps3;
  auto pstart = [&](int q) { return (q >= 1 ? ps1 : 0) + (q >= 2 ? ps2 - ps1 : 0) + (q >= 3 ? ps3 - ps2 : 0); };
  const int p0 = pstart(wave), p1 = (wave + 1 >= P) ? n : pstart(wave + 1);
  const StagedOps s = staged_ops(d, o, transposed);
  const double* T = s.T + (p0 / SPS_BLK) * (SPS_TW * SPS_TS);
  const double* G = s.G + (p0 / SPS_BLK) * (SPS_BLK * SPS_GS);
  double* b = reinterpret_cast<double*>(vA + p0);
  if (wave < P) sweep_first(T, G, p1 - p0, b, transposed);
  stage_late(d, regs, o, transposed);
  __syncthreads();
  // spikes (entry c of row i at c n + i) and the coupled system's inverse (column-major, at
  // rof), copied from the factors to the early set's space
  double* lsp = transposed ? s.G : s.T;
  const int nr = d.nrr[dir];
  if (wave < P) {
    sweep_second(T, G, p1 - p0, b, transposed);
  } else {
    const double2* src = reinterpret_cast<const double2*>(d.ops + (size_t)k * d.opsize + d.spk[dir]);
    double2* dst = reinterpret_cast<double2*>(lsp);
    const int h = (d.rof[dir] + nr * nr + 1) / 2, t0 = tid - P * SPS_WAVE, nth = blockDim.x - P * SPS_WAVE;
    double2 v[SPS_CP_REG];
#pragma unroll
    for (int i = 0; i < SPS_CP_REG; ++i) {
      const double2* q = src + min(t0 + i * nth, h - 1);
      v[i] = make_double2(q->x, q->y);
    }
#pragma unroll
    for (int i = 0; i < SPS_CP_REG; ++i)
      if (t0 + i * nth < h) dst[t0 + i * nth] = v[i];
  }
  __syncthreads();
  cplx* zs = vB;   // the coupled entries
  const int zb1 = d.zb1[dir], zb2 = d.zb2[dir], rs0 = d.rsh0[dir], rs1 = d.rsh1[dir], rs2 = d.rsh2[dir];
  const double* rinv = lsp + d.rof[dir];
  // row r = tid / 4 of z = R^{-1} g, four lanes per row, every fourth column; no branches inside
  // the sums (columns past the end read a valid entry and take a zero coefficient), in chunks
  // of six so that several LDS reads are in flight together
  const int r = tid >> 2, cc = tid & 3;
  if (r < nr) {
    cplx z = czero();
    for (int c0 = cc; c0 < nr; c0 += 24) {
      cplx g[6];
      double rv[6];
#pragma unroll
      for (int u = 0; u < 6; ++u) {
        const int c = min(c0 + 4 * u, nr - 1);
        g[u] = vA[c + rs0 + (c >= zb1 ? rs1 - rs0 : 0) + (c >= zb2 ? rs2 - rs1 : 0)];
        rv[u] = rinv[c * nr + r];
      }
#pragma unroll
      for (int u = 0; u < 6; ++u) z = cadd(z, cscale(g[u], (c0 + 4 * u < nr) ? rv[u] : 0.0));
    }
    z = group_sum<4>(z);
    if (cc == 0) zs[r] = z;
  }
  __syncthreads();
  if (tid < n) {
    const int wV = sm & 31, wW = (sm >> 5) & 31, zV = (sm >> 10) & 127, zW = (sm >> 17) & 127;
    const int w = wV + wW;
    cplx x = vA[tid];
    for (int c0 = 0; c0 < w; c0 += 6) {
      cplx g[6];
      double sv[6];
#pragma unroll
      for (int u = 0; u < 6; ++u) {
        const int c = min(c0 + u, w - 1);
        g[u] = zs[(c < wV) ? zV + c : zW + c - wV];
        sv[u] = lsp[soff + c * sstr];
      }
#pragma unroll
      for (int u = 0; u < 6; ++u) x = csub(x, cscale(g[u], (c0 + u < w) ? sv[u] : 0.0));
    }
    vA[tid] = x;
  }
  __syncthreads();
}

// The staged solves need stage_early(d, regs, lds, transposed) by every thread before the last
// barrier.
template <bool STREAM>
__device__ __forceinline__ void rbc_solve(const RbcDev& d, int k, const OpsRegs& regs, double* lds, cplx* vA,
                                          cplx* vB, bool transposed) {
  if (STREAM) rbc_solve_streamed(d, d.ops + (size_t)k * d.opsize, lds, vA, transposed);
  else if (d.part) rbc_solve_part(d, k, regs, lds, vA, vB, transposed);
  else rbc_solve_staged(d, regs, lds, vA, transposed);
}

// ---------------------------------------------------------------------------- per-wavenumber forward kernel
enum KfMode { KF_ZGRID = 0, KF_STAGE = 1, KF_EVALF = 3, KF_SOLVE = 4 };

// Implicit stages of the largest IMEX Runge-Kutta tableau the stage kernels take (ARS(4,4,3)).
constexpr int RK_MAXS = 4;

// The IMEX Runge-Kutta schemes of Ascher, Ruuth & Spiteri (1997) the 2D problem runs: explicit
// tableau A and implicit tableau H over stages 0 .. s, stage 0 the step's initial state.  Both
// have H's first column zero and one implicit diagonal value (one factorization of M + dt H_ii L
// serves every stage), and are stiffly accurate (the new state is the last stage).
struct RkTab {
  int s = 0;
  double A[RK_MAXS + 1][RK_MAXS + 1] = {};
  double H[RK_MAXS + 1][RK_MAXS + 1] = {};
};
inline RkTab rk_tableau(int scheme) {
  RkTab t;
  if (scheme == SPS_RK222) {
    // ARS(2,2,2): gamma = 1 - 1/sqrt(2), delta = 1 - 1/(2 gamma)
    const double g = 1.0 - 1.0 / std::sqrt(2.0), dl = 1.0 - 1.0 / (2.0 * g);
    t.s = 2;
    t.A[1][0] = g;
    t.A[2][0] = dl;
    t.A[2][1] = 1.0 - dl;
    t.H[1][1] = g;
    t.H[2][1] = 1.0 - g;
    t.H[2][2] = g;
  } else if (scheme == SPS_RK443) {
    // ARS(4,4,3): third order, implicit diagonal 1/2
    const double A[5][5] = {{0, 0, 0, 0, 0},
                            {1.0 / 2, 0, 0, 0, 0},
                            {11.0 / 18, 1.0 / 18, 0, 0, 0},
                            {5.0 / 6, -5.0 / 6, 1.0 / 2, 0, 0},
                            {1.0 / 4, 7.0 / 4, 3.0 / 4, -7.0 / 4, 0}};
    const double H[5][5] = {{0, 0, 0, 0, 0},
                            {0, 1.0 / 2, 0, 0, 0},
                            {0, 1.0 / 6, 1.0 / 2, 0, 0},
                            {0, -1.0 / 2, 1.0 / 2, 1.0 / 2, 0},
                            {0, 3.0 / 2, -3.0 / 2, 1.0 / 2, 1.0 / 2}};
    t.s = 4;
    for (int i = 0; i < 5; ++i)
      for (int j = 0; j < 5; ++j) {
        t.A[i][j] = A[i][j];
        t.H[i][j] = H[i][j];
      }
  }
  return t;
}

// Stage i of an IMEX Runge-Kutta step (Supplementary, "Initial value problems"; equ:imex):
//   (M + dt H_ii L) X_i = M X_0 + dt sum_{j<i} [A_ij F(X_j) - H_ij L X_j].
// The kernel that solves for X_i evaluates F(X_{i-1}) from the nonlinear terms of X_{i-1}'s
// grid fields and reads the earlier stages' states and F from their buffers.  H's first column
// is zero (stage 0 is explicit), so the implicit sum runs over j >= 1.
struct KfArgs {
  const cplx* X0;     // stage-0 state (ABI layout)
  const cplx* Xst;    // stage states X_1 .. X_{s-1}: X_j at Xst + (j - 1) sstr
  cplx* Xout;         // the stage's state (or F for KF_EVALF)
  const cplx* nl;     // [3][Ngz][K] nonlinear terms in x-spectral, z-grid form
  cplx* Fst;          // S10 N-hat of stages 0 .. s-2, [K][3][N] each: F_j at Fst + j fstr
  cplx* zg;           // [6][Ngz][K] output x-spectral z-grid fields (may be null)
  cplx* Xsave;        // second copy of the stage's new state (may be null)
  size_t sstr, fstr;  // stage-slot strides of Xst and Fst (complex entries, all instances)
  double dt;
  double fa[RK_MAXS]; // A_ij, j < i (zero beyond)
  double lh[RK_MAXS]; // H_ij, j < i (lh[0] = 0; zero beyond)
  double fself;       // A_{i,i-1}: the weight of the F evaluated in this launch
  double asum;        // sum_j A_ij: the weight of F's boundary data
  int stage, nst;     // i (1 .. s) and s
  int lx;             // some H_ij (j < i) is nonzero
  int mode;
};

// LDS: vA, vB (S complex each) persist; the rest is a union reused by the phases
// (transforms and right-hand side | block operators of the solve | output transforms).
// One entry of every length-S vector per thread (S + SPS_PAD <= NTK).
template <bool STREAM>
__global__ void __launch_bounds__(NTK) rbc_kfwd(RbcDev d, KfArgs a) {
  if (blockIdx.y) {
    const int b = blockIdx.y;
    const size_t st = (size_t)d.K * d.S, zs = (size_t)d.Ngz * d.K;
    rbc_inst(d, b);
    a.X0 = inst_ptr(a.X0, b, st);
    a.Xst = inst_ptr(a.Xst, b, st);
    a.Xout = inst_ptr(a.Xout, b, st);
    a.Xsave = inst_ptr(a.Xsave, b, st);
    a.nl = inst_ptr(a.nl, b, 3 * zs);
    a.zg = inst_ptr(a.zg, b, 6 * zs);
    a.Fst = inst_ptr(a.Fst, b, (size_t)d.K * 3 * d.N);
  } else if (d.nub) {
    rbc_inst(d, 0);
  }
  extern __shared__ double smem_d[];
  cplx* sm = reinterpret_cast<cplx*>(smem_d);
  const int k = xcd_wavenumber(blockIdx.x, d.K), tid = threadIdx.x;
  const int N = d.N, S = d.S, K = d.K, Ngz = d.Ngz, Hc = half_nodes(Ngz);
  const int mode = a.mode;
  cplx* vA = sm;                // S + SPS_PAD : right-hand side, then solution / state
  cplx* vB = vA + S + SPS_PAD;  // S : scratch
  cplx* un = vB + S;            // union
  // phase A views
  cplx* xa = un;                // S : stage-0 state
  cplx* xb = xa + S;            // S : sum_j H_ij X_j of the earlier stages
  cplx* rr = xb + S;            // S : right-hand side (equation slots)
  cplx* pq = rr + S;            // 6*Hc mirror sums of the three nonlinear terms
  cplx* nh = pq + 6 * Hc;       // 3*N  N-hat
  cplx* fr = nh + 3 * N;        // 3*N  S10 N-hat
  double* ct = reinterpret_cast<double*>(fr + 3 * N);   // 4*Ngz cosines
  const bool stage = mode == KF_STAGE;
  const bool nonlin = stage || mode == KF_EVALF;
  const int si = a.stage;

  // Global reads, in the order they are needed: the states and earlier F (combined as they
  // arrive), the mirror pair of the nonlinear terms and one cosine per thread first, then the
  // permutation maps and the block operators (needed last).
  const double kxk = d.kx[k];
  const cplx x0 = (mode != KF_EVALF && tid < S) ? a.X0[(size_t)k * S + tid] : czero();
  // (loops over the tableau's fixed size, so that the coefficients are read at constant
  // indices; the host zeroes them beyond the stage.  Loaded here, combined once every load is
  // issued: a sum taken as the loads arrive would wait for each before issuing the next.)
  cplx xs[RK_MAXS - 1], fs[RK_MAXS - 1];
#pragma unroll
  for (int j = 1; j < RK_MAXS; ++j)
    xs[j - 1] = (stage && j < si && a.lh[j] != 0.0 && tid < S)
                    ? a.Xst[(size_t)(j - 1) * a.sstr + (size_t)k * S + tid] : czero();
#pragma unroll
  for (int j = 0; j + 1 < RK_MAXS; ++j)
    fs[j] = (stage && j + 1 < si && a.fa[j] != 0.0 && tid < 3 * N)
                ? a.Fst[(size_t)j * a.fstr + (size_t)k * 3 * N + tid] : czero();
  const int pf = tid / Hc, pj = tid - pf * Hc, pjm = Ngz - 1 - pj;
  const bool pl = nonlin && tid < 3 * Hc;
  const cplx nvj = pl ? a.nl[((size_t)pf * Ngz + pj) * K + k] : czero();
  const cplx nvm = pl ? a.nl[((size_t)pf * Ngz + pjm) * K + k] : czero();
  const double cosr = (tid < 4 * Ngz) ? d.cosz[tid] : 0.0;
  OpsRegs opsr;
  MapRegs mr;
  // (issued in every mode, so that no load is under a branch; T blocks first: the first sweep
  // needs them, the G blocks arrive during it)
  load_maps(d, mr);
  if (!STREAM) ops_issue(d.ops + (size_t)k * d.opsize, d.tsz, d.blksz - d.tsz, opsr);
  cplx xc = czero(), fc = czero();
  if (stage) {
#pragma unroll
    for (int j = 1; j < RK_MAXS; ++j)
      if (j < si && a.lh[j] != 0.0) xc = cadd(xc, cscale(xs[j - 1], a.lh[j]));
#pragma unroll
    for (int j = 0; j + 1 < RK_MAXS; ++j)
      if (j + 1 < si && a.fa[j] != 0.0) fc = cadd(fc, cscale(fs[j], a.fa[j]));
  }
  if (stage) {
    if (tid < S) {
      xa[tid] = x0;
      xb[tid] = xc;
    }
    if (tid < 3 * N) vB[tid] = fc;    // sum_{j < i-1} A_ij F_j; vB is free until the solve
  }
  const cplx* f0s = vB;
  if (nonlin) {
    if (tid < 4 * Ngz) ct[tid] = cosr;
    if (pl) store_mirror_pair(nvj, nvm, pjm == pj, pq + 2 * (pf * Hc + pj));
    __syncthreads();
    // Chebyshev forward transform (truncating) of the three nonlinear terms: 8 lanes per mode
    for (int e = tid; e < 8 * N; e += NTK) {
      const int n = e >> 3, h = e & 7;
      cplx acc[3];
      nodes_to_mode<3, 8>(ct, pq, Hc, Ngz, n, h, acc);
      const double sc = (n == 0 ? 1.0 : 2.0) / Ngz;
      if (h == 0) {
#pragma unroll
        for (int f = 0; f < 3; ++f) nh[f * N + n] = cscale(acc[f], sc);
      }
    }
    __syncthreads();
    if (tid < 3 * N) {
      const int f = tid / N, n = tid - f * N;
      fr[tid] = s10_at(nh + f * N, n, N);
    }
    __syncthreads();
    if (mode == KF_EVALF) {
      if (tid < S) {
        cplx v = (tid < 3 * N) ? fr[tid] : czero();
        if (k == 0 && tid == 4 * N + 4) v = cadd(v, cmk(d.bc0, 0.0));
        a.Xout[(size_t)k * S + tid] = v;
      }
      return;
    }
    // F of stage i-1, kept for the later stages
    if (stage && si < a.nst && tid < 3 * N) a.Fst[(size_t)(si - 1) * a.fstr + (size_t)k * 3 * N + tid] = fr[tid];
  }
  if (stage) {
    const double dt = a.dt, fl = a.fself;
    if (tid < 4 * N) {
      const int s = tid;
      const MLRow r0 = ml_row(d, k, kxk, xa, s);
      cplx comb = (s < 3 * N) ? cadd(f0s[s], cscale(fr[s], fl)) : czero();
      if (a.lx) comb = csub(comb, ml_row(d, k, kxk, xb, s).l);
      rr[s] = cadd(r0.m, cscale(comb, dt));
    } else if (tid < 4 * N + 28) {
      // boundary and gauge rows: M is zero there and every stage's F holds the boundary data
      // (b = 1 at z = 0 for k = 0), so the row is dt (sum_j A_ij F - L sum_j H_ij X_j)
      const int q = (tid - 4 * N) >> 2, h = tid & 3;
      if (q < 6 || k != 0) {   // (the k = 0 gauge row: the last wave, below)
        const double fbc = (k == 0 && q == 4) ? d.bc0 : 0.0;
        cplx v = cmk(a.asum * fbc, 0.0);
        if (a.lx) v = csub(v, l_bc_row(d, k, xb, q, h));
        if (h == 0) rr[4 * N + q] = cscale(v, dt);
      }
    } else if (k == 0 && tid >= NTK - SPS_WAVE) {
      // the k = 0 gauge row, -dt (the mean of p): one mode per lane of the (otherwise idle) last
      // wave, so that the integration weights' divisions run side by side instead of sixteen in
      // a row on one quad
      const int m = tid - (NTK - SPS_WAVE);
      cplx v = (a.lx && m < N) ? cscale(xb[3 * N + m], -intw_at(m)) : czero();
      for (int o = SPS_WAVE / 2; o >= 1; o >>= 1) {
        v.x += __shfl_xor(v.x, o);
        v.y += __shfl_xor(v.y, o);
      }
      if (m == 0) rr[4 * N + 6] = cscale(v, dt);
    }
    __syncthreads();
  } else if (mode == KF_SOLVE) {
    if (tid < S) rr[tid] = x0;
    __syncthreads();
  }
  if (mode == KF_ZGRID) {
    if (tid < S) vA[tid] = x0;
    __syncthreads();
  } else {
    if (!STREAM) stage_early(d, opsr, reinterpret_cast<double*>(un), false);
    rbc_gather(d, mr, rr, vA);
    rbc_solve<STREAM>(d, k, opsr, reinterpret_cast<double*>(un), vA, vB, false);
    rbc_scatter(d, mr, vA, vB, vA);   // vA <- new state (ABI slots)
    if (tid < S) {
      const cplx v = vA[tid];
      a.Xout[(size_t)k * S + tid] = v;
      if (a.Xsave) a.Xsave[(size_t)k * S + tid] = v;
      if (stage && si == a.nst && __any(!(isfinite(v.x) && isfinite(v.y))) && lane_id() == 0) atomicOr(d.err, 2);
    }
  }
  if (a.zg == nullptr || mode == KF_SOLVE) return;
  // backward Chebyshev transforms of u, w, b (from vA) and of their z-derivatives
  double* ct2 = reinterpret_cast<double*>(un);
  cplx* dz = reinterpret_cast<cplx*>(ct2 + 4 * Ngz);   // 3*N
  if (tid < 4 * Ngz) ct2[tid] = cosr;
  if (tid < 3 * SPS_WAVE) dz_coefs_wave(vA, N, dz);
  __syncthreads();
  // a quad per (field group, mirror pair): group 0 = u, w, b; group 1 = their z-derivatives
  for (int e = tid; e < 8 * Hc; e += NTK) {
    const int h = e & 3, it = e >> 2, grp = it / Hc, j = it - grp * Hc, jm = Ngz - 1 - j;
    cplx val[3];
    modes_to_pair<3>(ct2, grp == 0 ? vA : dz, N, N, Ngz, j, h, val);
    if (h == 0 || (h == 1 && jm != j)) {
      const int jj = (h == 0) ? j : jm;
#pragma unroll
      for (int f = 0; f < 3; ++f) a.zg[((size_t)(3 * grp + f) * Ngz + jj) * K + k] = val[f];
    }
  }
}

// ---------------------------------------------------------------------------- grid-row kernels
// Hermitian packing of two half spectra U, V (K modes) into one length-n complex spectrum
// whose inverse DFT is u + i v (u, v real).  scale multiplies modes m >= 1.
__device__ __forceinline__ cplx pack_pair(const cplx* U, const cplx* V, int m, int n, int K, double scale) {
  if (m == 0) return cmk(U[0].x, V ? V[0].x : 0.0);
  if (m < K) {
    const cplx u = U[m], v = V ? V[m] : czero();
    return cscale(cmk(u.x - v.y, u.y + v.x), scale);
  }
  if (m > n - K) {
    const int q = n - m;
    const cplx u = U[q], v = V ? V[q] : czero();
    return cscale(cmk(u.x + v.y, v.x - u.y), scale);
  }
  return czero();
}

struct XfArgs {
  const cplx* zg;   // [6][Ngz][K] u, w, b, uz, wz, bz
  cplx* nl;         // [3][Ngz][K]
};

__global__ void __launch_bounds__(NTX) rbc_xfwd(RbcDev d, XfArgs a) {
  if (blockIdx.y) {
    const size_t zs = (size_t)d.Ngz * d.K;
    a.zg = inst_ptr(a.zg, blockIdx.y, 6 * zs);
    a.nl = inst_ptr(a.nl, blockIdx.y, 3 * zs);
  }
  extern __shared__ double smem_d[];
  cplx* sm = reinterpret_cast<cplx*>(smem_d);
  const int j = blockIdx.x, tid = threadIdx.x;
  const int K = d.K, Ngx = d.Ngx, Ngz = d.Ngz;
  cplx* spec = sm;                 // 9*K : u w b uz wz bz ux wx bx
  cplx* buf0 = spec + 9 * K;                // 4*Ngx (padded)
  cplx* buf1 = buf0 + fpad_size(4 * Ngx);   // 4*Ngx (padded)
  cplx* tw = buf1 + fpad_size(4 * Ngx);     // Ngx twiddles
  for (int e = tid; e < Ngx; e += NTX) tw[e] = d.twx[e];
  for (int e = tid; e < 6 * K; e += NTX) {
    const int f = e / K, m = e - f * K;
    spec[e] = a.zg[((size_t)f * Ngz + j) * K + m];
  }
  __syncthreads();
  for (int e = tid; e < 3 * K; e += NTX) {
    const int f = e / K, m = e - f * K;
    spec[(6 + f) * K + m] = cscale(cmul_i(spec[f * K + m]), d.kx[m]);
  }
  __syncthreads();
  // pairs: (u, w), (ux, uz), (wx, wz), (bx, bz)
  const int pu[4] = {0, 6, 7, 8};
  const int pv[4] = {1, 3, 4, 5};
  for (int e = tid; e < 4 * Ngx; e += NTX) {
    const int q = e / Ngx, m = e - q * Ngx;
    const cplx* U = spec + pu[q] * K;
    const cplx* V = spec + pv[q] * K;
    buf0[fpad(e)] = pack_pair(U, V, m, Ngx, K, 1.0);
  }
  __syncthreads();
  cplx* g = lds_fft(buf0, buf1, d.px, tw, +1, 4, Ngx, tid, NTX);
  cplx* o = (g == buf0) ? buf1 : buf0;
  for (int x = tid; x < Ngx; x += NTX) {
    const double u = g[fpad(x)].x, w = g[fpad(x)].y;
    const double ux = g[fpad(Ngx + x)].x, uz = g[fpad(Ngx + x)].y;
    const double wx = g[fpad(2 * Ngx + x)].x, wz = g[fpad(2 * Ngx + x)].y;
    const double bx = g[fpad(3 * Ngx + x)].x, bz = g[fpad(3 * Ngx + x)].y;
    const double Nu = -(u * ux + w * uz);
    const double Nw = -(u * wx + w * wz);
    const double Nb = -(u * bx + w * bz);
    o[fpad(x)] = cmk(Nu, Nw);
    o[fpad(Ngx + x)] = cmk(Nb, 0.0);
  }
  __syncthreads();
  cplx* h = lds_fft(o, g, d.px, tw, -1, 2, Ngx, tid, NTX);
  const double inv = 1.0 / Ngx;
  for (int e = tid; e < 3 * K; e += NTX) {
    const int f = e / K, m = e - f * K;
    const cplx* Z = h;
    const int zo = (f == 2) ? Ngx : 0;
    const cplx zm = Z[fpad(zo + m)], zq = Z[fpad(zo + (m == 0 ? 0 : Ngx - m))];
    cplx c;
    if (f == 0) c = cmk(0.5 * (zm.x + zq.x), 0.5 * (zm.y - zq.y));
    else if (f == 1) c = cmk(0.5 * (zm.y + zq.y), -0.5 * (zm.x - zq.x));
    else c = cmk(0.5 * (zm.x + zq.x), 0.5 * (zm.y - zq.y));
    a.nl[((size_t)f * Ngz + j) * K + m] = cscale(c, inv);
  }
}

struct XaArgs {
  const cplx* nlbar;  // [3][Ngz][K] cotangents of the x-spectra of N_u, N_w, N_b
  const cplx* zg;     // [6][Ngz][K] primal fields of the stage
  cplx* zbar;         // [6][Ngz][K] cotangents of u, w, b, uz, wz, bz x-spectra
};

__global__ void __launch_bounds__(NTX) rbc_xadj(RbcDev d, XaArgs a) {
  if (blockIdx.y) {
    const size_t zs = (size_t)d.Ngz * d.K;
    a.nlbar = inst_ptr(a.nlbar, blockIdx.y, 3 * zs);
    a.zg = inst_ptr(a.zg, blockIdx.y, 6 * zs);
    a.zbar = inst_ptr(a.zbar, blockIdx.y, 6 * zs);
  }
  extern __shared__ double smem_d[];
  cplx* sm = reinterpret_cast<cplx*>(smem_d);
  const int j = blockIdx.x, tid = threadIdx.x;
  const int K = d.K, Ngx = d.Ngx, Ngz = d.Ngz;
  cplx* spec = sm;                  // 12*K: u w b uz wz bz ux wx bx | nub nwb nbb
  cplx* buf0 = spec + 12 * K;               // 6*Ngx (padded)
  cplx* buf1 = buf0 + fpad_size(6 * Ngx);   // 6*Ngx (padded)
  cplx* tw = buf1 + fpad_size(6 * Ngx);     // Ngx twiddles
  for (int e = tid; e < Ngx; e += NTX) tw[e] = d.twx[e];
  for (int e = tid; e < 6 * K; e += NTX) {
    const int f = e / K, m = e - f * K;
    spec[e] = a.zg[((size_t)f * Ngz + j) * K + m];
  }
  for (int e = tid; e < 3 * K; e += NTX) {
    const int f = e / K, m = e - f * K;
    spec[(9 + f) * K + m] = a.nlbar[((size_t)f * Ngz + j) * K + m];
  }
  __syncthreads();
  for (int e = tid; e < 3 * K; e += NTX) {
    const int f = e / K, m = e - f * K;
    spec[(6 + f) * K + m] = cscale(cmul_i(spec[f * K + m]), d.kx[m]);
  }
  __syncthreads();
  // buffers 0..3: primal pairs; 4: (Nu_bar, Nw_bar) with halved m >= 1 weights; 5: (Nb_bar, 0)
  const int pu[6] = {0, 6, 7, 8, 9, 11};
  const int pv[6] = {1, 3, 4, 5, 10, -1};
  for (int e = tid; e < 6 * Ngx; e += NTX) {
    const int q = e / Ngx, m = e - q * Ngx;
    const cplx* U = spec + pu[q] * K;
    const cplx* V = (pv[q] >= 0) ? spec + pv[q] * K : nullptr;
    buf0[fpad(e)] = pack_pair(U, V, m, Ngx, K, q >= 4 ? 0.5 : 1.0);
  }
  __syncthreads();
  cplx* g = lds_fft(buf0, buf1, d.px, tw, +1, 6, Ngx, tid, NTX);
  cplx* o = (g == buf0) ? buf1 : buf0;
  const double inv = 1.0 / Ngx;
  for (int x = tid; x < Ngx; x += NTX) {
    const double u = g[fpad(x)].x, w = g[fpad(x)].y;
    const double ux = g[fpad(Ngx + x)].x, uz = g[fpad(Ngx + x)].y;
    const double wx = g[fpad(2 * Ngx + x)].x, wz = g[fpad(2 * Ngx + x)].y;
    const double bx = g[fpad(3 * Ngx + x)].x, bz = g[fpad(3 * Ngx + x)].y;
    const double Nub = g[fpad(4 * Ngx + x)].x * inv, Nwb = g[fpad(4 * Ngx + x)].y * inv;
    const double Nbb = g[fpad(5 * Ngx + x)].x * inv;
    const double ub = -(Nub * ux + Nwb * wx + Nbb * bx);
    const double wb = -(Nub * uz + Nwb * wz + Nbb * bz);
    o[fpad(x)] = cmk(ub, wb);
    o[fpad(Ngx + x)] = cmk(-Nub * u, -Nub * w);          // ux_bar, uz_bar
    o[fpad(2 * Ngx + x)] = cmk(-Nwb * u, -Nwb * w);      // wx_bar, wz_bar
    o[fpad(3 * Ngx + x)] = cmk(-Nbb * u, -Nbb * w);      // bx_bar, bz_bar
  }
  __syncthreads();
  cplx* h = lds_fft(o, g, d.px, tw, -1, 4, Ngx, tid, NTX);
  // unpack: A_m = (Z_m + conj Z_-m)/2, B_m = (Z_m - conj Z_-m)/(2i); weight 1 at m = 0, 2 else
  for (int e = tid; e < 3 * K; e += NTX) {
    const int f = e / K, m = e - f * K;
    const double wgt = (m == 0) ? 1.0 : 2.0;
    const double kx = d.kx[m];
    auto unpack = [&](int q, cplx& A, cplx& B) {
      const cplx zm = h[fpad(q * Ngx + m)], zq = h[fpad(q * Ngx + (m == 0 ? 0 : Ngx - m))];
      A = cscale(cmk(0.5 * (zm.x + zq.x), 0.5 * (zm.y - zq.y)), wgt);
      B = cscale(cmk(0.5 * (zm.y + zq.y), -0.5 * (zm.x - zq.x)), wgt);
    };
    cplx A0, B0, Ad, Bd;
    unpack(0, A0, B0);        // u_bar, w_bar
    unpack(1 + f, Ad, Bd);    // (ux_bar, uz_bar) / (wx_bar, wz_bar) / (bx_bar, bz_bar)
    // x-derivative transposed: conj(i kx) = -i kx
    const cplx dxt = cscale(cmul_mi(Ad), kx);
    cplx base = (f == 0) ? A0 : (f == 1 ? B0 : czero());
    a.zbar[((size_t)f * Ngz + j) * K + m] = cadd(base, dxt);
    a.zbar[((size_t)(3 + f) * Ngz + j) * K + m] = Bd;
  }
}

// Grid-row kernels with one wavefront per length-Ngx FFT (Ngx = 64 R1, R1 = 3 or 6, i.e. nx = 128
// or 256): the same transforms and products as rbc_xfwd / rbc_xadj, with the FFTs of wave_fft.h
// (registers, two in-wave LDS exchanges, no block barrier inside a transform).  Each wave packs
// its pair of real rows (Hermitian packing of two half spectra, read straight from global
// memory), the inverse FFTs leave the grid rows in the permuted layout, the products are formed
// in that layout, and the forward FFTs return natural-order spectra for the truncation.
template <int R1>
struct WaveRow {
  static constexpr int N = 64 * R1;      // Ngx
  static constexpr int K = N / 3;        // kept modes
  static constexpr int SC = (N + (N >> 3) + 1 + 1) & ~1;   // fpad_size(N), rounded to even
};

// Natural-layout entries a[q] = packed spectrum at m = l + 64 q of the pair (U, V): U the
// x-spectrum of field fu (times i kx when du), V that of field fv (none when fv < 0), modes
// m >= 1 scaled by sc.  src: [fields][Ngz][K] at row j.
template <int R1>
__device__ __forceinline__ void pack_pair_row(const RbcDev& d, const cplx* src, int j, int fu, bool du, int fv,
                                              double scl, cplx (&a)[R1]) {
  constexpr int N = WaveRow<R1>::N, K = WaveRow<R1>::K;
  const int l = lane_id(), Ngz = d.Ngz;
  const cplx* U = src + ((size_t)fu * Ngz + j) * K;
  // (without a V the U row is read in its place and the values dropped: every load is issued
  // unconditionally, since a load under a branch makes the first use wait for all of them)
  const cplx* V = src + ((size_t)(fv >= 0 ? fv : fu) * Ngz + j) * K;
  cplx uu[R1], vv[R1];
  double kk[R1];
#pragma unroll
  for (int q = 0; q < R1; ++q) {
    const int m = l + 64 * q;
    const int sidx = m < K ? m : (m > N - K ? N - m : 0);
    uu[q] = U[sidx];
    vv[q] = V[sidx];
    kk[q] = d.kx[sidx];
  }
#pragma unroll
  for (int q = 0; q < R1; ++q) {
    const int m = l + 64 * q;
    const bool lowm = m < K, highm = m > N - K;
    cplx u = czero(), v = czero();
    if (lowm || highm) {
      u = du ? cscale(cmul_i(uu[q]), kk[q]) : uu[q];
      v = fv >= 0 ? vv[q] : czero();
    }
    cplx r;
    if (m == 0) r = cmk(u.x, v.x);
    else if (lowm) r = cscale(cmk(u.x - v.y, u.y + v.x), scl);
    else if (highm) r = cscale(cmk(u.x + v.y, v.x - u.y), scl);
    else r = czero();
    a[q] = r;
  }
}

template <int R1>
__global__ void __launch_bounds__(256) rbc_xfwd_w(RbcDev d, XfArgs a) {
  if (blockIdx.y) {
    const size_t zs = (size_t)d.Ngz * d.K;
    a.zg = inst_ptr(a.zg, blockIdx.y, 6 * zs);
    a.nl = inst_ptr(a.nl, blockIdx.y, 3 * zs);
  }
  using W = WaveRow<R1>;
  constexpr int N = W::N, K = W::K, SC = W::SC;
  extern __shared__ double smem_d[];
  cplx* tw = reinterpret_cast<cplx*>(smem_d);   // N
  cplx* scr = tw + N;                            // 4 x SC: each wave's FFT exchange scratch
  // Grid rows in the permuted layout (8 registers x 8 R1 active lanes = N entries per wave).
  // Waves 0 and 1 go on to the products and the forward FFTs, so theirs get a region of their
  // own; waves 2 and 3 are done after the inverse FFT and keep theirs in their own scratch.
  // (The block takes 3 N + 4 SC complex entries, three blocks per CU.)
  static_assert(N <= SC, "a wave's grid rows fit its FFT scratch");
  cplx* G01 = scr + 4 * SC;                      // 2 x N
  const int j = blockIdx.x, tid = threadIdx.x, wv = tid >> 6, l = lane_id();
  cplx* sc = scr + wv * SC;
  // pair wv: (u, w), (ux, uz), (wx, wz), (bx, bz)
  cplx av[R1];
  pack_pair_row<R1>(d, a.zg, j, wv == 0 ? 0 : wv - 1, wv > 0, wv == 0 ? 1 : wv + 2, 1.0, av);
  for (int e = tid; e < N; e += 256) tw[e] = d.twx[e];
  __syncthreads();
  cplx pv[8];
  wfft_a_to_p<R1, +1>(av, pv, sc, tw);
  if (l < 8 * R1) {
    cplx* gw = wv < 2 ? G01 + wv * N : sc;
#pragma unroll
    for (int h = 0; h < 8; ++h) gw[h * 8 * R1 + l] = pv[h];
  }
  __syncthreads();
  if (wv >= 2) return;
  if (l < 8 * R1) {
    const cplx* G0 = G01;
    const cplx* G1 = G01 + N;
    const cplx* G2 = scr + 2 * SC;
    const cplx* G3 = scr + 3 * SC;
    // (the wave's branch outside the loops: a branch between the rows would make every row's
    // LDS reads wait for the previous row's)
    if (wv == 0) {
#pragma unroll
      for (int h = 0; h < 8; ++h) {
        const int e = h * 8 * R1 + l;
        const cplx uw = G0[e], ud = G1[e], wd = G2[e];
        pv[h] = cmk(-(uw.x * ud.x + uw.y * ud.y), -(uw.x * wd.x + uw.y * wd.y));   // N_u, N_w
      }
    } else {
#pragma unroll
      for (int h = 0; h < 8; ++h) {
        const int e = h * 8 * R1 + l;
        const cplx uw = G0[e], bd = G3[e];
        pv[h] = cmk(-(uw.x * bd.x + uw.y * bd.y), 0.0);                            // N_b
      }
    }
  }
  wfft_p_to_a<R1, -1>(pv, av, sc, tw);
#pragma unroll
  for (int q = 0; q < R1; ++q) sc[fpad(q * 64 + l)] = av[q];
  wave_lds_sync();
  constexpr double inv = 1.0 / N;
  const int Ngz = d.Ngz;
#pragma unroll
  for (int t = 0; t < (K + 63) / 64; ++t) {
    const int m = l + 64 * t;
    if (m >= K) break;
    const cplx zm = sc[fpad(m)], zq = sc[fpad(m == 0 ? 0 : N - m)];
    if (wv == 0) {
      a.nl[((size_t)0 * Ngz + j) * K + m] = cscale(cmk(0.5 * (zm.x + zq.x), 0.5 * (zm.y - zq.y)), inv);
      a.nl[((size_t)1 * Ngz + j) * K + m] = cscale(cmk(0.5 * (zm.y + zq.y), -0.5 * (zm.x - zq.x)), inv);
    } else {
      a.nl[((size_t)2 * Ngz + j) * K + m] = cscale(cmk(0.5 * (zm.x + zq.x), 0.5 * (zm.y - zq.y)), inv);
    }
  }
}

template <int R1>
__global__ void __launch_bounds__(384) rbc_xadj_w(RbcDev d, XaArgs a) {
  if (blockIdx.y) {
    const size_t zs = (size_t)d.Ngz * d.K;
    a.nlbar = inst_ptr(a.nlbar, blockIdx.y, 3 * zs);
    a.zg = inst_ptr(a.zg, blockIdx.y, 6 * zs);
    a.zbar = inst_ptr(a.zbar, blockIdx.y, 6 * zs);
  }
  using W = WaveRow<R1>;
  constexpr int N = W::N, K = W::K, SC = W::SC;
  extern __shared__ double smem_d[];
  cplx* tw = reinterpret_cast<cplx*>(smem_d);   // N
  cplx* scr = tw + N;                            // 6 x SC: each wave's FFT exchange scratch
  // Grid rows in the permuted layout (N entries per wave): waves 0-3 go on to the products and
  // the forward FFTs and get a region of their own; waves 4 and 5 (the cotangent pairs) are
  // done after the inverse FFT and keep theirs in their own scratch.  (The block takes
  // 5 N + 6 SC complex entries, two blocks per CU.)
  static_assert(N <= SC, "a wave's grid rows fit its FFT scratch");
  cplx* G03 = scr + 6 * SC;                      // 4 x N
  const int j = blockIdx.x, tid = threadIdx.x, wv = tid >> 6, l = lane_id();
  cplx* sc = scr + wv * SC;
  // pairs: (u, w), (ux, uz), (wx, wz), (bx, bz), (Nu_bar, Nw_bar) and (Nb_bar, 0) with halved
  // weights of the modes m >= 1 (the transposed forward transform of a real row)
  cplx av[R1];
  if (wv < 4) pack_pair_row<R1>(d, a.zg, j, wv == 0 ? 0 : wv - 1, wv > 0, wv == 0 ? 1 : wv + 2, 1.0, av);
  else pack_pair_row<R1>(d, a.nlbar, j, wv == 4 ? 0 : 2, false, wv == 4 ? 1 : -1, 0.5, av);
  for (int e = tid; e < N; e += 384) tw[e] = d.twx[e];
  __syncthreads();
  cplx pv[8];
  wfft_a_to_p<R1, +1>(av, pv, sc, tw);
  if (l < 8 * R1) {
    cplx* gw = wv < 4 ? G03 + wv * N : sc;
#pragma unroll
    for (int h = 0; h < 8; ++h) gw[h * 8 * R1 + l] = pv[h];
  }
  __syncthreads();
  if (wv < 4) {
    if (l < 8 * R1) {
      constexpr double inv = 1.0 / N;
      const cplx* G4 = scr + 4 * SC;
      const cplx* G5 = scr + 5 * SC;
      // (the wave's branch outside the loops: a branch between the rows would make every row's
      // LDS reads wait for the previous row's)
      if (wv == 0) {
#pragma unroll
        for (int h = 0; h < 8; ++h) {
          const int e = h * 8 * R1 + l;
          const cplx nb = G4[e];
          const double Nub = nb.x * inv, Nwb = nb.y * inv, Nbb = G5[e].x * inv;
          const cplx ud = G03[N + e], wd = G03[2 * N + e], bd = G03[3 * N + e];
          pv[h] = cmk(-(Nub * ud.x + Nwb * wd.x + Nbb * bd.x), -(Nub * ud.y + Nwb * wd.y + Nbb * bd.y));
        }
      } else {
        // (x-derivative bar, z-derivative bar) of u, w or b: the cotangent Nu_bar, Nw_bar or Nb_bar
        // of wave 1, 2 or 3 times (u, w)
        const cplx* Gc = wv == 3 ? G5 : G4;
        const bool im = wv == 2;
#pragma unroll
        for (int h = 0; h < 8; ++h) {
          const int e = h * 8 * R1 + l;
          const cplx nb = Gc[e];
          const double c = (im ? nb.y : nb.x) * inv;
          const cplx uw = G03[e];
          pv[h] = cmk(-c * uw.x, -c * uw.y);
        }
      }
    }
    wfft_p_to_a<R1, -1>(pv, av, sc, tw);
#pragma unroll
    for (int q = 0; q < R1; ++q) sc[fpad(q * 64 + l)] = av[q];
  }
  __syncthreads();
  // unpack A_m = (Z_m + conj Z_-m)/2, B_m = (Z_m - conj Z_-m)/(2i), weight 1 at m = 0, 2 else
  const int Ngz = d.Ngz;
  for (int e = tid; e < 3 * K; e += 384) {
    const int f = e / K, m = e - f * K;
    const double wgt = (m == 0) ? 1.0 : 2.0;
    auto unpack = [&](int q, cplx& A, cplx& B) {
      const cplx* Z = scr + q * SC;
      const cplx zm = Z[fpad(m)], zq = Z[fpad(m == 0 ? 0 : N - m)];
      A = cscale(cmk(0.5 * (zm.x + zq.x), 0.5 * (zm.y - zq.y)), wgt);
      B = cscale(cmk(0.5 * (zm.y + zq.y), -0.5 * (zm.x - zq.x)), wgt);
    };
    cplx A0, B0, Ad, Bd;
    unpack(0, A0, B0);
    unpack(1 + f, Ad, Bd);
    const cplx dxt = cscale(cmul_mi(Ad), d.kx[m]);
    const cplx base = (f == 0) ? A0 : (f == 1 ? B0 : czero());
    a.zbar[((size_t)f * Ngz + j) * K + m] = cadd(base, dxt);
    a.zbar[((size_t)(3 + f) * Ngz + j) * K + m] = Bd;
  }
}

// ---------------------------------------------------------------------------- per-wavenumber adjoint kernel
enum KaFlags { KA_C = 1, KA_A = 2, KA_B = 4, KA_G = 8, KA_SOLVE_T = 16 };

// Reverse of stage m of an IMEX Runge-Kutta step (Supplementary, RK adjoint equations), with
// Y_j the stage adjoints:
//   (M + dt H_mm L)^H Y_m = dF(X_m)^H (dt sum_{j>m} A_jm Y_j) - dt L^H sum_{j>m} H_jm Y_j
// (for m = s the right-hand side is the cotangent of the step's new state), and the step's
// initial-state cotangent M^H sum_j Y_j + dF(X_0)^H (dt sum_j A_j0 Y_j) (H's first column is
// zero).  The kernel of stage m (KA_A for m = s, KA_B below) solves for Y_m, hands the
// cotangent dt sum_{j>=m} A_{j,m-1} Y_j of F(X_{m-1}) to the grid-row adjoint, and (m = 1)
// forms M^H sum_j Y_j for the KA_C step that adds the last F-VJP.
struct KaArgs {
  const cplx* zbar;   // [6][Ngz][K]
  const cplx* Xb_in;  // cotangent of the step's final state (KA_A without KA_C) or F-bar (KA_G) or rhs (KA_SOLVE_T)
  cplx* Xb_out;       // cotangent of the step's initial state (KA_C) or solution (KA_SOLVE_T)
  cplx* acc;          // [K][S] M^H (Y_1 + ... + Y_s)
  cplx* Ybuf;         // stage adjoints Y_2 .. Y_s, [K][S] each: Y_j at Ybuf + (j - 2) sstr
  cplx* nlbar;        // [3][Ngz][K]
  const cplx* Xm;     // parameter gradient (may be null): the stage state X_m (X_s: the step's new state)
  double* pacc;       //   [K][2] accumulated dJ/dnu, dJ/dkappa of each wavenumber
  size_t sstr;        // stage-slot stride of Ybuf (complex entries, all instances)
  double dt;
  double hc[RK_MAXS + 1];   // H_jm, j = m+1 .. s (zero elsewhere)
  double fc[RK_MAXS + 1];   // A_{j,m-1}, j = m+1 .. s (zero elsewhere)
  double hself, fself;      // H_mm and A_{m,m-1}
  int stage, nst;           // m and s
  int flags;
};

// Row s < 3N of (dL/dp) X for p = nu (u, w rows) or kappa (b rows): the viscous or diffusive
// operator -(DZZ - kx^2 S10) of the row's field and its lifted first-order tau.
__device__ __forceinline__ cplx dl_row(const RbcDev& d, int k, const cplx* X, int s) {
  const int N = d.N, f = s / N, n = s - f * N;
  const double kx = d.kx[k];
  const cplx* c = X + f * N;
  cplx v = cadd(cscale(dzz_at(c, n, N), -1.0), cscale(s10_at(c, n, N), kx * kx));
  if (n == N - 2) v = csub(v, cscale(X[4 * N + f], 4.0));
  return v;
}

// pacc[k] += -dt <W_m, dL X_m> for dL = dL/dnu, dL/dkappa and W_m = sum_{j>=m} H_jm Y_j: stage
// m's share of -sum_i <Y_i, dR_i/dp>, the stage residuals' parameter derivatives
// dR_i/dp = dt sum_{j<=i} H_ij dL X_j against the stage adjoints (equ:efficient_gradient),
// regrouped by state.  w: this thread's entry of W_m; Xm in LDS (ABI slots); red: 2 * (NTK / 64)
// doubles.  Block-wide.
__device__ void param_accumulate(const RbcDev& d, const KaArgs& a, int k, cplx w, const cplx* Xm, double* red) {
  const int tid = threadIdx.x, N = d.N;
  double cn = 0.0, ck = 0.0;
  if (tid < 3 * N) {
    const cplx l = dl_row(d, k, Xm, tid);
    const double v = w.x * l.x + w.y * l.y;
    if (tid < 2 * N) cn = v;
    else ck = v;
  }
  for (int o = 32; o >= 1; o >>= 1) {
    cn += __shfl_xor(cn, o);
    ck += __shfl_xor(ck, o);
  }
  const int wv = tid >> 6;
  if ((tid & 63) == 0) {
    red[2 * wv] = cn;
    red[2 * wv + 1] = ck;
  }
  __syncthreads();
  if (tid == 0) {
    double sn = 0.0, sk = 0.0;
    for (int w = 0; w < NTK / 64; ++w) {
      sn += red[2 * w];
      sk += red[2 * w + 1];
    }
    a.pacc[2 * k] -= a.dt * sn;
    a.pacc[2 * k + 1] -= a.dt * sk;
  }
}

// The zbar entries of mirror pair (f, j) = (tid / Hc, tid % Hc), f < 6, read by each thread at
// kernel start (6 Hc <= NTK).
struct ZbarPair {
  cplx vj, vm;
  bool on;
};
__device__ __forceinline__ ZbarPair load_zbar_pair(const RbcDev& d, const KaArgs& a, int k, bool want) {
  const int Hc = half_nodes(d.Ngz), tid = threadIdx.x;
  const int f = tid / Hc, j = tid - f * Hc, jm = d.Ngz - 1 - j;
  ZbarPair z;
  z.on = want && tid < 6 * Hc;
  z.vj = z.on ? a.zbar[((size_t)f * d.Ngz + j) * d.K + k] : czero();
  z.vm = z.on ? a.zbar[((size_t)f * d.Ngz + jm) * d.K + k] : czero();
  return z;
}

// c_bar for u, w, b from zbar (adjoint Chebyshev backward transform + derivative transposes).
// pqz: 12*Hc, cb: 6*N, out: 3*N, ct: staged cosines.  Block-wide.
__device__ void zbar_to_coeffs(const RbcDev& d, const ZbarPair& zp, const double* ct, cplx* pqz, cplx* cb,
                               cplx* out) {
  const int tid = threadIdx.x, N = d.N, Ngz = d.Ngz, Hc = half_nodes(Ngz);
  if (zp.on) {
    const int f = tid / Hc, j = tid - f * Hc;
    store_mirror_pair(zp.vj, zp.vm, Ngz - 1 - j == j, pqz + 2 * (f * Hc + j));
  }
  __syncthreads();
  // transposed (unscaled) backward transform: 4 lanes per (field group of 3, mode)
  for (int e = tid; e < 8 * N; e += NTK) {
    const int h = e & 3, it = e >> 2, grp = it / N, n = it - grp * N;
    cplx acc[3];
    nodes_to_mode<3, 4>(ct, pqz + 6 * Hc * grp, Hc, Ngz, n, h, acc);
    if (h == 0) {
#pragma unroll
      for (int f = 0; f < 3; ++f) cb[(3 * grp + f) * N + n] = acc[f];
    }
  }
  __syncthreads();
  // out = cb + the transposed derivative map of the second group: field f on wave f, mode on
  // lane; entry n needs 4 n times the stride-2 prefix sum of y (y_0 halved) up to n - 1
  if (tid < 3 * SPS_WAVE) {
    const int f = tid >> 6, p = tid & 63;
    const cplx* y = cb + (3 + f) * N;
    cplx w = (p < N) ? cscale(y[p], p == 0 ? 0.5 : 1.0) : czero();
    for (int o = 2; o < 64; o <<= 1) {
      const double tx = __shfl_up(w.x, o), ty = __shfl_up(w.y, o);
      if (p >= o) {
        w.x += tx;
        w.y += ty;
      }
    }
    if (p + 1 < N) out[f * N + p + 1] = cadd(cb[f * N + p + 1], cscale(w, 4.0 * (p + 1)));
    if (p == 0) out[f * N] = cb[f * N];
  }
  __syncthreads();
}

// cotangent G (equation slots) of F -> nlbar (S10^T, then the transposed Chebyshev forward
// transform).  nhb: 3*N scratch.  Block-wide.
__device__ void g_to_nlbar(const RbcDev& d, const KaArgs& a, int k, const double* ct, const cplx* G, cplx* nhb) {
  const int tid = threadIdx.x, N = d.N, Ngz = d.Ngz, K = d.K, Hc = half_nodes(Ngz);
  for (int e = tid; e < 3 * N; e += NTK) {
    const int f = e / N, m = e - f * N;
    nhb[e] = cscale(s10t_at(G + f * N, m, N), (m == 0 ? 1.0 : 2.0) / Ngz);
  }
  __syncthreads();
  for (int e = tid; e < 4 * Hc; e += NTK) {
    const int h = e & 3, j = e >> 2, jm = Ngz - 1 - j;
    cplx val[3];
    modes_to_pair<3>(ct, nhb, N, N, Ngz, j, h, val);
    if (h == 0 || (h == 1 && jm != j)) {
      const int jj = (h == 0) ? j : jm;
#pragma unroll
      for (int f = 0; f < 3; ++f) a.nlbar[((size_t)f * Ngz + jj) * K + k] = val[f];
    }
  }
}

// LDS: vA, vB (S complex each) persist; the rest is a union of phase buffers and the
// staged block operators.  One entry of every length-S vector per thread.  The streamed form
// (launches of thousands of systems) is held to six waves per SIMD, i.e. 80 registers and three
// blocks per CU: it spills 72 bytes per thread and is still 13 % faster than at two blocks.
template <bool STREAM>
__global__ void __launch_bounds__(NTK, STREAM ? 6 : 1) rbc_kadj(RbcDev d, KaArgs a) {
  if (blockIdx.y) {
    const int b = blockIdx.y;
    const size_t st = (size_t)d.K * d.S, zs = (size_t)d.Ngz * d.K;
    rbc_inst(d, b);
    a.zbar = inst_ptr(a.zbar, b, 6 * zs);
    a.nlbar = inst_ptr(a.nlbar, b, 3 * zs);
    a.Xb_in = inst_ptr(a.Xb_in, b, st);
    a.Xb_out = inst_ptr(a.Xb_out, b, st);
    a.acc = inst_ptr(a.acc, b, st);
    a.Ybuf = inst_ptr(a.Ybuf, b, st);
    a.Xm = inst_ptr(a.Xm, b, st);
  } else if (d.nub) {
    rbc_inst(d, 0);
  }
  extern __shared__ double smem_d[];
  cplx* sm = reinterpret_cast<cplx*>(smem_d);
  const int k = xcd_wavenumber(blockIdx.x, d.K), tid = threadIdx.x;
  const int N = d.N, S = d.S, Ngz = d.Ngz, Hc = half_nodes(Ngz);
  const int fl = a.flags;
  const double dt = a.dt;
  const int m = a.stage;
  const bool sl = tid < S;
  const size_t ks = (size_t)k * S + tid;
  cplx* vA = sm;                // S + SPS_PAD : solver-order vector
  cplx* vB = vA + S + SPS_PAD;  // S : solve result in equation slots (Y)
  cplx* un = vB + S;            // union
  double* ops = reinterpret_cast<double*>(un);
  // phase views (before the solve)
  double* ct = reinterpret_cast<double*>(un);           // 4*Ngz
  cplx* xbar = reinterpret_cast<cplx*>(ct + 4 * Ngz);   // S   cotangent of a state
  cplx* y2 = xbar + S;                                  // S
  cplx* pqz = y2 + S;                                   // 12*Hc
  cplx* cb = pqz + 12 * Hc;                             // 6*N
  cplx* vv = cb + 6 * N;                                // 3*N
  // views after the solve
  cplx* p_t = y2;                                       // S  (Y1 + Y2)
  cplx* p_g = pqz;                                      // S  cotangent of F
  cplx* p_nh = p_g + S;                                 // 3*N
  cplx* p_x = p_nh + 3 * N;                             // S  (parameter gradient: X_m)
  double* p_red = reinterpret_cast<double*>(p_x + S);   // 2 * NTK / 64

  // global reads in the order they are needed, the block operators last
  const double kxk = d.kx[k];
  const bool in_x = (fl & (KA_SOLVE_T | KA_G)) || ((fl & KA_A) && !(fl & KA_C));
  const cplx xin = (in_x && sl) ? a.Xb_in[ks] : czero();
  const cplx accv = ((fl & KA_C) && a.acc && sl) ? a.acc[ks] : czero();
  // the later stages' adjoints, loaded here and combined once every load is issued (a sum
  // taken as they arrive would wait for each before issuing the next): yc = sum_{j>m} H_jm Y_j
  // (implicit coupling), fs = sum_{j>m} A_{j,m-1} Y_j (F cotangent of stage m-1),
  // ys = sum_{j>m} Y_j (loops over the tableau's fixed size: coefficients at constant indices)
  cplx yv[RK_MAXS - 1];
#pragma unroll
  for (int j = 2; j <= RK_MAXS; ++j)
    yv[j - 2] = ((fl & KA_B) && sl && j > m && j <= a.nst) ? a.Ybuf[(size_t)(j - 2) * a.sstr + ks] : czero();
  const bool par = (fl & (KA_A | KA_B)) && a.pacc;
  const cplx xmv = (par && sl) ? a.Xm[ks] : czero();
  const ZbarPair zp = load_zbar_pair(d, a, k, (fl & (KA_C | KA_B)) != 0);
  const double cosr = (tid < 4 * Ngz) ? d.cosz[tid] : 0.0;
  OpsRegs opsr;
  MapRegs mr;
  // (issued for every flag set, so that no load is under a branch; the transposed solve's first
  // sweep reads the G blocks: those first)
  load_maps(d, mr);
  if (!STREAM) ops_issue_gt(d.ops + (size_t)k * d.opsize, d.tsz, d.blksz - d.tsz, opsr);
  cplx yc = czero(), fs = czero(), ys = czero();
  if ((fl & KA_B) && sl) {
#pragma unroll
    for (int j = 2; j <= RK_MAXS; ++j) {
      if (j > m && j <= a.nst) {
        const cplx y = yv[j - 2];
        yc = cadd(yc, cscale(y, a.hc[j]));
        fs = cadd(fs, cscale(y, a.fc[j]));
        ys = cadd(ys, y);
      }
    }
  }
  if (tid < 4 * Ngz) ct[tid] = cosr;
  if (fl & KA_SOLVE_T) {
    if (sl) xbar[tid] = xin;
    __syncthreads();
  }
  if (fl & KA_G) {
    if (sl) p_g[tid] = xin;
    __syncthreads();
    g_to_nlbar(d, a, k, ct, p_g, p_nh);
    return;
  }
  if (fl & KA_C) {
    zbar_to_coeffs(d, zp, ct, pqz, cb, vv);
    if (sl) xbar[tid] = (tid < 3 * N) ? cadd(accv, vv[tid]) : accv;
    __syncthreads();
    if (!(fl & KA_A)) {
      if (sl) a.Xb_out[ks] = xbar[tid];
      return;
    }
  } else if (fl & KA_A) {
    if (sl) xbar[tid] = xin;
    __syncthreads();
  }
  if (fl & KA_B) {
    // xbar_m = F-VJP part - dt L^H sum_{j>m} H_jm Y_j
    zbar_to_coeffs(d, zp, ct, pqz, cb, vv);
    if (sl) y2[tid] = yc;
    __syncthreads();
    if (sl) {
      const MLRow t = mlt_col(d, k, kxk, y2, tid);
      cplx v = cscale(t.l, -dt);
      if (tid < 3 * N) v = cadd(v, vv[tid]);
      xbar[tid] = v;
    }
    __syncthreads();
  }
  // Y_m = (M + dt H_mm L)^{-H} xbar
  if (!STREAM) stage_early(d, opsr, ops, true);
  rbc_gather_h(d, mr, xbar, vA);
  rbc_solve<STREAM>(d, k, opsr, ops, vA, vB, true);
  rbc_scatter_h(d, mr, vA, vB);       // vB = Y_m
  if (fl & KA_SOLVE_T) {
    if (sl) a.Xb_out[ks] = vB[tid];
    return;
  }
  if (tid < 4 * Ngz) ct[tid] = cosr;
  const cplx ym = sl ? vB[tid] : czero();
  if (sl) {
    if (m >= 2) a.Ybuf[(size_t)(m - 2) * a.sstr + ks] = ym;
    if (m == 1) p_t[tid] = cadd(ys, ym);
    if (par) p_x[tid] = xmv;
    // F cotangent of stage m-1: dt sum_{j>=m} A_{j,m-1} Y_j
    p_g[tid] = cscale(cadd(fs, cscale(ym, a.fself)), dt);
  }
  __syncthreads();
  if (par) param_accumulate(d, a, k, cadd(yc, cscale(ym, a.hself)), p_x, p_red);
  if (m == 1 && sl) a.acc[ks] = mlt_col(d, k, kxk, p_t, tid).m;
  g_to_nlbar(d, a, k, ct, p_g, p_nh);
}

// ---------------------------------------------------------------------------- factor
// A batch (BLnu != null): instance blockIdx.y factors a M + b (BL + nu BLnu + kappa BLka) with
// its own nu and kappa (L is affine in them) into its own operators.
__global__ void __launch_bounds__(NT) rbc_factor(RbcDev d, const double* BM, const double* BL, double am,
                                                 double bl, double* ops, const double* BLnu = nullptr,
                                                 const double* BLka = nullptr) {
  extern __shared__ double smem_d[];
  __shared__ int sh[4];
  const int k = blockIdx.x, b = blockIdx.y, tid = threadIdx.x;
  const int bw = d.kl + d.ku + 1, ldab = 2 * d.kl + d.ku + 1;
  const size_t ko = (size_t)k * d.n * bw;
  const double nu = d.nub ? d.nub[b] : 0.0, ka = d.kab ? d.kab[b] : 0.0;
  double* O = ops + ((size_t)b * d.K + k) * d.opsize;
  const double* bnu = BLnu ? BLnu + ko : nullptr;
  const double* bka = BLka ? BLka + ko : nullptr;
  if (!d.part) {
    int* spiv = reinterpret_cast<int*>(smem_d + (size_t)d.n * ldab);
    band_factor_block(BM + ko, BL + ko, am, bl, d.n, d.kl, d.ku, smem_d, sh, spiv, O, d.err, bnu, bka, nu, ka);
    return;
  }
  // P partitions: each partition's factors and block operators, its spikes (its factors solved
  // with the columns that couple it to the next and to the previous partition, for A and for
  // A^T), then the inverses of the coupled entries' systems.  Layout from pmeta: per partition
  // p (8 ints): start, rows, then per direction the widths of V_p and W_p and the offset of its
  // spike rows (entry c of its row t at c n_p + t); per interface q (6 ints at 8 SPS_MAXPART):
  // per direction the widths of a_q (last entries of partition q) and c_q (first entries of
  // partition q + 1) and their offset in the coupled system.  Inverses column-major.
  const int P = d.part;
  const int* pm = d.pmeta;
  int mx = 0;
  for (int p = 0; p < P; ++p) mx = max(mx, pm[8 * p + 1]);
  double* ab = smem_d;                                                   // mx * ldab
  int* spiv = reinterpret_cast<int*>(ab + (size_t)mx * ldab);            // mx
  double* R = ab + (size_t)mx * ldab + ((mx + 1) & ~1) / 2 + 1;          // mx * SPS_SPIKE_W
  double* Rm = R + (size_t)mx * SPS_SPIKE_W;                             // nr * nr
  const int nrm = max(d.nrr[0], d.nrr[1]);
  double* aug = Rm + (size_t)nrm * nrm;                                  // nr * (2 nr + 1)
  auto Aat = [&](int i, int c) -> double {   // entry (i, c) of a M + b L of the whole system
    const int q = c - i + d.kl;
    if (q < 0 || q >= bw) return 0.0;
    const size_t e = ko + (size_t)i * bw + q;
    const double l = BLnu ? BL[e] + nu * BLnu[e] + ka * BLka[e] : BL[e];
    return am * BM[e] + bl * l;
  };
  for (int p = 0; p < P; ++p) {
    const int s0 = pm[8 * p], np = pm[8 * p + 1], s1 = s0 + np;
    band_lu_factor(BM + ko + (size_t)s0 * bw, BL + ko + (size_t)s0 * bw, am, bl, np, d.kl, d.ku, ab, sh, spiv, d.err,
                   bnu ? bnu + (size_t)s0 * bw : nullptr, bka ? bka + (size_t)s0 * bw : nullptr, nu, ka);
    band_condense(ab, spiv, np, d.kl, d.ku, O + (s0 / SPS_BLK) * (SPS_TW * SPS_TS),
                  O + d.tsz + (s0 / SPS_BLK) * (SPS_BLK * SPS_GS));
    for (int dir = 0; dir < 2; ++dir) {
      const int wV = pm[8 * p + 2 + 3 * dir], wW = pm[8 * p + 3 + 3 * dir], w = wV + wW;
      // columns c < wV: the first wV columns of partition p + 1; then the last wW of p - 1
      // (of A, or of A^T for the transposed direction)
      for (int e = threadIdx.x; e < np * w; e += blockDim.x) {
        const int i = e / w, c = e - i * w;
        const int col = (c < wV) ? s1 + c : s0 - wW + (c - wV);
        R[e] = dir ? Aat(col, s0 + i) : Aat(s0 + i, col);
      }
      band_lu_solve_cols(ab, spiv, np, d.kl, d.ku, R, w, dir == 1);
      double* out = O + (dir ? d.spk[1] : d.spk[0]) + pm[8 * p + 4 + 3 * dir];
      for (int e = threadIdx.x; e < np * w; e += blockDim.x) {
        const int i = e / w, c = e - i * w;
        out[(size_t)c * np + i] = R[e];
      }
      __syncthreads();   // R is refilled next
    }
  }
  for (int dir = 0; dir < 2; ++dir) {
    const int nr = dir ? d.nrr[1] : d.nrr[0];
    const double* spd = O + (dir ? d.spk[1] : d.spk[0]);
    for (int e = threadIdx.x; e < nr * nr; e += blockDim.x) Rm[e] = (e / nr == e % nr) ? 1.0 : 0.0;
    __syncthreads();
    // R z = g: a_q + V_q c_q + W_q a_{q-1} (rows of a_q, the last entries of partition q) and
    // c_q + V_{q+1} c_{q+1} + W_{q+1} a_q (rows of c_q, the first entries of partition q + 1)
    for (int q = 0; q + 1 < P; ++q) {
      const int* im = pm + 8 * SPS_MAXPART + 6 * q + 3 * dir;
      const int la = im[0], lc = im[1], zo = im[2];
      for (int side = 0; side < 2; ++side) {
        const int p = q + side;   // the partition whose rows these are
        const int* ppm = pm + 8 * p;
        const int np = ppm[1], wV = ppm[2 + 3 * dir], wW = ppm[3 + 3 * dir], w = wV + wW;
        const int nrow = side ? lc : la, row0 = side ? 0 : np - la, zrow = side ? zo + la : zo;
        // coupled-system columns of the spike columns: V_p -> c_p, W_p -> a_{p-1}
        const int zc = (p + 1 < P) ? pm[8 * SPS_MAXPART + 6 * p + 3 * dir + 2] + pm[8 * SPS_MAXPART + 6 * p + 3 * dir] : 0;
        const int za = (p > 0) ? pm[8 * SPS_MAXPART + 6 * (p - 1) + 3 * dir + 2] : 0;
        const double* rows = spd + ppm[4 + 3 * dir] + row0;   // entry c of the partition's row row0 + t
        for (int e = threadIdx.x; e < nrow * w; e += blockDim.x) {
          const int t = e / w, c = e - t * w;
          const int col = (c < wV) ? zc + c : za + (c - wV);
          Rm[(size_t)(zrow + t) * nr + col] = rows[(size_t)c * np + t];
        }
      }
    }
    block_inverse(Rm, nr, aug, O + (dir ? d.spk[1] + d.rof[1] : d.spk[0] + d.rof[0]), d.err, sh, true);
  }
}

// ---------------------------------------------------------------------------- linear boundary value problem
// L X = M f + c (Supplementary, "Linear boundary value problems"): the steady state of the IVP
// without its explicit term, driven by the forcing f (u, w, b blocks of a state-shaped array)
// with the IVP's boundary data c.  Right-hand side in equation-row slots: S10 f in the C2 rows
// of u, w, b, zero continuity and gauge rows, b(0) = bc0 at k = 0.  One block per wavenumber.
__global__ void __launch_bounds__(NT) rbc_lbvp_rhs(RbcDev d, const cplx* f, cplx* R) {
  const int k = blockIdx.x, N = d.N, S = d.S;
  const cplx* fk = f + (size_t)k * S;
  for (int s = threadIdx.x; s < S; s += NT) {
    cplx v = czero();
    if (s < 3 * N) {
      const int q = s / N, n = s - q * N;
      v = s10_at(fk + q * N, n, N);
    } else if (k == 0 && s == 4 * N + 4) {
      v = cmk(d.bc0, 0.0);
    }
    R[(size_t)k * S + s] = v;
  }
}
// The VJP of the right-hand side: fbar = M^H Y on the u, w, b blocks, zero in the other slots.
__global__ void __launch_bounds__(NT) rbc_lbvp_rhs_adj(RbcDev d, const cplx* Y, cplx* fbar) {
  const int k = blockIdx.x, N = d.N, S = d.S;
  const cplx* yk = Y + (size_t)k * S;
  for (int s = threadIdx.x; s < S; s += NT) {
    cplx v = czero();
    if (s < 3 * N) {
      const int q = s / N, m = s - q * N;
      v = s10t_at(yk + q * N, m, N);
    }
    fbar[(size_t)k * S + s] = v;
  }
}

// ---------------------------------------------------------------------------- eigenvalue problem
// Linear stability of the conduction state (Supplementary, "Eigenvalue problems"):
// (lambda M + L_s) X = 0 per wavenumber, L_s the IVP's L with -S10 w in the b rows.  The
// eigenvalue nearest a shift sigma comes from inverse iteration with A = sigma M + L_s:
// y = A^-1 M x, mu = <x, y> for |x| = 1, lambda = sigma - 1/mu; the adjoint eigenvector
// ((conj(lambda) M^H + L_s^H) Y = 0) from y = A^-H M^H x through the same factors.

// R = M X: S10 on the u, w, b blocks, zero in the other slots.  One block per wavenumber.
__global__ void __launch_bounds__(NT) rbc_apply_m(RbcDev d, const cplx* X, cplx* R) {
  const int k = blockIdx.x, N = d.N, S = d.S;
  const cplx* xk = X + (size_t)k * S;
  for (int s = threadIdx.x; s < S; s += NT) {
    cplx v = czero();
    if (s < 3 * N) {
      const int q = s / N, n = s - q * N;
      v = s10_at(xk + q * N, n, N);
    }
    R[(size_t)k * S + s] = v;
  }
}

// sum over the block of NT values per component (LDS tree); every thread gets the sums
template <int C>
__device__ __forceinline__ void block_sums(double (&v)[C], double (*red)[NT]) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int c = 0; c < C; ++c) red[c][tid] = v[c];
  __syncthreads();
  for (int h = NT / 2; h > 0; h >>= 1) {
    if (tid < h)
#pragma unroll
      for (int c = 0; c < C; ++c) red[c][tid] += red[c][tid + h];
    __syncthreads();
  }
#pragma unroll
  for (int c = 0; c < C; ++c) v[c] = red[c][0];
}

// One inverse-iteration update per wavenumber: mu = <x, y> (x has unit norm), x <- y / |y|,
// lam = sigma - 1/mu (lam may be null).
__global__ void __launch_bounds__(NT) rbc_evp_update(RbcDev d, cplx* x, const cplx* y, double sigma, cplx* lam) {
  __shared__ double red[3][NT];
  const int k = blockIdx.x, S = d.S;
  cplx* xk = x + (size_t)k * S;
  const cplx* yk = y + (size_t)k * S;
  double v[3] = {0.0, 0.0, 0.0};
  for (int s = threadIdx.x; s < S; s += NT) {
    const cplx a = xk[s], b = yk[s];
    v[0] += a.x * b.x + a.y * b.y;   // Re conj(a) b
    v[1] += a.x * b.y - a.y * b.x;   // Im conj(a) b
    v[2] += b.x * b.x + b.y * b.y;
  }
  block_sums<3>(v, red);
  const double inv = v[2] > 0.0 ? 1.0 / sqrt(v[2]) : 0.0;
  for (int s = threadIdx.x; s < S; s += NT) xk[s] = cscale(yk[s], inv);
  if (lam && threadIdx.x == 0) {
    const double m2 = v[0] * v[0] + v[1] * v[1];
    lam[k] = cmk(sigma - v[0] / m2, v[1] / m2);   // sigma - 1/mu
  }
}

// Eigenvalue sensitivities (equ:eigenvalue_sens, dM/dp = 0): out[k] = (d lambda/dRa,
// d lambda/dk) = -<Y, dL/dp X> / <Y, M X>, with dL/dRa = dnu dL/dnu + dka dL/dkappa (the
// viscous and diffusive blocks and their lifted taus) and dL/dk (the k^2 terms, i k p in the
// x-momentum rows, i k u in continuity).
__global__ void __launch_bounds__(NT) rbc_evp_sens(RbcDev d, const cplx* X, const cplx* Y, double dnu, double dka,
                                                   cplx* out) {
  __shared__ double red[6][NT];
  const int k = blockIdx.x, N = d.N, S = d.S;
  const cplx* xk = X + (size_t)k * S;
  const cplx* yk = Y + (size_t)k * S;
  const double kx = d.kx[k], k2 = kx * kx;
  double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};   // <Y,MX>, <Y,dL/dRa X>, <Y,dL/dk X> (re, im)
  auto acc = [&](int c, cplx yv, cplx w) {
    v[2 * c] += yv.x * w.x + yv.y * w.y;
    v[2 * c + 1] += yv.x * w.y - yv.y * w.x;
  };
  for (int s = threadIdx.x; s < 4 * N; s += NT) {
    const cplx yv = yk[s];
    if (s < 3 * N) {
      const int f = s / N, n = s - f * N;
      const cplx* c = xk + f * N;
      const double dif = (f == 2) ? d.ka : d.nu, ddif = (f == 2) ? dka : dnu;
      const cplx sc = s10_at(c, n, N);
      cplx dra = cscale(cadd(cscale(dzz_at(c, n, N), -1.0), cscale(sc, k2)), ddif);
      if (n == N - 2) dra = csub(dra, cscale(xk[4 * N + f], 4.0 * ddif));
      cplx dk = cscale(sc, 2.0 * kx * dif);
      if (f == 0) dk = cadd(dk, cmul_i(s10_at(xk + 3 * N, n, N)));
      acc(0, yv, sc);
      acc(1, yv, dra);
      acc(2, yv, dk);
    } else {
      const int n = s - 3 * N;
      acc(2, yv, cmul_i(s0_at(xk, n, N)));
    }
  }
  block_sums<6>(v, red);
  if (threadIdx.x == 0) {
    const double dr = v[0], di = v[1], m2 = dr * dr + di * di;
    // -num / den
    out[2 * k] = cmk(-(v[2] * dr + v[3] * di) / m2, -(v[3] * dr - v[2] * di) / m2);
    out[2 * k + 1] = cmk(-(v[4] * dr + v[5] * di) / m2, -(v[5] * dr - v[4] * di) / m2);
  }
}

// Eigenvector sensitivities (equ:eigenvector_sens, dM/dp = 0): z with (lambda M + L_s) z = r,
// r = -(dlambda/dp M + dL/dp) X, and <X, z> = 0, through the factors of A = sigma M + L_s:
// z <- P A^-1 (r - (lambda - sigma) M z), P = I - X (Y^H M .) / (Y^H M X) the spectral projector
// that removes the eigenvector (M^H Y is proportional to the left eigenvector of A^-1 M, and
// Y^H r = 0 makes the fixed point a solution); the iteration contracts by
// |lambda - sigma| / min_j |lambda_j - sigma| over the other eigenvalues.  Finally z loses its
// component along X.

// R = -(dlam[k][p] M X + dL/dp X) per wavenumber, p = 0 (Ra, via dnu and dka) or 1 (k); the
// rows as in rbc_evp_sens.
__global__ void __launch_bounds__(NT) rbc_evp_dlx(RbcDev d, const cplx* X, const cplx* dlam, int p, double dnu,
                                                  double dka, cplx* R) {
  const int k = blockIdx.x, N = d.N, S = d.S;
  const cplx* xk = X + (size_t)k * S;
  const double kx = d.kx[k], k2 = kx * kx;
  const cplx dl = dlam[2 * k + p];
  for (int s = threadIdx.x; s < S; s += NT) {
    cplx v = czero();
    if (s < 3 * N) {
      const int f = s / N, n = s - f * N;
      const cplx* c = xk + f * N;
      const double dif = (f == 2) ? d.ka : d.nu, ddif = (f == 2) ? dka : dnu;
      const cplx sc = s10_at(c, n, N);
      if (p == 0) {
        v = cscale(cadd(cscale(dzz_at(c, n, N), -1.0), cscale(sc, k2)), ddif);
        if (n == N - 2) v = csub(v, cscale(xk[4 * N + f], 4.0 * ddif));
      } else {
        v = cscale(sc, 2.0 * kx * dif);
        if (f == 0) v = cadd(v, cmul_i(s10_at(xk + 3 * N, n, N)));
      }
      v = cadd(v, cmul(dl, sc));
    } else if (s < 4 * N && p == 1) {
      v = cmul_i(s0_at(xk, s - 3 * N, N));
    }
    R[(size_t)k * S + s] = cscale(v, -1.0);
  }
}

// W = R - (lam[k] - sigma) MZ per wavenumber.
__global__ void __launch_bounds__(NT) rbc_vs_combine(RbcDev d, const cplx* R, const cplx* MZ, const cplx* lam,
                                                     double sigma, cplx* W) {
  const int k = blockIdx.x, S = d.S;
  const cplx c = cmk(lam[k].x - sigma, lam[k].y);
  for (int s = threadIdx.x; s < S; s += NT) {
    const size_t e = (size_t)k * S + s;
    W[e] = csub(R[e], cmul(c, MZ[e]));
  }
}

// Z -= X <Q, Z> / <Q, X> per wavenumber (complex inner products <a, b> = sum conj(a) b): the
// spectral projection with Q = M^H Y, or the orthogonal one with Q = X.
__global__ void __launch_bounds__(NT) rbc_vs_project(RbcDev d, cplx* Z, const cplx* X, const cplx* Q) {
  __shared__ double red[4][NT];
  const int k = blockIdx.x, S = d.S;
  cplx* zk = Z + (size_t)k * S;
  const cplx* xk = X + (size_t)k * S;
  const cplx* qk = Q + (size_t)k * S;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int s = threadIdx.x; s < S; s += NT) {
    const cplx q = qk[s], z = zk[s], x = xk[s];
    v[0] += q.x * z.x + q.y * z.y;
    v[1] += q.x * z.y - q.y * z.x;
    v[2] += q.x * x.x + q.y * x.y;
    v[3] += q.x * x.y - q.y * x.x;
  }
  block_sums<4>(v, red);
  const double m2 = v[2] * v[2] + v[3] * v[3];
  const cplx a = m2 > 0.0 ? cmk((v[0] * v[2] + v[1] * v[3]) / m2, (v[1] * v[2] - v[0] * v[3]) / m2) : czero();
  for (int s = threadIdx.x; s < S; s += NT) zk[s] = csub(zk[s], cmul(a, xk[s]));
}

// ---------------------------------------------------------------------------- shift-invert Arnoldi
// Several eigenvalues nearest a real shift per wavenumber (Supplementary, "Eigenvalue
// problems": a Krylov eigensolver on the shift-inverted pencil).  m Arnoldi steps on
// B = (sigma M + L_s)^-1 M through the factors of the inverse iteration: v_{j+1} h_{j+1,j} =
// B v_j - sum_{i<=j} h_ij v_i, the h_ij by classical Gram-Schmidt applied twice.  Basis V laid
// out vector-major, [m+1][K][S] (vector j of every wavenumber is a state); Hessenberg matrices
// Hb [K][(m+1) m], row-major.
constexpr int ARN_MAX_M = 64;
constexpr int ARN_CH = 8;   // inner products reduced together

// Sums of C values over the block (NT / 64 waves): each wave sums by xor shuffles, then the
// waves' partial sums meet in LDS (red: [C][NT / 64]); every thread gets the sums.  A barrier
// must separate two uses of red.
template <int C>
__device__ __forceinline__ void block_sums_w(double (&v)[C], double (*red)[NT / 64]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    double x = v[c];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    v[c] = x;
  }
  if (lane == 0)
#pragma unroll
    for (int c = 0; c < C; ++c) red[c][w] = v[c];
  __syncthreads();
#pragma unroll
  for (int c = 0; c < C; ++c) {
    double x = 0.0;
#pragma unroll
    for (int q = 0; q < NT / 64; ++q) x += red[c][q];
    v[c] = x;
  }
}

// Orthogonalizes w = V_{j+1} (in place, one block per wavenumber) against V_0..V_j and
// normalizes it, filling column j of Hb; j = -1 normalizes the start vector V_0.
__global__ void __launch_bounds__(NT) rbc_arnoldi_orth(RbcDev d, cplx* V, cplx* Hb, int j, int m) {
  extern __shared__ double smem_d[];
  __shared__ double red[2 * ARN_CH][NT / 64];
  __shared__ cplx hs[ARN_MAX_M];
  cplx* w = reinterpret_cast<cplx*>(smem_d);
  const int k = blockIdx.x, K = d.K, S = d.S, tid = threadIdx.x;
  auto vec = [&](int i) { return V + ((size_t)i * K + k) * S; };
  cplx* Hk = Hb + (size_t)k * (m + 1) * m;
  cplx* wg = vec(j + 1);
  for (int s = tid; s < S; s += NT) w[s] = wg[s];
  __syncthreads();
  for (int pass = 0; pass < 2 && j >= 0; ++pass) {
    for (int i0 = 0; i0 <= j; i0 += ARN_CH) {
      double v[2 * ARN_CH];
#pragma unroll
      for (int c = 0; c < 2 * ARN_CH; ++c) v[c] = 0.0;
      for (int s = tid; s < S; s += NT) {
        const cplx b = w[s];
#pragma unroll
        for (int c = 0; c < ARN_CH; ++c)
          if (i0 + c <= j) {
            const cplx a = vec(i0 + c)[s];
            v[2 * c] += a.x * b.x + a.y * b.y;       // Re conj(a) b
            v[2 * c + 1] += a.x * b.y - a.y * b.x;   // Im conj(a) b
          }
      }
      block_sums_w<2 * ARN_CH>(v, red);
      if (tid == 0)
#pragma unroll
        for (int c = 0; c < ARN_CH; ++c)
          if (i0 + c <= j) hs[i0 + c] = cmk(v[2 * c], v[2 * c + 1]);
      __syncthreads();   // red is reused by the next reduction; hs complete
    }
    for (int s = tid; s < S; s += NT) {
      cplx r = w[s];
      for (int i = 0; i <= j; ++i) r = csub(r, cmul(hs[i], vec(i)[s]));
      w[s] = r;
    }
    if (tid <= j) Hk[(size_t)tid * m + j] = pass == 0 ? hs[tid] : cadd(Hk[(size_t)tid * m + j], hs[tid]);
    __syncthreads();
  }
  double v[1] = {0.0};
  for (int s = tid; s < S; s += NT) v[0] += w[s].x * w[s].x + w[s].y * w[s].y;
  block_sums_w<1>(v, red);
  const double h = sqrt(v[0]);
  const double inv = h > 0.0 ? 1.0 / h : 0.0;
  for (int s = tid; s < S; s += NT) wg[s] = cscale(w[s], inv);
  if (j >= 0 && tid == 0) Hk[(size_t)(j + 1) * m + j] = cmk(h, 0.0);
  for (int i = j + 2 + tid; j >= 0 && i <= m; i += NT) Hk[(size_t)i * m + j] = czero();   // below the subdiagonal
}

__device__ __forceinline__ double cabs_d(cplx a) { return hypot(a.x, a.y); }
__device__ __forceinline__ double cabs1(cplx a) { return fabs(a.x) + fabs(a.y); }   // |re| + |im|
__device__ __forceinline__ cplx cdiv(cplx a, cplx b) {
  const double q = 1.0 / (b.x * b.x + b.y * b.y);
  return cmk((a.x * b.x + a.y * b.y) * q, (a.y * b.x - a.x * b.y) * q);
}
__device__ __forceinline__ cplx csqrt_d(cplx z) {
  const double r = hypot(z.x, z.y);
  if (r == 0.0) return czero();
  const double t = sqrt(0.5 * (r + fabs(z.x)));
  return z.x >= 0.0 ? cmk(t, z.y / (2.0 * t)) : cmk(fabs(z.y) / (2.0 * t), copysign(t, z.y));
}

// Eigenpairs of the m x m Hessenberg matrix of every wavenumber (one wave per wavenumber):
// complex Schur form H = Z T Z^H by shifted QR steps (Givens rotations, Wilkinson shift from
// the trailing 2 x 2 of the active block, an exceptional shift every 10 steps without
// deflation, deflation where |h_{l,l-1}| <= ulp (|h_ll| + |h_{l-1,l-1}|) with |z| measured as
// |re z| + |im z|), eigenvectors of T
// by back substitution, y = Z z normalized.  Out, per wavenumber, the nev pairs of largest
// |nu| (nearest the shift) in that order: lam = sigma - 1/nu, the residual |h_{m+1,m}| |y_m|
// (res, nullable) and y (Ysel [K][nev][m]).  Zw: [K][2][m][m] work in global memory, or, with
// zlds, the same 2 m^2 entries after sel in LDS.  No convergence within 30 m steps sets bit 4
// of d.err.
constexpr int ARN_NT = 64;
// offset (in complex entries) of the eigenvector work arrays in rbc_hess_eig's LDS: after H, Z,
// rotations and nu (2 n^2 + 3 n entries), residuals (n doubles) and selection (n ints), rounded
// up to a whole entry
__host__ __device__ inline int hess_zoff(int n) { return 2 * n * n + 3 * n + (8 * n + 4 * n + 15) / 16; }
__global__ void __launch_bounds__(ARN_NT) rbc_hess_eig(RbcDev d, const cplx* Hb, int m, int nev, double sigma,
                                                        cplx* lam, double* res, cplx* Ysel, cplx* Zw, int zlds) {
  extern __shared__ double smem_d[];
  const int k = blockIdx.x, t = threadIdx.x, n = m;
  cplx* H = reinterpret_cast<cplx*>(smem_d);
  cplx* Z = H + n * n;
  cplx* cs = Z + n * n;        // [2n] rotations of one QR step
  cplx* nu = cs + 2 * n;       // [n]
  double* rs = reinterpret_cast<double*>(nu + n);   // [n]
  int* sel = reinterpret_cast<int*>(rs + n);        // [n]
  const cplx* Hk = Hb + (size_t)k * (m + 1) * m;
  for (int e = t; e < n * n; e += ARN_NT) {
    const int i = e / n, j = e - i * n;
    H[e] = (i <= j + 1) ? Hk[(size_t)i * m + j] : czero();
    Z[e] = cmk(i == j ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  double anorm = 0.0;
  for (int e = 0; e < n * n; ++e) anorm = fmax(anorm, cabs1(H[e]));
  const double ulp = 2.220446049250313e-16;
  const double smlnum = fmax(anorm * ulp, 1e-300);
  int hi = n - 1, its = 0, total = 0;
  bool fail = false;
  while (hi > 0) {
    int l = hi;
    for (; l > 0; --l) {
      const double sub = cabs1(H[l * n + l - 1]);
      double tst = cabs1(H[(l - 1) * n + l - 1]) + cabs1(H[l * n + l]);
      if (tst == 0.0) tst = anorm;
      if (sub <= ulp * tst || sub <= smlnum) break;
    }
    __syncthreads();
    if (l > 0 && t == 0) H[l * n + l - 1] = czero();
    __syncthreads();
    if (l == hi) {
      --hi;
      its = 0;
      continue;
    }
    if (++total > 30 * n) {
      fail = true;
      break;
    }
    ++its;
    cplx mu;
    const cplx dd = H[hi * n + hi];
    if (its % 10 == 0) {
      mu = cmk(dd.x + 0.75 * cabs_d(H[hi * n + hi - 1]), dd.y);
    } else {
      const cplx a = H[(hi - 1) * n + hi - 1], b = H[(hi - 1) * n + hi], c = H[hi * n + hi - 1];
      const cplx half = cscale(csub(a, dd), 0.5), mid = cscale(cadd(a, dd), 0.5);
      const cplx disc = csqrt_d(cadd(cmul(half, half), cmul(b, c)));
      const cplx m1 = cadd(mid, disc), m2 = csub(mid, disc);
      mu = cabs_d(csub(m1, dd)) <= cabs_d(csub(m2, dd)) ? m1 : m2;
    }
    __syncthreads();
    for (int i = l + t; i <= hi; i += ARN_NT) H[i * n + i] = csub(H[i * n + i], mu);
    __syncthreads();
    // H - mu I = Q R: G_kk zeroes h_{kk+1,kk}, G = [[conj c, conj s], [-s, c]]
    for (int kk = l; kk < hi; ++kk) {
      const cplx x = H[kk * n + kk], y = H[(kk + 1) * n + kk];
      const double r2 = x.x * x.x + x.y * x.y + y.x * y.x + y.y * y.y;
      const double ir = r2 > 0.0 ? 1.0 / sqrt(r2) : 0.0;
      const cplx c = r2 > 0.0 ? cscale(x, ir) : cmk(1.0, 0.0);
      const cplx sg = cscale(y, ir);
      __syncthreads();
      for (int j = kk + t; j < n; j += ARN_NT) {
        const cplx a = H[kk * n + j], b = H[(kk + 1) * n + j];
        H[kk * n + j] = cadd(cmul(cconj(c), a), cmul(cconj(sg), b));
        H[(kk + 1) * n + j] = csub(cmul(c, b), cmul(sg, a));
      }
      if (t == 0) {
        cs[2 * (kk - l)] = c;
        cs[2 * (kk - l) + 1] = sg;
      }
      __syncthreads();
    }
    // R Q + mu I, Z Q: columns kk, kk+1 times G^H = [[c, -conj s], [s, conj c]]
    for (int kk = l; kk < hi; ++kk) {
      const cplx c = cs[2 * (kk - l)], sg = cs[2 * (kk - l) + 1];
      for (int i = t; i <= kk + 1; i += ARN_NT) {
        const cplx a = H[i * n + kk], b = H[i * n + kk + 1];
        H[i * n + kk] = cadd(cmul(a, c), cmul(b, sg));
        H[i * n + kk + 1] = csub(cmul(b, cconj(c)), cmul(a, cconj(sg)));
      }
      for (int i = t; i < n; i += ARN_NT) {
        const cplx a = Z[i * n + kk], b = Z[i * n + kk + 1];
        Z[i * n + kk] = cadd(cmul(a, c), cmul(b, sg));
        Z[i * n + kk + 1] = csub(cmul(b, cconj(c)), cmul(a, cconj(sg)));
      }
      __syncthreads();
    }
    for (int i = l + t; i <= hi; i += ARN_NT) H[i * n + i] = cadd(H[i * n + i], mu);
    __syncthreads();
  }
  if (fail && t == 0) atomicOr(d.err, 4);
  // eigenvector i of T (lane i), then y = Z z; entry j of vector i at [j n + i] (z) and
  // [(n + j) n + i] (y), so the lanes of a wave touch neighbouring entries
  cplx* zk = zlds ? reinterpret_cast<cplx*>(smem_d) + hess_zoff(n) : Zw + (size_t)k * 2 * n * n;
  const double hsub = cabs_d(Hk[(size_t)m * m + m - 1]);
  for (int i = t; i < n; i += ARN_NT) {
    cplx* z = zk + i;
    cplx* y = zk + (size_t)n * n + i;
    const cplx ti = H[i * n + i];
    for (int j = 0; j < n; ++j) z[(size_t)j * n] = cmk(j == i ? 1.0 : 0.0, 0.0);
    for (int j = i - 1; j >= 0; --j) {
      cplx acc = czero();
      for (int q = j + 1; q <= i; ++q) acc = cadd(acc, cmul(H[j * n + q], z[(size_t)q * n]));
      cplx den = csub(H[j * n + j], ti);
      if (cabs_d(den) < smlnum) den = cmk(smlnum, 0.0);
      z[(size_t)j * n] = cscale(cdiv(acc, den), -1.0);
    }
    double nrm = 0.0;
    for (int r = 0; r < n; ++r) {
      cplx acc = czero();
      for (int q = 0; q <= i; ++q) acc = cadd(acc, cmul(Z[r * n + q], z[(size_t)q * n]));
      y[(size_t)r * n] = acc;
      nrm += acc.x * acc.x + acc.y * acc.y;
    }
    const double inv = 1.0 / sqrt(nrm);
    for (int r = 0; r < n; ++r) y[(size_t)r * n] = cscale(y[(size_t)r * n], inv);
    nu[i] = ti;
    rs[i] = hsub * cabs_d(y[(size_t)(n - 1) * n]);
  }
  __syncthreads();
  if (t == 0) {
    for (int r = 0; r < nev; ++r) {
      int best = -1;
      double bv = -1.0;
      for (int i = 0; i < n; ++i) {
        bool used = false;
        for (int q = 0; q < r; ++q) used = used || sel[q] == i;
        const double a = cabs_d(nu[i]);
        if (!used && a > bv) {
          bv = a;
          best = i;
        }
      }
      sel[r] = best;
    }
  }
  __syncthreads();
  for (int r = t; r < nev; r += ARN_NT) {
    const int i = sel[r];
    const cplx inv_nu = cdiv(cmk(1.0, 0.0), nu[i]);
    lam[(size_t)k * nev + r] = cmk(sigma - inv_nu.x, -inv_nu.y);
    if (res) res[(size_t)k * nev + r] = rs[i];
    const cplx* y = zk + (size_t)n * n + i;
    for (int q = 0; q < n; ++q) Ysel[((size_t)k * nev + r) * m + q] = y[(size_t)q * n];
  }
}

// Ritz vectors X[k][r] = V_m y_r (unit norm), one block per (wavenumber, pair).
__global__ void __launch_bounds__(NT) rbc_ritz(RbcDev d, const cplx* V, const cplx* Ysel, int m, int nev, cplx* X) {
  __shared__ double red[1][NT];
  const int k = blockIdx.x, r = blockIdx.y, K = d.K, S = d.S, tid = threadIdx.x;
  const cplx* y = Ysel + ((size_t)k * nev + r) * m;
  cplx* xo = X + ((size_t)k * nev + r) * S;
  double v[1] = {0.0};
  for (int s = tid; s < S; s += NT) {
    cplx acc = czero();
    for (int i = 0; i < m; ++i) acc = cadd(acc, cmul(V[((size_t)i * K + k) * S + s], y[i]));
    xo[s] = acc;
    v[0] += acc.x * acc.x + acc.y * acc.y;
  }
  block_sums<1>(v, red);
  const double inv = v[0] > 0.0 ? 1.0 / sqrt(v[0]) : 0.0;
  for (int s = tid; s < S; s += NT) xo[s] = cscale(xo[s], inv);
}

// ---------------------------------------------------------------------------- initial state and its adjoint
// x pass: one block per scale-1 z node; b0 laid out [x][z].
__global__ void __launch_bounds__(NT) rbc_init_x(RbcDev d, const double* grid, cplx* tmp) {
  extern __shared__ double smem_d[];
  cplx* sm = reinterpret_cast<cplx*>(smem_d);
  const int zi = blockIdx.x, tid = threadIdx.x, n = d.Nx1, K = d.K;
  grid += (size_t)blockIdx.y * n * d.Nz1;
  tmp += (size_t)blockIdx.y * d.Nz1 * K;
  cplx* b0 = sm;
  cplx* b1 = sm + fpad_size(n);
  for (int x = tid; x < n; x += NT) b0[fpad(x)] = cmk(grid[(size_t)x * d.Nz1 + zi], 0.0);
  __syncthreads();
  cplx* h = lds_fft(b0, b1, d.px1, d.twx1, -1, 1, n, tid, NT);
  for (int m = tid; m < K; m += NT) tmp[(size_t)zi * K + m] = cscale(h[fpad(m)], 1.0 / n);
}

__global__ void __launch_bounds__(NT) rbc_init_z(RbcDev d, const cplx* tmp, cplx* X) {
  __shared__ double ct[4 * 256];
  __shared__ cplx col[256];
  const int k = blockIdx.x, tid = threadIdx.x, N = d.N, S = d.S, K = d.K, Nz1 = d.Nz1;
  tmp += (size_t)blockIdx.y * Nz1 * K;
  X += (size_t)blockIdx.y * K * S;
  stage_cos(d.cosz1, ct, Nz1);
  for (int z = tid; z < Nz1; z += NT) col[z] = tmp[(size_t)z * K + k];
  __syncthreads();
  for (int s = tid; s < S; s += NT) {
    cplx v = czero();
    if (s >= 2 * N && s < 3 * N) {
      const int n = s - 2 * N;
      v = cscale(cheb_sum_nodes(ct, col, n, Nz1), (n == 0 ? 1.0 : 2.0) / Nz1);
    }
    X[(size_t)k * S + s] = v;
  }
}

__global__ void __launch_bounds__(NT) rbc_init_adj_z(RbcDev d, const cplx* Xb, cplx* tmp) {
  __shared__ double ct[4 * 256];
  __shared__ cplx cw[128];
  const int k = blockIdx.x, tid = threadIdx.x, N = d.N, S = d.S, K = d.K, Nz1 = d.Nz1;
  Xb += (size_t)blockIdx.y * K * S;
  tmp += (size_t)blockIdx.y * Nz1 * K;
  stage_cos(d.cosz1, ct, Nz1);
  for (int n = tid; n < N; n += NT) cw[n] = cscale(Xb[(size_t)k * S + 2 * N + n], (n == 0 ? 1.0 : 2.0) / Nz1);
  __syncthreads();
  for (int z = tid; z < Nz1; z += NT) tmp[(size_t)z * K + k] = cheb_sum_modes(ct, cw, z, N, Nz1);
}

__global__ void __launch_bounds__(NT) rbc_init_adj_x(RbcDev d, const cplx* tmp, double* gbar) {
  extern __shared__ double smem_d[];
  cplx* sm = reinterpret_cast<cplx*>(smem_d);
  const int zi = blockIdx.x, tid = threadIdx.x, n = d.Nx1, K = d.K;
  tmp += (size_t)blockIdx.y * d.Nz1 * K;
  gbar += (size_t)blockIdx.y * n * d.Nz1;
  cplx* b0 = sm;
  cplx* b1 = sm + fpad_size(n);
  const cplx* t = tmp + (size_t)zi * K;
  for (int m = tid; m < n; m += NT) {
    cplx v = czero();
    if (m == 0) v = cmk(t[0].x, 0.0);
    else if (m < K) v = cscale(t[m], 0.5);
    else if (m > n - K) v = cscale(cconj(t[n - m]), 0.5);
    b0[fpad(m)] = v;
  }
  __syncthreads();
  cplx* h = lds_fft(b0, b1, d.px1, d.twx1, +1, 1, n, tid, NT);
  for (int x = tid; x < n; x += NT) gbar[(size_t)x * d.Nz1 + zi] = h[fpad(x)].x / n;
}

// ---------------------------------------------------------------------------- cost
// J = cost_scale/2 sum_k w_k Re(c_k^H G c_k) over the first ncost fields (u, w for the 2D
// problem; u_par, v, u_perp for the 3D one), w_k = 1 for the x wavenumber 0, else 2, the k = 0
// coefficients taken by their real parts; dJ/dX alongside.  One block per mode.
__global__ void __launch_bounds__(NT) rbc_cost(RbcDev d, const cplx* X, cplx* Xb, double* Jpart) {
  __shared__ double red[NT];
  __shared__ cplx cf[3][128];
  const int k = blockIdx.x, tid = threadIdx.x, N = d.N, S = d.S, nc = d.ncost;
  X += (size_t)blockIdx.y * d.K * S;
  Xb += (size_t)blockIdx.y * d.K * S;
  Jpart += (size_t)blockIdx.y * d.K;
  const double wk = (d.ckeep && !d.ckeep[k]) ? 0.0 : ((k / d.Kz == 0) ? 1.0 : 2.0);
  for (int e = tid; e < nc * N; e += NT) {
    const int f = e / N, n = e - f * N;
    cplx a = X[(size_t)k * S + e];
    if (k == 0) a.y = 0.0;
    cf[f][n] = a;
  }
  __syncthreads();
  double part = 0.0;
  for (int s = tid; s < S; s += NT) {
    cplx v = czero();
    if (s < nc * N) {
      const int f = s / N, m = s - f * N;
      const cplx* c = cf[f];
      double gr = 0.0, gi = 0.0;
      for (int n = 0; n < N; ++n) {
        const double G = d.gram[m * N + n];
        gr += G * c[n].x;
        gi += G * c[n].y;
      }
      part += c[m].x * gr + c[m].y * gi;   // Re(conj(c_m) (G c)_m)
      v = cmk(d.cost_scale * wk * gr, d.cost_scale * wk * gi);
      if (k == 0) v.y = 0.0;
    }
    Xb[(size_t)k * S + s] = v;
  }
  red[tid] = part;
  __syncthreads();
  for (int o = NT / 2; o > 0; o >>= 1) {
    if (tid < o) red[tid] += red[tid + o];
    __syncthreads();
  }
  if (tid == 0) Jpart[k] = 0.5 * d.cost_scale * wk * red[0];
}

// Plane Couette states between the physical layout (u, v, w, p; taus of u, v, w first order,
// then second order, then tau_p) and the library's (u_par, v, u_perp, p; the same taus in the
// wave-vector frame, scaled to unit wall distance).  e[k] = (kx, kz) / |(kx, kz)| of mode k
// ((1, 0) at the mean mode).  One thread per (mode, index): index n < N takes the four
// coefficients of mode n, index N + t the first-order (t = 0) or second-order (t = 1) taus, or
// tau_p (t = 2).  to_lib: rotate into the frame and multiply the taus by tscale; else rotate
// back and divide them by tscale.
__global__ void cou_frame(int K, int N, const double2* e, const cplx* in, cplx* out, int to_lib, double tscale) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int S = 4 * N + 7, per = N + 3;
  if (i >= K * per) return;
  const int k = i / per, idx = i - k * per;
  const double ex = e[k].x, ez = e[k].y;
  const cplx* a = in + (size_t)k * S;
  cplx* o = out + (size_t)k * S;
  auto rot = [&](int s0, int s2, double sc) {
    const cplx u = a[s0], w = a[s2];
    if (to_lib) {
      o[s0] = cscale(cadd(cscale(u, ex), cscale(w, ez)), sc);
      o[s2] = cscale(cadd(cscale(u, -ez), cscale(w, ex)), sc);
    } else {
      o[s0] = cscale(cadd(cscale(u, ex), cscale(w, -ez)), sc);
      o[s2] = cscale(cadd(cscale(u, ez), cscale(w, ex)), sc);
    }
  };
  const double ts = to_lib ? tscale : 1.0 / tscale;
  if (idx < N) {
    rot(idx, 2 * N + idx, 1.0);
    o[N + idx] = a[N + idx];
    o[3 * N + idx] = a[3 * N + idx];
  } else if (idx < N + 2) {
    const int b = 4 * N + 3 * (idx - N);
    rot(b, b + 2, ts);
    o[b + 1] = cscale(a[b + 1], ts);
  } else {
    o[4 * N + 6] = cscale(a[4 * N + 6], ts);
  }
}

__global__ void fill_zero(double* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

// out[0] = dJ/dRa, out[1] = dJ/dPr from the per-wavenumber dJ/dnu, dJ/dkappa (summed over k in
// order by one thread, so the result does not depend on scheduling) and the chain-rule factors.
__global__ void rbc_param_finish(const double* pacc, int K, double nu_ra, double ka_ra, double nu_pr, double ka_pr,
                                 double* out) {
  if (threadIdx.x != 0) return;
  double sn = 0.0, sk = 0.0;
  for (int k = 0; k < K; ++k) {
    sn += pacc[2 * k];
    sk += pacc[2 * k + 1];
  }
  out[0] = nu_ra * sn + ka_ra * sk;
  out[1] = nu_pr * sn + ka_pr * sk;
}

// out[b] = sum of part[b][0..n) in order; one block per instance b
__global__ void sum_parts(const double* part, int n, double* out) {
  if (threadIdx.x == 0) {
    const double* p = part + (size_t)blockIdx.x * n;
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += p[i];
    out[blockIdx.x] = s;
  }
}

// ---------------------------------------------------------------------------- host: banded systems
struct RbcHostBands {
  int kl = 0, ku = 0;
  std::vector<double> BM, BL;   // [K][S][kl+ku+1] row bands of D_r M R D_c and D_r L R D_c
  std::vector<int> rowmap, colmap;
  std::vector<signed char> rowph, colph;
  std::vector<double> rho;
};

// ABI-slot dense M_k, L_k (complex), written from the formulation of the header comment.
// M and L of one mode: horizontal wavenumber kx (the mean mode when `mean`), viscosity nu,
// diffusivity ka of the third field, coupling cp of that field into the w rows.
// cw: coupling of w into the b rows (-cw S10 w), the linearized advection of the conduction
// profile in the stability operator (0 for the IVP).
static void rbc_assemble(int N, double kx, double nu, double ka, double cp, double cw, bool mean, Cmat& M, Cmat& L) {
  const double k2 = kx * kx;
  const std::vector<double> S0 = op_S0(N), S1 = op_S1(N);
  const std::vector<double> S10 = matmul(S1, S0, N);
  const std::vector<double> D0 = op_D(N, 1.0, true), D1 = op_D(N, 2.0, false);
  const std::vector<double> D10 = matmul(D1, D0, N);
  const std::vector<double> S1D0 = matmul(S1, D0, N);
  const int U = 0, W = N, B = 2 * N, P = 3 * N, T = 4 * N;
  const double difs[3] = {nu, nu, ka};
  for (int f = 0; f < 3; ++f) {
    const int r0 = f * N, c0 = f * N;
    const double dif = difs[f];
    for (int i = 0; i < N; ++i)
      for (int j = 0; j < N; ++j) {
        const double s10 = S10[(size_t)i * N + j], dzz = 4.0 * D10[(size_t)i * N + j];
        if (s10 != 0.0) M.add(r0 + i, c0 + j, s10);
        const double lv = -dif * (dzz - k2 * s10);
        if (lv != 0.0) L.add(r0 + i, c0 + j, lv);
      }
    L.add(r0 + N - 2, T + f, -4.0 * dif);   // lifted first-order tau
    L.add(r0 + N - 1, T + 3 + f, 1.0);      // second tau
  }
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      const double s10 = S10[(size_t)i * N + j];
      if (s10 != 0.0) {
        L.add(U + i, P + j, 0.0, kx * s10);   // i kx S10 p in x-momentum
        if (cp != 0.0) L.add(W + i, B + j, -cp * s10);   // -b in z-momentum
        if (cw != 0.0) L.add(B + i, W + j, -cw * s10);   // -w in the buoyancy rows (stability)
      }
      const double sd = 2.0 * S1D0[(size_t)i * N + j];
      if (sd != 0.0) L.add(W + i, P + j, sd);   // dp/dz in z-momentum
      const double s0 = S0[(size_t)i * N + j];
      if (s0 != 0.0) L.add(P + i, U + j, 0.0, kx * s0);   // continuity i kx u
      const double d0 = 2.0 * D0[(size_t)i * N + j];
      if (d0 != 0.0) L.add(P + i, W + j, d0);             // continuity dw/dz
    }
  L.add(P + N - 1, T + 1, 1.0);  // lift(tau_w1) in continuity
  for (int f = 0; f < 3; ++f)
    for (int m = 0; m < N; ++m) {
      L.add(T + 2 * f, f * N + m, (m & 1) ? -1.0 : 1.0);   // value at z = 0
      L.add(T + 2 * f + 1, f * N + m, 1.0);                // value at z = 1
    }
  if (mean) {
    L.add(P + 0, T + 6, 1.0);
    for (int m = 0; m < N; m += 2) L.add(T + 6, P + m, 1.0 / (1.0 - (double)m * m));
  } else {
    L.add(T + 6, T + 6, 1.0);
  }
}


// Real-ified banded M and L of every mode (mode k has wavenumber kx[k]; mode 0 is the mean mode).
// Modes with equal wavenumbers share their assembly.
static void host_bands(int N, const std::vector<double>& kxs, double nu, double ka, double cp, RbcHostBands& hb,
                       double cw = 0.0, int force_kl = -1, int force_ku = -1) {
  const int S = 4 * N + 7, K = (int)kxs.size();
  // phases and recombination
  std::vector<signed char> rowph(S, 0), colph(S, 0);
  for (int i = 0; i < N; ++i) rowph[i] = 1;
  rowph[4 * N + 0] = rowph[4 * N + 1] = 1;   // u boundary rows
  for (int i = 0; i < N; ++i) colph[i] = 1;
  colph[4 * N + 0] = colph[4 * N + 3] = 1;   // tau_u1, tau_u2
  std::vector<double> rho(S, 0.0);
  for (int f = 0; f < 3; ++f)
    for (int m = 0; m + 2 < N; ++m) rho[f * N + m] = -1.0;
  auto iw = [](int j) { return 1.0 / (1.0 - (double)j * j); };
  for (int m = 0; m + 2 < N; ++m) {
    const int j = m + 2;
    rho[3 * N + m] = (j % 2 == 0) ? -(iw(j) / iw(j - 2)) : 0.0;
  }
  // interleaved orders
  std::vector<int> rowmap, colmap;
  rowmap.push_back(4 * N + 6);
  for (int q = 0; q < 6; ++q) rowmap.push_back(4 * N + q);
  for (int n = 0; n < N; ++n) {
    rowmap.push_back(3 * N + n);
    rowmap.push_back(n);
    rowmap.push_back(N + n);
    rowmap.push_back(2 * N + n);
  }
  colmap.push_back(4 * N + 6);
  for (int n = 0; n < N; ++n)
    for (int f = 0; f < 4; ++f) colmap.push_back(f * N + n);
  for (int q = 0; q < 6; ++q) colmap.push_back(4 * N + q);
  // B = D_r (A R) D_c per k, for A in {M, L}; find the band
  std::vector<std::vector<double>> bm(K), bl(K);
  int kl = 0, ku = 0;
  auto transform = [&](Cmat& A, std::vector<double>& out) {
    out.assign((size_t)S * S, 0.0);
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
        if (colph[c]) v = make_double2(-v.y, v.x);   // times i
        if (rowph[r]) v = make_double2(v.y, -v.x);   // times -i
        row[j] = v;
        rowmax = std::max(rowmax, std::hypot(v.x, v.y));
      }
      for (int j = 0; j < S; ++j) {
        double2 v = row[j];
        if (std::hypot(v.x, v.y) <= 1e-14 * rowmax) continue;   // exact cancellations of R
        if (std::fabs(v.y) > 1e-13 * rowmax) throw Error(SPS_E_ARG, "real-ified RBC block is not real");
        out[(size_t)i * S + j] = v.x;
        kl = std::max(kl, i - j);
        ku = std::max(ku, j - i);
      }
    }
  };
  std::map<double, int> seen;
  for (int k = 0; k < K; ++k) {
    auto it = (k == 0) ? seen.end() : seen.find(kxs[k]);
    if (it != seen.end()) {
      bm[k] = bm[it->second];
      bl[k] = bl[it->second];
      continue;
    }
    Cmat M(S), L(S);
    rbc_assemble(N, kxs[k], nu, ka, cp, cw, k == 0, M, L);
    transform(M, bm[k]);
    transform(L, bl[k]);
    if (k > 0) seen[kxs[k]] = k;
  }
  if (force_kl >= 0) {   // the band of another operator of the same family (a batch's common layout)
    SPS_REQUIRE(kl <= force_kl && ku <= force_ku, "operator band wider than the batch's common band");
    kl = force_kl;
    ku = force_ku;
  }
  const int bw = kl + ku + 1;
  hb.kl = kl;
  hb.ku = ku;
  hb.BM.assign((size_t)K * S * bw, 0.0);
  hb.BL.assign((size_t)K * S * bw, 0.0);
  for (int k = 0; k < K; ++k)
    for (int i = 0; i < S; ++i)
      for (int j = std::max(0, i - kl); j <= std::min(S - 1, i + ku); ++j) {
        hb.BM[((size_t)k * S + i) * bw + (j - i + kl)] = bm[k][(size_t)i * S + j];
        hb.BL[((size_t)k * S + i) * bw + (j - i + kl)] = bl[k][(size_t)i * S + j];
      }
  hb.rowmap = rowmap;
  hb.colmap = colmap;
  hb.rowph = rowph;
  hb.colph = colph;
  hb.rho = rho;
}

void rbc_host_bands(const sps_desc& desc, RbcHostBands& hb) {
  std::vector<double> kx(desc.nx / 2);
  for (int k = 0; k < desc.nx / 2; ++k) kx[k] = 2.0 * M_PI * k / desc.lx;
  host_bands(desc.nz, kx, std::pow(desc.param0 / desc.param1, -0.5), std::pow(desc.param0 * desc.param1, -0.5), 1.0,
             hb);
}

class RbcProblem : public ProblemImpl {
 public:
  // ra (batch > 1 or ra given): a batch of instances of the problem with Rayleigh numbers ra[b]
  // and the descriptor's other parameters; each instance has its own factors.
  RbcProblem(const sps_desc& desc, hipStream_t s, int batch = 1, const double* ra = nullptr) : desc_(desc) {
    stream = s;
    SPS_REQUIRE(batch >= 1 && batch <= 4096, "batch must be in [1, 4096]");
    B_ = batch;
    if (ra) {
      rab_.assign(ra, ra + batch);
      for (double r : rab_) SPS_REQUIRE(std::isfinite(r) && r > 0.0, "Rayleigh numbers must be positive");
    }
    SPS_REQUIRE(desc.scheme == SPS_RK222 || desc.scheme == SPS_RK443, "RBC supports the RK222 and RK443 schemes");
    tab_ = rk_tableau(desc.scheme);
    SPS_REQUIRE(desc.nx >= 8 && desc.nx % 2 == 0, "nx must be even and >= 8");
    SPS_REQUIRE(desc.nz >= 8 && desc.nz <= 128 && desc.nz % 2 == 0, "nz must be even in [8, 128]");
    SPS_REQUIRE(desc.dealias == 1.5, "RBC uses 3/2 dealiasing");
    SPS_REQUIRE(desc.dt > 0 && desc.checkpoint_every >= 1 && desc.max_steps >= 1, "bad dt / checkpoint / max_steps");
    K_ = desc.nx / 2;
    N_ = desc.nz;
    S_ = 4 * N_ + 7;
    Ngx_ = 3 * desc.nx / 2;
    Ngz_ = 3 * N_ / 2;
    SPS_REQUIRE(fft_plan(Ngx_, &dv_.px), "3/2 nx must factor into 2 and 3");
    SPS_REQUIRE(fft_plan(desc.nx, &dv_.px1), "nx must factor into 2 and 3");
    nu_ = std::pow(desc.param0 / desc.param1, -0.5);
    ka_ = std::pow(desc.param0 * desc.param1, -0.5);
    dt_ = desc.dt;
    kxs_.resize(K_);
    for (int k = 0; k < K_; ++k) kxs_[k] = 2.0 * M_PI * k / desc.lx;
    cp_ = 1.0;
    bc0_ = 1.0;
    cost_scale_ = desc.lx;
    Kz_ = 1;
    ncost_ = 2;
    SPS_HIP(hipGetDevice(&device_));
    init();
  }

  // 3D plane Couette flow (perturbation of U = y between walls y = -1, 1 moving with -1, 1):
  // the per-mode Stokes systems of the frame scaled to unit wall distance (y' = (y + 1)/2,
  // x' = x/2, z' = z/2, t' = t/2: nu' = 1/(2 Re), dt' = dt/2, U = 2y' - 1) in the variables
  // (u_par, v, u_perp, p) of the wave-vector frame, with no buoyancy coupling and homogeneous
  // walls; the explicit term from the plane kernels of cou.hip.
  RbcProblem(const CouetteSpec& c, hipStream_t s) {
    stream = s;
    SPS_REQUIRE(c.nx >= 4 && c.nx % 2 == 0 && c.nz >= 4 && c.nz % 2 == 0, "nx and nz must be even and >= 4");
    SPS_REQUIRE(c.ny >= 8 && c.ny <= 128 && c.ny % 2 == 0, "ny must be even in [8, 128]");
    SPS_REQUIRE(c.lx > 0 && c.lz > 0 && c.re > 0, "bad periods or Reynolds number");
    SPS_REQUIRE(c.dt > 0 && c.checkpoint_every >= 1 && c.max_steps >= 1, "bad dt / checkpoint / max_steps");
    desc_ = sps_desc{};
    desc_.equation = SPS_COUETTE3D;
    desc_.scheme = SPS_RK222;
    tab_ = rk_tableau(SPS_RK222);
    desc_.nx = c.nx;
    desc_.nz = c.ny;
    desc_.lx = c.lx;
    desc_.dealias = 1.5;
    desc_.dt = c.dt;
    desc_.checkpoint_every = c.checkpoint_every;
    desc_.max_steps = c.max_steps;
    cou_ = true;
    const int Kx = c.nx / 2;
    K_ = Kx * c.nz;
    N_ = c.ny;
    S_ = 4 * N_ + 7;
    Ngx_ = 3 * c.nx / 2;
    Ngz_ = 3 * N_ / 2;
    SPS_REQUIRE(fft_plan(Ngx_, &dv_.px) && fft_plan(c.nx, &dv_.px1), "nx and 3 nx / 2 must factor into 2 and 3");
    nu_ = ka_ = 1.0 / (2.0 * c.re);
    dt_ = 0.5 * c.dt;
    const double lx = 0.5 * c.lx, lz = 0.5 * c.lz;
    kxs_.resize(K_);
    ckeep_.resize(K_);
    for (int m = 0; m < Kx; ++m)
      for (int n = 0; n < c.nz; ++n) {
        const int ns = (n < c.nz / 2) ? n : n - c.nz;
        kxs_[m * c.nz + n] = std::hypot(2.0 * M_PI * m / lx, 2.0 * M_PI * ns / lz);
        ckeep_[m * c.nz + n] = (n != c.nz / 2);
      }
    cp_ = 0.0;
    bc0_ = 0.0;
    cost_scale_ = 2.0 * c.lx * c.lz;
    Kz_ = c.nz;
    ncost_ = 3;
    std::vector<double> unode(Ngz_);
    for (int j = 0; j < Ngz_; ++j)
      unode[j] = -(double)cosl(3.14159265358979323846264338327950288L * (2 * j + 1) / (2.0L * Ngz_));
    CouetteGeom g{Kx, c.nz, Ngx_, 3 * c.nz / 2, Ngz_, lx, lz, unode.data(), 2.0};
    planes_.reset(new CouettePlanes(g, stream));
    std::vector<double2> fr(K_);
    for (int m = 0; m < Kx; ++m)
      for (int n = 0; n < c.nz; ++n) {
        const int ns = (n < c.nz / 2) ? n : n - c.nz;
        const double kx = 2.0 * M_PI * m / c.lx, kz = 2.0 * M_PI * ns / c.lz, kh = std::hypot(kx, kz);
        fr[m * c.nz + n] = kh > 0.0 ? make_double2(kx / kh, kz / kh) : make_double2(1.0, 0.0);
      }
    frame_ = arena_.upload(fr, stream);
    init();
  }

  void init() {
    dv_.B = B_;
    cur_dt_ = dt_;
    stream_solve_ = (long long)K_ * B_ > 1024;
    build_tables();
    build_bands();
    alloc_work();
    // the reverse sweep recomputes segment j-1 on a second stream while the adjoint of segment
    // j runs on the caller's; non-blocking so a legacy default caller stream does not serialize
    SPS_HIP(hipStreamCreateWithFlags(&aux_, hipStreamNonBlocking));
    for (auto& e : ev_) SPS_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  ~RbcProblem() override {
    drop_graphs();
    if (host_ckpt_) (void)hipStreamSynchronize(stream);   // copies into pinned host memory
    close_ckpt_file();
    for (auto e : ckev_)
      if (e) (void)hipEventDestroy(e);
    if (cap_) (void)hipStreamDestroy(cap_);
    if (aux_) (void)hipStreamSynchronize(aux_);
    for (auto e : ev_)
      if (e) (void)hipEventDestroy(e);
    if (aux_) (void)hipStreamDestroy(aux_);
  }

  long long state_size() const override { return (long long)B_ * K_ * S_ * 2; }
  size_t st() const { return (size_t)B_ * K_ * S_; }   // complex entries of a state (all instances)
  void no_batch(const char* what) const {
    if (B_ > 1 || !rab_.empty()) throw Error(SPS_E_UNSUPPORTED, std::string(what) + " is not built for batches");
  }

  // the descriptor for factors of one unpartitioned system per wavenumber at ops (the boundary
  // value and eigenvalue problems' factor sets)
  RbcDev whole_dev(double* ops) const {
    RbcDev d = dv_;
    d.ops = ops;
    d.part = 0;
    d.blksz = d.opsize = blk_ops_size(S_);
    d.tsz = blk_t_size(S_);
    return d;
  }

  // M + dt H_ii L (the implicit diagonal is one value for every stage)
  void factor() override {
    if (factored_) return;
    factor_into(dt_, ops_);
    factored_ = true;
  }
  void factor_into(double dt, double* ops) {
    RbcDev d = dv_;
    d.ops = ops;
    hipLaunchKernelGGL(rbc_factor, dim3(K_, B_), dim3(NT), factor_lds(), stream, d, BM_, BL_, 1.0, dt * tab_.H[1][1],
                       ops, BLnu_, BLka_);
    SPS_CHECK_LAUNCH();
  }

  // Variable steps (equ:imex with step-dependent coefficients): step i of a run takes vdt_[i]
  // in its stage coefficients and its own factors M + vdt_[i] H_ii L, one factor set per
  // distinct step (kept for later calls); the reverse sweep uses the same step's set.
  static constexpr int kMaxStepSets = 16;
  void set_timesteps(const double* dts, int n) override {
    drop_graphs();
    tape_steps_ = -1;
    if (!dts || n == 0) {
      vdt_.clear();
      vset_.clear();
      return;
    }
    SPS_REQUIRE(n >= 1 && n <= desc_.max_steps, "n must be in [1, max_steps]");
    std::vector<double> v(n);
    std::vector<int> set(n);
    std::vector<double> distinct;
    for (int i = 0; i < n; ++i) {
      SPS_REQUIRE(std::isfinite(dts[i]) && dts[i] > 0.0, "steps must be positive");
      v[i] = cou_ ? 0.5 * dts[i] : dts[i];
      auto it = std::find(distinct.begin(), distinct.end(), v[i]);
      if (it == distinct.end()) {
        SPS_REQUIRE((int)distinct.size() < kMaxStepSets, "at most 16 distinct steps");
        distinct.push_back(v[i]);
        it = distinct.end() - 1;
      }
      set[i] = (int)(it - distinct.begin());
    }
    std::vector<double*> ops(distinct.size());
    for (size_t q = 0; q < distinct.size(); ++q) {
      auto c = opcache_.find(distinct[q]);
      if (c == opcache_.end()) {
        SPS_REQUIRE(opcache_.size() < 4 * kMaxStepSets, "too many distinct steps over the problem's lifetime");
        double* o = arena_.alloc<double>((size_t)B_ * K_ * dv_.opsize);
        factor_into(distinct[q], o);
        c = opcache_.emplace(distinct[q], o).first;
      }
      ops[q] = c->second;
    }
    vdt_ = v;
    vset_ = set;
    vops_ = ops;
  }
  // the step and factors of step n of the run (n < 0: the constant step) for the launches
  // enqueued next
  void step_setup(int n) {
    if (n < 0 || vdt_.empty()) {
      cur_dt_ = dt_;
      dv_.ops = ops_;
      return;
    }
    const int g = step_base_ + n;
    cur_dt_ = vdt_[g];
    dv_.ops = vops_[vset_[g]];
  }
  // every sweep leaves the constant step's settings behind, also when it throws
  struct StepScope {
    RbcProblem* p;
    ~StepScope() {
      p->step_base_ = 0;
      p->step_setup(-1);
    }
  };
  void check_run_length(int nsteps) const {
    if (!vdt_.empty() && nsteps > (int)vdt_.size())
      throw Error(SPS_E_ARG, "nsteps exceeds the number of variable steps set");
  }

  // A new step for the following runs: the matrices M + dt H_ii L of every wavenumber are
  // refactored at once (in the scaled frame for plane Couette); recorded runs and captured
  // graphs are dropped.
  void set_dt(double dt) override {
    SPS_REQUIRE(std::isfinite(dt) && dt > 0.0, "dt must be positive");
    drop_graphs();
    desc_.dt = dt;
    dt_ = cou_ ? 0.5 * dt : dt;
    cur_dt_ = dt_;
    factored_ = false;
    tape_steps_ = -1;
    factor();
  }

  void step(double* X, int nsteps) override {
    SPS_REQUIRE(X != nullptr, "X is null");
    SPS_REQUIRE(nsteps >= 1 && nsteps <= desc_.max_steps, "nsteps out of range");
    check_run_length(nsteps);
    factor();
    StepScope scope{this};
    forward(reinterpret_cast<cplx*>(X), nsteps);
  }

  // plane Couette: physical (u, v, w) layout <-> the library's wave-vector frame; a state's taus
  // are twice the physical ones in the library (unit wall distance), a cotangent's half
  void couette_frame(const double* in, double* out, int to_lib, int cotangent) override {
    if (!cou_) throw Error(SPS_E_UNSUPPORTED, "the frame conversion is for plane Couette states");
    SPS_REQUIRE(in && out, "null argument");
    const int n = K_ * (N_ + 3);
    hipLaunchKernelGGL(cou_frame, dim3((n + NT - 1) / NT), dim3(NT), 0, stream, K_, N_, frame_,
                       reinterpret_cast<const cplx*>(in), reinterpret_cast<cplx*>(out), to_lib ? 1 : 0,
                       cotangent ? 0.5 : 2.0);
    SPS_CHECK_LAUNCH();
  }

  void adjoint_step(double* Xbar, int nsteps) override {
    SPS_REQUIRE(Xbar != nullptr, "Xbar is null");
    if (tape_steps_ != nsteps) throw Error(SPS_E_STATE, "adjoint_step: nsteps does not match the recorded forward run");
    StepScope scope{this};
    reverse(reinterpret_cast<cplx*>(Xbar), nsteps);
  }

  void cost(const double* X, double* J, double* dJdX) override {
    SPS_REQUIRE(X && dJdX, "null argument");
    hipLaunchKernelGGL(rbc_cost, dim3(K_, B_), dim3(NT), 0, stream, dv_, reinterpret_cast<const cplx*>(X),
                       reinterpret_cast<cplx*>(dJdX), Jpart_);
    SPS_CHECK_LAUNCH();
    if (J) {
      hipLaunchKernelGGL(sum_parts, dim3(B_), dim3(64), 0, stream, Jpart_, K_, J);
      SPS_CHECK_LAUNCH();
    }
  }

  void set_graph(bool on) override {
    if (!on) drop_graphs();
    graph_on_ = on;
  }

  void gradient(const double* X0, int nsteps, const double* dJdXN, double* XN, double* dJdX0, double* dJdtheta,
                double* J) override {
    SPS_REQUIRE(X0 && dJdX0, "null argument");
    SPS_REQUIRE(nsteps >= 1 && nsteps <= desc_.max_steps, "nsteps out of range");
    check_run_length(nsteps);
    StepScope scope{this};
    if (dJdtheta) {
      no_batch("the parameter gradient");
      if (cou_) throw Error(SPS_E_UNSUPPORTED, "parameter gradients are built for the 2D problem");
      if (ckpt_mode_ != SPS_CKPT_UNIFORM)
        throw Error(SPS_E_UNSUPPORTED, "parameter gradients need the uniform checkpoint schedule");
      if (!sst_) {
        sst_ = arena_.alloc<cplx>((size_t)2 * seglen_ * tab_.s * K_ * S_);
        pacc_ = arena_.alloc<double>((size_t)2 * K_);
      }
    }
    factor();
    if (graph_on_ && ckpt_mode_ != SPS_CKPT_TWO_LEVEL) {
      const GraphKey key{X0, dJdXN, XN, dJdX0, dJdtheta, J, nsteps};
      for (const auto& g : graphs_)
        if (g.first == key) {
          SPS_HIP(hipGraphLaunch(g.second, stream));
          after_graph_gradient(nsteps);
          return;
        }
      graphs_.emplace_back(key, capture_gradient(X0, nsteps, dJdXN, XN, dJdX0, dJdtheta, J));
      SPS_HIP(hipGraphLaunch(graphs_.back().second, stream));
      after_graph_gradient(nsteps);
      return;
    }
    gradient_launches(X0, nsteps, dJdXN, XN, dJdX0, dJdtheta, J);
  }

  // the recorded-run state a replayed gradient leaves (as its eager launches would)
  void after_graph_gradient(int nsteps) {
    tape_steps_ = ckpt_mode_ == SPS_CKPT_BINOMIAL ? -1 : nsteps;
    const int ce = desc_.checkpoint_every;
    last_seg_ok_ = (nsteps + ce - 1) / ce < 3;
  }

  // the launch sequence of one gradient on `stream` (and the auxiliary stream)
  void gradient_launches(const double* X0, int nsteps, const double* dJdXN, double* XN, double* dJdX0,
                         double* dJdtheta, double* J) {
    // the parameter gradient records the stage states of every recorded step and accumulates
    // over the reverse sweep; it is on for this gradient only
    param_on_ = dJdtheta != nullptr;
    theta_out_ = dJdtheta;
    struct Off {
      RbcProblem* p;
      ~Off() { p->param_on_ = false; p->theta_out_ = nullptr; }
    } off{this};
    SPS_HIP(hipMemcpyAsync(Xg_, X0, sizeof(cplx) * st(), hipMemcpyDeviceToDevice, stream));
    forward(Xg_, nsteps);
    if (XN) SPS_HIP(hipMemcpyAsync(XN, Xg_, sizeof(cplx) * st(), hipMemcpyDeviceToDevice, stream));
    if (dJdXN) {
      if (dJdXN != dJdX0) SPS_HIP(hipMemcpyAsync(dJdX0, dJdXN, sizeof(cplx) * st(), hipMemcpyDeviceToDevice, stream));
    } else {
      cost(reinterpret_cast<const double*>(Xg_), J, dJdX0);
    }
    reverse(reinterpret_cast<cplx*>(dJdX0), nsteps);
  }

  void initial_state(const double* grid, double* X) override {
    if (cou_) throw Error(SPS_E_UNSUPPORTED, "Couette states are given as coefficients");
    SPS_REQUIRE(grid && X, "null argument");
    hipLaunchKernelGGL(rbc_init_x, dim3(N_, B_), dim3(NT), 2 * fpad_size(desc_.nx) * sizeof(cplx), stream, dv_, grid,
                       itmp_);
    SPS_CHECK_LAUNCH();
    hipLaunchKernelGGL(rbc_init_z, dim3(K_, B_), dim3(NT), 0, stream, dv_, itmp_, reinterpret_cast<cplx*>(X));
    SPS_CHECK_LAUNCH();
  }

  void initial_state_adjoint(const double* Xbar, double* grid) override {
    if (cou_) throw Error(SPS_E_UNSUPPORTED, "Couette states are given as coefficients");
    SPS_REQUIRE(grid && Xbar, "null argument");
    hipLaunchKernelGGL(rbc_init_adj_z, dim3(K_, B_), dim3(NT), 0, stream, dv_, reinterpret_cast<const cplx*>(Xbar),
                       itmp_);
    SPS_CHECK_LAUNCH();
    hipLaunchKernelGGL(rbc_init_adj_x, dim3(N_, B_), dim3(NT), 2 * fpad_size(desc_.nx) * sizeof(cplx), stream, dv_,
                       itmp_, grid);
    SPS_CHECK_LAUNCH();
  }

  void eval_F(const double* X, double* F) override {
    no_batch("this evaluation");
    SPS_REQUIRE(X && F, "null argument");
    launch_kf(KF_ZGRID, reinterpret_cast<const cplx*>(X), nullptr, zgA_);
    launch_xf(zgA_);
    launch_kf(KF_EVALF, nullptr, reinterpret_cast<cplx*>(F), nullptr);
  }

  // eval_F with its intermediates in the library's static per-device scratch: no device
  // allocation, no timer events, three launches on the problem's stream.  Calls that overlap
  // on one GPU share the scratch and race.
  void eval_F_noalloc(const double* X, double* F) override {
    no_batch("the allocation-free evaluation");
    if (cou_) throw Error(SPS_E_UNSUPPORTED, "the allocation-free evaluation is built for the 2D problem");
    SPS_REQUIRE(X && F, "null argument");
    const size_t need = (size_t)9 * Ngz_ * K_ * sizeof(cplx);
    if (need > SPS_SCRATCH_BYTES)
      throw Error(SPS_E_ARG, "eval_F_noalloc: the problem needs " + std::to_string(need) +
                                 " bytes of scratch, more than the library's " + std::to_string(SPS_SCRATCH_BYTES));
    cplx* zg = reinterpret_cast<cplx*>(scratch_address(device_));
    cplx* nl = zg + (size_t)6 * Ngz_ * K_;
    KfArgs a{};
    a.X0 = reinterpret_cast<const cplx*>(X);
    a.nl = nl;
    a.zg = zg;
    a.dt = dt_;
    a.mode = KF_ZGRID;
    hipLaunchKernelGGL(kfwd_fn(), dim3(K_), dim3(NTK), kf_lds(), stream, dv_, a);
    SPS_CHECK_LAUNCH();
    launch_xf_rows(zg, nl, stream);
    a.X0 = nullptr;
    a.Xout = reinterpret_cast<cplx*>(F);
    a.zg = nullptr;
    a.mode = KF_EVALF;
    hipLaunchKernelGGL(kfwd_fn(), dim3(K_), dim3(NTK), kf_lds(), stream, dv_, a);
    SPS_CHECK_LAUNCH();
  }

  void eval_F_vjp(const double* X, const double* Fbar, double* Xbar) override {
    no_batch("this evaluation");
    SPS_REQUIRE(X && Fbar && Xbar, "null argument");
    launch_kf(KF_ZGRID, reinterpret_cast<const cplx*>(X), nullptr, zgA_);
    KaArgs a = ka_args(KA_G);
    a.Xb_in = reinterpret_cast<const cplx*>(Fbar);
    launch_ka(a);
    launch_xa(zgA_);
    a = ka_args(KA_C);
    a.acc = nullptr;
    a.Xb_out = reinterpret_cast<cplx*>(Xbar);
    launch_ka(a);
  }

  void solve(const double* R, double* X, int adjoint) override {
    no_batch("this evaluation");
    SPS_REQUIRE(R && X, "null argument");
    factor();
    if (!adjoint) {
      launch_kf(KF_SOLVE, reinterpret_cast<const cplx*>(R), reinterpret_cast<cplx*>(X), nullptr);
    } else {
      KaArgs a = ka_args(KA_SOLVE_T);
      a.Xb_in = reinterpret_cast<const cplx*>(R);
      a.Xb_out = reinterpret_cast<cplx*>(X);
      launch_ka(a);
    }
  }

  // Linear boundary value problem L X = M f + c: L factored once (the same blocked LU as the
  // IVP's matrix, with a = 0, b = 1), the forward solve and the adjoint through those factors.
  void lbvp_factor() {
    if (lfactored_) return;
    if (!lops_) {
      lops_ = arena_.alloc<double>((size_t)K_ * dv_.opsize);
      lrhs_ = arena_.alloc<cplx>((size_t)K_ * S_);
    }
    hipLaunchKernelGGL(rbc_factor, dim3(K_), dim3(NT), factor_lds(), stream, whole_dev(lops_), BM_, BL_, 0.0, 1.0,
                       lops_);
    SPS_CHECK_LAUNCH();
    lfactored_ = true;
  }

  void lbvp_solve(const double* f, double* X) override {
    no_batch("the boundary value problem");
    if (cou_) throw Error(SPS_E_UNSUPPORTED, "the boundary value problem is built for the 2D problem");
    SPS_REQUIRE(f && X, "null argument");
    lbvp_factor();
    hipLaunchKernelGGL(rbc_lbvp_rhs, dim3(K_), dim3(NT), 0, stream, dv_, reinterpret_cast<const cplx*>(f), lrhs_);
    SPS_CHECK_LAUNCH();
    RbcDev dl = whole_dev(lops_);
    KfArgs a = kf_args(KF_SOLVE);
    a.X0 = lrhs_;
    a.Xout = reinterpret_cast<cplx*>(X);
    hipLaunchKernelGGL(kfwd_fn(), dim3(K_), dim3(NTK), kf_lds(), stream, dl, a);
    SPS_CHECK_LAUNCH();
  }

  void lbvp_adjoint(const double* Xbar, double* fbar) override {
    no_batch("the boundary value problem");
    if (cou_) throw Error(SPS_E_UNSUPPORTED, "the boundary value problem is built for the 2D problem");
    SPS_REQUIRE(Xbar && fbar, "null argument");
    lbvp_factor();
    RbcDev dl = whole_dev(lops_);
    KaArgs a = ka_args(KA_SOLVE_T);
    a.Xb_in = reinterpret_cast<const cplx*>(Xbar);
    a.Xb_out = lrhs_;
    hipLaunchKernelGGL(kadj_fn(), dim3(K_), dim3(NTK), ka_lds(), stream, dl, a);
    SPS_CHECK_LAUNCH();
    hipLaunchKernelGGL(rbc_lbvp_rhs_adj, dim3(K_), dim3(NT), 0, stream, dv_, lrhs_, reinterpret_cast<cplx*>(fbar));
    SPS_CHECK_LAUNCH();
  }

  // Eigenvalue problem of the conduction state's perturbations, every wavenumber at once: the
  // stability bands (built on first use), one factorization of sigma M + L_s, `iters` inverse
  // iterations for the right and for the left eigenvector through those factors, then the
  // sensitivities.  lam[K], dlam[K][2] complex; X, Y [K][S] complex (unit norm); device arrays.
  // Bands, factor storage and default start vector of the stability operator (first call),
  // then the factors of sigma M + L_s; returns the descriptor with that band.
  RbcDev evp_setup(double sigma) {
    if (!eops_) {
      RbcHostBands hb;
      host_bands(N_, kxs_, nu_, ka_, cp_, hb, 1.0);
      SPS_REQUIRE(hb.kl + SPS_BLK <= SPS_TW && SPS_BLK + hb.kl + hb.ku <= SPS_GW,
                  "stability band too wide for the block solver");
      ekl_ = hb.kl;
      eku_ = hb.ku;
      eBM_ = arena_.upload(hb.BM, stream);
      eBL_ = arena_.upload(hb.BL, stream);
      eops_ = arena_.alloc<double>((size_t)K_ * dv_.opsize);
      ework_ = arena_.alloc<cplx>((size_t)K_ * S_);
      std::vector<cplx> x0((size_t)K_ * S_, make_double2(0.0, 0.0));
      for (int k = 0; k < K_; ++k)
        for (int s = 0; s < 3 * N_; ++s) x0[(size_t)k * S_ + s] = make_double2(1.0 / (1 + s % N_), 0.5 / (1 + s / N_));
      estart_ = arena_.upload(x0, stream);
      const size_t lds = (size_t)(2 * ekl_ + eku_ + 1) * S_ * sizeof(double) + sizeof(int) * S_;
      SPS_REQUIRE(lds <= 160 * 1024, "problem too large for LDS");
      if (lds > factor_lds())
        SPS_HIP(hipFuncSetAttribute((const void*)rbc_factor, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    }
    RbcDev de = whole_dev(eops_);
    de.kl = ekl_;
    de.ku = eku_;
    de.uw = ekl_ + eku_ + 1;
    de.ops = eops_;
    const size_t lds = (size_t)(2 * ekl_ + eku_ + 1) * S_ * sizeof(double) + sizeof(int) * S_;
    hipLaunchKernelGGL(rbc_factor, dim3(K_), dim3(NT), lds, stream, de, eBM_, eBL_, sigma, 1.0, eops_);
    SPS_CHECK_LAUNCH();
    return de;
  }
  // y = (sigma M + L_s)^-1 M x for every wavenumber through the factors of evp_setup
  void evp_apply(const RbcDev& de, const cplx* x, cplx* y) {
    hipLaunchKernelGGL(rbc_apply_m, dim3(K_), dim3(NT), 0, stream, de, x, ework_);
    SPS_CHECK_LAUNCH();
    evp_solve(de, ework_, y);
  }
  // y = (sigma M + L_s)^-1 r
  void evp_solve(const RbcDev& de, const cplx* r, cplx* y) {
    KfArgs a = kf_args(KF_SOLVE);
    a.X0 = r;
    a.Xout = y;
    hipLaunchKernelGGL(kfwd_fn(), dim3(K_), dim3(NTK), kf_lds(), stream, de, a);
    SPS_CHECK_LAUNCH();
  }

  void stability(double sigma, int iters, double* lam, double* X, double* Y, double* dlam) override {
    no_batch("the eigenvalue problem");
    if (cou_) throw Error(SPS_E_UNSUPPORTED, "the eigenvalue problem is built for the 2D problem");
    SPS_REQUIRE(lam && X && Y && dlam, "null argument");
    SPS_REQUIRE(iters >= 1 && iters <= 10000, "iters must be in [1, 10000]");
    const RbcDev de = evp_setup(sigma);
    cplx* x = reinterpret_cast<cplx*>(X);
    cplx* y = reinterpret_cast<cplx*>(Y);
    cplx* l = reinterpret_cast<cplx*>(lam);
    // right eigenvector
    copy_state(x, estart_);
    for (int it = 0; it < iters; ++it) {
      evp_apply(de, x, y);   // y is scratch until the left iteration
      hipLaunchKernelGGL(rbc_evp_update, dim3(K_), dim3(NT), 0, stream, de, x, y, sigma, l);
      SPS_CHECK_LAUNCH();
    }
    // left (adjoint) eigenvector through the same factors
    copy_state(y, estart_);
    for (int it = 0; it < iters; ++it) {
      hipLaunchKernelGGL(rbc_lbvp_rhs_adj, dim3(K_), dim3(NT), 0, stream, de, y, ework_);   // M^H y
      SPS_CHECK_LAUNCH();
      KaArgs a = ka_args(KA_SOLVE_T);
      a.Xb_in = ework_;
      a.Xb_out = Xw_;
      hipLaunchKernelGGL(kadj_fn(), dim3(K_), dim3(NTK), ka_lds(), stream, de, a);
      SPS_CHECK_LAUNCH();
      hipLaunchKernelGGL(rbc_evp_update, dim3(K_), dim3(NT), 0, stream, de, y, Xw_, sigma, nullptr);
      SPS_CHECK_LAUNCH();
    }
    const double Ra = desc_.param0;
    hipLaunchKernelGGL(rbc_evp_sens, dim3(K_), dim3(NT), 0, stream, de, x, y, -0.5 * nu_ / Ra, -0.5 * ka_ / Ra,
                       reinterpret_cast<cplx*>(dlam));
    SPS_CHECK_LAUNCH();
  }

  void stability_vector_sens(double sigma, int iters, const double* lam, const double* X, const double* Y,
                             const double* dlam, double* dX) override {
    no_batch("the eigenvalue problem");
    if (cou_) throw Error(SPS_E_UNSUPPORTED, "the eigenvalue problem is built for the 2D problem");
    SPS_REQUIRE(lam && X && Y && dlam && dX, "null argument");
    SPS_REQUIRE(iters >= 1 && iters <= 10000, "iters must be in [1, 10000]");
    const RbcDev de = evp_setup(sigma);
    if (!vsR_) {
      vsR_ = arena_.alloc<cplx>((size_t)K_ * S_);
      vsW_ = arena_.alloc<cplx>((size_t)K_ * S_);
      vsQ_ = arena_.alloc<cplx>((size_t)K_ * S_);
    }
    const cplx* x = reinterpret_cast<const cplx*>(X);
    const cplx* l = reinterpret_cast<const cplx*>(lam);
    hipLaunchKernelGGL(rbc_lbvp_rhs_adj, dim3(K_), dim3(NT), 0, stream, de, reinterpret_cast<const cplx*>(Y), vsQ_);
    SPS_CHECK_LAUNCH();   // Q = M^H Y
    const double Ra = desc_.param0;
    for (int p = 0; p < 2; ++p) {
      cplx* z = reinterpret_cast<cplx*>(dX) + (size_t)p * K_ * S_;
      hipLaunchKernelGGL(rbc_evp_dlx, dim3(K_), dim3(NT), 0, stream, de, x, reinterpret_cast<const cplx*>(dlam), p,
                         -0.5 * nu_ / Ra, -0.5 * ka_ / Ra, vsR_);
      SPS_CHECK_LAUNCH();
      evp_solve(de, vsR_, z);
      hipLaunchKernelGGL(rbc_vs_project, dim3(K_), dim3(NT), 0, stream, de, z, x, vsQ_);
      SPS_CHECK_LAUNCH();
      for (int it = 1; it < iters; ++it) {
        hipLaunchKernelGGL(rbc_apply_m, dim3(K_), dim3(NT), 0, stream, de, z, ework_);
        SPS_CHECK_LAUNCH();
        hipLaunchKernelGGL(rbc_vs_combine, dim3(K_), dim3(NT), 0, stream, de, vsR_, ework_, l, sigma, vsW_);
        SPS_CHECK_LAUNCH();
        evp_solve(de, vsW_, z);
        hipLaunchKernelGGL(rbc_vs_project, dim3(K_), dim3(NT), 0, stream, de, z, x, vsQ_);
        SPS_CHECK_LAUNCH();
      }
      hipLaunchKernelGGL(rbc_vs_project, dim3(K_), dim3(NT), 0, stream, de, z, x, x);
      SPS_CHECK_LAUNCH();
    }
  }

  void stability_arnoldi(double sigma, int m, int nev, const double* v0, double* lam, double* X, double* res,
                         double* Hout) override {
    no_batch("the eigenvalue problem");
    if (cou_) throw Error(SPS_E_UNSUPPORTED, "the eigenvalue problem is built for the 2D problem");
    SPS_REQUIRE(lam != nullptr, "lam is null");
    SPS_REQUIRE(m >= 2 && m <= ARN_MAX_M, "m must be in [2, 64]");
    SPS_REQUIRE(nev >= 1 && nev <= m, "nev must be in [1, m]");
    SPS_REQUIRE(m <= 3 * N_, "m must not exceed the rank of M (3 nz)");
    const RbcDev de = evp_setup(sigma);
    if (!aV_) {
      aV_ = arena_.alloc<cplx>((size_t)(ARN_MAX_M + 1) * K_ * S_);
      aH_ = arena_.alloc<cplx>((size_t)K_ * (ARN_MAX_M + 1) * ARN_MAX_M);
      aZ_ = arena_.alloc<cplx>((size_t)K_ * 2 * ARN_MAX_M * ARN_MAX_M);
      aY_ = arena_.alloc<cplx>((size_t)K_ * ARN_MAX_M * ARN_MAX_M);
      SPS_HIP(hipFuncSetAttribute((const void*)rbc_hess_eig, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)kHessLdsMax));
    }
    auto vec = [&](int i) { return aV_ + (size_t)i * K_ * S_; };
    copy_state(vec(0), v0 ? reinterpret_cast<const cplx*>(v0) : estart_);
    const size_t wl = sizeof(cplx) * S_;
    hipLaunchKernelGGL(rbc_arnoldi_orth, dim3(K_), dim3(NT), wl, stream, de, aV_, aH_, -1, m);
    SPS_CHECK_LAUNCH();
    for (int j = 0; j < m; ++j) {
      evp_apply(de, vec(j), vec(j + 1));
      hipLaunchKernelGGL(rbc_arnoldi_orth, dim3(K_), dim3(NT), wl, stream, de, aV_, aH_, j, m);
      SPS_CHECK_LAUNCH();
    }
    if (Hout)
      SPS_HIP(hipMemcpyAsync(Hout, aH_, sizeof(cplx) * K_ * (m + 1) * m, hipMemcpyDeviceToDevice, stream));
    const int zlds = hess_lds(m, true) <= kHessLdsMax ? 1 : 0;
    hipLaunchKernelGGL(rbc_hess_eig, dim3(K_), dim3(ARN_NT), hess_lds(m, zlds != 0), stream, de, aH_, m, nev, sigma,
                       reinterpret_cast<cplx*>(lam), res, aY_, aZ_, zlds);
    SPS_CHECK_LAUNCH();
    if (X) {
      hipLaunchKernelGGL(rbc_ritz, dim3(K_, nev), dim3(NT), 0, stream, de, aV_, aY_, m, nev, reinterpret_cast<cplx*>(X));
      SPS_CHECK_LAUNCH();
    }
  }
  // LDS of rbc_hess_eig: H, Z, rotations, nu, residuals, selection, and with zlds the
  // eigenvector work arrays
  static size_t hess_lds(int m, bool zlds) {
    return sizeof(cplx) * ((size_t)hess_zoff(m) + (zlds ? (size_t)2 * m * m : 0));
  }
  static constexpr size_t kHessLdsMax = 160 * 1024;

  void timer_enable(int kind, bool on) override {
    SPS_REQUIRE(kind >= 0 && kind <= 3, "unknown timer kind");
    timer_kind_ = kind;
    timer_.enable(on);
  }
  // the timer's event pair for a launch of kernel class `kind` on stream s, if it is timed
  bool timed(int kind, hipStream_t s, hipEvent_t* e0, hipEvent_t* e1) {
    return kind == timer_kind_ && s == stream && !capturing_ && timer_.take(e0, e1);
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
  // ----------------------------------------------------------------- launches
  size_t factor_lds() const {
    const size_t ldab = 2 * kl_ + ku_ + 1;
    const size_t whole = ldab * S_ * sizeof(double) + sizeof(int) * S_;
    if (!dv_.part) return whole;
    size_t mx = 0;
    for (int p = 0; p < dv_.part; ++p) mx = std::max<size_t>(mx, pmeta_h_[8 * p + 1]);
    const size_t nr = std::max(dv_.nrr[0], dv_.nrr[1]);
    const size_t partd = mx * ldab + (mx + 1) / 2 + 1 + mx * SPS_SPIKE_W + nr * nr + nr * (2 * nr + 1);
    return std::max(whole, partd * sizeof(double));
  }
  // staged solves hold a system's block operators in LDS; streamed ones two chunk buffers
  size_t ops_bytes() const {
    if (stream_solve_) return sizeof(double) * 2 * (size_t)SOLVE_CHUNK_D;
    return sizeof(double) * (size_t)dv_.blksz;
  }
  // launches with many more systems than CUs stream the operators (several blocks per CU);
  // smaller ones stage them whole (one block per CU, shortest dependent chain)
  typedef void (*KfFn)(RbcDev, KfArgs);
  typedef void (*KaFn)(RbcDev, KaArgs);
  KfFn kfwd_fn() const { return stream_solve_ ? rbc_kfwd<true> : rbc_kfwd<false>; }
  KaFn kadj_fn() const { return stream_solve_ ? rbc_kadj<true> : rbc_kadj<false>; }
  // bytes of the stage kernels' phase buffers before the solve (from the union's start)
  size_t kf_pre() const {
    return sizeof(cplx) * (3 * S_ + 6 * half_nodes(Ngz_) + 6 * N_) + sizeof(double) * 4 * Ngz_;
  }
  size_t ka_pre() const {
    return sizeof(double) * 4 * Ngz_ + sizeof(cplx) * (2 * S_ + 12 * half_nodes(Ngz_) + 9 * N_);
  }
  size_t kf_lds() const {
    const size_t post = sizeof(double) * 4 * Ngz_ + sizeof(cplx) * 3 * N_;
    return sizeof(cplx) * (2 * S_ + SPS_PAD) + std::max({kf_pre(), post, ops_bytes()});
  }
  size_t ka_lds() const {
    const size_t post = sizeof(double) * (4 * Ngz_ + 2 * NTK / 64) + sizeof(cplx) * (5 * S_ + 3 * N_);
    return sizeof(cplx) * (2 * S_ + SPS_PAD) + std::max({ka_pre(), post, ops_bytes()});
  }
  size_t xf_lds() const { return sizeof(cplx) * (9 * K_ + 2 * fpad_size(4 * Ngx_) + Ngx_); }
  size_t xa_lds() const { return sizeof(cplx) * (12 * K_ + 2 * fpad_size(6 * Ngx_) + Ngx_); }

  // ----------------------------------------------------------------- graphs
  struct GraphKey {
    const double *X0, *dJN;
    double *XN, *dJ, *th, *J;
    int nsteps;
    bool operator==(const GraphKey& o) const {
      return X0 == o.X0 && dJN == o.dJN && XN == o.XN && dJ == o.dJ && th == o.th && J == o.J && nsteps == o.nsteps;
    }
  };
  // Record one gradient into a graph: the launches go to a private capture stream (the
  // caller's stream may be the legacy null stream, which cannot be captured); the
  // auxiliary stream joins the capture through the events of the reverse sweep.
  hipGraphExec_t capture_gradient(const double* X0, int nsteps, const double* dJdXN, double* XN, double* dJdX0,
                                  double* dJdtheta, double* J) {
    if (!cap_) SPS_HIP(hipStreamCreateWithFlags(&cap_, hipStreamNonBlocking));
    hipStream_t user = stream;
    stream = cap_;
    capturing_ = true;
    hipGraph_t graph = nullptr;
    SPS_HIP(hipStreamBeginCapture(cap_, hipStreamCaptureModeThreadLocal));
    try {
      gradient_launches(X0, nsteps, dJdXN, XN, dJdX0, dJdtheta, J);
    } catch (...) {
      (void)hipStreamEndCapture(cap_, &graph);
      if (graph) (void)hipGraphDestroy(graph);
      stream = user;
      capturing_ = false;
      throw;
    }
    const hipError_t e = hipStreamEndCapture(cap_, &graph);
    stream = user;
    capturing_ = false;
    SPS_HIP(e);
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    SPS_HIP(ei);
    return exec;
  }
  void drop_graphs() {
    if (!graphs_.empty()) (void)hipStreamSynchronize(stream);
    for (auto& g : graphs_) (void)hipGraphExecDestroy(g.second);
    graphs_.clear();
  }

  // a non-stage launch of the forward kernel (grid fields, F, a solve)
  void launch_kf(int mode, const cplx* X0, cplx* Xout, cplx* zg) { launch_kf_on(stream, mode, X0, Xout, zg); }
  void launch_kf_on(hipStream_t s, int mode, const cplx* X0, cplx* Xout, cplx* zg) {
    KfArgs a = kf_args(mode);
    a.X0 = X0;
    a.Xout = Xout;
    a.zg = zg;
    launch_kf_args(s, a);
  }
  KfArgs kf_args(int mode) const {
    KfArgs a{};
    a.Xst = Xst_;
    a.Fst = Fst_;
    a.nl = nl_;
    a.sstr = st();
    a.fstr = (size_t)B_ * K_ * 3 * N_;
    a.dt = cur_dt_;
    a.nst = tab_.s;
    a.mode = mode;
    return a;
  }
  // stage i (1 .. s) of a step from X: the stage's state goes to its slot of Xst_ (i < s) or
  // back into X (i = s, the new state); zg: where its grid fields go (nullable); save: a second
  // copy of its state (nullable)
  void launch_stage(hipStream_t s, int i, cplx* X, cplx* zg, cplx* save) {
    KfArgs a = kf_args(KF_STAGE);
    a.X0 = X;
    a.Xout = (i < tab_.s) ? Xst_ + (size_t)(i - 1) * st() : X;
    a.zg = zg;
    a.Xsave = save;
    a.stage = i;
    for (int j = 0; j < i; ++j) {
      a.fa[j] = tab_.A[i][j];
      a.lh[j] = tab_.H[i][j];
      a.asum += tab_.A[i][j];
      if (tab_.H[i][j] != 0.0) a.lx = 1;
    }
    a.fself = tab_.A[i][i - 1];
    launch_kf_args(s, a);
  }
  // stage launches on the caller's stream are timed (on the auxiliary stream a launch may share
  // the chip with the adjoint sweep)
  void launch_kf_args(hipStream_t s, const KfArgs& a) {
    hipEvent_t e0, e1;
    if (a.mode == KF_STAGE && timed(0, s, &e0, &e1))
      hipExtLaunchKernelGGL(kfwd_fn(), dim3(K_, B_), dim3(NTK), kf_lds(), s, e0, e1, 0, dv_, a);
    else
      hipLaunchKernelGGL(kfwd_fn(), dim3(K_, B_), dim3(NTK), kf_lds(), s, dv_, a);
    SPS_CHECK_LAUNCH();
  }
  void launch_xf(const cplx* zg, hipStream_t s = nullptr) {
    if (planes_) {
      planes_->forward(zg, nl_, s ? s : stream);
      return;
    }
    launch_xf_rows(zg, nl_, s ? s : stream);
  }
  // the grid-row forward kernel: one wave per FFT where the row length is 64 R1 (R1 = 3, 6)
  void launch_xf_rows(const cplx* zg, cplx* nl, hipStream_t s) {
    XfArgs a{zg, nl};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const bool t = timed(2, s, &e0, &e1);
    const dim3 g(Ngz_, B_);
    if (wave_r1_ == 6) hipExtLaunchKernelGGL(rbc_xfwd_w<6>, g, dim3(256), xfw_lds(), s, t ? e0 : nullptr, t ? e1 : nullptr, 0, dv_, a);
    else if (wave_r1_ == 3) hipExtLaunchKernelGGL(rbc_xfwd_w<3>, g, dim3(256), xfw_lds(), s, t ? e0 : nullptr, t ? e1 : nullptr, 0, dv_, a);
    else hipExtLaunchKernelGGL(rbc_xfwd, g, dim3(NTX), xf_lds(), s, t ? e0 : nullptr, t ? e1 : nullptr, 0, dv_, a);
    SPS_CHECK_LAUNCH();
  }
  size_t xfw_lds() const { return sizeof(cplx) * (3 * Ngx_ + 4 * wave_sc()); }
  size_t xaw_lds() const { return sizeof(cplx) * (5 * Ngx_ + 6 * wave_sc()); }
  int wave_sc() const { return wave_r1_ == 6 ? WaveRow<6>::SC : WaveRow<3>::SC; }
  // adjoint kernel arguments; stage m (1 .. s) for the stage reverses KA_A (m = s) and KA_B
  KaArgs ka_args(int flags, int m = 0) {
    KaArgs a{};
    a.zbar = zbar_;
    a.acc = acc_;
    a.Ybuf = Ybuf_;
    a.nlbar = nlbar_;
    a.sstr = st();
    a.dt = cur_dt_;
    a.stage = m;
    a.nst = tab_.s;
    if (m >= 1) {
      for (int j = m + 1; j <= tab_.s; ++j) {
        a.hc[j] = tab_.H[j][m];
        a.fc[j] = tab_.A[j][m - 1];
      }
      a.hself = tab_.H[m][m];
      a.fself = tab_.A[m][m - 1];
    }
    a.flags = flags;
    return a;
  }
  void launch_ka(const KaArgs& a) {
    hipEvent_t e0, e1;
    if ((a.flags & (KA_A | KA_B)) && !(a.flags & KA_SOLVE_T) && timed(1, stream, &e0, &e1))
      hipExtLaunchKernelGGL(kadj_fn(), dim3(K_, B_), dim3(NTK), ka_lds(), stream, e0, e1, 0, dv_, a);
    else
      hipLaunchKernelGGL(kadj_fn(), dim3(K_, B_), dim3(NTK), ka_lds(), stream, dv_, a);
    SPS_CHECK_LAUNCH();
  }
  void launch_xa(const cplx* zg) {
    if (planes_) {
      planes_->vjp(nlbar_, zg, zbar_, stream);
      return;
    }
    XaArgs a{nlbar_, zg, zbar_};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const bool t = timed(3, stream, &e0, &e1);
    if (!t) e0 = e1 = nullptr;
    const dim3 g(Ngz_, B_);
    if (wave_r1_ == 6) hipExtLaunchKernelGGL(rbc_xadj_w<6>, g, dim3(384), xaw_lds(), stream, e0, e1, 0, dv_, a);
    else if (wave_r1_ == 3) hipExtLaunchKernelGGL(rbc_xadj_w<3>, g, dim3(384), xaw_lds(), stream, e0, e1, 0, dv_, a);
    else hipExtLaunchKernelGGL(rbc_xadj, g, dim3(NTX), xa_lds(), stream, e0, e1, 0, dv_, a);
    SPS_CHECK_LAUNCH();
  }

  // segment store: two buffers of z-grid fields (step s, stage q < s_stages: the fields of the
  // states F is evaluated at), used by alternate segments
  cplx* slot(int buf, int s, int stage) {
    return seg_ + (((size_t)buf * seglen_ + s) * tab_.s + stage) * zsize_;
  }
  cplx* ckpt(int c) { return ckpt_ + (size_t)c * st(); }

  // One IMEX RK step from X (in place) on stream st.  z(q), q < s: the x-spectral z-grid fields
  // of stage q's state (z(0): those of X, given; the stages write the others); zout: where the
  // new state's fields go (or null).  sv(q) (nullable): where stage q+1's state is also stored
  // (the parameter gradient's records; sv(s-1) is the new state).
  template <class ZF, class SF>
  void rk_step(hipStream_t st, cplx* X, ZF z, cplx* zout, SF sv) {
    const int s = tab_.s;
    for (int i = 1; i <= s; ++i) {
      launch_xf(z(i - 1), st);
      launch_stage(st, i, X, (i < s) ? z(i) : zout, sv(i - 1));
    }
  }
  static cplx* no_save(int) { return nullptr; }
  // state records of the parameter gradient: two buffers of the s stage states per step
  cplx* sslot(int buf, int s, int q) { return sst_ + (((size_t)buf * seglen_ + s) * tab_.s + q) * K_ * S_; }

  // The adjoint launches of one step: its stages in reverse, each followed by the grid-row
  // adjoint of the F it differentiates.  z(q): the fields of stage q's state recorded by the
  // step's forward run; sv(q): stage q+1's state (parameter gradient only).  `first`: no step
  // has been reversed yet in this sweep (Xbar is the cotangent of the step's new state);
  // otherwise the stage-s kernel first completes the later step's initial-state cotangent.
  template <class ZF, class SF>
  void reverse_step(cplx* Xbar, bool& first, ZF z, SF sv) {
    const int s = tab_.s;
    for (int m = s; m >= 1; --m) {
      KaArgs a = ka_args(m == s ? (first ? KA_A : (KA_C | KA_A)) : KA_B, m);
      if (m == s) a.Xb_in = Xbar;
      if (param_on_) {
        a.Xm = sv(m - 1);
        a.pacc = pacc_;
      }
      launch_ka(a);
      first = false;
      launch_xa(z(m - 1));
    }
  }

  void forward(cplx* X, int nsteps) {
    if (ckpt_mode_ == SPS_CKPT_BINOMIAL) {
      forward_binomial(X, nsteps);
      return;
    }
    if (ckpt_mode_ == SPS_CKPT_TWO_LEVEL) {
      forward_two_level(X, nsteps);
      return;
    }
    const int ce = desc_.checkpoint_every;
    const int nseg = (nsteps + ce - 1) / ce;
    const int last0 = (nseg - 1) * ce;   // first step of the last segment: recorded now
    const int lb = (nseg - 1) & 1;
    // fields of step n, stage q: a single rolling buffer (kernels are stream ordered) or,
    // inside the last segment, the segment store read back by the reverse sweep
    auto zpos = [&](int n, int q) { return (n >= last0) ? slot(lb, n - last0, q) : zgA_; };
    auto spos = [&](int n, int q) { return (param_on_ && n >= last0) ? sslot(lb, n - last0, q) : nullptr; };
    launch_kf(KF_ZGRID, X, nullptr, zpos(0, 0));
    for (int n = 0; n < nsteps; ++n) {
      if (n % ce == 0) SPS_HIP(hipMemcpyAsync(ckpt(n / ce), X, sizeof(cplx) * st(), hipMemcpyDeviceToDevice, stream));
      step_setup(n);
      rk_step(stream, X, [&](int q) { return zpos(n, q); }, (n + 1 < nsteps) ? zpos(n + 1, 0) : nullptr,
              [&](int q) { return spos(n, q); });
    }
    tape_steps_ = nsteps;
    last_seg_ok_ = true;
  }

  // re-run segment seg from its checkpoint on stream s into segment buffer seg & 1
  void recompute(int seg, int len, hipStream_t s) {
    const int b = seg & 1;
    SPS_HIP(hipMemcpyAsync(Xw_, ckpt(seg), sizeof(cplx) * st(), hipMemcpyDeviceToDevice, s));
    launch_kf_on(s, KF_ZGRID, Xw_, nullptr, slot(b, 0, 0));
    for (int j = 0; j < len; ++j) {
      step_setup(seg * desc_.checkpoint_every + j);
      rk_step(s, Xw_, [&](int q) { return slot(b, j, q); }, (j + 1 < len) ? slot(b, j + 1, 0) : nullptr,
              [&](int q) { return param_on_ ? sslot(b, j, q) : nullptr; });
    }
  }

  // Reverse sweep.  The recompute of segment seg-1 (auxiliary stream, scratch Xst_, Xw_, nl_, Fst_,
  // segment buffer (seg-1)&1) overlaps the adjoint of segment seg (caller's stream, scratch
  // acc_, Ybuf_, nlbar_, zbar_, segment buffer seg&1).  Events order (i) every recompute after
  // the forward sweep, (ii) the adjoint of seg after its recompute, (iii) the recompute into a
  // buffer after the adjoint that last read it; the caller's stream waits for all of it.
  void reverse(cplx* Xbar, int nsteps) {
    if (ckpt_mode_ == SPS_CKPT_BINOMIAL) {
      reverse_binomial(Xbar, nsteps);
      return;
    }
    if (ckpt_mode_ == SPS_CKPT_TWO_LEVEL) {
      reverse_two_level(Xbar, nsteps);
      return;
    }
    const int ce = desc_.checkpoint_every;
    const int nseg = (nsteps + ce - 1) / ce;
    auto seglen = [&](int g) { return std::min(ce, nsteps - g * ce); };
    hipEvent_t ev_fwd = ev_[0], ev_rec = ev_[1], ev_adj = ev_[2];
    // A second reverse sweep of the same run: with three or more segments the previous sweep's
    // recompute of segment nseg-3 overwrote the buffer that held the last segment's stage
    // fields (both use buffer (nseg-1)&1), so the last segment is recomputed first.
    if (!last_seg_ok_) recompute(nseg - 1, seglen(nseg - 1), stream);
    if (param_on_) {
      hipLaunchKernelGGL(fill_zero, dim3((2 * K_ + NT - 1) / NT), dim3(NT), 0, stream, pacc_, 2 * K_);
      SPS_CHECK_LAUNCH();
    }
    SPS_HIP(hipEventRecord(ev_fwd, stream));
    SPS_HIP(hipStreamWaitEvent(aux_, ev_fwd, 0));
    bool first = true;
    for (int seg = nseg - 1; seg >= 0; --seg) {
      const int len = seglen(seg), b = seg & 1;
      if (seg != nseg - 1) SPS_HIP(hipStreamWaitEvent(stream, ev_rec, 0));
      if (seg >= 1) {
        if (seg != nseg - 1) SPS_HIP(hipStreamWaitEvent(aux_, ev_adj, 0));
        recompute(seg - 1, seglen(seg - 1), aux_);
        SPS_HIP(hipEventRecord(ev_rec, aux_));
      }
      for (int j = len - 1; j >= 0; --j) {
        step_setup(seg * ce + j);
        reverse_step(Xbar, first, [&](int q) { return slot(b, j, q); }, [&](int q) { return sslot(b, j, q); });
      }
      SPS_HIP(hipEventRecord(ev_adj, stream));
    }
    last_seg_ok_ = nseg < 3;
    KaArgs a = ka_args(KA_C);
    a.Xb_out = Xbar;
    launch_ka(a);
    if (param_on_) {
      // dJ/dRa and dJ/dPr from dJ/dnu and dJ/dkappa: nu = (Ra/Pr)^(-1/2), kappa = (Ra Pr)^(-1/2)
      const double Ra = desc_.param0, Pr = desc_.param1;
      hipLaunchKernelGGL(rbc_param_finish, dim3(1), dim3(64), 0, stream, pacc_, K_, -0.5 * nu_ / Ra,
                         -0.5 * ka_ / Ra, 0.5 * nu_ / Pr, -0.5 * ka_ / Pr, theta_out_);
      SPS_CHECK_LAUNCH();
    }
    // join the auxiliary stream explicitly (it may have waited without launching, nseg = 1)
    SPS_HIP(hipEventRecord(ev_rec, aux_));
    SPS_HIP(hipStreamWaitEvent(stream, ev_rec, 0));
  }

  // ----------------------------------------------------------------- binomial checkpointing
  // The schedule's actions on a working state (the caller's X in the forward sweep, Xw_ in the
  // reverse sweep) and rv_slots_ stored states, all on the problem's stream.  A turn records the
  // step's two stage-field sets in the first segment slot and runs the step's adjoint launches,
  // exactly those of the segment sweep.
  void set_checkpointing(int scheme, int slots) override {
    if (scheme != SPS_CKPT_UNIFORM) no_batch("this checkpoint schedule");
    SPS_REQUIRE(scheme == SPS_CKPT_UNIFORM || scheme == SPS_CKPT_BINOMIAL || scheme == SPS_CKPT_TWO_LEVEL,
                "unknown checkpointing scheme");
    if (scheme != SPS_CKPT_UNIFORM) {
      SPS_REQUIRE(slots >= 1 && slots <= desc_.max_steps + 1, "slots must be in [1, max_steps + 1]");
      if (slots > rv_cap_) {
        rv_ = arena_.alloc<cplx>((size_t)slots * K_ * S_);
        rv_cap_ = slots;
      }
    }
    if (scheme == SPS_CKPT_TWO_LEVEL) {
      if (ckfd_ < 0) alloc_host_ckpt();
      if (!Xs_) Xs_ = arena_.alloc<cplx>((size_t)K_ * S_);
    }
    drop_graphs();
    ckpt_mode_ = scheme;
    rv_slots_ = (scheme == SPS_CKPT_UNIFORM) ? 0 : slots;
    sched_.clear();
    tape_steps_ = -1;
  }
  cplx* rvslot(int i) { return rv_ + (size_t)i * K_ * S_; }
  // binomial schedule (forward and reverse actions) for a run of n steps with rv_slots_ slots
  const std::pair<std::vector<CkptAction>, std::vector<CkptAction>>& schedule(int n) {
    auto it = sched_.find(n);
    if (it == sched_.end()) {
      std::pair<std::vector<CkptAction>, std::vector<CkptAction>> v;
      binomial_schedule(n, rv_slots_, v.first, v.second);
      it = sched_.emplace(n, std::move(v)).first;
    }
    return it->second;
  }
  void copy_state(cplx* dst, const cplx* src) {
    SPS_HIP(hipMemcpyAsync(dst, src, sizeof(cplx) * K_ * S_, hipMemcpyDefault, stream));
  }
  void advance(cplx* X, int a, int b) {
    launch_kf(KF_ZGRID, X, nullptr, zgA_);
    for (int n = a; n < b; ++n) {
      step_setup(n);
      rk_step(stream, X, [&](int) { return zgA_; }, (n + 1 < b) ? zgA_ : nullptr, no_save);
    }
  }
  // forward actions of a schedule on the working state X (stored states in the slots); with
  // to_end false, the advance past the last stored state (to the run's final state) is skipped
  void run_forward_actions(cplx* X, const std::vector<CkptAction>& acts, bool to_end = true) {
    size_t last = acts.size();
    if (!to_end)
      while (last > 0 && acts[last - 1].op != CK_TAKESHOT) --last;
    for (size_t i = 0; i < last; ++i) {
      const CkptAction& c = acts[i];
      if (c.op == CK_TAKESHOT) copy_state(rvslot(c.a), X);
      else if (c.op == CK_ADVANCE) advance(X, c.a, c.b);
    }
  }
  // reverse actions on the working state Xw_; `first`: no reverse step has run yet in this sweep
  void run_reverse_actions(cplx* Xbar, const std::vector<CkptAction>& acts, bool& first) {
    for (const CkptAction& c : acts) {
      switch (c.op) {
        case CK_RESTORE: copy_state(Xw_, rvslot(c.a)); break;
        case CK_TAKESHOT: copy_state(rvslot(c.a), Xw_); break;
        case CK_ADVANCE: advance(Xw_, c.a, c.b); break;
        case CK_YOUTURN: {
          auto z = [&](int q) { return slot(0, 0, q); };
          launch_kf(KF_ZGRID, Xw_, nullptr, slot(0, 0, 0));
          step_setup(c.a);
          rk_step(stream, Xw_, z, nullptr, no_save);
          reverse_step(Xbar, first, z, no_save);
          break;
        }
        default: throw Error(SPS_E_STATE, "bad checkpoint action");
      }
    }
  }
  void finish_reverse(cplx* Xbar) {
    KaArgs a = ka_args(KA_C);
    a.Xb_out = Xbar;
    launch_ka(a);
  }
  void forward_binomial(cplx* X, int nsteps) {
    run_forward_actions(X, schedule(nsteps).first);
    tape_steps_ = nsteps;
  }
  void reverse_binomial(cplx* Xbar, int nsteps) {
    bool first = true;
    run_reverse_actions(Xbar, schedule(nsteps).second, first);
    finish_reverse(Xbar);
    tape_steps_ = -1;   // the reverse sweep reused the snapshot slots: the run is reversed once
  }
  // Two levels: the state at the start of every segment of checkpoint_every steps goes to
  // pinned host memory during the forward sweep; the reverse sweep brings the segments back
  // from the last, and reverses each with the binomial schedule of its length on the device
  // slots (the segment's own forward actions first, then its turns).
  int seg_len(int g, int nsteps) const { return std::min(desc_.checkpoint_every, nsteps - g * desc_.checkpoint_every); }
  // Nested schedule (outer slots fewer than the segments): the segment starts are placed by the
  // binomial schedule over segments on the outer slots; each outer turn reverses its segment
  // with the binomial schedule of the segment on the device slots.
  bool nested(int nseg) const { return outer_slots_ > 0 && outer_slots_ < nseg; }
  int seg_start(int g, int nsteps) const { return std::min(g * desc_.checkpoint_every, nsteps); }
  const std::pair<std::vector<CkptAction>, std::vector<CkptAction>>& outer_schedule(int nseg) {
    auto it = osched_.find(nseg);
    if (it == osched_.end()) {
      std::pair<std::vector<CkptAction>, std::vector<CkptAction>> sc;
      // (a segment's advance costs checkpoint_every forward steps; the outer costs are in steps)
      if (outer_wr_ >= 0.0) {
        // (the search takes nseg^2 min(slots, nseg) steps)
        SPS_REQUIRE((double)nseg * nseg * std::min(outer_slots_, nseg) <= 2e10,
                    "too many segments for the outer cost search");
        cost_schedule(nseg, outer_slots_, (double)desc_.checkpoint_every, outer_wr_, outer_rd_, sc.first, sc.second);
      } else {
        binomial_schedule(nseg, outer_slots_, sc.first, sc.second);
      }
      it = osched_.emplace(nseg, std::move(sc)).first;
    }
    return it->second;
  }
  // outer slot i <-> device state (host memory: stream-ordered copies; file: staged through
  // buffer 0 with the stream synchronized around each file access)
  void outer_store(int i, const cplx* src) {
    if (ckfd_ < 0) {
      copy_state(host_ckpt_.get() + (size_t)i * K_ * S_, src);
      return;
    }
    copy_state(ckstage_.get(), src);
    SPS_HIP(hipStreamSynchronize(stream));
    file_io(true, 0, i);
  }
  void outer_load(int i, cplx* dst) {
    if (ckfd_ < 0) {
      copy_state(dst, host_ckpt_.get() + (size_t)i * K_ * S_);
      return;
    }
    SPS_HIP(hipStreamSynchronize(stream));   // staging buffer 0 free
    file_io(false, 0, i);
    copy_state(dst, ckstage_.get());
  }
  void forward_nested(cplx* X, int nsteps, int nseg) {
    for (const CkptAction& c : outer_schedule(nseg).first) {
      if (c.op == CK_TAKESHOT) outer_store(c.a, X);
      else if (c.op == CK_ADVANCE) advance(X, seg_start(c.a, nsteps), seg_start(c.b, nsteps));
    }
    if (ckfd_ >= 0) SPS_HIP(hipStreamSynchronize(stream));
  }
  void reverse_nested(cplx* Xbar, int nsteps, int nseg) {
    if (!Xo_) Xo_ = arena_.alloc<cplx>((size_t)K_ * S_);
    bool first = true;
    for (const CkptAction& c : outer_schedule(nseg).second) {
      switch (c.op) {
        case CK_RESTORE: outer_load(c.a, Xo_); break;
        case CK_TAKESHOT: outer_store(c.a, Xo_); break;
        case CK_ADVANCE: advance(Xo_, seg_start(c.a, nsteps), seg_start(c.b, nsteps)); break;
        case CK_YOUTURN: {
          // the working state holds the start of segment c.a; the schedule restores before
          // it uses the working state again
          const auto& sc = schedule(seg_len(c.a, nsteps));
          copy_state(Xs_, Xo_);
          step_base_ = seg_start(c.a, nsteps);   // the segment's schedule counts its own steps
          run_forward_actions(Xs_, sc.first, false);
          run_reverse_actions(Xbar, sc.second, first);
          step_base_ = 0;
          break;
        }
        default: throw Error(SPS_E_STATE, "bad checkpoint action");
      }
    }
    finish_reverse(Xbar);
    tape_steps_ = -1;   // the outer slots were reused: the run is reversed once
  }

  void forward_two_level(cplx* X, int nsteps) {
    const int ce = desc_.checkpoint_every, nseg = (nsteps + ce - 1) / ce;
    if (nested(nseg)) {
      forward_nested(X, nsteps, nseg);
    } else if (ckfd_ >= 0) {
      forward_disk(X, nsteps, nseg);
    } else {
      for (int g = 0; g < nseg; ++g) {
        copy_state(host_ckpt_.get() + (size_t)g * K_ * S_, X);
        step_base_ = g * ce;
        advance(X, 0, seg_len(g, nsteps));
      }
      step_base_ = 0;
    }
    tape_steps_ = nsteps;
  }
  void reverse_two_level(cplx* Xbar, int nsteps) {
    const int ce = desc_.checkpoint_every, nseg = (nsteps + ce - 1) / ce;
    if (nested(nseg)) {
      reverse_nested(Xbar, nsteps, nseg);
      return;
    }
    bool first = true;
    // disk level: a host-to-device copy from staging buffer b may be in flight (also from an
    // earlier reverse sweep of the same run; waiting on an event never recorded returns at once)
    int pend[2] = {1, 1};
    for (int g = nseg - 1; g >= 0; --g) {
      const auto& sc = schedule(seg_len(g, nsteps));
      if (ckfd_ >= 0) {
        const int b = g & 1;
        if (pend[b]) SPS_HIP(hipEventSynchronize(ckev_[b]));
        file_io(false, b, g);
        copy_state(Xs_, ckstage_.get() + (size_t)b * K_ * S_);
        SPS_HIP(hipEventRecord(ckev_[b], stream));
        pend[b] = 1;
      } else {
        copy_state(Xs_, host_ckpt_.get() + (size_t)g * K_ * S_);
      }
      step_base_ = g * ce;
      run_forward_actions(Xs_, sc.first, false);
      run_reverse_actions(Xbar, sc.second, first);
      step_base_ = 0;
    }
    finish_reverse(Xbar);
  }
  // Disk level: segment starts staged through two pinned buffers; the write of segment g's
  // start waits for its device-to-host copy (an event) while later segments run.
  void forward_disk(cplx* X, int nsteps, int nseg) {
    int pend[2] = {-1, -1};
    auto flush = [&](int b) {
      if (pend[b] < 0) return;
      SPS_HIP(hipEventSynchronize(ckev_[b]));
      file_io(true, b, pend[b]);
      pend[b] = -1;
    };
    for (int g = 0; g < nseg; ++g) {
      const int b = g & 1;
      flush(b);
      copy_state(ckstage_.get() + (size_t)b * K_ * S_, X);
      SPS_HIP(hipEventRecord(ckev_[b], stream));
      pend[b] = g;
      step_base_ = g * desc_.checkpoint_every;
      advance(X, 0, seg_len(g, nsteps));
    }
    step_base_ = 0;
    flush(0);
    flush(1);
  }
  void file_io(bool write, int b, int g) {
    const size_t bytes = sizeof(cplx) * K_ * S_;
    char* p = reinterpret_cast<char*>(ckstage_.get() + (size_t)b * K_ * S_);
    const off_t off = (off_t)g * (off_t)bytes;
    size_t done = 0;
    while (done < bytes) {
      const ssize_t r = write ? pwrite(ckfd_, p + done, bytes - done, off + (off_t)done)
                              : pread(ckfd_, p + done, bytes - done, off + (off_t)done);
      if (r <= 0) throw Error(SPS_E_IO, write ? "checkpoint file write failed" : "checkpoint file read failed");
      done += (size_t)r;
    }
  }
  // pinned host states of the outer level: one per segment of the longest run, or the outer
  // slot count when that is smaller
  void alloc_host_ckpt() {
    const int nseg = (desc_.max_steps + desc_.checkpoint_every - 1) / desc_.checkpoint_every;
    const int need = outer_slots_ > 0 ? std::min(outer_slots_, nseg) : nseg;
    if (host_ckpt_ && host_cap_ >= need) return;
    if (host_ckpt_) SPS_HIP(hipStreamSynchronize(stream));
    host_ckpt_.reset();
    void* p = nullptr;
    SPS_HIP(hipHostMalloc(&p, sizeof(cplx) * K_ * S_ * (size_t)need, hipHostMallocDefault));
    host_ckpt_.reset(reinterpret_cast<cplx*>(p));
    host_cap_ = need;
  }
  void close_ckpt_file() {
    if (ckfd_ < 0) return;
    (void)hipStreamSynchronize(stream);
    (void)close(ckfd_);
    (void)unlink(ckpath_.c_str());
    ckfd_ = -1;
    ckpath_.clear();
  }

 public:
  void set_checkpoint_file(const char* path) override {
    no_batch("the disk checkpoint level");
    drop_graphs();
    SPS_HIP(hipStreamSynchronize(stream));   // copies into the host level may be in flight
    close_ckpt_file();
    tape_steps_ = -1;
    if (!path) {
      if (ckpt_mode_ == SPS_CKPT_TWO_LEVEL) alloc_host_ckpt();
      return;
    }
    SPS_REQUIRE(path[0] != '\0', "empty checkpoint file path");
    const int fd = open(path, O_RDWR | O_CREAT | O_TRUNC, 0600);
    if (fd < 0) throw Error(SPS_E_IO, std::string("cannot create the checkpoint file ") + path);
    ckfd_ = fd;
    ckpath_ = path;
    if (!ckstage_) {
      void* p = nullptr;
      SPS_HIP(hipHostMalloc(&p, sizeof(cplx) * K_ * S_ * 2, hipHostMallocDefault));
      ckstage_.reset(reinterpret_cast<cplx*>(p));
      for (auto& e : ckev_) SPS_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    }
    host_ckpt_.reset();
    host_cap_ = 0;
  }
  void set_outer_slots(int slots) override {
    no_batch("the nested checkpoint schedule");
    SPS_REQUIRE(slots >= 0, "outer slots must be >= 0");
    drop_graphs();
    SPS_HIP(hipStreamSynchronize(stream));
    outer_slots_ = slots;
    osched_.clear();
    tape_steps_ = -1;
    if (ckpt_mode_ == SPS_CKPT_TWO_LEVEL && ckfd_ < 0) alloc_host_ckpt();
  }
  void set_outer_costs(double write_cost, double read_cost) override {
    no_batch("the nested checkpoint schedule");
    const bool off = write_cost < 0.0 && read_cost < 0.0;
    SPS_REQUIRE(off || (write_cost >= 0.0 && read_cost >= 0.0 && std::isfinite(write_cost + read_cost)),
                "outer costs: both >= 0 and finite, or both negative");
    drop_graphs();
    SPS_HIP(hipStreamSynchronize(stream));
    outer_wr_ = off ? -1.0 : write_cost;
    outer_rd_ = off ? -1.0 : read_cost;
    osched_.clear();
    tape_steps_ = -1;
  }

 private:

  // ----------------------------------------------------------------- tables
  void build_tables() {
    const int N = N_, K = K_, Ngz = Ngz_, Nz1 = desc_.nz;
    // cos(pi m / (2 Ng)), m < 4 Ng, in extended precision
    auto costab = [](int Ng) {
      std::vector<double> c(4 * Ng);
      for (int m = 0; m < 4 * Ng; ++m)
        c[m] = (double)cosl((long double)m * 3.14159265358979323846264338327950288L / (2.0L * Ng));
      return c;
    };
    std::vector<double> gram((size_t)N * N);
    auto I = [](int j) { return (j % 2 == 0) ? 2.0 / (1.0 - (double)j * j) : 0.0; };
    for (int m = 0; m < N; ++m)
      for (int n = 0; n < N; ++n) gram[(size_t)m * N + n] = 0.25 * (I(m + n) + I(std::abs(m - n)));
    dv_.K = K;
    dv_.N = N;
    dv_.S = S_;
    dv_.Ngx = Ngx_;
    dv_.Ngz = Ngz;
    dv_.Nx1 = desc_.nx;
    dv_.Nz1 = Nz1;
    dv_.Lx = desc_.lx;
    dv_.nu = nu_;
    dv_.ka = ka_;
    dv_.kx = arena_.upload(kxs_, stream);
    dv_.cp = cp_;
    dv_.bc0 = bc0_;
    dv_.cost_scale = cost_scale_;
    dv_.Kz = Kz_;
    dv_.ncost = ncost_;
    dv_.ckeep = ckeep_.empty() ? nullptr : arena_.upload(ckeep_, stream);
    dv_.cosz = arena_.upload(costab(Ngz), stream);
    dv_.cosz1 = arena_.upload(costab(Nz1), stream);
    dv_.twx = arena_.upload(twiddles(Ngx_), stream);
    dv_.twx1 = arena_.upload(twiddles(desc_.nx), stream);
    dv_.gram = arena_.upload(gram, stream);
  }

  void build_bands() {
    RbcHostBands hb;
    host_bands(N_, kxs_, nu_, ka_, cp_, hb);
    kl_ = hb.kl;
    ku_ = hb.ku;
    if (!rab_.empty()) {
      // a batch: L = L0 + nu Lnu + kappa Lka on the common band, per-instance nu and kappa
      RbcHostBands h0, hn, hk;
      host_bands(N_, kxs_, 0.0, 0.0, cp_, h0, 0.0, kl_, ku_);
      host_bands(N_, kxs_, 1.0, 0.0, cp_, hn, 0.0, kl_, ku_);
      host_bands(N_, kxs_, 0.0, 1.0, cp_, hk, 0.0, kl_, ku_);
      for (size_t e = 0; e < hn.BL.size(); ++e) {
        hn.BL[e] -= h0.BL[e];
        hk.BL[e] -= h0.BL[e];
      }
      hb.BL = h0.BL;
      BLnu_ = arena_.upload(hn.BL, stream);
      BLka_ = arena_.upload(hk.BL, stream);
      blnu_h_ = hn.BL;
      blka_h_ = hk.BL;
      std::vector<double> nub(B_), kab(B_);
      for (int b = 0; b < B_; ++b) {
        nub[b] = std::pow(rab_[b] / desc_.param1, -0.5);
        kab[b] = std::pow(rab_[b] * desc_.param1, -0.5);
      }
      dv_.nub = arena_.upload(nub, stream);
      dv_.kab = arena_.upload(kab, stream);
    }
    SPS_REQUIRE(kl_ + SPS_BLK <= SPS_TW && SPS_BLK + kl_ + ku_ <= SPS_GW, "band too wide for the block solver");
    SPS_REQUIRE(N_ <= SPS_WAVE, "nz too large for the stage kernels");
    SPS_REQUIRE(S_ + SPS_PAD <= NTK && 4 * N_ + 28 <= NTK && 4 * Ngz_ <= NTK && 6 * half_nodes(Ngz_) <= NTK,
                "nz too large for one state entry per thread");
    BM_ = arena_.upload(hb.BM, stream);
    BL_ = arena_.upload(hb.BL, stream);
    plan_partition(hb);
    dv_.n = S_;
    dv_.kl = kl_;
    dv_.ku = ku_;
    dv_.uw = kl_ + ku_ + 1;
    dv_.rowmap = arena_.upload(hb.rowmap, stream);
    dv_.colmap = arena_.upload(hb.colmap, stream);
    dv_.rowph = arena_.upload(hb.rowph, stream);
    dv_.colph = arena_.upload(hb.colph, stream);
    dv_.rho = arena_.upload(hb.rho, stream);
    std::vector<int> gmap(S_), hmap(S_), sflag(S_);
    std::vector<double> hrho(S_, 0.0);
    for (int i = 0; i < S_; ++i) {
      const int r = hb.rowmap[i], c = hb.colmap[i];
      gmap[i] = r | (hb.rowph[r] ? (1 << 30) : 0);
      hmap[i] = c | (hb.colph[c] ? (1 << 30) : 0) | ((c >= 2 && hb.colph[c - 2]) ? (1 << 29) : 0);
      hrho[i] = (c >= 2) ? hb.rho[c - 2] : 0.0;
      sflag[i] = hb.colph[i];
    }
    SPS_REQUIRE(S_ < 0xffff, "nz too large for the per-thread maps");
    dv_.gmap = arena_.upload(gmap, stream);
    dv_.hmap = arena_.upload(hmap, stream);
    dv_.hrho = arena_.upload(hrho, stream);
    dv_.sflag = arena_.upload(sflag, stream);
  }

  // The staged path solves in P = 4, 3 or 2 partitions of whole 8-row blocks (spread as evenly
  // as possible), the most that the couplings allow: from the band pattern (over every
  // wavenumber and, for a batch, every part of L), rows of a partition may reach only the
  // neighbouring partitions, each interface's widths (cu: columns of the next partition that
  // rows above reach, cl: columns of the previous partition that rows below reach) at most 16,
  // a row's spike entries at most SPS_SPIKE_W and the coupled system at most SPS_RED_MAX
  // unknowns (and no more than S, its scratch).
  void plan_partition(const RbcHostBands& hb) {
    dv_.part = 0;
    if (stream_solve_) return;
    const int nblk = blk_count(S_), bw = kl_ + ku_ + 1;
    // the columns each row reaches
    std::vector<int> cmin(S_, S_), cmax(S_, -1);
    auto scan = [&](const std::vector<double>& band) {
      for (int k = 0; k < K_; ++k)
        for (int i = 0; i < S_; ++i)
          for (int q = 0; q < bw; ++q) {
            const int c = i + q - kl_;
            if (c < 0 || c >= S_ || band[((size_t)k * S_ + i) * bw + q] == 0.0) continue;
            cmin[i] = std::min(cmin[i], c);
            cmax[i] = std::max(cmax[i], c);
          }
    };
    scan(hb.BM);
    scan(hb.BL);
    if (!rab_.empty()) {   // the batch's nu and kappa parts of L (host copies)
      scan(blnu_h_);
      scan(blka_h_);
    }
    for (int P = SPS_MAXPART; P >= 2; --P) {
      if (nblk < 2 * P) continue;
      std::vector<int> st(P + 1, 0);
      for (int p = 0; p < P; ++p) st[p + 1] = st[p] + SPS_BLK * (nblk / P + (p < nblk % P ? 1 : 0));
      st[P] = S_;
      auto part_of = [&](int i) {
        int p = 0;
        while (p + 1 < P && i >= st[p + 1]) ++p;
        return p;
      };
      // interface q's widths for A (cu: columns of partition q + 1 that rows of q reach;
      // cl: columns of q that rows of q + 1 reach) and for A^T (cut: rows of q + 1 that reach
      // back into q; clt: rows of q that reach into q + 1)
      std::vector<int> cu(P - 1, 0), cl(P - 1, 0), cut(P - 1, 0), clt(P - 1, 0);
      bool ok = true;
      for (int i = 0; i < S_ && ok; ++i) {
        if (cmax[i] < 0) continue;
        const int pi = part_of(i), plo = part_of(cmin[i]), phi = part_of(cmax[i]);
        if (plo < pi - 1 || phi > pi + 1) ok = false;
        if (phi == pi + 1) {
          cu[pi] = std::max(cu[pi], cmax[i] - st[pi + 1] + 1);
          clt[pi] = std::max(clt[pi], st[pi + 1] - i);
        }
        if (plo == pi - 1) {
          cl[pi - 1] = std::max(cl[pi - 1], st[pi] - cmin[i]);
          cut[pi - 1] = std::max(cut[pi - 1], i - st[pi] + 1);
        }
      }
      if (!ok) continue;
      int nr0 = 0, nr1 = 0;
      for (int q = 0; q + 1 < P; ++q) {
        if (std::max({cu[q], cl[q], cut[q], clt[q]}) > 16) ok = false;
        nr0 += cu[q] + cl[q];
        nr1 += cut[q] + clt[q];
      }
      for (int p = 0; p < P; ++p) {
        const int w0 = (p + 1 < P ? cu[p] : 0) + (p > 0 ? cl[p - 1] : 0);
        const int w1 = (p + 1 < P ? cut[p] : 0) + (p > 0 ? clt[p - 1] : 0);
        if (std::max(w0, w1) > SPS_SPIKE_W || w0 == 0 || w1 == 0) ok = false;
      }
      const int nr = std::max(nr0, nr1);
      if (!ok || nr > SPS_RED_MAX || nr > S_) continue;
      // each direction's spikes (rounded to 4 doubles) and inverse must fit the space of the
      // early set of its solve (the T blocks for the forward solve, the G blocks for the
      // transposed one) and the copy's loads; offsets below 2^16
      int sz[2] = {0, 0};
      for (int p = 0; p < P; ++p) {
        const int np = st[p + 1] - st[p];
        sz[0] += np * ((p + 1 < P ? cu[p] : 0) + (p > 0 ? cl[p - 1] : 0));
        sz[1] += np * ((p + 1 < P ? cut[p] : 0) + (p > 0 ? clt[p - 1] : 0));
      }
      const int area0 = (sz[0] + 3) / 4 * 4 + nr0 * nr0, area1 = (sz[1] + 3) / 4 * 4 + nr1 * nr1;
      if (std::max(sz[0], sz[1]) >= 0xffff) continue;
      const int cap = SPS_CP_REG * 2 * (NTK - SPS_WAVE * P);
      if (area0 > blk_t_size(S_) || area1 > blk_g_size(S_) || area0 + 1 > cap || area1 + 1 > cap) continue;
      // accepted: descriptor fields and the tables of both directions
      dv_.part = P;
      dv_.ps1 = st[1];
      dv_.ps2 = P > 2 ? st[2] : S_;
      dv_.ps3 = P > 3 ? st[3] : S_;
      pmeta_h_.assign(8 * SPS_MAXPART + 6 * (SPS_MAXPART - 1), 0);
      smap_h_.assign(2 * (size_t)S_, int2{0, 0});
      for (int dir = 0; dir < 2; ++dir) {
        std::vector<int> la(P - 1), lc(P - 1), zo(P, 0);
        for (int q = 0; q + 1 < P; ++q) {
          la[q] = dir ? clt[q] : cl[q];   // last entries of partition q
          lc[q] = dir ? cut[q] : cu[q];   // first entries of partition q + 1
          zo[q + 1] = zo[q] + la[q] + lc[q];
          int* im = &pmeta_h_[8 * SPS_MAXPART + 6 * q + 3 * dir];
          im[0] = la[q];
          im[1] = lc[q];
          im[2] = zo[q];
        }
        int off = 0;
        for (int p = 0; p < P; ++p) {
          const int np = st[p + 1] - st[p];
          const int wV = (p + 1 < P) ? lc[p] : 0, wW = (p > 0) ? la[p - 1] : 0, w = wV + wW;
          const int zV = wV ? zo[p] + la[p] : 0, zW = wW ? zo[p - 1] : 0;
          int* pm = &pmeta_h_[8 * p];
          pm[0] = st[p];
          pm[1] = np;
          pm[2 + 3 * dir] = wV;
          pm[3 + 3 * dir] = wW;
          pm[4 + 3 * dir] = off;
          for (int i = st[p]; i < st[p + 1]; ++i)
            smap_h_[(size_t)dir * S_ + i] = int2{(off + (i - st[p])) | (np << 16), wV | (wW << 5) | (zV << 10) | (zW << 17)};
          off += np * w;
        }
        off = (off + 3) / 4 * 4;
        const int big = 1 << 20;
        dv_.rof[dir] = off;
        dv_.nrr[dir] = dir ? nr1 : nr0;
        dv_.zb1[dir] = P > 2 ? zo[1] : big;
        dv_.zb2[dir] = P > 3 ? zo[2] : big;
        dv_.rsh0[dir] = st[1] - la[0] - zo[0];
        dv_.rsh1[dir] = P > 2 ? st[2] - la[1] - zo[1] : 0;
        dv_.rsh2[dir] = P > 3 ? st[3] - la[2] - zo[2] : 0;
      }
      return;
    }
  }

  void alloc_work() {
    const size_t st = (size_t)B_ * K_ * S_;
    zsize_ = (size_t)B_ * 6 * Ngz_ * K_;
    // (partitions start at whole blocks: together they have the whole system's block count)
    dv_.tsz = blk_t_size(S_);
    dv_.blksz = dv_.opsize = blk_ops_size(S_);
    if (dv_.part) {
      dv_.spk[0] = dv_.blksz;
      dv_.spk[1] = dv_.spk[0] + (dv_.rof[0] + dv_.nrr[0] * dv_.nrr[0] + 3) / 4 * 4;
      dv_.opsize = (dv_.spk[1] + dv_.rof[1] + dv_.nrr[1] * dv_.nrr[1] + 3) / 4 * 4;
      dv_.smap = arena_.upload(smap_h_, stream);
      dv_.pmeta = arena_.upload(pmeta_h_, stream);
    }
    if (!stream_solve_) {
      // the staged solves: each thread's share of either set in registers, and the phase
      // buffers below the early set (the forward solve's is the T blocks, the transposed one's
      // the G blocks)
      const size_t gsz = dv_.blksz - dv_.tsz;
      SPS_REQUIRE((size_t)dv_.tsz <= 2 * SPS_OPS_REG_T * NTK && gsz <= 2 * SPS_OPS_REG_G * NTK,
                  "nz too large for the staged block solver");
      SPS_REQUIRE(kf_pre() <= sizeof(double) * gsz && ka_pre() <= sizeof(double) * dv_.tsz,
                  "stage buffers overlap the staged operators");
    }
    ops_ = arena_.alloc<double>((size_t)B_ * K_ * dv_.opsize);
    dv_.ops = ops_;
    err_ = arena_.alloc<int>(1);
    SPS_HIP(hipMemsetAsync(err_, 0, sizeof(int), stream));
    dv_.err = err_;
    const int ns = tab_.s;
    Xst_ = arena_.alloc<cplx>((size_t)(ns - 1) * st);
    Xw_ = arena_.alloc<cplx>(st);
    Xg_ = arena_.alloc<cplx>(st);
    acc_ = arena_.alloc<cplx>(st);
    Ybuf_ = arena_.alloc<cplx>((size_t)(ns - 1) * st);
    Fst_ = arena_.alloc<cplx>((size_t)(ns - 1) * B_ * K_ * 3 * N_);
    zgA_ = arena_.alloc<cplx>(zsize_);
    zbar_ = arena_.alloc<cplx>(zsize_);
    nl_ = arena_.alloc<cplx>((size_t)B_ * 3 * Ngz_ * K_);
    nlbar_ = arena_.alloc<cplx>((size_t)B_ * 3 * Ngz_ * K_);
    itmp_ = arena_.alloc<cplx>((size_t)B_ * desc_.nz * K_);
    Jpart_ = arena_.alloc<double>((size_t)B_ * K_);
    const int ce = desc_.checkpoint_every;
    const int nck = (desc_.max_steps + ce - 1) / ce;
    ckpt_ = arena_.alloc<cplx>((size_t)nck * st);
    seglen_ = std::min(ce, desc_.max_steps);
    seg_ = arena_.alloc<cplx>((size_t)2 * seglen_ * ns * zsize_);
    const size_t fac_lds = factor_lds();
    std::vector<std::pair<const void*, size_t>> lds = {
        {(const void*)kfwd_fn(), kf_lds()}, {(const void*)kadj_fn(), ka_lds()}, {(const void*)rbc_factor, fac_lds}};
    if (!cou_) {
      wave_r1_ = (Ngx_ == 384) ? 6 : (Ngx_ == 192 ? 3 : 0);
      if (wave_r1_ == 6) {
        lds.push_back({(const void*)rbc_xfwd_w<6>, xfw_lds()});
        lds.push_back({(const void*)rbc_xadj_w<6>, xaw_lds()});
      } else if (wave_r1_ == 3) {
        lds.push_back({(const void*)rbc_xfwd_w<3>, xfw_lds()});
        lds.push_back({(const void*)rbc_xadj_w<3>, xaw_lds()});
      } else {
        lds.push_back({(const void*)rbc_xfwd, xf_lds()});
        lds.push_back({(const void*)rbc_xadj, xa_lds()});
      }
    }
    for (const auto& fl : lds) {
      SPS_REQUIRE(fl.second <= 160 * 1024, "problem too large for LDS");
      SPS_HIP(hipFuncSetAttribute(fl.first, hipFuncAttributeMaxDynamicSharedMemorySize, (int)fl.second));
    }
    SPS_HIP(hipStreamSynchronize(stream));
  }

  sps_desc desc_;
  int K_, N_, S_, Ngx_, Ngz_, kl_ = 0, ku_ = 0;
  double nu_, ka_, dt_ = 0.0, cp_ = 1.0, bc0_ = 1.0, cost_scale_ = 1.0;
  int Kz_ = 1, ncost_ = 2;
  bool cou_ = false, stream_solve_ = false;
  int wave_r1_ = 0;                  // grid rows of 64*wave_r1_ points use the one-wave-per-FFT kernels (0: off)
  int B_ = 1;                        // instances of a batch
  std::vector<double> rab_;          // a batch's Rayleigh numbers (empty: a single problem)
  const double *BLnu_ = nullptr, *BLka_ = nullptr;   // a batch's nu and kappa parts of L
  std::vector<double> blnu_h_, blka_h_;               // (host copies, for the partition's coupling widths)
  std::vector<int> pmeta_h_;                          // partitioned solve: factor-kernel layout
  std::vector<int2> smap_h_;                          // partitioned solve: per-row spike offsets and widths
  const double2* frame_ = nullptr;   // plane Couette: unit wave vector of each mode
  std::vector<double> kxs_;
  std::vector<unsigned char> ckeep_;
  std::unique_ptr<CouettePlanes> planes_;
  RbcDev dv_{};
  DevArena arena_;
  double *BM_ = nullptr, *BL_ = nullptr, *ops_ = nullptr, *Jpart_ = nullptr;
  double* lops_ = nullptr;   // LU block operators of L alone (boundary value problem), built on first use
  double *eBM_ = nullptr, *eBL_ = nullptr, *eops_ = nullptr;   // stability operator bands and factors
  cplx *aV_ = nullptr, *aH_ = nullptr, *aZ_ = nullptr, *aY_ = nullptr;   // Arnoldi basis, Hessenberg, work
  cplx *vsR_ = nullptr, *vsW_ = nullptr, *vsQ_ = nullptr;   // eigenvector sensitivities: rhs, work, M^H Y
  cplx *ework_ = nullptr, *estart_ = nullptr;
  int ekl_ = 0, eku_ = 0;
  cplx* lrhs_ = nullptr;
  bool lfactored_ = false;
  int *err_ = nullptr;
  RkTab tab_;                        // the step's IMEX Runge-Kutta tableau
  double cur_dt_ = 0.0;              // the step of the launches being enqueued (step_setup)
  std::vector<double> vdt_;          // variable steps of a run (empty: the constant step)
  std::vector<int> vset_;            // factor set of each variable step
  std::vector<double*> vops_;        // factors of each distinct variable step
  std::map<double, double*> opcache_;   // factor sets built so far, by step
  int step_base_ = 0;                // run index of local step 0 (a segment's own schedule)
  cplx *Xst_, *Xw_, *Xg_, *acc_, *Ybuf_, *Fst_, *zgA_, *zbar_, *nl_, *nlbar_, *itmp_, *ckpt_, *seg_;
  size_t zsize_ = 0;
  int seglen_ = 0;
  hipStream_t aux_ = nullptr, cap_ = nullptr;
  hipEvent_t ev_[3] = {nullptr, nullptr, nullptr};
  bool graph_on_ = false, capturing_ = false;
  std::vector<std::pair<GraphKey, hipGraphExec_t>> graphs_;
  bool factored_ = false;
  int device_ = 0;   // the device current when the problem was built
  int tape_steps_ = -1;
  bool last_seg_ok_ = true;
  bool param_on_ = false;          // this gradient also accumulates dJ/dRa, dJ/dPr
  double* theta_out_ = nullptr;    // where they go
  cplx* sst_ = nullptr;            // state records of the parameter gradient (sslot)
  double* pacc_ = nullptr;         // [K][2] per-wavenumber dJ/dnu, dJ/dkappa   // uniform schedule: the last segment's stage fields are in their buffer
  int ckpt_mode_ = SPS_CKPT_UNIFORM, rv_slots_ = 0, rv_cap_ = 0;
  cplx* rv_ = nullptr;   // binomial schedule's stored states
  cplx* Xs_ = nullptr;   // working state of a two-level segment's forward actions
  std::map<int, std::pair<std::vector<CkptAction>, std::vector<CkptAction>>> sched_;   // by run length
  struct HostFree {
    void operator()(cplx* p) const { (void)hipHostFree(p); }
  };
  std::unique_ptr<cplx, HostFree> host_ckpt_;   // two-level: segment start states in pinned host memory
  std::unique_ptr<cplx, HostFree> ckstage_;     // disk level: two pinned staging buffers
  int host_cap_ = 0;                            // states held by host_ckpt_
  int outer_slots_ = 0;                         // outer-level slots (0: one per segment)
  double outer_wr_ = -1.0, outer_rd_ = -1.0;    // outer write/read costs in forward steps (< 0: binomial)
  std::map<int, std::pair<std::vector<CkptAction>, std::vector<CkptAction>>> osched_;
  cplx* Xo_ = nullptr;                          // working state of the nested outer schedule
  hipEvent_t ckev_[2] = {nullptr, nullptr};
  int ckfd_ = -1;                               // disk level: the checkpoint file, or -1
  std::string ckpath_;
  KernelTimer timer_;
  int timer_kind_ = 0;   // kernel class the timer follows (0 kfwd, 1 kadj, 2 x rows, 3 x rows adjoint)
};

}  // namespace

ProblemImpl* make_rbc(const sps_desc& d, hipStream_t s) { return new RbcProblem(d, s); }
ProblemImpl* make_rbc_batch(const sps_desc& d, int batch, const double* ra, hipStream_t s) {
  std::vector<double> r(batch > 0 ? batch : 0, d.param0);
  if (ra) r.assign(ra, ra + batch);
  return new RbcProblem(d, s, batch, r.data());
}
ProblemImpl* make_couette(const CouetteSpec& c, hipStream_t s) { return new RbcProblem(c, s); }

}  // namespace sps

extern "C" int sps_rbc_host_bands(const sps_desc* desc, int* kl, int* ku, double* BM, double* BL, int* rowmap,
                                  int* colmap, signed char* rowph, signed char* colph, double* rho) {
  try {
    if (!desc || !kl || !ku) return SPS_E_ARG;
    sps::RbcHostBands hb;
    sps::rbc_host_bands(*desc, hb);
    *kl = hb.kl;
    *ku = hb.ku;
    if (BM) std::copy(hb.BM.begin(), hb.BM.end(), BM);
    if (BL) std::copy(hb.BL.begin(), hb.BL.end(), BL);
    if (rowmap) std::copy(hb.rowmap.begin(), hb.rowmap.end(), rowmap);
    if (colmap) std::copy(hb.colmap.begin(), hb.colmap.end(), colmap);
    if (rowph) std::copy(hb.rowph.begin(), hb.rowph.end(), rowph);
    if (colph) std::copy(hb.colph.begin(), hb.colph.end(), colph);
    if (rho) std::copy(hb.rho.begin(), hb.rho.end(), rho);
    return SPS_OK;
  } catch (const sps::Error& e) {
    return e.code;
  }
}
