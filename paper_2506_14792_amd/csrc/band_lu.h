// Batched banded LU with partial pivoting (one real system per wavenumber) and its
// forward and transposed solves.  The factorization is LAPACK-style (row exchanges
// interleaved with the eliminations, kl sub- and ku super-diagonals, U fill up to
// kl + ku); its factors are then condensed into dense block operators (below) that the
// solves apply.
#pragma once
#include "sps_device.h"

// Uniform value v placed into lane `lane` of a wave-distributed value (a lane select).
__device__ __forceinline__ double writelane_d(double v, int lane, double old) {
  return (lane_id() == lane) ? v : old;
}

// Blocked solves.  The factor kernel turns the banded LU factors into dense block operators
// (one set per system) so that a solve is a short chain of small matrix-vector products
// with no per-row lane broadcasts:
//   T_t  (TW x TW): the row exchanges and eliminations of L-sweep steps t*BLK .. t*BLK+BLK-1
//        acting on the window [t*BLK, t*BLK + TW) (identity beyond BLK + kl); the L sweep is
//        T_last ... T_1 T_0.
//   G_t  (BLK x GW): back substitution of U rows t*BLK .. t*BLK+BLK-1,
//        x_block = G_t [y_block; x(t*BLK + BLK .. t*BLK + GW)], G_t = [U_tt^{-1} | -U_tt^{-1} U_t,off]
//        (zero beyond BLK + uw - 1); the U sweep applies G_t for t descending.
// The transposed solve applies G_t^T for t ascending, then T_t^T for t descending.
// Block shapes are compile-time so every read is unconditional: the right-hand side must
// be followed by at least SPS_PAD zero entries (positions n .. n + SPS_PAD - 1), which the
// operators keep at zero.
// Layout per system: T[nblk][TW][TS] (row-major, padded rows) followed by G[nblk][BLK][GS].
// One complex right-hand side per wave (lanes 0-31 the real parts, 32-63 the imaginary parts):
// b[2*i], b[2*i + 1] in LDS; operators in LDS.
#define SPS_BLK 8
#define SPS_TW 16     // T window: needs SPS_BLK + kl <= SPS_TW
#define SPS_GW 36     // G width: needs SPS_BLK + uw - 1 <= SPS_GW
#define SPS_TS 17     // row stride of T (odd: rows and columns are both read without LDS bank conflicts)
#define SPS_GS 37     // row stride of G
#define SPS_PAD 40    // zero tail after the right-hand side (>= SPS_GW)

__host__ __device__ inline int blk_count(int n) { return (n + SPS_BLK - 1) / SPS_BLK; }
// doubles of the T blocks and of the G blocks of an n-row system (multiples of 4, so every
// set of operators starts 32-byte aligned), and of both
__host__ __device__ inline int blk_t_size(int n) { return blk_count(n) * SPS_TW * SPS_TS; }
__host__ __device__ inline int blk_g_size(int n) { return blk_count(n) * SPS_BLK * SPS_GS; }
__host__ __device__ inline int blk_ops_size(int n) { return blk_t_size(n) + blk_g_size(n); }
static_assert((SPS_TW * SPS_TS) % 4 == 0 && (SPS_BLK * SPS_GS) % 4 == 0, "block sizes keep 32-byte alignment");

// The four sweeps over a range of blocks [t0, t1), with the operators of that range at T (T
// blocks t0 .. t1-1) or G (G blocks t0 .. t1-1): forward L sweep (t ascending) and U sweep
// (t descending), transposed U^T sweep (t ascending) and L^T sweep (t descending).  One wave
// per complex right-hand side: lanes 0-31 take the real parts, lanes 32-63 the imaginary parts
// (element x at b[2x + part]), both halves reading the same operator entries.  Entries at
// nrow and beyond are read (the operators multiply them by zero, or copy them) but never
// written, so a system whose rows are followed by another system's live rows can be solved
// in place while that one is solved by another wave.
// L sweep: output r = l/2, half h = l&1 sums columns 8h .. 8h+7 (l = lane within the half)
__device__ inline void blk_L_range(const double* T, int t0, int t1, double* b, int nrow) {
  const int lane = lane_id(), l = lane & 31;
  const int r = l >> 1, h = l & 1;
  double* bc = b + (lane >> 5);
  for (int t = t0; t < t1; ++t) {
    const double* v = bc + 2 * (t * SPS_BLK + 8 * h);
    const double* Tr = T + ((t - t0) * SPS_TW + r) * SPS_TS + 8 * h;
    double a0 = 0.0, a1 = 0.0;
#pragma unroll
    for (int c = 0; c < 8; c += 2) {
      a0 = fma(Tr[c], v[2 * (c)], a0);
      a1 = fma(Tr[c + 1], v[2 * (c + 1)], a1);
    }
    double s = a0 + a1;
    s += dpp_xor1(s);
    if (h == 0 && t * SPS_BLK + r < nrow) bc[2 * (t * SPS_BLK + r)] = s;
  }
}
// U sweep: output i = l/4, quarter q = l&3 sums columns 9q .. 9q+8
__device__ inline void blk_U_range(const double* G, int t0, int t1, double* b, int nrow) {
  const int lane = lane_id(), l = lane & 31;
  const int i = l >> 2, q = l & 3;
  double* bc = b + (lane >> 5);
  for (int t = t1 - 1; t >= t0; --t) {
    const double* v = bc + 2 * (t * SPS_BLK + 9 * q);
    const double* Gr = G + ((t - t0) * SPS_BLK + i) * SPS_GS + 9 * q;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
#pragma unroll
    for (int c = 0; c < 9; c += 3) {
      a0 = fma(Gr[c], v[2 * (c)], a0);
      a1 = fma(Gr[c + 1], v[2 * (c + 1)], a1);
      a2 = fma(Gr[c + 2], v[2 * (c + 2)], a2);
    }
    double s = (a0 + a1) + a2;
    s += dpp_xor1(s);
    s += dpp_xor2(s);
    if (q == 0 && t * SPS_BLK + i < nrow) bc[2 * (t * SPS_BLK + i)] = s;
  }
}
// U^T sweep: output column c = l sums the BLK rows of its column; lanes l < GW - 32 also take
// column l + 32 (the others compute a copy of column GW - 1 that they do not store)
__device__ inline void blk_Ut_range(const double* G, int t0, int t1, double* b, int nrow) {
  const int lane = lane_id(), c = lane & 31, c2 = min(c + 32, SPS_GW - 1);
  double* bc = b + (lane >> 5);
  for (int t = t0; t < t1; ++t) {
    const double* v = bc + 2 * (t * SPS_BLK);
    const double* Gc = G + (t - t0) * SPS_BLK * SPS_GS;
    double a0 = 0.0, a1 = 0.0, e0 = 0.0, e1 = 0.0;
#pragma unroll
    for (int i = 0; i < SPS_BLK; i += 2) {
      const double v0 = v[2 * (i)], v1 = v[2 * (i + 1)];
      a0 = fma(Gc[i * SPS_GS + c], v0, a0);
      a1 = fma(Gc[(i + 1) * SPS_GS + c], v1, a1);
      e0 = fma(Gc[i * SPS_GS + c2], v0, e0);
      e1 = fma(Gc[(i + 1) * SPS_GS + c2], v1, e1);
    }
    const double keep = (c >= SPS_BLK) ? v[2 * (c)] : 0.0;
    const double keep2 = v[2 * (c2)];
    if (t * SPS_BLK + c < nrow) bc[2 * (t * SPS_BLK + c)] = keep + (a0 + a1);
    if (c + 32 < SPS_GW && t * SPS_BLK + c2 < nrow) bc[2 * (t * SPS_BLK + c2)] = keep2 + (e0 + e1);
  }
}
// L^T sweep: output column c = l/2, half h = l&1 sums rows 8h .. 8h+7 of column c
__device__ inline void blk_Lt_range(const double* T, int t0, int t1, double* b, int nrow) {
  const int lane = lane_id(), l = lane & 31;
  const int c = l >> 1, h = l & 1;
  double* bc = b + (lane >> 5);
  for (int t = t1 - 1; t >= t0; --t) {
    const double* v = bc + 2 * (t * SPS_BLK + 8 * h);
    const double* Tc = T + ((t - t0) * SPS_TW + 8 * h) * SPS_TS + c;
    double a0 = 0.0, a1 = 0.0;
#pragma unroll
    for (int r = 0; r < 8; r += 2) {
      a0 = fma(Tc[r * SPS_TS], v[2 * (r)], a0);
      a1 = fma(Tc[(r + 1) * SPS_TS], v[2 * (r + 1)], a1);
    }
    double s = a0 + a1;
    s += dpp_xor1(s);
    if (h == 0 && t * SPS_BLK + c < nrow) bc[2 * (t * SPS_BLK + c)] = s;
  }
}
// One system's block operators are brought into LDS in two steps so that their memory
// latency overlaps other work: ops_issue() starts all global loads of this thread's share
// into registers, ops_store_part() writes one set of them into LDS once the destination is free.
// The T blocks and the G blocks of a system are loaded and stored separately, so that the set
// the first sweep needs can go to LDS before the other has arrived.  Counts (doubles) must be
// multiples of 2; at most SPS_OPS_REG_T / SPS_OPS_REG_G 16-byte loads per thread.
#define SPS_OPS_REG_T 9
#define SPS_OPS_REG_G 10
struct OpsRegs {
  double2 t[SPS_OPS_REG_T];
  double2 g[SPS_OPS_REG_G];
};
// Every load is issued (an index past the end is clamped to the last element, whose copy is
// not stored): a load under a branch would leave the compiler unsure how many loads are in
// flight after an earlier one, and it then waits for all of them before using that one.
template <int NS>
__device__ __forceinline__ void ops_issue_part(const double* g, int count, double2 (&v)[NS]) {
  const double2* g2 = reinterpret_cast<const double2*>(g);
  const int h = count / 2;
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    // (field by field: a whole-struct copy from global memory keeps v in scratch memory)
    const double2* p = g2 + min((int)(threadIdx.x + i * blockDim.x), h - 1);
    v[i] = make_double2(p->x, p->y);
  }
}
template <int NS>
__device__ __forceinline__ void ops_store_part(const double2 (&v)[NS], int count, double* dst) {
  double2* d2 = reinterpret_cast<double2*>(dst);
  const int h = count / 2;
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    const int e = threadIdx.x + i * blockDim.x;
    if (e < h) d2[e] = v[i];
  }
}
// a system's operators at g: tsz doubles of T blocks, then gsz of G blocks.  The loads return
// in issue order, so a wait for the set issued first does not wait for the other.
__device__ __forceinline__ void ops_issue(const double* g, int tsz, int gsz, OpsRegs& r) {
  ops_issue_part(g, tsz, r.t);
  ops_issue_part(g + tsz, gsz, r.g);
}
// the same with the G blocks issued first
__device__ __forceinline__ void ops_issue_gt(const double* g, int tsz, int gsz, OpsRegs& r) {
  ops_issue_part(g + tsz, gsz, r.g);
  ops_issue_part(g, tsz, r.t);
}

// ---------------------------------------------------------------------------- factor
// One block (>= 64 threads) per system.  AB: row-band input for this system,
// band[i*(kl+ku+1) + (c - i + kl)] = A[i][c], combined as a*BM + b*BL; entries whose column
// falls outside [0, n) are dropped (so a band pointer offset by m rows with n = n - m gives the
// trailing diagonal block, and n = m the leading one).
// LDS layout (LAPACK band with fill rows): ab[c*ldab + (kv + i - c)] = A[i][c],
// ldab = 2kl + ku + 1, kv = kl + ku.
// With BLnu and BLka given, the L band is BL + nu BLnu + ka BLka (an operator affine in two
// parameters, here the diffusivities of one instance of a batch).
__device__ inline void band_lu_factor(const double* __restrict__ BM, const double* __restrict__ BL, double a,
                                      double bcoef, int n, int kl, int ku, double* ab, int* sh, int* spiv, int* err,
                                      const double* __restrict__ BLnu = nullptr,
                                      const double* __restrict__ BLka = nullptr, double nu = 0.0, double ka = 0.0) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int ldab = 2 * kl + ku + 1, kv = kl + ku, bw = kl + ku + 1;
  for (int e = tid; e < n * ldab; e += nt) ab[e] = 0.0;
  __syncthreads();
  for (int e = tid; e < n * bw; e += nt) {
    const int i = e / bw, d = e - i * bw;
    const int c = i + d - kl;
    if (c >= 0 && c < n) {
      const double l = BLnu ? BL[e] + nu * BLnu[e] + ka * BLka[e] : BL[e];
      ab[c * ldab + (kv + i - c)] = a * BM[e] + bcoef * l;
    }
  }
  __syncthreads();
  // the column steps on wave 0 alone (a step touches at most (kl + 1) x (kl + ku + 1) entries;
  // the LDS operations of one wave complete in order, so no block barrier is needed per step)
  if (tid < SPS_WAVE) {
    const int lane = tid;
    auto wsync = [] {
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
    };
    for (int j = 0; j < n; ++j) {
      const int km = min(kl, n - 1 - j);
      const int wd = min(kv, n - 1 - j);  // columns right of j that can hold fill
      // pivot: the first row of largest magnitude among j .. j + km (lanes 0 .. 7, DPP merge)
      int jp = lane;
      double best = (lane <= km && lane < 8) ? fabs(ab[j * ldab + kv + lane]) : -1.0;
      auto merge = [&](double ob, int op) {
        if (ob > best || (ob == best && op < jp)) {
          best = ob;
          jp = op;
        }
      };
      merge(dpp_xor1(best), __builtin_amdgcn_mov_dpp(jp, 0xB1, 0xF, 0xF, false));
      merge(dpp_xor2(best), __builtin_amdgcn_mov_dpp(jp, 0x4E, 0xF, 0xF, false));
      merge(dpp_mirror8(best), __builtin_amdgcn_mov_dpp(jp, 0x141, 0xF, 0xF, false));
      jp = __builtin_amdgcn_readfirstlane(jp);
      best = __shfl(best, 0);
      if (lane == 0) {
        spiv[j] = j + jp;
        if (!(best > 0.0) || !isfinite(best)) atomicOr(err, 1);
      }
      if (jp != 0 && lane <= wd) {
        const int c = j + lane;
        double* p0 = &ab[c * ldab + kv + j - c];
        double* p1 = &ab[c * ldab + kv + j + jp - c];
        const double t0 = *p0, t1 = *p1;
        *p0 = t1;
        *p1 = t0;
      }
      wsync();
      const double rinv = 1.0 / ab[j * ldab + kv];
      if (lane >= 1 && lane <= km) ab[j * ldab + kv + lane] *= rinv;
      wsync();
      // rank-1 update: lane (row j + 1 + (lane & 7), columns j + 1 + (lane >> 3) + 8 q)
      {
        const int i = 1 + (lane & 7), c0 = j + 1 + (lane >> 3);
        if (i <= km) {
          const double l = ab[j * ldab + kv + i];
          double u[4], v[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int c = c0 + 8 * q;
            if (c <= j + wd) {
              u[q] = ab[c * ldab + kv + j - c];
              v[q] = ab[c * ldab + kv + j + i - c];
            }
          }
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int c = c0 + 8 * q;
            if (c <= j + wd) ab[c * ldab + kv + j + i - c] = v[q] - l * u[q];
          }
        }
      }
      wsync();
    }
  }
  __syncthreads();
}

// Block operators (see above) of the factors in ab; T_t column c is the image of the window's
// unit vector e_c.
__device__ inline void band_condense(const double* ab, const int* spiv, int n, int kl, int ku, double* T, double* G) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int ldab = 2 * kl + ku + 1, kv = kl + ku;
  __syncthreads();
  const int nblk = blk_count(n);
  for (int e = tid; e < nblk * SPS_TW; e += nt) {
    const int t = e / SPS_TW, c = e - t * SPS_TW, tb = t * SPS_BLK;
    double v[SPS_TW];
#pragma unroll
    for (int r = 0; r < SPS_TW; ++r) v[r] = (r == c) ? 1.0 : 0.0;
    for (int q = 0; q < SPS_BLK; ++q) {
      const int j = tb + q;
      if (j >= n) break;
      const int p = spiv[j] - j;
      double vq = 0.0, vp = 0.0;
#pragma unroll
      for (int r = 0; r < SPS_TW; ++r) {
        if (r == q) vq = v[r];
        if (r == q + p) vp = v[r];
      }
#pragma unroll
      for (int r = 0; r < SPS_TW; ++r) {
        if (r == q) v[r] = vp;
        else if (r == q + p) v[r] = vq;
      }
      const int km = min(kl, n - 1 - j);
#pragma unroll
      for (int r = 0; r < SPS_TW; ++r) {
        const int i = r - q;   // row j + i
        if (i >= 1 && i <= km) v[r] -= ab[j * ldab + kv + i] * vp;
      }
    }
    for (int r = 0; r < SPS_TW; ++r) T[(t * SPS_TW + r) * SPS_TS + c] = v[r];
  }
  // G_t row i: Ui[i][c] for c < BLK (row i of the inverse of the diagonal block of U),
  // then -sum_i' Ui[i][i'] U[tb+i'][tb+c] for BLK <= c < GW
  auto Uat = [&](int i, int c) -> double {   // U[i][c] of the factored band
    return (i < n && c < n && c >= i && c - i <= kv) ? ab[c * ldab + kv + i - c] : 0.0;
  };
  for (int e = tid; e < nblk * SPS_BLK; e += nt) {
    const int t = e / SPS_BLK, i = e - t * SPS_BLK, tb = t * SPS_BLK;
    double ui[SPS_BLK];
#pragma unroll
    for (int c = 0; c < SPS_BLK; ++c) ui[c] = 0.0;
    if (tb + i < n) {
#pragma unroll
      for (int c = 0; c < SPS_BLK; ++c) {
        if (c < i || tb + c >= n) continue;
        double sacc = (c == i) ? 1.0 : 0.0;
#pragma unroll
        for (int ip = 0; ip < SPS_BLK; ++ip)
          if (ip >= i && ip < c) sacc -= ui[ip] * Uat(tb + ip, tb + c);
        ui[c] = sacc / Uat(tb + c, tb + c);
      }
    }
    double* Gr = G + (t * SPS_BLK + i) * SPS_GS;
#pragma unroll
    for (int c = 0; c < SPS_BLK; ++c) Gr[c] = ui[c];
    for (int c = SPS_BLK; c < SPS_GS; ++c) {
      double sacc = 0.0;
#pragma unroll
      for (int ip = 0; ip < SPS_BLK; ++ip) sacc -= ui[ip] * Uat(tb + ip, tb + c);
      Gr[c] = sacc;
    }
  }
}

__device__ inline void band_factor_block(const double* __restrict__ BM, const double* __restrict__ BL,
                                         double a, double bcoef, int n, int kl, int ku, double* ab,
                                         int* sh, int* spiv, double* OPS, int* err,
                                         const double* __restrict__ BLnu = nullptr,
                                         const double* __restrict__ BLka = nullptr, double nu = 0.0,
                                         double ka = 0.0) {
  band_lu_factor(BM, BL, a, bcoef, n, kl, ku, ab, sh, spiv, err, BLnu, BLka, nu, ka);
  band_condense(ab, spiv, n, kl, ku, OPS, OPS + blk_t_size(n));
}

// Solves with the factors in ab for nr <= blockDim.x / 8 right-hand sides, the columns of the
// n x nr row-major matrix R (LDS): A x = r (row interchanges and L, then U) or, transposed,
// A^T x = r (U^T, then L^T and the interchanges in reverse).  Column c is taken by the eight
// lanes 8c .. 8c + 7 of one wave, so a step needs no block barrier: lane i updates the rows
// j + i (L, kl <= 7) or j - i, j - i - 8, ... (U), or sums those products for the transposed
// solve (an eight-lane DPP sum).  Used for the partitioned solve's coupling blocks at
// factorization time.  Block-wide (ends with a barrier).
__device__ inline void band_lu_solve_cols(const double* ab, const int* spiv, int n, int kl, int ku, double* R,
                                          int nr, bool transposed) {
  constexpr int KV = SPS_GW - SPS_BLK;   // the widest band of the block operators, kl + ku <= KV
  const int c = threadIdx.x >> 3, i = threadIdx.x & 7, ldab = 2 * kl + ku + 1, kv = kl + ku;
  __syncthreads();
  if (c < nr) {
    auto x = [&](int r) -> double& { return R[(size_t)r * nr + c]; };
    auto wsync = [] {
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
    };
    if (!transposed) {
      for (int j = 0; j < n; ++j) {
        // row j takes x(p) (the interchange); row j + i, i <= km, the old entry of row j + i
        // (or of row j if j + i = p) minus l_i times it
        const int p = spiv[j], km = min(kl, n - 1 - j);
        const double xj = x(p);
        double v = 0.0, l = 0.0;
        if (i >= 1 && i <= km) {
          v = (j + i == p) ? x(j) : x(j + i);
          l = ab[j * ldab + kv + i];
        }
        wsync();
        if (i == 0) x(j) = xj;
        else if (i <= km) x(j + i) = v - l * xj;
        wsync();
      }
      for (int j = n - 1; j >= 0; --j) {
        const double xj = x(j) / ab[j * ldab + kv];
        const int ku2 = min(kv, j);
        double v[KV / 8 + 1], u[KV / 8 + 1];
#pragma unroll
        for (int q = 0; q <= KV / 8; ++q) {
          const int r = i + 8 * q;
          if (r >= 1 && r <= ku2) {
            v[q] = x(j - r);
            u[q] = ab[j * ldab + kv - r];
          }
        }
        wsync();
        if (i == 0) x(j) = xj;
#pragma unroll
        for (int q = 0; q <= KV / 8; ++q) {
          const int r = i + 8 * q;
          if (r >= 1 && r <= ku2) x(j - r) = v[q] - u[q] * xj;
        }
        wsync();
      }
    } else {
      for (int j = 0; j < n; ++j) {
        const int ku2 = min(kv, j);
        double s = 0.0;
#pragma unroll
        for (int q = 0; q <= KV / 8; ++q) {
          const int r = i + 8 * q;
          if (r >= 1 && r <= ku2) s = fma(ab[j * ldab + kv - r], x(j - r), s);
        }
        s = group_sum<8>(s);
        const double xj = (x(j) - s) / ab[j * ldab + kv];
        wsync();
        if (i == 0) x(j) = xj;
        wsync();
      }
      for (int j = n - 2; j >= 0; --j) {
        const int km = min(kl, n - 1 - j);
        double s = (i >= 1 && i <= km) ? ab[j * ldab + kv + i] * x(j + i) : 0.0;
        s = group_sum<8>(s);
        const double xjv = x(j) - s;
        const int p = spiv[j];
        const double xp = x(p);
        wsync();
        if (i == 0) {
          if (p != j) {
            x(j) = xp;
            x(p) = xjv;
          } else {
            x(j) = xjv;
          }
        }
        wsync();
      }
    }
  }
  __syncthreads();
}

// Inverse of the nr x nr matrix A (row-major, LDS) into Ainv (global, row-major, or
// column-major if colmajor) by Gauss-Jordan elimination with partial pivoting on [A | I] in LDS
// (aug: nr x 2nr doubles, then nr doubles of multipliers); sh: one int of LDS.  Thread t takes column t mod 2nr of the augmented matrix and every
// (blockDim / 2nr)-th row.  Block-wide (ends with a barrier).
__device__ inline void block_inverse(const double* A, int nr, double* aug, double* Ainv, int* err, int* sh,
                                     bool colmajor = false) {
  const int tid = threadIdx.x, nt = blockDim.x, w = 2 * nr;
  double* f = aug + (size_t)nr * w;
  const int groups = max(nt / w, 1), g = tid / w, c = tid - g * w;
  __syncthreads();
  for (int e = tid; e < nr * w; e += nt) {
    const int i = e / w, cc = e - i * w;
    aug[e] = (cc < nr) ? A[i * nr + cc] : ((cc - nr == i) ? 1.0 : 0.0);
  }
  __syncthreads();
  for (int j = 0; j < nr; ++j) {
    if (tid < 8) {
      // pivot: the first row i >= j of largest |aug[i][j]| (eight lanes, every eighth row,
      // then a DPP reduction over the eight that keeps the smaller index of equal values)
      int p = j;
      double best = -1.0;
      for (int i = j + tid; i < nr; i += 8) {
        const double v = fabs(aug[i * w + j]);
        if (v > best) {
          best = v;
          p = i;
        }
      }
      auto merge = [&](double ob, int op) {
        if (ob > best || (ob == best && op < p)) {
          best = ob;
          p = op;
        }
      };
      merge(dpp_xor1(best), __builtin_amdgcn_mov_dpp(p, 0xB1, 0xF, 0xF, false));
      merge(dpp_xor2(best), __builtin_amdgcn_mov_dpp(p, 0x4E, 0xF, 0xF, false));
      merge(dpp_mirror8(best), __builtin_amdgcn_mov_dpp(p, 0x141, 0xF, 0xF, false));
      if (tid == 0) {
        if (!(best > 0.0)) atomicOr(err, 1);
        sh[0] = p;
      }
    }
    __syncthreads();
    const int p = sh[0];
    const double rinv = 1.0 / aug[p * w + j];
    if (g == 0 && c < w) {
      // rows j and p exchanged, the new row j scaled by the pivot's reciprocal
      const double a = aug[j * w + c], b = aug[p * w + c];
      aug[j * w + c] = b * rinv;
      if (p != j) aug[p * w + c] = a;
    }
    __syncthreads();
    for (int i = tid; i < nr; i += nt) f[i] = (i == j) ? 0.0 : aug[i * w + j];
    __syncthreads();
    if (g < groups && c < w) {
      // (four rows at a time: their reads in flight together)
      const double pj = aug[j * w + c];
      int i = g;
      for (; i + 3 * groups < nr; i += 4 * groups) {
        double v[4], fv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          v[u] = aug[(i + u * groups) * w + c];
          fv[u] = f[i + u * groups];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) aug[(i + u * groups) * w + c] = v[u] - fv[u] * pj;
      }
      for (; i < nr; i += groups) aug[i * w + c] -= f[i] * pj;
    }
    __syncthreads();
  }
  for (int e = tid; e < nr * nr; e += nt) {
    const int i = e / nr, cc = e - i * nr;
    Ainv[colmajor ? cc * nr + i : e] = aug[i * w + nr + cc];
  }
  __syncthreads();
}
