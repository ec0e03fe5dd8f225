// Host-side dense ultraspherical operators shared by the problems' band assembly: Chebyshev T
// (first kind), C1 = U and C2 bases on [-1, 1], each matrix N x N with column n the image of
// basis function n in the output basis (paper: Sparse spectral methods).
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

namespace sps {

// dense complex matrix in row-major order
struct Cmat {
  int n;
  std::vector<double2> a;
  explicit Cmat(int n_) : n(n_), a((size_t)n_ * n_, make_double2(0.0, 0.0)) {}
  double2& at(int i, int j) { return a[(size_t)i * n + j]; }
  void add(int i, int j, double re, double im = 0.0) {
    at(i, j).x += re;
    at(i, j).y += im;
  }
};

// T -> C1 conversion: T_0 = U_0, T_1 = U_1 / 2, T_n = (U_n - U_{n-2}) / 2
inline std::vector<double> op_S0(int N) {
  std::vector<double> S((size_t)N * N, 0.0);
  for (int n = 0; n < N; ++n) {
    S[(size_t)n * N + n] = (n == 0) ? 1.0 : 0.5;
    if (n >= 2) S[(size_t)(n - 2) * N + n] = -0.5;
  }
  return S;
}
// C1 -> C2 conversion: U_n = (C2_n - C2_{n-2}) / (n + 1)
inline std::vector<double> op_S1(int N) {
  std::vector<double> S((size_t)N * N, 0.0);
  for (int n = 0; n < N; ++n) {
    S[(size_t)n * N + n] = 1.0 / (n + 1);
    if (n >= 2) S[(size_t)(n - 2) * N + n] = -1.0 / (n + 1);
  }
  return S;
}
// derivative one basis up: D[n-1][n] = v n (T -> C1 with v = 1) or v (C1 -> C2 with v = 2)
inline std::vector<double> op_D(int N, double v, bool scaled_by_index) {
  std::vector<double> D((size_t)N * N, 0.0);
  for (int n = 1; n < N; ++n) D[(size_t)(n - 1) * N + n] = scaled_by_index ? v * n : v;
  return D;
}
// C = A B for N x N row-major matrices
inline std::vector<double> matmul(const std::vector<double>& A, const std::vector<double>& B, int N) {
  std::vector<double> C((size_t)N * N, 0.0);
  for (int i = 0; i < N; ++i)
    for (int k = 0; k < N; ++k) {
      const double a = A[(size_t)i * N + k];
      if (a == 0.0) continue;
      for (int j = 0; j < N; ++j) C[(size_t)i * N + j] += a * B[(size_t)k * N + j];
    }
  return C;
}

}  // namespace sps
