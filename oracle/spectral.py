"""Spectral bases, transforms and sparse ultraspherical operators as plain dense matrices.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Paper passages followed:
* "Sparse spectral methods": trial/test bases giving banded operators (the
  ultraspherical method), nonlinear terms on a collocation grid, boundary
  conditions through tau terms.
* Methods, "Spectral transforms": f_hat = T f, f = T^{-1} f_hat; the adjoint of a
  matrix transform is its Hermitian transpose.

Readings where the paper is silent:
* Fourier: real data, half spectrum m = 0..K-1 stored (Nyquist dropped).
  backward  u_j = Re(c_0) + 2 Re sum_{m>=1} c_m exp(i k_m x_j),
  forward   c_m = (1/Ng) sum_j u_j exp(-i k_m x_j),   x_j = j L / Ng, k_m = 2 pi m / L.
* Chebyshev on [a, b]: Gauss (root) nodes, ascending:
  x_j = -cos(pi (j + 1/2) / Ng), z_j = a + (b - a)(x_j + 1)/2,
  backward  f_j = sum_{n<N} a_n T_n(x_j),
  forward   a_n = (2 - delta_{n0}) / Ng * sum_j f_j T_n(x_j).
* Dealiasing: evaluate on a padded grid of Ng = 3/2 * (modes) points (2x for
  cubic products), transform forward and truncate back to the stored modes.
"""
import numpy as np


# ----------------------------------------------------------------------------- Fourier


def fourier_grid(Ng, L):
    """Uniform periodic grid x_j = j L / Ng."""
    return np.arange(Ng) * (L / Ng)


def fourier_wavenumbers(K, L):
    """Wavenumbers k_m = 2 pi m / L of the stored half spectrum m = 0..K-1."""
    return 2.0 * np.pi * np.arange(K) / L


def grid_phase(m, Ng):
    """exp(i k_m x_j) on the grid x_j = j L / Ng, as a (len(j) = Ng) x len(m) array, for integer
    (possibly negative) mode numbers m.  Since k_m x_j = 2 pi m j / Ng, the angle is reduced
    exactly in integers first (m j mod Ng), so every entry is correct to the rounding of one
    cosine and sine, independent of L and of the sizes of m and j."""
    j = np.arange(Ng)
    r = np.mod(np.outer(j, np.asarray(m, dtype=np.int64)), Ng)
    return np.exp(2j * np.pi * r / Ng)


def fourier_backward_matrix(K, Ng, L):
    """Complex matrix B (Ng x K) such that the real grid values are u = Re(B @ c).

    B[j, m] = w_m exp(i k_m x_j) with w_0 = 1 and w_m = 2 for m >= 1, so that
    u_j = Re(c_0) + 2 Re sum_{m>=1} c_m exp(i k_m x_j).
    """
    w = np.full(K, 2.0)
    w[0] = 1.0
    return w[None, :] * grid_phase(np.arange(K), Ng)


def fourier_forward_matrix(K, Ng, L):
    """Complex matrix F (K x Ng): c_m = (1/Ng) sum_j u_j exp(-i k_m x_j) (truncating)."""
    return np.conj(grid_phase(np.arange(K), Ng)).T / Ng


def fourier_backward(c, B):
    """Real grid values from half-spectrum coefficients along axis 0 of c."""
    return np.real(np.tensordot(B, c, axes=(1, 0)))


def fourier_backward_adjoint(ubar, B):
    """Adjoint (real inner products) of fourier_backward: cbar = B^H ubar."""
    return np.tensordot(B.conj(), ubar, axes=(0, 0))


def fourier_forward(u, F):
    """Half-spectrum coefficients of real grid values along axis 0 of u."""
    return np.tensordot(F, u, axes=(1, 0))


def fourier_forward_adjoint(cbar, F):
    """Adjoint (real inner products) of fourier_forward: ubar = Re(F^H cbar)."""
    return np.real(np.tensordot(F.conj(), cbar, axes=(0, 0)))


# ----------------------------------------------------------------------------- complex Fourier (full spectrum)


def complex_fourier_modes(Nc):
    """Signed mode numbers of a full complex spectrum of a periodic direction with Nc
    grid points at scale 1, Nyquist dropped: 0..Nc/2-1, then -Nc/2+1..-1 (Nc - 1 modes),
    stored in the usual FFT order with the Nyquist slot kept as an unused zero."""
    m = np.arange(Nc)
    m = np.where(m < Nc // 2, m, m - Nc)
    return m


def complex_fourier_backward_matrix(Nc, Ng, L):
    """(Ng x Nc): u_j = sum_m c_m exp(i k_m x_j); the Nyquist slot (m = -Nc/2) is not used."""
    m = complex_fourier_modes(Nc)
    keep = (np.abs(m) < Nc // 2).astype(float)
    return keep[None, :] * grid_phase(m, Ng)


def complex_fourier_forward_matrix(Nc, Ng, L):
    """(Nc x Ng): c_m = (1/Ng) sum_j u_j exp(-i k_m x_j), Nyquist slot set to zero."""
    m = complex_fourier_modes(Nc)
    keep = (np.abs(m) < Nc // 2).astype(float)
    return keep[:, None] * np.conj(grid_phase(m, Ng)).T / Ng


# ----------------------------------------------------------------------------- Chebyshev


def chebyshev_nodes(Ng):
    """Gauss-Chebyshev (root) nodes on [-1, 1], ascending."""
    return -np.cos(np.pi * (np.arange(Ng) + 0.5) / Ng)


def chebyshev_T(nmax, x):
    """Matrix T[j, n] = T_n(x_j) = cos(n arccos x_j), n < nmax."""
    x = np.asarray(x, dtype=float)
    th = np.arccos(np.clip(x, -1.0, 1.0))
    return np.cos(np.outer(th, np.arange(nmax)))


def chebyshev_T_nodes(nmax, Ng):
    """T[j, n] = T_n(x_j) at the ascending Gauss nodes x_j = -cos(pi (j + 1/2) / Ng):
    T_n(x_j) = cos(n arccos x_j) = cos(pi n (2 (Ng - j) - 1) / (2 Ng)), with the angle reduced
    exactly in integers (mod 4 Ng) so that every entry is correct to the rounding of one cosine
    (cos(n arccos x_j) of the rounded node loses about n ulps of the angle)."""
    j = np.arange(Ng)
    n = np.arange(nmax, dtype=np.int64)
    M = np.mod(np.outer(2 * (Ng - j) - 1, n), 4 * Ng)
    return np.cos(np.pi * M / (2.0 * Ng))


def chebyshev_backward_matrix(N, Ng):
    """(Ng x N): f_j = sum_n a_n T_n(x_j) on the Gauss nodes."""
    return chebyshev_T_nodes(N, Ng)


def chebyshev_forward_matrix(N, Ng):
    """(N x Ng): a_n = (2 - delta_{n0}) / Ng * sum_j f_j T_n(x_j), truncated to n < N."""
    T = chebyshev_T_nodes(N, Ng)
    c = np.full(N, 2.0)
    c[0] = 1.0
    return (c[:, None] * T.T) / Ng


def z_of_x(x, a, b):
    """Map the reference interval [-1, 1] onto [a, b]."""
    return a + (b - a) * (np.asarray(x) + 1.0) / 2.0


# ----------------------------------------------------------------------------- ultraspherical operators
#
# Bases: T_n (Chebyshev first kind), C1_n = U_n (Gegenbauer lambda = 1), C2_n (lambda = 2).
# Column n of each matrix holds the image of the n-th input basis function expanded in
# the output basis; all matrices are N x N (degree is never raised).


def D0(N):
    """d/dx: T -> C1.  d/dx T_n = n U_{n-1}."""
    D = np.zeros((N, N))
    for n in range(1, N):
        D[n - 1, n] = n
    return D


def D1(N):
    """d/dx: C1 -> C2.  d/dx U_n = 2 C2_{n-1}."""
    D = np.zeros((N, N))
    for n in range(1, N):
        D[n - 1, n] = 2.0
    return D


def S0(N):
    """Conversion T -> C1.  T_0 = U_0, T_1 = U_1 / 2, T_n = (U_n - U_{n-2}) / 2."""
    S = np.zeros((N, N))
    S[0, 0] = 1.0
    for n in range(1, N):
        S[n, n] = 0.5
        if n >= 2:
            S[n - 2, n] = -0.5
    return S


def S1(N):
    """Conversion C1 -> C2.  U_n = (C2_n - C2_{n-2}) / (n + 1)."""
    S = np.zeros((N, N))
    for n in range(N):
        S[n, n] = 1.0 / (n + 1)
        if n >= 2:
            S[n - 2, n] = -1.0 / (n + 1)
    return S


def cheb_derivative_T(N):
    """d/dx within the T basis (dense upper triangle):
    d/dx T_n = sum_{m<n, m+n odd} (2n / c_m) T_m with c_0 = 2, c_m = 1 otherwise."""
    D = np.zeros((N, N))
    for n in range(N):
        for m in range(n):
            if (m + n) % 2 == 1:
                D[m, n] = 2.0 * n / (2.0 if m == 0 else 1.0)
    return D


def boundary_row(N, side):
    """Evaluation row of a T series at x = -1 (side=-1) or x = +1 (side=+1)."""
    n = np.arange(N)
    return np.ones(N) if side > 0 else (-1.0) ** n


def integral_row(N, a, b):
    """Row r with r @ a = int_a^b sum_n a_n T_n dz: (b - a)/(1 - n^2) for even n, 0 for odd."""
    r = np.zeros(N)
    for n in range(0, N, 2):
        r[n] = (b - a) / (1.0 - n * n)
    return r


def gram_T(N, a, b):
    """G[m, n] = int_a^b T_m T_n dz, using T_m T_n = (T_{m+n} + T_{|m-n|}) / 2."""
    def I(j):  # int_{-1}^{1} T_j dx
        return 2.0 / (1.0 - j * j) if j % 2 == 0 else 0.0
    G = np.zeros((N, N))
    for m in range(N):
        for n in range(N):
            G[m, n] = 0.25 * (b - a) * (I(m + n) + I(abs(m - n)))
    return G
