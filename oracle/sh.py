"""2D Swift-Hohenberg equation on a doubly periodic square as an FP64 oracle.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

u_t = r u - (1 + Laplacian)^2 u - u^3 in the paper's IVP form M dX/dt + L X = F(X)
(Supplementary, "Initial value problems") with one unknown per Fourier mode:
M = 1, L_k = -r + (1 - |k|^2)^2, F = -u^3 with the cube formed on a grid padded by 2 in
each direction (the cubic term needs twice the modes; Supplementary example details).

Modes of an N x N instance on [0, L)^2: k_x = 2 pi i_x / L for i_x < N/2 (half spectrum,
Nyquist dropped), k_y = 2 pi i_y / L for i_y in FFT order 0 .. N/2-1, -N/2+1 .. -1, the
Nyquist row i_y = N/2 kept as an unused zero.  The state is c[i_y, i_x], shape (N, N/2),
flattened to (N N/2, 1) for the timesteppers.  The real field is
u(x, y) = Re sum_{i_y, i_x} w_{i_x} c e^{i (k_x x + k_y y)},  w_0 = 1, w_{i_x >= 1} = 2.

Transforms are numpy FFTs (a library step), used as explicit sums: to_grid places the
coefficients in an Ng x (Ng/2 + 1) half spectrum and returns Ng^2 irfft2 (numpy's inverse
takes the real part of the k_x = 0 column, which is the weight-1 column above);
from_grid is rfft2 / Ng^2 restricted to the kept modes.  Both are pinned against direct
sums on small grids.  Objective: J = 1/2 mean of u^2 over the N x N grid, which equals
(1 / 2 L^2) times the integral of u^2 exactly (u^2 has no modes that alias onto the mean on
that grid).  The gradient is reported with respect to the initial grid field u0, through
X0 = from_grid(u0) on the N x N grid.
"""
import numpy as np


class SH:
    def __init__(self, N, r, L=16.0 * np.pi, dealias=2):
        assert N % 2 == 0
        self.N, self.r, self.Lx = N, r, L
        self.Ng = int(dealias * N)
        iy = np.arange(N)
        iy = np.where(iy < N // 2, iy, iy - N)          # N/2 -> -N/2: the Nyquist row
        self.iy = iy
        self.ix = np.arange(N // 2)
        self.keep = np.ones((N, N // 2), bool)
        self.keep[N // 2, :] = False                    # Nyquist row unused
        ky = 2.0 * np.pi * iy / L
        kx = 2.0 * np.pi * self.ix / L
        self.ky, self.kx = ky, kx
        k2 = ky[:, None] ** 2 + kx[None, :] ** 2
        lin = np.where(self.keep, -r + (1.0 - k2) ** 2, 1.0)   # unused slots: identity rows
        self.K = N * (N // 2)
        self.S = 1
        self.M = np.ones((self.K, 1, 1), dtype=complex)
        self.L = lin.astype(complex).reshape(self.K, 1, 1)

    # -- transforms --------------------------------------------------------------------
    def _rows(self, Ng):
        """Row index of each i_y in an Ng-point FFT-ordered spectrum."""
        return np.where(self.iy >= 0, self.iy, self.iy + Ng)

    def to_grid(self, c, Ng=None, weighted=True):
        """Grid values (Ng x Ng, [y, x]) of Re sum w c e^{i k.x}; weighted=False uses weight 1
        for every kept mode (the transpose of from_grid up to 1/Ng^2)."""
        Ng = Ng or self.Ng
        c = np.where(self.keep, c, 0.0)
        if not weighted:
            c = c.copy()
            c[:, 1:] *= 0.5
        H = np.zeros((Ng, Ng // 2 + 1), dtype=complex)
        H[self._rows(Ng), : self.N // 2] = c
        return np.fft.irfft2(H, s=(Ng, Ng)) * Ng * Ng

    def from_grid(self, u, Ng=None):
        """Kept-mode coefficients (1/Ng^2) sum u e^{-i k.x} of Ng x Ng grid values."""
        Ng = Ng or u.shape[0]
        U = np.fft.rfft2(u) / (Ng * Ng)
        c = U[self._rows(Ng), : self.N // 2]
        return np.where(self.keep, c, 0.0)

    # -- IVP pieces ---------------------------------------------------------------------
    def _c(self, X):
        return X.reshape(self.N, self.N // 2)

    def F(self, X):
        u = self.to_grid(self._c(X))
        return (-self.from_grid(u ** 3)).reshape(self.K, 1)

    def F_vjp(self, X, Ybar):
        """(dF/dX)^H Ybar with the real inner product Re(a^H b) of the coefficients:
        F = -T_f(u^3), u = T_b c, so F_vjp = T_b^T (3 u^2 T_f^T(-Ybar)), where
        T_f^T d = Re sum_k d_k e^{i k.x} / Ng^2 (weight 1) and T_b^T v = w sum_x v e^{-i k.x}."""
        u = self.to_grid(self._c(X))
        Ng = self.Ng
        ub = 3.0 * u * u * self.to_grid(-self._c(Ybar), Ng, weighted=False) / (Ng * Ng)
        w = np.full(self.N // 2, 2.0)
        w[0] = 1.0
        cb = self.from_grid(ub, Ng) * (Ng * Ng) * w[None, :]
        return cb.reshape(self.K, 1)

    # -- objective and initial transform ---------------------------------------------
    def initial_state(self, u0):
        return self.from_grid(u0, self.N).reshape(self.K, 1)

    def initial_state_adjoint(self, Xbar):
        """Transpose of initial_state: Re sum_k Xbar_k e^{i k.x} / N^2 (weight 1)."""
        return self.to_grid(self._c(Xbar), self.N, weighted=False) / (self.N * self.N)

    def energy(self, X):
        u = self.to_grid(self._c(X), self.N)
        return 0.5 * np.mean(u * u)

    def energy_grad(self, X):
        """dJ/dX = T_b^T (u / N^2) on the N x N grid."""
        N = self.N
        u = self.to_grid(self._c(X), N)
        w = np.full(N // 2, 2.0)
        w[0] = 1.0
        return (self.from_grid(u / (N * N), N) * (N * N) * w[None, :]).reshape(self.K, 1)
