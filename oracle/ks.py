"""1D Kuramoto-Sivashinsky equation on a periodic interval as a dense FP64 oracle.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

u_t + u_xx + u_xxxx + u u_x = 0 in the paper's IVP form M dX/dt + L X = F(X)
(Supplementary, "Initial value problems") with one unknown per Fourier mode:
M = 1, L_m = -k_m^2 + k_m^4, F = -1/2 d/dx (u^2) evaluated on the 3/2-padded grid
("Sparse spectral methods"; dealiasing as in the Supplementary example details).
The state is (K, 1): the stored half spectrum m = 0..K-1, K = Nx/2.
"""
import numpy as np

from . import spectral as sp


class KS:
    def __init__(self, Nx=64, L=32.0 * np.pi, dealias=1.5):
        self.Nx, self.Lx = Nx, L
        self.K = Nx // 2
        self.S = 1
        self.Ng = int(round(dealias * Nx))
        self.k = sp.fourier_wavenumbers(self.K, L)
        self.B = sp.fourier_backward_matrix(self.K, self.Ng, L)
        self.Fm = sp.fourier_forward_matrix(self.K, self.Ng, L)
        self.M = np.ones((self.K, 1, 1), dtype=complex)
        self.L = (-self.k ** 2 + self.k ** 4).astype(complex).reshape(self.K, 1, 1)

    def F(self, X):
        u = sp.fourier_backward(X[:, 0], self.B)
        sq = sp.fourier_forward(u * u, self.Fm)
        return (-0.5j * self.k * sq)[:, None]

    def F_vjp(self, X, Ybar):
        u = sp.fourier_backward(X[:, 0], self.B)
        sqb = np.conj(-0.5j * self.k) * Ybar[:, 0]
        ub = 2.0 * u * sp.fourier_forward_adjoint(sqb, self.Fm)
        return sp.fourier_backward_adjoint(ub, self.B)[:, None]

    def energy(self, X):
        """J = 1/2 (1/L) int u^2 dx = 1/2 sum_m w_m |c_m|^2 (Parseval), w_0 = 1, w_m = 2,
        with c_0 taken by its real part."""
        c = X[:, 0].copy()
        c[0] = c[0].real
        w = np.full(self.K, 2.0); w[0] = 1.0
        return 0.5 * np.sum(w * np.abs(c) ** 2)

    def energy_grad(self, X):
        c = X[:, 0].copy()
        c[0] = c[0].real
        w = np.full(self.K, 2.0); w[0] = 1.0
        return (w * c)[:, None]
