"""3D plane Couette flow, Fourier (x) x Fourier (z) x Chebyshev (y), as a dense FP64 oracle.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Perturbation u = (u, v, w) of the laminar flow U = y between walls y = -1, +1 moving with
U = -1, +1, on [0, Lx) x [-1, 1] x [0, Lz), viscosity nu = 1/Re:
    u_t + (u.grad) u + U u_x + v U' e_x + grad p - nu Laplacian u = 0,   div u = 0,
    u = 0 at y = -1, +1.
IVP form M dX/dt + L X = F(X) (Supplementary, "Initial value problems"): the Stokes part
(time derivative, viscous term, pressure gradient, continuity, boundary and gauge rows) is
implicit, F = -(u.grad) u - U u_x - v U' e_x (products on the 3/2 padded grid).  The
tau formulation is the first-order lifted one of oracle/rbc.py on [-1, 1]:
    slots per mode: u[0:N], v[N:2N], w[2N:3N], p[3N:4N],
                    tau_u1, tau_v1, tau_w1, tau_u2, tau_v2, tau_w2, tau_p;
    momentum rows (C2): S10 u_t - nu (DYY - k^2 S10) u + (pressure gradient) S10
                         - 2 nu lift(tau_1) + tau_2 e_{N-1};
    continuity (C1): i kx S0 u + D0 v + i kz S0 w + tau_v1 e_{N-1} (+ tau_p e_0 at k = 0);
    six wall rows, and the gauge int p dy = 0 at k = 0 (tau_p = 0 elsewhere).
Modes: kx = 2 pi m / Lx for m < Nx/2 (half spectrum), kz = 2 pi n / Lz for n < Nz in FFT order;
mode index k = m Nz + n.  The z Nyquist mode n = Nz/2 is kept as an unforced mode (its
explicit term is zero).  Grid values are u(x, y, z) = Re sum_k w_m c_k(y) e^{i(kx x + kz z)}
(w_0 = 1, w_m = 2); transforms use numpy FFTs (a library step) with explicit padding.
Cost: J = 1/2 int |u|^2 dV = 1/2 Lx Lz sum_k w_m int_{-1}^{1} Re(c_k^H c_k) dy over u, v, w,
the k = 0 coefficients taken by their real parts, z Nyquist modes excluded (the energy of the
field for states whose m = 0 modes are Hermitian in n).
"""
import numpy as np

from . import spectral as sp


class Couette:
    def __init__(self, Nx, Ny, Nz, Lx=4.0 * np.pi, Lz=2.0 * np.pi, Re=400.0, dealias=1.5):
        assert Nx % 2 == 0 and Nz % 2 == 0
        self.Nx, self.Ny, self.Nz, self.Lx, self.Lz, self.Re = Nx, Ny, Nz, Lx, Lz, Re
        self.Kx = Nx // 2
        self.N = Ny
        self.K = self.Kx * Nz
        self.S = 4 * Ny + 7
        self.nu = 1.0 / Re
        self.Ngx = int(round(dealias * Nx))
        self.Ngy = int(round(dealias * Ny))
        self.Ngz = int(round(dealias * Nz))
        m = np.arange(self.Kx)
        n = np.arange(Nz)
        ns = np.where(n < Nz // 2, n, n - Nz)
        self.kx = np.repeat(2.0 * np.pi * m / Lx, Nz)           # per mode k = m Nz + n
        self.kz = np.tile(2.0 * np.pi * ns / Lz, self.Kx)
        self.m = np.repeat(m, Nz)
        self.ns = np.tile(ns, self.Kx)
        self.keep = np.tile(n != Nz // 2, self.Kx)               # z Nyquist: unforced
        self.By = sp.chebyshev_backward_matrix(Ny, self.Ngy)
        self.Fy = sp.chebyshev_forward_matrix(Ny, self.Ngy)
        self.Dy = sp.cheb_derivative_T(Ny)                        # d/dy within T on [-1, 1]
        self.S10 = sp.S1(Ny) @ sp.S0(Ny)
        self.y = sp.chebyshev_nodes(self.Ngy)                    # ascending Gauss nodes
        self.M, self.L = self._build_matrices()

    # ------------------------------------------------------------------ slots
    def sl(self, name):
        N = self.N
        base = {"u": 0, "v": N, "w": 2 * N, "p": 3 * N}
        if name in base:
            return slice(base[name], base[name] + N)
        taus = ["tau_u1", "tau_v1", "tau_w1", "tau_u2", "tau_v2", "tau_w2", "tau_p"]
        return 4 * N + taus.index(name)

    def _build_matrices(self):
        N, K, S, nu = self.N, self.K, self.S, self.nu
        S0, S1, D0, D1 = sp.S0(N), sp.S1(N), sp.D0(N), sp.D1(N)
        S10 = S1 @ S0
        DYY = D1 @ D0                     # d2/dy2: T -> C2 on [-1, 1]
        SD = S1 @ D0                      # d/dy: T -> C2
        eN1 = np.zeros(N); eN1[N - 1] = 1.0
        eN2 = np.zeros(N); eN2[N - 2] = 1.0
        e0 = np.zeros(N); e0[0] = 1.0
        lift_dy = 2.0                     # d/dy U_{N-1}(y) = 2 C2_{N-2}(y)
        bot, top = sp.boundary_row(N, -1), sp.boundary_row(N, +1)
        integ = sp.integral_row(N, -1.0, 1.0)
        u, v, w, p = self.sl("u"), self.sl("v"), self.sl("w"), self.sl("p")
        t1 = [self.sl("tau_u1"), self.sl("tau_v1"), self.sl("tau_w1")]
        t2 = [self.sl("tau_u2"), self.sl("tau_v2"), self.sl("tau_w2")]
        tp = self.sl("tau_p")
        M = np.zeros((K, S, S), dtype=complex)
        L = np.zeros((K, S, S), dtype=complex)
        for k in range(K):
            kx, kz = self.kx[k], self.kz[k]
            lap = DYY - (kx * kx + kz * kz) * S10
            grads = [1j * kx * S10, SD, 1j * kz * S10]
            for f, blk in enumerate((u, v, w)):
                M[k][blk, blk] = S10
                L[k][blk, blk] = -nu * lap
                L[k][blk, p] = grads[f]
                L[k][blk, t1[f]] = -nu * lift_dy * eN2
                L[k][blk, t2[f]] = eN1
            # continuity (C1 rows, in the slots of p)
            L[k][p, u] = 1j * kx * S0
            L[k][p, v] = D0
            L[k][p, w] = 1j * kz * S0
            L[k][p, t1[1]] = eN1
            # wall rows: field f at y = -1 (row tau_f1) and y = +1 (row tau_f2)
            for f, blk in enumerate((u, v, w)):
                L[k][t1[f], blk] = bot
                L[k][t2[f], blk] = top
            if k == 0:
                L[k][p, tp] = e0
                L[k][tp, p] = integ
            else:
                L[k][tp, tp] = 1.0
        return M, L

    # ------------------------------------------------------------------ transforms of (K, N) fields
    def _rows_z(self):
        n = self.ns
        return np.where(n >= 0, n, n + self.Ngz)

    def to_grid(self, c):
        """(K, N) coefficients -> grid values [y, z, x] (Ngy, Ngz, Ngx)."""
        cy = c @ self.By.T                                         # (K, Ngy)
        H = np.zeros((self.Ngy, self.Ngz, self.Ngx // 2 + 1), dtype=complex)
        kk = np.nonzero(self.keep)[0]
        H[:, self._rows_z()[kk], self.m[kk]] = cy[kk].T
        return np.fft.irfft2(H, s=(self.Ngz, self.Ngx), axes=(1, 2)) * (self.Ngz * self.Ngx)

    def from_grid(self, g):
        """Grid values [y, z, x] -> (K, N) coefficients (truncating; z Nyquist zero)."""
        U = np.fft.rfft2(g, axes=(1, 2)) / (self.Ngz * self.Ngx)
        cy = U[:, self._rows_z(), self.m].T                        # (K, Ngy)
        cy = np.where(self.keep[:, None], cy, 0.0)
        return cy @ self.Fy.T

    def to_grid_adjoint(self, gbar):
        """Transpose of to_grid for the real inner products: w_m sum over grid e^{-i k.x}."""
        U = np.fft.rfft2(gbar, axes=(1, 2))                       # sum g e^{-i k.x}
        cy = U[:, self._rows_z(), self.m].T
        wm = np.where(self.m == 0, 1.0, 2.0)
        cy = np.where(self.keep[:, None], cy * wm[:, None], 0.0)
        return cy @ self.By

    def from_grid_adjoint(self, cbar):
        """Transpose of from_grid: Re sum_k (Fy^T cbar)_k e^{i k.x} / (Ngz Ngx) (weight 1)."""
        cy = cbar @ self.Fy                                        # (K, Ngy)
        cy = np.where(self.keep[:, None], cy, 0.0).astype(complex)
        cy[self.m >= 1] *= 0.5
        H = np.zeros((self.Ngy, self.Ngz, self.Ngx // 2 + 1), dtype=complex)
        H[:, self._rows_z(), self.m] = cy.T
        return np.fft.irfft2(H, s=(self.Ngz, self.Ngx), axes=(1, 2))

    # ------------------------------------------------------------------ explicit term
    def _fields(self, X):
        g = {}
        ikx, ikz = 1j * self.kx[:, None], 1j * self.kz[:, None]
        for f in ("u", "v", "w"):
            c = X[:, self.sl(f)]
            g[f] = self.to_grid(c)
            g[f + "x"] = self.to_grid(ikx * c)
            g[f + "y"] = self.to_grid(c @ self.Dy.T)
            g[f + "z"] = self.to_grid(ikz * c)
        return g

    def products(self, X):
        """Grid values of the explicit-term densities N_u, N_v, N_w."""
        g = self._fields(X)
        U = self.y[:, None, None]
        out = []
        for f in ("u", "v", "w"):
            n = -(g["u"] * g[f + "x"] + g["v"] * g[f + "y"] + g["w"] * g[f + "z"]) - U * g[f + "x"]
            if f == "u":
                n = n - g["v"]                                     # v U', U' = 1
            out.append(n)
        return out

    def F(self, X):
        out = np.zeros_like(X)
        for f, n in zip(("u", "v", "w"), self.products(X)):
            out[:, self.sl(f)] = self.from_grid(n) @ self.S10.T
        return out

    def F_vjp(self, X, Ybar):
        """(dF/dX)^H Ybar: transposes of the conversion, the forward and backward transforms and
        the derivatives, and the product rule of the densities."""
        g = self._fields(X)
        U = self.y[:, None, None]
        nb = {f: self.from_grid_adjoint(Ybar[:, self.sl(f)] @ self.S10) for f in ("u", "v", "w")}
        gb = {}
        for a in ("u", "v", "w"):
            gb[a] = -(nb["u"] * g["u" + _d(a)] + nb["v"] * g["v" + _d(a)] + nb["w"] * g["w" + _d(a)])
        gb["v"] = gb["v"] - nb["u"]                                # from -v U' in N_u
        for f in ("u", "v", "w"):
            gb[f + "x"] = -nb[f] * (g["u"] + U)
            gb[f + "y"] = -nb[f] * g["v"]
            gb[f + "z"] = -nb[f] * g["w"]
        ikx, ikz = 1j * self.kx[:, None], 1j * self.kz[:, None]
        Xb = np.zeros_like(Ybar)
        for f in ("u", "v", "w"):
            Xb[:, self.sl(f)] = (self.to_grid_adjoint(gb[f])
                                 + np.conj(ikx) * self.to_grid_adjoint(gb[f + "x"])
                                 + self.to_grid_adjoint(gb[f + "y"]) @ self.Dy
                                 + np.conj(ikz) * self.to_grid_adjoint(gb[f + "z"]))
        return Xb

    # ------------------------------------------------------------------ cost
    def energy(self, X):
        G = sp.gram_T(self.N, -1.0, 1.0)                          # int_{-1}^{1} T_a T_b dy
        wm = np.where(self.m == 0, 1.0, 2.0) * self.keep
        J = 0.0
        for f in ("u", "v", "w"):
            c = X[:, self.sl(f)].copy()
            c[0] = c[0].real
            J += 0.5 * self.Lx * self.Lz * np.sum(wm * np.real(np.einsum("km,mn,kn->k", c.conj(), G, c)))
        return J

    def energy_grad(self, X):
        G = sp.gram_T(self.N, -1.0, 1.0)
        wm = np.where(self.m == 0, 1.0, 2.0) * self.keep
        Xb = np.zeros_like(X)
        for f in ("u", "v", "w"):
            c = X[:, self.sl(f)].copy()
            c[0] = c[0].real
            Xb[:, self.sl(f)] = self.Lx * self.Lz * wm[:, None] * (c @ G.T)
        return Xb


def _d(a):
    return {"u": "x", "v": "y", "w": "z"}[a]
