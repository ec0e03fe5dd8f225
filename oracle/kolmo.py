"""2D Kolmogorov flow (vorticity form) on the periodic square [0, 2 pi)^2 as an FP64 oracle,
optionally with a learned closure added to its explicit term.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

omega_t + u . grad omega = nu Laplacian omega - drag omega + f,  u = (d_y psi, -d_x psi),
Laplacian psi = -omega, nu = 1 / Re, f = -4 cos(4 y) (the curl of the body force sin(4y) x^).
The linear drag (bottom friction) is the usual companion of this forcing: without it the forced
flow keeps accelerating at Re = 1000 and has no statistically steady state.
IVP form M dX/dt + L X = F(X) (Supplementary, "Initial value problems") with one unknown per
Fourier mode: M = 1, L_k = nu |k|^2 + drag, F = -u . grad omega + f (+ closure), the advection on the
3/2-padded grid.  Modes, layout and transforms are those of the Swift-Hohenberg oracle
(oracle/sh.py) on L = 2 pi.  The closure evaluates the network of oracle/closure.py on the
vorticity at the N x N grid points and adds the coefficients of its output to F.

Rollout loss (the closure's training objective): J = (1/n) sum_{k=1..n} mean over the N x N
grid of (omega_k - target_k)^2, with targets given as coefficients; its direct cotangents
enter the reverse sweep at every state (injected cotangents).
"""
import numpy as np

from . import closure as cl
from . import imex
from .sh import SH


class Kolmogorov:
    def __init__(self, N, Re=1000.0, L=2.0 * np.pi, params=None, bf=True, drag=0.0):
        self.T = SH(N, 0.0, L=L, dealias=1.5)
        T = self.T
        self.N, self.Nh, self.Ng, self.Lx = N, N // 2, T.Ng, L
        self.nu = 1.0 / Re
        self.drag = drag
        self.params, self.bf = params, bf
        ky, kx = T.ky[:, None], T.kx[None, :]
        k2 = ky ** 2 + kx ** 2
        self.kx, self.ky = np.broadcast_to(kx, k2.shape), np.broadcast_to(ky, k2.shape)
        self.inv_k2 = np.where(k2 > 0, 1.0 / np.where(k2 > 0, k2, 1.0), 0.0)
        lin = np.where(T.keep, self.nu * k2 + drag, 1.0)
        self.K = N * (N // 2)
        self.S = 1
        self.M = np.ones((self.K, 1, 1), dtype=complex)
        self.L = lin.astype(complex).reshape(self.K, 1, 1)
        self.w = np.full(N // 2, 2.0)
        self.w[0] = 1.0
        f = np.zeros((N, N // 2), complex)
        iy4 = int(np.where(T.iy == 4)[0][0]) if N > 8 else None
        if iy4 is not None:
            f[iy4, 0] = -2.0
            f[int(np.where(T.iy == -4)[0][0]), 0] = -2.0
        self.f = f

    def _c(self, X):
        return X.reshape(self.N, self.Nh)

    def spectral_fields(self, c):
        psi = c * self.inv_k2
        return (1j * self.ky * psi, -1j * self.kx * psi, 1j * self.kx * c, 1j * self.ky * c)

    # -- explicit term ------------------------------------------------------------------
    def advection(self, c):
        Ng = self.Ng
        u, v, wx, wy = (self.T.to_grid(h, Ng) for h in self.spectral_fields(c))
        return self.T.from_grid(-(u * wx + v * wy), Ng)

    def closure_term(self, c):
        if self.params is None:
            return np.zeros_like(c)
        w = self.T.to_grid(c, self.N)
        y, _ = cl.forward(self.params, w, self.bf)
        return self.T.from_grid(y, self.N)

    def F(self, X):
        c = self._c(X)
        return (self.advection(c) + self.f + self.closure_term(c)).reshape(self.K, 1)

    def _Tb_t(self, v, Ng):
        """Transpose of to_grid (weighted) on an Ng grid: w_m sum_x v e^{-i k.x}."""
        return self.T.from_grid(v, Ng) * (Ng * Ng) * self.w[None, :]

    def F_vjp(self, X, Ybar, with_params=False):
        """(dF/dX)^H Ybar (real inner product of the coefficients); with_params also returns the
        closure parameters' cotangent (dF/dtheta)^H Ybar as a flat vector."""
        c, g = self._c(X), self._c(Ybar)
        Ng, N = self.Ng, self.N
        u, v, wx, wy = (self.T.to_grid(h, Ng) for h in self.spectral_fields(c))
        qb = self.T.to_grid(g, Ng, weighted=False) / (Ng * Ng)
        ub, vb, wxb, wyb = (self._Tb_t(-qb * a, Ng) for a in (wx, wy, u, v))
        cb = (np.conj(1j * self.ky * self.inv_k2) * ub + np.conj(-1j * self.kx * self.inv_k2) * vb
              + np.conj(1j * self.kx) * wxb + np.conj(1j * self.ky) * wyb)
        pb = None
        if self.params is not None:
            w = self.T.to_grid(c, N)
            yb = self.T.to_grid(g, N, weighted=False) / (N * N)
            xb, pbd = cl.vjp(self.params, w, yb, self.bf)
            cb = cb + self._Tb_t(xb, N)
            pb = cl.flatten(pbd)
        cb = np.where(self.T.keep, cb, 0.0).reshape(self.K, 1)
        return (cb, pb) if with_params else cb

    # -- loss ---------------------------------------------------------------------------
    def snapshot_loss(self, X, target):
        e = self.T.to_grid(self._c(X) - self._c(target), self.N)
        return np.mean(e * e)

    def snapshot_loss_grad(self, X, target):
        e = self.T.to_grid(self._c(X) - self._c(target), self.N)
        return self._Tb_t(2.0 * e / (self.N * self.N), self.N).reshape(self.K, 1)


def rollout_loss_and_gradients(P, X0, targets, dt, n):
    """J = (1/n) sum_{k=1..n} snapshot_loss(X_k, targets[k-1]) of an SBDF2 rollout and its
    gradients with respect to X0 and the closure parameters (the reverse sweep with injected
    cotangents, imex.sbdf_adjoint_general)."""
    XN, states = imex.sbdf_forward(P, X0, dt, n)
    J = sum(P.snapshot_loss(states[k], targets[k - 1]) for k in range(1, n + 1)) / n
    inject = [None] + [P.snapshot_loss_grad(states[k], targets[k - 1]) / n for k in range(1, n + 1)]
    g0, gp = imex.sbdf_adjoint_general(P, states, dt, inject=inject, param_vjp=P.params is not None)
    return J, g0, gp, states
