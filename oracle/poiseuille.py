"""Linear stability of plane Poiseuille flow as a dense FP64 oracle: the eigenvalue problem of
the paper's neutral-curve example (Results, "Parametric sensitivity and numerical
continuation"; Supplementary, "Eigenvalue problems": equ:eigenvalue_sens).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Flow between walls y = 0 and y = 2 with base flow U = y (2 - y) along x at Reynolds number Re.
Two-dimensional perturbations (u, v, p) ~ exp(i alpha x + lambda t) of streamwise wavenumber
alpha satisfy

    lambda u + i alpha U u + U' v + i alpha p - (1/Re) (D^2 - alpha^2) u = 0
    lambda v + i alpha U v        + D p       - (1/Re) (D^2 - alpha^2) v = 0
    i alpha u + D v = 0,          u = v = 0 at both walls,

i.e. (lambda M + L) X = 0 with Re(lambda) the growth rate.  Readings the paper leaves open:

* with x = y - 1 in [-1, 1] (D = d/dx, U = 1 - x^2, U' = -2 x) the unknowns are Chebyshev-T
  series and the equations use the ultraspherical method of the 2D problem (oracle/rbc.py):
  momentum rows in C2 coefficients, continuity in C1, first-order lifted taus (the first tau
  of u and v lifted into the last C1 mode of their gradient, the second entering the momentum
  row as the last C2 mode, the first tau of v also lifted into continuity), four boundary rows
  and, alpha being nonzero, the row tau_p = 0;
* products with the polynomial base flow are exact: a row holds the first N C2 coefficients of
  the product series (degree N + 1), not a product of truncated matrices;
* slots (S = 3N + 5): u[0:N], v[N:2N], p[2N:3N], tau_u1, tau_v1, tau_u2, tau_v2, tau_p;
  equation rows use the same slot numbers (u- and v-momentum, continuity, boundary rows
  u(-1), u(1), v(-1), v(1), the tau_p row).
"""
import numpy as np
import scipy.linalg as sla

from . import spectral as sp


def mult_x(N):
    """Multiplication by x of a T series of N terms, exactly: an (N + 1) x N matrix
    (x T_0 = T_1, x T_n = (T_{n+1} + T_{n-1}) / 2)."""
    A = np.zeros((N + 1, N))
    A[1, 0] = 1.0
    for n in range(1, N):
        A[n + 1, n] += 0.5
        A[n - 1, n] += 0.5
    return A


def S10_ext(N):
    """T -> C2 conversion of a series of N terms (the square N x N conversion)."""
    return sp.S1(N) @ sp.S0(N)


class Poiseuille:
    def __init__(self, N=64):
        self.N = N
        self.S = 3 * N + 5
        S0, S1, D0, D1 = sp.S0(N), sp.S1(N), sp.D0(N), sp.D1(N)
        self.S10 = S1 @ S0
        self.S0m = S0
        self.DZ1 = D0                    # d/dx: T -> C1
        self.DZZ = D1 @ D0               # d2/dx2: T -> C2
        self.SD = S1 @ D0                # d/dx: T -> C2
        # base-flow products (first N C2 coefficients of exact product series)
        X1 = mult_x(N)                            # (N+1) x N
        X2 = mult_x(N + 1) @ X1                   # (N+2) x N: x^2
        Uext = np.eye(N + 2, N) - X2              # U = 1 - x^2
        self.SU = (S10_ext(N + 2) @ Uext)[:N]     # C2 coefficients of U u
        self.SdU = (S10_ext(N + 1) @ (-2.0 * X1))[:N]   # C2 coefficients of U' v

    def sl(self, name):
        N = self.N
        base = {"u": 0, "v": N, "p": 2 * N}
        if name in base:
            return slice(base[name], base[name] + N)
        taus = ["tau_u1", "tau_v1", "tau_u2", "tau_v2", "tau_p"]
        return 3 * N + taus.index(name)

    def matrices(self, alpha, Re):
        """Dense (M, L) of wavenumber alpha at Reynolds number Re."""
        N, S = self.N, self.S
        nu = 1.0 / Re
        M = np.zeros((S, S), dtype=complex)
        L = np.zeros((S, S), dtype=complex)
        u, v, p = self.sl("u"), self.sl("v"), self.sl("p")
        tu1, tv1, tu2, tv2, tp = (self.sl(n) for n in ("tau_u1", "tau_v1", "tau_u2", "tau_v2", "tau_p"))
        ru, rv, rc = u, v, p
        eN1 = np.zeros(N); eN1[N - 1] = 1.0
        eN2 = np.zeros(N); eN2[N - 2] = 1.0
        lift_dz = 2.0                     # d/dx U_{N-1}(x) = 2 C2_{N-2}
        lap = self.DZZ - alpha * alpha * self.S10
        M[ru, u] = self.S10
        M[rv, v] = self.S10
        # u-momentum
        L[ru, u] = 1j * alpha * self.SU - nu * lap
        L[ru, v] = self.SdU
        L[ru, p] = 1j * alpha * self.S10
        L[ru, tu1] = -nu * lift_dz * eN2
        L[ru, tu2] = eN1
        # v-momentum
        L[rv, v] = 1j * alpha * self.SU - nu * lap
        L[rv, p] = self.SD
        L[rv, tv1] = -nu * lift_dz * eN2
        L[rv, tv2] = eN1
        # continuity
        L[rc, u] = 1j * alpha * self.S0m
        L[rc, v] = self.DZ1
        L[rc, tv1] = eN1
        # boundary rows and the tau_p row
        bot, top = sp.boundary_row(N, -1), sp.boundary_row(N, +1)
        L[tu1, u] = bot
        L[tv1, u] = top
        L[tu2, v] = bot
        L[tv2, v] = top
        L[tp, tp] = 1.0
        return M, L

    def dL(self, alpha, Re):
        """(dL/dRe, dL/dalpha), exactly: L is affine in nu = 1/Re (a difference at nu-values
        1 and 0, times dnu/dRe = -1/Re^2) and quadratic in alpha (a central difference)."""
        _, L1 = self.matrices(alpha, 1.0)
        _, Linf = self.matrices(alpha, np.inf)
        dRe = -(L1 - Linf) / (Re * Re)
        h = 0.5
        dal = (self.matrices(alpha + h, Re)[1] - self.matrices(alpha - h, Re)[1]) / (2.0 * h)
        return dRe, dal

    def eig(self, alpha, Re, sigma):
        """The eigenvalue nearest sigma with right and left (adjoint) eigenvectors, from the
        dense generalized problem L X = -lambda M X (M singular: infinite eigenvalues dropped)."""
        M, L = self.matrices(alpha, Re)
        w, vl, vr = sla.eig(L, -M, left=True, right=True)
        ok = np.isfinite(w)
        i = np.flatnonzero(ok)[np.argmin(np.abs(w[ok] - sigma))]
        return w[i], vr[:, i], vl[:, i]

    def eigenvalues(self, alpha, Re):
        M, L = self.matrices(alpha, Re)
        w = sla.eigvals(L, -M)
        return w[np.isfinite(w)]

    def sensitivity(self, alpha, Re, X, Y):
        """(dlambda/dRe, dlambda/dalpha) by equ:eigenvalue_sens (M does not depend on either):
        -<Y, dL/dp X> / <Y, M X>."""
        M, _ = self.matrices(alpha, Re)
        dRe, dal = self.dL(alpha, Re)
        den = np.vdot(Y, M @ X)
        return -np.vdot(Y, dRe @ X) / den, -np.vdot(Y, dal @ X) / den

    def neutral_Re(self, alpha, Re0, sigma0, tol=1e-14, maxit=20):
        """Newton on the growth rate Re(lambda)(Re) = 0 at fixed alpha, the derivative from the
        eigenvalue sensitivity, each solve targeting the previous eigenvalue.  Returns
        (Re, lambda, number of eigenvalue solves, history of (Re, lambda))."""
        Re, sigma, hist = Re0, sigma0, []
        for it in range(1, maxit + 1):
            lam, X, Y = self.eig(alpha, Re, sigma)
            hist.append((Re, lam))
            if abs(lam.real) <= tol:
                return Re, lam, it, hist
            dRe, _ = self.sensitivity(alpha, Re, X, Y)
            Re = Re - lam.real / dRe.real
            sigma = lam
        return Re, lam, maxit, hist
