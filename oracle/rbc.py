"""2D Rayleigh-Benard convection, Fourier (x) x Chebyshev (z), as a dense FP64 oracle.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The equations are written in the paper's IVP form M dX/dt + L X = F(X)
(Supplementary, "Initial value problems"); the sparse ultraspherical
discretization with tau terms follows "Sparse spectral methods".  Readings the
paper leaves open:

* free-fall units: nu = (Ra/Pr)^(-1/2), kappa = (Ra Pr)^(-1/2); buoyancy b with
  b(z=0) = 1, b(z=1) = 0 and no-slip walls u = w = 0;
* first-order lifted-tau formulation: grad(u) is augmented by e_z lift(tau_1) with
  lift into the last C1 mode, the second tau of each field enters its C2 equation
  as the last C2 mode, the pressure gauge int p dz = 0 carries tau_p at k = 0;
* every block has S = 4N + 7 slots:
      u[0:N], w[N:2N], b[2N:3N], p[3N:4N],
      tau_u1, tau_w1, tau_b1, tau_u2, tau_w2, tau_b2, tau_p;
  equation rows use the same slot numbers: u-, w-, b-momentum (C2 coefficients),
  continuity (C1), six boundary rows u(0), u(1), w(0), w(1), b(0), b(1), and the
  gauge row (k = 0) or the row tau_p = 0 (k != 0).
"""
import numpy as np

from . import spectral as sp


class RBC:
    def __init__(self, Nx=256, Nz=64, Lx=4.0, Ra=1e6, Pr=1.0, dealias=1.5):
        assert Nx % 2 == 0
        self.Nx, self.Nz, self.Lx, self.Ra, self.Pr = Nx, Nz, Lx, Ra, Pr
        self.K = Nx // 2
        self.N = Nz
        self.S = 4 * Nz + 7
        self.nu = (Ra / Pr) ** -0.5
        self.kappa = (Ra * Pr) ** -0.5
        self.Ngx = int(round(dealias * Nx))
        self.Ngz = int(round(dealias * Nz))
        self.kx = sp.fourier_wavenumbers(self.K, Lx)
        # transforms on the dealiased grid
        self.Bx = sp.fourier_backward_matrix(self.K, self.Ngx, Lx)
        self.Fx = sp.fourier_forward_matrix(self.K, self.Ngx, Lx)
        self.Bz = sp.chebyshev_backward_matrix(self.N, self.Ngz)
        self.Fz = sp.chebyshev_forward_matrix(self.N, self.Ngz)
        # derivative d/dz within the T basis on [0, 1]: dz = 2 d/dx
        self.Dz = 2.0 * sp.cheb_derivative_T(self.N)
        self.S10 = sp.S1(self.N) @ sp.S0(self.N)
        self.M, self.L, self.Fconst = self._build_matrices()

    # ------------------------------------------------------------------ slots
    def sl(self, name):
        N = self.N
        base = {"u": 0, "w": N, "b": 2 * N, "p": 3 * N}
        if name in base:
            return slice(base[name], base[name] + N)
        taus = ["tau_u1", "tau_w1", "tau_b1", "tau_u2", "tau_w2", "tau_b2", "tau_p"]
        return 4 * N + taus.index(name)

    # ------------------------------------------------------------------ matrices
    def _build_matrices(self):
        N, K, S = self.N, self.K, self.S
        nu, ka = self.nu, self.kappa
        S0, S1, D0, D1 = sp.S0(N), sp.S1(N), sp.D0(N), sp.D1(N)
        S10 = S1 @ S0
        DZ1 = 2.0 * D0                      # d/dz: T -> C1 on [0, 1]
        DZZ = 4.0 * (D1 @ D0)               # d2/dz2: T -> C2
        SD = S1 @ DZ1                       # d/dz: T -> C2
        eN1 = np.zeros(N); eN1[N - 1] = 1.0
        eN2 = np.zeros(N); eN2[N - 2] = 1.0
        e0 = np.zeros(N); e0[0] = 1.0
        lift_dz = 4.0                        # d/dz U_{N-1}(2z-1) = 4 C2_{N-2}
        bot, top = sp.boundary_row(N, -1), sp.boundary_row(N, +1)
        integ = sp.integral_row(N, 0.0, 1.0)
        u, w, b, p = self.sl("u"), self.sl("w"), self.sl("b"), self.sl("p")
        tu1, tw1, tb1 = self.sl("tau_u1"), self.sl("tau_w1"), self.sl("tau_b1")
        tu2, tw2, tb2, tp = self.sl("tau_u2"), self.sl("tau_w2"), self.sl("tau_b2"), self.sl("tau_p")
        # equation rows share the slot numbers of the unknown blocks
        ru, rw, rb, rc = u, w, b, p
        bc_rows = [tu1, tw1, tb1, tu2, tw2, tb2]   # 6 boundary rows
        r_gauge = tp
        M = np.zeros((K, S, S), dtype=complex)
        L = np.zeros((K, S, S), dtype=complex)
        Fc = np.zeros((K, S), dtype=complex)
        for k in range(K):
            kx = self.kx[k]
            lap = DZZ - kx * kx * S10
            # mass matrix: d/dt of u, w, b in the C2 rows
            M[k][ru, u] = S10
            M[k][rw, w] = S10
            M[k][rb, b] = S10
            # x-momentum
            L[k][ru, u] = -nu * lap
            L[k][ru, p] = 1j * kx * S10
            L[k][ru, tu1] = -nu * lift_dz * eN2
            L[k][ru, tu2] = eN1
            # z-momentum
            L[k][rw, w] = -nu * lap
            L[k][rw, p] = SD
            L[k][rw, b] = -S10
            L[k][rw, tw1] = -nu * lift_dz * eN2
            L[k][rw, tw2] = eN1
            # buoyancy
            L[k][rb, b] = -ka * lap
            L[k][rb, tb1] = -ka * lift_dz * eN2
            L[k][rb, tb2] = eN1
            # continuity (C1 rows): div u + lift(tau_w1) (+ tau_p at k = 0)
            L[k][rc, u] = 1j * kx * S0
            L[k][rc, w] = DZ1
            L[k][rc, tw1] = eN1
            # boundary rows
            L[k][bc_rows[0], u] = bot
            L[k][bc_rows[1], u] = top
            L[k][bc_rows[2], w] = bot
            L[k][bc_rows[3], w] = top
            L[k][bc_rows[4], b] = bot
            L[k][bc_rows[5], b] = top
            if k == 0:
                L[k][rc, tp] = e0
                L[k][r_gauge, p] = integ
                Fc[k, bc_rows[4]] = 1.0     # b(z=0) = 1 for the horizontal mean
            else:
                L[k][r_gauge, tp] = 1.0     # tau_p = 0 away from k = 0
        return M, L, Fc

    # ------------------------------------------------------------------ transforms of (K, N) coefficient fields
    def to_grid(self, c):
        """(K, N) complex coefficients -> (Ngx, Ngz) real grid values."""
        return sp.fourier_backward(c @ self.Bz.T, self.Bx)

    def to_grid_adjoint(self, g):
        return sp.fourier_backward_adjoint(g, self.Bx) @ self.Bz

    def from_grid(self, g):
        """(Ngx, Ngz) real grid values -> (K, N) coefficients (truncating)."""
        return sp.fourier_forward(g, self.Fx) @ self.Fz.T

    def from_grid_adjoint(self, cbar):
        return sp.fourier_forward_adjoint(cbar @ self.Fz, self.Fx)

    def ddx(self, c):
        return 1j * self.kx[:, None] * c

    def ddz(self, c):
        return c @ self.Dz.T

    # ------------------------------------------------------------------ explicit term
    def _grid_fields(self, X):
        u, w, b = X[:, self.sl("u")], X[:, self.sl("w")], X[:, self.sl("b")]
        g = {}
        g["u"], g["w"] = self.to_grid(u), self.to_grid(w)
        g["ux"], g["uz"] = self.to_grid(self.ddx(u)), self.to_grid(self.ddz(u))
        g["wx"], g["wz"] = self.to_grid(self.ddx(w)), self.to_grid(self.ddz(w))
        g["bx"], g["bz"] = self.to_grid(self.ddx(b)), self.to_grid(self.ddz(b))
        return g

    def nonlinear_coeffs(self, X):
        """T coefficients (first N) of N_u, N_w, N_b = -(u.grad) of (u, w, b)."""
        g = self._grid_fields(X)
        Nu = -(g["u"] * g["ux"] + g["w"] * g["uz"])
        Nw = -(g["u"] * g["wx"] + g["w"] * g["wz"])
        Nb = -(g["u"] * g["bx"] + g["w"] * g["bz"])
        return self.from_grid(Nu), self.from_grid(Nw), self.from_grid(Nb)

    def F(self, X):
        Nu, Nw, Nb = self.nonlinear_coeffs(X)
        out = self.Fconst.copy()
        out[:, self.sl("u")] += Nu @ self.S10.T
        out[:, self.sl("w")] += Nw @ self.S10.T
        out[:, self.sl("b")] += Nb @ self.S10.T
        return out

    def F_vjp(self, X, Ybar):
        """(dF/dX)^H Ybar: transposes of the conversion, of the forward and backward
        transforms and of the derivatives, and the product rule."""
        g = self._grid_fields(X)
        # conversion S10 and forward transform, transposed
        Nub = self.from_grid_adjoint(Ybar[:, self.sl("u")] @ self.S10)
        Nwb = self.from_grid_adjoint(Ybar[:, self.sl("w")] @ self.S10)
        Nbb = self.from_grid_adjoint(Ybar[:, self.sl("b")] @ self.S10)
        # product rule
        ub = -(Nub * g["ux"] + Nwb * g["wx"] + Nbb * g["bx"])
        wb = -(Nub * g["uz"] + Nwb * g["wz"] + Nbb * g["bz"])
        uxb, uzb = -Nub * g["u"], -Nub * g["w"]
        wxb, wzb = -Nwb * g["u"], -Nwb * g["w"]
        bxb, bzb = -Nbb * g["u"], -Nbb * g["w"]
        # backward transforms and derivatives, transposed
        ikx = 1j * self.kx[:, None]
        Xb = np.zeros_like(Ybar)
        Xb[:, self.sl("u")] = (self.to_grid_adjoint(ub)
                              + np.conj(ikx) * self.to_grid_adjoint(uxb)
                              + self.to_grid_adjoint(uzb) @ self.Dz)
        Xb[:, self.sl("w")] = (self.to_grid_adjoint(wb)
                              + np.conj(ikx) * self.to_grid_adjoint(wxb)
                              + self.to_grid_adjoint(wzb) @ self.Dz)
        Xb[:, self.sl("b")] = (np.conj(ikx) * self.to_grid_adjoint(bxb)
                              + self.to_grid_adjoint(bzb) @ self.Dz)
        return Xb

    # ------------------------------------------------------------------ scale-1 grid, initial state, cost
    def scale1(self):
        """Transforms on the un-padded Nx x Nz grid used for inputs and gradients."""
        Fx = sp.fourier_forward_matrix(self.K, self.Nx, self.Lx)
        Fz = sp.chebyshev_forward_matrix(self.N, self.Nz)
        return Fx, Fz

    def grid_points(self):
        """Scale-1 grid: x_j = j Lx / Nx, z on the Nz Gauss nodes mapped to [0, 1]."""
        return sp.fourier_grid(self.Nx, self.Lx), sp.z_of_x(sp.chebyshev_nodes(self.Nz), 0.0, 1.0)

    def initial_state(self, b0_grid):
        """State with u = w = p = taus = 0 and b from its (Nx, Nz) scale-1 grid values."""
        Fx, Fz = self.scale1()
        X = np.zeros((self.K, self.S), dtype=complex)
        X[:, self.sl("b")] = sp.fourier_forward(b0_grid, Fx) @ Fz.T
        return X

    def initial_state_adjoint(self, Xbar):
        """Gradient with respect to the scale-1 grid values of b0."""
        Fx, Fz = self.scale1()
        return sp.fourier_forward_adjoint(Xbar[:, self.sl("b")] @ Fz, Fx)

    def kinetic_energy(self, X):
        """J = 1/2 int_0^Lx int_0^1 (u^2 + w^2) dz dx, exactly, from the coefficients:
        J = Lx/2 sum_k w_k Re(u_k^H G u_k + w_k^H G w_k), w_0 = 1, w_k = 2, with the
        k = 0 coefficients taken by their real parts."""
        G = sp.gram_T(self.N, 0.0, 1.0)
        wk = np.full(self.K, 2.0); wk[0] = 1.0
        J = 0.0
        for f in ("u", "w"):
            c = X[:, self.sl(f)].copy()
            c[0] = c[0].real
            J += 0.5 * self.Lx * np.sum(wk * np.real(np.einsum("km,mn,kn->k", c.conj(), G, c)))
        return J

    def kinetic_energy_grad(self, X):
        G = sp.gram_T(self.N, 0.0, 1.0)
        wk = np.full(self.K, 2.0); wk[0] = 1.0
        Xb = np.zeros_like(X)
        for f in ("u", "w"):
            c = X[:, self.sl(f)].copy()
            c[0] = c[0].real
            Xb[:, self.sl(f)] = self.Lx * wk[:, None] * (c @ G.T)
        return Xb

    # ------------------------------------------------------------------ linear boundary value problem
    # Supplementary, "Linear boundary value problems": L X = F(p), adjoint state equation
    # L^H Y = G through the same LU factors, then the VJP of F.  Here F(f) = M f + c: the steady
    # state of the IVP without its explicit term, driven by body forces and a heat source f
    # (the u, w, b blocks of a state-shaped array, T coefficients; other slots ignored) with the
    # IVP's boundary data c.  Its solution is an admissible IVP initial state (no-slip,
    # divergence-free, the IVP's buoyancy boundary values), the Cartesian counterpart of the
    # paper's LBVP-then-IVP chain.

    def lbvp_rhs(self, f):
        R = self.Fconst.copy()
        for name in ("u", "w", "b"):
            R[:, self.sl(name)] += f[:, self.sl(name)] @ self.S10.T
        return R

    def lbvp_solve(self, f):
        """X with L_k X_k = (M f + c)_k for every wavenumber k (dense LU, partial pivoting)."""
        R = self.lbvp_rhs(f)
        return np.stack([np.linalg.solve(self.L[k], R[k]) for k in range(self.K)])

    def lbvp_adjoint(self, Xbar):
        """fbar = M^H L^-H Xbar, the cotangent of f (p and tau slots zero)."""
        Y = np.stack([np.linalg.solve(self.L[k].conj().T, Xbar[k]) for k in range(self.K)])
        fb = np.zeros_like(Y)
        for name in ("u", "w", "b"):
            fb[:, self.sl(name)] = Y[:, self.sl(name)] @ self.S10
        return fb

    # ------------------------------------------------------------------ linear stability (eigenvalue problem)
    # Supplementary, "Eigenvalue problems": (lambda M + L) X = 0, the adjoint problem
    # (conj(lambda) M^H + L^H) Y = 0, and the eigenvalue sensitivity equ:eigenvalue_sens,
    # d lambda / dp = -<Y, (lambda dM/dp + dL/dp) X> / <Y, M X>.  The operator is that of a
    # perturbation of the conduction state b0 = 1 - z, u = 0: the IVP's L plus the linearized
    # advection of b0 by w (w db0/dz = -w), -S10 w in the b rows; lambda is the growth rate
    # (perturbations ~ exp(lambda t)).  M does not depend on Ra or k.

    def stability_operator(self):
        Ls = self.L.copy()
        for k in range(self.K):
            Ls[k][self.sl("b"), self.sl("w")] -= self.S10
        return Ls

    def stability_eig(self, k, sigma):
        """Eigenvalue of wavenumber k nearest sigma, with right and left (adjoint) eigenvectors,
        from the dense generalized eigenproblem L X = -lambda M X (scipy; M singular, so the
        infinite eigenvalues are dropped)."""
        import scipy.linalg as sla
        Ls = self.stability_operator()[k]
        w, vl, vr = sla.eig(Ls, -self.M[k], left=True, right=True)
        ok = np.isfinite(w)
        i = np.flatnonzero(ok)[np.argmin(np.abs(w[ok] - sigma))]
        return w[i], vr[:, i], vl[:, i]

    def stability_vector_sensitivity(self, k, lam, X, Y):
        """Eigenvector sensitivities (equ:eigenvector_sens, dM/dp = 0): for p = Ra and p = k the
        solution z of (lambda M + L_s) z = -(M dlambda/dp + dL/dp) X with <X, z> = 0, which is
        unique because the right-hand side is orthogonal to the adjoint eigenvector Y.  Solved
        as the consistent stacked system [lambda M + L_s; X^H] z = [rhs; 0] (least squares, exact
        here).  Returns the two vectors as columns."""
        A = lam * self.M[k] + self.stability_operator()[k]
        dRa, dk = self.stability_sensitivity(k, lam, X, Y)
        dLRa, dLk = self.stability_dL(k)
        out = []
        for dl, dL in ((dRa, dLRa), (dk, dLk)):
            rhs = -(dl * (self.M[k] @ X) + dL @ X)
            Ab = np.vstack([A, X.conj()[None, :]])
            z = np.linalg.lstsq(Ab, np.concatenate([rhs, [0.0]]), rcond=None)[0]
            out.append(z)
        return np.stack(out, axis=1)

    def stability_arnoldi(self, k, sigma, v0, m):
        """Several eigenvalues nearest the real shift sigma at once (Supplementary, "Eigenvalue
        problems": shift-invert about a target with a Krylov eigensolver): m steps of Arnoldi on
        B = (sigma M + L_s)^-1 M from the start vector v0, each new vector orthogonalized by
        classical Gram-Schmidt applied twice, then the eigenpairs (nu, y) of the m x m
        Hessenberg matrix.  B X = nu X turns into (lambda M + L_s) X = 0 with
        lambda = sigma - 1/nu.  Returns, ordered by decreasing |nu| (nearest sigma first): lambda,
        the Ritz vectors V_m y (unit norm) as columns, the residuals |h_{m+1,m}| |e_m^T y| of the
        pairs of B (y of unit norm), and the Arnoldi basis V (S x (m+1)) and matrix
        Hbar ((m+1) x m)."""
        import scipy.linalg as sla
        A = sigma * self.M[k] + self.stability_operator()[k]
        lu = sla.lu_factor(A)
        S = A.shape[0]
        V = np.zeros((S, m + 1), dtype=complex)
        Hbar = np.zeros((m + 1, m), dtype=complex)
        V[:, 0] = v0 / np.linalg.norm(v0)
        for j in range(m):
            w = sla.lu_solve(lu, self.M[k] @ V[:, j])
            for _ in range(2):
                h = V[:, :j + 1].conj().T @ w
                w = w - V[:, :j + 1] @ h
                Hbar[:j + 1, j] += h
            Hbar[j + 1, j] = np.linalg.norm(w)
            V[:, j + 1] = w / Hbar[j + 1, j]
        nu, Y = np.linalg.eig(Hbar[:m, :])
        order = np.argsort(-np.abs(nu), kind="stable")
        nu, Y = nu[order], Y[:, order]
        Y = Y / np.linalg.norm(Y, axis=0)
        X = V[:, :m] @ Y
        X = X / np.linalg.norm(X, axis=0)
        res = np.abs(Hbar[m, m - 1]) * np.abs(Y[m - 1, :])
        return sigma - 1.0 / nu, X, res, V, Hbar

    def _L_with(self, k, nu=None, ka=None, kx=None):
        saved = (self.nu, self.kappa, self.kx[k])
        if nu is not None:
            self.nu = nu
        if ka is not None:
            self.kappa = ka
        if kx is not None:
            self.kx[k] = kx
        _, L, _ = self._build_matrices()
        self.nu, self.kappa, self.kx[k] = saved
        return L[k]

    def param_dL(self):
        """dL/dRa and dL/dPr of every wavenumber, (K, S, S) each, exactly: L is affine in
        nu = (Ra/Pr)^(-1/2) and kappa = (Ra Pr)^(-1/2) (differences at unit and zero values), and
        dnu/dRa = -nu/(2 Ra), dnu/dPr = nu/(2 Pr), dkappa/dRa = -kappa/(2 Ra),
        dkappa/dPr = -kappa/(2 Pr).  M and F do not depend on Ra or Pr."""
        Lnu = np.array([self._L_with(k, nu=1.0, ka=0.0) - self._L_with(k, nu=0.0, ka=0.0) for k in range(self.K)])
        Lka = np.array([self._L_with(k, nu=0.0, ka=1.0) - self._L_with(k, nu=0.0, ka=0.0) for k in range(self.K)])
        nu, ka = self.nu, self.kappa
        dRa = (-0.5 * nu / self.Ra) * Lnu + (-0.5 * ka / self.Ra) * Lka
        dPr = (0.5 * nu / self.Pr) * Lnu + (-0.5 * ka / self.Pr) * Lka
        return [dRa, dPr]

    def stability_dL(self, k):
        """dL/dRa and dL/dk of wavenumber k, exactly: L is affine in nu and kappa (differences
        at unit and zero values), quadratic in k (a central difference is exact), and the
        stability coupling depends on neither."""
        Lnu = self._L_with(k, nu=1.0, ka=0.0) - self._L_with(k, nu=0.0, ka=0.0)
        Lka = self._L_with(k, nu=0.0, ka=1.0) - self._L_with(k, nu=0.0, ka=0.0)
        dnu = -0.5 * self.nu / self.Ra
        dka = -0.5 * self.kappa / self.Ra
        h = 0.5
        dLk = (self._L_with(k, kx=self.kx[k] + h) - self._L_with(k, kx=self.kx[k] - h)) / (2 * h)
        return dnu * Lnu + dka * Lka, dLk

    def stability_sensitivity(self, k, lam, X, Y):
        """(d lambda/dRa, d lambda/dk) by equ:eigenvalue_sens (dM/dp = 0)."""
        dLRa, dLk = self.stability_dL(k)
        den = np.vdot(Y, self.M[k] @ X)
        return -np.vdot(Y, dLRa @ X) / den, -np.vdot(Y, dLk @ X) / den
