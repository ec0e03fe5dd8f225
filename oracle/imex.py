"""IMEX timesteppers and their discrete adjoints, written out stage by stage.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

A problem has the initial-value form  M dX/dt + L X = F(X)  (Supplementary,
"Initial value problems").  The state X is an array of shape (K, S): K independent
blocks (one per Fourier wavenumber or mode) of S unknowns each.  A problem object
provides

    P.M, P.L        dense (K, S, S) complex matrices
    P.F(X)          explicit term, shape (K, S)
    P.F_vjp(X, Yb)  vector-Jacobian product (dF/dX)^H Yb at X, shape (K, S)

Linear systems are assembled densely per block and solved by LU with partial
pivoting; adjoint solves reuse the same factors through the conjugate transpose
(Methods, "Linear system solves").
"""
import numpy as np
import scipy.linalg as sla


# ----------------------------------------------------------------------------- dense LU per block


class BlockLU:
    """LU factors of A_k = a M_k + b L_k for every block k.  Blocks of size 1 (problems
    whose operators are diagonal in the spectral basis) are solved by the division the
    1x1 LU reduces to."""

    def __init__(self, M, L, a, b):
        A = a * M + b * L
        self.diag = A.shape[1] == 1
        if self.diag:
            self.d = A[:, 0, 0]
        else:
            self.factors = [sla.lu_factor(A[k]) for k in range(A.shape[0])]

    def solve(self, R):
        if self.diag:
            return R / self.d[:, None]
        return np.stack([sla.lu_solve(f, R[k]) for k, f in enumerate(self.factors)])

    def solve_adjoint(self, G):
        """Solve A_k^H y = g through the same factors."""
        if self.diag:
            return G / np.conj(self.d)[:, None]
        return np.stack([sla.lu_solve(f, G[k], trans=2) for k, f in enumerate(self.factors)])


def apply_blocks(A, X):
    return np.einsum("kij,kj->ki", A, X)


def apply_blocks_H(A, Y):
    return np.einsum("kji,kj->ki", A.conj(), Y)


# ----------------------------------------------------------------------------- IMEX Runge-Kutta


def ars222_tableau():
    """ARS(2,2,2) of Ascher, Ruuth & Spiteri (1997), the second-order IMEX RK scheme.

    gamma = 1 - 1/sqrt(2), delta = 1 - 1/(2 gamma).  A is the explicit tableau, H the
    implicit one; stage 0 is the step's initial state.
    """
    g = 1.0 - 1.0 / np.sqrt(2.0)
    d = 1.0 - 1.0 / (2.0 * g)
    A = np.array([[0.0, 0.0, 0.0], [g, 0.0, 0.0], [d, 1.0 - d, 0.0]])
    H = np.array([[0.0, 0.0, 0.0], [0.0, g, 0.0], [0.0, 1.0 - g, g]])
    return A, H


def ars443_tableau():
    """ARS(4,4,3) of Ascher, Ruuth & Spiteri (1997): three stages past the initial state plus
    the final one, implicit diagonal 1/2 (one matrix serves every stage), third order, both
    parts stiffly accurate (X_{n+1} is the last stage)."""
    A = np.array([[0.0, 0.0, 0.0, 0.0, 0.0],
                  [1.0 / 2.0, 0.0, 0.0, 0.0, 0.0],
                  [11.0 / 18.0, 1.0 / 18.0, 0.0, 0.0, 0.0],
                  [5.0 / 6.0, -5.0 / 6.0, 1.0 / 2.0, 0.0, 0.0],
                  [1.0 / 4.0, 7.0 / 4.0, 3.0 / 4.0, -7.0 / 4.0, 0.0]])
    H = np.array([[0.0, 0.0, 0.0, 0.0, 0.0],
                  [0.0, 1.0 / 2.0, 0.0, 0.0, 0.0],
                  [0.0, 1.0 / 6.0, 1.0 / 2.0, 0.0, 0.0],
                  [0.0, -1.0 / 2.0, 1.0 / 2.0, 1.0 / 2.0, 0.0],
                  [0.0, 3.0 / 2.0, -3.0 / 2.0, 1.0 / 2.0, 1.0 / 2.0]])
    return A, H


def rk_forward(P, X0, dt, nsteps, tableau=None):
    """IMEX RK: (M + dt H_ii L) X_{n,i} = M X_{n,0} + dt sum_{j<i} [A_ij F_{n,j} - H_ij L X_{n,j}].

    Returns the final state and the list of stage states [X_{n,0}, ..., X_{n,s-1}] of
    every step (all of them are stored; no checkpointing).
    """
    A, H = tableau if tableau is not None else ars222_tableau()
    s = A.shape[0] - 1
    lus = {}
    for i in range(1, s + 1):
        if H[i, i] not in lus:
            lus[H[i, i]] = BlockLU(P.M, P.L, 1.0, dt * H[i, i])
    X = np.array(X0, dtype=complex)
    history = []
    for _ in range(nsteps):
        Xs = [X]
        Fs = [P.F(X)]
        MX0 = apply_blocks(P.M, X)
        for i in range(1, s + 1):
            rhs = MX0.copy()
            for j in range(i):
                if A[i, j] != 0.0:
                    rhs += dt * A[i, j] * Fs[j]
                if H[i, j] != 0.0:
                    rhs -= dt * H[i, j] * apply_blocks(P.L, Xs[j])
            Xi = lus[H[i, i]].solve(rhs)
            Xs.append(Xi)
            if i < s:
                Fs.append(P.F(Xi))
        history.append(Xs[:s])
        X = Xs[s]
    return X, history


def rk_adjoint(P, Xbar_N, history, dt, tableau=None, dLs=None, XN=None):
    """Reverse sweep of the IMEX RK scheme (Supplementary, RK adjoint equations).

    With Y_{n+1,0} the cotangent of X_{n+1} = X_{n,s}:
      (M + dt H_ss L)^H Y_{n,s} = Y_{n+1,0}
      (M + dt H_ii L)^H Y_{n,i} = sum_{j>i} dt (A_ji dF_{n,i} - H_ji L)^H Y_{n,j},  0 < i < s
      Y_{n,0} = sum_{j>=1} (M^H + dt [A_j0 dF_{n,0} - H_j0 L]^H) Y_{n,j}
    and Y_{n,0} is the cotangent of X_n.  Returns dJ/dX_0 = Y_{0,0}.

    Parameter gradients (equ:efficient_gradient): with dLs a list of per-wavenumber blocks
    dL/dp (one (K, S, S) array per parameter p of L) and XN the final state, also returns
    dJ/dp = -sum_n sum_{i>=1} <Y_{n,i}, dR_{n,i}/dp>, the residual of stage i being
    R_{n,i} = (M + dt H_ii L) X_{n,i} - M X_{n,0} - dt sum_{j<i} [A_ij F_{n,j} - H_ij L X_{n,j}],
    so dR_{n,i}/dp = dt sum_{j<=i} H_ij (dL/dp) X_{n,j} with X_{n,s} = X_{n+1}; <a, b> is the
    real inner product Re(a^H b) of the state layout.  Result: (dJ/dX_0, array of dJ/dp).
    """
    A, H = tableau if tableau is not None else ars222_tableau()
    s = A.shape[0] - 1
    lus = {}
    for i in range(1, s + 1):
        if H[i, i] not in lus:
            lus[H[i, i]] = BlockLU(P.M, P.L, 1.0, dt * H[i, i])
    Ynext = np.array(Xbar_N, dtype=complex)
    grads = np.zeros(0 if dLs is None else len(dLs))
    Xend = None if dLs is None else np.array(XN, dtype=complex)
    for Xs in reversed(history):
        Y = [None] * (s + 1)
        Y[s] = lus[H[s, s]].solve_adjoint(Ynext)
        for i in range(s - 1, 0, -1):
            acc = np.zeros_like(Ynext)
            Fcot = np.zeros_like(Ynext)
            for j in range(i + 1, s + 1):
                Fcot += dt * A[j, i] * Y[j]
                if H[j, i] != 0.0:
                    acc -= dt * H[j, i] * apply_blocks_H(P.L, Y[j])
            acc += P.F_vjp(Xs[i], Fcot)
            Y[i] = lus[H[i, i]].solve_adjoint(acc)
        Y0 = np.zeros_like(Ynext)
        Fcot = np.zeros_like(Ynext)
        for j in range(1, s + 1):
            Y0 += apply_blocks_H(P.M, Y[j])
            Fcot += dt * A[j, 0] * Y[j]
            if H[j, 0] != 0.0:
                Y0 -= dt * H[j, 0] * apply_blocks_H(P.L, Y[j])
        Y0 += P.F_vjp(Xs[0], Fcot)
        if dLs is not None:
            stages = list(Xs) + [Xend]
            for q, dL in enumerate(dLs):
                for i in range(1, s + 1):
                    r = np.zeros_like(Ynext)
                    for j in range(i + 1):
                        if H[i, j] != 0.0:
                            r += dt * H[i, j] * apply_blocks(dL, stages[j])
                    grads[q] -= np.real(np.vdot(Y[i], r))
            Xend = Xs[0]
        Ynext = Y0
    if dLs is not None:
        return Ynext, grads
    return Ynext


# ----------------------------------------------------------------------------- IMEX multistep (SBDF)


# SBDF-k at a constant step (Wang & Ruuth 2008): the k-step backward difference for M dX/dt
# (a_i dt, i = 0..k) and the k-th order extrapolation of F from the previous k steps (c_i,
# i = 1..k); L is implicit at the new step only (b_0 = 1).
SBDF_ROWS = {
    1: ([1.0, -1.0], [1.0]),
    2: ([1.5, -2.0, 0.5], [2.0, -1.0]),
    3: ([11.0 / 6.0, -3.0, 1.5, -1.0 / 3.0], [3.0, -3.0, 1.0]),
    4: ([25.0 / 12.0, -4.0, 3.0, -4.0 / 3.0, 0.25], [4.0, -6.0, 4.0, -1.0]),
}


def sbdf_coefficients(n, dt, order=2):
    """Coefficients (a_i, b_i, c_i) of step n (n = 1, 2, ...) of the multistep scheme
    (a_0 M + b_0 L) X_n = sum_{i>=1} [c_i F(X_{n-i}) - (a_i M + b_i L) X_{n-i}] (equ:imex):
    SBDF-order, reverting to SBDF-n while fewer than `order` previous steps exist."""
    q = min(n, order)
    al, be = SBDF_ROWS[q]
    a = np.array(al) / dt
    b = np.zeros(q + 1)
    b[0] = 1.0
    c = np.concatenate([[0.0], be])
    return a, b, c


def sbdf_variable_coefficients(h, n, order=2):
    """Coefficients of step n for step sizes h (h[i] = t_{i+1} - t_i; step n advances from
    t_{n-1} by h[n-1]), the variable-step form of the scheme of sbdf_coefficients (equ:imex:
    coefficients that depend on the timestep, lower order while the history is short).  With
    q = min(n, order) and the nodes tau_j = t_{n-j} - t_n, j = 0..q, the row is defined by its
    order conditions: sum_j a_j tau_j^p = [p == 1] for p = 0..q (the backward difference of
    dX/dt at t_n is exact for polynomials of degree q) and sum_{i>=1} c_i tau_i^p = [p == 0]
    for p = 0..q-1 (F extrapolated to t_n exactly for degree q - 1), solved as Vandermonde
    systems."""
    q = min(n, order)
    tau = np.zeros(q + 1)
    for j in range(1, q + 1):
        tau[j] = tau[j - 1] - h[n - j]
    V = np.vander(tau, q + 1, increasing=True).T          # V[p, j] = tau_j^p
    rhs = np.zeros(q + 1)
    rhs[1] = 1.0
    a = np.linalg.solve(V, rhs)
    W = np.vander(tau[1:], q, increasing=True).T          # W[p, i] = tau_i^p
    e0 = np.zeros(q)
    e0[0] = 1.0
    c = np.concatenate([[0.0], np.linalg.solve(W, e0)])
    b = np.zeros(q + 1)
    b[0] = 1.0
    return a, b, c


def _coefficients(n, dt, order):
    """Row of step n: constant step (scalar dt) or the variable-step row (dt a sequence)."""
    if np.ndim(dt) == 0:
        return sbdf_coefficients(n, dt, order)
    return sbdf_variable_coefficients(dt, n, order)


def sbdf_forward(P, X0, dt, nsteps, order=2):
    """Multistep IMEX forward run; returns X_N and all states [X_0, ..., X_N].  dt is the
    constant step or the sequence of step sizes (one LU per distinct a_0, rebuilt when the
    step changes)."""
    states = [np.array(X0, dtype=complex)]
    Fs = [P.F(states[0])]
    lus = {}
    for n in range(1, nsteps + 1):
        a, b, c = _coefficients(n, dt, order)
        key = (a[0], b[0])
        if key not in lus:
            lus[key] = BlockLU(P.M, P.L, a[0], b[0])
        rhs = np.zeros_like(states[0])
        for i in range(1, len(a)):
            Xi = states[n - i]
            rhs += c[i] * Fs[n - i] - a[i] * apply_blocks(P.M, Xi) - b[i] * apply_blocks(P.L, Xi)
        Xn = lus[key].solve(rhs)
        states.append(Xn)
        Fs.append(P.F(Xn) if n < nsteps else None)
    return states[-1], states


def sbdf_adjoint(P, Xbar_N, states, dt, order=2):
    """Reverse sweep of the multistep scheme (Supplementary, multistep adjoint equation),
    in accumulated-cotangent form: with Xbar_N = dJ/dX_N, for n = N..1 solve
    (a_0^n M + b_0^n L)^H Y_n = Xbar_n, then for each i >= 1 add
    (c_i^n dF(X_{n-i}) - (a_i^n M + b_i^n L))^H Y_n into Xbar_{n-i}.  Returns Xbar_0."""
    N = len(states) - 1
    Xbar = [np.zeros_like(states[0]) for _ in range(N + 1)]
    Xbar[N] = np.array(Xbar_N, dtype=complex)
    lus = {}
    for n in range(N, 0, -1):
        a, b, c = _coefficients(n, dt, order)
        key = (a[0], b[0])
        if key not in lus:
            lus[key] = BlockLU(P.M, P.L, a[0], b[0])
        Y = lus[key].solve_adjoint(Xbar[n])
        for i in range(1, len(a)):
            Xbar[n - i] += P.F_vjp(states[n - i], c[i] * Y)
            Xbar[n - i] -= a[i] * apply_blocks_H(P.M, Y) + b[i] * apply_blocks_H(P.L, Y)
    return Xbar[0]


def sbdf_adjoint_general(P, states, dt, Xbar_N=None, inject=None, param_vjp=False, order=2):
    """The multistep reverse sweep of sbdf_adjoint with two additions: cotangents inject[k]
    that a cost depending on intermediate states X_k adds to Xbar_k (entering before the solve
    of step k), and, with param_vjp, the gradient with respect to parameters of F,
    sum over steps n and i >= 1 of (dF/dp (X_{n-i}))^H c_i^n Y_n (equ:efficient_gradient),
    from P.F_vjp(X, Ybar, with_params=True).  Returns (Xbar_0, pbar)."""
    N = len(states) - 1
    Xbar = [np.zeros_like(states[0]) for _ in range(N + 1)]
    if Xbar_N is not None:
        Xbar[N] += Xbar_N
    pbar = None
    lus = {}
    for n in range(N, 0, -1):
        if inject is not None and inject[n] is not None:
            Xbar[n] += inject[n]
        a, b, c = _coefficients(n, dt, order)
        key = (a[0], b[0])
        if key not in lus:
            lus[key] = BlockLU(P.M, P.L, a[0], b[0])
        Y = lus[key].solve_adjoint(Xbar[n])
        for i in range(1, len(a)):
            if param_vjp:
                v, pv = P.F_vjp(states[n - i], c[i] * Y, with_params=True)
                pbar = pv if pbar is None else pbar + pv
            else:
                v = P.F_vjp(states[n - i], c[i] * Y)
            Xbar[n - i] += v
            Xbar[n - i] -= a[i] * apply_blocks_H(P.M, Y) + b[i] * apply_blocks_H(P.L, Y)
    if inject is not None and inject[0] is not None:
        Xbar[0] += inject[0]
    return Xbar[0], pbar
