"""Pins of the oracle's eigenvalue problem and eigenvalue sensitivities (Supplementary,
"Eigenvalue problems", equ:eigenvalue_sens) on the onset of Rayleigh-Benard convection between
no-slip walls: Newton steps on the growth rate with the adjoint sensitivity converge to the
textbook critical Rayleigh number 1707.762 at k = 3.1163 with a real leading eigenvalue
(exchange of stabilities) and a neutral curve with zero slope there; the sensitivities equal
central differences of the eigenvalues; the left eigenvector solves the adjoint problem.
The shift-invert Arnoldi: the Arnoldi relation and orthonormal basis, its converged Ritz
values equal the dense generalized eigenvalues nearest the shift in the same order, its Ritz
vectors solve the pencil, and its leading value at the onset has zero growth rate."""
import numpy as np

from oracle.rbc import RBC

KC, RAC = 3.1163, 1707.762


def problem(Ra, k=KC, N=32):
    return RBC(Nx=4, Nz=N, Lx=2.0 * np.pi / k, Ra=Ra, Pr=1.0)


def growth(Ra, k=KC):
    P = problem(Ra, k)
    lam, X, Y = P.stability_eig(1, 0.0)
    return P, lam, X, Y


def test_newton_on_the_growth_rate_finds_the_textbook_onset():
    Ra = 1500.0
    for _ in range(8):
        P, lam, X, Y = growth(Ra)
        dRa, _ = P.stability_sensitivity(1, lam, X, Y)
        Ra -= lam.real / dRa.real
    P, lam, X, Y = growth(Ra)
    assert abs(Ra - RAC) < 2e-3, Ra
    assert abs(lam) < 1e-12 and abs(lam.imag) < 1e-12
    # the critical wavenumber is the minimum of the neutral curve: dRa/dk = -(dl/dk)/(dl/dRa)
    dRa, dk = P.stability_sensitivity(1, lam, X, Y)
    assert abs(dk.real / dRa.real) < 0.1
    P2, lam2, X2, Y2 = growth(Ra, k=2.5)
    dRa2, dk2 = P2.stability_sensitivity(1, lam2, X2, Y2)
    assert -dk2.real / dRa2.real < -100.0      # Ra rises steeply below k_c


def test_sensitivities_equal_central_differences():
    Ra, h = 1800.0, 0.5
    P, lam, X, Y = growth(Ra, k=2.8)
    dRa, dk = P.stability_sensitivity(1, lam, X, Y)
    fd_Ra = (growth(Ra + h, k=2.8)[1] - growth(Ra - h, k=2.8)[1]) / (2 * h)
    hk = 1e-4
    fd_k = (growth(Ra, k=2.8 + hk)[1] - growth(Ra, k=2.8 - hk)[1]) / (2 * hk)
    assert abs(dRa - fd_Ra) < 1e-6 * abs(dRa)
    assert abs(dk - fd_k) < 1e-5 * abs(dk)


def test_left_eigenvector_solves_the_adjoint_problem():
    P, lam, X, Y = growth(3000.0, k=4.0)
    Ls = P.stability_operator()[1]
    r = (np.conj(lam) * P.M[1].conj().T + Ls.conj().T) @ Y
    assert np.linalg.norm(r) < 1e-11 * np.linalg.norm(Ls) * np.linalg.norm(Y)
    assert np.linalg.norm((lam * P.M[1] + Ls) @ X) < 1e-11 * np.linalg.norm(Ls) * np.linalg.norm(X)


def dense_nearest(P, k, sigma, count):
    import scipy.linalg as sla
    w = sla.eig(P.stability_operator()[k], -P.M[k], right=False)
    w = w[np.isfinite(w)]
    return w[np.argsort(np.abs(w - sigma), kind="stable")][:count]


def test_arnoldi_relation_and_orthonormal_basis():
    import workloads as wl
    P = problem(3000.0, k=2.5, N=16)
    m, sigma = 12, 0.5
    v0 = wl.random_state(7, (P.K, P.M[1].shape[0]))[1]
    lam, X, res, V, Hbar = P.stability_arnoldi(1, sigma, v0, m)
    B = np.linalg.solve(sigma * P.M[1] + P.stability_operator()[1], P.M[1])
    assert np.linalg.norm(B @ V[:, :m] - V @ Hbar) < 1e-12 * np.linalg.norm(B)
    assert np.linalg.norm(V.conj().T @ V - np.eye(m + 1)) < 1e-13
    assert np.allclose(np.tril(Hbar, -2), 0.0) and np.all(np.diag(Hbar, -1).real > 0)
    assert np.allclose(V[:, 0], v0 / np.linalg.norm(v0))


def test_arnoldi_ritz_values_are_the_eigenvalues_nearest_the_shift():
    import workloads as wl
    for Ra, k, sigma in ((5000.0, 3.0, 0.05), (3000.0, 2.5, -0.3)):
        P = problem(Ra, k=k, N=24)
        v0 = wl.random_state(8, (P.K, P.M[1].shape[0]))[1]
        lam, X, res, V, Hbar = P.stability_arnoldi(1, sigma, v0, 30)
        nu = 1.0 / (sigma - lam)
        conv = res < 1e-10 * np.abs(nu)
        nconv = int(np.argmin(conv)) if not conv.all() else len(conv)
        assert nconv >= 4, res
        ref = dense_nearest(P, 1, sigma, nconv)
        assert np.max(np.abs(lam[:nconv] - ref) / np.maximum(np.abs(ref), 1.0)) < 1e-9
        Ls, M = P.stability_operator()[1], P.M[1]
        for i in range(nconv):
            r = (lam[i] * M + Ls) @ X[:, i]
            assert np.linalg.norm(r) < 1e-7 * np.linalg.norm(Ls)


def test_arnoldi_leading_value_at_the_onset_has_zero_growth():
    import workloads as wl
    P = problem(RAC, k=KC, N=32)
    v0 = wl.random_state(9, (P.K, P.M[1].shape[0]))[1]
    lam, X, res, V, Hbar = P.stability_arnoldi(1, 0.0, v0, 20)
    assert abs(lam[0]) < 1e-6 and abs(lam[0].imag) < 1e-12
    lr, Xr, _ = P.stability_eig(1, 0.0)
    assert abs(lam[0] - lr) < 1e-12
    assert abs(abs(np.vdot(X[:, 0], Xr)) / np.linalg.norm(Xr) - 1.0) < 1e-10


def normalized_eig(P, k, sigma, X0):
    """Eigenvector nearest sigma scaled so that <X0, X> = <X0, X0>."""
    lam, X, _ = P.stability_eig(k, sigma)
    return lam, X * (np.vdot(X0, X0) / np.vdot(X0, X))


def test_eigenvector_sensitivity_equals_central_differences():
    """equ:eigenvector_sens with <X, dX/dp> = 0 is the derivative of the eigenvector normalized by
    <X(p0), X(p)> = <X(p0), X(p0)>: central differences in Ra and in k agree, and z solves the
    singular equation with a right-hand side orthogonal to Y."""
    Ra, kx, h, hk = 1800.0, 2.8, 0.5, 1e-4
    P, lam, X, Y = growth(Ra, k=kx)
    X = X / np.linalg.norm(X)
    Z = P.stability_vector_sensitivity(1, lam, X, Y)
    A = lam * P.M[1] + P.stability_operator()[1]
    dRa, dk = P.stability_sensitivity(1, lam, X, Y)
    dLRa, dLk = P.stability_dL(1)
    for i, (dl, dL) in enumerate(((dRa, dLRa), (dk, dLk))):
        rhs = -(dl * (P.M[1] @ X) + dL @ X)
        assert abs(np.vdot(Y, rhs)) < 1e-10 * np.linalg.norm(Y) * np.linalg.norm(rhs)
        assert np.linalg.norm(A @ Z[:, i] - rhs) < 1e-9 * np.linalg.norm(rhs)
        assert abs(np.vdot(X, Z[:, i])) < 1e-12 * np.linalg.norm(Z[:, i])
    Xp = normalized_eig(problem(Ra + h, k=kx), 1, lam.real, X)[1]
    Xm = normalized_eig(problem(Ra - h, k=kx), 1, lam.real, X)[1]
    fd = (Xp - Xm) / (2 * h)
    assert np.linalg.norm(fd - Z[:, 0]) < 1e-5 * np.linalg.norm(Z[:, 0])
    Xp = normalized_eig(problem(Ra, k=kx + hk), 1, lam.real, X)[1]
    Xm = normalized_eig(problem(Ra, k=kx - hk), 1, lam.real, X)[1]
    fd = (Xp - Xm) / (2 * hk)
    assert np.linalg.norm(fd - Z[:, 1]) < 1e-5 * np.linalg.norm(Z[:, 1])
