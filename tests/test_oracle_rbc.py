"""Pins of the Rayleigh-Benard oracle: textbook onset (linear operators), closed-form
diffusion at k = 0 (tau rows, boundary rows, gauge, timestepper), exact dealiased
products, the inner-product test on F, Taylor remainders and brute-force finite
differences of the full discrete gradient (Supplementary, "Verification")."""
import numpy as np
import numpy.polynomial.chebyshev as npc
import scipy.linalg as sla
import pytest

from conftest import load_golden
from oracle import imex
from oracle import spectral as sp
from oracle.rbc import RBC
import workloads as wl


def growth_rate(Ra, kx, Nz=32):
    """Largest real part of lambda in (lambda M + L_lin) X = 0 at wavenumber kx, with
    L_lin = L minus the linearized advection of the conduction profile b = 1 - z."""
    P = RBC(Nx=4, Nz=Nz, Lx=2 * np.pi / kx, Ra=Ra, Pr=1.0)
    M, L = P.M[1].copy(), P.L[1].copy()
    L[P.sl("b"), P.sl("w")] += -P.S10
    lam = sla.eig(-L, M, right=False)
    return np.max(lam[np.isfinite(lam)].real)


def test_onset_matches_textbook():
    g = {r[0]: float(r[1]) for r in load_golden("rbc_onset.txt")}
    Ra_c, k_c = g["Ra_c"], g["k_c"]
    assert growth_rate(0.97 * Ra_c, k_c) < -1e-3
    assert growth_rate(1.03 * Ra_c, k_c) > 1e-3
    # secant iterations for the root of the growth rate in Ra
    a, b = 1650.0, 1770.0
    ga, gb = growth_rate(a, k_c), growth_rate(b, k_c)
    for _ in range(4):
        a, ga, b = b, gb, b - gb * (b - a) / (gb - ga)
        gb = growth_rate(b, k_c)
    assert abs(b - Ra_c) < 0.05
    assert abs(growth_rate(Ra_c, k_c)) < 2e-5


def test_k0_diffusion_closed_form():
    """At k = 0 with u0 = A sin(pi z), b0 = 1 - z + B sin(pi z) and w = 0, the flow decays
    by pure diffusion: u = A exp(-nu pi^2 t) sin(pi z), b = 1 - z + B exp(-kappa pi^2 t)
    sin(pi z), and the gauge fixes p = z - z^2/2 - B exp(..) cos(pi z)/pi - 1/3."""
    Ra, Pr = 400.0, 2.0
    P = RBC(Nx=4, Nz=24, Lx=4.0, Ra=Ra, Pr=Pr)
    A, B, T = 0.3, 0.2, 2.0
    xq = sp.chebyshev_nodes(P.N)
    zq = sp.z_of_x(xq, 0.0, 1.0)
    Fz = sp.chebyshev_forward_matrix(P.N, P.N)
    X0 = np.zeros((P.K, P.S), dtype=complex)
    X0[0, P.sl("u")] = Fz @ (A * np.sin(np.pi * zq))
    X0[0, P.sl("b")] = Fz @ (1 - zq + B * np.sin(np.pi * zq))
    errs = []
    zt = np.linspace(0, 1, 11)
    for n in (50, 100, 200):
        XN, _ = imex.rk_forward(P, X0, T / n, n)
        u = npc.chebval(2 * zt - 1, XN[0, P.sl("u")].real)
        b = npc.chebval(2 * zt - 1, XN[0, P.sl("b")].real)
        p = npc.chebval(2 * zt - 1, XN[0, P.sl("p")].real)
        eb = B * np.exp(-P.kappa * np.pi ** 2 * T)
        ue = A * np.exp(-P.nu * np.pi ** 2 * T) * np.sin(np.pi * zt)
        be = 1 - zt + eb * np.sin(np.pi * zt)
        pe = zt - zt ** 2 / 2 - eb * np.cos(np.pi * zt) / np.pi - 1.0 / 3.0
        errs.append(max(np.abs(u - ue).max(), np.abs(b - be).max(), np.abs(p - pe).max()))
        assert np.abs(XN[0, P.sl("w")]).max() < 1e-13
        assert np.abs(XN[1:]).max() < 1e-30
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(rates - 2.0) < 0.1), (errs, rates)


def test_nonlinear_term_is_exact_dealiased_product():
    """With 3/2 padding the quadratic products of the stored modes are exact: compare with
    the products evaluated on a 4x finer grid by numpy's FFT and Chebyshev routines."""
    P = RBC(Nx=8, Nz=10, Lx=3.0, Ra=1e4, Pr=1.0)
    rng = np.random.default_rng(3)
    X = wl.random_state(4, (P.K, P.S))
    Nu, Nw, Nb = P.nonlinear_coeffs(X)
    # independent evaluation: physical fields on a fine tensor grid
    Mx, Mz = 4 * P.Nx, 4 * P.N
    x = np.arange(Mx) * P.Lx / Mx
    zx = np.cos(np.pi * (np.arange(Mz) + 0.5) / Mz)  # Gauss nodes (any order)
    kx = 2 * np.pi * np.arange(P.K) / P.Lx

    def phys(c):
        cz = np.array([npc.chebval(zx, c[k]) for k in range(P.K)])      # (K, Mz)
        pad = np.zeros((Mx // 2 + 1, Mz), dtype=complex)
        pad[:P.K] = cz
        pad[0] = pad[0].real
        return np.fft.irfft(pad, Mx, axis=0) * Mx                        # (Mx, Mz)

    def dz(c):
        return np.array([np.append(2.0 * npc.chebder(c[k]), 0.0) for k in range(P.K)])

    def coeffs(f):
        ck = np.fft.rfft(f, axis=0)[:P.K] / Mx
        return np.array([npc.chebfit(zx, ck[k].real, P.N - 1) + 1j * npc.chebfit(zx, ck[k].imag, P.N - 1)
                         for k in range(P.K)])

    u, w, b = (X[:, P.sl(f)] for f in "uwb")
    ux, wx, bx = (phys(1j * kx[:, None] * c) for c in (u, w, b))
    uz, wz, bz = (phys(dz(c)) for c in (u, w, b))
    U, W = phys(u), phys(w)
    # the products have Chebyshev degree up to 2N - 2; project them with a fine-grid fit
    def proj(f):
        ck = np.fft.rfft(f, axis=0)[:P.K] / Mx
        full = np.array([npc.chebfit(zx, ck[k].real, 2 * P.N) + 1j * npc.chebfit(zx, ck[k].imag, 2 * P.N)
                         for k in range(P.K)])
        return full[:, :P.N]
    for got, ref in ((Nu, proj(-(U * ux + W * uz))), (Nw, proj(-(U * wx + W * wz))),
                     (Nb, proj(-(U * bx + W * bz)))):
        assert np.max(np.abs(got - ref)) < 1e-11 * np.max(np.abs(ref))


def test_F_vjp_inner_product():
    """F is quadratic, so its central difference with unit step is exactly F'(X) v."""
    P = RBC(Nx=16, Nz=12, Lx=4.0, Ra=1e5, Pr=0.7)
    X = wl.random_state(10, (P.K, P.S))
    v = wl.random_state(11, (P.K, P.S))
    Yb = wl.random_state(12, (P.K, P.S), real_first_row=False)
    Fv = (P.F(X + v) - P.F(X - v)) / 2.0
    lhs = np.real(np.vdot(Yb, Fv))
    rhs = np.real(np.vdot(P.F_vjp(X, Yb), v))
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_kinetic_energy_matches_quadrature():
    P = RBC(Nx=8, Nz=10, Lx=4.0)
    X = wl.random_state(13, (P.K, P.S))
    Mx, Mz = 64, 40
    from numpy.polynomial.legendre import leggauss
    xq, wq = leggauss(Mz)
    x = np.arange(Mx) * P.Lx / Mx
    Bx = sp.fourier_backward_matrix(P.K, Mx, P.Lx)
    T = sp.chebyshev_T(P.N, xq)
    J = 0.0
    for f in "uw":
        g = sp.fourier_backward(X[:, P.sl(f)] @ T.T, Bx)
        J += 0.5 * np.sum(g ** 2 * wq[None, :]) * 0.5 * (P.Lx / Mx)
    assert abs(P.kinetic_energy(X) - J) < 1e-12 * J
    # and its gradient by the inner-product identity J(X) = 1/2 <grad, X> (homogeneous, degree 2)
    assert abs(0.5 * np.real(np.vdot(P.kinetic_energy_grad(X), X)) - P.kinetic_energy(X)) < 1e-12 * J


def gradient(P, b0, dt, n):
    X0 = P.initial_state(b0)
    XN, hist = imex.rk_forward(P, X0, dt, n)
    J = P.kinetic_energy(XN)
    g = imex.rk_adjoint(P, P.kinetic_energy_grad(XN), hist, dt)
    return J, P.initial_state_adjoint(g)


def test_taylor_remainder_rate():
    P = RBC(Nx=16, Nz=16, Lx=4.0, Ra=1e6, Pr=1.0)
    b0 = wl.rbc_b0(seed=2, Nx=16, Nz=16, amp=0.05)
    dt, n = 2e-3, 20
    J, g = gradient(P, b0, dt, n)
    d = np.random.default_rng(21).standard_normal(b0.shape)
    eps = np.array([1e-2, 5e-3, 2.5e-3, 1.25e-3])
    rem = []
    for e in eps:
        Je = P.kinetic_energy(imex.rk_forward(P, P.initial_state(b0 + e * d), dt, n)[0])
        rem.append(abs(Je - J - e * np.sum(g * d)))
    rates = np.log2(np.array(rem[:-1]) / np.array(rem[1:]))
    paper = [float(r[1]) for r in load_golden("paper_taylor_rates.txt")]
    assert min(paper) > 1.95 and max(paper) < 2.05
    assert np.all(np.abs(rates - 2.0) < 0.05), rates


def test_brute_force_finite_differences_every_component():
    P = RBC(Nx=8, Nz=8, Lx=4.0, Ra=1e5, Pr=1.0)
    b0 = wl.rbc_b0(seed=3, Nx=8, Nz=8, amp=0.3)
    dt, n = 1e-2, 3
    J, g = gradient(P, b0, dt, n)
    h = 1e-5
    fd = np.zeros_like(b0)
    for idx in np.ndindex(b0.shape):
        e = np.zeros_like(b0)
        e[idx] = h
        Jp = P.kinetic_energy(imex.rk_forward(P, P.initial_state(b0 + e), dt, n)[0])
        Jm = P.kinetic_energy(imex.rk_forward(P, P.initial_state(b0 - e), dt, n)[0])
        fd[idx] = (Jp - Jm) / (2 * h)
    assert np.max(np.abs(fd - g)) <= 1e-7 * np.max(np.abs(g))


def test_parameter_gradient_against_central_differences():
    """dJ/dRa and dJ/dPr of the kinetic energy after a few RK222 steps from the reverse sweep's
    stage adjoints (equ:efficient_gradient: minus the adjoints against the parameter derivative
    of each stage residual) against brute-force central differences of the whole forward run in
    Ra and in Pr (Richardson-extrapolated steps of 1e-3 and 5e-4 relative), on a tiny grid."""
    import workloads as wl
    from oracle import imex
    Ra, Pr, dt, n = 1e5, 0.7, 2e-3, 3

    def run(ra, pr):
        P = RBC(Nx=8, Nz=8, Lx=3.0, Ra=ra, Pr=pr)
        X0 = P.initial_state(wl.rbc_b0(seed=3, Nx=8, Nz=8, amp=0.3))
        XN, hist = imex.rk_forward(P, X0, dt, n)
        return P, XN, hist

    P, XN, hist = run(Ra, Pr)
    _, gp = imex.rk_adjoint(P, P.kinetic_energy_grad(XN), hist, dt, dLs=P.param_dL(), XN=XN)

    def J(ra, pr):
        Q, XQ, _ = run(ra, pr)
        return Q.kinetic_energy(XQ)

    for q, (dra, dpr) in enumerate(((Ra, 0.0), (0.0, Pr))):
        def cd(h):
            return (J(Ra + h * dra, Pr + h * dpr) - J(Ra - h * dra, Pr - h * dpr)) / (2 * h * (dra + dpr))
        fd = (4 * cd(5e-4) - cd(1e-3)) / 3.0
        assert abs(fd - gp[q]) <= 1e-8 * abs(gp[q]), (q, fd, gp[q])
