"""Pins of the oracle's linear boundary value problem L X = M f + c (the steady state of the
Rayleigh-Benard IVP without its explicit term) and of its adjoint (Supplementary, "Linear
boundary value problems"): closed-form steady solutions at k = 0, a manufactured polynomial
solution at k != 0 that the tau method must reproduce exactly, the dot-product test of the
adjoint, and the gradient of an IVP cost through the LBVP-then-IVP chain against central
differences."""
import numpy as np
from numpy.polynomial import Chebyshev, Polynomial

import workloads as wl
from oracle import imex
from oracle.rbc import RBC


def cheb01(p, N):
    """First N Chebyshev coefficients on [0, 1] of a polynomial given in powers of z."""
    c = Polynomial(p, domain=[0, 1], window=[0, 1]).convert(kind=Chebyshev, domain=[0, 1]).coef
    out = np.zeros(N, dtype=complex)
    out[: len(c)] = c
    return out


def test_k0_steady_stokes_and_conduction_closed_form():
    """At k = 0 a uniform force c on u gives u = c z (1 - z) / (2 nu), w = 0, the conduction
    profile b = 1 - z, and the hydrostatic pressure p = z - z^2/2 - 1/3 (p' = b, zero mean)."""
    P = RBC(Nx=8, Nz=12, Lx=3.0, Ra=1e5, Pr=0.7)
    N = P.N
    c = 0.37
    f = np.zeros((P.K, P.S), dtype=complex)
    f[0, P.sl("u")][0] = c
    X = P.lbvp_solve(f)
    u_ref = cheb01([0.0, c / (2 * P.nu), -c / (2 * P.nu)], N)
    b_ref = cheb01([1.0, -1.0], N)
    p_ref = cheb01([-1.0 / 3.0, 1.0, -0.5], N)
    scale = np.abs(u_ref).max()
    assert np.abs(X[0, P.sl("u")] - u_ref).max() < 1e-12 * scale
    assert np.abs(X[0, P.sl("w")]).max() < 1e-12 * scale
    assert np.abs(X[0, P.sl("b")] - b_ref).max() < 1e-12
    assert np.abs(X[0, P.sl("p")] - p_ref).max() < 1e-12
    assert np.abs(X[0, 4 * N:]).max() < 1e-10 * scale
    # no forcing and homogeneous boundary data: every other wavenumber stays at rest
    assert np.abs(X[1:]).max() < 1e-14


def test_manufactured_solution_at_nonzero_wavenumber():
    """Streamfunction psi = z^2 (1 - z)^2 at wavenumber kx: u = psi', w = -i kx psi is
    divergence-free and no-slip; with p = z^3 - z and b = z (1 - z) the forcing
    f_u = -nu (u'' - kx^2 u) + i kx p, f_w = -nu (w'' - kx^2 w) + p' - b,
    f_b = -kappa (b'' - kx^2 b) is polynomial, so the tau solution is the manufactured one with
    zero taus."""
    P = RBC(Nx=12, Nz=12, Lx=2.5, Ra=3e4, Pr=0.9)
    N = P.N
    psi = Polynomial([0, 0, 1, -2, 1])
    p = Polynomial([0, -1, 0, 1])
    b = Polynomial([0, 1, -1])
    for k in (1, 4):
        kx = P.kx[k]
        u = psi.deriv()
        w_c = -1j * kx   # w = w_c psi
        fu = [-P.nu * (u.deriv(2) - kx ** 2 * u), 1j * kx * p]
        fw = [-P.nu * w_c * (psi.deriv(2) - kx ** 2 * psi), p.deriv(), -b]
        fb = -P.kappa * (b.deriv(2) - kx ** 2 * b)
        f = np.zeros((P.K, P.S), dtype=complex)
        f[k, P.sl("u")] = cheb01(fu[0].coef, N) + cheb01(fu[1].coef, N)
        f[k, P.sl("w")] = sum(cheb01(q.coef, N) for q in fw)
        f[k, P.sl("b")] = cheb01(fb.coef, N)
        X = P.lbvp_solve(f)
        ref = {"u": cheb01(u.coef, N), "w": w_c * cheb01(psi.coef, N), "b": cheb01(b.coef, N),
               "p": cheb01(p.coef, N)}
        for name, r in ref.items():
            assert np.abs(X[k, P.sl(name)] - r).max() < 1e-12 * max(1.0, np.abs(r).max()), (k, name)
        assert np.abs(X[k, 4 * N:]).max() < 1e-11
        # k = 0 keeps the conduction state, every other wavenumber stays at rest
        assert np.abs(X[0, P.sl("b")] - cheb01([1.0, -1.0], N)).max() < 1e-12
        rest = [j for j in range(1, P.K) if j != k]
        assert np.abs(X[rest]).max() < 1e-14


def test_adjoint_dot_product():
    """<G, X(f) - X(0)> = <fbar, f> with fbar = lbvp_adjoint(G) (the map f -> X is affine)."""
    P = RBC(Nx=16, Nz=14, Lx=3.0, Ra=2e5, Pr=1.3)
    f = wl.random_state(21, (P.K, P.S))
    G = wl.random_state(22, (P.K, P.S), real_first_row=False)
    dX = P.lbvp_solve(f) - P.lbvp_solve(np.zeros_like(f))
    fb = P.lbvp_adjoint(G)
    lhs = np.real(np.vdot(G, dX))
    rhs = np.real(np.vdot(fb, f))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    # the adjoint ignores nothing it should see and produces nothing outside the forced slots
    assert np.abs(fb[:, 3 * P.N:]).max() == 0.0


def forcing(P, seed, amp, nmodes=4):
    """Smooth forcing: random complex coefficients in the first nmodes Chebyshev modes of u, w,
    b at every wavenumber (real at k = 0), of size amp."""
    rng = np.random.default_rng(seed)
    f = np.zeros((P.K, P.S), dtype=complex)
    for name in ("u", "w", "b"):
        sl = P.sl(name)
        blk = amp * (rng.standard_normal((P.K, nmodes)) + 1j * rng.standard_normal((P.K, nmodes)))
        f[:, sl.start:sl.start + nmodes] = blk
    f[0] = f[0].real
    return f


def chain(P, f, dt, n):
    X0 = P.lbvp_solve(f)
    XN, hist = imex.rk_forward(P, X0, dt, n)
    J = P.kinetic_energy(XN)
    X0b = imex.rk_adjoint(P, P.kinetic_energy_grad(XN), hist, dt)
    return J, P.lbvp_adjoint(X0b)


def test_chained_gradient_central_differences():
    """J = kinetic energy after n RK222 steps from the LBVP solution: the chained adjoint
    (IVP reverse sweep, then L^H Y = Xbar_0 and M^H Y) against central differences in every
    forced coefficient of two wavenumbers, and the Taylor remainder rate along a random
    direction."""
    P = RBC(Nx=8, Nz=10, Lx=3.0, Ra=5e4, Pr=1.0)
    f = forcing(P, 5, 1e-2)
    dt, n = 0.02, 4
    J, g = chain(P, f, dt, n)
    assert 1e-8 < J < 1.0   # a flow of moderate amplitude, far from blow-up
    h = 1e-6
    for k in (0, 2):
        for s in [q * P.N + m for q in range(3) for m in range(4)]:
            for part in ((1.0,) if k == 0 else (1.0, 1j)):
                e = np.zeros_like(f)
                e[k, s] = h * part
                Jp = chain(P, f + e, dt, n)[0]
                Jm = chain(P, f - e, dt, n)[0]
                fd = (Jp - Jm) / (2 * h)
                an = np.real(np.conj(part) * g[k, s])
                assert abs(fd - an) <= 1e-6 * np.max(np.abs(g)), (k, s, part, fd, an)
    d = forcing(P, 7, 1e-2)
    eps = np.array([1.0, 0.5, 0.25])
    rem = [abs(chain(P, f + e * d, dt, n)[0] - J - e * np.real(np.vdot(g, d))) for e in eps]
    rates = np.log2(np.array(rem[:-1]) / np.array(rem[1:]))
    assert np.all(np.abs(rates - 2.0) < 0.1), rates
