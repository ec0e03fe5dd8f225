"""Pins of the plane Couette oracle: closed-form viscous decay of a streak and of a spanwise mean
flow (second-order convergence to the exact solution), the explicit term against products
evaluated independently on a finer grid, the F-VJP inner-product test, the energy formula
against quadrature, the energy budget of the explicit term (advection conserves energy, the
base flow produces -int u v), the divergence-free perturbation generator, and the gradient of the
final energy by Taylor remainders and brute-force central differences of every component."""
import numpy as np
import numpy.polynomial.chebyshev as npc

import workloads as wl
from oracle import imex
from oracle import spectral as sp
from oracle.couette import Couette


def state_from_uvw(P, c):
    """(K, 3, N) velocity coefficients -> oracle state (K, S)."""
    X = np.zeros((P.K, P.S), complex)
    for f, name in enumerate("uvw"):
        X[:, P.sl(name)] = c[:, f]
    return X


def hermitian(P, X):
    """Make the m = 0 modes Hermitian in n (a real field) and the mean mode real."""
    X = X.copy()
    for n in range(1, P.Nz // 2):
        X[P.Nz - n] = np.conj(X[n])
    X[0] = X[0].real
    X[P.Nz // 2] = 0.0
    return X


def test_viscous_decay_of_a_streak_and_a_mean_flow_closed_form():
    """u = A cos(pi y / 2) cos(kz z) (a streak, kx = 0) and, separately, w = B cos(pi y / 2) (a
    spanwise mean flow) carry no advection, pressure or lift-up: they decay as
    exp(-nu (pi^2/4 + kz^2) t).  The RK222 error converges at second order."""
    for case in ("streak", "mean"):
        P = Couette(Nx=4, Ny=24, Nz=4, Lx=2.0 * np.pi, Lz=2.0 * np.pi, Re=50.0)
        A, T = 0.3, 1.0
        yq = sp.chebyshev_nodes(P.N)
        Fy = sp.chebyshev_forward_matrix(P.N, P.N)
        prof = Fy @ np.cos(np.pi * yq / 2.0)
        X0 = np.zeros((P.K, P.S), complex)
        if case == "streak":
            X0[1, P.sl("u")] = 0.5 * A * prof            # n = 1 and n = -1 (index Nz - 1)
            X0[P.Nz - 1, P.sl("u")] = 0.5 * A * prof
            lam, slot, ks = -P.nu * (np.pi ** 2 / 4 + 1.0), "u", [1, P.Nz - 1]
        else:
            X0[0, P.sl("w")] = A * prof
            lam, slot, ks = -P.nu * np.pi ** 2 / 4, "w", [0]
        errs = []
        yt = np.linspace(-1, 1, 11)
        for n in (25, 50, 100):
            XN, _ = imex.rk_forward(P, X0, T / n, n)
            ref = (0.5 * A if case == "streak" else A) * np.exp(lam * T) * np.cos(np.pi * yt / 2)
            err = 0.0
            for k in ks:
                err = max(err, np.abs(npc.chebval(yt, XN[k, P.sl(slot)].real) - ref).max())
                err = max(err, np.abs(XN[k, P.sl("p")]).max())
            others = np.delete(np.arange(P.K), ks)
            assert np.abs(XN[others][:, : 4 * P.N]).max() < 1e-14
            errs.append(err)
        rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
        assert np.all(np.abs(rates - 2.0) < 0.1), (case, errs, rates)


def fine_products(P, X, Mx, My, Mz):
    """The explicit-term densities evaluated independently: fields summed mode by mode on a fine
    tensor grid (numpy chebval and complex exponentials), products, then projected onto the
    stored modes with numpy's FFT and a Chebyshev least-squares fit of degree 3N."""
    x = np.arange(Mx) * P.Lx / Mx
    z = np.arange(Mz) * P.Lz / Mz
    yq = np.cos(np.pi * (np.arange(My) + 0.5) / My)
    wm = np.where(P.m == 0, 1.0, 2.0)

    def phys(c):
        out = np.zeros((My, Mz, Mx))
        for k in np.nonzero(P.keep)[0]:
            cy = npc.chebval(yq, c[k])
            e = np.exp(1j * (P.kz[k] * z[:, None] + P.kx[k] * x[None, :]))
            out += np.real(wm[k] * cy[:, None, None] * e[None])
        return out

    def dy(c):
        return np.array([np.append(npc.chebder(c[k]), 0.0) for k in range(P.K)])

    g = {}
    for f in "uvw":
        c = X[:, P.sl(f)]
        g[f] = phys(c)
        g[f + "x"] = phys(1j * P.kx[:, None] * c)
        g[f + "z"] = phys(1j * P.kz[:, None] * c)
        g[f + "y"] = phys(dy(c))
    Y = yq[:, None, None]
    dens = {}
    for f in "uvw":
        d = -(g["u"] * g[f + "x"] + g["v"] * g[f + "y"] + g["w"] * g[f + "z"]) - Y * g[f + "x"]
        if f == "u":
            d = d - g["v"]
        dens[f] = d

    def proj(f):
        U = np.fft.rfft2(f, axes=(1, 2)) / (Mx * Mz)
        rows = np.where(P.ns >= 0, P.ns, P.ns + Mz)
        cy = U[:, rows, P.m]                                      # (My, K)
        out = np.zeros((P.K, P.N), complex)
        for k in np.nonzero(P.keep)[0]:
            full = npc.chebfit(yq, cy[:, k].real, 3 * P.N) + 1j * npc.chebfit(yq, cy[:, k].imag, 3 * P.N)
            out[k] = full[: P.N]
        return out

    return [proj(dens[f]) for f in "uvw"]


def test_explicit_term_is_the_exact_dealiased_product():
    P = Couette(Nx=6, Ny=8, Nz=6, Lx=3.0, Lz=2.0, Re=100.0)
    X = hermitian(P, wl.random_state(5, (P.K, P.S)))
    got = [P.from_grid(n) for n in P.products(X)]
    ref = fine_products(P, X, 4 * P.Nx, 4 * P.Ny, 4 * P.Nz)
    for a, b in zip(got, ref):
        assert np.max(np.abs(a - b)) < 1e-11 * np.max(np.abs(b))


def test_F_vjp_inner_product():
    """F is quadratic plus linear, so its central difference with unit step is exactly F'(X) v."""
    P = Couette(Nx=6, Ny=10, Nz=6, Lx=4.0, Lz=3.0, Re=300.0)
    X = wl.random_state(10, (P.K, P.S))
    v = wl.random_state(11, (P.K, P.S))
    Yb = wl.random_state(12, (P.K, P.S), real_first_row=False)
    Fv = (P.F(X + v) - P.F(X - v)) / 2.0
    lhs = np.real(np.vdot(Yb, Fv))
    rhs = np.real(np.vdot(P.F_vjp(X, Yb), v))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_energy_matches_quadrature():
    P = Couette(Nx=6, Ny=8, Nz=6, Lx=4.0, Lz=3.0)
    X = hermitian(P, wl.random_state(13, (P.K, P.S)))
    from numpy.polynomial.legendre import leggauss
    My, Mx, Mz = 24, 24, 24
    yq, wq = leggauss(My)
    x = np.arange(Mx) * P.Lx / Mx
    z = np.arange(Mz) * P.Lz / Mz
    wm = np.where(P.m == 0, 1.0, 2.0)
    J = 0.0
    for f in "uvw":
        c = X[:, P.sl(f)]
        g = np.zeros((My, Mz, Mx))
        for k in np.nonzero(P.keep)[0]:
            e = np.exp(1j * (P.kz[k] * z[:, None] + P.kx[k] * x[None, :]))
            g += np.real(wm[k] * npc.chebval(yq, c[k])[:, None, None] * e[None])
        J += 0.5 * np.sum(g ** 2 * wq[:, None, None]) * (P.Lx / Mx) * (P.Lz / Mz)
    assert abs(P.energy(X) - J) < 1e-12 * J
    assert abs(0.5 * np.real(np.vdot(P.energy_grad(X), X)) - P.energy(X)) < 1e-12 * J


def test_generator_is_divergence_free_with_no_slip_and_given_energy():
    P = Couette(Nx=8, Ny=16, Nz=8)
    c = wl.couette_perturbation(seed=2, Nx=8, Ny=16, Nz=8, energy=1e-6)
    X = state_from_uvw(P, c)
    for k in range(P.K):
        dv = np.append(npc.chebder(c[k, 1]), 0.0)
        div = 1j * P.kx[k] * c[k, 0] + dv + 1j * P.kz[k] * c[k, 2]
        assert np.abs(div).max() < 1e-14
        for f in range(3):
            assert abs(npc.chebval(1.0, c[k, f])) < 1e-15 and abs(npc.chebval(-1.0, c[k, f])) < 1e-15
    assert abs(P.energy(X) - 1e-6) < 1e-18


def test_energy_budget_of_the_explicit_term():
    """For a divergence-free field with no-slip walls whose products stay within the stored
    modes, <u, F> = -int u v dV exactly: advection conserves energy and the base flow U = y
    produces -int u v U' dV."""
    P = Couette(Nx=8, Ny=24, Nz=8, Lx=4.0, Lz=3.0)
    c = wl.couette_perturbation(seed=4, Nx=8, Ny=24, Nz=8, Lx=4.0, Lz=3.0, energy=1.0, mmax=2, nmax=2, deg=2)
    X = state_from_uvw(P, c)
    G = sp.gram_T(P.N, -1.0, 1.0)
    wm = np.where(P.m == 0, 1.0, 2.0)

    def inner(a, b):
        return P.Lx * P.Lz * np.sum(wm * np.real(np.einsum("km,mn,kn->k", a.conj(), G, b)))

    N = [P.from_grid(n) for n in P.products(X)]
    lhs = sum(inner(c[:, f], N[f]) for f in range(3))
    prod = -inner(c[:, 0], c[:, 1])
    assert abs(lhs - prod) < 1e-12 * abs(prod)
    assert abs(prod) > 1e-3


def gradient(P, X0, dt, n):
    XN, hist = imex.rk_forward(P, X0, dt, n)
    return P.energy(XN), imex.rk_adjoint(P, P.energy_grad(XN), hist, dt)


def test_taylor_remainder_rate():
    P = Couette(Nx=8, Ny=12, Nz=8, Re=400.0)
    X0 = state_from_uvw(P, wl.couette_perturbation(seed=6, Nx=8, Ny=12, Nz=8, energy=1e-2))
    dt, n = 0.02, 10
    J, g = gradient(P, X0, dt, n)
    d = state_from_uvw(P, wl.couette_perturbation(seed=7, Nx=8, Ny=12, Nz=8, energy=1e-2))
    eps = np.array([1e-1, 5e-2, 2.5e-2, 1.25e-2])
    rem = []
    for e in eps:
        Je = P.energy(imex.rk_forward(P, X0 + e * d, dt, n)[0])
        rem.append(abs(Je - J - e * np.real(np.vdot(g, d))))
    rates = np.log2(np.array(rem[:-1]) / np.array(rem[1:]))
    assert np.all(np.abs(rates - 2.0) < 0.05), rates


def test_brute_force_finite_differences_every_component():
    P = Couette(Nx=4, Ny=8, Nz=4, Lx=3.0, Lz=2.0, Re=100.0)
    X0 = state_from_uvw(P, wl.couette_perturbation(seed=8, Nx=4, Ny=8, Nz=4, Lx=3.0, Lz=2.0, energy=1.0))
    dt, n = 0.02, 3
    J, g = gradient(P, X0, dt, n)
    h = 1e-5
    for k in range(P.K):
        for s in range(3 * P.N):
            for part in (1.0, 1j):
                e = np.zeros_like(X0)
                e[k, s] = h * part
                Jp = P.energy(imex.rk_forward(P, X0 + e, dt, n)[0])
                Jm = P.energy(imex.rk_forward(P, X0 - e, dt, n)[0])
                fd = (Jp - Jm) / (2 * h)
                an = np.real(np.conj(part) * g[k, s])
                assert abs(fd - an) <= 1e-7 * np.max(np.abs(g)), (k, s, part, fd, an)
