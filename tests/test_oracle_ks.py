"""Pins of the Kuramoto-Sivashinsky oracle: energy conservation of the dealiased
nonlinearity, exact products against numpy's FFT on a fine grid, the inner-product
test on F, Taylor remainders and brute-force finite differences."""
import numpy as np
import pytest

from oracle import imex
from oracle.ks import KS
import workloads as wl


def test_nonlinearity_conserves_energy():
    P = KS()
    X = wl.ks_c0(seed=5, amp=1.0)[:, None]
    # <u, F(u)> in the Parseval inner product: sum_m w_m Re(conj(c_m) F_m)
    w = np.full(P.K, 2.0); w[0] = 1.0
    dot = np.sum(w * np.real(np.conj(X[:, 0]) * P.F(X)[:, 0]))
    scale = np.sum(w * np.abs(X[:, 0]) * np.abs(P.F(X)[:, 0]))
    assert abs(dot) < 1e-14 * scale


def test_nonlinearity_is_exact_product():
    P = KS(Nx=32, L=10.0)
    c = wl.random_state(6, (P.K,))
    F = P.F(c[:, None])[:, 0]
    Mg = 8 * P.Nx
    pad = np.zeros(Mg // 2 + 1, dtype=complex); pad[:P.K] = c; pad[0] = pad[0].real
    u = np.fft.irfft(pad, Mg) * Mg
    k = 2 * np.pi * np.arange(P.K) / P.Lx
    ref = -0.5j * k * (np.fft.rfft(u * u)[:P.K] / Mg)
    assert np.max(np.abs(F - ref)) < 1e-13 * np.max(np.abs(ref))


def test_F_vjp_inner_product():
    P = KS()
    X = wl.random_state(7, (P.K, 1))
    v = wl.random_state(8, (P.K, 1))
    Yb = wl.random_state(9, (P.K, 1), real_first_row=False)
    Fv = (P.F(X + v) - P.F(X - v)) / 2.0
    lhs = np.real(np.vdot(Yb, Fv))
    rhs = np.real(np.vdot(P.F_vjp(X, Yb), v))
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def gradient(P, X0, dt, n, order=2):
    XN, states = imex.sbdf_forward(P, X0, dt, n, order=order)
    return P.energy(XN), imex.sbdf_adjoint(P, P.energy_grad(XN), states, dt, order=order)


@pytest.mark.parametrize("order", [2, 3, 4])
def test_taylor_remainder_rate(order):
    P = KS()
    X0 = wl.ks_c0(seed=0)[:, None]
    dt = 0.05
    J, g = gradient(P, X0, dt, 200, order)
    d = wl.random_state(10, (P.K, 1))
    rem = []
    for e in (1e-4, 5e-5, 2.5e-5, 1.25e-5):
        Je = P.energy(imex.sbdf_forward(P, X0 + e * d, dt, 200, order=order)[0])
        rem.append(abs(Je - J - e * np.real(np.vdot(g, d))))
    rates = np.log2(np.array(rem[:-1]) / np.array(rem[1:]))
    assert np.all(np.abs(rates - 2.0) < 0.05), rates


@pytest.mark.parametrize("order", [2, 3, 4])
def test_brute_force_finite_differences_every_component(order):
    """8 modes x 10 steps: every real and imaginary component of the initial state."""
    P = KS(Nx=16, L=8.0)
    X0 = wl.ks_c0(seed=1, Nx=16, amp=0.5)[:, None]
    dt, n = 0.05, 10
    J, g = gradient(P, X0, dt, n, order)
    h = 1e-6
    for m in range(P.K):
        for part in (1.0, 1j):
            if m == 0 and part == 1j:
                continue
            e = np.zeros_like(X0); e[m, 0] = h * part
            fd = (P.energy(imex.sbdf_forward(P, X0 + e, dt, n, order=order)[0])
                  - P.energy(imex.sbdf_forward(P, X0 - e, dt, n, order=order)[0])) / (2 * h)
            an = np.real(np.conj(part) * g[m, 0])
            assert abs(fd - an) <= 1e-7 * np.max(np.abs(g))


@pytest.mark.parametrize("order", [2, 3])
def test_variable_step_taylor_remainder_rate(order):
    """200 steps whose sizes vary by +-30 % around 0.05: the gradient's Taylor remainder falls at
    second order."""
    P = KS()
    X0 = wl.ks_c0(seed=0)[:, None]
    h = 0.05 * (1.0 + 0.3 * np.sin(np.arange(200) * 0.37))
    XN, states = imex.sbdf_forward(P, X0, h, 200, order=order)
    J = P.energy(XN)
    g = imex.sbdf_adjoint(P, P.energy_grad(XN), states, h, order=order)
    d = wl.random_state(10, (P.K, 1))
    rem = []
    for e in (1e-4, 5e-5, 2.5e-5, 1.25e-5):
        Je = P.energy(imex.sbdf_forward(P, X0 + e * d, h, 200, order=order)[0])
        rem.append(abs(Je - J - e * np.real(np.vdot(g, d))))
    rates = np.log2(np.array(rem[:-1]) / np.array(rem[1:]))
    assert np.all(np.abs(rates - 2.0) < 0.05), rates


def test_rk443_gradient_taylor_rate_and_brute_force():
    """KS with ARS(4,4,3): Taylor remainder rate 2 of the gradient (64 modes, 100 steps) and
    brute-force central differences of every component (8 modes, 6 steps)."""
    tab = imex.ars443_tableau()
    P = KS()
    X0 = wl.ks_c0(seed=0)[:, None]
    XN, hist = imex.rk_forward(P, X0, 0.05, 100, tableau=tab)
    J = P.energy(XN)
    g = imex.rk_adjoint(P, P.energy_grad(XN), hist, 0.05, tableau=tab)
    d = wl.random_state(10, (P.K, 1))
    rem = []
    for e in (1e-4, 5e-5, 2.5e-5):
        Je = P.energy(imex.rk_forward(P, X0 + e * d, 0.05, 100, tableau=tab)[0])
        rem.append(abs(Je - J - e * np.real(np.vdot(g, d))))
    rates = np.log2(np.array(rem[:-1]) / np.array(rem[1:]))
    assert np.all(np.abs(rates - 2.0) < 0.05), rates
    P = KS(Nx=16, L=8.0)
    X0 = wl.ks_c0(seed=1, Nx=16, amp=0.5)[:, None]
    XN, hist = imex.rk_forward(P, X0, 0.05, 6, tableau=tab)
    g = imex.rk_adjoint(P, P.energy_grad(XN), hist, 0.05, tableau=tab)
    h = 1e-6
    for m in range(P.K):
        for part in (1.0, 1j):
            if m == 0 and part == 1j:
                continue
            e = np.zeros_like(X0); e[m, 0] = h * part
            fd = (P.energy(imex.rk_forward(P, X0 + e, 0.05, 6, tableau=tab)[0])
                  - P.energy(imex.rk_forward(P, X0 - e, 0.05, 6, tableau=tab)[0])) / (2 * h)
            assert abs(fd - np.real(np.conj(part) * g[m, 0])) <= 1e-7 * np.max(np.abs(g))
