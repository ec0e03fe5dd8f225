"""Pins of the oracle's transforms (Methods, "Spectral transforms") against library
routines, closed-form identities and the inner-product (dot-product) test."""
import numpy as np
import numpy.polynomial.chebyshev as npc
import scipy.fft
import pytest

from oracle import spectral as sp

RNG = np.random.default_rng(1234)


def rand_coeffs(K, real0=True):
    c = RNG.standard_normal(K) + 1j * RNG.standard_normal(K)
    if real0:
        c[0] = c[0].real
    return c


@pytest.mark.parametrize("Nx,L", [(16, 2 * np.pi), (64, 32 * np.pi), (256, 4.0)])
def test_fourier_forward_is_numpy_rfft(Nx, L):
    K, Ng = Nx // 2, 3 * Nx // 2
    u = RNG.standard_normal(Ng)
    c = sp.fourier_forward(u, sp.fourier_forward_matrix(K, Ng, L))
    ref = np.fft.rfft(u)[:K] / Ng
    assert np.max(np.abs(c - ref)) < 1e-14 * np.max(np.abs(ref)) * 10


@pytest.mark.parametrize("Nx,L", [(16, 2 * np.pi), (64, 32 * np.pi), (256, 4.0)])
def test_fourier_backward_is_padded_numpy_irfft(Nx, L):
    K, Ng = Nx // 2, 3 * Nx // 2
    c = rand_coeffs(K)
    u = sp.fourier_backward(c, sp.fourier_backward_matrix(K, Ng, L))
    pad = np.zeros(Ng // 2 + 1, dtype=complex)
    pad[:K] = c
    ref = np.fft.irfft(pad, Ng) * Ng
    assert np.max(np.abs(u - ref)) < 1e-13 * np.max(np.abs(ref))


def test_fourier_roundtrip_and_truncation():
    K, Ng, L = 32, 96, 7.0
    c = rand_coeffs(K)
    B, F = sp.fourier_backward_matrix(K, Ng, L), sp.fourier_forward_matrix(K, Ng, L)
    c2 = sp.fourier_forward(sp.fourier_backward(c, B), F)
    assert np.max(np.abs(c2 - c)) < 1e-13
    # a pure mode above the kept band is truncated away
    x = sp.fourier_grid(Ng, L)
    u = np.cos(2 * np.pi * (K + 3) * x / L)
    assert np.max(np.abs(sp.fourier_forward(u, F))) < 1e-14


@pytest.mark.parametrize("N,Ng", [(8, 12), (64, 96), (64, 64)])
def test_chebyshev_backward_is_chebval(N, Ng):
    a = RNG.standard_normal(N)
    f = sp.chebyshev_backward_matrix(N, Ng) @ a
    ref = npc.chebval(sp.chebyshev_nodes(Ng), a)
    assert np.max(np.abs(f - ref)) < 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("N,Ng", [(8, 12), (64, 96), (64, 64)])
def test_chebyshev_forward_is_scipy_dct2(N, Ng):
    """sum_j f_j T_n(x_j) on ascending Gauss nodes equals (-1)^n DCT-II(f)_n / 2."""
    f = RNG.standard_normal(Ng)
    a = sp.chebyshev_forward_matrix(N, Ng) @ f
    y = scipy.fft.dct(f, type=2)[:N]
    n = np.arange(N)
    ref = (2.0 - (n == 0)) / Ng * ((-1.0) ** n) * y / 2.0
    assert np.max(np.abs(a - ref)) < 1e-13 * np.max(np.abs(ref))


def test_chebyshev_forward_inverts_backward():
    N, Ng = 64, 96
    a = RNG.standard_normal(N)
    a2 = sp.chebyshev_forward_matrix(N, Ng) @ (sp.chebyshev_backward_matrix(N, Ng) @ a)
    assert np.max(np.abs(a2 - a)) < 1e-13


def inner(a, b):
    return np.real(np.vdot(a, b))


@pytest.mark.parametrize("Nx", [16, 256])
def test_fourier_adjoints_dot_product(Nx):
    K, Ng, L = Nx // 2, 3 * Nx // 2, 4.0
    B, F = sp.fourier_backward_matrix(K, Ng, L), sp.fourier_forward_matrix(K, Ng, L)
    c, ub = rand_coeffs(K), RNG.standard_normal(Ng)
    lhs = inner(ub, sp.fourier_backward(c, B))
    rhs = inner(sp.fourier_backward_adjoint(ub, B), c)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)
    u, cb = RNG.standard_normal(Ng), rand_coeffs(K, real0=False)
    lhs = inner(cb, sp.fourier_forward(u, F))
    rhs = inner(sp.fourier_forward_adjoint(cb, F), u)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_complex_fourier_roundtrip():
    Nc, Ng, L = 16, 24, 3.0
    B = sp.complex_fourier_backward_matrix(Nc, Ng, L)
    F = sp.complex_fourier_forward_matrix(Nc, Ng, L)
    c = RNG.standard_normal(Nc) + 1j * RNG.standard_normal(Nc)
    c[Nc // 2] = 0.0
    assert np.max(np.abs(F @ (B @ c) - c)) < 1e-14
    u = RNG.standard_normal(Ng)
    ref = np.fft.fft(u) / Ng
    m = sp.complex_fourier_modes(Nc)
    keep = np.abs(m) < Nc // 2
    assert np.max(np.abs((F @ u)[keep] - ref[m[keep] % Ng])) < 1e-14


def test_transform_matrix_entries_to_full_precision():
    """The matrix entries are evaluated with their angles reduced exactly in integers: the
    Chebyshev T_n at the Gauss nodes and the Fourier phases agree with an 80-bit evaluation of the
    same exact angles to a few ulps (the angle of a rounded node, cos(n arccos x_j), would be off
    by about n ulps: 7e-14 at 64 modes), and both are consistent with numpy's FFT and chebval."""
    pi = np.longdouble("3.14159265358979323846264338327950288")
    Ng, N = 96, 64
    j = np.arange(Ng)
    M = np.mod(np.outer(2 * (Ng - j) - 1, np.arange(N)), 4 * Ng).astype(np.longdouble)
    ref = np.cos(pi * M / (2 * Ng))
    assert float(np.max(np.abs(sp.chebyshev_T_nodes(N, Ng) - ref))) < 2e-15
    # chebval evaluates at the rounded nodes: equal up to T_n' times the node's rounding
    x = sp.chebyshev_nodes(Ng)
    cv = np.array([np.polynomial.chebyshev.chebval(x, np.eye(N)[n]) for n in range(N)]).T
    assert np.max(np.abs(sp.chebyshev_T_nodes(N, Ng) - cv)) < 1e-13
    Nx = 384
    r = np.mod(np.outer(np.arange(Nx), np.arange(128)), Nx).astype(np.longdouble)
    ph = sp.grid_phase(np.arange(128), Nx)
    assert float(np.max(np.abs(ph.real - np.cos(2 * pi * r / Nx)))) < 2e-15
    assert float(np.max(np.abs(ph.imag - np.sin(2 * pi * r / Nx)))) < 2e-15
    u = np.random.default_rng(0).standard_normal(Nx)
    F = sp.fourier_forward_matrix(128, Nx, 4.0)
    assert np.max(np.abs(F @ u - np.fft.fft(u)[:128] / Nx)) < 1e-15
