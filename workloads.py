"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module draws random numbers and lays them out on the problem's grid points;
it holds none of the solver's arithmetic (no transforms, operators or timesteps).
All generators use numpy's PCG64 (numpy.random.default_rng(seed)) in FP64.
"""
import math

import numpy as np


def gauss_nodes_unit(Nz):
    """Gauss-Chebyshev (root) nodes mapped to [0, 1], ascending."""
    return 0.5 * (1.0 - np.cos(np.pi * (np.arange(Nz) + 0.5) / Nz))


def rbc_b0(seed=0, Nx=256, Nz=64, amp=1e-3):
    """Initial buoyancy on the (Nx, Nz) scale-1 grid: the conduction profile 1 - z plus
    i.i.d. standard normal noise of amplitude amp damped at the walls by 4 z (1 - z)."""
    rng = np.random.default_rng(seed)
    xi = rng.standard_normal((Nx, Nz))
    z = gauss_nodes_unit(Nz)
    return (1.0 - z)[None, :] + amp * xi * (4.0 * z * (1.0 - z))[None, :]


def rbc_forcing(seed=0, Nx=256, Nz=64, amp=1e-5, nmodes=4):
    """Forcing of the 2D boundary value problem in the state layout (K = Nx/2 wavenumbers,
    S = 4 Nz + 7 slots): i.i.d. complex normal coefficients of size amp in the first nmodes
    Chebyshev modes of the u, w, b blocks at every wavenumber (real at k = 0), zero elsewhere."""
    rng = np.random.default_rng(seed)
    K, S = Nx // 2, 4 * Nz + 7
    f = np.zeros((K, S), dtype=complex)
    for q in range(3):
        f[:, q * Nz:q * Nz + nmodes] = amp * (rng.standard_normal((K, nmodes)) + 1j * rng.standard_normal((K, nmodes)))
    f[0] = f[0].real
    return f


def ks_c0(seed=0, Nx=64, amp=1e-2):
    """Initial half-spectrum coefficients c_m = amp (1 + m)^-2 (xi + i eta), m < Nx/2,
    with a real mean mode; returned as an (Nx/2,) complex array."""
    rng = np.random.default_rng(seed)
    K = Nx // 2
    xi = rng.standard_normal(K)
    eta = rng.standard_normal(K)
    m = np.arange(K)
    c = amp * (1.0 + m) ** -2.0 * (xi + 1j * eta)
    c[0] = c[0].real
    return c


def random_state(seed, shape, real_first_row=True):
    """Complex normal test vector of the given shape; the first block (the mean mode)
    is made real when real_first_row is set."""
    rng = np.random.default_rng(seed)
    X = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    if real_first_row:
        X[0] = X[0].real
    return X


def sh_batch(seed=0, batch=128, sizes=(64, 96, 128, 192), rmin=0.1, rmax=0.5, amp=0.1):
    """A batch of Swift-Hohenberg instances: sizes drawn uniformly from `sizes`, r uniform in
    [rmin, rmax], initial grid fields uniform in [-amp, amp] on each N x N grid.  Returns
    (sizes, r, list of (N, N) arrays)."""
    rng = np.random.default_rng(seed)
    n = rng.choice(np.array(sizes), size=batch)
    r = rng.uniform(rmin, rmax, size=batch)
    u0 = [rng.uniform(-amp, amp, size=(int(k), int(k))) for k in n]
    return [int(k) for k in n], [float(v) for v in r], u0


def kolmo_vorticity(seed=0, N=64, batch=1, amp=0.4):
    """Random initial vorticity coefficients of 2D Kolmogorov flow on [0, 2 pi)^2 with an
    energy spectrum E(k) ~ k^-3: |omega_k| ~ amp |k|^-1 (complex Gaussian per mode, the k_x = 0
    column Hermitian so that the field is real, mean and Nyquist row zero).  The expected mean
    square velocity is about 6 amp^2 (a lattice sum of |k|^-4), so amp = 0.4 gives about 1.  Returns (batch, N, N/2) complex arrays c[iy, m] (iy in FFT order)."""
    rng = np.random.default_rng(seed)
    iy = np.arange(N)
    ky = np.where(iy < N // 2, iy, iy - N).astype(float)
    kx = np.arange(N // 2).astype(float)
    k = np.sqrt(ky[:, None] ** 2 + kx[None, :] ** 2)
    out = np.zeros((batch, N, N // 2), complex)
    for b in range(batch):
        c = (rng.standard_normal((N, N // 2)) + 1j * rng.standard_normal((N, N // 2))) / np.sqrt(2.0)
        c *= amp / np.where(k > 0, k, 1.0)
        c[0, 0] = 0.0
        c[N // 2, :] = 0.0
        c[N // 2 + 1:, 0] = np.conj(c[1:N // 2, 0][::-1])
        out[b] = c
    return out


def couette_perturbation(seed=0, Nx=128, Ny=64, Nz=64, Lx=4.0 * np.pi, Lz=2.0 * np.pi, energy=1e-6,
                         mmax=3, nmax=3, deg=8):
    """Random divergence-free velocity perturbation of plane Couette flow with no-slip walls, as
    Chebyshev coefficients per Fourier mode.  Modes k = m Nz + n (m < Nx/2, n < Nz in FFT order),
    only |m| < mmax, |n| < nmax excited.  Per mode with kh = |(kx, kz)| > 0:
        v = (1 - y^2)^2 q(y),  s = (1 - y^2) r(y),
        (u, w) = i (kx, kz) v' / kh^2 + (-kz, kx) s / kh,
    with q, r random complex polynomials of degree deg (coefficients decaying as 2^-j), so that
    i kx u + v' + i kz w = 0 and u = v = w = 0 at y = -1, 1; the mean mode holds
    u, w = (1 - y^2) r(y), v = 0 (real).  The m = 0 modes are Hermitian in n (a real field).
    Scaled to kinetic energy `energy` = 1/2 int |u|^2 dV.  Returns (K, 3, Ny) complex
    coefficients (u, v, w)."""
    C = np.polynomial.chebyshev
    rng = np.random.default_rng(seed)
    Kx = Nx // 2
    out = np.zeros((Kx * Nz, 3, Ny), complex)
    one_m_y2 = np.array([0.5, 0.0, -0.5])          # 1 - y^2 in the T basis
    wall2 = C.chebmul(one_m_y2, one_m_y2)

    def poly():
        dec = 2.0 ** -np.arange(deg + 1)
        return dec * (rng.standard_normal(deg + 1) + 1j * rng.standard_normal(deg + 1))

    def fit(c):
        v = np.zeros(Ny, complex)
        v[: min(Ny, len(c))] = c[:Ny]
        return v

    for m in range(min(mmax, Kx)):
        for ns in range(-(nmax - 1), nmax):
            if m == 0 and ns < 0:
                continue
            n = ns % Nz
            k = m * Nz + n
            kx, kz = 2.0 * np.pi * m / Lx, 2.0 * np.pi * ns / Lz
            kh = np.hypot(kx, kz)
            if kh == 0.0:
                r1, r2 = poly().real, poly().real
                out[k, 0] = fit(C.chebmul(one_m_y2, r1))
                out[k, 2] = fit(C.chebmul(one_m_y2, r2))
                continue
            v = C.chebmul(wall2, poly())
            s = C.chebmul(one_m_y2, poly())
            dv = C.chebder(v)
            out[k, 1] = fit(v)
            out[k, 0] = fit(1j * kx * dv / kh ** 2) - fit(kz * s / kh)
            out[k, 2] = fit(1j * kz * dv / kh ** 2) + fit(kx * s / kh)
            if m == 0:
                out[(-ns) % Nz] = np.conj(out[k])
    # kinetic energy: 1/2 Lx Lz sum_k w_m int_{-1}^{1} |c_k(y)|^2 dy
    e = 0.0
    for k in range(Kx * Nz):
        wm = 1.0 if k < Nz else 2.0
        for f in range(3):
            c = out[k, f]
            sq = C.chebadd(C.chebmul(c.real, c.real), C.chebmul(c.imag, c.imag))
            integ = C.chebint(sq)
            e += 0.5 * Lx * Lz * wm * (C.chebval(1.0, integ) - C.chebval(-1.0, integ))
    return out * np.sqrt(energy / e)


CLOSURE_PARAM_ORDER = ("w1", "b1", "w2", "b2", "w3", "b3")


def closure_params(seed=0, C=32, scale=1.0):
    """Seeded initial weights of the closure network (3x3 convolutions 1 -> C -> C -> 1):
    He-style normal draws for w1 and w2, a last layer 1e-2 smaller so that the network starts
    as a small perturbation of the explicit term, zero biases.  Returns a dict of arrays with
    the shapes w1 (C, 1, 3, 3), b1 (C,), w2 (C, C, 3, 3), b2 (C,), w3 (1, C, 3, 3), b3 (1,)."""
    rng = np.random.default_rng(seed)
    return {
        "w1": rng.standard_normal((C, 1, 3, 3)) * math.sqrt(2.0 / 9.0) * scale,
        "b1": np.zeros(C),
        "w2": rng.standard_normal((C, C, 3, 3)) * math.sqrt(2.0 / (9.0 * C)) * scale,
        "b2": np.zeros(C),
        "w3": rng.standard_normal((1, C, 3, 3)) * math.sqrt(1.0 / (9.0 * C)) * scale * 1e-2,
        "b3": np.zeros(1),
    }


def closure_theta(seed=0, C=32, scale=1.0):
    """closure_params as one FP64 vector in the library's parameter order (w1, b1, w2, b2, w3,
    b3, each row-major)."""
    p = closure_params(seed, C, scale)
    return np.concatenate([np.asarray(p[k], dtype=np.float64).ravel() for k in CLOSURE_PARAM_ORDER])
