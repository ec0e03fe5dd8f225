"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module draws random numbers and lays them out on the problem's grid points;
it holds none of the solver's arithmetic (no transforms, operators or timesteps).
All generators use numpy's PCG64 (numpy.random.default_rng(seed)) in FP64.
"""
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
