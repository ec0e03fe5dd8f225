"""3D plane Couette flow on the GPU against the FP64 oracle (error <= 1e-11 of each field's own
largest entry: u_par, v, u_perp, p and the taus, the mean mode and the other modes apart, see
tests/parity.py), and the full 128 x 64 x 64 configuration's gradient against central
differences of the GPU's own forward runs.

The library stores each mode's horizontal velocity in the frame of its wave vector,
u_par = (kx u + kz w)/kh, u_perp = (-kz u + kx w)/kh, and solves the problem scaled to unit wall
distance (time t/2, tau values twice those of the unscaled equations, explicit term twice the
unscaled one); `to_lib` maps an oracle state into that layout (an orthogonal rotation of the
velocity slots per mode and the factor 2 on the taus)."""
import numpy as np
import pytest

import workloads as wl
from oracle import imex
from oracle.couette import Couette
from parity import check_fields

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2506_14792_amd as sps  # noqa: E402
from paper_2506_14792_amd import autograd as sa  # noqa: E402


def frame(P):
    kh = np.hypot(P.kx, P.kz)
    ex = np.where(kh > 0, P.kx / np.where(kh > 0, kh, 1.0), 1.0)
    ez = np.where(kh > 0, P.kz / np.where(kh > 0, kh, 1.0), 0.0)
    return ex[:, None], ez[:, None]


def to_lib(P, X, tau_scale=2.0):
    """Oracle state (K, S) in (u, v, w, p, taus) -> library layout (u_par, v, u_perp, p, taus)."""
    N = P.N
    ex, ez = frame(P)
    Y = np.zeros_like(X)
    u, v, w = X[:, 0:N], X[:, N:2 * N], X[:, 2 * N:3 * N]
    Y[:, 0:N] = ex * u + ez * w
    Y[:, N:2 * N] = v
    Y[:, 2 * N:3 * N] = -ez * u + ex * w
    Y[:, 3 * N:4 * N] = X[:, 3 * N:4 * N]
    t = X[:, 4 * N:]
    ex1, ez1 = ex[:, 0], ez[:, 0]
    for off in (0, 3):   # first- and second-order taus of (u, v, w) -> (par, v, perp)
        tu, tv, tw = t[:, off], t[:, off + 1], t[:, off + 2]
        Y[:, 4 * N + off] = tau_scale * (ex1 * tu + ez1 * tw)
        Y[:, 4 * N + off + 1] = tau_scale * tv
        Y[:, 4 * N + off + 2] = tau_scale * (-ez1 * tu + ex1 * tw)
    Y[:, 4 * N + 6] = tau_scale * t[:, 6]
    return Y


def dev(Y):
    return torch.from_numpy(np.ascontiguousarray(Y).view(np.float64).ravel().copy()).cuda()


def host(t, P):
    return t.cpu().numpy().view(np.complex128).reshape(P.K, P.S)


def rel(a, b):
    return np.max(np.abs(a - b)) / np.max(np.abs(b))


NAMES = ("u_par", "v", "u_perp", "p")


def fields(got, ref, P, what, tol=1e-11):
    return check_fields(got, ref, P.N, tol, what=what, names=NAMES)


def state(P, seed, energy):
    c = wl.couette_perturbation(seed=seed, Nx=P.Nx, Ny=P.N, Nz=P.Nz, Lx=P.Lx, Lz=P.Lz, energy=energy,
                                mmax=min(4, P.Kx), nmax=min(4, P.Nz // 2))
    X = np.zeros((P.K, P.S), complex)
    for f in range(3):
        X[:, f * P.N:(f + 1) * P.N] = c[:, f]
    return X


CFGS = [dict(Nx=8, Ny=12, Nz=8, Lx=4.0 * np.pi, Lz=2.0 * np.pi), dict(Nx=24, Ny=16, Nz=12, Lx=3.0, Lz=2.5)]
# more than 1024 modes: the per-mode kernels stream their block operators through LDS
BIG = dict(Nx=64, Ny=16, Nz=48, Lx=4.0 * np.pi, Lz=2.0 * np.pi)


@pytest.mark.parametrize("cfg", CFGS, ids=["8x12x8", "24x16x12"])
def test_couette_explicit_term_and_solve(cfg):
    print(f"couette F/solve {cfg}", flush=True)
    P = Couette(Re=400.0, **cfg)
    G = sps.Couette(cfg["Nx"], cfg["Ny"], cfg["Nz"], cfg["Lx"], cfg["Lz"], Re=400.0, dt=0.01, checkpoint_every=2,
                    max_steps=4)
    X = state(P, 1, 1.0) + 0.01 * wl.random_state(2, (P.K, P.S))
    X[:, 3 * P.N:] = 0.0
    F = torch.zeros(G.n, dtype=torch.float64, device="cuda")
    G.eval_F(dev(to_lib(P, X)), F)
    ef = fields(host(F, P), to_lib(P, 2.0 * P.F(X)), P, "F")
    Yb = wl.random_state(3, (P.K, P.S), real_first_row=False)
    Xb = torch.zeros_like(F)
    G.eval_F_vjp(dev(to_lib(P, X)), dev(to_lib(P, Yb, 1.0)), Xb)
    ev = fields(host(Xb, P)[:, :3 * P.N], to_lib(P, 2.0 * P.F_vjp(X, Yb), 1.0)[:, :3 * P.N], P, "F vjp")
    print(f"  F rel {ef:.2e}  F_vjp rel {ev:.2e}", flush=True)


@pytest.mark.parametrize("cfg", CFGS + [BIG], ids=["8x12x8", "24x16x12", "64x16x48-streamed"])
def test_couette_forward_and_gradient(cfg):
    print(f"couette gradient {cfg}", flush=True)
    P = Couette(Re=400.0, **cfg)
    dt, n, ce = 0.01, 5, 2
    G = sps.Couette(cfg["Nx"], cfg["Ny"], cfg["Nz"], cfg["Lx"], cfg["Lz"], Re=400.0, dt=dt, checkpoint_every=ce,
                    max_steps=n)
    X0 = state(P, 5, 0.5)
    XN, hist = imex.rk_forward(P, X0, dt, n)
    Jo = P.energy(XN)
    go = imex.rk_adjoint(P, P.energy_grad(XN), hist, dt)
    Xd = dev(to_lib(P, X0))
    XNg = torch.zeros_like(Xd)
    g = torch.zeros_like(Xd)
    J = torch.zeros(1, dtype=torch.float64, device="cuda")
    G.gradient(Xd, n, XNg, g, J)
    G.sync()
    ex = fields(host(XNg, P), to_lib(P, XN), P, "X_N")
    eg = fields(host(g, P), to_lib(P, go, 1.0), P, "dJ/dX0")
    eJ = abs(J.item() - Jo) / Jo
    print(f"  XN rel {ex:.2e}  J rel {eJ:.2e}  dJ/dX0 rel {eg:.2e}", flush=True)
    assert eJ <= 1e-11
    # the forward sweep alone, then the adjoint of the recorded run with an external cotangent
    X = Xd.clone()
    G.step(X, n)
    Xbar = dev(to_lib(P, P.energy_grad(XN), 1.0))
    G.adjoint_step(Xbar, n)
    G.sync()
    fields(host(X, P), to_lib(P, XN), P, "step X_N")
    fields(host(Xbar, P), to_lib(P, go, 1.0), P, "adjoint_step dJ/dX0")


def test_couette_full_size_gradient_central_differences():
    """128 x 64 x 64, Re = 400, dt = 0.01, 20 steps with checkpoints every 10: the gradient of the
    final energy along random directions equals central differences of the GPU forward runs
    (the map is smooth and nearly linear at energy 1e-6, so the O(eps^2) error is negligible)."""
    print("couette 128x64x64 directional differences", flush=True)
    nx, ny, nz, n = 128, 64, 64, 20
    G = sps.Couette(nx, ny, nz, Re=400.0, dt=0.01, checkpoint_every=10, max_steps=n)
    K, S = (nx // 2) * nz, 4 * ny + 7
    c = wl.couette_perturbation(seed=0, Nx=nx, Ny=ny, Nz=nz, energy=1e-6)
    X0 = np.zeros((K, S), complex)
    Pf = type("F", (), {})()
    Pf.kx = np.repeat(2 * np.pi * np.arange(nx // 2) / (4 * np.pi), nz)
    ns = np.arange(nz)
    Pf.kz = np.tile(2 * np.pi * np.where(ns < nz // 2, ns, ns - nz) / (2 * np.pi), nx // 2)
    Pf.N, Pf.K, Pf.S = ny, K, S
    for f in range(3):
        X0[:, f * ny:(f + 1) * ny] = c[:, f]
    Xd = dev(to_lib(Pf, X0))
    g = torch.zeros_like(Xd)
    J = torch.zeros(1, dtype=torch.float64, device="cuda")
    G.gradient(Xd, n, None, g, J)
    G.sync()
    print(f"  J = {J.item():.6e}", flush=True)
    for trial in range(2):
        d = np.zeros((K, S), complex)
        cd = wl.couette_perturbation(seed=10 + trial, Nx=nx, Ny=ny, Nz=nz, energy=1e-6)
        for f in range(3):
            d[:, f * ny:(f + 1) * ny] = cd[:, f]
        dd = dev(to_lib(Pf, d))
        eps = 1e-3
        Jp = torch.zeros_like(J)
        Jm = torch.zeros_like(J)
        tmp = torch.zeros_like(Xd)
        G.gradient(Xd + eps * dd, n, None, tmp, Jp)
        G.gradient(Xd - eps * dd, n, None, tmp, Jm)
        G.sync()
        fd = (Jp.item() - Jm.item()) / (2 * eps)
        an = float(torch.dot(g, dd).item())
        print(f"  direction {trial}: central difference {fd:.10e}  gradient {an:.10e}", flush=True)
        assert abs(fd - an) <= 1e-7 * abs(an)


def test_couette_energy_gain_through_autograd():
    """The energy gain J = E(T) / E(0) built from the autograd Functions (Step with
    checkpoint-and-recompute every 4 steps, Cost): backward() against the oracle's gradient of the
    same quotient and against central differences of the GPU forward map."""
    print("couette autograd energy gain", flush=True)
    cfg = CFGS[0]
    P = Couette(Re=400.0, **cfg)
    dt, n = 0.01, 10
    G = sps.Couette(cfg["Nx"], cfg["Ny"], cfg["Nz"], cfg["Lx"], cfg["Lz"], Re=400.0, dt=dt, checkpoint_every=4,
                    max_steps=n)
    X0 = state(P, 9, 1e-6)
    x0 = dev(to_lib(P, X0)).requires_grad_(True)

    def gain(x):
        return sa.cost(sa.step(x, G, n), G) / sa.cost(x, G)

    J = gain(x0)
    (g,) = torch.autograd.grad(J, x0)
    XN, hist = imex.rk_forward(P, X0, dt, n)
    E0, ET = P.energy(X0), P.energy(XN)
    gT = imex.rk_adjoint(P, P.energy_grad(XN), hist, dt)
    gref = gT / E0 - (ET / E0 ** 2) * P.energy_grad(X0)
    eg = fields(host(g, P), to_lib(P, gref, 1.0), P, "gain gradient")
    print(f"  gain {J.item():.10f} vs {ET / E0:.10f}  gradient rel {eg:.2e}", flush=True)
    assert abs(J.item() - ET / E0) <= 1e-11 * ET / E0
    d = dev(to_lib(P, state(P, 12, 1e-6)))
    eps = 1e-3
    with torch.no_grad():
        fd = (gain(x0.detach() + eps * d).item() - gain(x0.detach() - eps * d).item()) / (2 * eps)
    an = float(torch.dot(g, d).item())
    print(f"  central difference {fd:.10e}  gradient {an:.10e}", flush=True)
    assert abs(fd - an) <= 1e-6 * abs(an)


def test_couette_frame_conversion_through_the_abi():
    """sps_couette_frame against the test's own rotation (to_lib): states (taus doubled) and
    cotangents (taus halved) into the library's frame, and back (round trip to rounding)."""
    print("couette frame conversion", flush=True)
    cfg = CFGS[1]
    P = Couette(Re=400.0, **cfg)
    G = sps.Couette(cfg["Nx"], cfg["Ny"], cfg["Nz"], cfg["Lx"], cfg["Lz"], Re=400.0, dt=0.01, checkpoint_every=1,
                    max_steps=1)
    X = wl.random_state(40, (P.K, P.S), real_first_row=False)
    out = torch.zeros(G.n, dtype=torch.float64, device="cuda")
    back = torch.zeros_like(out)
    for cot, ts in ((False, 2.0), (True, 0.5)):
        G.frame(dev(X), out, to_library=True, cotangent=cot)
        G.frame(out, back, to_library=False, cotangent=cot)
        G.sync()
        ref = to_lib(P, X, ts)
        e1 = np.max(np.abs(host(out, P) - ref)) / np.max(np.abs(ref))
        e2 = np.max(np.abs(host(back, P) - X)) / np.max(np.abs(X))
        print(f"  cotangent={cot}: to library {e1:.1e}, round trip {e2:.1e}", flush=True)
        assert e1 <= 1e-15 and e2 <= 1e-15
    R = sps.Problem(sps.RBC2D, 16, 12, 4.0, 1e6, 1.0, 1.5, 1e-3, 1, 1)
    Z = torch.zeros(R.n, dtype=torch.float64, device="cuda")
    with pytest.raises(sps.SpsError) as e:
        R.frame(Z, Z.clone())
    assert e.value.code == -7
