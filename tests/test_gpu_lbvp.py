"""GPU parity of the boundary value problem L X = M f + c of the 2D operator and of its adjoint
(Supplementary, "Linear boundary value problems") against the FP64 oracle, through the C ABI:
the solve and the adjoint at three sizes, the LBVP-then-IVP gradient (sps_lbvp_solve,
sps_gradient, sps_lbvp_adjoint) against the oracle's chain, and the same chain at the full
256 x 64 configuration through torch.autograd against central differences of GPU runs.
Tolerance: 1e-11 of each field's own largest entry (u, w, b, p and the taus, the k = 0 row
and the rows k >= 1 apart, the solution with the conduction state subtracted; tests/parity.py)
(L is conditioned at about 1e5 at 256 x 64)."""
import sys

import numpy as np
import pytest

import workloads as wl
from oracle import imex
from oracle.rbc import RBC
from parity import check_fields

pytestmark = pytest.mark.gpu

TOL = 1e-11

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2506_14792_amd as sps  # noqa: E402
from paper_2506_14792_amd import autograd as sa  # noqa: E402

SMALL = (24, 16, 3.0, 1e5, 0.7, 2e-3)
ODD = (24, 14, 2.5, 3e4, 0.9, 2e-3)
FULL = (256, 64, 4.0, 1e6, 1.0, 1e-3)


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(X):
    return torch.from_numpy(np.ascontiguousarray(X).view(np.float64).ravel().copy()).cuda()


def from_dev(t, shape):
    return t.cpu().numpy().view(np.complex128).reshape(shape)


def rel(a, b):
    return np.max(np.abs(a - b)) / np.max(np.abs(b))


def build(cfg, ce=1, max_steps=1):
    nx, nz, lx, Ra, Pr, dt = cfg
    P = RBC(Nx=nx, Nz=nz, Lx=lx, Ra=Ra, Pr=Pr)
    G = sps.Problem(sps.RBC2D, nx, nz, lx, Ra, Pr, 1.5, dt, ce, max_steps)
    return P, G


def forcing(P, seed, amp, nmodes=4):
    """Smooth forcing: random coefficients in the first nmodes Chebyshev modes of u, w, b at
    every wavenumber (real at k = 0)."""
    rng = np.random.default_rng(seed)
    f = np.zeros((P.K, P.S), dtype=complex)
    for name in ("u", "w", "b"):
        sl = P.sl(name)
        f[:, sl.start:sl.start + nmodes] = amp * (rng.standard_normal((P.K, nmodes))
                                                  + 1j * rng.standard_normal((P.K, nmodes)))
    f[0] = f[0].real
    return f


@pytest.mark.parametrize("cfg", [SMALL, ODD, FULL], ids=["small", "odd", "full"])
def test_lbvp_solve_and_adjoint(cfg):
    note(f"lbvp solve/adjoint parity {cfg}")
    P, G = build(cfg)
    shape = (P.K, P.S)
    f = wl.random_state(31, shape)          # every slot set: p and tau slots must be ignored
    Xb = wl.random_state(32, shape, real_first_row=False)
    X = torch.zeros(G.n, dtype=torch.float64, device="cuda")
    fb = torch.zeros_like(X)
    G.lbvp_solve(to_dev(f), X)
    G.lbvp_adjoint(to_dev(Xb), fb)
    G.sync()
    base = P.lbvp_solve(np.zeros(shape, complex))
    ex = check_fields(from_dev(X, shape), P.lbvp_solve(f), P.Nz, TOL, base=base, what="LBVP X")
    ref = P.lbvp_adjoint(Xb)
    got = from_dev(fb, shape)
    ea = check_fields(got[:, :3 * P.N], ref[:, :3 * P.N], P.Nz, TOL, what="LBVP fbar")
    note(f"  X rel {ex:.2e}  fbar rel {ea:.2e}")
    assert np.abs(got[:, 3 * P.N:]).max() == 0.0
    # a second call reuses the factors and gives the same result bit for bit
    X2 = torch.zeros_like(X)
    G.lbvp_solve(to_dev(f), X2)
    G.sync()
    assert torch.equal(X, X2)


def test_lbvp_then_ivp_gradient_against_oracle():
    note("lbvp -> ivp gradient vs oracle")
    cfg = SMALL
    n, ce = 6, 2
    P, G = build(cfg, ce=ce, max_steps=n)
    shape = (P.K, P.S)
    dt = cfg[5]
    f = forcing(P, 3, 1e-2)
    X0 = P.lbvp_solve(f)
    XN, hist = imex.rk_forward(P, X0, dt, n)
    Jo = P.kinetic_energy(XN)
    fbo = P.lbvp_adjoint(imex.rk_adjoint(P, P.kinetic_energy_grad(XN), hist, dt))
    X0g = torch.zeros(G.n, dtype=torch.float64, device="cuda")
    G.lbvp_solve(to_dev(f), X0g)
    g = torch.zeros_like(X0g)
    J = torch.zeros(1, dtype=torch.float64, device="cuda")
    G.gradient(X0g, n, None, g, J)
    fb = torch.zeros_like(X0g)
    G.lbvp_adjoint(g, fb)
    G.sync()
    eJ = abs(J.item() - Jo) / Jo
    ef = check_fields(from_dev(fb, shape)[:, :3 * P.N], fbo[:, :3 * P.N], P.Nz, TOL, what="dJ/df")
    note(f"  J {J.item():.6e} rel {eJ:.2e}  dJ/df rel {ef:.2e}")
    assert eJ <= TOL


def test_lbvp_chain_full_size_autograd_central_differences():
    """256 x 64, Ra = 1e6: J = kinetic energy after 100 RK222 steps from the LBVP solution,
    differentiated through torch.autograd (Lbvp, Step with checkpoints every 50, Cost); the
    gradient along two random smooth directions against central differences of GPU runs."""
    note("lbvp -> ivp chain 256x64 through autograd")
    n = 100
    P, G = build(FULL, ce=50, max_steps=n)
    f = to_dev(forcing(P, 4, 1e-5)).requires_grad_(True)

    def objective(x):
        return sa.cost(sa.step(sa.lbvp(x, G), G, n), G)

    J = objective(f)
    (gf,) = torch.autograd.grad(J, f)
    note(f"  J = {J.item():.6e}")
    assert 1e-12 < J.item() < 1.0
    for trial in range(2):
        d = to_dev(forcing(P, 10 + trial, 1e-5))
        eps = 1e-2
        with torch.no_grad():
            fd = (objective(f.detach() + eps * d).item() - objective(f.detach() - eps * d).item()) / (2 * eps)
        an = float(torch.dot(gf, d).item())
        note(f"  direction {trial}: central difference {fd:.10e}  gradient {an:.10e}")
        assert abs(fd - an) <= 1e-6 * abs(an)


def test_lbvp_unsupported_for_other_problems():
    note("lbvp on a KS problem")
    G = sps.Problem(sps.KS1D, 64, 0, 32.0 * np.pi, 0.0, 0.0, 1.5, 0.05, 1, 4)
    X = torch.zeros(G.n, dtype=torch.float64, device="cuda")
    with pytest.raises(sps.SpsError) as e:
        G.lbvp_solve(X, X)
    assert e.value.code == -7
