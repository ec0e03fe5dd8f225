"""Variable steps inside one recorded run of the 2D problem (sps_set_timesteps: step i + 1 takes
dts[i] in its stage coefficients and its own factors of M + dts[i] H_ii L) against the FP64
oracle's chain of single steps of the same sizes and their adjoints: the final state, J, dJ/dX0,
dJ/dRa and dJ/dPr, under ARS(2,2,2) and ARS(4,4,3), with ragged checkpoint segments; the
binomial and two-level schedules and graph replay give the uniform schedule's bits; a batch;
refusals.  Bounds: tests/parity.py (1e-11 of each field group)."""
import sys

import numpy as np
import pytest

from oracle import imex
from oracle.rbc import RBC
import workloads as wl
from parity import check_fields

pytestmark = pytest.mark.gpu

TOL = 1e-11

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2506_14792_amd as sps  # noqa: E402

SMALL = (24, 16, 3.0, 1e5, 0.7)
FULL = (256, 64, 4.0, 1e6, 1.0)
TABS = {sps.RK222: None, sps.RK443: imex.ars443_tableau()}


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(X):
    return torch.from_numpy(np.ascontiguousarray(X).view(np.float64).ravel().copy()).cuda()


def from_dev(t, shape):
    return t.cpu().numpy().view(np.complex128).reshape(shape)


def oracle_chain(P, X0, dts, tab, params=False):
    """Forward run of single steps of sizes dts and the reverse sweep step by step."""
    X, hists, states = np.array(X0, complex), [], [np.array(X0, complex)]
    for dt in dts:
        X, h = imex.rk_forward(P, X, dt, 1, tableau=tab)
        hists.append(h)
        states.append(X)
    J = P.kinetic_energy(X)
    Y = P.kinetic_energy_grad(X)
    th = np.zeros(2)
    for n in range(len(dts) - 1, -1, -1):
        if params:
            Y, g = imex.rk_adjoint(P, Y, hists[n], dts[n], tableau=tab, dLs=P.param_dL(), XN=states[n + 1])
            th += g
        else:
            Y = imex.rk_adjoint(P, Y, hists[n], dts[n], tableau=tab)
    return X, J, Y, th


def build(cfg, scheme, ce, max_steps):
    nx, nz, lx, Ra, Pr = cfg
    P = RBC(Nx=nx, Nz=nz, Lx=lx, Ra=Ra, Pr=Pr)
    G = sps.Problem(sps.RBC2D, nx, nz, lx, Ra, Pr, 1.5, 2e-3, ce, max_steps, scheme=scheme)
    return P, G


@pytest.mark.parametrize("scheme", [sps.RK222, sps.RK443], ids=["rk222", "rk443"])
def test_variable_steps_small(scheme):
    dts = [2e-3, 2e-3, 1e-3, 1e-3, 1.5e-3, 2e-3, 7e-4]
    n = len(dts)
    note(f"variable steps 24x16 scheme {scheme}: {dts}")
    P, G = build(SMALL, scheme, 3, n)
    G.set_timesteps(dts)
    X0 = P.initial_state(wl.rbc_b0(seed=51, Nx=SMALL[0], Nz=SMALL[1], amp=0.1))
    XN_r, J_r, g_r, th_r = oracle_chain(P, X0, dts, TABS[scheme], params=True)
    x0 = to_dev(X0)
    XN, g = torch.zeros_like(x0), torch.zeros_like(x0)
    J = torch.zeros(1, dtype=torch.float64, device="cuda")
    th = torch.zeros(2, dtype=torch.float64, device="cuda")
    G.gradient(x0, n, XN, g, J, dJdtheta=th)
    G.sync()
    base = P.lbvp_solve(np.zeros((P.K, P.S), complex))
    check_fields(from_dev(XN, X0.shape), XN_r, P.Nz, TOL, base=base, what="X_N")
    check_fields(from_dev(g, X0.shape), g_r, P.Nz, TOL, what="dJ/dX0")
    eJ = abs(J.item() - J_r) / abs(J_r)
    e = np.abs(th.cpu().numpy() - th_r) / np.abs(th_r)
    note(f"  J rel {eJ:.1e}; dJ/dRa rel {e[0]:.1e}, dJ/dPr rel {e[1]:.1e}")
    assert eJ <= TOL and np.all(e <= TOL)
    # graph replay, binomial and two-level schedules: the same bits
    G.set_graph(True)
    for _ in range(2):
        g2 = torch.zeros_like(g)
        G.gradient(x0, n, None, g2, None)
        G.sync()
        assert torch.equal(g2, g)
    G.set_graph(False)
    for ck, slots in ((sps.CKPT_BINOMIAL, 2), (sps.CKPT_TWO_LEVEL, 1)):
        G.set_checkpointing(ck, slots)
        g2 = torch.zeros_like(g)
        G.gradient(x0, n, None, g2, None)
        G.sync()
        note(f"  schedule {ck}: bit-identical {torch.equal(g2, g)}")
        assert torch.equal(g2, g)
    G.set_checkpointing(sps.CKPT_UNIFORM)
    # back to the constant step: the constant-step run of the oracle
    G.set_timesteps(None)
    X = x0.clone()
    G.step(X, 3)
    G.sync()
    Xc, _ = imex.rk_forward(P, X0, 2e-3, 3, tableau=TABS[scheme])
    check_fields(from_dev(X, X0.shape), Xc, P.Nz, TOL, base=base, what="constant-step X_3")


def test_variable_steps_full_size():
    dts = [1e-3, 5e-4, 5e-4, 1e-3]
    note(f"variable steps 256x64: {dts}")
    P, G = build(FULL, sps.RK222, 2, len(dts))
    G.set_timesteps(dts)
    X0 = P.initial_state(wl.rbc_b0(seed=52, Nx=FULL[0], Nz=FULL[1], amp=0.1))
    XN_r, J_r, g_r, _ = oracle_chain(P, X0, dts, None)
    x0 = to_dev(X0)
    g = torch.zeros_like(x0)
    J = torch.zeros(1, dtype=torch.float64, device="cuda")
    G.gradient(x0, len(dts), None, g, J)
    G.sync()
    check_fields(from_dev(g, X0.shape), g_r, P.Nz, TOL, what="dJ/dX0")
    assert abs(J.item() - J_r) <= TOL * abs(J_r)


def test_variable_steps_batch_and_refusals():
    nx, nz, lx, _, Pr = SMALL
    ras, dts = (1e5, 3e4), [2e-3, 1e-3, 1e-3, 1.5e-3]
    note("variable steps, batch of two")
    G = sps.RbcBatch(list(ras), nx, nz, lx, Pr, dt=2e-3, checkpoint_every=2, max_steps=len(dts))
    G.set_timesteps(dts)
    Ps = [RBC(Nx=nx, Nz=nz, Lx=lx, Ra=r, Pr=Pr) for r in ras]
    Xs = [P.initial_state(wl.rbc_b0(seed=53 + b, Nx=nx, Nz=nz, amp=0.1)) for b, P in enumerate(Ps)]
    X0 = torch.from_numpy(np.concatenate([X.view(np.float64).ravel() for X in Xs])).cuda()
    g = torch.zeros_like(X0)
    G.gradient(X0, len(dts), None, g, None)
    G.sync()
    gh = g.cpu().numpy().view(np.complex128).reshape((2,) + Xs[0].shape)
    for b, P in enumerate(Ps):
        _, _, g_r, _ = oracle_chain(P, Xs[b], dts, None)
        check_fields(gh[b], g_r, nz, TOL, what=f"instance {b} dJ/dX0")
    # a run longer than the steps set, too many distinct steps, a non-positive step
    with pytest.raises(sps.SpsError) as e:
        G2 = sps.Problem(sps.RBC2D, nx, nz, lx, 1e5, Pr, 1.5, 2e-3, 2, 20)
        G2.set_timesteps([1e-3, 2e-3])
        G2.step(torch.zeros(G2.n, dtype=torch.float64, device="cuda"), 3)
    assert e.value.code == -1
    with pytest.raises(sps.SpsError) as e:
        G2.set_timesteps([1e-3 * (1 + k) for k in range(17)])
    assert e.value.code == -1
    with pytest.raises(sps.SpsError) as e:
        G2.set_timesteps([1e-3, 0.0])
    assert e.value.code == -1
