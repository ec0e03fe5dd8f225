"""Graph mode of sps_gradient: the recorded graph, replayed several times with eager work
and synchronizations in between, gives exactly (bitwise) the eager result every time, for
a run with several checkpoint segments (two streams in the reverse sweep) and for a
single-segment run."""
import numpy as np
import pytest

from oracle.rbc import RBC
import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2506_14792_amd as sps  # noqa: E402

SMALL = (24, 16, 3.0, 1e5, 0.7, 2e-3)
FULL = (256, 64, 4.0, 1e6, 1.0, 1e-3)


@pytest.mark.parametrize("cfg,nsteps,ce", [(SMALL, 7, 3), (SMALL, 3, 5), (FULL, 6, 4)],
                         ids=["small-3seg", "small-1seg", "full-2seg"])
def test_graph_replays_match_eager(cfg, nsteps, ce):
    print(f"graph replay {cfg} x {nsteps} ce={ce}", flush=True)
    nx, nz, lx, Ra, Pr, dt = cfg
    P = RBC(Nx=nx, Nz=nz, Lx=lx, Ra=Ra, Pr=Pr)
    G = sps.Problem(sps.RBC2D, nx, nz, lx, Ra, Pr, 1.5, dt, ce, nsteps)
    X0 = torch.from_numpy(P.initial_state(wl.rbc_b0(seed=31, Nx=nx, Nz=nz, amp=0.1)).view(np.float64).ravel().copy()).cuda()
    XN = torch.zeros(G.n, dtype=torch.float64, device="cuda")
    g = torch.zeros_like(XN)
    J = torch.zeros(1, dtype=torch.float64, device="cuda")
    G.gradient(X0, nsteps, XN, g, J)
    G.sync()
    ref = (XN.clone(), g.clone(), J.clone())
    G.set_graph(True)
    scratch = torch.zeros_like(XN)
    for rep in range(3):
        XN.zero_()
        g.zero_()
        J.zero_()
        G.gradient(X0, nsteps, XN, g, J)
        G.sync()
        assert torch.equal(XN, ref[0]) and torch.equal(g, ref[1]) and torch.equal(J, ref[2]), f"replay {rep}"
        # eager work of the program between replays
        G.eval_F(X0, scratch)
        G.sync()
        torch.cuda.synchronize()
    # a second argument tuple records its own graph
    g2 = torch.zeros_like(g)
    G.gradient(X0, nsteps, None, g2, None)
    G.sync()
    assert torch.equal(g2, ref[1])
    G.set_graph(False)
    g.zero_()
    G.gradient(X0, nsteps, None, g, None)
    G.sync()
    assert torch.equal(g, ref[1])


def test_graph_mode_unsupported_for_ks():
    G = sps.Problem(sps.KS1D, 64, 0, 32.0 * np.pi, 0.0, 0.0, 1.5, 0.05, 1, 4)
    with pytest.raises(sps.SpsError):
        G.set_graph(True)
