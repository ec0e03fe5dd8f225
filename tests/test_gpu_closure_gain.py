"""What the trained closure gains over the unclosed coarse solver.

Fine runs of the unclosed solver (512 x 512 modes, Re = 1000, drag 0.1, step 0.00025) from
seeded k^-3 vorticity provide the truth: their states every 8 steps truncated to the 64 x 64
coarse modes.  The closure network is trained on the GPU (rollout loss over 200 coarse steps of
0.002, gradients through the adjoint, Adam) on four runs, and judged on two held-out runs: the
mean rollout error against the truncated fine states must drop by at least 10 % relative to the
coarse solver without the closure, on the same windows."""
import numpy as np
import pytest

import workloads
from oracle import closure as cl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2506_14792_amd import closure_train as ct  # noqa: E402

NF, FAC, RE, DRAG, DT = 512, 8, 1000.0, 0.1, 0.002
NC = NF // FAC


def test_trained_closure_beats_no_closure():
    print("closure gain: fine runs", flush=True)
    ntrain, ntest, n = 4, 2, 200
    c = workloads.kolmo_vorticity(seed=100, N=NF, batch=ntrain + ntest)
    X0 = torch.from_numpy(np.ascontiguousarray(np.transpose(c, (0, 2, 1))).view(np.float64).ravel().copy()).cuda()
    S = ct.fine_snapshots(X0, NF, FAC, RE, DRAG, DT, spinup=16000, nsnap=600)
    assert torch.isfinite(S).all()
    Str, Ste = S[:, :ntrain].contiguous(), S[:, ntrain:].contiguous()
    picks = [(s, b) for s in range(0, 401, 100) for b in range(ntest)]
    J_plain = ct.rollout_losses(Ste, picks, n, NC, RE, DRAG, DT, None)
    theta0 = torch.from_numpy(workloads.closure_theta(seed=0, C=32, scale=1.0)).cuda()
    print("closure gain: training", flush=True)
    theta, losses = ct.train(Str, theta0, n, NC, RE, DRAG, DT, batch=8, iters=40, lr=1e-3,
                             starts=list(range(0, 401, 10)), seed=0)
    assert np.all(np.isfinite(losses))
    J_closed = ct.rollout_losses(Ste, picks, n, NC, RE, DRAG, DT, theta)
    ratio = J_plain.mean() / J_closed.mean()
    print(f"held-out rollout error: no closure {J_plain.mean():.4e}  trained closure {J_closed.mean():.4e}  "
          f"ratio {ratio:.3f}", flush=True)
    assert J_closed.mean() <= 0.9 * J_plain.mean()
