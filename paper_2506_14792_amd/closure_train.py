"""Training of the Kolmogorov-flow closure network on the GPU (argument marshalling and the
training loop only; every step runs in libsps.so).

Data: fine runs of the unclosed solver (N_f x N_f modes, step dt / factor), whose states every
`factor` steps are truncated to the N_c x N_c modes of the coarse grid (N_f = factor N_c).
Objective: the rollout loss of a coarse run with the closure started from a truncated fine state,
J = (1/n) sum_k mean over the coarse grid of (omega_k - truncated fine omega_k)^2, differentiated
through the discrete adjoint of the coarse solver (equ:efficient_gradient), with Adam on the
network's parameters.  The unclosed coarse run on the same windows is the baseline the closure
is judged against.
"""
import numpy as np

from .sps import Kolmogorov, lib


def fine_snapshots(X0, n_fine, factor, re, drag, dt, spinup, nsnap):
    """Run the fine instances in X0 (device state, batch * n_fine^2 doubles) for spinup +
    nsnap * factor fine steps of size dt / factor, keeping every factor-th state truncated to
    the coarse modes (n_fine / factor).  Returns a device tensor [nsnap + 1][batch][coarse
    state]: snapshot 0 is the state after `spinup` steps (a multiple of factor, >= factor)."""
    import torch
    if spinup < factor or spinup % factor:
        raise ValueError("spinup must be a positive multiple of factor")
    nc = n_fine // factor
    B = X0.numel() // (n_fine * n_fine)
    G = Kolmogorov(B, n_fine, Re=re, dt=dt / factor, max_steps=1, closure=False, keep_history=False, drag=drag)
    total = spinup + nsnap * factor
    snap = torch.empty((total // factor) * B * nc * nc, dtype=torch.float64, device=X0.device)
    G.forward(X0, total, snap=snap, every=factor, nc=nc)
    torch.cuda.synchronize()
    G.close()
    return snap.view(total // factor, B, nc * nc)[spinup // factor - 1:].contiguous()


def gather_windows(S, picks, n):
    """Initial states and targets of coarse rollouts: picks = [(start, instance)], S the
    snapshots [T][B][state].  Returns (X0 [len(picks) * state], targets [n][len(picks)][state])."""
    import torch
    s = torch.as_tensor([p[0] for p in picks], device=S.device)
    b = torch.as_tensor([p[1] for p in picks], device=S.device)
    X0 = S[s, b].reshape(-1).contiguous()
    steps = s[None, :] + torch.arange(1, n + 1, device=S.device)[:, None]
    T = S[steps, b[None, :].expand_as(steps)].contiguous()
    return X0, T.reshape(-1)


def rollout_losses(S, picks, n, nc, re, drag, dt, theta=None):
    """Per-window rollout loss of the coarse solver, with the closure (parameters theta) or
    without it (theta None)."""
    import torch
    X0, T = gather_windows(S, picks, n)
    G = Kolmogorov(len(picks), nc, Re=re, dt=dt, max_steps=n, closure=theta is not None, keep_history=True,
                   drag=drag)
    if theta is not None:
        G.set_params(theta)
    J = torch.zeros(len(picks), dtype=torch.float64, device=S.device)
    G.rollout(X0, T, n, J=J)
    torch.cuda.synchronize()
    G.close()
    return J.cpu().numpy()


def train(S, theta0, n, nc, re, drag, dt, batch, iters, lr, starts, seed=0, log=None):
    """Adam on the closure parameters: each iteration draws `batch` windows (start step from
    `starts`, instance uniform), runs the coarse rollout with the closure, its reverse sweep and
    one Adam update with the gradient of the batch's summed loss.  Returns (theta, losses per iteration)."""
    import torch
    rng = np.random.default_rng(seed)
    B = S.shape[1]
    G = Kolmogorov(batch, nc, Re=re, dt=dt, max_steps=n, closure=True, keep_history=True, drag=drag)
    npar = int(lib().sps_cnn_nparam())
    theta = theta0.clone()
    m1 = torch.zeros(npar, dtype=torch.float64, device=S.device)
    m2 = torch.zeros_like(m1)
    g = torch.zeros_like(m1)
    J = torch.zeros(batch, dtype=torch.float64, device=S.device)
    G.set_params(theta)
    losses = []
    for it in range(1, iters + 1):
        picks = [(int(rng.choice(starts)), int(rng.integers(B))) for _ in range(batch)]
        X0, T = gather_windows(S, picks, n)
        G.rollout(X0, T, n, J=J, dJdtheta=g)
        G.adam(theta, g, m1, m2, lr, it)
        losses.append(float(J.mean()))
        if log is not None:
            log(it, losses[-1])
    G.close()
    return theta, losses
