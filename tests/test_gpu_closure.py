"""The closure network on the GPU (bf16 weights and activations, FP32 accumulation, MFMA for
the 32 -> 32 layer) against the FP64 oracle that emulates the same bf16 roundings.

Bound.  Every output pixel, input-cotangent pixel and parameter-cotangent entry is held to an
element-wise bound derived from the two implementations' arithmetic (tests/closure_bound.py):
FP32 accumulation of K terms (K u times the sum of magnitudes, u = 2^-24, with a factor 2),
FP32 GELU evaluation, and one bf16 spacing for exactly those activations whose oracle value
lies within the propagated difference of a bf16 rounding boundary (a possible flip), carried
through the following layers by the absolute weights.  A pixel with no nearby boundary is thus
held at the accumulation level (about 3e-5 of its sum of magnitudes), and a wrong tap anywhere,
the periodic border included, shows at once; the border rows and columns are also reported on
their own."""
import numpy as np
import pytest

from oracle import closure as cl
import workloads
from closure_bound import forward_bound, vjp_bound

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2506_14792_amd as sps  # noqa: E402


def params(seed):
    rng = np.random.default_rng(seed)
    p = workloads.closure_params(seed=seed, C=32, scale=1.0)
    p["w3"] = p["w3"] * 100.0
    for k in ("b1", "b2", "b3"):
        p[k] = 0.2 * rng.standard_normal(p[k].shape)
    return p


@pytest.mark.parametrize("shape", [(3, 64, 64), (2, 16, 32)], ids=["64x64", "16x32"])
def test_closure_net_forward_and_vjp(shape):
    print(f"closure net {shape}", flush=True)
    B, H, W = shape
    p = params(7)
    theta = torch.from_numpy(cl.flatten(p)).cuda()
    rng = np.random.default_rng(8)
    x = rng.standard_normal((B, H, W))
    yb = rng.standard_normal((B, H, W))
    net = sps.ClosureNet(B, H, W)
    assert net.nparam == theta.numel()
    net.set_params(theta)
    xd = torch.from_numpy(x.ravel().copy()).cuda()
    y = torch.zeros_like(xd)
    net.forward(xd, y)
    xb = torch.zeros_like(xd)
    tb = torch.zeros_like(theta)
    net.vjp(xd, torch.from_numpy(yb.ravel().copy()).cuda(), xb, tb)
    net.vjp(xd, torch.from_numpy(yb.ravel().copy()).cuda(), xb, tb)   # theta_bar accumulates
    torch.cuda.synchronize()
    y, xb, tb = y.cpu().numpy().reshape(B, H, W), xb.cpu().numpy().reshape(B, H, W), tb.cpu().numpy() / 2
    ry, rx, tr, tbound = [], [], None, None
    border = np.zeros((H, W), bool)
    border[[0, -1], :] = True
    border[:, [0, -1]] = True
    flips = [0, 0]
    for i in range(B):
        yo, by, cache, dl = forward_bound(p, x[i])
        flips[0] += dl["flips1"]
        flips[1] += dl["flips2"]
        ry.append(np.abs(y[i] - yo) / by)
        xo, po = cl.vjp(p, x[i], yb[i], bf=True)
        bx, bp = vjp_bound(p, x[i], yb[i], cache, dl)
        rx.append(np.abs(xb[i] - xo) / bx)
        f = cl.flatten(po)
        g = cl.flatten(bp)
        tr = f if tr is None else tr + f
        tbound = g if tbound is None else tbound + g
    ry, rx = np.stack(ry), np.stack(rx)
    print(f"possible bf16 flips: layer 1 {flips[0]}, layer 2 {flips[1]} of {B * H * W * 32} activations each",
          flush=True)
    print(f"forward: max |dy| / bound {ry.max():.3f} (border {ry[:, border].max():.3f})", flush=True)
    print(f"input cotangent: max |dx| / bound {rx.max():.3f} (border {rx[:, border].max():.3f})", flush=True)
    assert ry.max() <= 1.0 and rx.max() <= 1.0
    # and the bulk: median errors far below the bounds' rounding level
    xr = np.stack([cl.vjp(p, x[i], yb[i], bf=True)[0] for i in range(B)])
    ex = np.abs(xb - xr) / np.max(np.abs(xr))
    print(f"input cotangent: median {np.median(ex):.2e} of the largest", flush=True)
    assert np.median(ex) <= 2.0 ** -13
    tp, to, tbd = cl.unflatten(tb), cl.unflatten(tr), cl.unflatten(tbound)
    for k in cl.PARAM_ORDER:
        r = np.abs(tp[k] - to[k]) / tbd[k]
        e = np.abs(tp[k] - to[k]) / np.max(np.abs(to[k]))
        print(f"{k}: max |d| / bound {r.max():.3f}, median {np.median(e):.2e} of the largest", flush=True)
        assert r.max() <= 1.0 and np.median(e) <= 2.0 ** -13, k
