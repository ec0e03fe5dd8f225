"""The closure network on the GPU (bf16 weights and activations, FP32 accumulation, MFMA for
the 32 -> 32 layer) against the FP64 oracle that emulates the same bf16 roundings.

Bound.  Both sides round the same values to bf16; they differ by FP32 versus FP64
accumulation (at most K 2^-24 of the sum of magnitudes, K = 288 terms) and by an occasional
activation that lands on the other side of a bf16 rounding boundary (one bf16 ulp, 2^-8 of
that activation).  Per output pixel, with S_p = sum |w3| |a2| over the pixel's 3x3 x 32
inputs (the magnitude the output is a sum of), the test requires
max_p |y_gpu - y_oracle| / S_p <= 2^-5 (a few flips, amplified once by a layer) and the median
<= 2^-13.  Cotangents (FP32 on the GPU, FP64 in the oracle) of the input and of every parameter
array: max error <= 2^-7 and median <= 2^-13 relative to the array's largest magnitude."""
import numpy as np
import pytest

from oracle import closure as cl
import workloads

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
    yr, xr, tr = [], [], None
    ratios = []
    for i in range(B):
        yo, cache = cl.forward(p, x[i], bf=True)
        a2, w3 = cache[4], cache[7]
        S = cl.conv3(np.abs(a2), np.abs(w3), np.zeros(1))[0]
        ratios.append(np.abs(y[i] - yo) / S)
        xo, po = cl.vjp(p, x[i], yb[i], bf=True)
        xr.append(xo)
        f = cl.flatten(po)
        tr = f if tr is None else tr + f
    ratios = np.concatenate([r.ravel() for r in ratios])
    print(f"forward: max {ratios.max():.3e} median {np.median(ratios):.3e} of S_p", flush=True)
    assert ratios.max() <= 2.0 ** -5 and np.median(ratios) <= 2.0 ** -13
    ex = np.abs(xb - np.stack(xr)) / np.max(np.abs(xr))
    print(f"input cotangent: max {ex.max():.3e} median {np.median(ex):.3e}", flush=True)
    assert ex.max() <= 2.0 ** -7 and np.median(ex) <= 2.0 ** -13
    tp = cl.unflatten(tb)
    to = cl.unflatten(tr)
    for k in cl.PARAM_ORDER:
        e = np.abs(tp[k] - to[k]) / np.max(np.abs(to[k]))
        print(f"{k}: max {e.max():.3e} median {np.median(e):.3e}", flush=True)
        assert e.max() <= 2.0 ** -7 and np.median(e) <= 2.0 ** -13, k
