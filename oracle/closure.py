"""Closure network for a coarse periodic 2D run: three 3x3 periodic convolutions
1 -> C -> C -> 1 channels with GELU between them, as an FP64 oracle.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The network is not part of the paper's method; its output is added to the explicit term F
of the coarse problem and its parameters receive gradients through the discrete adjoint
like any parameter of F (equ:efficient_gradient: dJ/dp collects (dF/dp)^H of the step
cotangents).  Precision model: weights and activations are rounded to bfloat16
(round-to-nearest-even) where the GPU stores them in bfloat16, products are accumulated in
FP64 here (FP32 on the GPU); `bf16=False` switches every rounding off for exact-arithmetic
checks.

Layout: a field is (H, W) with x along W; channels first, (C, H, W).  conv(a, w)[o, y, x] =
sum_{c, dy, dx} w[o, c, dy+1, dx+1] a[c, (y+dy) mod H, (x+dx) mod W] + b[o].
GELU is the exact form x Phi(x) = x (1 + erf(x / sqrt 2)) / 2.
"""
import math

import numpy as np
from scipy.special import erf


def bf16(x):
    """Round FP64 values to the nearest bfloat16 (ties to even), returned as FP64."""
    f = np.asarray(x, dtype=np.float32)   # FP64 -> FP32 is itself round-to-nearest-even
    b = f.view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    b = (b + 0x7FFF + lsb) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def conv3(a, w, b):
    """Periodic 3x3 convolution, channels first: a (C, H, W), w (O, C, 3, 3), b (O,)."""
    O = w.shape[0]
    out = np.zeros((O,) + a.shape[1:])
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            sh = np.roll(a, shift=(-dy, -dx), axis=(1, 2))   # sh[c, y, x] = a[c, y+dy, x+dx]
            out += np.einsum("oc,cyx->oyx", w[:, :, dy + 1, dx + 1], sh)
    return out + b[:, None, None]


def conv3_adjoint_input(g, w):
    """Transpose of a -> conv3(a, w, 0) applied to g (O, H, W) -> (C, H, W)."""
    C = w.shape[1]
    out = np.zeros((C,) + g.shape[1:])
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            t = np.einsum("oc,oyx->cyx", w[:, :, dy + 1, dx + 1], g)
            out += np.roll(t, shift=(dy, dx), axis=(1, 2))
    return out


def conv3_adjoint_weight(a, g):
    """d/dw of sum(g * conv3(a, w, b)): (O, C, 3, 3); d/db: (O,)."""
    O, C = g.shape[0], a.shape[0]
    dw = np.zeros((O, C, 3, 3))
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            sh = np.roll(a, shift=(-dy, -dx), axis=(1, 2))
            dw[:, :, dy + 1, dx + 1] = np.einsum("oyx,cyx->oc", g, sh)
    return dw, g.sum(axis=(1, 2))


def init_params(seed=0, C=32, scale=1.0):
    """Seeded initial weights (random draws only, from the shared input generators)."""
    import workloads
    return workloads.closure_params(seed, C, scale)


def forward(p, x, bf=True):
    """Network output for one field x (H, W).  Returns (y (H, W), cache)."""
    r = bf16 if bf else (lambda v: np.asarray(v, dtype=np.float64))
    w1, w2, w3 = r(p["w1"]), r(p["w2"]), r(p["w3"])
    a0 = r(x)[None]
    z1 = conv3(a0, w1, p["b1"])
    a1 = r(gelu(z1))
    z2 = conv3(a1, w2, p["b2"])
    a2 = r(gelu(z2))
    y = conv3(a2, w3, p["b3"])[0]
    return y, (a0, z1, a1, z2, a2, w1, w2, w3)


def vjp(p, x, ybar, bf=True):
    """Cotangents of the input field and of every parameter for output cotangent ybar (H, W).
    The backward pass keeps FP64 cotangents (the GPU keeps FP32); stored bf16 activations and
    weights are the ones the forward pass used."""
    _, (a0, z1, a1, z2, a2, w1, w2, w3) = forward(p, x, bf)
    g3 = ybar[None]
    dw3, db3 = conv3_adjoint_weight(a2, g3)
    g2 = conv3_adjoint_input(g3, w3) * gelu_grad(z2)
    dw2, db2 = conv3_adjoint_weight(a1, g2)
    g1 = conv3_adjoint_input(g2, w2) * gelu_grad(z1)
    dw1, db1 = conv3_adjoint_weight(a0, g1)
    xbar = conv3_adjoint_input(g1, w1)[0]
    return xbar, {"w1": dw1, "b1": db1, "w2": dw2, "b2": db2, "w3": dw3, "b3": db3}


PARAM_ORDER = ("w1", "b1", "w2", "b2", "w3", "b3")


def flatten(p):
    return np.concatenate([np.asarray(p[k], dtype=np.float64).ravel() for k in PARAM_ORDER])


def unflatten(v, C=32):
    shapes = {"w1": (C, 1, 3, 3), "b1": (C,), "w2": (C, C, 3, 3), "b2": (C,), "w3": (1, C, 3, 3), "b3": (1,)}
    out, o = {}, 0
    for k in PARAM_ORDER:
        n = int(np.prod(shapes[k]))
        out[k] = v[o:o + n].reshape(shapes[k])
        o += n
    return out
