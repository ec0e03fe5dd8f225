"""Element-wise error bounds of the closure network on the GPU (bf16 weights and activations,
FP32 arithmetic, MFMA for the 32 -> 32 layer) against the FP64 oracle that rounds the same values
to bf16, derived from the two implementations' arithmetic and evaluated on the oracle's own
intermediate values.

Rounding model (u = 2^-24, the FP32 unit roundoff):
* A sum of K products and a bias accumulated in FP32 (any order, FMA or not) differs from the
  exact sum by at most K u times the sum of the magnitudes; the bias's own rounding to FP32 is
  one more term.  Every accumulation bound below carries a factor 2 on top.
* GELU and its derivative in FP32 (erff, expf and a few products, each within 2 ulps) are
  within GE(z) = 2^-21 |gelu(z)| + 2^-23 |z| (the second term: erff's absolute error times |z|/2
  where 1 + erf cancels) and GDE(z) = 2^-20 (1 + |z|) of the exact functions (a factor 2 over
  the ulp counts).
* Both sides round an activation to bf16 (round to nearest even, through FP32).  If the FP32
  value on the GPU and the FP64 value of the oracle differ by at most d, the rounded
  activations are equal unless a bf16 rounding boundary (the midpoint between two neighbouring
  bf16 numbers) lies within d (+ u |v| for the FP32 step) of the oracle's value; then they differ
  by one bf16 spacing.  The bound counts exactly those possible flips, per activation.
* Differences propagate through a layer by the absolute weights (|W| |da|), and through GELU by
  |gelu'| (plus the curvature over the interval, |gelu''| <= 0.8 times the interval's half-width).

Parameter gradients accumulate in FP32 over chunks of pixels (64 for the small arrays, 128 per
wave then 4 waves for the 32 x 32 layer) before an FP64 sum over chunks; their bounds use those
chunk lengths.  The oracle's FP64 rounding is negligible beside all of this.
"""
import numpy as np

from oracle import closure as cl

U = 2.0 ** -24


def _absconv(a, w):
    return cl.conv3(np.abs(a), np.abs(w), np.zeros(w.shape[0]))


def _absconv_t(g, w):
    return cl.conv3_adjoint_input(np.abs(g), np.abs(w))


def _absconv_w(a, g):
    return cl.conv3_adjoint_weight(np.abs(a), np.abs(g))[0]


def gelu_err(z):
    return 2.0 ** -21 * np.abs(cl.gelu(z)) + 2.0 ** -23 * np.abs(z)


def gelu_d_err(z):
    return 2.0 ** -20 * (1.0 + np.abs(z))


def bf16_flip(v, d):
    """Largest possible difference of bf16(v') and bf16(v) for |v' - v| <= d: one bf16 spacing
    where a rounding boundary lies within d (+ the FP32 step) of v, else zero.  Also returns
    the mask of possible flips."""
    v = np.asarray(v, dtype=np.float64)
    b = cl.bf16(v)
    bits = b.astype(np.float32).view(np.uint32).astype(np.int64)
    up = ((bits + 0x10000) & 0xFFFFFFFF).astype(np.uint32).view(np.float32).astype(np.float64)
    dn = ((bits - 0x10000) & 0xFFFFFFFF).astype(np.uint32).view(np.float32).astype(np.float64)
    # at zero both neighbours are the smallest normal bf16 of either sign
    tiny = 2.0 ** -126
    up = np.where(b == 0.0, tiny, up)
    dn = np.where(b == 0.0, -tiny, dn)
    dist = np.minimum(np.abs(v - 0.5 * (b + up)), np.abs(v - 0.5 * (b + dn)))
    flip = dist <= d + U * np.abs(v)
    spacing = np.maximum(np.abs(up - b), np.abs(b - dn))
    return np.where(flip, spacing, 0.0), flip


def forward_bound(p, x):
    """Per-pixel bound of |y_gpu - y_oracle| for one image x (H, W), and the oracle's
    intermediates.  Returns (y_oracle, bound, cache, deltas) with deltas the bounds on the
    pre-activations and activations that the backward bound reuses."""
    y, cache = cl.forward(p, x, bf=True)
    a0, z1, a1, z2, a2, w1, w2, w3 = cache
    b1, b2, b3 = (np.asarray(p[k], dtype=np.float64) for k in ("b1", "b2", "b3"))
    dz1 = 2.0 * 10 * U * (_absconv(a0, w1) + np.abs(b1)[:, None, None])
    dv1 = (np.abs(cl.gelu_grad(z1)) + 0.8 * dz1) * dz1 + gelu_err(z1)
    da1, f1 = bf16_flip(cl.gelu(z1), dv1)
    dz2 = 2.0 * 289 * U * (_absconv(a1, w2) + np.abs(b2)[:, None, None]) + _absconv(da1, w2)
    dv2 = (np.abs(cl.gelu_grad(z2)) + 0.8 * dz2) * dz2 + gelu_err(z2)
    da2, f2 = bf16_flip(cl.gelu(z2), dv2)
    dy = 2.0 * 289 * U * (_absconv(a2, w3)[0] + abs(float(b3[0]))) + _absconv(da2, w3)[0]
    return y, dy, cache, dict(dz1=dz1, da1=da1, dz2=dz2, da2=da2, flips1=int(f1.sum()), flips2=int(f2.sum()))


def vjp_bound(p, x, ybar, cache, dl):
    """Bounds of |gpu - oracle| for the input cotangent (H, W) and the parameter cotangents
    (dict of arrays) of one image, given forward_bound's cache and deltas."""
    a0, z1, a1, z2, a2, w1, w2, w3 = cache
    g3 = np.asarray(ybar, dtype=np.float64)[None]
    dg3 = U * np.abs(g3)
    a2bar = cl.conv3_adjoint_input(g3, w3)
    da2bar = 2.0 * 10 * U * _absconv_t(g3, w3) + _absconv_t(dg3, w3)
    gd2 = cl.gelu_grad(z2)
    g2 = a2bar * gd2
    dg2 = da2bar * (np.abs(gd2) + 0.8 * dl["dz2"]) + np.abs(a2bar) * (0.8 * dl["dz2"] + gelu_d_err(z2)) + U * np.abs(g2)
    a1bar = cl.conv3_adjoint_input(g2, w2)
    da1bar = 2.0 * 289 * U * _absconv_t(g2, w2) + _absconv_t(dg2, w2)
    gd1 = cl.gelu_grad(z1)
    g1 = a1bar * gd1
    dg1 = da1bar * (np.abs(gd1) + 0.8 * dl["dz1"]) + np.abs(a1bar) * (0.8 * dl["dz1"] + gelu_d_err(z1)) + U * np.abs(g1)
    dxb = 2.0 * 289 * U * _absconv_t(g1, w1)[0] + _absconv_t(dg1, w1)[0]
    # parameter cotangents: FP32 chunks (64 pixels; 128 per wave + 4 waves for w2) before FP64
    da1, da2 = dl["da1"], dl["da2"]
    out = {
        "w3": 2.0 * 64 * U * _absconv_w(a2, g3) + _absconv_w(a2, dg3) + _absconv_w(da2, g3),
        "b3": np.array([2.0 * 64 * U * np.abs(g3).sum() + dg3.sum()]),
        "w2": 2.0 * 132 * U * _absconv_w(a1, g2) + _absconv_w(a1, dg2) + _absconv_w(da1, np.abs(g2) + dg2),
        "b2": 2.0 * 64 * U * np.abs(g2).sum(axis=(1, 2)) + dg2.sum(axis=(1, 2)),
        "w1": 2.0 * 64 * U * _absconv_w(a0, g1) + _absconv_w(a0, dg1),
        "b1": 2.0 * 64 * U * np.abs(g1).sum(axis=(1, 2)) + dg1.sum(axis=(1, 2)),
    }
    return dxb, out
