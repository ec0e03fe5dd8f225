"""Pins of the closure-network oracle: periodic convolution against numpy FFT circular
convolution, dot-product tests of both adjoints, GELU against x Phi(x) from scipy, bfloat16
rounding against torch's bfloat16 conversion, and central differences of the exact-arithmetic
VJP for inputs and every parameter array."""
import numpy as np
from scipy.stats import norm

from oracle import closure as cl


def test_conv_is_circular_convolution():
    rng = np.random.default_rng(0)
    a = rng.standard_normal((3, 8, 10))
    w = rng.standard_normal((2, 3, 3, 3))
    b = rng.standard_normal(2)
    got = cl.conv3(a, w, b)
    # correlation with a 3x3 stencil = circular convolution with the flipped stencil
    ref = np.zeros_like(got)
    for o in range(2):
        for c in range(3):
            k = np.zeros((8, 10))
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    k[(-dy) % 8, (-dx) % 10] = w[o, c, dy + 1, dx + 1]
            ref[o] += np.real(np.fft.ifft2(np.fft.fft2(a[c]) * np.fft.fft2(k)))
        ref[o] += b[o]
    assert np.allclose(got, ref, atol=1e-12)


def test_adjoints_inner_products():
    rng = np.random.default_rng(1)
    a = rng.standard_normal((4, 6, 7))
    w = rng.standard_normal((5, 4, 3, 3))
    g = rng.standard_normal((5, 6, 7))
    lhs = np.sum(cl.conv3(a, w, np.zeros(5)) * g)
    assert np.isclose(lhs, np.sum(a * cl.conv3_adjoint_input(g, w)), rtol=1e-12)
    dw, db = cl.conv3_adjoint_weight(a, g)
    assert np.isclose(lhs, np.sum(w * dw), rtol=1e-12)
    assert np.allclose(db, g.sum(axis=(1, 2)))


def test_gelu_and_its_derivative():
    x = np.linspace(-6, 6, 241)
    assert np.allclose(cl.gelu(x), x * norm.cdf(x), atol=1e-15)
    h = 1e-5
    fd = (cl.gelu(x + h) - cl.gelu(x - h)) / (2 * h)
    assert np.allclose(cl.gelu_grad(x), fd, atol=1e-9)


def test_bf16_rounding_matches_torch():
    import torch
    rng = np.random.default_rng(2)
    v = np.concatenate([rng.standard_normal(2000) * 10.0 ** rng.integers(-6, 6, 2000),
                        [1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -(1.0 + 2.0 ** -8), 0.0, 65504.0]])
    ref = torch.from_numpy(v).to(torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(cl.bf16(v), ref)


def test_vjp_central_differences():
    rng = np.random.default_rng(3)
    C = 4
    p = cl.init_params(seed=4, C=C, scale=1.0)
    p["w3"] = p["w3"] * 100.0
    for k in ("b1", "b2", "b3"):
        p[k] = 0.1 * rng.standard_normal(p[k].shape)
    x = rng.standard_normal((6, 5))
    ybar = rng.standard_normal((6, 5))
    xbar, pbar = cl.vjp(p, x, ybar, bf=False)

    def J(pp, xx):
        return np.sum(ybar * cl.forward(pp, xx, bf=False)[0])

    h = 1e-6
    for idx in [(0, 0), (3, 4), (5, 2)]:
        e = np.zeros_like(x)
        e[idx] = h
        fd = (J(p, x + e) - J(p, x - e)) / (2 * h)
        assert np.isclose(fd, xbar[idx], rtol=1e-6, atol=1e-9)
    for k in cl.PARAM_ORDER:
        flat = p[k].ravel()
        for i in range(0, flat.size, max(1, flat.size // 5)):
            pp, pm = {q: v.copy() for q, v in p.items()}, {q: v.copy() for q, v in p.items()}
            pp[k].ravel()[i] += h
            pm[k].ravel()[i] -= h
            fd = (J(pp, x) - J(pm, x)) / (2 * h)
            assert np.isclose(fd, pbar[k].ravel()[i], rtol=1e-6, atol=1e-9), (k, i)
