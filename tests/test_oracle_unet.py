"""Pins of the network oracle (learned coarse-grid correction): the
convolution against a library correlation, pooling / upsampling adjointness
and closed forms, every parameter gradient against central finite
differences of the forward pass, BF16 rounding against torch's conversion,
and the first Adam step against its closed form."""
import numpy as np
import pytest
import scipy.ndimage as ndi
import torch

from oracle import unet


def test_conv_single_channel_is_library_correlation():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((1, 6, 6, 6, 1))
    w = rng.standard_normal((1, 27, 1))
    K = np.zeros((3, 3, 3))
    for t, dx, dy, dz in unet.taps():
        K[dz + 1, dy + 1, dx + 1] = w[0, t, 0]
    ref = ndi.correlate(x[0, ..., 0], K, mode="constant", cval=0.0)
    np.testing.assert_allclose(unet.conv(x, w)[0, ..., 0], ref, rtol=1e-13, atol=1e-13)


def test_conv_multichannel_is_sum_of_single_channel():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, 4, 4, 4, 3))
    w = rng.standard_normal((2, 27, 3))
    y = unet.conv(x, w)
    for b in range(2):
        for co in range(2):
            ref = 0
            for ci in range(3):
                K = np.zeros((3, 3, 3))
                for t, dx, dy, dz in unet.taps():
                    K[dz + 1, dy + 1, dx + 1] = w[co, t, ci]
                ref = ref + ndi.correlate(x[b, ..., ci], K, mode="constant")
            np.testing.assert_allclose(y[b, ..., co], ref, rtol=1e-12, atol=1e-12)


def test_pool_and_up_adjoint_and_closed_forms():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, 8, 8, 8, 3))
    y = rng.standard_normal((2, 4, 4, 4, 3))
    assert np.isclose((unet.pool(x) * y).sum(), (x * unet.pool_bwd(y)).sum(), rtol=1e-12)
    assert np.isclose((unet.up(y) * x).sum(), (y * unet.up_bwd(x)).sum(), rtol=1e-12)
    c = np.full((1, 4, 4, 4, 1), 2.5)
    np.testing.assert_allclose(unet.pool(c), 2.5)
    np.testing.assert_allclose(unet.pool(unet.up(y)), y, rtol=1e-14)
    # one child block: the mean of its 8 values
    assert np.isclose(unet.pool(x)[1, 2, 3, 1, 2], x[1, 4:6, 6:8, 2:4, 2].mean())


def _problem(seed, G=8, B=2):
    rng = np.random.default_rng(seed)
    # He-scaled weights keep activations O(1), so +-eps rarely crosses a ReLU kink
    theta = np.concatenate([np.concatenate([rng.standard_normal(co * 27 * ci) * np.sqrt(2.0 / (27 * ci)),
                                            0.1 * rng.standard_normal(co)]) for ci, co, _, _ in unet.LAYERS])
    inp = np.zeros((B, G, G, G, 2))
    inp[..., 0] = rng.standard_normal((B, G, G, G))
    mask = np.zeros((G, G, G))
    mask[1:G - 2, 1:G - 1, 1:G - 3] = 1.0
    inp[..., 1] = mask
    inp[..., 0] *= mask
    target = rng.standard_normal((B, G, G, G)) * mask
    return theta, inp, target


def _fd(theta, inp, target, d, eps):
    return (unet.loss(unet.forward(theta + eps * d, inp)[0], target, inp) -
            unet.loss(unet.forward(theta - eps * d, inp)[0], target, inp)) / (2 * eps)


def _agrees(theta, inp, target, d, exact, floor):
    """Central differences at three step sizes: a step that crosses a ReLU
    kink disagrees by chance at one size; a wrong gradient at all of them."""
    errs = []
    for eps in (1e-6, 3e-7, 1e-7):
        fd = _fd(theta, inp, target, d, eps)
        errs.append(abs(fd - exact) / max(abs(fd), floor))
    return min(errs) <= 1e-6, errs


def test_gradient_matches_finite_differences():
    theta, inp, target = _problem(4)
    L, g = unet.backward(theta, inp, target)
    out, _ = unet.forward(theta, inp)
    assert np.isclose(L, unet.loss(out, target, inp), rtol=1e-14)
    rng = np.random.default_rng(5)
    # directional derivatives, one direction per layer (weights and biases)
    o = 0
    for ci, co, _, _ in unet.LAYERS:
        n = co * 27 * ci + co
        d = np.zeros_like(theta)
        d[o:o + n] = rng.standard_normal(n)
        ok, errs = _agrees(theta, inp, target, d, g @ d, 1e-3)
        assert ok, (ci, co, errs)
        o += n
    # single coordinates: first weight, a middle one and the last bias
    for i in (0, unet.n_params() // 2, unet.n_params() - 1):
        d = np.zeros_like(theta)
        d[i] = 1.0
        ok, errs = _agrees(theta, inp, target, d, g[i], 1e-4)
        assert ok, (i, errs)


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(6)
    v = np.concatenate([rng.standard_normal(2000) * 10.0 ** rng.integers(-8, 8, 2000),
                        [0.0, -0.0, 1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 65504.0, 3.4e38, 1e-40]])
    ref = torch.tensor(v, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(unet.round_bf16(v), ref)
    assert np.isnan(unet.round_bf16(np.array([np.nan]))[0])


def test_first_adam_step_closed_form():
    rng = np.random.default_rng(7)
    theta = rng.standard_normal(50)
    g = rng.standard_normal(50)
    g += 0.5 * np.sign(g)  # |g| >= 0.5: eps = 1e-8 is negligible against sqrt(v)
    t1, m, v = unet.adam(theta, g, np.zeros(50), np.zeros(50), 1, lr=1e-2)
    # bias-corrected first moments are g and g^2: a step of lr * sign(g)
    np.testing.assert_allclose(theta - t1, 1e-2 * np.sign(g), rtol=1e-6)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_parameter_count():
    assert unet.n_params() == 181217
