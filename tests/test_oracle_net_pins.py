"""Pins of the surrogate-network oracle: convolution against a library
routine, gradients against finite differences, Adam against its closed-form
first step, bf16 rounding against its definition."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import net as N


def test_conv_matches_scipy_wrap_correlate():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((4, 7, 9))
    w = rng.standard_normal((3, 4, 3, 3))
    b = rng.standard_normal(3)
    z = N.conv3x3(x, w, b)
    for co in range(3):
        ref = b[co] + sum(ndimage.correlate(x[ci], w[co, ci], mode="wrap") for ci in range(4))
        assert np.max(np.abs(z[co] - ref)) < 1e-12


def _small_net(seed):
    rng = np.random.default_rng(seed)
    layers = [(5, 4), (4, 4), (4, 3)]
    params = [{"w": rng.standard_normal((co, ci, 3, 3)) * 0.3, "b": rng.standard_normal(co) * 0.1}
              for ci, co in layers]
    return params


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(1)
    f = rng.random((3, 5, 6))
    x = N.net_input(f, 1.2, 0.7)
    t = rng.random((3, 5, 6))
    params = _small_net(2)
    v, acts = N.forward(params, x, f)
    grads = N.backward(params, acts, v, t)
    h = 1e-6
    for li in range(len(params)):
        for key in ("w", "b"):
            flat = params[li][key].reshape(-1)
            gflat = grads[li][key].reshape(-1)
            for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
                old = flat[idx]
                flat[idx] = old + h
                lp = N.mse(N.forward(params, x, f)[0], t)
                flat[idx] = old - h
                lm = N.mse(N.forward(params, x, f)[0], t)
                flat[idx] = old
                fd = (lp - lm) / (2 * h)
                assert abs(fd - gflat[idx]) < 1e-6 * max(1.0, abs(fd)), (li, key, idx)


def test_input_gradient_adjoint_identity():
    """<conv(x), g> - <b, sum g> = <x, grad_input(g)> for any x, g."""
    rng = np.random.default_rng(3)
    x = rng.standard_normal((4, 6, 8))
    g = rng.standard_normal((5, 6, 8))
    w = rng.standard_normal((5, 4, 3, 3))
    b = np.zeros(5)
    assert abs(np.sum(N.conv3x3(x, w, b) * g) - np.sum(x * N.conv3x3_grad_input(g, w))) < 1e-10


def test_adam_first_step_closed_form():
    """After one step from zero moments, each parameter moves by
    -lr * g / (|g| + eps) (bias correction cancels the (1 - beta) factors)."""
    params = [{"w": np.array([0.5, -1.0, 2.0]), "b": np.array([0.0])}]
    grads = [{"w": np.array([0.3, -2.0, 1e-9]), "b": np.array([4.0])}]
    st = N.adam_init(params)
    before = {k: v.copy() for k, v in params[0].items()}
    N.adam_step(params, grads, st, lr=0.01)
    for k in ("w", "b"):
        exp = before[k] - 0.01 * grads[0][k] / (np.abs(grads[0][k]) + 1e-8)
        assert np.allclose(params[0][k], exp, rtol=1e-12, atol=1e-15)


def test_bf16_round():
    # bf16 keeps 8 significant bits: the spacing just above 1.0 is 2^-7
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7 + 2 ** -9, -3.14159, 0.0, 1.0 + 2 ** -8 + 2 ** -10,
                     1.0 + 3 * 2 ** -8], dtype=np.float32)
    r = N.bf16_round(vals)
    assert r[0] == 1.0
    assert r[1] == 1.0                    # tie -> even (1.0)
    assert r[2] == 1.0 + 2 ** -7          # below half a spacing -> down
    assert r[5] == 1.0 + 2 ** -7          # above half a spacing -> up
    assert r[6] == 1.0 + 2 ** -6          # tie -> even (mantissa ...10)
    assert abs(r[3] - (-3.140625)) < 1e-12
    assert r[4] == 0.0
    # every result has a zero low half-word
    assert np.all((r.astype(np.float32).view(np.uint32) & 0xFFFF) == 0)


@pytest.mark.parametrize("seed", [0, 1])
def test_full_network_shapes_and_residual(seed):
    params = N.init_params(seed)
    f = np.random.default_rng(seed).random((3, 8, 8))
    v, acts = N.forward(params, N.net_input(f, 1.0, 0.8), f)
    assert v.shape == f.shape and len(acts) == 7
    assert acts[1].shape == (32, 8, 8) and np.all(acts[1] >= 0)
