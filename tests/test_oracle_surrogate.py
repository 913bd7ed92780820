"""Pins of the learned-form oracle: convolutions against scipy's
correlate2d, the backward pass against central finite differences of the
forward pass, pooling in closed form, Adam against hand-computed steps, and
stamp extraction on a constructed image."""
import numpy as np
import pytest
import scipy.signal

import oracle.surrogate as NN
import synth


def test_conv_forward_matches_correlate2d():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 3, 9, 9))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    for stride in (1, 2):
        y = NN.conv_forward(x, w, b, stride)
        for n in range(2):
            for co in range(4):
                ref = sum(scipy.signal.correlate2d(x[n, ci], w[co, ci], mode="same", boundary="fill")
                          for ci in range(3)) + b[co]
                assert np.allclose(y[n, co], ref[::stride, ::stride], rtol=0, atol=1e-12)


def _tiny_params(n_out, seed):
    rng = np.random.default_rng(seed)
    flat = synth.surrogate_init(n_out, seed)
    return NN.unflatten(flat, n_out), rng


def test_param_count():
    assert NN.n_params(732) == 960812


@pytest.mark.parametrize("name", ["conv1.w", "conv2.w", "conv3.b", "conv4.w", "fc1.w", "fc2.b", "fc3.w"])
def test_backward_matches_finite_differences(name):
    n_out = 7
    params, rng = _tiny_params(n_out, 3)
    B, S = 2, 3
    stamps = rng.standard_normal((B, S, 2, 32, 32))
    pos = rng.uniform(-1, 1, (B, S, 2))
    target = rng.standard_normal((B, n_out))
    pred, cache = NN.forward(params, stamps, pos)
    _, gpred = NN.mse_loss(pred, target)
    grads = NN.backward(params, cache, gpred)
    flat_idx = rng.choice(params[name].size, size=min(6, params[name].size), replace=False)
    h = 1e-6
    for k in flat_idx:
        p1 = {kk: vv.copy() for kk, vv in params.items()}
        p2 = {kk: vv.copy() for kk, vv in params.items()}
        p1[name].flat[k] += h
        p2[name].flat[k] -= h
        l1, _ = NN.mse_loss(NN.forward(p1, stamps, pos)[0], target)
        l2, _ = NN.mse_loss(NN.forward(p2, stamps, pos)[0], target)
        fd = (l1 - l2) / (2 * h)
        an = grads[name].flat[k]
        assert abs(fd - an) <= 1e-6 * max(abs(fd), abs(an)) + 1e-10, (name, k, fd, an)


def test_input_gradient_matches_finite_differences():
    n_out = 5
    params, rng = _tiny_params(n_out, 9)
    stamps = rng.standard_normal((1, 2, 2, 32, 32))
    pos = rng.uniform(-1, 1, (1, 2, 2))
    target = rng.standard_normal((1, n_out))
    pred, cache = NN.forward(params, stamps, pos)
    _, gpred = NN.mse_loss(pred, target)
    gin = NN.backward(params, cache, gpred)["input"]
    h = 1e-6
    for idx in [(0, 1, 1, 10, 17), (0, 0, 0, 0, 0), (0, 1, 0, 31, 5)]:
        s1, s2 = stamps.copy(), stamps.copy()
        s1[idx] += h
        s2[idx] -= h
        fd = (NN.mse_loss(NN.forward(params, s1, pos)[0], target)[0]
              - NN.mse_loss(NN.forward(params, s2, pos)[0], target)[0]) / (2 * h)
        assert abs(fd - gin[idx]) <= 1e-6 * max(abs(fd), abs(gin[idx])) + 1e-10


def test_pooling_closed_form():
    """Identical per-stamp features h pool to h times the mean monomial."""
    n_out = 4
    params, rng = _tiny_params(n_out, 1)
    stamp = rng.standard_normal((2, 32, 32))
    stamps = np.broadcast_to(stamp, (1, 5, 2, 32, 32)).copy()
    pos = rng.uniform(-1, 1, (1, 5, 2))
    _, cache = NN.forward(params, stamps, pos)
    h = cache["h"][0]
    mono = NN.monomials2(pos[0, :, 0], pos[0, :, 1]).mean(axis=0)
    assert np.allclose(cache["u"][0].reshape(6, -1), mono[:, None] * h[None, :], atol=1e-13)


def test_adam_two_steps_by_hand():
    p, g1, g2 = np.array([1.0, -2.0]), np.array([0.5, -1.0]), np.array([0.1, 0.2])
    m = v = np.zeros(2)
    p1, m, v = NN.adam_step(p, g1, m, v, 1, lr=0.01)
    # first step: m_hat = g, v_hat = g^2 -> p -= lr * sign(g) (up to eps)
    assert np.allclose(p1, p - 0.01 * np.sign(g1), atol=1e-7)
    p2, m, v = NN.adam_step(p1, g2, m, v, 2, lr=0.01)
    m2 = 0.9 * 0.1 * g1 + 0.1 * g2
    v2 = 0.999 * 0.001 * g1 ** 2 + 0.001 * g2 ** 2
    want = p1 - 0.01 * (m2 / (1 - 0.81)) / (np.sqrt(v2 / (1 - 0.999 ** 2)) + 1e-8)
    assert np.allclose(p2, want, rtol=1e-14, atol=0)


def test_extract_stamps_constructed():
    W, H = 64, 48
    R = np.full((H, W), 10.0)
    S = np.full((H, W), 20.0)
    R[20, 30] += 50.0            # a single bright pixel at the stamp centre
    S[20, 30] += 25.0
    out = NN.extract_stamps(R, S, [(30, 20)], size=8, scale=1.0)
    # window rows 16..23, cols 26..33; the centre pixel sits at (4, 4)
    assert out.shape == (1, 2, 8, 8)
    assert abs(out[0, 0, 4, 4] - 1.0) < 1e-15 and abs(out[0, 0].sum() - 1.0) < 1e-13
    assert abs(out[0, 1, 4, 4] - 0.5) < 1e-15
    assert np.count_nonzero(out[0, 0]) == 1


def test_mse_loss_hand_values():
    """Mean over every output of every pair: pred - target = [[1, -2, 0],
    [3, 0, 2]] gives (1 + 4 + 0 + 9 + 0 + 4) / 6 = 3, gradient 2 d / 6."""
    pred = np.array([[1.0, 0.0, 5.0], [4.0, 1.0, 2.0]])
    target = np.array([[0.0, 2.0, 5.0], [1.0, 1.0, 0.0]])
    loss, g = NN.mse_loss(pred, target)
    assert loss == 3.0
    assert np.array_equal(g, np.array([[2.0, -4.0, 0.0], [6.0, 0.0, 4.0]]) / 6.0)
