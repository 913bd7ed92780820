"""CPU pins of the real-bogus scorer oracle (oracle/realbogus.py): its
convolution against scipy's 2-D correlation, exact rotation invariance of the
score, the residual identity path, a hand-computed network through every
layer of the parameter layout, and the stamp extraction."""
import numpy as np
import pytest
import scipy.signal

from oracle import realbogus as RB


@pytest.mark.parametrize("stride,k", [(1, 3), (2, 3), (2, 1)])
def test_conv_matches_scipy_correlate(stride, k):
    rng = np.random.default_rng(stride * 10 + k)
    x = rng.normal(size=(3, 10, 12))
    w = rng.normal(size=(4, 3, k, k)) if k == 3 else rng.normal(size=(4, 3))
    got = RB.conv(x, w, stride)
    for o in range(4):
        ref = np.zeros((10, 12))
        for c in range(3):
            if k == 3:
                ref += scipy.signal.correlate2d(x[c], w[o, c], mode="same", boundary="fill")
            else:
                ref += w[o, c] * x[c]
        assert np.allclose(got[o], ref[::stride, ::stride], rtol=1e-12, atol=1e-12)


def _params(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    lay = RB.param_layout()
    p = np.zeros(lay["_total"])
    for name, (ow, shape, ob, nb) in [(k, v) for k, v in lay.items() if k != "_total"]:
        fan = int(np.prod(shape[1:]))
        p[ow:ow + int(np.prod(shape))] = rng.uniform(-1, 1, int(np.prod(shape))) * np.sqrt(6.0 / fan) * scale
        p[ob:ob + nb] = rng.uniform(-0.1, 0.1, nb)
    return p


@pytest.mark.parametrize("rounded,tol", [(False, 1e-12), (True, 1e-5)])
def test_score_is_rotation_invariant(rounded, tol):
    # exact in FP64 up to the order of the 4-copy mean; with the bf16
    # rounding points a last-bit difference of an FP64 sum (numpy's summation
    # order can depend on memory alignment) occasionally moves a value across
    # a rounding boundary, one bf16 unit, hence the looser bound
    rng = np.random.default_rng(3)
    s = rng.normal(size=(2, 3, 32, 32))
    p = _params(4)
    l0, _ = RB.score(s, p, rounded)
    for k in (1, 2, 3):
        lk, _ = RB.score(np.rot90(s, k=k, axes=(2, 3)), p, rounded)
        assert np.allclose(lk, l0, rtol=tol, atol=tol)


def test_residual_identity_path():
    # block 1 with zero weights and biases passes its input through (ReLU of
    # a non-negative input): the trunk equals the one with block 1 removed
    rng = np.random.default_rng(5)
    x = rng.normal(size=(3, 32, 32))
    p = _params(6)
    P = RB.unpack(p)
    P0 = dict(P)
    P0["b1a"] = (np.zeros_like(P["b1a"][0]), np.zeros_like(P["b1a"][1]))
    P0["b1b"] = (np.zeros_like(P["b1b"][0]), np.zeros_like(P["b1b"][1]))
    f0 = RB.trunk(x, P0, rounded=False)
    # the same trunk written out without block 1
    w, b = P["stem"]
    a1 = RB.relu(RB.conv(x, w, 1) + b[:, None, None])
    w, b = P["b2a"]
    t = RB.relu(RB.conv(a1, w, 2) + b[:, None, None])
    w, b = P["b2b"]
    wp, bp = P["b2p"]
    a3 = RB.relu(RB.conv(t, w, 1) + b[:, None, None] + RB.conv(a1, wp, 2) + bp[:, None, None])
    w, b = P["b3a"]
    t = RB.relu(RB.conv(a3, w, 2) + b[:, None, None])
    w, b = P["b3b"]
    wp, bp = P["b3p"]
    a4 = RB.relu(RB.conv(t, w, 1) + b[:, None, None] + RB.conv(a3, wp, 2) + bp[:, None, None])
    assert np.allclose(f0, a4.mean(axis=(1, 2)), rtol=1e-13)


def test_hand_computed_network():
    # every weight zero; biases chosen so that each layer's output is a known
    # constant: stem 1, b1a 0.5, b1b -> relu(0.25 + 1) = 1.25, b2a 2, b2b +
    # projection biases -> 3 + 0.5, b3a 1, b3b + projection -> 4 - 1 = 3;
    # features 3 for all 128 channels; fc1 row i has weight (i + 1) / 128 on
    # channel 0 only, bias -1 -> h_i = 3 (i + 1) / 128 - 1 (ReLU keeps
    # i >= 43); fc2 weight 1 on h_63, bias 0.5 -> logit 3 * 64 / 128 - 1 + 0.5
    lay = RB.param_layout()
    p = np.zeros(lay["_total"])

    def bias(name, v):
        ow, shape, ob, nb = lay[name]
        p[ob:ob + nb] = v
    bias("stem", 1.0)
    bias("b1a", 0.5)
    bias("b1b", 0.25)
    bias("b2a", 2.0)
    bias("b2b", 3.0)
    bias("b2p", 0.5)
    bias("b3a", 1.0)
    bias("b3b", 4.0)
    bias("b3p", -1.0)
    ow, shape, ob, nb = lay["fc1"]
    w1 = np.zeros(shape)
    w1[:, 0] = (np.arange(64) + 1) / 128.0
    p[ow:ow + w1.size] = w1.ravel()
    p[ob:ob + nb] = -1.0
    ow, shape, ob, nb = lay["fc2"]
    w2 = np.zeros(shape)
    w2[0, 63] = 1.0
    p[ow:ow + w2.size] = w2.ravel()
    p[ob] = 0.5
    x = np.random.default_rng(7).normal(size=(1, 3, 32, 32))
    for rounded in (True, False):
        logit, prob = RB.score(x, p, rounded)
        assert logit[0] == pytest.approx(3.0 * 64 / 128 - 1.0 + 0.5, abs=1e-12)
        assert prob[0] == pytest.approx(1.0 / (1.0 + np.exp(-1.0)), abs=1e-12)
    assert RB.num_params() == lay["_total"] == 315009


def test_extract_periodic_and_scaled():
    H, W = 20, 24
    sci = np.arange(H * W, dtype=np.float64).reshape(H, W)
    ref = -sci
    diff = sci * 0.5
    st = RB.extract(sci, ref, diff, np.array([[2, 3]]), (1.0, 2.0, 3.0), (0.5, 0.25, 2.0))
    # element (i, j) of channel 0 is the science pixel (3 - 16 + i, 2 - 16 + j) mod size
    for i, j in [(0, 0), (16, 16), (31, 5), (7, 31)]:
        y, x = (3 - 16 + i) % H, (2 - 16 + j) % W
        assert st[0, 0, i, j] == (sci[y, x] - 1.0) * 0.5
        assert st[0, 1, i, j] == (ref[y, x] - 2.0) * 0.25
        assert st[0, 2, i, j] == (diff[y, x] - 3.0) * 2.0
