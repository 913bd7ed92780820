"""CPU pins of the fit-mode oracle (oracle/modes.py): the output-pixel kernel
convention and the masked fit, against definitions that share none of its
code paths: a pure-Python per-pixel model loop, exact recovery of a planted
output-pixel kernel, the input-pixel oracle on masked images, and the
convention-independent DK = 0 case."""
import numpy as np
import pytest

import oracle as O
from oracle import modes as M


def _py_model_outpix(Rm, a, b, L, DK, DB):
    """Per-pixel loop: M(x) = sum_i p_i(x) sum_delta a R(x - delta) + bg."""
    H, W = Rm.shape
    r = (L - 1) // 2
    xt = [2.0 * x / (W - 1) - 1.0 for x in range(W)]
    yt = [2.0 * y / (H - 1) - 1.0 for y in range(H)]
    mk = [(d - e, e) for d in range(DK + 1) for e in range(d + 1)]
    mb = [(d - e, e) for d in range(DB + 1) for e in range(d + 1)]
    out = np.zeros((H, W))
    for y in range(H):
        for x in range(W):
            s = 0.0
            for i, (ea, eb) in enumerate(mk):
                p = xt[x] ** ea * yt[y] ** eb
                for dy in range(-r, r + 1):
                    for dx in range(-r, r + 1):
                        s += a[i][dy + r][dx + r] * p * Rm[(y - dy) % H][(x - dx) % W]
            for c, (ea, eb) in enumerate(mb):
                s += b[c] * xt[x] ** ea * yt[y] ** eb
            out[y, x] = s
    return out


def _texture(W, H, seed):
    rng = np.random.default_rng(seed)
    return 1000.0 + rng.normal(0, 30, size=(H, W)) + 200 * np.exp(
        -((np.arange(W)[None, :] - W / 3) ** 2 + (np.arange(H)[:, None] - H / 2) ** 2) / 8.0)


def test_outpix_model_matches_pixel_loop():
    W, H, L, DK, DB = 13, 11, 3, 2, 1
    R = _texture(W, H, 1)
    rng = np.random.default_rng(2)
    theta = rng.normal(size=O.n_unknowns(L, DK, DB))
    a, b = O.split_theta(theta, L, DK, DB)
    want = _py_model_outpix(R - 3.0, a, b, L, DK, DB)
    got = M.model_image_outpix(R, theta, L, DK, DB, ref_pedestal=3.0)
    assert np.allclose(got, want, rtol=1e-12, atol=1e-9)
    # the design matrix of the output-pixel problem reproduces the model on
    # the frame-masked reference
    Rm = (R - 3.0) * M.frame_mask(W, H, 1)
    A = M.design_matrix_ex(R, L, DK, DB, ref_pedestal=3.0, outpix=True)
    assert np.allclose(A @ theta, _py_model_outpix(Rm, a, b, L, DK, DB).ravel(), rtol=1e-12, atol=1e-9)


@pytest.mark.parametrize("W,H,L,DK,DB", [(16, 14, 3, 2, 2), (20, 18, 5, 1, 1), (24, 20, 3, 2, 0)])
def test_outpix_exact_recovery(W, H, L, DK, DB):
    # noise-free science planted from the frame-masked reference with a known
    # output-pixel kernel and background: the fit returns them exactly
    R = _texture(W, H, W)
    Rm = R * M.frame_mask(W, H, (L - 1) // 2)
    rng = np.random.default_rng(H)
    a = rng.normal(0, 0.1, size=(O.n_mono(DK), L, L))
    b = rng.normal(0, 5.0, size=O.n_mono(DB))
    S = _py_model_outpix(Rm, a, b, L, DK, DB)
    theta = M.solve_ex(R, S, L, DK, DB, outpix=True)
    want = np.concatenate([a.ravel(), b])
    assert np.linalg.norm(theta - want) / np.linalg.norm(want) <= 1e-9


def test_outpix_dk0_is_the_input_pixel_fit_on_the_frame_masked_reference():
    W, H, L = 18, 16, 5
    R = _texture(W, H, 5)
    S = np.roll(R, (1, -1), axis=(0, 1)) * 0.8 + 40.0 + np.random.default_rng(6).normal(0, 3, size=R.shape)
    t_out = M.solve_ex(R, S, L, 0, 1, outpix=True)
    Rm = R * M.frame_mask(W, H, 2)
    t_in = O.solve_bruteforce(Rm, S, L, 0, 1)
    assert np.allclose(t_out, t_in, rtol=1e-9, atol=1e-9)


def test_masked_fit_is_the_plain_fit_on_masked_images():
    W, H, L, DK, DB = 20, 16, 3, 1, 1
    R = _texture(W, H, 7)
    S = 0.9 * np.roll(R, (0, 1), axis=(0, 1)) + np.random.default_rng(8).normal(0, 2, size=R.shape)
    mask = np.zeros((H, W), dtype=np.uint8)
    mask[3:10, 4:15] = 1
    mask[12:15, 2:6] = 1
    c_r, c_s = 1000.0, 900.0
    G, h = M.normal_ex(R, S, L, DK, DB, c_r, c_s, mask=mask)
    Rm = (R - c_r) * mask
    Sm = (S - c_s) * mask
    G0, h0 = O.normal_bruteforce(Rm, Sm, L, DK, DB)
    assert np.allclose(G, G0, rtol=1e-13, atol=1e-9)
    assert np.allclose(h, h0, rtol=1e-13, atol=1e-9)
    # an all-ones mask is the plain problem
    G1, h1 = M.normal_ex(R, S, L, DK, DB, c_r, c_s, mask=np.ones((H, W)))
    G2, h2 = O.normal_bruteforce(R, S, L, DK, DB, c_r, c_s)
    assert np.allclose(G1, G2, rtol=1e-13) and np.allclose(h1, h2, rtol=1e-13)


def test_subtract_ex_conventions():
    W, H, L, DK, DB = 15, 12, 3, 1, 1
    R = _texture(W, H, 9)
    S = _texture(W, H, 10)
    rng = np.random.default_rng(11)
    theta = rng.normal(size=O.n_unknowns(L, DK, DB))
    a, b = O.split_theta(theta, L, DK, DB)
    D = M.subtract_ex(R, S, theta, L, DK, DB, 5.0, 7.0, outpix=True)
    assert np.allclose(D, (S - 7.0) - _py_model_outpix(R - 5.0, a, b, L, DK, DB), rtol=1e-12, atol=1e-8)
    D0 = M.subtract_ex(R, S, theta, L, DK, DB, 5.0, 7.0, outpix=False)
    assert np.allclose(D0, O.subtract64(R, S, theta, L, DK, DB, 5.0, 7.0))
