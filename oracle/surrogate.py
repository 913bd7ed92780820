"""FP64 CPU oracle of the learned form: a small convolutional network that
predicts the kernel and background coefficients of the SFFT fit from
star-stamp pairs, its backward pass, the training loss and the Adam update.

TEST INFRASTRUCTURE ONLY: only tests/, the smoke check and the CPU baseline
may use it; the GPU library shares no code with it.

The network (the paper's transient pipeline runs a learned model beside the
image differencing, Sec. 2.3; its architecture here is this project's own):
  per stamp s (2 channels: reference, science; 32 x 32):
    conv 3x3 2->16 (stride 1) ReLU, 16->32 (stride 2) ReLU,
    32->64 (stride 2) ReLU, 64->64 (stride 2) ReLU -> 64 x 4 x 4,
    linear 1024 -> 128 ReLU = h_s
  position-weighted pooling over the S stamps of a pair:
    pooled[i, c] = (1/S) sum_s p_i(xt_s, yt_s) h_s[c], p_i the DK = 2
    monomials (1, xt, yt, xt^2, xt yt, yt^2) of the stamp centre
  linear 768 -> 512 ReLU, linear 512 -> n_out (standardised coefficients).
Convolutions are cross-correlations with zero padding 1:
  out[co, oy, ox] = b[co] + sum_{ci, ky, kx} w[co, ci, ky, kx] in[ci, s oy + ky - 1, s ox + kx - 1].
Loss: mean over pairs and outputs of (pred - target)^2.
Adam (Kingma and Ba 2015): m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
  p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
"""
from __future__ import annotations

import numpy as np

STAMP = 32
N_MONO = 6
CONVS = [(2, 16, 1), (16, 32, 2), (32, 64, 2), (64, 64, 2)]   # (cin, cout, stride)
FC1 = (1024, 128)
FC2 = (N_MONO * 128, 512)


def param_shapes(n_out: int):
    """(name, shape) in the order of the flat parameter vector."""
    out = []
    for k, (ci, co, _) in enumerate(CONVS):
        out += [(f"conv{k + 1}.w", (co, ci, 3, 3)), (f"conv{k + 1}.b", (co,))]
    out += [("fc1.w", (FC1[1], FC1[0])), ("fc1.b", (FC1[1],)),
            ("fc2.w", (FC2[1], FC2[0])), ("fc2.b", (FC2[1],)),
            ("fc3.w", (n_out, FC2[1])), ("fc3.b", (n_out,))]
    return out


def n_params(n_out: int) -> int:
    return int(sum(np.prod(s) for _, s in param_shapes(n_out)))


def unflatten(flat, n_out: int) -> dict:
    p, o = {}, 0
    for name, shape in param_shapes(n_out):
        n = int(np.prod(shape))
        p[name] = np.asarray(flat[o:o + n], dtype=np.float64).reshape(shape)
        o += n
    return p


def flatten(d: dict, n_out: int) -> np.ndarray:
    return np.concatenate([np.ravel(d[name]) for name, _ in param_shapes(n_out)])


def monomials2(xt, yt):
    """The six DK = 2 monomials in the fit's order: 1, xt, yt, xt^2, xt yt, yt^2."""
    xt, yt = np.asarray(xt, np.float64), np.asarray(yt, np.float64)
    return np.stack([np.ones_like(xt), xt, yt, xt * xt, xt * yt, yt * yt], axis=-1)


def _patches(x, stride):
    """x: (n, c, h, w) -> (n, c, 3, 3, ho, wo) zero-padded input windows."""
    n, c, h, w = x.shape
    xp = np.zeros((n, c, h + 2, w + 2))
    xp[:, :, 1:-1, 1:-1] = x
    ho, wo = (h - 1) // stride + 1, (w - 1) // stride + 1
    out = np.empty((n, c, 3, 3, ho, wo))
    for ky in range(3):
        for kx in range(3):
            out[:, :, ky, kx] = xp[:, :, ky:ky + stride * (ho - 1) + 1:stride,
                                   kx:kx + stride * (wo - 1) + 1:stride]
    return out


def conv_forward(x, w, b, stride):
    P = _patches(x, stride)
    return np.einsum("ncijhw,ocij->nohw", P, w, optimize=True) + b[None, :, None, None]


def conv_backward(x, w, stride, gy):
    """Gradients of conv_forward with respect to x, w and b."""
    P = _patches(x, stride)
    gw = np.einsum("nohw,ncijhw->ocij", gy, P, optimize=True)
    gb = gy.sum(axis=(0, 2, 3))
    gP = np.einsum("nohw,ocij->ncijhw", gy, w, optimize=True)
    n, c, h, ww = x.shape
    gxp = np.zeros((n, c, h + 2, ww + 2))
    ho, wo = gy.shape[2], gy.shape[3]
    for ky in range(3):
        for kx in range(3):
            gxp[:, :, ky:ky + stride * (ho - 1) + 1:stride, kx:kx + stride * (wo - 1) + 1:stride] += gP[:, :, ky, kx]
    return gxp[:, :, 1:-1, 1:-1], gw, gb


def forward(params: dict, stamps, pos):
    """stamps: (B, S, 2, 32, 32); pos: (B, S, 2) = (xt, yt). Returns (pred, cache)."""
    stamps = np.asarray(stamps, np.float64)
    B, S = stamps.shape[:2]
    x = stamps.reshape(B * S, 2, STAMP, STAMP)
    cache = {"x0": x}
    for k, (_, _, st) in enumerate(CONVS):
        z = conv_forward(x, params[f"conv{k + 1}.w"], params[f"conv{k + 1}.b"], st)
        x = np.maximum(z, 0.0)
        cache[f"a{k + 1}"] = x
    f = x.reshape(B * S, -1)
    h = np.maximum(f @ params["fc1.w"].T + params["fc1.b"], 0.0)
    mono = monomials2(pos[..., 0], pos[..., 1])                      # (B, S, 6)
    hs = h.reshape(B, S, -1)
    pooled = np.einsum("bsi,bsc->bic", mono, hs) / S                 # (B, 6, 128)
    u = pooled.reshape(B, -1)
    g = np.maximum(u @ params["fc2.w"].T + params["fc2.b"], 0.0)
    pred = g @ params["fc3.w"].T + params["fc3.b"]
    cache.update(f=f, h=h, mono=mono, u=u, g=g, B=B, S=S)
    return pred, cache


def backward(params: dict, cache: dict, gpred):
    """Gradients of every parameter (and of the input stamps, key "input")
    for d(loss)/d(pred) = gpred."""
    grads = {}
    B, S = cache["B"], cache["S"]
    g, u, h, f = cache["g"], cache["u"], cache["h"], cache["f"]
    grads["fc3.w"] = gpred.T @ g
    grads["fc3.b"] = gpred.sum(0)
    gg = (gpred @ params["fc3.w"]) * (g > 0)
    grads["fc2.w"] = gg.T @ u
    grads["fc2.b"] = gg.sum(0)
    gu = gg @ params["fc2.w"]
    gpooled = gu.reshape(B, N_MONO, -1)
    gh = (np.einsum("bsi,bic->bsc", cache["mono"], gpooled) / S).reshape(B * S, -1) * (h > 0)
    grads["fc1.w"] = gh.T @ f
    grads["fc1.b"] = gh.sum(0)
    gx = (gh @ params["fc1.w"]).reshape(cache["a4"].shape)
    for k in range(len(CONVS), 0, -1):
        a = cache[f"a{k}"]
        gz = gx * (a > 0)
        xin = cache[f"a{k - 1}"] if k > 1 else cache["x0"]
        gx, gw, gb = conv_backward(xin, params[f"conv{k}.w"], CONVS[k - 1][2], gz)
        grads[f"conv{k}.w"] = gw
        grads[f"conv{k}.b"] = gb
    grads["input"] = gx.reshape(B, S, 2, STAMP, STAMP)
    return grads


def mse_loss(pred, target):
    """Mean squared error over every output of every pair, and its gradient."""
    d = np.asarray(pred, np.float64) - np.asarray(target, np.float64)
    return float(np.mean(d * d)), 2.0 * d / d.size


def adam_step(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (t counts from 1). Returns new (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def extract_stamps(R, S, centers, size=STAMP, scale=100.0):
    """Normalised stamp pairs of the learned form: the size x size windows
    starting at (cx - size/2, cy - size/2) (periodic), each channel minus the
    mean of its window's border pixels, both divided by the reference
    window's sky-subtracted sum (1 when that sum is not positive) and
    multiplied by `scale`. Returns (S, 2, size, size)."""
    R = np.asarray(R, np.float64)
    Sc = np.asarray(S, np.float64)
    H, W = R.shape
    out = np.empty((len(centers), 2, size, size))
    off = np.arange(size) - size // 2
    border = np.ones((size, size), bool)
    border[1:-1, 1:-1] = False
    for k, (cx, cy) in enumerate(np.asarray(centers).reshape(-1, 2)):
        ys = (cy + off) % H
        xs = (cx + off) % W
        r = R[np.ix_(ys, xs)]
        s = Sc[np.ix_(ys, xs)]
        r = r - r[border].mean()
        s = s - s[border].mean()
        f = r.sum()
        f = f if f > 0 else 1.0
        out[k, 0] = scale * r / f
        out[k, 1] = scale * s / f
    return out
