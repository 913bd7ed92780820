"""FP64 CPU oracle for the real-bogus scorer's inference.

TEST INFRASTRUCTURE ONLY. Only tests/, the smoke check in __graft_entry__.py
and the CPU-baseline leg of bench.py may import or run anything in oracle/.
The GPU library never calls it and shares no code with it.

Paper Sec. 2.3.4 scores every candidate of a difference image with a
rotation-invariant convolutional network with residual connections (after
ResNet-18): the input is a three-channel stamp (science, template,
difference) centred on the candidate, the output a probability that the
candidate is real. The trained weights and the layer sizes are not
published; this build scores throughput with seeded random weights, and the
network is this reading of the description:

* the stamp (3 x 32 x 32) is rotated by 0, 90, 180 and 270 degrees; each
  copy goes through the same trunk:
    stem    conv 3x3 3 -> 32, ReLU                                   32 x 32
    block 1 conv 3x3 32 -> 32, ReLU; conv 3x3 32 -> 32, + input, ReLU  32 x 32
    block 2 conv 3x3 s2 32 -> 64, ReLU; conv 3x3 64 -> 64
            + conv 1x1 s2 32 -> 64 of the block input, ReLU            16 x 16
    block 3 conv 3x3 s2 64 -> 128, ReLU; conv 3x3 128 -> 128
            + conv 1x1 s2 64 -> 128 of the block input, ReLU            8 x 8
    global average pool -> 128 features;
* the four feature vectors are averaged (cyclic pooling: a rotation of the
  input permutes the copies, so the mean, and the score, is invariant);
* linear 128 -> 64, ReLU, linear 64 -> 1 = logit; probability = sigmoid.
Convolutions: zero padding 1 (3x3), cross-correlation, output (i, j) reads
input (s i + ky - 1, s j + kx - 1).

Precision (the GPU form runs the convolutions on bf16 matrix cores): the
stamp values, the convolution weights and every trunk activation are
rounded to bfloat16 (round to nearest even) where the GPU stores them; sums
are exact here (FP64) and FP32 on the GPU; the pooling and the linear layers
are unrounded (FP32 on the GPU). Biases are not rounded.

Parameters: one flat FP32 vector, layers in the order above, each conv
weight [out][in][ky][kx] then its bias [out]; block 2 and 3 are (conv a,
conv b, projection) with the projection weight [out][in]; then fc1 weight
[64][128], bias [64], fc2 weight [1][64], bias [1].
"""
from __future__ import annotations

import numpy as np

from . import sfft_oracle as O

STAMP = 32
CONV_SHAPES = [  # (name, out, in, k)
    ("stem", 32, 3, 3),
    ("b1a", 32, 32, 3), ("b1b", 32, 32, 3),
    ("b2a", 64, 32, 3), ("b2b", 64, 64, 3), ("b2p", 64, 32, 1),
    ("b3a", 128, 64, 3), ("b3b", 128, 128, 3), ("b3p", 128, 64, 1),
]
FC_SHAPES = [("fc1", 64, 128), ("fc2", 1, 64)]


def param_layout():
    """name -> (offset of weight, weight shape, offset of bias, bias size)."""
    out, o = {}, 0
    for name, co, ci, k in CONV_SHAPES:
        shape = (co, ci, k, k) if k == 3 else (co, ci)
        n = int(np.prod(shape))
        out[name] = (o, shape, o + n, co)
        o += n + co
    for name, co, ci in FC_SHAPES:
        out[name] = (o, (co, ci), o + co * ci, co)
        o += co * ci + co
    out["_total"] = o
    return out


def num_params() -> int:
    return param_layout()["_total"]


def unpack(params):
    lay = param_layout()
    p = np.asarray(params, dtype=np.float64)
    out = {}
    for name, v in lay.items():
        if name == "_total":
            continue
        ow, shape, ob, nb = v
        out[name] = (p[ow:ow + int(np.prod(shape))].reshape(shape), p[ob:ob + nb])
    return out


def bf16(x):
    return O.bf16_rne(np.asarray(x, dtype=np.float64))


def conv(x, w, stride):
    """Cross-correlation, zero padding (k - 1) / 2: x (C, H, W), w (O, C, k, k)
    or (O, C) for k = 1; output (O, Ho, Wo), Ho = ceil(H / stride)."""
    if w.ndim == 2:
        return np.einsum("oc,chw->ohw", w, x[:, ::stride, ::stride])
    C, H, W = x.shape
    k = w.shape[-1]
    p = (k - 1) // 2
    xp = np.zeros((C, H + 2 * p, W + 2 * p))
    xp[:, p:p + H, p:p + W] = x
    Ho, Wo = -(-H // stride), -(-W // stride)
    out = np.zeros((w.shape[0], Ho, Wo))
    for ky in range(k):
        for kx in range(k):
            patch = xp[:, ky:ky + stride * (Ho - 1) + 1:stride, kx:kx + stride * (Wo - 1) + 1:stride]
            out += np.einsum("oc,chw->ohw", w[:, :, ky, kx], patch)
    return out


def relu(x):
    return np.maximum(x, 0.0)


def trunk(x, P, rounded=True):
    """Features (128,) of one rotated stamp copy x (3, 32, 32)."""
    q = bf16 if rounded else (lambda v: np.asarray(v, dtype=np.float64))

    def W(name):
        w, b = P[name]
        return q(w), b

    a0 = q(x)
    w, b = W("stem")
    a1 = q(relu(conv(a0, w, 1) + b[:, None, None]))
    w, b = W("b1a")
    t = q(relu(conv(a1, w, 1) + b[:, None, None]))
    w, b = W("b1b")
    a2 = q(relu(conv(t, w, 1) + b[:, None, None] + a1))
    w, b = W("b2a")
    t = q(relu(conv(a2, w, 2) + b[:, None, None]))
    w, b = W("b2b")
    wp, bp = W("b2p")
    a3 = q(relu(conv(t, w, 1) + b[:, None, None] + conv(a2, wp, 2) + bp[:, None, None]))
    w, b = W("b3a")
    t = q(relu(conv(a3, w, 2) + b[:, None, None]))
    w, b = W("b3b")
    wp, bp = W("b3p")
    a4 = q(relu(conv(t, w, 1) + b[:, None, None] + conv(a3, wp, 2) + bp[:, None, None]))
    return a4.mean(axis=(1, 2))


def score(stamps, params, rounded=True):
    """(logits, probabilities) of n stamps (n, 3, 32, 32)."""
    P = unpack(params)
    stamps = np.asarray(stamps, dtype=np.float64)
    logits = np.zeros(len(stamps))
    for n, s in enumerate(stamps):
        feats = [trunk(np.ascontiguousarray(np.rot90(s, k=rot, axes=(1, 2))), P, rounded) for rot in range(4)]
        f = np.mean(feats, axis=0)
        w1, b1 = P["fc1"]
        w2, b2 = P["fc2"]
        h = relu(w1 @ f + b1)
        logits[n] = float((w2 @ h + b2)[0])
    return logits, 1.0 / (1.0 + np.exp(-logits))


def extract(sci, ref, diff, centers, offsets, scales):
    """Stamps (n, 3, 32, 32): channel c of candidate k is
    (I_c[cy - 16 + i, cx - 16 + j] - offsets[c]) * scales[c] with
    I = (science, template, difference), indices periodic."""
    imgs = [np.asarray(a, dtype=np.float64) for a in (sci, ref, diff)]
    H, W = imgs[0].shape
    out = np.zeros((len(centers), 3, STAMP, STAMP))
    ii = np.arange(STAMP) - STAMP // 2
    for k, (cx, cy) in enumerate(np.asarray(centers)):
        ys = (int(cy) + ii) % H
        xs = (int(cx) + ii) % W
        for c in range(3):
            out[k, c] = (imgs[c][np.ix_(ys, xs)] - offsets[c]) * scales[c]
    return out
