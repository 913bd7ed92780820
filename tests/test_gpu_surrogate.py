"""GPU parity of the learned form's hand-written kernels against the FP64
network oracle: stamp extraction, forward pass, every parameter gradient,
the Adam update, and the bfloat16 forward pass against the FP32 one.

Tolerances: the GPU runs in FP32 (the oracle in FP64); outputs and gradients
are compared by relative L2 error per parameter group, <= 1e-4 (sums of at
most ~6e4 FP32 products with relative rounding 6e-8 each; ReLU kinks that
flip between precisions are rare at these sizes). The bfloat16 forward pass
rounds every activation to 8 significant bits: its relative L2 deviation
from the FP32 pass must stay below 0.05 (a few 2^-8 per layer over 7
layers)."""
import numpy as np
import pytest

import oracle.surrogate as NN
import synth

pytestmark = pytest.mark.gpu

N_OUT = 732


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    return torch


def _sf():
    import paper_2603_08593_amd as sf
    sf.lib()
    return sf


def _rel(a, b):
    a, b = np.ravel(a).astype(np.float64), np.ravel(b).astype(np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _inputs(B, S, seed):
    rng = np.random.default_rng(seed)
    # stamp-like inputs: a positive blob per stamp plus noise, so that
    # pre-activations are not all near zero
    yy, xx = np.mgrid[0:32, 0:32] - 16.0
    blob = np.exp(-(xx ** 2 + yy ** 2) / 8.0)
    x = rng.standard_normal((B, S, 2, 32, 32)) * 0.3 + 3.0 * blob
    pos = rng.uniform(-1, 1, (B, S, 2))
    target = rng.standard_normal((B, N_OUT))
    return x.astype(np.float32), pos.astype(np.float32), target.astype(np.float32)


def test_num_params():
    assert _sf().sfft_surrogate_num_params(N_OUT) == NN.n_params(N_OUT) == 960812


def test_extract_stamps_matches_oracle():
    torch, sf = _torch(), _sf()
    p = synth.make_pair(256, 192, 5, 1, 1, seed=41, nstars=60, dtype=np.float32)
    c = np.array([[40, 50], [0, 0], [255, 191], [128, 100]], dtype=np.int32)
    want = NN.extract_stamps(p.R, p.S, c)
    h = sf.Handle()
    d = sf.make_desc(256, 192, 5, 1, 1)
    st = torch.empty((4, 2, 32, 32), dtype=torch.float32, device="cuda")
    pos = torch.empty((4, 2), dtype=torch.float32, device="cuda")
    sf.sfft_extract_stamps(h, d, torch.from_numpy(p.R).cuda(), torch.from_numpy(p.S).cuda(),
                           torch.from_numpy(c).cuda(), st, pos)
    torch.cuda.synchronize()
    got = st.cpu().numpy()
    err = _rel(got, want)
    print(f"  extract rel err {err:.2e}", flush=True)
    assert err <= 1e-6
    xt = 2 * c[:, 0] / 255 - 1
    yt = 2 * c[:, 1] / 191 - 1
    assert np.allclose(pos.cpu().numpy(), np.stack([xt, yt], 1), atol=1e-7)


def _gpu_state(B, S, seed):
    torch, sf = _torch(), _sf()
    flat = synth.surrogate_init(N_OUT, seed)
    net = sf.Surrogate(flat, N_OUT, n_stamps=S, max_pairs=B)
    x, pos, target = _inputs(B, S, seed + 1)
    X = torch.from_numpy(x).cuda()
    P = torch.from_numpy(pos).cuda()
    T = torch.from_numpy(target).cuda()
    return net, flat, x, pos, target, X, P, T


def test_forward_and_gradients_match_oracle():
    torch = _torch()
    B, S = 3, 8
    net, flat, x, pos, target, X, P, T = _gpu_state(B, S, 7)
    pred = net.forward(X, P, B)
    grads, loss = net.grad(X, P, T, B)
    torch.cuda.synchronize()
    params = NN.unflatten(flat, N_OUT)
    want_pred, cache = NN.forward(params, x, pos)
    want_loss, gpred = NN.mse_loss(want_pred, target)
    want = NN.backward(params, cache, gpred)
    ep = _rel(pred.cpu().numpy(), want_pred)
    el = abs(float(loss.item()) - want_loss) / want_loss
    print(f"  forward rel err {ep:.2e}, loss rel err {el:.2e}", flush=True)
    assert ep <= 1e-4 and el <= 1e-4
    g = NN.unflatten(grads.cpu().numpy(), N_OUT)
    for name, _ in NN.param_shapes(N_OUT):
        e = _rel(g[name], want[name])
        print(f"  grad {name:8s} rel err {e:.2e}", flush=True)
        assert e <= 1e-4, name


def test_adam_matches_oracle():
    torch = _torch()
    B, S = 2, 4
    net, flat, x, pos, target, X, P, T = _gpu_state(B, S, 11)
    net.grad(X, P, T, B)
    torch.cuda.synchronize()
    g = net.grads.cpu().numpy().astype(np.float64)
    p0 = net.params.cpu().numpy().astype(np.float64)
    net.adam(1e-3)
    torch.cuda.synchronize()
    want, m, v = NN.adam_step(p0, g, np.zeros_like(g), np.zeros_like(g), 1, lr=1e-3)
    got = net.params.cpu().numpy()
    assert np.max(np.abs(got - want)) <= 1e-6
    assert np.allclose(net.m.cpu().numpy(), m, rtol=1e-6, atol=1e-12)


def test_bf16_forward_close_to_fp32():
    torch, sf = _torch(), _sf()
    B, S = 4, 16
    net, flat, x, pos, target, X, P, T = _gpu_state(B, S, 3)
    p32 = net.forward(X, P, B, precision=sf.SFFT_NET_FP32).clone()
    p16 = net.forward(X, P, B, precision=sf.SFFT_NET_BF16)
    torch.cuda.synchronize()
    e = _rel(p16.cpu().numpy(), p32.cpu().numpy())
    print(f"  bf16 vs fp32 forward rel err {e:.2e}", flush=True)
    assert e <= 0.05


def test_gradients_deterministic():
    torch = _torch()
    B, S = 2, 8
    net, flat, x, pos, target, X, P, T = _gpu_state(B, S, 5)
    g1 = net.grad(X, P, T, B)[0].clone()
    g2 = net.grad(X, P, T, B)[0].clone()
    torch.cuda.synchronize()
    assert torch.equal(g1, g2)
