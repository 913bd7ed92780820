"""GPU parity of the real-bogus scorer (sfft_rb_extract, sfft_rb_score)
through the C ABI against the FP64 CPU oracle (oracle/realbogus.py) with the
same bf16 rounding points.

Bound on the logits: the GPU sums in FP32 in another order than the oracle's
FP64 sums, so an activation whose exact value lies within ~1e-6 of a bf16
rounding boundary can round to the neighbouring bf16 value (one unit, 2^-8
relative) on one side only; a few such activations per copy move the logit
by far less than 1e-3 (measured below and printed). The unrounded FP64
network differs from the rounded one by ~1e-2, so the bound separates the
two. Stamp extraction is exact (FP64 arithmetic, one rounding to FP32)."""
import numpy as np
import pytest

import synth
from oracle import realbogus as RB

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _env():
    import torch
    import paper_2603_08593_amd as sf
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    sf.lib()
    return torch, sf


def _images(W, H, seed):
    p = synth.make_pair(W, H, 5, 1, 1, seed=seed, nstars=max(20, W * H // 800), dtype=np.float32)
    D = (p.S.astype(np.float64) - p.R.astype(np.float64) * float(p.a[0].sum())).astype(np.float32)
    return p, D


def test_extract_matches_oracle():
    torch, sf = _env()
    W, H = 200, 150
    p, D = _images(W, H, 8100)
    c = synth.rb_candidates((H, W), 40, seed=8101, margin=0)
    c[:3] = [[0, 0], [W - 1, H - 1], [5, 140]]           # windows that wrap
    # the call takes the offsets and scales as FP32: the oracle gets the same values
    off = tuple(float(np.float32(v)) for v in (1000.0, 990.0, 0.5))
    sc = tuple(float(np.float32(v)) for v in (0.01, 0.02, 0.05))
    want = RB.extract(p.S, p.R, D, c, off, sc).astype(np.float32)
    h = sf.Handle()
    try:
        t = [torch.from_numpy(a).cuda() for a in (p.S, p.R, D)]
        cd = torch.from_numpy(c).cuda()
        st = torch.zeros((len(c), 3, 32, 32), dtype=torch.float32, device="cuda")
        sf.sfft_rb_extract(h, sf.image_desc(t[0]), t[0], t[1], t[2], cd, off, sc, st)
        torch.cuda.synchronize()
        got = st.cpu().numpy()
    finally:
        h.close()
    assert np.array_equal(got, want)


@pytest.mark.parametrize("n,seed", [(7, 1), (64, 2)])
def test_score_matches_oracle(n, seed):
    torch, sf = _env()
    p, D = _images(256, 256, 8200 + seed)
    c = synth.rb_candidates((256, 256), n, seed=8300 + seed)
    stamps = RB.extract(p.S, p.R, D, c, (1000.0, 1000.0, 0.0), (0.01, 0.01, 0.05)).astype(np.float32)
    params = synth.rb_init(seed)
    _say(f"real-bogus score n={n} seed={seed}")
    check = min(n, 8)                          # the oracle is slow: the first 8 candidates
    ref, _ = RB.score(stamps[:check], params, rounded=True)
    unr, _ = RB.score(stamps[:check], params, rounded=False)
    h = sf.Handle()
    try:
        sd = torch.from_numpy(stamps).cuda()
        pd = torch.from_numpy(params).cuda()
        lg = torch.zeros(n, dtype=torch.float32, device="cuda")
        pr = torch.zeros(n, dtype=torch.float32, device="cuda")
        ws = torch.empty(sf.sfft_rb_workspace_size(n), dtype=torch.uint8, device="cuda")
        sf.sfft_rb_score(h, pd, sd, lg, pr, ws)
        torch.cuda.synchronize()
        got = lg.cpu().numpy().astype(np.float64)
        prob = pr.cpu().numpy().astype(np.float64)
    finally:
        h.close()
    err = np.abs(got[:check] - ref) / (1.0 + np.abs(ref))
    sep = np.abs(unr - ref) / (1.0 + np.abs(ref))
    _say(f"  max |logit - oracle| / (1 + |logit|): {err.max():.2e} (bf16 vs unrounded oracle: {sep.max():.2e})")
    assert np.all(err <= 1e-3)
    assert np.allclose(prob, 1.0 / (1.0 + np.exp(-got)), rtol=1e-6, atol=1e-7)


def test_score_rotation_invariant_on_gpu():
    # a quarter turn of every stamp permutes the four copies: the features are
    # the same, added in another order (FP32), so the logits agree to ~1e-6
    torch, sf = _env()
    n = 32
    p, D = _images(256, 256, 8400)
    c = synth.rb_candidates((256, 256), n, seed=8401)
    stamps = RB.extract(p.S, p.R, D, c, (1000.0, 1000.0, 0.0), (0.01, 0.01, 0.05)).astype(np.float32)
    params = torch.from_numpy(synth.rb_init(3)).cuda()
    h = sf.Handle()
    try:
        ws = torch.empty(sf.sfft_rb_workspace_size(n), dtype=torch.uint8, device="cuda")
        outs = []
        for k in range(4):
            sd = torch.from_numpy(np.ascontiguousarray(np.rot90(stamps, k=k, axes=(2, 3)))).cuda()
            lg = torch.zeros(n, dtype=torch.float32, device="cuda")
            sf.sfft_rb_score(h, params, sd, lg, None, ws)
            torch.cuda.synchronize()
            outs.append(lg.cpu().numpy().astype(np.float64))
    finally:
        h.close()
    for k in (1, 2, 3):
        d = np.max(np.abs(outs[k] - outs[0]) / (1.0 + np.abs(outs[0])))
        _say(f"  rotation {90 * k}: max rel logit change {d:.2e}")
        assert d <= 1e-5
