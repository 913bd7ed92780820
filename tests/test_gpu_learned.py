"""Learned form on the GPU.

* Training: the library's forward, backward and Adam kernels lower the loss
  of a fixed mini-batch of real samples (labels fitted by the plain GPU path
  on GPU-rendered CCD pairs) step after step.
* Gain: the committed network (trained with
  `python -m paper_2603_08593_amd.train_surrogate` on 8,000 synthetic pairs)
  run through the gated path on held-out pairs (seeds never used in
  training): every pair ends with a difference image that passes the chi2
  judge (prediction accepted, or the fallback fit), and the network scores a
  higher acceptance rate and a lower median chi2 than the trivial predictor
  (the training-mean coefficients, background refitted the same way).
"""
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

WEIGHTS = os.path.join(os.path.dirname(__file__), "..", "paper_2603_08593_amd", "weights",
                       "surrogate_L11_DK2_DB2.npz")


def test_training_steps_lower_the_batch_loss():
    import torch
    import paper_2603_08593_amd as sf
    from paper_2603_08593_amd import train_surrogate as TS
    from paper_2603_08593_amd.learned import Standardizer
    assert torch.cuda.is_available()
    diff = sf.Differencer(2048, 4096, 11, 2, 2, image_dtype="float32")
    X, P, T, C, kept = TS.build_dataset(np.arange(20000, 20016), diff, torch, log_every=8)
    assert len(kept) == 16 and np.all(C <= 1.05)
    std = Standardizer.fit(T)
    Tt = torch.from_numpy(std.forward(T).astype(np.float32)).cuda()
    net = sf.Surrogate(synth.surrogate_init(diff.N, 3), diff.N, n_stamps=64, max_pairs=16)
    losses = [float(net.train_step(X.contiguous(), P.contiguous(), Tt.contiguous(), 16, 1e-3)[0].item())
              for _ in range(60)]
    print("  batch loss:", " ".join(f"{v:.3f}" for v in losses[::5]), f"... {losses[-1]:.3f}", flush=True)
    assert all(np.isfinite(losses))
    assert losses[-1] < 0.5 * losses[0]
    assert np.mean(np.diff(losses) < 0) > 0.8


def test_trained_network_gain_over_trivial_predictor():
    import torch
    from paper_2603_08593_amd import train_surrogate as TS
    from paper_2603_08593_amd.learned import load_weights
    params, std, meta = load_weights(WEIGHTS)
    assert int(meta["pairs"]) == 10000
    res = TS.evaluate(params, std, np.arange(9000, 9040), torch)
    print(f"  held-out: {res}", flush=True)
    assert res["pairs"] >= 30
    assert res["max_chi2_final"] <= 1.05
    assert res["accept_net"] >= 0.6
    assert res["accept_net"] > res["accept_trivial"]
    assert res["median_chi2_net"] < res["median_chi2_trivial"]
