"""Train the learned form's network on synthetic CCD pairs and measure what
it gains over the plain path.

    python -m paper_2603_08593_amd.train_surrogate --pairs 10000 --out weights.npz

Data: seeded 2048 x 4096 pairs rendered on the GPU (synth.gpu: random PSF
FWHM 2.5-6 px with random spatial gradients, random planted kernels and
backgrounds); labels are the coefficients the plain GPU path fits
(L = 11, DK = 2, DB = 2, FP64 build and solve); inputs are the 64 brightest
isolated stars' 32 x 32 stamp pairs (library stamp extraction). Split
80/5/15 % into training, validation and held-out pairs. Training runs the
library's forward, backward and Adam kernels. The held-out evaluation runs
the gated path (bfloat16 prediction, chi2 judge at 1.05, full fit on
rejection) against the plain path and against a trivial predictor (the
training-mean coefficients), and prints one JSON line of results.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def _log(msg):
    print(msg, flush=True)


def build_dataset(indices, diff, torch, log_every=200):
    import synth
    import synth.gpu as sg
    from . import sfft_extract_stamps
    n = len(indices)
    dev = torch.device("cuda")
    stamps = torch.empty((n, 64, 2, 32, 32), dtype=torch.float32, device=dev)
    pos = torch.empty((n, 64, 2), dtype=torch.float32, device=dev)
    thetas = np.empty((n, diff.N))
    chi2 = np.empty(n)
    keep = np.zeros(n, bool)
    t0 = time.perf_counter()
    for j, k in enumerate(indices):
        pr = sg.make_learned_pair(int(k))
        c = synth.pick_centers(pr["xs"], pr["ys"], pr["flux"], 2048, 4096, 64, 32, 5)
        if len(c) < 64:
            continue
        diff.run(pr["R"], pr["S"], max_refine=1)
        ct = torch.from_numpy(c).to(dev)
        sfft_extract_stamps(diff.handle, diff.desc, pr["R"], pr["S"], ct, stamps[j], pos[j])
        thetas[j] = diff.buf.coef.cpu().numpy()
        chi2[j] = float(diff.buf.chi2.item())
        keep[j] = diff.info().status == 0
        if (j + 1) % log_every == 0:
            _log(f"  data {j + 1}/{n} pairs, {time.perf_counter() - t0:.1f} s")
    idx = np.nonzero(keep)[0]
    it = torch.from_numpy(idx).to(dev)
    return stamps.index_select(0, it), pos.index_select(0, it), thetas[idx], chi2[idx], np.asarray(indices)[idx]


def evaluate(net_params, std, test_indices, torch, threshold=1.05, log=_log, refit_background=True):
    """Gated vs plain vs trivial on held-out pairs; times exclude rendering."""
    import synth
    import synth.gpu as sg
    from .learned import GatedDifferencer
    g = GatedDifferencer(2048, 4096, 11, 2, 2, net_params, std, threshold=threshold,
                         refit_background=refit_background)
    d = g.diff
    trivial = torch.as_tensor(std.mean, dtype=torch.float64, device="cuda")
    acc_net = acc_triv = 0
    chi_net, chi_triv, chi_plain, chi_final = [], [], [], []
    t_gated = t_plain = 0.0
    n = 0
    for k in test_indices:
        pr = sg.make_learned_pair(int(k))
        c = synth.pick_centers(pr["xs"], pr["ys"], pr["flux"], 2048, 4096, 64, 32, 5)
        if len(c) < 64:
            continue
        ct = torch.from_numpy(c).cuda()
        R, S = pr["R"], pr["S"]
        torch.cuda.synchronize()
        t = time.perf_counter()
        d.run(R, S, max_refine=1)
        chi_plain.append(float(d.buf.chi2.item()))
        t_plain += time.perf_counter() - t
        t = time.perf_counter()
        ok, cp, cf = g.run(R, S, ct)
        torch.cuda.synchronize()
        t_gated += time.perf_counter() - t
        acc_net += ok
        chi_net.append(cp)
        chi_final.append(cf)
        trivial.copy_(torch.as_tensor(std.mean, dtype=torch.float64, device="cuda"))
        if refit_background:
            d.refit_background(R, S, coef=trivial)   # the same background refit as the gated path
        d.subtract(R, S, coef=trivial)
        ct2 = float(d.buf.chi2.item())
        chi_triv.append(ct2)
        acc_triv += ct2 <= threshold
        n += 1
        if n % 50 == 0:
            log(f"  eval {n} pairs: net accepted {acc_net}, trivial accepted {acc_triv}")
    return dict(pairs=n, accept_net=acc_net / max(n, 1), accept_trivial=acc_triv / max(n, 1),
                median_chi2_net=float(np.median(chi_net)), median_chi2_trivial=float(np.median(chi_triv)),
                median_chi2_plain=float(np.median(chi_plain)), max_chi2_final=float(np.max(chi_final)),
                pairs_per_s_gated=n / t_gated if t_gated else None,
                pairs_per_s_plain=n / t_plain if t_plain else None)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--pairs", type=int, default=10000)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--eval-pairs", type=int, default=200)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--out", default="surrogate.npz")
    ap.add_argument("--eval-only", default=None, help="evaluate saved weights instead of training")
    ap.add_argument("--eval-start", type=int, default=None, help="first held-out pair index")
    ap.add_argument("--no-refit", action="store_true", help="use the network's background coefficients")
    a = ap.parse_args(argv)
    import torch
    import synth
    from . import Differencer, Surrogate
    from .learned import Standardizer, load_weights, save_weights, train
    if a.eval_only:
        params, std, _ = load_weights(a.eval_only)
        start = a.eval_start if a.eval_start is not None else int(0.85 * a.pairs)
        res = evaluate(params, std, np.arange(start, start + a.eval_pairs), torch,
                       refit_background=not a.no_refit)
        res.update(weights=a.eval_only, refit_background=not a.no_refit)
        print(json.dumps(res), flush=True)
        return 0
    diff = Differencer(2048, 4096, 11, 2, 2, image_dtype="float32")
    n_tr, n_va = int(0.80 * a.pairs), int(0.05 * a.pairs)
    idx = np.arange(a.pairs)
    _log(f"building {n_tr + n_va} training/validation pairs")
    X, P, T, C, kept = build_dataset(idx[:n_tr + n_va], diff, torch)
    tr = kept < n_tr
    va = ~tr
    _log(f"kept {int(tr.sum())} training and {int(va.sum())} validation pairs; "
         f"median chi2 of the labels {np.median(C):.4f}")
    std = Standardizer.fit(T[tr])
    Tt = torch.from_numpy(std.forward(T).astype(np.float32)).cuda()
    itr = torch.from_numpy(np.nonzero(tr)[0]).cuda()
    iva = torch.from_numpy(np.nonzero(va)[0]).cuda()
    Xtr, Ptr, Ttr = X.index_select(0, itr), P.index_select(0, itr), Tt.index_select(0, itr)
    Xva, Pva, Tva = X.index_select(0, iva), P.index_select(0, iva), Tt.index_select(0, iva)
    del X, P
    net = Surrogate(synth.surrogate_init(diff.N, a.seed), diff.N, n_stamps=64, max_pairs=a.batch)

    def val_loss():
        tot, m = 0.0, 0
        for s in range(0, Xva.shape[0] - a.batch + 1, a.batch):
            pred = net.forward(Xva[s:s + a.batch].contiguous(), Pva[s:s + a.batch].contiguous(), a.batch)
            tot += float(((pred - Tva[s:s + a.batch]) ** 2).mean().item()) * a.batch
            m += a.batch
        return tot / max(m, 1)

    t0 = time.perf_counter()
    hist = []
    for ep in range(a.epochs):
        lr0 = a.lr * 0.5 * (1 + np.cos(np.pi * ep / a.epochs))
        lr1 = a.lr * max(0.5 * (1 + np.cos(np.pi * (ep + 1) / a.epochs)), 0.02)
        h = train(net, Xtr, Ptr, Ttr, epochs=1, batch=a.batch, lr=lr0, lr_final=lr1, seed=a.seed + ep)
        hist.append((h[0], val_loss()))
        _log(f"epoch {ep + 1}/{a.epochs}: train {hist[-1][0]:.4f} val {hist[-1][1]:.4f} "
             f"({time.perf_counter() - t0:.0f} s)")
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    params = net.params.cpu().numpy()
    save_weights(a.out, params, std, train_loss=[x[0] for x in hist], val_loss=[x[1] for x in hist],
                 pairs=a.pairs, epochs=a.epochs, batch=a.batch, lr=a.lr)
    _log(f"saved {a.out}; evaluating on {a.eval_pairs} held-out pairs")
    res = evaluate(params, std, idx[n_tr + n_va:n_tr + n_va + a.eval_pairs], torch,
                   refit_background=not a.no_refit)
    res.update(train_seconds=train_s, final_train_loss=hist[-1][0], final_val_loss=hist[-1][1])
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
