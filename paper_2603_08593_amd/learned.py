"""Learned form: training of the coefficient network with the library's own
forward, backward and Adam kernels, and gated inference with the chi2 judge.

A pair is differenced with the predicted kernel first (its background
re-fitted exactly for that kernel, a 6-unknown least-squares problem from
image moments); when the difference image's reduced chi2 exceeds the
threshold (1.05), the full build + solve runs and the pair is differenced
again with its own fit.
Every step runs in the HIP library (argument marshalling only here).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import (SFFT_NET_BF16, Differencer, Surrogate, sfft_extract_stamps, sfft_subtract,
               sfft_surrogate_destandardize)

N_STAMPS = 64
STAMP = 32


@dataclass
class Standardizer:
    """Per-coefficient affine map between coefficients and network outputs:
    coef = mean + scale * pred."""
    mean: np.ndarray
    scale: np.ndarray

    @staticmethod
    def fit(thetas: np.ndarray) -> "Standardizer":
        t = np.asarray(thetas, dtype=np.float64)
        mean = t.mean(axis=0)
        scale = t.std(axis=0)
        scale = np.where(scale > 1e-12 * max(float(np.abs(t).max()), 1e-300), scale, 1.0)
        return Standardizer(mean, scale)

    def forward(self, thetas):
        return (np.asarray(thetas, np.float64) - self.mean) / self.scale


def save_weights(path, params, std: Standardizer, **meta):
    np.savez(path, params=np.asarray(params, np.float32), mean=std.mean, scale=std.scale,
             **{k: np.asarray(v) for k, v in meta.items()})


def load_weights(path):
    z = np.load(path, allow_pickle=False)
    meta = {k: z[k] for k in z.files if k not in ("params", "mean", "scale")}
    return z["params"], Standardizer(z["mean"], z["scale"]), meta


def save_checkpoint(path, net: Surrogate, std: Standardizer | None = None, **meta):
    """Training state for resuming: parameters, both Adam moment vectors and
    the step count (copied from the device after a synchronisation)."""
    net.torch.cuda.synchronize()
    extra = {} if std is None else dict(mean=std.mean, scale=std.scale)
    np.savez(path, params=net.params.cpu().numpy(), adam_m=net.m.cpu().numpy(), adam_v=net.v.cpu().numpy(),
             step=np.int64(net.step), **extra, **{k: np.asarray(v) for k, v in meta.items()})


def load_checkpoint(path, net: Surrogate):
    """Restores the state written by save_checkpoint into `net` (same n_out);
    returns the Standardizer when the checkpoint holds one."""
    z = np.load(path, allow_pickle=False)
    t = net.torch
    for name in ("params", "adam_m", "adam_v"):
        if z[name].shape != (net.params.numel(),):
            raise ValueError(f"checkpoint {name} has {z[name].shape}, network needs {net.params.numel()}")
    net.params.copy_(t.from_numpy(z["params"]).to(net.params.device))
    net.m.copy_(t.from_numpy(z["adam_m"]).to(net.m.device))
    net.v.copy_(t.from_numpy(z["adam_v"]).to(net.v.device))
    net.step = int(z["step"])
    return Standardizer(z["mean"], z["scale"]) if "mean" in z.files else None


def train(net: Surrogate, stamps, pos, targets, *, epochs: int, batch: int, lr: float, seed: int = 0,
          lr_final: float | None = None, log=None):
    """Adam on mini-batches of pairs. stamps (N, S, 2, 32, 32), pos (N, S, 2),
    targets (N, n_out) standardised: FP32 device tensors. Cosine learning-rate
    decay to lr_final. Returns the mean loss of every epoch."""
    import torch
    N = stamps.shape[0]
    rng = np.random.default_rng(seed)
    steps_per_epoch = N // batch
    total = epochs * steps_per_epoch
    lr_final = lr * 0.05 if lr_final is None else lr_final
    history = []
    step = 0
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(N)).to(stamps.device)
        acc = torch.zeros((), dtype=torch.float64, device=stamps.device)
        for k in range(steps_per_epoch):
            idx = perm[k * batch:(k + 1) * batch]
            x = stamps.index_select(0, idx).contiguous()
            p = pos.index_select(0, idx).contiguous()
            t = targets.index_select(0, idx).contiguous()
            cur = lr_final + 0.5 * (lr - lr_final) * (1.0 + math.cos(math.pi * step / max(total, 1)))
            loss = net.train_step(x, p, t, batch, cur)
            acc += loss[0]
            step += 1
        history.append(float(acc.item()) / max(steps_per_epoch, 1))
        if log:
            log(f"epoch {ep + 1}/{epochs}: train loss {history[-1]:.4f}")
    return history


class GatedDifferencer:
    """Difference one pair with the network's coefficients, falling back to
    the full fit when the chi2 judge rejects them."""

    def __init__(self, width, height, L, dk, db, params, std: Standardizer, *, threshold=1.05,
                 precision=SFFT_NET_BF16, image_dtype="float32", n_stamps=N_STAMPS, device="cuda",
                 refit_background=True, max_pairs=1, in_flight=1, solve_team=0):
        import torch
        self.torch = torch
        if in_flight < 1:
            raise ValueError("in_flight must be >= 1")
        self.diff = Differencer(width, height, L, dk, db, image_dtype=image_dtype, device=device,
                                solve_team=solve_team)
        # run_batch: pair k of a group is refitted, subtracted (and, if
        # rejected, fitted in full) in slot k % in_flight, each slot a
        # Differencer (handle, workspace, result buffers) with its own stream
        self.slots = [self.diff] + [Differencer(width, height, L, dk, db, image_dtype=image_dtype, device=device,
                                                solve_team=solve_team) for _ in range(in_flight - 1)]
        self.slot_streams = [torch.cuda.Stream() for _ in range(in_flight)] if in_flight > 1 else None
        self.max_pairs = int(max_pairs)
        self.net = Surrogate(params, self.diff.N, n_stamps=n_stamps, max_pairs=self.max_pairs,
                             handle=self.diff.handle, device=device)
        self.threshold = float(threshold)
        self.precision = precision
        self.refit = bool(refit_background)
        self.n_stamps = n_stamps
        dev = torch.device(device)
        self.mean = torch.as_tensor(std.mean, dtype=torch.float64, device=dev)
        self.scale = torch.as_tensor(std.scale, dtype=torch.float64, device=dev)
        B = self.max_pairs
        self.stamps_all = torch.empty((B, n_stamps, 2, STAMP, STAMP), dtype=torch.float32, device=dev)
        self.pos_all = torch.empty((B, n_stamps, 2), dtype=torch.float32, device=dev)
        self.pred_all = torch.empty((B, self.diff.N), dtype=torch.float32, device=dev)
        self.coef_all = torch.empty((B, self.diff.N), dtype=torch.float64, device=dev)
        self.chi2_all = torch.empty((B,), dtype=torch.float64, device=dev)
        self.stamps, self.pos = self.stamps_all[0], self.pos_all[0]
        self.pred, self.coef_pred = self.pred_all[:1], self.coef_all[0]

    def predict(self, R, S, centers, refit_background=None, stream=None):
        """Coefficients for the pair (device FP64 [N]); asynchronous. The
        kernel part is the network's; the background part is the network's,
        or (default) the least-squares background for that kernel: the
        sky-subtracted stamps carry no information on the images' sky levels."""
        d = self.diff
        sfft_extract_stamps(d.handle, d.desc, R, S, centers, self.stamps, self.pos, stream)
        self.net.forward(self.stamps, self.pos, 1, precision=self.precision, out=self.pred, stream=stream)
        sfft_surrogate_destandardize(d.handle, self.pred, self.mean, self.scale, 1, d.N, self.coef_pred, stream)
        if self.refit if refit_background is None else refit_background:
            d.refit_background(R, S, coef=self.coef_pred, stream=stream)
        return self.coef_pred

    def run(self, R, S, centers, max_refine=1, stream=None):
        """Returns (accepted, chi2 of the prediction, final chi2)."""
        d = self.diff
        self.predict(R, S, centers, stream=stream)
        d.subtract(R, S, coef=self.coef_pred, stream=stream)
        chi_pred = float(d.buf.chi2.item())          # the judge's decision needs the value on the host
        if chi_pred <= self.threshold:
            return True, chi_pred, chi_pred
        d.run(R, S, max_refine=max_refine, stream=stream)
        return False, chi_pred, float(d.buf.chi2.item())

    def close(self):
        """Release the slots' handles now (the network shares the first)."""
        for sd in self.slots:
            sd.close()

    def run_batch(self, pairs, max_refine=1, stream=None):
        """Gated differencing of up to max_pairs pairs [(R, S, centers), ...]
        with one network launch for all of them and one host read of their
        chi2 values; the rejected pairs are then fitted in full. Pair k is
        refitted and subtracted in slot k % in_flight, and the rejected ones
        are fitted in full in rounds of one per slot; with several slots, each
        on its own stream, one pair's refit (small, latency-bound kernels)
        overlaps other pairs' subtracts. Difference images go through the
        slots' output buffers (slots[j].buf.diff), each overwritten by the
        slot's next pair. Every pair's chi2 values are those of the
        single-slot path with the same solve team. Returns (accepted, chi2 of
        the predictions, final chi2) as lists."""
        torch = self.torch
        B = len(pairs)
        if B > self.max_pairs:
            raise ValueError(f"{B} pairs > max_pairs = {self.max_pairs}")
        d = self.diff
        for k, (R, S, C) in enumerate(pairs):
            sfft_extract_stamps(d.handle, d.desc, R, S, C, self.stamps_all[k], self.pos_all[k], stream)
        self.net.forward(self.stamps_all[:B], self.pos_all[:B], B, precision=self.precision,
                         out=self.pred_all[:B], stream=stream)
        sfft_surrogate_destandardize(d.handle, self.pred_all[:B], self.mean, self.scale, B, d.N,
                                     self.coef_all[:B], stream)
        nsl = len(self.slots)
        main = stream if stream is not None else torch.cuda.current_stream()
        if nsl > 1:
            for s in self.slot_streams:
                s.wait_stream(main)        # the predicted coefficients, and the inputs

        def on_slot(k, j):
            st = self.slot_streams[j] if nsl > 1 else stream
            if nsl > 1:
                for t in pairs[k][:2]:
                    t.record_stream(st)
            return self.slots[j], st

        for k, (R, S, C) in enumerate(pairs):
            sd, st = on_slot(k, k % nsl)
            if self.refit:
                sd.refit_background(R, S, coef=self.coef_all[k], stream=st)
            sfft_subtract(sd.handle, sd.desc, R, S, self.coef_all[k], sd.buf.diff, self.chi2_all[k:k + 1],
                          sd.buf.ws, st)
        if nsl > 1:
            for s in self.slot_streams:
                main.wait_stream(s)
        chi_pred = self.chi2_all[:B].cpu().tolist()     # the judge's decisions need the values on the host
        accepted = [c <= self.threshold for c in chi_pred]
        final = list(chi_pred)
        rejected = [k for k in range(B) if not accepted[k]]
        for i in range(0, len(rejected), nsl):         # rounds of full fits, one pair per slot
            group = rejected[i:i + nsl]
            for j, k in enumerate(group):
                sd, st = on_slot(k, j)
                sd.run(pairs[k][0], pairs[k][1], max_refine=max_refine, stream=st)
            if nsl > 1:
                for s in self.slot_streams:
                    main.wait_stream(s)
            for j, k in enumerate(group):
                final[k] = float(self.slots[j].buf.chi2.item())
        return accepted, chi_pred, final
