"""Seeded synthetic CCD pairs rendered on the GPU with torch, for the
learned form's training and held-out sets (thousands of 2048 x 4096 pairs,
too many for the NumPy renderer). Same model as synth.make_pair: Moffat
(beta = 3) stars with a spatially varying FWHM, a reference model, a
planted spatially varying kernel plus background applied with periodic
FFT convolution, independent Poisson noise (gain 1). Random numbers come
from the pair's seeded PCG64 stream (catalogue, PSF, kernel, background)
and a seeded torch generator (Poisson noise)."""
from __future__ import annotations

import math

import numpy as np

from . import (mono_exponents, n_mono, pack_theta, pixel_gaussian_kernel, seed_for)

CFG_LEARNED = 5


def _norm(n, device, dtype):
    import torch
    return (2.0 * torch.arange(n, device=device, dtype=dtype) / (n - 1) - 1.0) if n > 1 else \
        torch.zeros(1, device=device, dtype=dtype)


def render_moffat(W, H, xs, ys, fl, fwhms, beta=3.0, radius=12, ss=2, device="cuda"):
    """Sum of pixel-integrated (ss x ss supersampled) Moffat profiles, each
    truncated to a (2 radius + 1)^2 patch, normalised to unit sum there and
    scaled by its flux; periodic placement. Returns an (H, W) float64 tensor."""
    import torch
    dt = torch.float64
    xs_t = torch.as_tensor(xs, device=device, dtype=dt)
    ys_t = torch.as_tensor(ys, device=device, dtype=dt)
    fl_t = torch.as_tensor(fl, device=device, dtype=dt)
    alpha = torch.as_tensor(fwhms, device=device, dtype=dt) / (2.0 * math.sqrt(2.0 ** (1.0 / beta) - 1.0))
    ix = torch.floor(xs_t)
    iy = torch.floor(ys_t)
    off = torch.arange(-radius, radius + 1, device=device, dtype=dt)
    sub = (torch.arange(ss, device=device, dtype=dt) + 0.5) / ss - 0.5
    # sample points relative to the star centre: pixel centre at integer + 0.5
    px = (ix[:, None, None] + off[None, :, None] + 0.5 + sub[None, None, :]) - xs_t[:, None, None]
    py = (iy[:, None, None] + off[None, :, None] + 0.5 + sub[None, None, :]) - ys_t[:, None, None]
    a2 = (alpha ** 2)[:, None, None, None, None]
    r2 = px[:, None, None, :, :] ** 2 + py[:, :, :, None, None] ** 2     # (n, y, sy, x, sx)
    prof = (1.0 + r2 / a2) ** (-beta)
    prof = prof.mean(dim=(2, 4))                                          # (n, y, x)
    prof = prof / prof.sum(dim=(1, 2), keepdim=True) * fl_t[:, None, None]
    gy = (iy[:, None] + off[None, :]).long() % H
    gx = (ix[:, None] + off[None, :]).long() % W
    flat = (gy[:, :, None] * W + gx[:, None, :]).reshape(-1)
    img = torch.zeros(H * W, device=device, dtype=dt)
    img.index_add_(0, flat, prof.reshape(-1))
    return img.reshape(H, W)


def plant(src, a, b, DK, DB):
    """Periodic spatially varying convolution of src (torch float64, H x W)
    with kernel coefficients a[i, dy + r, dx + r] (polynomial weight at the
    input pixel) plus background b[c]: the model of synth.plant."""
    import torch
    H, W = src.shape
    dev, dt = src.device, src.dtype
    L = a.shape[-1]
    r = (L - 1) // 2
    xt, yt = _norm(W, dev, dt), _norm(H, dev, dt)
    acc = None
    for i, (ea, eb) in enumerate(mono_exponents(DK)):
        kimg = torch.zeros((H, W), device=dev, dtype=dt)
        ki = torch.as_tensor(a[i], device=dev, dtype=dt)
        rows = torch.arange(-r, r + 1, device=dev) % H
        cols = torch.arange(-r, r + 1, device=dev) % W
        kimg[rows[:, None], cols[None, :]] = ki
        p = (yt[:, None] ** eb) * (xt[None, :] ** ea)
        term = torch.fft.rfft2(p * src) * torch.fft.rfft2(kimg)
        acc = term if acc is None else acc + term
    out = torch.fft.irfft2(acc, s=(H, W))
    for c, (ea, eb) in enumerate(mono_exponents(DB)):
        out = out + float(b[c]) * (yt[:, None] ** eb) * (xt[None, :] ** ea)
    return out


def learned_kernel(rng, L, DK):
    """Random two-Gaussian planted kernel of the learned-form set: widths
    sigma_a ~ U[0.5, 1.0], sigma_b ~ U[1.2, 2.2] px, common sub-pixel centre,
    flux scale s ~ U[0.8, 1.2], mixing polynomial t = sum tau_i p_i with
    tau_0 ~ U[0.3, 0.7], linear terms ~ U[-0.15, 0.15], quadratic ~ U[-0.05, 0.05]."""
    s = float(rng.uniform(0.8, 1.2))
    sa = float(rng.uniform(0.5, 1.0))
    sb = float(rng.uniform(1.2, 2.2))
    mu = tuple(rng.uniform(-0.5, 0.5, size=2))
    ga = pixel_gaussian_kernel(L, sa, mu)
    gb = pixel_gaussian_kernel(L, sb, mu)
    nK = n_mono(DK)
    tau = np.zeros(nK)
    for i, (ea, eb) in enumerate(mono_exponents(DK)):
        d = ea + eb
        tau[i] = rng.uniform(0.3, 0.7) if d == 0 else (rng.uniform(-0.15, 0.15) if d == 1
                                                        else rng.uniform(-0.05, 0.05))
    a = np.empty((nK, L, L))
    for i in range(nK):
        a[i] = s * ((1.0 if i == 0 else 0.0) * ga + tau[i] * (gb - ga))
    return a, dict(s=s, sigma_a=sa, sigma_b=sb, mu=mu, tau=tau)


def make_learned_pair(index: int, W: int = 2048, H: int = 4096, nstars: int = 3000, L: int = 11,
                      DK: int = 2, DB: int = 2, device="cuda"):
    """Pair `index` of the learned-form set: FWHM_R = clip(f0 + gx xt + gy yt,
    2.5, 6) with f0 ~ U[3, 5.5], gx, gy ~ U[-0.5, 0.5] (random spatial
    gradients); flux log-uniform 1e2..1e6; sky U[800, 1500] per image.
    Returns dict(R, S: float32 device tensors; theta: planted coefficients;
    xs, ys, flux: catalogue; meta)."""
    import torch
    seed = seed_for(CFG_LEARNED, index)
    rng = np.random.Generator(np.random.PCG64(seed))
    xs = rng.uniform(0, W, nstars)
    ys = rng.uniform(0, H, nstars)
    fl = np.exp(rng.uniform(math.log(1e2), math.log(1e6), nstars))
    f0 = rng.uniform(3.0, 5.5)
    gxy = rng.uniform(-0.5, 0.5, size=2)
    fw = np.clip(f0 + gxy[0] * (2 * xs / (W - 1) - 1) + gxy[1] * (2 * ys / (H - 1) - 1), 2.5, 6.0)
    sky_R = float(rng.uniform(800, 1500))
    sky_S = float(rng.uniform(800, 1500))
    a, kmeta = learned_kernel(rng, L, DK)
    nB = n_mono(DB)
    b = np.zeros(nB)
    b[0] = sky_S - float(a[0].sum()) * sky_R
    for c, (ea, eb) in enumerate(mono_exponents(DB)):
        if c > 0:
            b[c] = rng.uniform(-20, 20) if ea + eb == 1 else rng.uniform(-10, 10)
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    R_model = sky_R + render_moffat(W, H, xs, ys, fl, fw, device=device)
    S_model = plant(R_model, a, b, DK, DB)
    R = torch.poisson(R_model, generator=g).to(torch.float32)
    S = torch.poisson(torch.clamp(S_model, min=0.0), generator=g).to(torch.float32)
    meta = dict(seed=seed, f0=f0, grad=tuple(gxy), sky_R=sky_R, sky_S=sky_S, **kmeta)
    return dict(R=R, S=S, theta=pack_theta(a, b), xs=xs, ys=ys, flux=fl, meta=meta)


CFG_BATCH = 4


def smooth235(lo: int, hi: int):
    """Even {2,3,5}-smooth integers in [lo, hi]."""
    out = []
    for v in range(lo + (lo & 1), hi + 1, 2):
        x = v
        for f in (2, 3, 5):
            while x % f == 0:
                x //= f
        if x == 1:
            out.append(v)
    return out


def batch_shapes(n_ccd: int = 60, n_cut: int = 40):
    """Shapes (W, H, L) of one exposure: n_ccd 2048 x 4096 CCD pairs and n_cut
    cutouts with {2,3,5}-smooth W in [512, 1536] and H in [512, 2048]; L is 11
    or 15 with equal probability, all drawn from the exposure's seed."""
    rng = np.random.Generator(np.random.PCG64(seed_for(CFG_BATCH, 0)))
    ws = smooth235(512, 1536)
    hs = smooth235(512, 2048)
    shapes = []
    for k in range(n_ccd + n_cut):
        L = 11 if rng.uniform() < 0.5 else 15
        if k < n_ccd:
            shapes.append((2048, 4096, L))
        else:
            shapes.append((int(rng.choice(ws)), int(rng.choice(hs)), L))
    return shapes


def make_batch_pair(index: int, W: int, H: int, L: int, device="cuda"):
    """Pair `index` of the batched-form exposure: the one-CCD recipe (Moffat
    beta = 3, FWHM 3.5 -> 5.0 px along y, ~3000 stars per 2048 x 4096 at the
    same density, flux log-uniform 1e2..1e6, sky U[800, 1500]) with a planted
    two-Gaussian DK = 2 kernel of size L and a quadratic background."""
    import torch
    from . import random_planted_kernel
    seed = seed_for(CFG_BATCH, 1 + index)
    rng = np.random.Generator(np.random.PCG64(seed))
    nstars = max(8, int(round(3000 * (W * H) / (2048 * 4096))))
    xs = rng.uniform(0, W, nstars)
    ys = rng.uniform(0, H, nstars)
    fl = np.exp(rng.uniform(math.log(1e2), math.log(1e6), nstars))
    fw = 3.5 + 1.5 * ys / max(H - 1, 1)
    sky_R = float(rng.uniform(800, 1500))
    sky_S = float(rng.uniform(800, 1500))
    a, kmeta = random_planted_kernel(rng, L, 2, s=float(rng.uniform(0.8, 1.2)))
    b = np.zeros(6)
    b[0] = sky_S - float(a[0].sum()) * sky_R
    for c, (ea, eb) in enumerate(mono_exponents(2)):
        if c > 0:
            b[c] = rng.uniform(-20, 20) if ea + eb == 1 else rng.uniform(-10, 10)
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    R_model = sky_R + render_moffat(W, H, xs, ys, fl, fw, device=device)
    S_model = plant(R_model, a, b, 2, 2)
    R = torch.poisson(R_model, generator=g).to(torch.float32)
    S = torch.poisson(torch.clamp(S_model, min=0.0), generator=g).to(torch.float32)
    return dict(R=R, S=S, theta=pack_theta(a, b), xs=xs, ys=ys, flux=fl, meta=dict(seed=seed, **kmeta))
