"""Seeded synthetic reference/science image pairs for the SFFT differencing path.

This module is the one shared input source for both the CPU oracle and the GPU
library. It renders star fields, plants a known matching kernel and
differential background, and adds Poisson noise. It contains no fitting,
normal-equation, solve or subtraction arithmetic: the planted science image is
produced by FFT convolution of rendered images with rendered kernel images,
which is the data model, not the method.

Workloads stand in for the DECam CCD pairs the paper differences (Sec. 2.3.2,
image differencing; DECam has 62 science CCDs of 2048x4096 pixels, Sec. 1).

Conventions shared with the method's unknown layout (documented beside the
C header): images are (H, W) row-major arrays indexed [y, x]; normalised
coordinates are xt = 2x/(W-1) - 1, yt = 2y/(H-1) - 1; the monomials of total
degree <= D are ordered for d = 0..D, for b = 0..d: (a = d - b, b), i.e.
1, xt, yt, xt^2, xt*yt, yt^2, ...; kernel coefficient (i, dy, dx) lives at
i*L*L + (dy + r)*L + (dx + r), background coefficients follow.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.fft
from scipy.special import erf

BASE_SEED = 260308593


def seed_for(cfg: int, index: int = 0) -> int:
    """Seed of pair `index` of workload `cfg` (PCG64)."""
    return BASE_SEED + 1000 * cfg + index


def rng_for(cfg: int, index: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed_for(cfg, index)))


def n_mono(D: int) -> int:
    return (D + 1) * (D + 2) // 2


def mono_exponents(D: int):
    return [(d - b, b) for d in range(D + 1) for b in range(d + 1)]


def _norm_coord(n: int) -> np.ndarray:
    if n == 1:
        return np.zeros(1)
    return 2.0 * np.arange(n, dtype=np.float64) / (n - 1) - 1.0


def _mono_images(W: int, H: int, D: int):
    xt = _norm_coord(W)[None, :]
    yt = _norm_coord(H)[:, None]
    return [np.broadcast_to(xt ** a * yt ** b, (H, W)) for (a, b) in mono_exponents(D)]


# ----------------------------------------------------------------------------
# star rendering (periodic: a star near an edge wraps to the opposite edge)
# ----------------------------------------------------------------------------

def _pix_gauss_1d(offsets: np.ndarray, centre: float, sigma: float) -> np.ndarray:
    """Pixel-integrated unit Gaussian on pixels centred at `offsets`."""
    s = sigma * math.sqrt(2.0)
    return 0.5 * (erf((offsets + 0.5 - centre) / s) - erf((offsets - 0.5 - centre) / s))


def render_gaussian_stars(W, H, xs, ys, fluxes, sigma, radius=None):
    img = np.zeros((H, W), dtype=np.float64)
    rad = int(radius if radius is not None else math.ceil(6 * sigma) + 1)
    offs = np.arange(-rad, rad + 1)
    for x0, y0, f in zip(xs, ys, fluxes):
        ix, iy = int(round(x0)), int(round(y0))
        gx = _pix_gauss_1d(ix + offs, x0, sigma)
        gy = _pix_gauss_1d(iy + offs, y0, sigma)
        cols = (ix + offs) % W
        rows = (iy + offs) % H
        np.add.at(img, (rows[:, None], cols[None, :]), f * np.outer(gy, gx))
    return img


def render_moffat_stars(W, H, xs, ys, fluxes, fwhms, beta=3.0, oversample=4, max_radius=40):
    """Moffat profiles, pixel-integrated by oversample x oversample sampling."""
    img = np.zeros((H, W), dtype=np.float64)
    sub = (np.arange(oversample) + 0.5) / oversample - 0.5
    for x0, y0, f, fw in zip(xs, ys, fluxes, fwhms):
        alpha = fw / (2.0 * math.sqrt(2.0 ** (1.0 / beta) - 1.0))
        # radius where the enclosed-flux deficit drops below ~1e-5 of the flux
        rad = int(min(max_radius, math.ceil(alpha * (1e5 ** (1.0 / (2 * (beta - 1))))) + 1))
        ix, iy = int(round(x0)), int(round(y0))
        offs = np.arange(-rad, rad + 1)
        px = (ix + offs)[:, None] + sub[None, :]          # (n, os)
        py = (iy + offs)[:, None] + sub[None, :]
        dx2 = (px - x0) ** 2
        dy2 = (py - y0) ** 2
        r2 = dy2[:, None, :, None] + dx2[None, :, None, :]   # (ny, nx, os, os)
        prof = (beta - 1.0) / (math.pi * alpha * alpha) * (1.0 + r2 / (alpha * alpha)) ** (-beta)
        stamp = prof.mean(axis=(2, 3)) * f
        cols = (ix + offs) % W
        rows = (iy + offs) % H
        np.add.at(img, (rows[:, None], cols[None, :]), stamp)
    return img


def pixel_gaussian_kernel(L: int, sigma: float, mu=(0.0, 0.0), total: float = 1.0) -> np.ndarray:
    """L x L pixel-integrated Gaussian indexed [dy + r, dx + r], centred at
    (mu_x, mu_y) pixels, normalised to sum `total`."""
    r = (L - 1) // 2
    offs = np.arange(-r, r + 1, dtype=np.float64)
    k = np.outer(_pix_gauss_1d(offs, mu[1], sigma), _pix_gauss_1d(offs, mu[0], sigma))
    return k * (total / k.sum())


# ----------------------------------------------------------------------------
# planting: S_model = sum_i (p_i * src) (*) k_i + sum_c b_c q_c, circular
# ----------------------------------------------------------------------------

def plant(src: np.ndarray, a: np.ndarray, b: np.ndarray, DK: int, DB: int) -> np.ndarray:
    """Apply a planted spatially varying kernel (coefficients a[i, dy+r, dx+r],
    polynomial weight evaluated at the input pixel) and background b[c] to
    `src`, with periodic boundaries. Implemented as FFT convolution with
    kernel images."""
    H, W = src.shape
    L = a.shape[-1]
    r = (L - 1) // 2
    monos = _mono_images(W, H, DK)
    acc = None
    for i, p in enumerate(monos):
        kimg = np.zeros((H, W))
        for dy in range(-r, r + 1):
            for dx in range(-r, r + 1):
                kimg[dy % H, dx % W] += a[i, dy + r, dx + r]
        term = scipy.fft.rfft2(p * src, workers=-1) * scipy.fft.rfft2(kimg, workers=-1)
        acc = term if acc is None else acc + term
    out = scipy.fft.irfft2(acc, s=(H, W), workers=-1)
    for c, q in enumerate(_mono_images(W, H, DB)):
        out = out + b[c] * q
    return out


def pack_theta(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    return np.concatenate([a.reshape(-1), np.asarray(b, dtype=np.float64).reshape(-1)])


@dataclass
class Pair:
    R: np.ndarray
    S: np.ndarray
    L: int
    DK: int
    DB: int
    a: np.ndarray            # planted kernel coefficients (nK, L, L)
    b: np.ndarray            # planted background (nB,)
    R_model: np.ndarray | None = None
    S_model: np.ndarray | None = None
    meta: dict = field(default_factory=dict)

    @property
    def theta(self) -> np.ndarray:
        return pack_theta(self.a, self.b)


def random_planted_kernel(rng, L, DK, s=1.0, sigma_a=0.6, sigma_b=1.6, lin=0.10, quad=0.03):
    """Two-Gaussian kernel mixed by a polynomial t(u) = sum_i tau_i p_i(u):
    a_(i, delta) = s ([i == 0] g_a(delta) + tau_i (g_b - g_a)(delta)). Its
    kernel sums are exactly s (i = 0) and 0 (i > 0)."""
    mu = tuple(rng.uniform(-0.5, 0.5, size=2))
    ga = pixel_gaussian_kernel(L, sigma_a, mu)
    gb = pixel_gaussian_kernel(L, sigma_b, mu)
    nK = n_mono(DK)
    tau = np.zeros(nK)
    for i, (ea, eb) in enumerate(mono_exponents(DK)):
        d = ea + eb
        if d == 0:
            tau[i] = rng.uniform(0.4, 0.6)
        elif d == 1:
            tau[i] = rng.uniform(-lin, lin)
        else:
            tau[i] = rng.uniform(-quad, quad)
    a = np.empty((nK, L, L))
    for i in range(nK):
        a[i] = s * ((1.0 if i == 0 else 0.0) * ga + tau[i] * (gb - ga))
    return a, dict(mu=mu, tau=tau)


def make_pair(W, H, L, DK, DB, *, seed, nstars=60, psf="gaussian", fwhm=3.0,
              fwhm_end=None, flux=(1e3, 1e5), sky_R=1000.0, sky_S=None,
              kernel=None, b=None, s=None, noise_R=True, noise_S=True,
              source="model", dtype=np.float64) -> Pair:
    """Generic seeded pair.

    source="model": S is planted from the noise-free reference model (the
    workloads as described: reference and science noised independently).
    source="noisy": S is planted from the noisy R itself, so that with
    noise_S=False the pair lies exactly in the model class.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    xs = rng.uniform(0, W, nstars)
    ys = rng.uniform(0, H, nstars)
    fl = np.exp(rng.uniform(math.log(flux[0]), math.log(flux[1]), nstars))
    if psf == "gaussian":
        stars = render_gaussian_stars(W, H, xs, ys, fl, fwhm / (2 * math.sqrt(2 * math.log(2))))
    else:
        fe = fwhm if fwhm_end is None else fwhm_end
        fw = fwhm + (fe - fwhm) * (ys / max(H - 1, 1))
        stars = render_moffat_stars(W, H, xs, ys, fl, fw)
    R_model = sky_R + stars
    R = rng.poisson(R_model).astype(np.float64) if noise_R else R_model.copy()
    if s is None:
        s = float(rng.uniform(0.8, 1.2))
    if kernel is None:
        a, kmeta = random_planted_kernel(rng, L, DK, s=s)
    else:
        a, kmeta = np.asarray(kernel, dtype=np.float64), {}
    nB = n_mono(DB)
    if b is None:
        b = np.zeros(nB)
        tgt = sky_S if sky_S is not None else float(rng.uniform(800, 1500))
        b[0] = tgt - float(a[0].sum()) * sky_R
        for c, (ea, eb) in enumerate(mono_exponents(DB)):
            if c > 0:
                b[c] = rng.uniform(-20, 20) if ea + eb == 1 else rng.uniform(-10, 10)
    b = np.asarray(b, dtype=np.float64)
    src = R_model if source == "model" else R
    S_model = plant(src, a, b, DK, DB)
    if noise_S:
        S = rng.poisson(np.maximum(S_model, 0.0)).astype(np.float64)
    else:
        S = S_model.copy()
    meta = dict(seed=seed, xs=xs, ys=ys, flux=fl, s=s, sky_R=sky_R, psf=psf, **kmeta)
    return Pair(R.astype(dtype), S.astype(dtype), L, DK, DB, a, b, R_model, S_model, meta)


# ----------------------------------------------------------------------------
# the named workloads
# ----------------------------------------------------------------------------

def make_cfg1(index: int = 0) -> Pair:
    """256x256 FP64: 60 Gaussian stars (FWHM 3 px, flux log-uniform 1e3..1e5),
    sky 1000 + Poisson. Science = reference model convolved with a constant
    7x7 pixel-integrated Gaussian (sigma^2 = s_3.6^2 - s_3.0^2, centred at
    +0.3 px in x, sum 0.9) + linear background + fresh Poisson noise. Fit
    L=7, DK=0, DB=1."""
    seed = seed_for(1, index)
    rng = np.random.Generator(np.random.PCG64(seed + 7919))
    sig = math.sqrt((3.6 / 2.3548200450309493) ** 2 - (3.0 / 2.3548200450309493) ** 2)
    k = pixel_gaussian_kernel(7, sig, (0.3, 0.0), 0.9)[None]
    b = np.array([rng.uniform(80, 120), rng.uniform(-20, 20), rng.uniform(-20, 20)])
    return make_pair(256, 256, 7, 0, 1, seed=seed, nstars=60, psf="gaussian", fwhm=3.0,
                     flux=(1e3, 1e5), sky_R=1000.0, kernel=k, b=b, s=0.9,
                     dtype=np.float64)


def make_cfg2(index: int = 0, W: int = 2048, H: int = 4096, nstars: int | None = None,
              L: int = 11, cfg: int = 2) -> Pair:
    """One DECam-CCD-shaped pair (default 2048x4096 FP32): ~3000 Moffat(beta=3)
    stars with FWHM varying linearly 3.5 -> 5.0 px along y, flux log-uniform
    1e2..1e6, sky U[800,1500] per image + Poisson; science PSF broadened by a
    spatially quadratic (DK=2) kernel, quadratic background. Fit L, DK=2, DB=2.
    Smaller W, H keep the star density."""
    seed = seed_for(cfg, index)
    rng = np.random.Generator(np.random.PCG64(seed + 104729))
    if nstars is None:
        nstars = max(8, int(round(3000 * (W * H) / (2048 * 4096))))
    sky_R = float(rng.uniform(800, 1500))
    sky_S = float(rng.uniform(800, 1500))
    return make_pair(W, H, L, 2, 2, seed=seed, nstars=nstars, psf="moffat", fwhm=3.5,
                     fwhm_end=5.0, flux=(1e2, 1e6), sky_R=sky_R, sky_S=sky_S,
                     dtype=np.float32)


def pick_centers(xs, ys, fl, W, H, n, size, r):
    """The n brightest stars at least size//2 + r + 1 px from every edge with
    no other star brighter than 1% of their flux within `size` px; ties by
    catalogue index; centre = nearest pixel (round half to even). Returns
    int32 array (n, 2) of (x, y) (fewer rows if fewer stars qualify)."""
    xs, ys, fl = np.asarray(xs), np.asarray(ys), np.asarray(fl)
    margin = size // 2 + r + 1
    order = sorted(range(len(fl)), key=lambda k: (-fl[k], k))
    out = []
    for k in order:
        cx, cy = int(np.rint(xs[k])), int(np.rint(ys[k]))
        if not (margin <= cx < W - margin and margin <= cy < H - margin):
            continue
        d = np.hypot(xs - xs[k], ys - ys[k])
        bad = (d < size) & (fl > 0.01 * fl[k])
        bad[k] = False
        if bad.any():
            continue
        out.append((cx, cy))
        if len(out) == n:
            break
    return np.asarray(out, dtype=np.int32).reshape(-1, 2)


def pick_stamps(pair: Pair, n: int = 64, size: int = 41):
    """Stamp centres of a pair (pick_centers on its catalogue)."""
    H, W = pair.R.shape
    return pick_centers(pair.meta["xs"], pair.meta["ys"], pair.meta["flux"], W, H, n, size,
                        (pair.L - 1) // 2)


def surrogate_init(n_out: int, seed: int) -> np.ndarray:
    """Seeded initial parameters of the learned form's network as one flat
    FP32 vector, in the layout (conv1..conv4 weight, bias; fc1..fc3 weight,
    bias): weights uniform in +-sqrt(6 / fan_in) (He), biases zero."""
    rng = np.random.default_rng(seed)
    shapes = []
    for ci, co in ((2, 16), (16, 32), (32, 64), (64, 64)):
        shapes += [((co, ci, 3, 3), ci * 9), ((co,), 0)]
    shapes += [((128, 1024), 1024), ((128,), 0), ((512, 768), 768), ((512,), 0),
               ((n_out, 512), 512), ((n_out,), 0)]
    parts = []
    for shape, fan_in in shapes:
        n = int(np.prod(shape))
        if fan_in:
            lim = np.sqrt(6.0 / fan_in)
            parts.append(rng.uniform(-lim, lim, n))
        else:
            parts.append(np.zeros(n))
    return np.concatenate(parts).astype(np.float32)


# ----------------------------------------------------------------------------
# multi-template workload and photometry positions
# ----------------------------------------------------------------------------

@dataclass
class MultiTemplate:
    S: np.ndarray                 # science image (H, W)
    templates: list               # n_temp reference images (H, W)
    zp_sci: float                 # science zero point
    zp_templates: np.ndarray      # zero point of each template
    transients: np.ndarray        # (n, 3): x, y, flux in science counts
    meta: dict = field(default_factory=dict)


def make_multi_template(W, H, n_temp=5, *, seed, nstars=None, fwhm_sci=4.2, fwhm_tmpl=(2.8, 3.6),
                        flux=(1e2, 1e5), n_transients=6, transient_flux=(2e3, 2e4), zp_sci=30.0,
                        background=True, dtype=np.float32) -> MultiTemplate:
    """One science image and n_temp aligned templates of the same star field
    (the multi-exposure template set of the paper's Sec. 2.2.1, N_TEMP = 5
    by default). Templates: Gaussian PSFs with FWHM U[fwhm_tmpl], flux
    scales U[0.7, 1.4] (so zero points zp_sci + 2.5 log10(scale)), skies
    U[800, 1500], Poisson noise. Science: a broader Gaussian PSF (fwhm_sci),
    sky U[800, 1500] plus a linear gradient, point-source transients present
    in it only, Poisson noise. Each template maps onto the science image by a
    Gaussian kernel of variance sigma_sci^2 - sigma_t^2 and sum 1/scale_t (up
    to pixel integration), so the fit of every template is close to the
    model class."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if nstars is None:
        nstars = max(8, int(round(3000 * (W * H) / (2048 * 4096))))
    xs = rng.uniform(0, W, nstars)
    ys = rng.uniform(0, H, nstars)
    fl = np.exp(rng.uniform(math.log(flux[0]), math.log(flux[1]), nstars))
    k = 2.0 * math.sqrt(2.0 * math.log(2.0))
    templates, zps, fws, scales = [], [], [], []
    for _ in range(n_temp):
        fw = float(rng.uniform(*fwhm_tmpl))
        sc = float(rng.uniform(0.7, 1.4))
        sky = float(rng.uniform(800, 1500))
        model = sky + sc * render_gaussian_stars(W, H, xs, ys, fl, fw / k)
        templates.append(rng.poisson(model).astype(dtype))
        zps.append(zp_sci + 2.5 * math.log10(sc))
        fws.append(fw)
        scales.append(sc)
    # transients: away from the edges, in the science image only
    m = 16
    tx = rng.uniform(m, W - m, n_transients)
    ty = rng.uniform(m, H - m, n_transients)
    tf = np.exp(rng.uniform(math.log(transient_flux[0]), math.log(transient_flux[1]), n_transients))
    sky_s = float(rng.uniform(800, 1500))
    smodel = sky_s + render_gaussian_stars(W, H, np.concatenate([xs, tx]), np.concatenate([ys, ty]),
                                           np.concatenate([fl, tf]), fwhm_sci / k)
    if background:
        xt = _norm_coord(W)[None, :]
        yt = _norm_coord(H)[:, None]
        smodel = smodel + rng.uniform(-20, 20) * xt + rng.uniform(-20, 20) * yt
    S = rng.poisson(np.maximum(smodel, 0.0)).astype(dtype)
    return MultiTemplate(S, templates, zp_sci, np.array(zps), np.stack([tx, ty, tf], axis=1),
                         dict(seed=seed, fwhm_templates=fws, scales=scales, fwhm_sci=fwhm_sci))


def background_positions(W, H, n, radius, *, seed, avoid=None, avoid_radius=0.0):
    """n aperture centres (x, y) drawn uniformly with the whole aperture
    inside the image (at least radius + 1 px from every edge); positions
    closer than avoid_radius to any (x, y) row of `avoid` are redrawn. Real
    positions (sub-pixel). float64 array (n, 2)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m = radius + 1.0
    out = []
    av = None if avoid is None else np.asarray(avoid, dtype=np.float64)[:, :2]
    while len(out) < n:
        x = float(rng.uniform(m, W - 1 - m))
        y = float(rng.uniform(m, H - 1 - m))
        if av is not None and len(av) and np.min(np.hypot(av[:, 0] - x, av[:, 1] - y)) < avoid_radius:
            continue
        out.append((x, y))
    return np.asarray(out, dtype=np.float64)


def rb_init(seed: int, n_params: int = 315009) -> np.ndarray:
    """Seeded random parameters of the real-bogus scorer as one flat FP32
    vector in its parameter layout: conv and
    linear weights uniform in +-sqrt(6 / fan_in) (He), biases uniform in
    +-0.05. The layout: conv (out, in, k) in the order stem (32, 3, 3),
    b1a (32, 32, 3), b1b (32, 32, 3), b2a (64, 32, 3), b2b (64, 64, 3),
    b2p (64, 32, 1), b3a (128, 64, 3), b3b (128, 128, 3), b3p (128, 64, 1),
    each weight then bias; fc1 (64, 128), fc2 (1, 64)."""
    rng = np.random.default_rng(seed)
    convs = [(32, 3, 3), (32, 32, 3), (32, 32, 3), (64, 32, 3), (64, 64, 3), (64, 32, 1),
             (128, 64, 3), (128, 128, 3), (128, 64, 1)]
    parts = []
    for co, ci, k in convs:
        fan = ci * k * k
        parts.append(rng.uniform(-1, 1, co * ci * k * k) * math.sqrt(6.0 / fan))
        parts.append(rng.uniform(-0.05, 0.05, co))
    for co, ci in ((64, 128), (1, 64)):
        parts.append(rng.uniform(-1, 1, co * ci) * math.sqrt(6.0 / ci))
        parts.append(rng.uniform(-0.05, 0.05, co))
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == n_params
    return p


def rb_candidates(pair_or_shape, n, *, seed, margin=20):
    """n candidate centres (x, y) (int32) uniformly inside the image, at least
    `margin` px from the edges (positions of detections on a difference image
    stand in for a detector's output)."""
    H, W = pair_or_shape
    rng = np.random.Generator(np.random.PCG64(seed))
    xs = rng.integers(margin, W - margin, n)
    ys = rng.integers(margin, H - margin, n)
    return np.stack([xs, ys], axis=1).astype(np.int32)
