"""FP64 CPU oracle for the products made from difference images.

TEST INFRASTRUCTURE ONLY. Only tests/, the smoke check in __graft_entry__.py
and the CPU-baseline leg of bench.py may import or run anything in oracle/.
The GPU library never calls it and shares no code with it.

1. Multi-template differencing (paper Sec. 2.3.2, image differencing; the
   template set of N_TEMP exposures, default 5, from Sec. 2.2.1): the science
   image is differenced against each template separately, every difference
   image is brought to one common photometric zero point, and the stack is
   median-combined pixel by pixel.
   Readings: a difference image with zero point zp_t is scaled by
   10^(0.4 (zp_common - zp_t)) (magnitudes m = zp - 2.5 log10(flux)); the
   median of an even count is the mean of the two middle values (the usual
   definition); each template is fitted with the same L, DK, DB.

2. Aperture photometry on a difference image (paper Sec. 2.3.3,
   differential photometry; forced photometry at fixed positions,
   Sec. 2.4.3): the flux in a circular aperture of radius r is the sum over
   pixels of the pixel value times the area of the pixel square
   [x - 1/2, x + 1/2] x [y - 1/2, y + 1/2] that lies inside the circle
   (pixel centres at integer coordinates; pixels outside the image
   contribute nothing). The limiting magnitude: aperture fluxes at n random
   background positions, sigma = their sample standard deviation (n - 1 in
   the denominator), m_lim = zp - 2.5 log10(nsigma * sigma) with nsigma = 5.
   Forced photometry: the aperture flux at given positions, its magnitude
   zp - 2.5 log10(flux) (NaN when flux <= 0) and the magnitude error
   (2.5 / ln 10) sigma / |flux| with sigma from the background apertures.

Pins (tests/test_oracle_products.py): the median against a sort-based
middle element in pure Python, the zero-point scale against known magnitude
differences, the overlap area against a fine sub-pixel grid count and the
disk area, the aperture sum of a constant image, the limiting magnitude of
a hand-computed case.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.integrate

from . import sfft_oracle as O

# ---------------------------------------------------------------------------
# 1. multi-template differencing and the median combine
# ---------------------------------------------------------------------------


def zp_scale(zp_from: float, zp_to: float) -> float:
    """Factor that brings fluxes measured with zero point zp_from to zero
    point zp_to: m = zp - 2.5 log10(f) is the same magnitude for both."""
    return 10.0 ** (0.4 * (zp_to - zp_from))


def median_combine(diffs, zps, zp_common) -> np.ndarray:
    """Pixelwise median of the zero-point-normalised difference images."""
    stack = np.stack([np.asarray(D, dtype=np.float64) * zp_scale(z, zp_common)
                      for D, z in zip(diffs, zps)])
    return np.median(stack, axis=0)


def difference_multi(templates, S, L, DK, DB, zps, zp_common, ref_pedestals=None,
                     sci_pedestal=0.0, refine=2):
    """The science image against every template (O2 build + Cholesky +
    direct subtraction each), then the normalised median."""
    outs = []
    for t, R in enumerate(templates):
        cR = 0.0 if ref_pedestals is None else float(ref_pedestals[t])
        outs.append(O.difference(R, S, L, DK, DB, cR, sci_pedestal, refine))
    comb = median_combine([o["D"] for o in outs], zps, zp_common)
    return dict(each=outs, combined=comb)


# ---------------------------------------------------------------------------
# 2. aperture photometry
# ---------------------------------------------------------------------------


def overlap_area(cx: float, cy: float, radius: float, px: int, py: int) -> float:
    """Area of the pixel square centred on (px, py) inside the circle of
    `radius` around (cx, cy): the integral over x of the length of the
    vertical chord of the circle that lies within the pixel's y range,
    evaluated by adaptive quadrature with the chord's kinks as breakpoints."""
    x0, x1 = px - 0.5 - cx, px + 0.5 - cx
    y0, y1 = py - 0.5 - cy, py + 0.5 - cy
    a, b = max(x0, -radius), min(x1, radius)
    if a >= b:
        return 0.0
    r2 = radius * radius

    def chord(u):
        s = math.sqrt(max(r2 - u * u, 0.0))
        return max(0.0, min(y1, s) - max(y0, -s))

    pts = [u for yy in (y0, y1) if abs(yy) < radius
           for u in (-math.sqrt(r2 - yy * yy), math.sqrt(r2 - yy * yy)) if a < u < b]
    val, _ = scipy.integrate.quad(chord, a, b, points=sorted(pts) or None, epsabs=1e-14, epsrel=1e-12,
                                  limit=200)
    return float(val)


def aperture_weights(cx: float, cy: float, radius: float, W: int, H: int):
    """(ys, xs, w): every image pixel with a nonzero overlap and its area."""
    ys, xs, ws = [], [], []
    for py in range(int(math.floor(cy - radius - 1)), int(math.ceil(cy + radius + 1)) + 1):
        if py < 0 or py >= H:
            continue
        for px in range(int(math.floor(cx - radius - 1)), int(math.ceil(cx + radius + 1)) + 1):
            if px < 0 or px >= W:
                continue
            w = overlap_area(cx, cy, radius, px, py)
            if w > 0.0:
                ys.append(py)
                xs.append(px)
                ws.append(w)
    return np.array(ys, dtype=np.int64), np.array(xs, dtype=np.int64), np.array(ws)


def aperture_flux(image, xy, radius: float) -> np.ndarray:
    """Aperture sums at the positions xy[k] = (x, y) (pixel coordinates)."""
    img = np.asarray(image, dtype=np.float64)
    H, W = img.shape
    out = np.zeros(len(xy))
    for k, (cx, cy) in enumerate(np.asarray(xy, dtype=np.float64)):
        ys, xs, w = aperture_weights(float(cx), float(cy), radius, W, H)
        out[k] = float(np.sum(w * img[ys, xs])) if len(w) else 0.0
    return out


def limiting_magnitude(image, xy, radius: float, zp: float, nsigma: float = 5.0):
    """(sigma, m_lim, fluxes) from aperture sums at background positions."""
    f = aperture_flux(image, xy, radius)
    sigma = float(np.std(f, ddof=1))
    return sigma, zp - 2.5 * math.log10(nsigma * sigma), f


def forced_photometry(image, xy, radius: float, zp: float, sigma: float):
    """(flux, mag, mag_err) at fixed positions."""
    f = aperture_flux(image, xy, radius)
    mag = np.full(len(f), np.nan)
    err = np.full(len(f), np.nan)
    pos = f > 0
    mag[pos] = zp - 2.5 * np.log10(f[pos])
    nz = f != 0
    err[nz] = 2.5 / math.log(10.0) * sigma / np.abs(f[nz])
    return f, mag, err
