"""FP64 CPU oracle for the two optional fit modes of the SFFT build.

TEST INFRASTRUCTURE ONLY. Only tests/, the smoke check in __graft_entry__.py
and the CPU-baseline leg of bench.py may import or run anything in oracle/.
The GPU library never calls it and shares no code with it.

The paper (Sec. 1, the SFFT description) fits a spatially varying kernel in a
delta-function basis; it does not say where its polynomial is evaluated, nor
how SFFT restricts a fit to star stamps. Two readings beside the plain one
(input-pixel polynomial, all pixels):

* Output-pixel convention: the kernel's polynomial is evaluated at the output
  pixel,
      M(x) = sum_i p_i(x) sum_delta a_(i,delta) R'(x - delta) + sum_c b_c q_c(x),
  design column (i, delta) = p_i(x) R'((x - delta) mod (W, H)).
* Masked fit: R' and S' are multiplied by a 0/1 mask (pixels outside it
  become zero in both images, the usual way SFFT keeps only star stamps)
  and the plain periodic problem is solved on the masked images; the
  difference image is then formed from the unmasked images.

With the output-pixel convention the fit also drops the reference pixels
within r = (L - 1) / 2 of an edge (they take part only through the periodic
wrap, where an output-pixel polynomial is not a shift of an input-pixel one):
the reference's effective mask is the given mask (or all ones) times the
interior frame; the science image keeps the given mask.

Both are brute force: the explicit design matrix and lstsq (O1 style), for
tiny images only.
"""
from __future__ import annotations

import numpy as np

from . import sfft_oracle as O


def frame_mask(W: int, H: int, r: int) -> np.ndarray:
    """1 on pixels at least r from every edge, 0 on the r-pixel frame."""
    m = np.zeros((H, W), dtype=np.float64)
    if W > 2 * r and H > 2 * r:
        m[r:H - r, r:W - r] = 1.0
    return m


def effective_mask(W, H, L, mask=None, outpix=False) -> np.ndarray:
    """The reference image's mask (with the frame for the output-pixel
    convention)."""
    m = np.ones((H, W)) if mask is None else (np.asarray(mask) != 0).astype(np.float64)
    if outpix:
        m = m * frame_mask(W, H, (L - 1) // 2)
    return m


def science_mask(W, H, mask=None) -> np.ndarray:
    return np.ones((H, W)) if mask is None else (np.asarray(mask) != 0).astype(np.float64)


def design_matrix_ex(R, L, DK, DB, ref_pedestal=0.0, mask=None, outpix=False) -> np.ndarray:
    """A (H*W x N) of the masked / output-pixel problem."""
    Rp = np.asarray(R, dtype=np.float64) - ref_pedestal
    H, W = Rp.shape
    Rm = Rp * effective_mask(W, H, L, mask, outpix)
    mono = O.poly_images(W, H, DK)
    Q = O.poly_images(W, H, DB)
    cols = []
    for i in range(mono.shape[0]):
        for dy, dx in zip(*O.kernel_offsets(L)):
            if outpix:
                col = mono[i] * np.roll(Rm, shift=(int(dy), int(dx)), axis=(0, 1))
            else:
                col = np.roll(mono[i] * Rm, shift=(int(dy), int(dx)), axis=(0, 1))
            cols.append(col.ravel())
    for c in range(Q.shape[0]):
        cols.append(Q[c].ravel())
    return np.stack(cols, axis=1)


def target_ex(S, L, sci_pedestal=0.0, mask=None, outpix=False) -> np.ndarray:
    Sp = np.asarray(S, dtype=np.float64) - sci_pedestal
    H, W = Sp.shape
    return (Sp * science_mask(W, H, mask)).ravel()


def normal_ex(R, S, L, DK, DB, ref_pedestal=0.0, sci_pedestal=0.0, mask=None, outpix=False):
    A = design_matrix_ex(R, L, DK, DB, ref_pedestal, mask, outpix)
    y = target_ex(S, L, sci_pedestal, mask, outpix)
    return A.T @ A, A.T @ y


def solve_ex(R, S, L, DK, DB, ref_pedestal=0.0, sci_pedestal=0.0, mask=None, outpix=False) -> np.ndarray:
    A = design_matrix_ex(R, L, DK, DB, ref_pedestal, mask, outpix)
    y = target_ex(S, L, sci_pedestal, mask, outpix)
    theta, *_ = np.linalg.lstsq(A, y, rcond=None)
    return theta


def model_image_outpix(R, theta, L, DK, DB, ref_pedestal=0.0) -> np.ndarray:
    """M(x) = sum_i p_i(x) sum_delta a_(i,delta) R'(x - delta) + background,
    on the unmasked reference (periodic)."""
    Rp = np.asarray(R, dtype=np.float64) - ref_pedestal
    H, W = Rp.shape
    a, b = O.split_theta(theta, L, DK, DB)
    mono = O.poly_images(W, H, DK)
    r = (L - 1) // 2
    M = np.zeros((H, W))
    for i in range(mono.shape[0]):
        conv = np.zeros((H, W))
        for dy in range(-r, r + 1):
            for dx in range(-r, r + 1):
                c = a[i, dy + r, dx + r]
                if c != 0.0:
                    conv += c * np.roll(Rp, shift=(dy, dx), axis=(0, 1))
        M += mono[i] * conv
    Q = O.poly_images(W, H, DB)
    for c in range(Q.shape[0]):
        M += b[c] * Q[c]
    return M


def subtract_ex(R, S, theta, L, DK, DB, ref_pedestal=0.0, sci_pedestal=0.0, outpix=False) -> np.ndarray:
    """Difference image of the unmasked images in the chosen convention."""
    Sp = np.asarray(S, dtype=np.float64) - sci_pedestal
    if outpix:
        return Sp - model_image_outpix(R, theta, L, DK, DB, ref_pedestal)
    return Sp - O.model_image(R, theta, L, DK, DB, ref_pedestal)
