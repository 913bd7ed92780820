"""FP64 CPU oracle for the SFFT image-differencing hot path.

TEST INFRASTRUCTURE ONLY. Only tests/, the smoke check in __graft_entry__.py
and the CPU-baseline leg of bench.py may import or run anything in oracle/.
The GPU library never calls it, shares no code with it, and no stored
expected value comes from the GPU path.

What the method computes (paper Sec. 1 and Sec. 2.3.2): SFFT fits, between an
aligned reference R and science image S, a matching kernel in a delta-function
basis (free pixel values on an L x L grid) whose values vary over the image as
a polynomial of degree DK, plus a differential background polynomial of degree
DB, by least squares formulated in the Fourier domain; then it convolves the
reference with the fitted kernel and subtracts. The paper prints none of the
equations, so the plain definition below is written out from linear least
squares and the convolution theorem:

    theta* = argmin sum_x ( S'(x) - M_theta(x) )^2,
    M_theta(x) = sum_i sum_delta a_(i,delta) p_i(x - delta) R'(x - delta)
                 + sum_c b_c q_c(x),
    D = S' - M_theta*,

with R' = R - c_R, S' = S - c_S (scalar pedestals), every index taken modulo
the image size (periodic boundary), p_i and q_c the monomials of total degree
<= DK resp. <= DB in xt = 2x/(W-1) - 1, yt = 2y/(H-1) - 1, ordered
for d = 0..D, for b = 0..d: (xt^(d-b) yt^b). The polynomial weight of the
kernel is evaluated at the input (reference) pixel. Unknown (i, dy, dx) is at
i*L*L + (dy+r)*L + (dx+r), r = (L-1)/2; background c follows all kernel terms.

Two independent routes to theta*:
  O1 (solve_bruteforce): explicit design matrix built with np.roll, lstsq.
  O2 (build_fft64 + solve_cholesky64): the normal equations G theta = h with
     every block filled by an FFT cross-correlation, then an equilibrated
     Cholesky solve with iterative refinement.
Subtraction (subtract64) is the direct tap-by-tap sum; chi2_nu is the
residual judge used to accept a difference image.

Every function is pinned by tests marked "not gpu" (brute force on tiny
inputs, exact recovery of a planted kernel, kernel-sum invariant, textbook
special cases, orthogonality of the residual, chi2 ~ 1 on in-model noise).
"""
from __future__ import annotations

import re
from dataclasses import dataclass

import numpy as np
import scipy.fft
import scipy.linalg

# ---------------------------------------------------------------------------
# conventions
# ---------------------------------------------------------------------------


def n_mono(D: int) -> int:
    """Number of monomials of total degree <= D in two variables."""
    return (D + 1) * (D + 2) // 2


def monomials(D: int):
    """Exponent pairs (a, b) of xt^a yt^b in the unknown layout's order."""
    return [(d - b, b) for d in range(D + 1) for b in range(d + 1)]


def n_unknowns(L: int, DK: int, DB: int) -> int:
    return L * L * n_mono(DK) + n_mono(DB)


def norm_coord(n: int) -> np.ndarray:
    """2 k / (n - 1) - 1 for k = 0..n-1 (0 for n == 1)."""
    if n == 1:
        return np.zeros(1)
    return 2.0 * np.arange(n, dtype=np.float64) / (n - 1) - 1.0


def poly_images(W: int, H: int, D: int) -> np.ndarray:
    """(n_mono(D), H, W) stack of monomial images."""
    xt = norm_coord(W)[None, :]
    yt = norm_coord(H)[:, None]
    return np.stack([np.broadcast_to(xt ** a * yt ** b, (H, W)) for a, b in monomials(D)])


def kernel_offsets(L: int):
    """(dy, dx) of the L*L kernel taps in layout order (dy major)."""
    r = (L - 1) // 2
    dy, dx = np.meshgrid(np.arange(-r, r + 1), np.arange(-r, r + 1), indexing="ij")
    return dy.ravel(), dx.ravel()


def split_theta(theta: np.ndarray, L: int, DK: int, DB: int):
    nK = n_mono(DK)
    a = np.asarray(theta[: nK * L * L], dtype=np.float64).reshape(nK, L, L)
    b = np.asarray(theta[nK * L * L:], dtype=np.float64)
    return a, b


def _prep(R, S, ref_pedestal, sci_pedestal):
    Rp = np.asarray(R, dtype=np.float64) - float(ref_pedestal)
    Sp = None if S is None else np.asarray(S, dtype=np.float64) - float(sci_pedestal)
    return Rp, Sp


# ---------------------------------------------------------------------------
# O1: brute-force least squares on the explicit design matrix
# ---------------------------------------------------------------------------


def design_matrix(R, L, DK, DB, ref_pedestal=0.0) -> np.ndarray:
    """A (H*W x N): column (i, delta) is the image p_i R' shifted by +delta
    (value at x is (p_i R')(x - delta), periodic); column c is q_c."""
    Rp, _ = _prep(R, None, ref_pedestal, 0.0)
    H, W = Rp.shape
    P = poly_images(W, H, DK) * Rp
    Q = poly_images(W, H, DB)
    cols = []
    for i in range(P.shape[0]):
        for dy, dx in zip(*kernel_offsets(L)):
            cols.append(np.roll(P[i], shift=(int(dy), int(dx)), axis=(0, 1)).ravel())
    for c in range(Q.shape[0]):
        cols.append(Q[c].ravel())
    return np.stack(cols, axis=1)


def normal_bruteforce(R, S, L, DK, DB, ref_pedestal=0.0, sci_pedestal=0.0):
    """G = A^T A, h = A^T S' from the explicit design matrix."""
    A = design_matrix(R, L, DK, DB, ref_pedestal)
    y = (np.asarray(S, dtype=np.float64) - sci_pedestal).ravel()
    return A.T @ A, A.T @ y


def solve_bruteforce(R, S, L, DK, DB, ref_pedestal=0.0, sci_pedestal=0.0) -> np.ndarray:
    """theta* by SVD-based lstsq on the explicit design matrix."""
    A = design_matrix(R, L, DK, DB, ref_pedestal)
    y = (np.asarray(S, dtype=np.float64) - sci_pedestal).ravel()
    theta, *_ = np.linalg.lstsq(A, y, rcond=None)
    return theta


# ---------------------------------------------------------------------------
# O2: FP64 FFT normal equations
# ---------------------------------------------------------------------------


def fft_correlation(f: np.ndarray, g: np.ndarray) -> np.ndarray:
    """C[dy, dx] = sum_u f(u) g(u + (dy, dx)), periodic, via the convolution
    theorem: C = IDFT( conj(DFT f) * DFT g )."""
    H, W = f.shape
    Ff = scipy.fft.rfft2(f, workers=-1)
    Fg = scipy.fft.rfft2(g, workers=-1)
    return scipy.fft.irfft2(np.conj(Ff) * Fg, s=(H, W), workers=-1)


def build_fft64(R, S, L, DK, DB, ref_pedestal=0.0, sci_pedestal=0.0):
    """Normal equations of the periodic least-squares problem, every block
    from a full (unpruned) FFT cross-correlation:
      G[(i,d),(j,d')] = C_{P_i,P_j}(d - d'),  G[(i,d),c] = C_{P_i,q_c}(d),
      G[c,c'] = sum q_c q_c',  h[(i,d)] = C_{P_i,S'}(d),  h[c] = sum q_c S',
    with P_i = p_i R' and C_{f,g}(D) = sum_u f(u) g(u + D)."""
    Rp, Sp = _prep(R, S, ref_pedestal, sci_pedestal)
    H, W = Rp.shape
    nK, nB = n_mono(DK), n_mono(DB)
    L2 = L * L
    N = nK * L2 + nB
    P = poly_images(W, H, DK) * Rp
    Q = poly_images(W, H, DB)
    FP = [scipy.fft.rfft2(P[i], workers=-1) for i in range(nK)]
    FQ = [scipy.fft.rfft2(Q[c], workers=-1) for c in range(nB)]
    FS = scipy.fft.rfft2(Sp, workers=-1)

    def corr(Fa, Fb):
        return scipy.fft.irfft2(np.conj(Fa) * Fb, s=(H, W), workers=-1)

    dy, dx = kernel_offsets(L)
    ddy = (dy[:, None] - dy[None, :]) % H
    ddx = (dx[:, None] - dx[None, :]) % W
    G = np.zeros((N, N))
    h = np.zeros(N)
    kb = nK * L2
    for i in range(nK):
        si = slice(i * L2, (i + 1) * L2)
        for j in range(i, nK):
            sj = slice(j * L2, (j + 1) * L2)
            C = corr(FP[i], FP[j])
            blk = C[ddy, ddx]
            G[si, sj] = blk
            G[sj, si] = blk.T
        for c in range(nB):
            C = corr(FP[i], FQ[c])
            col = C[dy % H, dx % W]
            G[si, kb + c] = col
            G[kb + c, si] = col
        C = corr(FP[i], FS)
        h[si] = C[dy % H, dx % W]
    for c in range(nB):
        for c2 in range(nB):
            G[kb + c, kb + c2] = float(np.sum(Q[c] * Q[c2]))
        h[kb + c] = float(np.sum(Q[c] * Sp))
    return G, h


@dataclass
class SolveInfo:
    status: str            # "ok" or "not_spd"
    failed_pivot: int      # 0-based failing pivot (-1 when ok)
    refine_iters: int
    backward_err: float    # ||h - G theta||_inf / (||G||_inf ||theta||_inf + ||h||_inf)
    cond_est: float        # 2-norm condition number of the equilibrated G


def solve_cholesky64(G, h, refine: int = 2, cond: bool = False):
    """theta = G^-1 h: equilibrate (D = diag(G)^-1/2), Cholesky factor the
    equilibrated matrix, two triangular solves, then `refine` steps of
    iterative refinement with the residual h - G theta in FP64.
    Returns (theta, SolveInfo); theta is None when G is not positive definite."""
    G = np.asarray(G, dtype=np.float64)
    h = np.asarray(h, dtype=np.float64)
    dg = np.diag(G).copy()
    bad = np.where(~(dg > 0) | ~np.isfinite(dg))[0]
    if bad.size:
        return None, SolveInfo("not_spd", int(bad[0]), 0, np.inf, np.inf)
    s = 1.0 / np.sqrt(dg)
    Gt = G * s[:, None] * s[None, :]
    try:
        cf = scipy.linalg.cho_factor(Gt, lower=True, check_finite=True)
    except np.linalg.LinAlgError as e:
        m = re.search(r"(\d+)", str(e))
        piv = int(m.group(1)) - 1 if m else -1
        return None, SolveInfo("not_spd", piv, 0, np.inf, np.inf)
    x = scipy.linalg.cho_solve(cf, h * s)
    for _ in range(refine):
        rres = h * s - Gt @ x
        x = x + scipy.linalg.cho_solve(cf, rres)
    theta = x * s
    res = h - G @ theta
    berr = float(np.max(np.abs(res)) /
                 (np.max(np.sum(np.abs(G), axis=1)) * np.max(np.abs(theta)) + np.max(np.abs(h))))
    kappa = float(np.linalg.cond(Gt)) if cond else float("nan")
    return theta, SolveInfo("ok", -1, refine, berr, kappa)


# ---------------------------------------------------------------------------
# convolve-and-subtract, chi2 judge
# ---------------------------------------------------------------------------


def model_image(R, theta, L, DK, DB, ref_pedestal=0.0) -> np.ndarray:
    """M_theta(x) by direct summation over the L*L taps and the monomials."""
    Rp, _ = _prep(R, None, ref_pedestal, 0.0)
    H, W = Rp.shape
    a, b = split_theta(theta, L, DK, DB)
    P = poly_images(W, H, DK) * Rp
    M = np.zeros((H, W))
    r = (L - 1) // 2
    for i in range(P.shape[0]):
        for dy in range(-r, r + 1):
            for dx in range(-r, r + 1):
                c = a[i, dy + r, dx + r]
                if c != 0.0:
                    M += c * np.roll(P[i], shift=(dy, dx), axis=(0, 1))
    Q = poly_images(W, H, DB)
    for c in range(Q.shape[0]):
        M += b[c] * Q[c]
    return M


def subtract64(R, S, theta, L, DK, DB, ref_pedestal=0.0, sci_pedestal=0.0) -> np.ndarray:
    """Difference image D = S' - M_theta."""
    Sp = np.asarray(S, dtype=np.float64) - sci_pedestal
    return Sp - model_image(R, theta, L, DK, DB, ref_pedestal)


def model_image_conv(R, theta, L, DK, DB, ref_pedestal=0.0) -> np.ndarray:
    """M_theta(x) as one periodic 2-D convolution per monomial:
    M = sum_i k_i * P_i + sum_c b_c q_c, P_i = p_i R', k_i[dy, dx] =
    a_(i,(dy,dx)), (k * P)(x) = sum_delta k(delta) P(x - delta) with indices
    modulo the image. scipy.ndimage.convolve (mode "wrap", centred odd
    kernel) is that sum; it serves full-size images, where the tap-by-tap
    roll of model_image takes a minute."""
    import scipy.ndimage
    Rp, _ = _prep(R, None, ref_pedestal, 0.0)
    H, W = Rp.shape
    a, b = split_theta(theta, L, DK, DB)
    P = poly_images(W, H, DK) * Rp
    M = np.zeros((H, W))
    for i in range(P.shape[0]):
        M += scipy.ndimage.convolve(P[i], a[i], mode="wrap")
    Q = poly_images(W, H, DB)
    for c in range(Q.shape[0]):
        M += b[c] * Q[c]
    return M


def subtract_conv64(R, S, theta, L, DK, DB, ref_pedestal=0.0, sci_pedestal=0.0) -> np.ndarray:
    """D = S' - M_theta with the model from model_image_conv."""
    Sp = np.asarray(S, dtype=np.float64) - sci_pedestal
    return Sp - model_image_conv(R, theta, L, DK, DB, ref_pedestal)


def kernel_sums(theta, L, DK, DB=0) -> np.ndarray:
    """kappa_i = sum_delta a_(i,delta): the flux-ratio polynomial."""
    a, _ = split_theta(theta, L, DK, DB)
    return a.reshape(a.shape[0], -1).sum(axis=1)


def variance_image(R, S, theta, L, DK, DB) -> np.ndarray:
    """V(x) = max(S(x), 1) + kappa2(x) max(R(x), 1) with kappa2(x) =
    sum_delta (sum_i a_(i,delta) p_i(x))^2: Poisson variance (gain 1) of S
    plus that of the convolved reference, on raw (pedestal-free) images."""
    R = np.asarray(R, dtype=np.float64)
    S = np.asarray(S, dtype=np.float64)
    H, W = R.shape
    a, _ = split_theta(theta, L, DK, DB)
    A = a.reshape(a.shape[0], -1)
    Qm = A @ A.T
    mono = poly_images(W, H, DK)
    k2 = np.einsum("ij,ihw,jhw->hw", Qm, mono, mono)
    return np.maximum(S, 1.0) + k2 * np.maximum(R, 1.0)


def chi2_nu(R, S, D, theta, L, DK, DB) -> float:
    """Reduced chi^2 of D over the image minus an r-pixel frame,
    dof = |Omega| - N."""
    H, W = np.asarray(R).shape
    r = (L - 1) // 2
    V = variance_image(R, S, theta, L, DK, DB)
    Dm = np.asarray(D, dtype=np.float64)[r:H - r, r:W - r]
    Vm = V[r:H - r, r:W - r]
    dof = Dm.size - n_unknowns(L, DK, DB)
    return float(np.sum(Dm * Dm / Vm) / dof)


# ---------------------------------------------------------------------------
# one-call path
# ---------------------------------------------------------------------------


def difference(R, S, L, DK, DB, ref_pedestal=0.0, sci_pedestal=0.0, refine=2):
    """Build (O2) + solve + subtract + chi2. Returns dict."""
    G, h = build_fft64(R, S, L, DK, DB, ref_pedestal, sci_pedestal)
    theta, info = solve_cholesky64(G, h, refine)
    out = dict(G=G, h=h, theta=theta, info=info)
    if theta is not None:
        D = subtract64(R, S, theta, L, DK, DB, ref_pedestal, sci_pedestal)
        out["D"] = D
        out["chi2"] = chi2_nu(R, S, D, theta, L, DK, DB)
    return out


def model_at(R, theta, L, DK, DB, ys, xs, ref_pedestal=0.0) -> np.ndarray:
    """M_theta at the listed pixels only, by direct summation (for sampled
    checks of full-size images)."""
    R = np.asarray(R)
    H, W = R.shape
    a, b = split_theta(theta, L, DK, DB)
    r = (L - 1) // 2
    xt, yt = norm_coord(W), norm_coord(H)
    out = np.zeros(len(ys))
    for n, (y, x) in enumerate(zip(ys, xs)):
        m = 0.0
        for dy in range(-r, r + 1):
            uy = (y - dy) % H
            for dx in range(-r, r + 1):
                ux = (x - dx) % W
                rv = float(R[uy, ux]) - ref_pedestal
                for i, (ea, eb) in enumerate(monomials(DK)):
                    m += a[i, dy + r, dx + r] * xt[ux] ** ea * yt[uy] ** eb * rv
        for c, (ea, eb) in enumerate(monomials(DB)):
            m += b[c] * xt[x] ** ea * yt[y] ** eb
        out[n] = m
    return out


def normal_entry(R, L, DK, row, col, ref_pedestal=0.0) -> float:
    """One kernel-kernel normal-matrix entry by a direct periodic sum:
    G[(i,d),(j,d')] = sum_x P_i(x - d) P_j(x - d')."""
    Rp = np.asarray(R, dtype=np.float64) - ref_pedestal
    H, W = Rp.shape
    L2 = L * L
    r = (L - 1) // 2
    mons = monomials(DK)
    xt, yt = norm_coord(W)[None, :], norm_coord(H)[:, None]
    i, d = divmod(row, L2)
    j, d2 = divmod(col, L2)
    Pi = xt ** mons[i][0] * yt ** mons[i][1] * Rp
    Pj = xt ** mons[j][0] * yt ** mons[j][1] * Rp
    a = np.roll(Pi, shift=(d // L - r, d % L - r), axis=(0, 1))
    b = np.roll(Pj, shift=(d2 // L - r, d2 % L - r), axis=(0, 1))
    return float(np.sum(a * b))


# ---------------------------------------------------------------------------
# O3: the least-squares problem restricted to star stamps (precision form)
# ---------------------------------------------------------------------------
# The same design matrix as O1, keeping only the rows of pixels that lie in
# square stamps of side `size` centred on the given pixels (periodic
# indexing). Its normal equations are the Gram sums G_s = A_s^T A_s,
# h_s = A_s^T S'_s. The precision form evaluates these sums on matrix cores
# with each FP32 operand split into bfloat16 terms; stamp_normal_split gives
# the exact value of that split-product sum (before any FP32 accumulation
# rounding), and bf16_rne / split_bf16 / split_bf16_3 define the splits.


def stamp_pixels(W: int, H: int, centers, size: int):
    """(ys, xs) of every stamp pixel: stamps in the given order, row-major
    inside a stamp, coordinates wrapped into the image."""
    centers = np.asarray(centers, dtype=np.int64).reshape(-1, 2)
    h = size // 2
    off = np.arange(size) - h
    ys = (centers[:, 1, None, None] + off[None, :, None]) % H
    xs = (centers[:, 0, None, None] + off[None, None, :]) % W
    ys, xs = np.broadcast_arrays(ys, xs)
    return ys.reshape(-1), xs.reshape(-1)


def stamp_design(R, centers, size, L, DK, DB, ref_pedestal=0.0) -> np.ndarray:
    """A_s: rows of the design matrix at the stamp pixels. Column (i, delta)
    holds p_i(u) R'(u) at u = x - delta; column c holds q_c(x)."""
    Rp, _ = _prep(R, None, ref_pedestal, 0.0)
    H, W = Rp.shape
    ys, xs = stamp_pixels(W, H, centers, size)
    P = poly_images(W, H, DK) * Rp
    Q = poly_images(W, H, DB)
    cols = []
    for i in range(P.shape[0]):
        for dy, dx in zip(*kernel_offsets(L)):
            cols.append(P[i][(ys - dy) % H, (xs - dx) % W])
    for c in range(Q.shape[0]):
        cols.append(Q[c][ys, xs])
    return np.stack(cols, axis=1)


def stamp_normal64(R, S, centers, size, L, DK, DB, ref_pedestal=0.0, sci_pedestal=0.0):
    """Exact FP64 stamp normal equations (G_s, h_s)."""
    A = stamp_design(R, centers, size, L, DK, DB, ref_pedestal)
    _, Sp = _prep(R, S, ref_pedestal, sci_pedestal)
    ys, xs = stamp_pixels(Sp.shape[1], Sp.shape[0], centers, size)
    s = Sp[ys, xs]
    return A.T @ A, A.T @ s


def bf16_rne(x) -> np.ndarray:
    """Round FP32 values to bfloat16 (8 significant bits), ties to even;
    returned as float32. Finite inputs only."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def split_bf16(a):
    """a (FP32) = hi + lo + e with hi = bf16(a), lo = bf16(a - hi) (a - hi is
    exact in FP32); |e| <= 2^-16 |a|."""
    a = np.asarray(a, dtype=np.float32)
    hi = bf16_rne(a)
    lo = bf16_rne(a - hi)
    return hi, lo


def split_bf16_3(a):
    """a (FP32) = hi + mid + lo with hi = bf16(a), mid = bf16(a - hi),
    lo = bf16(a - hi - mid). Both differences are exact in FP32, and the
    decomposition itself is exact whenever |a| >= 2^-100: a - hi is a whole
    number of units in the last place of a below 2^15, a - hi - mid one below
    2^7, which 8 significant bits hold."""
    a = np.asarray(a, dtype=np.float32)
    hi = bf16_rne(a)
    r1 = a - hi
    mid = bf16_rne(r1)
    lo = bf16_rne(r1 - mid)
    return hi, mid, lo


def split_product_terms(terms: int):
    """Index pairs (s, t) of the split terms kept in a product a*b: with two
    terms per operand (hi, lo) hi*hi + hi*lo + lo*hi; with three
    (hi, mid, lo) every pair of total order s + t <= 2: hi*hi, hi*mid,
    mid*hi, hi*lo, lo*hi, mid*mid."""
    if terms == 2:
        return [(0, 0), (0, 1), (1, 0)]
    if terms == 3:
        return [(0, 0), (0, 1), (1, 0), (0, 2), (2, 0), (1, 1)]
    raise ValueError("terms must be 2 or 3")


def stamp_normal_split(R, S, centers, size, L, DK, DB, ref_pedestal=0.0, sci_pedestal=0.0, terms=3):
    """The Gram sums the split-product form computes, evaluated exactly:
    every design value and stamp value is first rounded to FP32, split into
    `terms` bfloat16 terms, and each product a*b is replaced by the term
    products of split_product_terms; all sums in FP64 (exact products).
    Returns (G, h)."""
    A = stamp_design(R, centers, size, L, DK, DB, ref_pedestal).astype(np.float32)
    _, Sp = _prep(R, S, ref_pedestal, sci_pedestal)
    ys, xs = stamp_pixels(Sp.shape[1], Sp.shape[0], centers, size)
    s = Sp[ys, xs].astype(np.float32)
    split = split_bf16 if terms == 2 else split_bf16_3
    As = [t.astype(np.float64) for t in split(A)]
    ss = [t.astype(np.float64) for t in split(s)]
    G = np.zeros((A.shape[1], A.shape[1]))
    h = np.zeros(A.shape[1])
    for p, q in split_product_terms(terms):
        G += As[p].T @ As[q]
        h += As[p].T @ ss[q]
    return G, h


def stamp_abs_gram(R, S, centers, size, L, DK, DB, ref_pedestal=0.0, sci_pedestal=0.0):
    """|A_s|^T |A_s| and |A_s|^T |S'_s|: the scale of each Gram entry's
    rounding-error bound."""
    A = np.abs(stamp_design(R, centers, size, L, DK, DB, ref_pedestal))
    _, Sp = _prep(R, S, ref_pedestal, sci_pedestal)
    ys, xs = stamp_pixels(Sp.shape[1], Sp.shape[0], centers, size)
    return A.T @ A, A.T @ np.abs(Sp[ys, xs])
