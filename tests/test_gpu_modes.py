"""GPU parity of the two optional fit modes through the C ABI against the
brute-force oracle (oracle/modes.py): the masked fit (R' and S' zero outside
a star-stamp mask) and the output-pixel kernel convention (the polynomial
evaluated at the output pixel; R' zero on the r-pixel frame), alone and
together, and at full size the orthogonality of the output-pixel residual to
sampled design columns.

Tolerances: normal matrix and right-hand side 1e-11 relative to their
largest entry (FP64 FFT build against explicit sums); kernel coefficients
1e-5 relative (FP64 form); difference image 1e-3 of the sky noise; chi2
1e-6 relative."""
import numpy as np
import pytest
import scipy.ndimage

import oracle as O
from oracle import modes as M
import synth

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _env():
    import torch
    import paper_2603_08593_amd as sf
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    sf.lib()
    return torch, sf


def _sigma_sky(D, r):
    H, W = D.shape
    Dm = D[r:H - r, r:W - r]
    return 1.4826 * float(np.median(np.abs(Dm - np.median(Dm))))


def _stamp_mask(p, W, H, size, n):
    # squares of side `size` around the n brightest stars whose square lies
    # inside the image (overlaps allowed): the star-stamp mask of a sparse field
    h = size // 2
    xs, ys, fl = p.meta["xs"], p.meta["ys"], p.meta["flux"]
    m = np.zeros((H, W), dtype=np.uint8)
    k = 0
    for j in np.argsort(-fl, kind="stable"):
        cx, cy = int(np.rint(xs[j])), int(np.rint(ys[j]))
        if h <= cx < W - h and h <= cy < H - h:
            m[cy - h:cy + h + 1, cx - h:cx + h + 1] = 1
            k += 1
            if k == n:
                break
    return m, k


CASES = [
    # W, H, L, DK, DB, masked, outpix, dtype
    (64, 48, 5, 2, 1, True, False, np.float64),
    (96, 64, 7, 1, 2, True, False, np.float32),
    (64, 48, 5, 2, 1, False, True, np.float64),
    (80, 60, 5, 1, 1, False, True, np.float32),
    (72, 54, 5, 2, 2, True, True, np.float64),
    (64, 40, 3, 0, 1, False, True, np.float64),     # DK = 0: the conventions coincide (frame aside)
]


@pytest.mark.parametrize("W,H,L,DK,DB,masked,outpix,dtype", CASES)
def test_mode_matches_bruteforce(W, H, L, DK, DB, masked, outpix, dtype):
    torch, sf = _env()
    p = synth.make_pair(W, H, L, DK, DB, seed=synth.seed_for(7, W * 7 + H + L), nstars=max(12, W * H // 250),
                        dtype=dtype)
    mask = None
    if masked:
        mask, ns = _stamp_mask(p, W, H, 13, 12)
        assert ns >= 4
    tag = f"{W}x{H} L={L} DK={DK} DB={DB} masked={masked} outpix={outpix} {np.dtype(dtype).name}"
    _say(f"fit mode {tag}")
    Gr, hr = M.normal_ex(p.R, p.S, L, DK, DB, mask=mask, outpix=outpix)
    th_r = M.solve_ex(p.R, p.S, L, DK, DB, mask=mask, outpix=outpix)
    D_r = M.subtract_ex(p.R, p.S, th_r, L, DK, DB, outpix=outpix)
    chi_r = O.chi2_nu(p.R, p.S, D_r, th_r, L, DK, DB)
    d = sf.Differencer(W, H, L, DK, DB, image_dtype="float32" if dtype == np.float32 else "float64",
                       convention="output" if outpix else "input")
    try:
        R = torch.from_numpy(p.R).cuda()
        S = torch.from_numpy(p.S).cuda()
        md = None if mask is None else torch.from_numpy(mask).cuda()
        d.run(R, S, max_refine=2, mask=md)
        torch.cuda.synchronize()
        info = d.info()
        assert info.status == 0, info.status
        G, h = d.buf.G.cpu().numpy(), d.buf.h.cpu().numpy()
        th = d.buf.coef.cpu().numpy()
        D = d.buf.diff.cpu().numpy().astype(np.float64)
        chi = float(d.buf.chi2.item())
    finally:
        d.close()
    gerr = np.max(np.abs(G - Gr)) / np.max(np.abs(Gr))
    herr = np.max(np.abs(h - hr)) / np.max(np.abs(hr))
    nk = O.n_mono(DK) * L * L
    cerr = np.linalg.norm(th[:nk] - th_r[:nk]) / np.linalg.norm(th_r[:nk])
    sig = _sigma_sky(D_r, (L - 1) // 2)
    drms = float(np.sqrt(np.mean((D - D_r) ** 2)))
    _say(f"  G {gerr:.1e}  h {herr:.1e}  coef {cerr:.1e}  D rms/sigma {drms / sig:.1e}  chi2 {chi:.6f} "
         f"(oracle {chi_r:.6f})")
    assert gerr <= 1e-11 and herr <= 1e-11
    assert cerr <= 1e-5
    assert drms <= 1e-3 * sig
    assert abs(chi - chi_r) <= 1e-6 * chi_r


def test_modes_rejected_where_unsupported():
    torch, sf = _env()
    lib = sf.lib()
    h = sf.Handle()
    try:
        d = sf.make_desc(128, 128, 5, 2, 1, convention=sf.SFFT_CONV_OUTPUT_PIXEL)
        n = sf.ctypes.c_size_t()
        assert lib.sfft_stamps_workspace_size(h.ptr, d, 4, 21, sf.ctypes.byref(n)) == sf.SFFT_ERR_UNSUPPORTED
        bad = sf.make_desc(128, 128, 5, 2, 1, convention=2)
        assert sf.sfft_validate(bad) == sf.SFFT_ERR_INVALID_ARG
    finally:
        h.close()


def test_outpix_full_size_residual_orthogonal_to_design():
    # 2048 x 4096, L = 11, DK = DB = 2 in the output-pixel convention: the
    # residual of the fitted model (recomputed in FP64 from the GPU
    # coefficients) is orthogonal to sampled columns of the output-pixel
    # design, p_i(x) R'_f(x - d) with R'_f zero on the r-pixel frame
    # The fit drops the reference's frame, so the sky is taken out first
    # (image-mean pedestals), as for any masked fit: with the raw sky of
    # ~1000 ADU the missing frame leaves a sky-sized hole in the model beside
    # the edges and the fit is pulled by it (chi2 ~2.9 on a 256 x 256 crop,
    # 1.01 with pedestals, oracle on the CPU)
    torch, sf = _env()
    p = synth.make_cfg2()
    W, H, L, DK, DB = 2048, 4096, 11, 2, 2
    r = (L - 1) // 2
    cR = float(np.mean(p.R, dtype=np.float64))
    cS = float(np.mean(p.S, dtype=np.float64))
    _say("output-pixel convention, 2048x4096 L=11 DK=2 DB=2, image-mean pedestals: residual orthogonality")
    d = sf.Differencer(W, H, L, DK, DB, convention="output", ref_pedestal=cR, sci_pedestal=cS)
    try:
        R = torch.from_numpy(p.R).cuda()
        S = torch.from_numpy(p.S).cuda()
        d.run(R, S, max_refine=1)
        torch.cuda.synchronize()
        assert d.info().status == 0
        th = d.buf.coef.cpu().numpy()
        chi = float(d.buf.chi2.item())
    finally:
        d.close()
    Rf = (p.R.astype(np.float64) - cR) * M.frame_mask(W, H, r)
    a, b = O.split_theta(th, L, DK, DB)
    mono = O.poly_images(W, H, DK)
    model = np.zeros((H, W))
    for i in range(mono.shape[0]):
        model += mono[i] * scipy.ndimage.convolve(Rf, a[i], mode="wrap")
    Q = O.poly_images(W, H, DB)
    for c in range(Q.shape[0]):
        model += b[c] * Q[c]
    e = (p.S.astype(np.float64) - cS) - model
    rng = np.random.default_rng(11)
    worst = 0.0
    N = O.n_unknowns(L, DK, DB)
    cols = list(rng.choice(O.n_mono(DK) * L * L, size=24, replace=False)) + list(range(O.n_mono(DK) * L * L, N))
    for j in cols:
        if j < O.n_mono(DK) * L * L:
            i, dd = divmod(int(j), L * L)
            dy, dx = dd // L - r, dd % L - r
            col = mono[i] * np.roll(Rf, shift=(dy, dx), axis=(0, 1))
        else:
            col = Q[j - O.n_mono(DK) * L * L]
        v = abs(float(np.sum(col * e))) / (np.linalg.norm(col) * np.linalg.norm(e))
        worst = max(worst, v)
    _say(f"  max |A_j^T e| / (|A_j| |e|) over {len(cols)} columns: {worst:.2e}; chi2 {chi:.5f}")
    assert worst <= 1e-10
    assert chi <= 1.05
