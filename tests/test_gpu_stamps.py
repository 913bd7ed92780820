"""GPU parity of the stamp Gram (precision form: every FP32 operand split
into three bfloat16 terms, the six term products of order <= 2 on matrix
cores) against the stamp oracle.

Bounds, per Gram entry, relative to the sum of absolute products
(|A|^T |A|): the split itself is evaluated exactly by the oracle
(stamp_normal_split, terms=3), so the GPU may differ from it only by FP32
accumulation, which runs over at most 8 chunks of 6 products each before it
is flushed into FP64: at most 48 + 32 roundings of 2^-24 each per run, and
each run's error is bounded by its own share of |A|^T |A|. Against the exact
FP64 Gram add the dropped term products (2^-23) and the FP32 rounding of both
operands (2 x 2^-24)."""
import numpy as np
import pytest

import oracle as O
import synth

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    return torch


def _sf():
    import paper_2603_08593_amd as sf
    sf.lib()
    return sf


def _say(msg):
    print(msg, flush=True)


FLUSH_CHUNKS = 8          # chunks of FP32 accumulation before each FP64 flush
PRODUCTS = 6              # term products per operand pair


def _acc_bound():
    return (PRODUCTS * FLUSH_CHUNKS + 32) * 2.0 ** -24


def _run(p, centers, size, refine=2, subtract=False, peds=(0.0, 0.0)):
    torch, sf = _torch(), _sf()
    H, W = p.R.shape
    dt = "float32" if p.R.dtype == np.float32 else "float64"
    d = sf.Differencer(W, H, p.L, p.DK, p.DB, image_dtype=dt, stamps=(len(centers), size),
                       ref_pedestal=peds[0], sci_pedestal=peds[1])
    R = torch.from_numpy(p.R).cuda()
    S = torch.from_numpy(p.S).cuda()
    c = torch.from_numpy(np.ascontiguousarray(centers, dtype=np.int32)).cuda()
    d.build_stamps(R, S, c, size)
    d.solve(max_refine=refine)
    if subtract:
        d.subtract(R, S)
    torch.cuda.synchronize()
    return dict(G=d.buf.G.cpu().numpy(), h=d.buf.h.cpu().numpy(), theta=d.buf.coef.cpu().numpy(),
                D=d.buf.diff.cpu().numpy().astype(np.float64) if subtract else None,
                chi2=float(d.buf.chi2.item()), info=d.info(), d=d, R=R, S=S, c=c)


def _check_gram(p, centers, size, g, peds=(0.0, 0.0)):
    L, DK, DB = p.L, p.DK, p.DB
    Gs, hs = O.stamp_normal_split(p.R, p.S, centers, size, L, DK, DB, *peds, terms=3)
    Ga, ha = O.stamp_abs_gram(p.R, p.S, centers, size, L, DK, DB, *peds)
    G64, h64 = O.stamp_normal64(p.R, p.S, centers, size, L, DK, DB, *peds)
    tol = _acc_bound()
    eg = np.max(np.abs(g["G"] - Gs) / np.maximum(Ga, 1e-300))
    eh = np.max(np.abs(g["h"] - hs) / np.maximum(ha, 1e-300))
    eg64 = np.max(np.abs(g["G"] - G64) / np.maximum(Ga, 1e-300))
    _say(f"  |G - G_split|/|A|'|A| max {eg:.2e}, h {eh:.2e} (bound {tol:.1e}); "
         f"vs exact FP64 {eg64:.2e}")
    assert eg <= tol and eh <= tol
    assert eg64 <= tol + 2.0 ** -23 + 2 * 2.0 ** -24
    assert np.array_equal(g["G"], g["G"].T)
    return G64, h64


@pytest.mark.parametrize("W,H,L,DK,DB,size,n,dtype", [
    (160, 128, 5, 2, 1, 21, 10, np.float32),     # several tiles, planes per tile vary
    (96, 64, 3, 0, 0, 9, 3, np.float64),         # one tile, FP64 images
    (210, 150, 7, 1, 2, 15, 7, np.float32),      # W = 2 3 5 7: no FFT, so any width
    (64, 64, 1, 0, 1, 1, 40, np.float32),        # single-pixel stamps, single tap
])
def test_stamp_gram_small(W, H, L, DK, DB, size, n, dtype):
    p = synth.make_pair(W, H, L, DK, DB, seed=500 + W + size, nstars=max(8, W * H // 1500),
                        psf="moffat", fwhm=3.0, fwhm_end=4.5, flux=(1e2, 1e5), dtype=dtype)
    rng = np.random.default_rng(W + H + size)
    c = np.stack([rng.integers(0, W, n), rng.integers(0, H, n)], axis=1).astype(np.int32)
    c[0] = (0, 0)                     # wraps over all four corners
    if n > 1:
        c[1] = (W - 1, H // 2)        # wraps over the right edge
    _say(f"stamps {W}x{H} L={L} DK={DK} DB={DB} size={size} n={n} {np.dtype(dtype).name}")
    g = _run(p, c, size)
    _check_gram(p, c, size, g)


def test_stamp_solve_cfg2_full_size():
    """64 stamps of 41 x 41 on the 2048 x 4096 CCD pair with the FP64 image
    means as pedestals (the precision form's reading: the sky level stays
    out of the bfloat16 split): Gram parity, and the model image of the GPU
    stamp fit within 1e-3 of the sky noise of the oracle's exact FP64 stamp
    fit with the same pedestals (the bound every GPU form meets). The fit
    must pass the chi2 judge (<= 1.05)."""
    p = synth.make_cfg2()
    c = synth.pick_stamps(p, 64, 41)
    assert len(c) == 64
    L, DK, DB = p.L, p.DK, p.DB
    peds = (float(np.mean(p.R, dtype=np.float64)), float(np.mean(p.S, dtype=np.float64)))
    _say(f"cfg2 stamps: 64 x 41^2, L=11 DK=2 DB=2, pedestals {peds[0]:.3f} {peds[1]:.3f}")
    g = _run(p, c, 41, subtract=True, peds=peds)
    assert g["info"].status == 0
    G64, h64 = _check_gram(p, c, 41, g, peds)
    t64, info = O.solve_cholesky64(G64, h64, refine=2, cond=True)
    G0, _ = O.stamp_normal64(p.R, p.S, c, 41, L, DK, DB)
    s0 = 1.0 / np.sqrt(np.diag(G0))
    cond0 = float(np.linalg.cond(G0 * s0[:, None] * s0[None, :]))
    rng = np.random.default_rng(2)
    H, W = p.R.shape
    ys, xs = rng.integers(0, H, 1500), rng.integers(0, W, 1500)
    m_gpu = O.model_at(p.R, g["theta"], L, DK, DB, ys, xs, ref_pedestal=peds[0])
    m64 = O.model_at(p.R, t64, L, DK, DB, ys, xs, ref_pedestal=peds[0])
    sig = np.sqrt(np.median(p.S))          # Poisson sky noise, gain 1
    d64 = float(np.sqrt(np.mean((m_gpu - m64) ** 2)) / sig)
    nk = O.n_mono(DK) * L * L
    err64 = np.linalg.norm(g["theta"][:nk] - t64[:nk]) / np.linalg.norm(t64[:nk])
    _say(f"  precision-form error vs FP64 stamp fit: model {d64:.2e} sigma, coef {err64:.2e}; "
         f"cond of the equilibrated stamp system {info.cond_est:.2e} with pedestals, {cond0:.2e} "
         f"without; chi2 of the stamp fit {g['chi2']:.4f}")
    assert d64 <= 1e-3
    assert 0.5 < g["chi2"] <= 1.05


def test_stamp_nonfinite_flag():
    torch, sf = _torch(), _sf()
    p = synth.make_pair(64, 64, 3, 0, 0, seed=9, nstars=10, dtype=np.float32)
    R = p.R.copy()
    R[20, 20] = np.nan
    p = synth.Pair(R=R, S=p.S, L=p.L, DK=p.DK, DB=p.DB, a=p.a, b=p.b, R_model=p.R_model,
                   S_model=p.S_model, meta=p.meta)
    g = _run(p, np.array([[20, 20]], dtype=np.int32), 9)
    assert g["info"].status == 4      # SFFT_ERR_NONFINITE


def test_stamp_bad_arguments():
    torch, sf = _torch(), _sf()
    d = sf.Differencer(64, 64, 3, 0, 0, stamps=(2, 9))
    R = torch.zeros((64, 64), dtype=torch.float32, device="cuda")
    c = torch.zeros((2, 2), dtype=torch.int32, device="cuda")
    for size in (8, 0, 129, 65):
        with pytest.raises(sf.SfftError) as e:
            d.build_stamps(R, R, c, size)
        assert e.value.status == sf.SFFT_ERR_INVALID_ARG
    with pytest.raises(sf.SfftError) as e:
        d.build_stamps(R, R, c[:0], 9)
    assert e.value.status == sf.SFFT_ERR_INVALID_ARG
