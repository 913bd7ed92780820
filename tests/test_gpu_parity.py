"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle on
the same seeded inputs. Tolerances: kernel coefficients relative error
<= 1e-5 (FP64-internal build), difference image RMS deviation <= 1e-3 of the
sky noise (1.4826 MAD of the oracle's D over the frame interior)."""
import numpy as np
import pytest

import oracle as O
import synth

pytestmark = pytest.mark.gpu

COEF_TOL = 1e-5
DRMS_TOL = 1e-3


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    return torch


def _sf():
    import paper_2603_08593_amd as sf
    sf.lib()      # fails loudly when the HIP library is missing
    return sf


def _say(msg):
    print(msg, flush=True)


def _sigma_sky(D, r):
    H, W = D.shape
    Dm = D[r:H - r, r:W - r]
    return 1.4826 * float(np.median(np.abs(Dm - np.median(Dm))))


def _run_gpu(p, compute="fp64", peds=(0.0, 0.0), refine=2, radix_order=0):
    torch = _torch()
    sf = _sf()
    H, W = p.R.shape
    dt = "float32" if p.R.dtype == np.float32 else "float64"
    d = sf.Differencer(W, H, p.L, p.DK, p.DB, image_dtype=dt, compute=compute,
                       ref_pedestal=peds[0], sci_pedestal=peds[1], radix_order=radix_order)
    R = torch.from_numpy(p.R).cuda()
    S = torch.from_numpy(p.S).cuda()
    d.run(R, S, max_refine=refine)
    torch.cuda.synchronize()
    out = dict(G=d.buf.G.cpu().numpy(), h=d.buf.h.cpu().numpy(), theta=d.buf.coef.cpu().numpy(),
               D=d.buf.diff.cpu().numpy().astype(np.float64), chi2=float(d.buf.chi2.item()),
               info=d.info(), d=d, R=R, S=S)
    return out


def _compare(p, g, peds=(0.0, 0.0), coef_tol=COEF_TOL, check_G=True):
    L, DK, DB = p.L, p.DK, p.DB
    ref = O.difference(p.R, p.S, L, DK, DB, *peds)
    assert g["info"].status == 0, g["info"].status
    if check_G:
        gerr = np.max(np.abs(g["G"] - ref["G"])) / np.max(np.abs(ref["G"]))
        herr = np.max(np.abs(g["h"] - ref["h"])) / np.max(np.abs(ref["h"]))
        _say(f"  G rel err {gerr:.2e}  h rel err {herr:.2e}")
        assert gerr <= 1e-11 and herr <= 1e-11
    nk = O.n_mono(DK) * L * L
    cerr = np.linalg.norm(g["theta"][:nk] - ref["theta"][:nk]) / np.linalg.norm(ref["theta"][:nk])
    sig = _sigma_sky(ref["D"], (L - 1) // 2)
    drms = float(np.sqrt(np.mean((g["D"] - ref["D"]) ** 2)))
    _say(f"  coef rel err {cerr:.2e}  D rms/sigma {drms / sig:.2e}  chi2 {g['chi2']:.6f} "
         f"(oracle {ref['chi2']:.6f})  berr {g['info'].backward_err:.1e}")
    assert cerr <= coef_tol
    assert drms <= DRMS_TOL * sig
    assert abs(g["chi2"] - ref["chi2"]) <= 1e-6 * ref["chi2"] + 1e-9
    return ref


def test_cfg1_full_path():
    p = synth.make_cfg1()
    _say("cfg1 256x256 FP64 L=7 DK=0 DB=1")
    _compare(p, _run_gpu(p))


@pytest.mark.parametrize("W,H,L,DK,DB,dtype", [
    (256, 512, 11, 2, 2, np.float32),     # several column groups, 5 row blocks (ragged)
    (64, 200, 7, 1, 2, np.float64),       # ragged rows, DK = 1
    (32, 40, 15, 0, 2, np.float64),       # H < block: halo wraps the image
    (128, 64, 1, 0, 0, np.float32),       # single tap, constant background
    (16, 48, 3, 0, 2, np.float64),        # smallest width
    (512, 128, 9, 2, 1, np.float32),
    (96, 80, 5, 1, 1, np.float64),        # W = 2^5 3: radix-3 row FFT
    (160, 120, 7, 2, 2, np.float32),      # W = 2^5 5: radix-5 row FFT
    (1500, 40, 3, 1, 1, np.float32),      # W = 2^2 3 5^3: 6 row elements per thread
    (768, 256, 15, 2, 2, np.float32),     # L = 15, DK = 2 (N = 1356)
])
def test_small_shapes(W, H, L, DK, DB, dtype):
    p = synth.make_pair(W, H, L, DK, DB, seed=1000 + W + H + L, nstars=max(8, W * H // 2000),
                        psf="moffat", fwhm=3.5, fwhm_end=5.0, flux=(1e2, 1e6), dtype=dtype)
    _say(f"shape {W}x{H} L={L} DK={DK} DB={DB} {np.dtype(dtype).name}")
    _compare(p, _run_gpu(p))


@pytest.mark.parametrize("W,H,L,DK,DB,dtype", [
    (2048, 64, 7, 2, 2, np.float32),      # CCD width: stages 4, 8, 8, 8
    (1500, 40, 3, 1, 1, np.float32),      # 2^2 3 5^3: stages 5, 5, 5, 3, 4
    (96, 80, 5, 1, 1, np.float64),        # stages 3, 4, 8
    (160, 120, 7, 2, 2, np.float32),      # stages 5, 4, 8
])
def test_reversed_radix_order(W, H, L, DK, DB, dtype):
    """Row FFTs with their stages in reversed order (sfft_set_radix_order 1):
    the same oracle bounds as the default order, and G within rounding of
    the default order's G."""
    p = synth.make_pair(W, H, L, DK, DB, seed=2000 + W + H + L, nstars=max(8, W * H // 2000),
                        psf="moffat", fwhm=3.5, fwhm_end=5.0, flux=(1e2, 1e6), dtype=dtype)
    _say(f"reversed radix order: {W}x{H} L={L} DK={DK} DB={DB} {np.dtype(dtype).name}")
    g1 = _run_gpu(p, radix_order=1)
    assert g1["d"].handle is not None
    _compare(p, g1)
    g0 = _run_gpu(p)
    dg = np.max(np.abs(g1["G"] - g0["G"])) / np.max(np.abs(g0["G"]))
    _say(f"  G order 1 vs order 0: {dg:.1e} of max")
    assert dg <= 1e-13


def test_pedestals_fp64():
    p = synth.make_pair(128, 160, 7, 2, 2, seed=77, nstars=30, dtype=np.float32)
    peds = (float(np.mean(p.R.astype(np.float64))), float(np.mean(p.S.astype(np.float64))))
    _say(f"pedestals {peds}")
    _compare(p, _run_gpu(p, peds=peds), peds=peds)


def test_fp32_precision_form_difference_image():
    """FP32 spectra/products with FP32 accumulation, FP64 solve: held to the
    difference-image bound; the coefficient error is reported."""
    p = synth.make_pair(256, 256, 11, 2, 2, seed=78, nstars=60, psf="moffat", fwhm=3.5,
                        fwhm_end=5.0, flux=(1e2, 1e6), dtype=np.float32)
    peds = (float(np.mean(p.R.astype(np.float64))), float(np.mean(p.S.astype(np.float64))))
    g = _run_gpu(p, compute="fp32", peds=peds)
    ref = O.difference(p.R, p.S, 11, 2, 2, *peds)
    nk = 6 * 121
    cerr = np.linalg.norm(g["theta"][:nk] - ref["theta"][:nk]) / np.linalg.norm(ref["theta"][:nk])
    sig = _sigma_sky(ref["D"], 5)
    drms = float(np.sqrt(np.mean((g["D"] - ref["D"]) ** 2)))
    _say(f"fp32 form: coef rel err {cerr:.2e} (reported), D rms/sigma {drms / sig:.2e}")
    assert drms <= DRMS_TOL * sig


def test_subtract_alone_matches_oracle():
    torch = _torch()
    sf = _sf()
    W, H, L, DK, DB = 128, 64, 5, 2, 2
    rng = np.random.default_rng(5)
    R = rng.normal(1000, 30, (H, W))
    S = rng.normal(1000, 30, (H, W))
    theta = rng.normal(0, 0.05, O.n_unknowns(L, DK, DB))
    d = sf.Differencer(W, H, L, DK, DB, image_dtype="float64", ref_pedestal=12.5, sci_pedestal=-3.0)
    coef = torch.from_numpy(theta).cuda()
    d.subtract(torch.from_numpy(R).cuda(), torch.from_numpy(S).cuda(), coef=coef)
    torch.cuda.synchronize()
    D = d.buf.diff.cpu().numpy()
    Do = O.subtract64(R, S, theta, L, DK, DB, 12.5, -3.0)
    assert np.max(np.abs(D - Do)) <= 1e-9 * np.max(np.abs(Do))
    chi = O.chi2_nu(R, S, Do, theta, L, DK, DB)
    assert abs(d.buf.chi2.item() - chi) <= 1e-9 * chi


def test_deterministic_bitwise():
    p = synth.make_pair(128, 96, 7, 2, 2, seed=79, nstars=20, dtype=np.float32)
    a = _run_gpu(p)
    b = _run_gpu(p)
    assert np.array_equal(a["G"], b["G"]) and np.array_equal(a["D"], b["D"])
    assert a["chi2"] == b["chi2"]


def test_nonfinite_input_reported():
    p = synth.make_pair(64, 64, 5, 0, 1, seed=80, nstars=10, dtype=np.float64)
    p.R[10, 20] = np.nan
    g = _run_gpu(p)
    sf = _sf()
    assert g["info"].nonfinite != 0
    assert g["info"].status == sf.SFFT_ERR_NONFINITE


def test_constant_reference_not_spd():
    sf = _sf()
    p = synth.make_pair(64, 64, 3, 0, 0, seed=81, nstars=10, dtype=np.float64)
    p.R[:] = 5.0
    g = _run_gpu(p)
    assert g["info"].status == sf.SFFT_ERR_NOT_SPD
    assert g["info"].failed_pivot >= 0
    assert np.all(np.isnan(g["theta"]))


def test_bad_arguments_raise():
    torch = _torch()
    sf = _sf()
    d = sf.Differencer(64, 64, 5, 0, 0, image_dtype="float32")
    R = torch.zeros((64, 64), device="cuda")
    small_ws = d.buf.ws[:256]
    with pytest.raises(sf.SfftError) as e:
        sf.sfft_build_system(d.handle, d.desc, R, R, d.buf.G, d.buf.h, small_ws)
    assert e.value.status == sf.SFFT_ERR_WORKSPACE
    with pytest.raises(sf.SfftError) as e:
        sf.sfft_subtract(d.handle, d.desc, R, R, d.buf.coef, R, None, d.buf.ws)
    assert e.value.status == sf.SFFT_ERR_INVALID_ARG


def test_cfg2_full_size_sampled():
    """2048x4096 FP32, L=11, DK=2, DB=2 (N=732) in the benchmark's launch
    configuration: coefficients against the full FP64 oracle solve; sampled
    normal-matrix entries and difference pixels against direct sums; the
    residual's orthogonality to sampled design columns."""
    torch = _torch()
    sf = _sf()
    p = synth.make_cfg2()
    _say("cfg2 2048x4096 FP32 L=11 DK=2 DB=2 (sampled checks), max_refine=1")
    g = _run_gpu(p, refine=1)
    assert g["info"].status == 0
    G_o, h_o = O.build_fft64(p.R, p.S, 11, 2, 2)
    th_o, _ = O.solve_cholesky64(G_o, h_o)
    nk = 726
    cerr = np.linalg.norm(g["theta"][:nk] - th_o[:nk]) / np.linalg.norm(th_o[:nk])
    gerr = np.max(np.abs(g["G"] - G_o)) / np.max(np.abs(G_o))
    _say(f"  G rel err {gerr:.2e}  coef rel err {cerr:.2e}")
    assert gerr <= 1e-11 and cerr <= COEF_TOL
    rng = np.random.default_rng(3)
    for _ in range(6):
        row, col = rng.integers(0, nk, 2)
        e = O.normal_entry(p.R, 11, 2, int(row), int(col))
        assert abs(g["G"][row, col] - e) <= 1e-11 * np.max(np.abs(G_o))
    ys = rng.integers(0, 4096, 40)
    xs = rng.integers(0, 2048, 40)
    ys[:4] = [0, 4095, 3, 4090]
    xs[:4] = [0, 2047, 2040, 5]
    M = O.model_at(p.R, g["theta"], 11, 2, 2, ys, xs)
    Dref = p.S.astype(np.float64)[ys, xs] - M
    # FP32 output: compare at the output precision
    assert np.max(np.abs(g["D"][ys, xs] - Dref)) <= 2e-3
    # orthogonality with an FP64 difference image from the GPU coefficients
    d64 = sf.Differencer(2048, 4096, 11, 2, 2, image_dtype="float64")
    R64 = g["R"].double()
    S64 = g["S"].double()
    d64.subtract(R64, S64, coef=g["d"].buf.coef)
    torch.cuda.synchronize()
    D64 = d64.buf.diff.cpu().numpy()
    A_cols = []
    xt, yt = O.norm_coord(2048)[None, :], O.norm_coord(4096)[:, None]
    Rd = p.R.astype(np.float64)
    worst = 0.0
    for _ in range(4):
        col = int(rng.integers(0, nk))
        i, dd = divmod(col, 121)
        ea, eb = O.monomials(2)[i]
        P = np.roll(xt ** ea * yt ** eb * Rd, shift=(dd // 11 - 5, dd % 11 - 5), axis=(0, 1))
        v = abs(float(np.sum(P * D64))) / (np.linalg.norm(P) * np.linalg.norm(D64))
        worst = max(worst, v)
    _say(f"  orthogonality |a^T D|/(|a||D|) max {worst:.2e}")
    assert worst <= 1e-10


def test_refit_background_matches_oracle():
    """Least-squares background for a fixed (perturbed) kernel: GPU against
    b = G_bb^-1 (h_b - G_kb^T a) from the oracle's normal equations; and for
    the full fit's own kernel it returns the fit's background."""
    torch, sf = _torch(), _sf()
    p = synth.make_pair(256, 192, 7, 2, 2, seed=77, nstars=60, psf="moffat", fwhm=3.5,
                       fwhm_end=4.5, flux=(1e2, 1e6), dtype=np.float32)
    G, h = O.build_fft64(p.R, p.S, 7, 2, 2)
    th, _ = O.solve_cholesky64(G, h)
    nk = O.n_mono(2) * 49
    rng = np.random.default_rng(1)
    a = th[:nk] * (1 + 0.05 * rng.standard_normal(nk))
    want = np.linalg.solve(G[nk:, nk:], h[nk:] - G[nk:, :nk] @ a)
    d = sf.Differencer(256, 192, 7, 2, 2, image_dtype="float32")
    R, S = torch.from_numpy(p.R).cuda(), torch.from_numpy(p.S).cuda()
    coef = torch.from_numpy(np.concatenate([a, np.zeros(6)])).cuda()
    d.refit_background(R, S, coef=coef)
    torch.cuda.synchronize()
    got = coef.cpu().numpy()
    e = np.max(np.abs(got[nk:] - want)) / np.max(np.abs(want))
    _say(f"  refit background rel err {e:.2e}")
    assert e <= 1e-9
    assert np.array_equal(got[:nk], a)
    coef2 = torch.from_numpy(np.concatenate([th[:nk], np.zeros(6)])).cuda()
    d.refit_background(R, S, coef=coef2)
    torch.cuda.synchronize()
    assert np.max(np.abs(coef2.cpu().numpy()[nk:] - th[nk:])) <= 1e-8 * np.max(np.abs(th[nk:]))
