"""GPU parity of the difference-image products through the C ABI against the
FP64 CPU oracle (oracle/products.py): the zero-point-normalised median
combine, the whole multi-template path (each template's fit, difference
image and chi2, and the combined image), exact-overlap aperture fluxes, the
limiting magnitude and forced photometry.

Tolerances: the median of identical inputs is bit-exact (both sides scale in
FP64 and select the same middle value; the result is rounded once to the
image type); the multi-template fits meet the single-pair bounds (kernel
coefficients 1e-5 relative, difference image RMS 1e-3 of the sky noise, and
the median is 1-Lipschitz in the maximum norm, so the combined image meets
the same bound); aperture sums are FP64 sums of FP64 area weights (1e-11
relative to the sum of absolute terms), magnitudes 1e-11 absolute."""
import math

import numpy as np
import pytest

import synth
from oracle import products as P
import oracle as O

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


@pytest.mark.parametrize("n,W,H,dtype", [(5, 200, 72, np.float32), (1, 64, 8, np.float32), (4, 131, 17, np.float64),
                                         (7, 1030, 3, np.float32), (16, 96, 40, np.float64)])
def test_median_combine_matches_oracle(n, W, H, dtype):
    torch, sf = _env()
    rng = np.random.default_rng(5000 + n * 7 + W)
    diffs = [rng.normal(0, 30, size=(H, W)).astype(dtype) for _ in range(n)]
    # ties and a NaN exercise the selection and the NaN rule
    if n >= 3:
        diffs[1][0, :5] = diffs[0][0, :5]
        diffs[2][1, 3] = np.nan
    zps = list(rng.uniform(29, 31, size=n))
    _say(f"median combine n={n} {W}x{H} {np.dtype(dtype).name}")
    ref = P.median_combine(diffs, zps, 30.0).astype(dtype)
    h = sf.Handle()
    try:
        dd = [torch.from_numpy(d).cuda() for d in diffs]
        out = torch.full_like(dd[0], 7.0)
        sf.sfft_median_combine(h, sf.image_desc(dd[0]), dd, zps, 30.0, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
    finally:
        h.close()
    assert np.array_equal(np.isnan(got), np.isnan(ref))
    m = ~np.isnan(ref)
    assert np.array_equal(got[m], ref[m])


@pytest.mark.parametrize("W,H,L,DK,DB,n,dtype,refine", [
    (512, 512, 7, 2, 1, 5, np.float32, 2),     # the science spectrum is reused across templates
    (96, 80, 5, 1, 1, 3, np.float64, 1),       # workspace too small to keep it: full builds
])
def test_multi_template_matches_oracle(W, H, L, DK, DB, n, dtype, refine):
    torch, sf = _env()
    mt = synth.make_multi_template(W, H, n, seed=synth.seed_for(6, W + n), dtype=dtype)
    zps = [mt.zp_sci] * n
    zps[-1] += 0.25            # one difference on another zero point: scaled before the median
    _say(f"multi-template {W}x{H} L={L} DK={DK} DB={DB} n={n} {np.dtype(dtype).name}")
    ref = P.difference_multi(mt.templates, mt.S, L, DK, DB, zps, 29.5, refine=refine)
    md = sf.MultiDifferencer(W, H, L, DK, DB, n, image_dtype="float32" if dtype == np.float32 else "float64")
    try:
        refs = [torch.from_numpy(t).cuda() for t in mt.templates]
        sci = torch.from_numpy(mt.S).cuda()
        md.run(refs, sci, zps, 29.5, max_refine=refine)
        torch.cuda.synchronize()
        nk = O.n_mono(DK) * L * L
        r = (L - 1) // 2
        coefs = md.coefs.cpu().numpy()
        chis = md.chi2s.cpu().numpy()
        for t in range(n):
            assert md.info(t).status == 0
            o = ref["each"][t]
            cerr = np.linalg.norm(coefs[t, :nk] - o["theta"][:nk]) / np.linalg.norm(o["theta"][:nk])
            D = md.diffs[t].cpu().numpy().astype(np.float64)
            sig = _sigma_sky(o["D"], r)
            drms = float(np.sqrt(np.mean((D - o["D"]) ** 2)))
            _say(f"  template {t}: coef rel err {cerr:.2e}  D rms/sigma {drms / sig:.2e}  chi2 {chis[t]:.5f} "
                 f"(oracle {o['chi2']:.5f})")
            assert cerr <= 1e-5
            assert drms <= 1e-3 * sig
            assert abs(chis[t] - o["chi2"]) <= 1e-6 * o["chi2"]
        C = md.combined.cpu().numpy().astype(np.float64)
        sigc = _sigma_sky(ref["combined"], r)
        cmax = float(np.max(np.abs(C - ref["combined"])))
        crms = float(np.sqrt(np.mean((C - ref["combined"]) ** 2)))
        _say(f"  combined: rms/sigma {crms / sigc:.2e}  max/sigma {cmax / sigc:.2e}")
        assert crms <= 1e-3 * sigc
    finally:
        md.close()


def test_multi_template_reuse_equals_single_pairs():
    # the builds that reuse the science spectrum give the systems of
    # independent single pairs up to rounding (the FFT packs two real
    # signals per complex transform, so the science spectrum's rounding
    # depends on its partner signal): coefficients to 1e-9 relative, chi2 to
    # 1e-10, difference images to 1e-6 of the sky noise
    torch, sf = _env()
    W, H, L, DK, DB, n = 512, 512, 7, 2, 1, 4
    mt = synth.make_multi_template(W, H, n, seed=synth.seed_for(6, 77))
    _say(f"multi-template reuse vs single pairs {W}x{H} L={L} n={n}")
    md = sf.MultiDifferencer(W, H, L, DK, DB, n)
    d = sf.Differencer(W, H, L, DK, DB)
    try:
        refs = [torch.from_numpy(t).cuda() for t in mt.templates]
        sci = torch.from_numpy(mt.S).cuda()
        md.run(refs, sci, [30.0] * n, 30.0, max_refine=2)
        for t in range(n):
            d.run(refs[t], sci, max_refine=2)
            torch.cuda.synchronize()
            c1, c2 = d.buf.coef.cpu().numpy(), md.coefs[t].cpu().numpy()
            cerr = np.linalg.norm(c1 - c2) / np.linalg.norm(c1)
            D1 = d.buf.diff.cpu().numpy().astype(np.float64)
            D2 = md.diffs[t].cpu().numpy().astype(np.float64)
            sig = _sigma_sky(D1, (L - 1) // 2)
            dmax = float(np.max(np.abs(D1 - D2)))
            x1, x2 = float(d.buf.chi2.item()), float(md.chi2s[t].item())
            _say(f"  template {t}: coef rel diff {cerr:.1e}  D max diff/sigma {dmax / sig:.1e}  "
                 f"chi2 {x1:.6f} / {x2:.6f}")
            assert cerr <= 1e-9
            assert dmax <= 1e-6 * sig
            assert abs(x1 - x2) <= 1e-10 * x1
    finally:
        md.close()
        d.close()


def test_multi_template_nonfinite_science_flags_every_template():
    torch, sf = _env()
    W, H, L, DK, DB, n = 512, 512, 7, 2, 1, 3
    mt = synth.make_multi_template(W, H, n, seed=synth.seed_for(6, 78))
    S = mt.S.copy()
    S[100, 200] = np.nan
    _say("multi-template with a NaN science pixel")
    md = sf.MultiDifferencer(W, H, L, DK, DB, n)
    try:
        md.run([torch.from_numpy(t).cuda() for t in mt.templates], torch.from_numpy(S).cuda(), [30.0] * n, 30.0)
        torch.cuda.synchronize()
        for t in range(n):
            info = md.info(t)
            assert info.nonfinite != 0 and info.status == sf.SFFT_ERR_NONFINITE
    finally:
        md.close()


def _photometry_image(W, H, seed, dtype):
    rng = np.random.default_rng(seed)
    img = rng.normal(0, 12.0, size=(H, W))
    pts = rng.uniform(0, [W, H], size=(12, 2))
    img += synth.render_gaussian_stars(W, H, pts[:, 0], pts[:, 1], rng.uniform(1e3, 1e4, 12), 1.6)
    return img.astype(dtype), pts


@pytest.mark.parametrize("W,H,dtype,radius", [(300, 200, np.float32, 3.0), (257, 131, np.float64, 5.7),
                                              (64, 64, np.float32, 0.8)])
def test_aperture_flux_matches_oracle(W, H, dtype, radius):
    torch, sf = _env()
    img, pts = _photometry_image(W, H, 7100 + W, dtype)
    rng = np.random.default_rng(W)
    xy = np.concatenate([rng.uniform(-3, [W + 2, H + 2], size=(200, 2)),     # some cut by the edges
                         np.array([[0.0, 0.0], [W - 1.0, H - 1.0], [10.5, 7.5], [12.0, 9.0]]), pts])
    _say(f"aperture flux {W}x{H} {np.dtype(dtype).name} r={radius} n={len(xy)}")
    ref = P.aperture_flux(img, xy, radius)
    scale = P.aperture_flux(np.abs(img.astype(np.float64)), xy, radius)
    h = sf.Handle()
    try:
        im = torch.from_numpy(img).cuda()
        xyd = torch.from_numpy(np.ascontiguousarray(xy)).cuda()
        f = torch.zeros(len(xy), dtype=torch.float64, device="cuda")
        sf.sfft_aperture_flux(h, sf.image_desc(im), im, xyd, radius, f)
        torch.cuda.synchronize()
        got = f.cpu().numpy()
    finally:
        h.close()
    err = np.abs(got - ref) / np.maximum(scale, 1e-300)
    _say(f"  max rel err {err.max():.2e}")
    assert np.all(err <= 1e-11)


def test_limiting_magnitude_and_forced_photometry_match_oracle():
    torch, sf = _env()
    W, H = 1024, 768
    img, pts = _photometry_image(W, H, 7300, np.float32)
    xy = synth.background_positions(W, H, 1024, 3.0, seed=7301, avoid=pts, avoid_radius=12.0)
    _say(f"limiting magnitude {W}x{H} 1024 apertures r=3, forced photometry at {len(pts)} positions")
    sigma, mlim, fl = P.limiting_magnitude(img, xy, 3.0, 30.0)
    f_ref, m_ref, e_ref = P.forced_photometry(img, pts, 3.0, 30.0, sigma)
    h = sf.Handle()
    try:
        im = torch.from_numpy(img).cuda()
        desc = sf.image_desc(im)
        xyd = torch.from_numpy(xy).cuda()
        flux = torch.zeros(len(xy), dtype=torch.float64, device="cuda")
        res = torch.zeros(3, dtype=torch.float64, device="cuda")
        sf.sfft_limiting_magnitude(h, desc, im, xyd, 3.0, 30.0, flux, res)
        pd = torch.from_numpy(np.ascontiguousarray(pts)).cuda()
        ff = torch.zeros(len(pts), dtype=torch.float64, device="cuda")
        mm = torch.zeros_like(ff)
        ee = torch.zeros_like(ff)
        sf.sfft_forced_photometry(h, desc, im, pd, 3.0, 30.0, res[0:1], ff, mm, ee)
        torch.cuda.synchronize()
        r = res.cpu().numpy()
        _say(f"  sigma {r[0]:.6f} (oracle {sigma:.6f})  m_lim {r[1]:.9f} (oracle {mlim:.9f})")
        assert abs(r[0] - sigma) <= 1e-11 * sigma
        assert abs(r[1] - mlim) <= 1e-11
        assert np.allclose(flux.cpu().numpy(), fl, rtol=1e-11, atol=1e-9)
        fg, mg, eg = ff.cpu().numpy(), mm.cpu().numpy(), ee.cpu().numpy()
        assert np.allclose(fg, f_ref, rtol=1e-11, atol=1e-9)
        assert np.array_equal(np.isnan(mg), np.isnan(m_ref))
        ok = ~np.isnan(m_ref)
        assert np.all(np.abs(mg[ok] - m_ref[ok]) <= 1e-11)
        assert np.allclose(eg, e_ref, rtol=1e-11)
    finally:
        h.close()


def test_multi_template_transients_recovered_by_forced_photometry():
    # end to end: the transients planted in the science image only appear in
    # the median-combined difference with their injected flux (within the
    # aperture's enclosed fraction and the noise)
    torch, sf = _env()
    W, H, L, n = 512, 512, 9, 5
    mt = synth.make_multi_template(W, H, n, seed=synth.seed_for(6, 99), n_transients=8,
                                   transient_flux=(1.5e4, 5e4))
    md = sf.MultiDifferencer(W, H, L, 1, 1, n)
    h = sf.Handle()
    try:
        refs = [torch.from_numpy(t).cuda() for t in mt.templates]
        sci = torch.from_numpy(mt.S).cuda()
        comb = md.run(refs, sci, [mt.zp_sci] * n, mt.zp_sci)
        xy = torch.from_numpy(np.ascontiguousarray(mt.transients[:, :2])).cuda()
        f = torch.zeros(len(xy), dtype=torch.float64, device="cuda")
        rad = 6.0
        sf.sfft_aperture_flux(h, sf.image_desc(comb), comb, xy, rad, f)
        torch.cuda.synchronize()
        got = f.cpu().numpy()
    finally:
        md.close()
        h.close()
    sig_psf = mt.meta["fwhm_sci"] / 2.3548200450309493
    enclosed = 1.0 - math.exp(-rad * rad / (2 * sig_psf * sig_psf))
    want = mt.transients[:, 2] * enclosed
    _say(f"  transient flux ratio {np.round(got / want, 3)}")
    # aperture noise (r = 6 on the combined image) is ~ 0.03 of the faintest flux
    assert np.all(np.abs(got / want - 1.0) <= 0.15)
