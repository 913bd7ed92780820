"""GPU parity of the batched form: a batch of unequal pairs (different
sizes, {2,3,5}-smooth widths, L = 11 and 15) run in one launch per phase
must give the same results as each pair run alone through the single-pair
calls with the same precision (FP32 spectra, FP64 solve) and pedestals (each
item's FP64 image means), and the same
again when replayed from a captured HIP graph (several replays, with eager
work and synchronisations between them) and after autotuning.

Bounds: the batched kernels run the same per-item arithmetic as the
single-pair ones with the same row FFT radix order, so coefficients must
agree to 1e-12 relative (observed: bit-identical) and chi2 to 1e-12, for
every launch configuration the autotuner can choose (rows per workgroup,
radix order, subtract tile height, solve team)."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

SHAPES = [(256, 256, 11), (240, 200, 15), (512, 128, 11), (96, 96, 7), (160, 320, 15)]


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    return torch


def _sf():
    import paper_2603_08593_amd as sf
    sf.lib()
    return sf


def _pairs():
    out = []
    for k, (W, H, L) in enumerate(SHAPES):
        out.append(synth.make_pair(W, H, L, 2, 2, seed=700 + k, nstars=max(10, W * H // 1500),
                                   psf="moffat", fwhm=3.5, fwhm_end=5.0, flux=(1e2, 1e6),
                                   sky_R=1000.0, dtype=np.float32))
    return out


def _single(p, torch, sf, peds, radix_order=0):
    H, W = p.R.shape
    d = sf.Differencer(W, H, p.L, 2, 2, image_dtype="float32", compute="fp32",
                       ref_pedestal=peds[0], sci_pedestal=peds[1], radix_order=radix_order)
    d.run(torch.from_numpy(p.R).cuda(), torch.from_numpy(p.S).cuda(), max_refine=1)
    torch.cuda.synchronize()
    return d.buf.coef.cpu().numpy(), float(d.buf.chi2.item()), d.buf.diff.cpu().numpy()


def _check(b, refs, tag):
    for k, (coef, chi2, D) in enumerate(refs):
        got = b.bufs[k].coef.cpu().numpy()
        gchi = float(b.bufs[k].chi2.item())
        assert b.info(k).status == 0
        e = np.linalg.norm(got - coef) / np.linalg.norm(coef)
        print(f"  {tag} item {k} {SHAPES[k]}: coef rel diff {e:.1e}, chi2 {gchi:.6f} vs {chi2:.6f}, "
              f"bitwise {np.array_equal(got, coef)}", flush=True)
        assert e <= 1e-12
        assert abs(gchi - chi2) <= 1e-12 * chi2
        assert np.allclose(b.bufs[k].diff.cpu().numpy(), D, rtol=0, atol=1e-3)


def test_batch_matches_single_pairs_eager_graph_and_tuned():
    torch, sf = _torch(), _sf()
    pairs = _pairs()
    b = sf.Batch(SHAPES, dk=2, db=2, max_refine=1)
    for k, p in enumerate(pairs):
        b.load(k, torch.from_numpy(p.R).cuda(), torch.from_numpy(p.S).cuda())
    refs = [_single(p, torch, sf, b.peds[k]) for k, p in enumerate(pairs)]
    b.run()
    torch.cuda.synchronize()
    _check(b, refs, "eager")
    s = torch.cuda.Stream()
    for rep in range(3):
        for k in range(len(SHAPES)):
            b.bufs[k].coef.zero_()
            b.bufs[k].chi2.zero_()
        x = torch.randn(1000, device="cuda").sum()        # eager work between replays
        with torch.cuda.stream(s):
            b.run_graph(s)
        s.synchronize()
        torch.cuda.synchronize()
        assert torch.isfinite(x)
        _check(b, refs, f"graph replay {rep}")
    rpb, team = b.tune()
    torch.cuda.synchronize()
    kn = b.knobs()
    print(f"  tuned: {kn}", flush=True)
    assert (kn["rows_per_block"], kn["team"]) == (rpb, team)
    if kn["radix_order"] != 0:     # singles with the same row FFT plans
        refs = [_single(p, torch, sf, b.peds[k], radix_order=kn["radix_order"]) for k, p in enumerate(pairs)]
    b.run()
    torch.cuda.synchronize()
    _check(b, refs, "tuned")
    b.close()


def test_batch_knob_grid():
    """Every radix order and subtract tile height, with several row blockings
    and teams: each item equals the single-pair result with the same radix
    order; invalid knobs are rejected and leave the batch as it was."""
    torch, sf = _torch(), _sf()
    pairs = _pairs()
    b = sf.Batch(SHAPES, dk=2, db=2, max_refine=1)
    for k, p in enumerate(pairs):
        b.load(k, torch.from_numpy(p.R).cuda(), torch.from_numpy(p.S).cuda())
    refs = {ro: [_single(p, torch, sf, b.peds[k], radix_order=ro) for k, p in enumerate(pairs)]
            for ro in (0, 1)}
    grid = [(2, 0, 16, 8), (4, 1, 16, 0), (8, 0, 64, 16), (16, 1, 64, 4), (4, 1, 32, 32), (1, 0, 32, 3)]
    for rpb, ro, tr, team in grid:
        b.set_knobs(rows_per_block=rpb, radix_order=ro, tile_rows=tr, team=team)
        kn = b.knobs()
        assert (kn["rows_per_block"], kn["radix_order"], kn["tile_rows"]) == (rpb, ro, tr)
        for k in range(len(SHAPES)):
            b.bufs[k].coef.zero_()
            b.bufs[k].chi2.zero_()
        b.run()
        torch.cuda.synchronize()
        _check(b, refs[ro], f"knobs {kn}")
    before = b.knobs()
    for bad in (dict(tile_rows=24), dict(radix_order=2), dict(rows_per_block=0), dict(team=129)):
        with pytest.raises(sf.SfftError) as e:
            b.set_knobs(**bad)
        assert e.value.status == sf.SFFT_ERR_INVALID_ARG
    assert b.knobs() == before
    b.close()


def test_batch_fixed_plans_small_solve_teams():
    """Solve teams of 1, 2 and 3 workgroups: with one workgroup it runs the
    diagonal chain and the panel / trailing work in turn, with two the bulk
    role has a single workgroup; odd row-pass blockings."""
    torch, sf = _torch(), _sf()
    pairs = _pairs()
    b = sf.Batch(SHAPES, dk=2, db=2, max_refine=1)
    for k, p in enumerate(pairs):
        b.load(k, torch.from_numpy(p.R).cuda(), torch.from_numpy(p.S).cuda())
    refs = [_single(p, torch, sf, b.peds[k]) for k, p in enumerate(pairs)]
    for rpb, team in [(1, 1), (3, 2), (16, 3), (4, 0)]:
        b.plan(rpb, team)
        for k in range(len(SHAPES)):
            b.bufs[k].coef.zero_()
        b.run()
        torch.cuda.synchronize()
        _check(b, refs, f"rows per workgroup {rpb}, team {team}")
    with pytest.raises(sf.SfftError) as e:
        b.plan(0, 1)
    assert e.value.status == sf.SFFT_ERR_INVALID_ARG
    with pytest.raises(sf.SfftError) as e:
        b.plan(4, 129)
    assert e.value.status == sf.SFFT_ERR_INVALID_ARG
    b.close()


def test_batch_rejects_unsupported():
    torch, sf = _torch(), _sf()
    with pytest.raises(sf.SfftError) as e:
        sf.Batch([(4096, 64, 5)], dk=2, db=2)          # width > 2048
    assert e.value.status == sf.SFFT_ERR_UNSUPPORTED


def test_bad_items_do_not_poison_the_batch():
    """An item with a NaN pixel reports SFFT_ERR_NONFINITE and an item whose
    reference is constant (zero after its pedestal) reports SFFT_ERR_NOT_SPD;
    the other items of the same launches give the results they give alone."""
    torch, sf = _torch(), _sf()
    pairs = _pairs()
    bad_nan = pairs[1].R.copy()
    bad_nan[17, 33] = np.nan
    bad_const = np.full_like(pairs[3].R, 1234.0)
    b = sf.Batch(SHAPES, dk=2, db=2, max_refine=1)
    for k, p in enumerate(pairs):
        R = bad_nan if k == 1 else (bad_const if k == 3 else p.R)
        b.load(k, torch.from_numpy(np.ascontiguousarray(R)).cuda(), torch.from_numpy(p.S).cuda())
    good = [0, 2, 4]
    refs = {k: _single(pairs[k], torch, sf, b.peds[k]) for k in good}
    b.run()
    torch.cuda.synchronize()
    assert b.info(1).status == sf.SFFT_ERR_NONFINITE
    assert b.info(3).status == sf.SFFT_ERR_NOT_SPD and b.info(3).failed_pivot >= 0
    assert np.all(np.isnan(b.bufs[3].coef.cpu().numpy()))
    for k in good:
        coef, chi2, D = refs[k]
        assert b.info(k).status == 0
        got = b.bufs[k].coef.cpu().numpy()
        print(f"  good item {k}: bitwise {np.array_equal(got, coef)}", flush=True)
        assert np.linalg.norm(got - coef) <= 1e-12 * np.linalg.norm(coef)
        assert abs(float(b.bufs[k].chi2.item()) - chi2) <= 1e-12 * chi2
    b.close()
