"""The allocation-free subtract (sfft_subtract_noalloc) against sfft_subtract,
through the C ABI: two calls in a row, the second on a smaller pair, each
compared with the workspace entry point on the same inputs and coefficients.
Both run the same kernels in the same order, so the difference image and the
chi2 value agree bit for bit."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _case(sf, torch, W, H, L, DK, DB, seed, dtype):
    p = synth.make_pair(W, H, L, DK, DB, seed=seed, nstars=max(20, W * H // 2000), dtype=dtype)
    dt = "float32" if dtype == np.float32 else "float64"
    _say(f"no-alloc subtract {W}x{H} L={L} DK={DK} DB={DB} {dt} seed={seed}")
    d = sf.Differencer(W, H, L, DK, DB, image_dtype=dt)
    R = torch.from_numpy(p.R).cuda()
    S = torch.from_numpy(p.S).cuda()
    d.run(R, S, max_refine=1)
    torch.cuda.synchronize()
    assert d.info().status == 0
    ref_D = d.buf.diff.clone()
    ref_chi2 = d.buf.chi2.clone()
    D2 = torch.full_like(ref_D, float("nan"))
    chi2 = torch.full_like(ref_chi2, float("nan"))
    sf.sfft_subtract_noalloc(d.handle, d.desc, R, S, d.buf.coef, D2, chi2)
    torch.cuda.synchronize()
    assert torch.equal(D2, ref_D)
    assert torch.equal(chi2, ref_chi2)
    # without chi2 (null pointer): the same difference image
    D3 = torch.full_like(ref_D, float("nan"))
    sf.sfft_subtract_noalloc(d.handle, d.desc, R, S, d.buf.coef, D3, None)
    torch.cuda.synchronize()
    assert torch.equal(D3, ref_D)
    _say(f"  identical; chi2 {chi2.item():.6f}")
    d.close()


def test_noalloc_subtract_matches_workspace_entry_point():
    import torch
    import paper_2603_08593_amd as sf
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    sf.lib()
    # first call on the larger pair, second on a smaller one: the shared
    # scratch holds the first call's partials when the second starts
    _case(sf, torch, 640, 480, 11, 2, 2, 9101, np.float32)
    _case(sf, torch, 200, 136, 7, 1, 1, 9102, np.float64)


def test_noalloc_subtract_rejects_oversize_and_bad_args():
    import torch
    import paper_2603_08593_amd as sf
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    lib = sf.lib()
    h = sf.Handle()
    try:
        # 8192 x 16416: 128 x 513 tiles of 64 x 32 > 65536 -> workspace error, nothing launched
        big = sf.make_desc(8192, 16416, 11, 2, 2)
        dummy = torch.zeros(16, dtype=torch.float32, device="cuda")
        coef = torch.zeros(732, dtype=torch.float64, device="cuda")
        rc = lib.sfft_subtract_noalloc(h.ptr, big, sf._dp(dummy), sf._dp(dummy), sf._dp(coef),
                                       sf._dp(torch.zeros_like(dummy)), None, None)
        assert rc == sf.SFFT_ERR_WORKSPACE
        small = sf.make_desc(64, 64, 5, 0, 0)
        rc = lib.sfft_subtract_noalloc(h.ptr, small, sf._dp(dummy), sf._dp(dummy), sf._dp(coef),
                                       sf._dp(dummy), None, None)     # diff aliases ref
        assert rc == sf.SFFT_ERR_INVALID_ARG
    finally:
        h.close()
