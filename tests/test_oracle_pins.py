"""Pins of the FP64 CPU oracle against things other than itself: brute-force
least squares on tiny images, exact recovery of planted kernels, the
kernel-sum invariant, textbook special cases, direct-sum subtraction, the
orthogonality of the residual and chi2 ~ 1 on in-model noise."""
import json
import os

import numpy as np
import pytest

import oracle as O
import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


# 1. brute force: the FFT normal equations equal A^T A, A^T S' of the explicit
#    design matrix, and the Cholesky solution equals the SVD least-squares one.
@pytest.mark.parametrize("W,H,L,DK,DB", [
    (32, 32, 1, 0, 0), (32, 32, 3, 1, 1), (32, 32, 5, 0, 2), (48, 40, 5, 2, 2),
    (40, 48, 3, 2, 0), (96, 96, 7, 0, 1), (128, 96, 5, 2, 2), (33, 31, 3, 1, 2),
    (64, 24, 11, 0, 0),
])
def test_fft_normal_equations_equal_bruteforce(W, H, L, DK, DB):
    p = synth.make_pair(W, H, L, DK, DB, seed=11 + W + H + L, nstars=10, source="noisy")
    ped = (float(np.mean(p.R)), float(np.mean(p.S))) if DK == 0 else (0.0, 0.0)
    G, h = O.build_fft64(p.R, p.S, L, DK, DB, *ped)
    Gb, hb = O.normal_bruteforce(p.R, p.S, L, DK, DB, *ped)
    assert np.max(np.abs(G - Gb)) <= 1e-12 * np.max(np.abs(Gb))
    assert np.max(np.abs(h - hb)) <= 1e-12 * np.max(np.abs(hb))
    th, info = O.solve_cholesky64(G, h, refine=2, cond=True)
    assert info.status == "ok"
    tb = O.solve_bruteforce(p.R, p.S, L, DK, DB, *ped)
    # forward error of a backward-stable solve scales with the condition number
    assert _rel(th, tb) <= max(1e-10, 1e-15 * info.cond_est)


# 2. exact recovery of a planted kernel + background on noise-free in-model pairs
@pytest.mark.parametrize("W,H,L,DK,DB,n", [
    (96, 96, 5, 1, 1, 40), (128, 96, 7, 2, 2, 60), (64, 64, 3, 0, 2, 20),
])
def test_planted_exact_recovery(W, H, L, DK, DB, n):
    p = synth.make_pair(W, H, L, DK, DB, seed=101 + L, nstars=n, source="noisy",
                        noise_S=False)
    G, h = O.build_fft64(p.R, p.S, L, DK, DB)
    th, info = O.solve_cholesky64(G, h, refine=2, cond=True)
    assert info.status == "ok"
    err = _rel(th, p.theta)
    assert err <= max(1e-9, 1e-15 * info.cond_est), (err, info.cond_est)


# 3. kernel sum = flux ratio: exactly s (i = 0) and 0 (i > 0) on noise-free pairs;
#    within 5 sigma of the least-squares error on noisy science images.
def test_kernel_sum_invariant_noise_free():
    p = synth.make_pair(96, 80, 5, 2, 1, seed=7, nstars=40, source="noisy", noise_S=False, s=0.87)
    G, h = O.build_fft64(p.R, p.S, 5, 2, 1)
    th, _ = O.solve_cholesky64(G, h)
    k = O.kernel_sums(th, 5, 2, 1)
    assert abs(k[0] - 0.87) <= 1e-9
    assert np.max(np.abs(k[1:])) <= 1e-9


def test_kernel_sum_invariant_noisy_within_ls_error():
    L, DK, DB = 5, 0, 1
    p = synth.make_pair(128, 128, L, DK, DB, seed=8, nstars=60, source="noisy", noise_S=True, s=1.13)
    G, h = O.build_fft64(p.R, p.S, L, DK, DB)
    th, _ = O.solve_cholesky64(G, h)
    D = O.subtract64(p.R, p.S, th, L, DK, DB)
    N = O.n_unknowns(L, DK, DB)
    sigma2 = float(np.sum(D * D) / (D.size - N))
    u = np.zeros(N)
    u[: L * L] = 1.0
    sig_k = np.sqrt(sigma2 * u @ np.linalg.solve(G, u))
    assert abs(O.kernel_sums(th, L, DK, DB)[0] - 1.13) <= 5 * sig_k


# 4. textbook special cases
def test_single_tap_is_linear_regression():
    p = synth.make_pair(64, 48, 1, 0, 0, seed=3, nstars=20)
    G, h = O.build_fft64(p.R, p.S, 1, 0, 0)
    th, _ = O.solve_cholesky64(G, h)
    R, S = p.R.ravel(), p.S.ravel()
    a = np.mean((R - R.mean()) * (S - S.mean())) / np.var(R)
    b = S.mean() - a * R.mean()
    assert abs(th[0] - a) <= 1e-9 * abs(a)
    assert abs(th[1] - b) <= 1e-7 * max(abs(b), 1.0)


def test_golden_worked_example():
    g = json.load(open(os.path.join(HERE, "golden", "ols_worked_example.json")))
    R, S = np.array(g["R"]), np.array(g["S"])
    G, h = O.build_fft64(R, S, g["L"], g["DK"], g["DB"])
    th, _ = O.solve_cholesky64(G, h)
    assert np.allclose(th, g["theta"], rtol=0, atol=1e-12)
    D = O.subtract64(R, S, th, g["L"], g["DK"], g["DB"])
    assert np.allclose(D, g["D"], rtol=0, atol=1e-12)


@pytest.mark.parametrize("L,DK,DB", [(5, 1, 1), (3, 2, 2)])
def test_scaled_reference_is_scaled_delta(L, DK, DB):
    p = synth.make_pair(48, 56, L, DK, DB, seed=4, nstars=25)
    S = 0.73 * p.R
    th = O.difference(p.R, S, L, DK, DB)["theta"]
    expect = np.zeros_like(th)
    r = (L - 1) // 2
    expect[r * L + r] = 0.73
    assert np.max(np.abs(th - expect)) <= 1e-10


def test_offset_reference_is_delta_plus_constant():
    L, DK, DB = 3, 1, 1
    p = synth.make_pair(40, 40, L, DK, DB, seed=5, nstars=15)
    th = O.difference(p.R, p.R + 42.5, L, DK, DB)["theta"]
    expect = np.zeros_like(th)
    expect[(L * L) // 2] = 1.0
    expect[O.n_mono(DK) * L * L] = 42.5
    assert np.max(np.abs(th - expect)) <= 1e-9


@pytest.mark.parametrize("t", [(2, -1), (-3, 0), (0, 1)])
def test_pure_shift_is_one_hot(t):
    L, DK, DB = 7, 0, 0
    p = synth.make_pair(50, 44, L, DK, DB, seed=6, nstars=25)
    S = np.roll(p.R, shift=t, axis=(0, 1))      # S(y, x) = R(y - t0, x - t1)
    th = O.difference(p.R, S, L, DK, DB)["theta"]
    r = (L - 1) // 2
    expect = np.zeros_like(th)
    expect[(t[0] + r) * L + (t[1] + r)] = 1.0
    assert np.max(np.abs(th - expect)) <= 1e-9


# 5. subtraction against a pure-Python per-pixel loop
def test_subtract_matches_pixel_loop():
    W, H, L, DK, DB = 9, 7, 3, 2, 1
    rng = np.random.default_rng(0)
    R = rng.normal(100, 10, (H, W))
    S = rng.normal(100, 10, (H, W))
    th = rng.normal(0, 1, O.n_unknowns(L, DK, DB))
    D = O.subtract64(R, S, th, L, DK, DB, ref_pedestal=3.0, sci_pedestal=-2.0)
    r = 1
    mons = O.monomials(DK)
    bgm = O.monomials(DB)
    xt = lambda x: 2 * x / (W - 1) - 1
    yt = lambda y: 2 * y / (H - 1) - 1
    for y in range(H):
        for x in range(W):
            m = 0.0
            for i, (ea, eb) in enumerate(mons):
                for dy in range(-r, r + 1):
                    for dx in range(-r, r + 1):
                        uy, ux = (y - dy) % H, (x - dx) % W
                        coef = th[i * L * L + (dy + r) * L + (dx + r)]
                        m += coef * xt(ux) ** ea * yt(uy) ** eb * (R[uy, ux] - 3.0)
            for c, (ea, eb) in enumerate(bgm):
                m += th[len(mons) * L * L + c] * xt(x) ** ea * yt(y) ** eb
            assert abs(D[y, x] - ((S[y, x] + 2.0) - m)) <= 1e-9


# 6. chi2 ~ 1 when reference and science carry independent Poisson noise
def test_chi2_near_one_in_model():
    L, DK, DB = 5, 1, 1
    p = synth.make_pair(192, 160, L, DK, DB, seed=9, nstars=40, source="model",
                        flux=(1e3, 3e4))
    out = O.difference(p.R, p.S, L, DK, DB)
    dof = (192 - 4) * (160 - 4) - O.n_unknowns(L, DK, DB)
    assert abs(out["chi2"] - 1.0) <= 5 * np.sqrt(2.0 / dof) + 0.02


# 7. orthogonality of the residual to every design column (direct sums)
def test_residual_orthogonal_to_design():
    L, DK, DB = 5, 2, 2
    p = synth.make_pair(80, 72, L, DK, DB, seed=10, nstars=30)
    out = O.difference(p.R, p.S, L, DK, DB)
    A = O.design_matrix(p.R, L, DK, DB)
    D = out["D"].ravel()
    g = A.T @ D
    assert np.linalg.norm(g) <= 1e-10 * np.linalg.norm(A) * np.linalg.norm(D)


# 8. a rank-deficient system is reported, not pseudo-inverted
def test_constant_reference_is_not_spd():
    R = np.full((32, 32), 5.0)
    S = np.random.default_rng(1).normal(0, 1, (32, 32))
    G, h = O.build_fft64(R, S, 3, 0, 0)
    th, info = O.solve_cholesky64(G, h)
    assert th is None and info.status == "not_spd" and info.failed_pivot >= 0


# 9. generator: the named workloads have the stated shapes and statistics
def test_workload_cfg1_shape_and_kernel():
    p = synth.make_cfg1()
    assert p.R.shape == (256, 256) and p.R.dtype == np.float64
    assert (p.L, p.DK, p.DB) == (7, 0, 1)
    assert abs(p.a.sum() - 0.9) < 1e-12
    assert 900 < np.median(p.R) < 1100


# 10. the single-output checkers used at full size: model_at against the
#     tap-by-tap model image, normal_entry against the explicit design matrix,
#     and the convolution form of the model against the same model image
@pytest.mark.parametrize("L,DK,DB,ped", [(5, 2, 2, 0.0), (3, 1, 0, 7.5), (7, 0, 1, -2.0)])
def test_model_at_matches_model_image(L, DK, DB, ped):
    W, H = 36, 28
    rng = np.random.default_rng(L + DK)
    R = rng.normal(100, 20, (H, W))
    th = rng.normal(0, 0.3, O.n_unknowns(L, DK, DB))
    M = O.model_image(R, th, L, DK, DB, ref_pedestal=ped)
    ys = np.array([0, H - 1, 0, H - 1, 3, 17, 2])
    xs = np.array([0, W - 1, W - 1, 0, 1, 20, 34])
    got = O.model_at(R, th, L, DK, DB, ys, xs, ref_pedestal=ped)
    assert np.max(np.abs(got - M[ys, xs])) <= 1e-10 * np.max(np.abs(M))
    Mc = O.model_image_conv(R, th, L, DK, DB, ref_pedestal=ped)
    assert np.max(np.abs(Mc - M)) <= 1e-11 * np.max(np.abs(M))
    S = rng.normal(90, 20, (H, W))
    Dc = O.subtract_conv64(R, S, th, L, DK, DB, ped, 1.25)
    assert np.max(np.abs(Dc - O.subtract64(R, S, th, L, DK, DB, ped, 1.25))) <= 1e-11 * np.max(np.abs(M))


def test_model_conv_one_hot_shift():
    """A one-hot kernel at delta = (dy, dx) moves the reference by +delta."""
    W, H, L = 20, 16, 5
    R = np.random.default_rng(3).normal(0, 1, (H, W))
    th = np.zeros(O.n_unknowns(L, 0, 0))
    th[(1 + 2) * L + (-2 + 2)] = 1.0          # dy = 1, dx = -2
    M = O.model_image_conv(R, th, L, 0, 0)
    assert np.array_equal(M, np.roll(R, shift=(1, -2), axis=(0, 1)))


def test_normal_entry_matches_design_matrix():
    W, H, L, DK = 30, 26, 5, 2
    rng = np.random.default_rng(12)
    R = rng.normal(50, 10, (H, W))
    A = O.design_matrix(R, L, DK, 0, ref_pedestal=4.0)
    G = A.T @ A
    nk = O.n_mono(DK) * L * L
    for row, col in [(0, 0), (nk - 1, 0), (12, 31), (60, 74), (nk - 1, nk - 1), (26, 51)]:
        e = O.normal_entry(R, L, DK, row, col, ref_pedestal=4.0)
        assert abs(e - G[row, col]) <= 1e-12 * np.max(np.abs(G))
