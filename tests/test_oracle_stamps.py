"""Pins of the stamp (precision-form) oracle: stamps that tile the image
reproduce the full-image FFT normal equations; a planted kernel is recovered
exactly from stamps alone; one stamp with a single tap is ordinary linear
regression; the bfloat16 split follows round-to-nearest-even on worked
values and obeys its error bounds."""
import numpy as np
import pytest

import oracle as O
import synth


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def _tiling_centers(W, H, size):
    h = size // 2
    return np.array([(x + h, y + h) for y in range(0, H, size) for x in range(0, W, size)],
                    dtype=np.int32)


# Stamps that cover every pixel exactly once see every row of the full design
# matrix once: their Gram sums equal the FFT-built normal equations (a
# different route: spectra products, not row gathers).
@pytest.mark.parametrize("W,H,size,L,DK,DB", [
    (28, 21, 7, 3, 1, 1), (40, 40, 5, 5, 2, 2), (36, 24, 3, 1, 0, 2), (45, 27, 9, 7, 0, 0),
])
def test_tiling_stamps_equal_full_normal_equations(W, H, size, L, DK, DB):
    p = synth.make_pair(W, H, L, DK, DB, seed=300 + W + L, nstars=8, source="noisy")
    c = _tiling_centers(W, H, size)
    Gs, hs = O.stamp_normal64(p.R, p.S, c, size, L, DK, DB)
    G, h = O.build_fft64(p.R, p.S, L, DK, DB)
    assert np.max(np.abs(Gs - G)) <= 1e-12 * np.max(np.abs(G))
    assert np.max(np.abs(hs - h)) <= 1e-12 * np.max(np.abs(h))


# Stamps wrap periodically: a stamp centred on a corner covers the four corners.
def test_stamp_pixels_wrap():
    ys, xs = O.stamp_pixels(10, 8, [(0, 0)], 3)
    assert list(zip(ys.tolist(), xs.tolist())) == [
        (7, 9), (7, 0), (7, 1), (0, 9), (0, 0), (0, 1), (1, 9), (1, 0), (1, 1)]


# A noise-free in-model pair is fitted exactly by the stamp rows alone.
def test_planted_recovery_from_stamps():
    W, H, L, DK, DB = 128, 128, 5, 2, 2
    p = synth.make_pair(W, H, L, DK, DB, seed=77, nstars=60, source="noisy", noise_S=False)
    rng = np.random.default_rng(5)
    c = np.stack([rng.integers(0, W, 24), rng.integers(0, H, 24)], axis=1)
    G, h = O.stamp_normal64(p.R, p.S, c, 15, L, DK, DB)
    th, info = O.solve_cholesky64(G, h, refine=2, cond=True)
    assert info.status == "ok"
    assert _rel(th, p.theta) <= max(1e-9, 1e-15 * info.cond_est)


# L = 1, DK = DB = 0 on one stamp: S = a R + b by ordinary least squares.
def test_single_tap_single_stamp_is_regression():
    p = synth.make_pair(64, 64, 1, 0, 0, seed=3, nstars=12, source="noisy")
    G, h = O.stamp_normal64(p.R, p.S, [(30, 20)], 11, 1, 0, 0)
    th = np.linalg.solve(G, h)
    r = p.R[15:26, 25:36].ravel()
    s = p.S[15:26, 25:36].ravel()
    a = np.cov(r, s, bias=True)[0, 1] / np.var(r)
    b = s.mean() - a * r.mean()
    assert abs(th[0] - a) <= 1e-10 * abs(a)
    assert abs(th[1] - b) <= 1e-9 * max(abs(b), 1.0)


# bfloat16 rounding on hand-checked values (8 significant bits, ties to even).
@pytest.mark.parametrize("x,want", [
    (1.0, 1.0),
    (1.0 + 2.0 ** -8, 1.0),                              # tie -> even (1.0)
    (1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -6),              # tie -> even (mantissa ...10)
    (1.0 + 2.0 ** -8 + 2.0 ** -20, 1.0 + 2.0 ** -7),     # above the tie
    (-(1.0 + 2.0 ** -8 + 2.0 ** -20), -(1.0 + 2.0 ** -7)),
    (3.0, 3.0),
    (255.5, 256.0),                                      # 255.5 = 0xFF.8: tie -> even 256
    (257.0, 256.0),                                      # 257 = 1.00000001b x 2^8: tie -> even
    (259.0, 260.0),                                      # tie between 258 and 260 -> 260
    (2.0 ** -130, 2.0 ** -130),                          # subnormal kept
])
def test_bf16_rne_worked_values(x, want):
    assert float(O.bf16_rne(np.float32(x))) == want


def test_split_error_bounds():
    rng = np.random.default_rng(0)
    a = (rng.standard_normal(20000) * np.exp(rng.uniform(-20, 20, 20000))).astype(np.float32)
    b = (rng.standard_normal(20000) * np.exp(rng.uniform(-20, 20, 20000))).astype(np.float32)
    ah, al = O.split_bf16(a)
    bh, bl = O.split_bf16(b)
    # hi and lo are bfloat16 values (low 16 bits zero)
    assert not np.any(ah.view(np.uint32) & 0xFFFF) and not np.any(al.view(np.uint32) & 0xFFFF)
    a64, b64 = a.astype(np.float64), b.astype(np.float64)
    e = np.abs(a64 - ah.astype(np.float64) - al.astype(np.float64))
    assert np.all(e <= 2.0 ** -16 * np.abs(a64))
    ah, al, bh, bl = (t.astype(np.float64) for t in (ah, al, bh, bl))
    prod = ah * bh + ah * bl + al * bh
    assert np.all(np.abs(prod - a64 * b64) <= 3 * 2.0 ** -16 * np.abs(a64 * b64))


# The two-term split-product Gram is the exact Gram up to the split bound.
def test_split_gram_within_split_bound():
    W, H, L, DK, DB = 96, 64, 5, 2, 1
    p = synth.make_pair(W, H, L, DK, DB, seed=21, nstars=30, source="noisy", dtype=np.float32)
    c = [(20, 20), (70, 40), (50, 10)]
    G, h = O.stamp_normal64(p.R, p.S, c, 13, L, DK, DB)
    Gs, hs = O.stamp_normal_split(p.R, p.S, c, 13, L, DK, DB, terms=2)
    Ga, ha = O.stamp_abs_gram(p.R, p.S, c, 13, L, DK, DB)
    # FP32 rounding of each operand (2^-24 each) plus the split (3 * 2^-16)
    tol = 3 * 2.0 ** -16 + 3 * 2.0 ** -24
    assert np.all(np.abs(Gs - G) <= tol * Ga)
    assert np.all(np.abs(hs - h) <= tol * ha)


# Three-term split on hand-checked values: (1 + 2^-10 + 2^-19) keeps its
# three bits in three terms; (1 + 2^-8 + 2^-9) rounds hi up and leaves a
# negative mid.
@pytest.mark.parametrize("x,want", [
    (1.0 + 2.0 ** -10 + 2.0 ** -19, (1.0, 2.0 ** -10, 2.0 ** -19)),
    (1.0 + 2.0 ** -8 + 2.0 ** -9, (1.0 + 2.0 ** -7, -(2.0 ** -9), 0.0)),
    (-3.0, (-3.0, 0.0, 0.0)),
    (1.0 + 2.0 ** -23, (1.0, 2.0 ** -23, 0.0)),
])
def test_split3_worked_values(x, want):
    got = tuple(float(t) for t in O.split_bf16_3(np.float32(x)))
    assert got == want


def test_split3_is_exact_and_products_within_bound():
    rng = np.random.default_rng(1)
    a = (rng.standard_normal(50000) * np.exp(rng.uniform(-40, 40, 50000))).astype(np.float32)
    b = (rng.standard_normal(50000) * np.exp(rng.uniform(-40, 40, 50000))).astype(np.float32)
    parts_a = O.split_bf16_3(a)
    parts_b = O.split_bf16_3(b)
    for t in parts_a + parts_b:
        assert not np.any(t.view(np.uint32) & 0xFFFF)          # bfloat16 values
    a64, b64 = a.astype(np.float64), b.astype(np.float64)
    A = [t.astype(np.float64) for t in parts_a]
    B = [t.astype(np.float64) for t in parts_b]
    assert np.array_equal(A[0] + A[1] + A[2], a64)              # exact decomposition
    assert np.array_equal(B[0] + B[1] + B[2], b64)
    # kept: every term pair of order <= 2; dropped: mid*lo, lo*mid, lo*lo,
    # each below 2^-24 |ab|
    prod = sum(A[p] * B[q] for p, q in O.split_product_terms(3))
    assert np.all(np.abs(prod - a64 * b64) <= 2.0 ** -23 * np.abs(a64 * b64))
    # the two-term form is coarser: its products sit near 2^-16
    A2 = [t.astype(np.float64) for t in O.split_bf16(a)]
    B2 = [t.astype(np.float64) for t in O.split_bf16(b)]
    prod2 = sum(A2[p] * B2[q] for p, q in O.split_product_terms(2))
    assert np.max(np.abs(prod2 - a64 * b64) / np.abs(a64 * b64)) > 2.0 ** -20


# The three-term split Gram is the exact Gram up to the operands' FP32
# rounding (2^-24 each) and the dropped term products (2^-23).
def test_split3_gram_within_bound():
    W, H, L, DK, DB = 96, 64, 5, 2, 1
    p = synth.make_pair(W, H, L, DK, DB, seed=21, nstars=30, source="noisy", dtype=np.float32)
    c = [(20, 20), (70, 40), (50, 10)]
    G, h = O.stamp_normal64(p.R, p.S, c, 13, L, DK, DB)
    Gs, hs = O.stamp_normal_split(p.R, p.S, c, 13, L, DK, DB, terms=3)
    Ga, ha = O.stamp_abs_gram(p.R, p.S, c, 13, L, DK, DB)
    tol = 2.0 ** -23 + 3 * 2.0 ** -24
    assert np.all(np.abs(Gs - G) <= tol * Ga)
    assert np.all(np.abs(hs - h) <= tol * ha)
    # a planted error in the kept terms (mid*mid dropped) breaks the bound
    A = O.stamp_design(p.R, c, 13, L, DK, DB).astype(np.float32)
    Ah, Am, Al = (t.astype(np.float64) for t in O.split_bf16_3(A))
    Gbad = Ah.T @ Ah + Ah.T @ Am + Am.T @ Ah + Ah.T @ Al + Al.T @ Ah
    assert np.any(np.abs(Gbad - G) > tol * Ga)
