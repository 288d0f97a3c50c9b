"""Pins of the FP64 oracle against what the method and the mathematics fix.

Each test checks the oracle against something other than itself: a library
routine (scipy.ndimage, numpy least squares / sort / solve), a closed form of
Farneback's two-frame method (a quadratic shifted by d is recovered exactly),
or an invariant (identical frames, integer shifts, DC offset, intensity scale,
transposition). Tolerances are FP64 rounding-level unless stated.
"""
import json
import os

import numpy as np
import pytest

import bruteforce as bf
import oracle
from paper_2511_14419_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rnd(shape, seed, scale=100.0):
    return np.random.default_rng(seed).standard_normal(shape) * scale


def quad_image(h, w, A, b, c, shift=(0.0, 0.0)):
    """f(x) = x^T A x + b^T x + c at x = (col, row) - shift."""
    yy, xx = np.meshgrid(np.arange(h, dtype=np.float64), np.arange(w, dtype=np.float64), indexing="ij")
    x = xx - shift[0]
    y = yy - shift[1]
    return A[0][0] * x * x + 2 * A[0][1] * x * y + A[1][1] * y * y + b[0] * x + b[1] * y + c


# --------------------------------------------------------------------------- pyramid

@pytest.mark.parametrize("shape", [(16, 16), (17, 23), (9, 8), (31, 5)])
def test_pyr_down_matches_scipy(shape):
    img = rnd(shape, 1)
    np.testing.assert_allclose(oracle.pyr_down(img), bf.pyr_down(img), rtol=0, atol=1e-12)


def test_pyr_down_constant_and_quadratic():
    img = np.full((20, 14), 7.25)
    assert np.all(oracle.pyr_down(img) == 7.25)
    A = [[0.03, -0.011], [-0.011, 0.02]]
    f = quad_image(40, 36, A, (0.4, -0.7), 3.0)
    g = oracle.pyr_down(f)
    # blur with a unit-variance binomial in each axis adds A_xx + A_yy; keeping
    # the even pixels doubles every coordinate: g(i, j) = f(2j, 2i) + A_xx + A_yy
    h2, w2 = g.shape
    ref = quad_image(h2, w2, [[4 * A[0][0], 4 * A[0][1]], [4 * A[1][0], 4 * A[1][1]]],
                     (0.8, -1.4), 3.0 + A[0][0] + A[1][1])
    np.testing.assert_allclose(g[1:-1, 1:-1], ref[1:-1, 1:-1], rtol=0, atol=1e-11)


# --------------------------------------------------------------------------- expansion

@pytest.mark.parametrize("shape,n,sigma", [((16, 16), 5, 1.1), ((23, 17), 5, 1.1), ((18, 21), 7, 1.5),
                                           ((12, 40), 5, 0.8)])
def test_poly_expand_matches_lstsq(shape, n, sigma):
    img = rnd(shape, 2)
    np.testing.assert_allclose(oracle.poly_expand(img, n, sigma), bf.poly_expand(img, n, sigma),
                               rtol=0, atol=1e-9)


def test_poly_expand_recovers_global_quadratic():
    A = [[0.021, 0.0135], [0.0135, -0.034]]
    b = (1.7, -0.6)
    f = quad_image(30, 26, A, b, 11.0)
    r = oracle.poly_expand(f, 5, 1.1)
    yy, xx = np.meshgrid(np.arange(30.0), np.arange(26.0), indexing="ij")
    sl = (slice(2, -2), slice(2, -2))
    # local linear term at pixel p is b + 2 A p
    np.testing.assert_allclose(r[0][sl], (b[0] + 2 * (A[0][0] * xx + A[0][1] * yy))[sl], atol=1e-10)
    np.testing.assert_allclose(r[1][sl], (b[1] + 2 * (A[1][0] * xx + A[1][1] * yy))[sl], atol=1e-10)
    np.testing.assert_allclose(r[2][sl], A[0][0], atol=1e-12)
    np.testing.assert_allclose(r[3][sl], A[1][1], atol=1e-12)
    np.testing.assert_allclose(r[4][sl], 2 * A[0][1], atol=1e-12)


# --------------------------------------------------------------------------- sampling

def test_bilinear_matches_scipy_and_clamps():
    p = rnd((9, 13), 3)
    rng = np.random.default_rng(4)
    for x, y in zip(rng.uniform(-3, 16, 200), rng.uniform(-3, 12, 200)):
        ref = bf.sample(p, np.array(x), np.array(y))
        assert abs(oracle.bilinear(p, x, y) - ref) < 1e-12
    assert oracle.bilinear(p, 4, 7) == p[7, 4]
    assert oracle.bilinear(p, -5, -5) == p[0, 0]
    assert oracle.bilinear(p, 99, 99) == p[-1, -1]


def test_flow_upsample():
    c = rnd((6, 7, 2), 5, 1.0)
    f = oracle.flow_upsample(c, 12, 13)
    np.testing.assert_array_equal(f[::2, ::2], 2 * c)
    np.testing.assert_allclose(f, bf.upsample(c, 12, 13), atol=1e-12)
    # odd fine pixels sit half-way between coarse pixels
    np.testing.assert_allclose(f[1:-1:2, 0], c[:-1, 0] + c[1:, 0], atol=1e-12)


# --------------------------------------------------------------------------- update / window / solve

def test_update_terms_match_bruteforce():
    r1 = rnd((5, 14, 11), 6, 1.0)
    r2 = rnd((5, 14, 11), 7, 1.0)
    fl = rnd((14, 11, 2), 8, 2.0)
    np.testing.assert_allclose(oracle.update_terms(r1, r2, fl), bf.update_terms(r1, r2, fl), atol=1e-12)


def test_update_terms_closed_form():
    """Quadratic and its shift by d: h = G d at every pixel whatever the prior."""
    A = [[0.02, 0.007], [0.007, 0.015]]
    d = (0.37, -1.81)
    f1 = quad_image(40, 40, A, (0.5, 0.2), 1.0)
    f2 = quad_image(40, 40, A, (0.5, 0.2), 1.0, shift=d)
    r1, r2 = oracle.poly_expand(f1), oracle.poly_expand(f2)
    prior = rnd((40, 40, 2), 9, 0.8)
    gh = oracle.update_terms(r1, r2, prior)
    sl = (slice(6, -6), slice(6, -6))
    g11, g12, g22, h1, h2 = (g[sl] for g in gh)
    np.testing.assert_allclose(h1, g11 * d[0] + g12 * d[1], atol=1e-12)
    np.testing.assert_allclose(h2, g12 * d[0] + g22 * d[1], atol=1e-12)
    Am = np.array(A)
    G = Am.T @ Am
    np.testing.assert_allclose(g11, G[0, 0], atol=1e-14)
    np.testing.assert_allclose(g12, G[0, 1], atol=1e-14)
    np.testing.assert_allclose(g22, G[1, 1], atol=1e-14)


@pytest.mark.parametrize("win", [1, 3, 7, 15])
def test_box_sum_matches_uniform_filter(win):
    x = rnd((3, 19, 23), 10)
    np.testing.assert_allclose(oracle.box_sum(x, win), bf.box_sum(x, win), rtol=1e-12, atol=1e-9)


def test_solve_matches_numpy_and_regularises():
    rng = np.random.default_rng(11)
    M = rng.standard_normal((2, 2, 8, 8))
    G = np.einsum("kihw,kjhw->ijhw", M, M)
    hv = rng.standard_normal((2, 8, 8))
    gh = np.stack([G[0, 0], G[0, 1], G[1, 1], hv[0], hv[1]])
    np.testing.assert_allclose(oracle.solve(gh, 1e-3), bf.solve(gh, 1e-3), atol=1e-9)
    # rank-one G: det = 0 < eps tr^2, so den = eps tr^2 and d = adj(G) h / den
    gh1 = np.zeros((5, 1, 2))
    gh1[:, 0, 0] = [4.0, 2.0, 1.0, 3.0, -1.0]
    gh1[:, 0, 1] = [0.0, 0.0, 0.0, 5.0, 5.0]  # tr = 0 -> zero flow
    d = oracle.solve(gh1, 1e-3)
    np.testing.assert_allclose(d[0, 0], [(1 * 3 - 2 * -1) / (1e-3 * 25), (4 * -1 - 2 * 3) / (1e-3 * 25)])
    assert np.all(d[0, 1] == 0.0)


# --------------------------------------------------------------------------- whole flow

@pytest.mark.parametrize("levels,iters", [(1, 1), (2, 2), (3, 3), (3, 1)])
def test_quadratic_shift_recovered_exactly(levels, iters):
    A = [[0.004, 0.0012], [0.0012, 0.003]]
    d = (0.37, -1.81)
    n = 192
    f1 = quad_image(n, n, A, (0.3, -0.2), 10.0)
    f2 = quad_image(n, n, A, (0.3, -0.2), 10.0, shift=d)
    fl = oracle.flow(f1, f2, levels=levels, iterations=iters)
    m = 72
    np.testing.assert_allclose(fl[m:-m, m:-m, 0], d[0], atol=1e-9)
    np.testing.assert_allclose(fl[m:-m, m:-m, 1], d[1], atol=1e-9)


def test_identical_frames_zero_flow_empty_mask():
    f = synth.pair_512_u8(3)[0][:96, :80].astype(np.float64)
    for mode, thr in [(0, 1.0), (1, 0.2)]:
        fl, mask, _ = oracle.roi_mask(f, f, thresh_mode=mode, thresh=thr)
        assert np.all(fl == 0.0)
        assert not mask.any()


def shifted_pair(h, w, d, seed, sigma=2.0):
    T = synth.smooth_texture(h, w, seed, sigma=sigma, pad=16)
    p = 16
    prev = T[p:p + h, p:p + w]
    nxt = T[p - d[1]:p - d[1] + h, p - d[0]:p - d[0] + w]  # next(y) = prev(y - d)
    return prev, nxt


@pytest.mark.parametrize("d", [(1, 0), (0, -2), (2, 1), (-3, 2)])
def test_integer_shift_is_fixed_point(d):
    prev, nxt = shifted_pair(80, 72, d, 12)
    init = np.zeros((80, 72, 2))
    init[..., 0], init[..., 1] = d
    fl = oracle.flow(prev, nxt, levels=1, iterations=2, init=init)
    # each iteration is exact where its whole window saw exact terms (poly
    # half-width 2 + window half-width 7 + |d| + 1 from the border), so the
    # exact region shrinks by that much per iteration
    m = 2 * (2 + 7 + 4)
    np.testing.assert_allclose(fl[m:-m, m:-m, 0], d[0], atol=1e-9)
    np.testing.assert_allclose(fl[m:-m, m:-m, 1], d[1], atol=1e-9)


@pytest.mark.parametrize("d", [(1, 0), (0, -2), (2, 1), (-3, 2)])
def test_integer_shift_from_zero_converges(d):
    prev, nxt = shifted_pair(160, 160, d, 13)
    fl = oracle.flow(prev, nxt)
    m = 40
    err = np.hypot(fl[m:-m, m:-m, 0] - d[0], fl[m:-m, m:-m, 1] - d[1])
    assert err.max() <= 0.05 and np.median(err) <= 0.01, (err.max(), np.median(err))


def test_dc_scale_transpose_invariance():
    f0, f1, _ = synth.pair_512_u8(1)
    a, b = f0[100:196, 60:140].astype(np.float64), f1[100:196, 60:140].astype(np.float64)
    ref = oracle.flow(a, b)
    np.testing.assert_allclose(oracle.flow(a + 517.0, b + 517.0), ref, atol=1e-9)
    np.testing.assert_allclose(oracle.flow(3.5 * a, 3.5 * b), ref, atol=1e-9)
    t = oracle.flow(a.T.copy(), b.T.copy())
    np.testing.assert_allclose(t[..., 0], ref[..., 1].T, atol=1e-9)
    np.testing.assert_allclose(t[..., 1], ref[..., 0].T, atol=1e-9)


@pytest.mark.parametrize("shape,levels,win,poly_n", [((24, 20), 1, 5, 5), ((32, 28), 2, 7, 5),
                                                     ((40, 36), 2, 3, 7), ((36, 36), 3, 5, 5)])
def test_flow_matches_bruteforce(shape, levels, win, poly_n):
    f0, f1, _ = synth.pair_512_u8(2)
    a = f0[200:200 + shape[0], 210:210 + shape[1]].astype(np.float64)
    b = f1[200:200 + shape[0], 210:210 + shape[1]].astype(np.float64)
    kw = dict(levels=levels, winsize=win, iterations=2, poly_n=poly_n, poly_sigma=1.1 if poly_n == 5 else 1.5)
    np.testing.assert_allclose(oracle.flow(a, b, **kw), bf.flow(a, b, **kw), atol=1e-8)


def test_init_flow_used_at_coarsest_level():
    f0, f1, _ = synth.pair_512_u8(4)
    a, b = f0[:64, :48].astype(np.float64), f1[:64, :48].astype(np.float64)
    init = np.random.default_rng(5).uniform(-2, 2, (64, 48, 2))
    kw = dict(levels=2, winsize=5, iterations=1)
    np.testing.assert_allclose(oracle.flow(a, b, init=init, **kw), bf.flow(a, b, init=init, **kw), atol=1e-8)


def test_moving_blob_flow_points_along_motion():
    h = w = 96
    yy, xx = np.meshgrid(np.arange(h, dtype=float), np.arange(w, dtype=float), indexing="ij")
    blob = lambda cx, cy: 100 * np.exp(-((xx - cx) ** 2 + (yy - cy) ** 2) / (2 * 6.0 ** 2))
    fl = oracle.flow(blob(45.0, 48.0), blob(47.0, 49.0))  # moved +2 columns, +1 row
    dx, dy = fl[48, 45]
    assert abs(dx - 2.0) < 0.1 and abs(dy - 1.0) < 0.1, (dx, dy)


# --------------------------------------------------------------------------- threshold / dilation

def test_threshold_top_matches_sort_with_ties():
    rng = np.random.default_rng(14)
    fl = rng.standard_normal((37, 29, 2))
    fl[:5, :5] = 0.5  # a block of ties
    for q in [0.01, 0.2, 0.5, 0.97]:
        pre, t2 = oracle.threshold_top(fl, q)
        ref, rt2 = bf.threshold_top(fl, q)
        assert t2 == rt2
        np.testing.assert_array_equal(pre, ref)
        assert pre.sum() <= int(np.floor(q * pre.size))


def test_threshold_top_all_zero_and_exact_count():
    pre, t2 = oracle.threshold_top(np.zeros((10, 10, 2)), 0.2)
    assert t2 == 0.0 and not pre.any()
    fl = np.zeros((10, 10, 2))
    fl[..., 0] = np.arange(100).reshape(10, 10)  # distinct magnitudes
    pre, _ = oracle.threshold_top(fl, 0.2)
    assert pre.sum() == 20 and pre.ravel()[80:].all()


def test_threshold_abs_strict():
    fl = np.array([[[1.0, 0.0], [0.6, 0.8], [0.0, 1.0000001], [0.3, 0.2]]])
    np.testing.assert_array_equal(oracle.threshold_abs(fl, 1.0), [[0, 0, 1, 0]])


def test_top_fraction_golden_example():
    """The paper's example: an RoI threshold of 0.2 keeps the top 20 %."""
    with open(os.path.join(GOLDEN, "top_fraction_example.json")) as fh:
        g = json.load(fh)
    mags = np.array(g["magnitudes"], dtype=np.float64)
    fl = np.stack([mags, np.zeros_like(mags)], -1)[None]
    pre, _ = oracle.threshold_top(fl, g["q"])
    assert sorted(np.nonzero(pre[0])[0].tolist()) == g["selected"]


@pytest.mark.parametrize("r,shape", [(0, 0), (1, 0), (2, 0), (3, 1), (2, 1)])
def test_dilate_matches_scipy(r, shape):
    pre = (np.random.default_rng(15).uniform(size=(33, 27)) > 0.93).astype(np.uint8)
    pre[0, 0] = pre[-1, -1] = 1
    np.testing.assert_array_equal(oracle.dilate(pre, r, shape), bf.dilate(pre, r, shape))


def test_dilate_single_pixel_gives_structuring_element():
    pre = np.zeros((11, 11), np.uint8)
    pre[5, 5] = 1
    for r, shape in [(2, 0), (3, 1)]:
        m = oracle.dilate(pre, r, shape)
        se = bf.structuring_element(r, shape).astype(np.uint8)
        np.testing.assert_array_equal(m[5 - r:6 + r, 5 - r:6 + r], se)
        assert m.sum() == se.sum()


# --------------------------------------------------------------------------- denoising pre-stage

@pytest.mark.parametrize("r", [1, 2])
def test_median_matches_scipy(r):
    from scipy import ndimage
    img = np.random.default_rng(20).integers(0, 4096, (23, 31)).astype(np.float64)
    np.testing.assert_array_equal(oracle.median(img, r), ndimage.median_filter(img, size=2 * r + 1, mode="nearest"))


def test_bilateral_limits():
    from scipy import ndimage
    img = rnd((21, 26), 21, 50.0)
    # huge range sigma: a normalised Gaussian blur
    t = np.arange(-2, 3, dtype=np.float64)
    k = np.exp(-t * t / (2 * 1.5 ** 2))
    k /= k.sum()
    blur = ndimage.correlate1d(ndimage.correlate1d(img, k, axis=0, mode="nearest"), k, axis=1, mode="nearest")
    np.testing.assert_allclose(oracle.bilateral(img, 2, 1.5, 1e9), blur, atol=1e-9)
    # tiny range sigma on distinct values: only the centre weighs
    np.testing.assert_allclose(oracle.bilateral(img, 2, 1.5, 1e-6), img, atol=1e-12)
    # constants stay constant
    assert np.allclose(oracle.bilateral(np.full((9, 9), 7.5), 2, 1.5, 3.0), 7.5)


def test_bilateral_matches_bruteforce():
    img = rnd((13, 17), 22, 30.0)
    ref = np.empty_like(img)
    pad = np.pad(img, 2, mode="edge")
    for i in range(13):
        for j in range(17):
            win = pad[i:i + 5, j:j + 5]
            u, v = np.meshgrid(np.arange(-2, 3), np.arange(-2, 3), indexing="ij")
            wt = np.exp(-(u * u + v * v) / (2 * 1.2 ** 2)) * np.exp(-(win - img[i, j]) ** 2 / (2 * 8.0 ** 2))
            ref[i, j] = (wt * win).sum() / wt.sum()
    np.testing.assert_allclose(oracle.bilateral(img, 2, 1.2, 8.0), ref, atol=1e-10)


def test_denoise_composes_median_then_bilateral():
    img = np.random.default_rng(23).integers(0, 255, (19, 22)).astype(np.float64)
    np.testing.assert_array_equal(oracle.denoise(img, 1, 2, 1.5, 20.0),
                                  oracle.bilateral(oracle.median(img, 1), 2, 1.5, 20.0))
    np.testing.assert_array_equal(oracle.denoise(img, 0, 0), img)


def test_ensemble_is_union_of_recent_masks():
    rng = np.random.default_rng(30)
    masks = [(rng.uniform(size=(7, 9)) > 0.8).astype(np.uint8) for _ in range(6)]
    for k in (0, 1, 2, 5):
        out = oracle.ensemble(masks, k)
        for t in range(6):
            ref = np.logical_or.reduce(masks[max(0, t - k):t + 1]).astype(np.uint8)
            np.testing.assert_array_equal(out[t], ref)
    assert all(np.array_equal(a, b) for a, b in zip(oracle.ensemble(masks, 0), masks))


# --------------------------------------------------------------------------- the paper's RoI rule

def test_open_close_matches_scipy():
    from scipy import ndimage
    pre = (np.random.default_rng(31).uniform(size=(40, 37)) > 0.55).astype(np.uint8)
    for r in (1, 2):
        se = np.ones((2 * r + 1, 2 * r + 1), bool)
        ero = lambda m: ndimage.binary_erosion(m, se, border_value=1)
        dil = lambda m: ndimage.binary_dilation(m, se, border_value=0)
        ref = ero(dil(dil(ero(pre.astype(bool))))).astype(np.uint8)
        np.testing.assert_array_equal(oracle.open_close(pre, r), ref)


def test_cc_filter_matches_scipy_label():
    from scipy import ndimage
    m = (np.random.default_rng(32).uniform(size=(50, 45)) > 0.6).astype(np.uint8)
    lab, n = ndimage.label(m, structure=np.ones((3, 3)))
    area = np.bincount(lab.ravel())
    for a in (1, 3, 10, 40):
        keep = area >= a
        keep[0] = False
        np.testing.assert_array_equal(oracle.cc_filter(m, a), keep[lab].astype(np.uint8))


def test_saliency_bruteforce_and_closed_form():
    rng = np.random.default_rng(33)
    fl = rng.normal(size=(17, 23, 2))
    M = np.hypot(fl[..., 0], fl[..., 1])
    P = np.pad(M, 1, mode="edge")
    G = np.hypot(0.5 * (P[1:-1, 2:] - P[1:-1, :-2]), 0.5 * (P[2:, 1:-1] - P[:-2, 1:-1]))
    S = 0.7 * M / M.max() + 0.3 * G / G.max()
    np.testing.assert_allclose(oracle.saliency(fl, 0.7), S / S.max(), atol=1e-14)
    # uniform motion: no gradient, saliency 1 everywhere; no motion: 0
    np.testing.assert_array_equal(oracle.saliency(np.ones((5, 6, 2)), 0.7), np.ones((5, 6)))
    np.testing.assert_array_equal(oracle.saliency(np.zeros((5, 6, 2)), 0.7), np.zeros((5, 6)))
    # magnitude growing linearly along x (interior): constant gradient term
    xx = np.tile(np.arange(1.0, 11.0), (4, 1))
    s = oracle.saliency(np.stack([xx, np.zeros_like(xx)], -1), 1.0)
    np.testing.assert_allclose(s, xx / 10.0, atol=1e-15)


def test_saliency_mask_top_fraction():
    f0, f1, _ = synth.pair_512_u8(2)
    fl = oracle.flow(f0[:128, :128].astype(float), f1[:128, :128].astype(float))
    mask, s, tau = oracle.saliency_mask(fl, 1, 0.2)
    assert (s > tau).sum() <= int(np.floor(0.2 * s.size))
    assert mask.any() and mask.mean() < 0.6


# --------------------------------------------------------------------------- stabilisation (phase correlation)

def _dft2(x):
    """Textbook 2-D DFT by explicit sums: X(k, l) = sum x(m, n) e^{-2 pi i (km/M + ln/N)}."""
    M, N = x.shape
    m = np.arange(M)
    n = np.arange(N)
    Fm = np.exp(-2j * np.pi * np.outer(m, m) / M)
    Fn = np.exp(-2j * np.pi * np.outer(n, n) / N)
    out = np.zeros((M, N), complex)
    for k in range(M):
        for l in range(N):
            out[k, l] = np.sum(x * np.outer(Fm[k], Fn[l]))
    return out


def test_phase_correlation_matches_textbook_definition():
    rng = np.random.default_rng(41)
    a, b = rng.uniform(0, 255, (11, 13)), rng.uniform(0, 255, (11, 13))
    r, P, y0, x0 = oracle.phase_correlation(a, b)
    assert (P, y0, x0) == (8, 1, 2)
    win = np.outer(0.5 - 0.5 * np.cos(2 * np.pi * np.arange(8) / 7), 0.5 - 0.5 * np.cos(2 * np.pi * np.arange(8) / 7))
    A = _dft2(a[1:9, 2:10] * win)
    B = _dft2(b[1:9, 2:10] * win)
    X = B * np.conj(A)
    R = X / np.abs(X)
    # inverse DFT by the same explicit sums: x(m, n) = (1/MN) sum X(k, l) e^{+2 pi i (...)}
    ref = np.conj(_dft2(np.conj(R))).real / 64
    np.testing.assert_allclose(r, ref, atol=1e-12)


def test_phase_shift_circular_closed_form():
    """For a circular shift inside the window the normalised cross power is a
    pure phase ramp when no window is applied; with the Hann window the peak
    still lands exactly on the shift for a broadband texture."""
    tex = synth.smooth_texture(256, 256, 3, sigma=1.0, pad=0)
    for s in [(0, 0), (3, -5), (-7, 2), (12, 0), (0, -13)]:
        moved = np.roll(tex, s, axis=(0, 1))
        sy, sx, peak = oracle.phase_shift(tex, moved)
        assert (sy, sx) == s and peak > 0.3


def test_phase_shift_sign_and_align_on_translated_frames():
    """next = prev moved by s (next(x) = prev(x - s)): the estimate is s and
    aligning next by it gives back prev away from the entering border."""
    big = synth.smooth_texture(300, 340, 7, sigma=1.5, pad=40)
    for s in [(4, -6), (-9, 3), (0, 0), (1, 1)]:
        prev = big[40:340, 40:380]
        nxt = big[40 - s[0]:340 - s[0], 40 - s[1]:380 - s[1]]
        sy, sx, _ = oracle.phase_shift(prev, nxt)
        assert (sy, sx) == s
        al = oracle.align(nxt, sy, sx)
        m = 16
        np.testing.assert_array_equal(al[m:-m, m:-m], prev[m:-m, m:-m])


def test_phase_size_and_align_edges():
    assert oracle.phase_size(2048, 2448) == 2048
    assert oracle.phase_size(1536, 1536) == 1024
    assert oracle.phase_size(5, 300) == 4
    assert oracle.phase_size(1, 300) == 0
    assert oracle.phase_shift(np.ones((1, 7)), np.ones((1, 7))) == (0, 0, 0.0)
    x = np.arange(12.0).reshape(3, 4)
    np.testing.assert_array_equal(oracle.align(x, 1, -2), x[np.ix_([1, 2, 2], [0, 0, 0, 1])])
    # identical frames: zero shift, peak 1 (the surface is a unit delta)
    f = synth.smooth_texture(64, 64, 2, pad=0)
    sy, sx, peak = oracle.phase_shift(f, f)
    assert (sy, sx) == (0, 0) and abs(peak - 1.0) < 1e-12


def test_stabilized_path_recovers_translated_pair():
    """A globally translated pair: with stabilisation the flow is the residual
    (near zero), without it the flow carries the translation."""
    big = synth.smooth_texture(96, 128, 9, sigma=2.0, pad=16)
    prev = big[16:112, 16:144]
    nxt = big[16 - 2:112 - 2, 16 + 3:144 + 3]  # next(x) = prev(x - (2, -3))
    f0, _, _ = oracle.roi_mask(prev, nxt)
    f1, _, _ = oracle.roi_mask(prev, nxt, stabilize=True)
    c = (slice(24, -24), slice(24, -24))
    assert abs(np.median(f0[c][..., 0]) + 3) < 0.2 and abs(np.median(f0[c][..., 1]) - 2) < 0.2
    assert np.abs(f1[c]).max() < 0.05
