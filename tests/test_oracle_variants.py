"""Pins for the oracle's variants of the update, the start volume, the metric
and the stop rule (CPU only).

The paper names none of these variants; each is pinned by what fixes it
mathematically:

* background b in the image model A x + b: the update is still EM for Poisson
  data with mean A x + b, so a consistent solution is a fixed point and the
  likelihood never decreases; with one depth and Nnum = 1 it is 2-D RL with a
  background, written here with scipy's convolution;
* ISRA, x * A^T y / A^T(A x + b): a multiplicative majorise-minimise step for
  non-negative least squares, so a consistent solution is a fixed point, the
  squared residual never increases and the KKT conditions hold at
  convergence; the 2-D special case again goes through scipy;
* without a background both updates are unchanged when x^0 is scaled;
* the back projection start is A^T y (the dense transpose of A, built from
  deltas, and the 2-D correlation);
* the rectangle and whole-matrix regions, the region-only norm and the
  spectral norm against closed forms built through scipy's inverse DCT
  (tests/golden/metric_variants.json), and the spectral norm of a rank-one
  image against the Frobenius norm;
* the window-mean stop rule against worked sequences and against the identity
  mean(e_{k-w+1..k}) < mean(e_{k-w..k-1})  <=>  e_k < e_{k-w}.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy.fft import idctn
from scipy.signal import convolve2d

import oracle
from lfrl_synth import bead_volume, gaussian_psf, measure

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "metric_variants.json")


def golden():
    with open(GOLDEN) as f:
        return json.load(f)


def small_problem(seed=0, n=3, ly=6, nz=3, k=9):
    psf = gaussian_psf(n, nz, k, seed=seed, sigma0=0.8)
    h = w = n * ly
    x_true = bead_volume(nz, h, w, 6, seed + 1).astype(np.float64) + 0.01
    y = measure(oracle.forward(psf, x_true), 500.0, 2.0, seed + 2)
    return psf, x_true, y.astype(np.float64)


# --------------------------------------------------------------------------
# background term
# --------------------------------------------------------------------------
def test_background_consistent_solution_is_fixed_point():
    psf, x_true, _ = small_problem(seed=11)
    b = 3.5
    y = oracle.forward(psf, x_true) + b
    x1 = oracle.rl(psf, y, 1, x0=x_true, background=b)
    np.testing.assert_allclose(x1, x_true, rtol=1e-12)
    # without the background term in the model the same data is not a fixed point
    assert np.max(np.abs(oracle.rl(psf, y, 1, x0=x_true) / x_true - 1)) > 1e-3


def test_background_loglik_monotone_and_nonnegative():
    psf, _, y = small_problem(seed=12)
    b = 2.0
    xs = oracle.rl(psf, y, 10, keep_all=True, background=b)
    ll = [oracle.poisson_loglik(y, oracle.forward(psf, x) + b) for x in xs]
    for x in xs:
        assert (x >= 0).all()
    assert all(q >= p - 1e-9 * abs(p) for p, q in zip(ll, ll[1:]))
    assert ll[-1] > ll[0]


def test_background_plain_2d_special_case():
    rng = np.random.default_rng(14)
    k, h, w, b = 5, 17, 21, 0.7
    psf = rng.uniform(0, 1, size=(1, 1, 1, k, k)).astype(np.float32)
    y = rng.uniform(1, 10, size=(h, w))
    hk = psf[0, 0, 0].astype(np.float64)
    flip = hk[::-1, ::-1]
    x = np.ones((h, w))
    norm = convolve2d(np.ones((h, w)), flip, mode="same")
    for _ in range(4):
        est = convolve2d(x, hk, mode="same") + b
        x = x * convolve2d(y / est, flip, mode="same") / norm
    np.testing.assert_allclose(oracle.rl(psf, y, 4, background=b)[0], x, rtol=1e-11)


# --------------------------------------------------------------------------
# ISRA
# --------------------------------------------------------------------------
@pytest.mark.parametrize("b", [0.0, 1.5])
def test_isra_consistent_solution_is_fixed_point(b):
    psf, x_true, _ = small_problem(seed=21)
    y = oracle.forward(psf, x_true) + b
    x1 = oracle.rl(psf, y, 1, x0=x_true, update="isra", background=b)
    np.testing.assert_allclose(x1, x_true, rtol=1e-12)


@pytest.mark.parametrize("b", [0.0, 2.0])
def test_isra_residual_never_increases(b):
    psf, _, y = small_problem(seed=22)
    xs = oracle.rl(psf, y, 12, keep_all=True, update="isra", background=b)
    res = [float(np.sum((y - oracle.forward(psf, x) - b) ** 2)) for x in xs]
    for x in xs:
        assert (x >= 0).all()
    assert all(q <= p * (1 + 1e-12) for p, q in zip(res, res[1:]))
    assert res[-1] < 0.5 * res[0]


def test_isra_kkt_at_convergence():
    """Non-negative least squares: the gradient A^T(A x + b - y) vanishes where x
    stays clearly positive and is >= 0 where x has gone to 0."""
    rng = np.random.default_rng(23)
    n, nz, k = 2, 1, 3
    psf = rng.uniform(0.2, 1.0, size=(nz, n, n, k, k)).astype(np.float32)
    h = w = 6
    b = 0.3
    x_true = rng.uniform(0.5, 2.0, size=(nz, h, w))
    y = (oracle.forward(psf, x_true) + b) * rng.uniform(0.95, 1.05, size=(h, w))
    x = oracle.rl(psf, y, 20000, update="isra", background=b)
    grad = oracle.backward(psf, oracle.forward(psf, x) + b - y)
    scale = oracle.backward(psf, y)
    big = x > 1e-2 * x.max()
    assert np.max(np.abs(grad[big] / scale[big])) < 1e-4
    assert (grad[~big] > -1e-4 * scale[~big]).all()


def test_isra_plain_2d_special_case():
    rng = np.random.default_rng(24)
    k, h, w, b = 7, 19, 16, 0.4
    psf = rng.uniform(0, 1, size=(1, 1, 1, k, k)).astype(np.float32)
    y = rng.uniform(1, 10, size=(h, w))
    hk = psf[0, 0, 0].astype(np.float64)
    flip = hk[::-1, ::-1]
    x = np.ones((h, w))
    num = convolve2d(y, flip, mode="same")
    for _ in range(5):
        den = convolve2d(convolve2d(x, hk, mode="same") + b, flip, mode="same")
        x = x * num / den
    np.testing.assert_allclose(oracle.rl(psf, y, 5, update="isra", background=b)[0], x,
                               rtol=1e-11)


@pytest.mark.parametrize("update", ["rl", "isra"])
def test_updates_ignore_the_scale_of_the_start(update):
    psf, _, y = small_problem(seed=25)
    rng = np.random.default_rng(26)
    x0 = rng.uniform(0.5, 2.0, size=(psf.shape[0],) + y.shape)
    a = oracle.rl(psf, y, 2, x0=x0, update=update)
    b = oracle.rl(psf, y, 2, x0=37.0 * x0, update=update)
    np.testing.assert_allclose(a, b, rtol=1e-12)
    # a background breaks the homogeneity of A x + b
    c = oracle.rl(psf, y, 2, x0=37.0 * x0, update=update, background=1.0)
    assert np.max(np.abs(c / a - 1)) > 1e-3


# --------------------------------------------------------------------------
# back projection start
# --------------------------------------------------------------------------
def test_backprojection_start_is_dense_transpose():
    rng = np.random.default_rng(31)
    n, k, nz, h, w = 2, 5, 2, 6, 6
    psf = rng.uniform(0.0, 1.0, size=(nz, n, n, k, k)).astype(np.float32)
    nv = nz * h * w
    a = np.zeros((h * w, nv))
    for i in range(nv):
        x = np.zeros(nv)
        x[i] = 1.0
        a[:, i] = oracle.forward(psf, x.reshape(nz, h, w)).ravel()
    y = rng.uniform(0, 5, size=(h, w))
    x0 = oracle.initial_volume(psf, y, "backprojection")
    np.testing.assert_allclose(x0.ravel(), a.T @ y.ravel(), rtol=1e-13)


def test_backprojection_start_plain_2d_is_correlation():
    rng = np.random.default_rng(32)
    k, h, w = 5, 12, 15
    psf = rng.uniform(0, 1, size=(1, 1, 1, k, k)).astype(np.float32)
    y = rng.uniform(0, 3, size=(h, w))
    flip = psf[0, 0, 0].astype(np.float64)[::-1, ::-1]
    np.testing.assert_allclose(oracle.initial_volume(psf, y, "backprojection")[0],
                               convolve2d(y, flip, mode="same"), rtol=1e-12)


# --------------------------------------------------------------------------
# metric variants
# --------------------------------------------------------------------------
@pytest.mark.parametrize("case", golden()["rectangle_counts"])
def test_rectangle_sizes(case):
    m = oracle.region_mask(case["h"], case["w"], case["xs"], case["ys"], "rectangle")
    assert int(m.sum()) == case["count"]


@pytest.mark.parametrize("case", golden()["equal_coefficients"])
def test_region_closed_forms(case):
    h, w = case["h"], case["w"]
    f = np.zeros((h, w))
    for (v, u), sgn in zip(case["positions"], case["signs"]):
        f[v, u] = 1.25 * sgn
    img = idctn(f, type=2, norm="ortho")
    e = oracle.dct_entropy(img, case["xs"], case["ys"], region=case["region"])
    assert e == pytest.approx(case["value"], rel=1e-12)
    k = len(case["positions"])
    g = h * w if case["region"] == "whole" else case["xs"] * case["ys"]
    assert case["value"] == pytest.approx(math.sqrt(k) * math.log2(k) / (2 * g), rel=1e-12)


def test_region_norm_closed_form():
    c = golden()["region_norm"]
    f = np.zeros((c["h"], c["w"]))
    for v, u in c["inside"]:
        f[v, u] = 1.0
    for i, (v, u) in enumerate(c["outside"]):
        f[v, u] = -1.0 if i % 2 == 0 else 1.0
    img = idctn(f, type=2, norm="ortho")
    assert oracle.dct_entropy(img, c["xs"], c["ys"], norm="full") == pytest.approx(
        c["full"], rel=1e-12)
    assert oracle.dct_entropy(img, c["xs"], c["ys"], norm="region") == pytest.approx(
        c["region"], rel=1e-12)


def test_region_norm_ignores_energy_outside():
    """Adding coefficients outside the triangle leaves the region-norm entropy
    unchanged and lowers nothing inside; the full-norm entropy changes."""
    rng = np.random.default_rng(41)
    h = w = 24
    xs, ys = 5.0, 6.0
    mask = oracle.triangle_mask(h, w, xs, ys)
    f = np.where(mask, rng.normal(size=(h, w)), 0.0)
    g = f + np.where(mask, 0.0, rng.normal(size=(h, w)))
    e_f = oracle.dct_entropy(idctn(f, type=2, norm="ortho"), xs, ys, norm="region")
    e_g = oracle.dct_entropy(idctn(g, type=2, norm="ortho"), xs, ys, norm="region")
    assert e_g == pytest.approx(e_f, rel=1e-10)
    assert oracle.dct_entropy(idctn(g, type=2, norm="ortho"), xs, ys) != pytest.approx(
        e_f, rel=1e-3)


@pytest.mark.parametrize("region", ["rectangle", "whole"])
@pytest.mark.parametrize("norm", ["full", "region", "spectral"])
def test_variants_scale_invariant_and_zero_for_constants(region, norm):
    img = np.random.default_rng(42).uniform(size=(18, 22))
    e = oracle.dct_entropy(img, 4.0, 3.5, region, norm)
    assert oracle.dct_entropy(9.5 * img, 4.0, 3.5, region, norm) == pytest.approx(e, rel=1e-12)
    assert abs(oracle.dct_entropy(np.full((18, 22), 2.0), 4.0, 3.5, region, norm)) < 1e-12


def test_whole_region_of_a_single_coefficient_is_zero():
    f = np.zeros((10, 14))
    f[3, 7] = 2.0
    assert abs(oracle.dct_entropy(idctn(f, type=2, norm="ortho"), 1.0, 1.0, "whole")) < 1e-14


# --------------------------------------------------------------------------
# window-mean stop rule
# --------------------------------------------------------------------------
@pytest.mark.parametrize("trace,patience,window,want", [
    # s_2 = 2, s_3 = 2.5, s_4 = 2.25: decrease at k = 4; e peaks at k = 2
    ([1, 3, 2, 2.5, 2.4, 2.0], 1, 2, (True, 4, 2)),
    # the raw values dip at k = 3, the means only at k = 7 (3.5 -> 3.3)
    ([1, 3, 2.9, 3.5, 3.4, 3.6, 3.0, 2.0], 1, 2, (True, 7, 6)),
    # means 2, 3, 10/3, 3, 2 from k = 3: decreases at k = 6 and 7
    ([1, 2, 3, 4, 3, 2, 1], 2, 3, (True, 7, 4)),
    # fewer values than the window: no trend yet
    ([1, 2, 1], 1, 4, (False, 3, 2)),
    # window 1 is the plain rule
    ([1, 2, 3, 2.5, 4], 1, 1, (True, 4, 3)),
])
def test_window_stop_rule(trace, patience, window, want):
    assert oracle.stop_decision(trace, patience, window) == want


def test_window_means_decrease_iff_values_w_apart_decrease():
    """Consecutive window means share w - 1 values, so the later one is smaller
    exactly when e_k < e_{k-w}.  Integer traces keep every mean exact."""
    rng = np.random.default_rng(43)
    for _ in range(300):
        w = int(rng.integers(1, 5))
        p = int(rng.integers(1, 3))
        trace = [float(v) for v in rng.integers(0, 6, size=int(rng.integers(0, 14)))]
        run, best, best_e, want = 0, 0, -np.inf, None
        for i, e in enumerate(trace):
            k = i + 1
            if k >= w + 1:
                run = run + 1 if trace[k - 1] < trace[k - 1 - w] else 0
            if e >= best_e:
                best, best_e = k, e
            if run >= p:
                want = (True, k, best)
                break
        if want is None:
            want = (False, len(trace), best)
        assert oracle.stop_decision(trace, p, w) == want


def test_deconvolve_variants_run_through():
    """oracle.deconvolve composes the pieces: ISRA with a background from the back
    projection start, scored on the rectangle with the region norm."""
    psf, _, y = small_problem(seed=51)
    x, best, ran, trace = oracle.deconvolve(psf, y, 6, 3.0, 3.0, update="isra", background=2.0,
                                            init="backprojection", region="rectangle",
                                            norm="region", window=2)
    assert len(trace) == ran and 1 <= best <= ran
    xs = oracle.rl(psf, y, ran, keep_all=True, update="isra", background=2.0,
                   init="backprojection")
    np.testing.assert_allclose(x, xs[best], rtol=1e-15)
    want = [oracle.metric(v, 3.0, 3.0, "rectangle", "region") for v in xs[1:]]
    np.testing.assert_allclose(trace, want, rtol=1e-15)


def test_spectral_norm_closed_form():
    """Two coefficients on the diagonal, 2 and -1: the largest singular value
    is 2 (tests/golden/metric_variants.json)."""
    c = golden()["spectral_norm"]
    f = np.zeros((c["h"], c["w"]))
    for v, u, val in c["coefficients"]:
        f[v, u] = val
    img = idctn(f, type=2, norm="ortho")
    assert oracle.dct_entropy(img, c["xs"], c["ys"], norm="spectral") == pytest.approx(
        c["value"], rel=1e-12)


def test_spectral_norm_of_rank_one_image_is_frobenius():
    """For a rank-one image the spectral and Frobenius norms coincide, so both
    readings give the same entropy; for a generic image the spectral norm is
    smaller and the entropy differs."""
    rng = np.random.default_rng(44)
    a, b = rng.uniform(0.5, 2.0, 20), rng.uniform(0.5, 2.0, 24)
    img = np.outer(a, b)
    for region in ("triangle", "rectangle", "whole"):
        assert oracle.dct_entropy(img, 5.0, 4.0, region, "spectral") == pytest.approx(
            oracle.dct_entropy(img, 5.0, 4.0, region, "full"), rel=1e-12)
    img2 = rng.uniform(size=(20, 24))
    assert oracle.dct_entropy(img2, 5.0, 4.0, norm="spectral") != pytest.approx(
        oracle.dct_entropy(img2, 5.0, 4.0, norm="full"), rel=1e-3)
