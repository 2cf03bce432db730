"""Pins for the oracle's DCT-entropy metric and stop rule (CPU only).

The DCT is checked against scipy's orthonormal DCT-II and against Parseval;
the entropy against closed forms built through scipy's inverse DCT; the region
against hand-counted triangles (tests/golden/metric_closed_forms.json)."""
import json
import math
import os

import numpy as np
import pytest
from scipy.fft import dctn, idctn

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "metric_closed_forms.json")


def golden():
    with open(GOLDEN) as f:
        return json.load(f)


@pytest.mark.parametrize("h,w", [(8, 8), (7, 12), (55, 55), (31, 20)])
def test_dct_matches_scipy_orthonormal_dct2(h, w):
    img = np.random.default_rng(h * w).uniform(size=(h, w))
    np.testing.assert_allclose(oracle.dct2(img), dctn(img, type=2, norm="ortho"),
                               rtol=1e-12, atol=1e-12)


def test_dct_axes_follow_height_and_width():
    """A pattern that varies only along the width puts its energy in row v = 0."""
    h, w = 6, 10
    img = np.tile(np.cos((2 * np.arange(w) + 1) * np.pi * 3 / (2 * w)), (h, 1))
    f = oracle.dct2(img)
    assert abs(f[0, 3]) > 1.0
    f[0, 3] = 0.0
    assert np.max(np.abs(f)) < 1e-12


def test_parseval():
    img = np.random.default_rng(2).uniform(size=(13, 21))
    assert np.sum(oracle.dct2(img) ** 2) == pytest.approx(np.sum(img ** 2), rel=1e-12)


def test_triangle_sizes():
    g = golden()["triangle_counts"]
    for case in g["cases"]:
        m = oracle.triangle_mask(case["h"], case["w"], case["xs"], case["ys"])
        assert int(m.sum()) == case["count"], case


def test_constant_image_has_zero_entropy():
    # only the DC coefficient survives (others are rounding noise of order 1e-16)
    assert abs(oracle.dct_entropy(np.full((20, 30), 3.7), 5.0, 4.0)) < 1e-12


@pytest.mark.parametrize("case", golden()["equal_coefficients"]["cases"])
def test_equal_coefficients_closed_form(case):
    """k coefficients of equal magnitude inside S and nothing else: each p is
    1/sqrt(k), so e = sqrt(k) * log2(k) / (X_S * Y_S)."""
    h, w, xs, ys = case["h"], case["w"], case["xs"], case["ys"]
    f = np.zeros((h, w))
    for (v, u), sgn in zip(case["positions"], case["signs"]):
        f[v, u] = 0.75 * sgn
    img = idctn(f, type=2, norm="ortho")
    k = len(case["positions"])
    assert oracle.dct_entropy(img, xs, ys) == pytest.approx(case["value"], rel=1e-12)
    assert case["value"] == pytest.approx(math.sqrt(k) * math.log2(k) / (xs * ys), rel=1e-12)


def test_energy_outside_region_only_enters_through_the_norm():
    """Two equal coefficients inside S plus two of the same size outside it:
    p = 1/2 for the inside pair, so e = -(2/(X_S Y_S)) * 2 * (1/2) log2(1/2)."""
    h = w = 16
    xs = ys = 4.0
    f = np.zeros((h, w))
    f[0, 1] = f[2, 0] = 1.0
    f[9, 9] = -1.0
    f[15, 3] = 1.0
    img = idctn(f, type=2, norm="ortho")
    assert oracle.dct_entropy(img, xs, ys) == pytest.approx(2.0 / 16.0, rel=1e-12)


def test_scale_invariance():
    img = np.random.default_rng(3).uniform(size=(24, 24))
    e = oracle.dct_entropy(img, 6.0, 6.0)
    assert oracle.dct_entropy(17.5 * img, 6.0, 6.0) == pytest.approx(e, rel=1e-12)


def test_metric_uses_z_maximum_projection():
    rng = np.random.default_rng(4)
    vol = rng.uniform(size=(3, 10, 12))
    assert oracle.metric(vol, 3.0, 2.5) == pytest.approx(
        oracle.dct_entropy(vol.max(axis=0), 3.0, 2.5), rel=1e-15)


@pytest.mark.parametrize("trace,patience,want", [
    ([1, 2, 3, 2.5, 4], 1, (True, 4, 3)),
    ([1, 2, 3, 4, 5], 1, (False, 5, 5)),
    ([3, 2, 5], 1, (True, 2, 1)),
    ([1, 3, 3, 2], 1, (True, 4, 3)),          # a tie is not a decrease
    ([1, 3, 2, 2.5, 2, 1.5], 2, (True, 6, 2)),
    ([1, 3, 2, 2.5, 2, 1.5], 3, (False, 6, 2)),
    ([5], 1, (False, 1, 1)),
    ([], 1, (False, 0, 0)),
])
def test_stop_rule(trace, patience, want):
    assert oracle.stop_decision(trace, patience) == want


def test_cutoff_equations():
    g = golden()["cutoff"]
    xs, ys = oracle.cutoff(g["d_ml"], g["mag"], g["nnum"], g["wavelength"], g["na"],
                           g["h"], g["w"])
    assert xs == pytest.approx(g["xs"], rel=1e-9)
    assert ys == pytest.approx(g["ys"], rel=1e-9)


def test_synthetic_cutoff():
    assert oracle.synthetic_cutoff(5, 1.0, 55, 55) == (5.5, 5.5)
    assert oracle.synthetic_cutoff(15, 2.0, 600, 600) == (10.0, 10.0)
