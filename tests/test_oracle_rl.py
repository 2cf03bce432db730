"""Pins for the oracle's Richardson-Lucy loop (CPU only).

Richardson-Lucy is the EM algorithm for Poisson data, which fixes properties
that any correct implementation has and that the usual slips break:

* flux: <A^T 1, x^k> equals the total counts over pixels with positive
  prediction (dropping the division by A^T 1 breaks it at the borders);
* the Poisson log-likelihood never decreases (inverting the ratio breaks it);
* a consistent exact solution is a fixed point;
* at convergence the KKT conditions of the likelihood hold;
* with one depth and Nnum = 1 it is plain 2-D Richardson-Lucy, written here
  with scipy's 2-D convolution.
"""
import numpy as np
import pytest
from scipy.signal import convolve2d

import oracle
from lfrl_synth import bead_volume, gaussian_psf, measure


def small_problem(seed=0, n=3, ly=6, nz=3, k=9):
    psf = gaussian_psf(n, nz, k, seed=seed, sigma0=0.8)
    h = w = n * ly
    x_true = bead_volume(nz, h, w, 6, seed + 1).astype(np.float64) + 0.01
    y = measure(oracle.forward(psf, x_true), 500.0, 2.0, seed + 2)
    return psf, x_true, y.astype(np.float64)


def test_flux_invariant_every_iteration():
    psf, _, y = small_problem()
    h, w = y.shape
    c = oracle.sensitivity(psf, h, w)
    xs = oracle.rl(psf, y, 6, keep_all=True)
    for k in range(1, len(xs)):
        yhat = oracle.forward(psf, xs[k - 1])
        want = y[yhat > 0].sum()
        assert np.sum(c * xs[k]) == pytest.approx(want, rel=1e-12)


def test_nonnegative_and_loglik_monotone():
    psf, _, y = small_problem(seed=5)
    xs = oracle.rl(psf, y, 10, keep_all=True)
    ll = [oracle.poisson_loglik(y, oracle.forward(psf, x)) for x in xs]
    for x in xs:
        assert (x >= 0).all()
    assert all(b >= a - 1e-9 * abs(a) for a, b in zip(ll, ll[1:]))
    assert ll[-1] > ll[0]


def test_exact_solution_is_fixed_point():
    psf, x_true, _ = small_problem(seed=9)
    y = oracle.forward(psf, x_true)
    x1 = oracle.rl(psf, y, 1, x0=x_true)
    np.testing.assert_allclose(x1, x_true, rtol=1e-12)


def test_kkt_at_convergence():
    """For a tiny, well-determined problem many iterations drive the KKT ratio
    A^T(y / A x) / A^T 1 to 1 wherever x stays clearly positive."""
    rng = np.random.default_rng(3)
    n, nz, k = 2, 1, 3
    psf = rng.uniform(0.2, 1.0, size=(nz, n, n, k, k)).astype(np.float32)
    h = w = 6
    x_true = rng.uniform(0.5, 2.0, size=(nz, h, w))
    y = oracle.forward(psf, x_true) * rng.uniform(0.9, 1.1, size=(h, w))
    x = oracle.rl(psf, y, 3000)
    c = oracle.sensitivity(psf, h, w)
    g = oracle.backward(psf, y / oracle.forward(psf, x)) / c
    big = x > 1e-3 * x.max()
    assert np.max(np.abs(g[big] - 1.0)) < 1e-3


def test_plain_2d_rl_special_case():
    rng = np.random.default_rng(4)
    k, h, w = 7, 20, 23
    psf = rng.uniform(0, 1, size=(1, 1, 1, k, k)).astype(np.float32)
    y = rng.uniform(1, 10, size=(h, w))
    hk = psf[0, 0, 0].astype(np.float64)
    flip = hk[::-1, ::-1]
    x = np.ones((h, w))
    norm = convolve2d(np.ones((h, w)), flip, mode="same")
    for _ in range(4):
        est = convolve2d(x, hk, mode="same")
        x = x * convolve2d(y / est, flip, mode="same") / norm
    np.testing.assert_allclose(oracle.rl(psf, y, 4)[0], x, rtol=1e-11)


def test_zero_prediction_and_zero_sensitivity_rules():
    """Pixels the volume cannot reach get ratio 0; voxels that reach no pixel
    (a zero kernel) are set to 0 rather than divided by zero."""
    n, nz, k = 2, 2, 3
    psf = np.zeros((nz, n, n, k, k), dtype=np.float32)
    psf[0, :, :, 1, 1] = 1.0           # plane 0: identity imaging
    h = w = 4                          # plane 1: all-zero kernels -> c = 0
    y = np.arange(1.0, 17.0).reshape(h, w)
    x = oracle.rl(psf, y, 2)
    np.testing.assert_array_equal(x[1], 0.0)
    np.testing.assert_allclose(x[0], y, rtol=1e-15)


@pytest.mark.parametrize("win", [(0, 6, 0, 6), (9, 15, 3, 12), (14, 18, 20, 24)])
def test_windowed_iterates_match_whole_volume_iterates(win):
    """rl_window (iterates evaluated only where the next step reads them)
    equals the whole-volume iteration cropped to the window, for corner,
    interior and edge windows over three iterations, with and without a
    background."""
    n, k, nz = 3, 7, 2
    h, w = 18, 24
    psf = np.random.default_rng(41).uniform(0.0, 1.0, size=(nz, n, n, k, k)).astype(np.float32)
    y = np.random.default_rng(42).uniform(1.0, 50.0, size=(h, w))
    r0, r1, s0, s1 = win
    for bg in (0.0, 3.0):
        full = oracle.rl(psf, y, 3, keep_all=True, background=bg)
        xs, c = oracle.rl_window(psf, y, 3, r0, r1, s0, s1, background=bg)
        np.testing.assert_allclose(c, oracle.sensitivity(psf, h, w)[:, r0:r1, s0:s1], rtol=1e-13)
        for m in range(3):
            np.testing.assert_allclose(xs[m], full[m + 1][:, r0:r1, s0:s1], rtol=1e-12)
