"""Pins for the oracle's light-field projections (CPU only).

The forward projection is fixed by two facts that do not come from the oracle:
a single bright voxel must image to its own PSF, centred on its own pixel
(that is what a PSF is), and the projection is linear.  The back projection
is fixed by being the adjoint.  The Nnum = 1 case is an ordinary sum of 2-D
convolutions and is checked against scipy."""
import numpy as np
import pytest
from scipy.signal import convolve2d

import oracle
from lfrl_synth import gaussian_psf


def random_psf(nz, n, k, seed):
    """Asymmetric random kernels, so a flipped or transposed tap index fails."""
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 1.0, size=(nz, n, n, k, k)).astype(np.float32)


def place(psf, j, r, s, h, w):
    """Image of a unit point source at voxel (j, r, s), built by slicing the
    kernel into an empty image (cropped at the borders)."""
    nz, n, _, k, _ = psf.shape
    c0 = (k - 1) // 2
    big = np.zeros((h + 2 * k, w + 2 * k))
    big[k + r - c0:k + r - c0 + k, k + s - c0:k + s - c0 + k] += psf[j, r % n, s % n]
    return big[k:k + h, k:k + w]


@pytest.mark.parametrize("n,k", [(3, 7), (4, 5), (5, 9)])
def test_delta_voxel_images_to_its_psf(n, k):
    nz, ly, lx = 2, 4, 5
    h, w = n * ly, n * lx
    psf = random_psf(nz, n, k, seed=1)
    for (j, r, s) in [(0, h // 2, w // 2), (1, h // 2 + 1, w // 2 - 1), (1, 0, 0),
                      (0, h - 1, w - 2), (1, 2, w - 1)]:
        x = np.zeros((nz, h, w))
        x[j, r, s] = 1.0
        got = oracle.forward(psf, x)
        np.testing.assert_array_equal(got, place(psf, j, r, s, h, w))


def test_interior_delta_reproduces_whole_kernel():
    n, k, nz = 3, 7, 2
    h, w = 30, 33
    psf = random_psf(nz, n, k, seed=2)
    c0 = (k - 1) // 2
    j, r, s = 1, 14, 16
    x = np.zeros((nz, h, w))
    x[j, r, s] = 1.0
    img = oracle.forward(psf, x)
    np.testing.assert_array_equal(img[r - c0:r + c0 + 1, s - c0:s + c0 + 1],
                                  psf[j, r % n, s % n].astype(np.float64))
    assert img.sum() == pytest.approx(psf[j, r % n, s % n].astype(np.float64).sum(), rel=1e-15)


def test_superposition_of_point_sources():
    n, k, nz = 3, 7, 3
    h, w = 12, 15
    psf = random_psf(nz, n, k, seed=3)
    rng = np.random.default_rng(4)
    x = np.zeros((nz, h, w))
    expect = np.zeros((h, w))
    for _ in range(12):
        j, r, s = rng.integers(nz), rng.integers(h), rng.integers(w)
        a = rng.uniform(0.1, 2.0)
        x[j, r, s] += a
    for j, r, s in zip(*np.nonzero(x)):
        expect += x[j, r, s] * place(psf, j, r, s, h, w)
    np.testing.assert_allclose(oracle.forward(psf, x), expect, rtol=1e-13, atol=1e-13)


def test_nnum1_is_sum_of_2d_convolutions():
    nz, k, h, w = 3, 9, 17, 20
    psf = random_psf(nz, 1, k, seed=5)
    rng = np.random.default_rng(6)
    x = rng.uniform(0, 1, size=(nz, h, w))
    y = rng.uniform(0, 1, size=(h, w))
    want_f = sum(convolve2d(x[j], psf[j, 0, 0].astype(np.float64), mode="same") for j in range(nz))
    np.testing.assert_allclose(oracle.forward(psf, x), want_f, rtol=1e-12, atol=1e-12)
    want_b = np.stack([convolve2d(y, psf[j, 0, 0, ::-1, ::-1].astype(np.float64), mode="same")
                       for j in range(nz)])
    np.testing.assert_allclose(oracle.backward(psf, y), want_b, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("n,k,ly,lx,nz", [(3, 7, 4, 5, 2), (5, 25, 3, 4, 2), (2, 3, 6, 3, 4)])
def test_adjointness(n, k, ly, lx, nz):
    h, w = n * ly, n * lx
    psf = random_psf(nz, n, k, seed=7)
    rng = np.random.default_rng(8)
    x = rng.normal(size=(nz, h, w))
    y = rng.normal(size=(h, w))
    lhs = np.sum(oracle.forward(psf, x) * y)
    rhs = np.sum(x * oracle.backward(psf, y))
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_dense_matrix_transpose():
    """Build A column by column from deltas and A^T column by column from image
    deltas; the two matrices must be transposes of each other exactly."""
    n, k, nz, h, w = 3, 5, 2, 6, 6
    psf = random_psf(nz, n, k, seed=9)
    nv = nz * h * w
    a = np.zeros((h * w, nv))
    for i in range(nv):
        x = np.zeros(nv)
        x[i] = 1.0
        a[:, i] = oracle.forward(psf, x.reshape(nz, h, w)).ravel()
    at = np.zeros((nv, h * w))
    for p in range(h * w):
        y = np.zeros(h * w)
        y[p] = 1.0
        at[:, p] = oracle.backward(psf, y.reshape(h, w)).ravel()
    np.testing.assert_array_equal(a.T, at)


def test_lenslet_translation_equivariance():
    n, k, nz = 3, 7, 2
    ly, lx = 8, 9
    h, w = n * ly, n * lx
    psf = random_psf(nz, n, k, seed=10)
    rng = np.random.default_rng(11)
    x = np.zeros((nz, h, w))
    x[:, 9:12, 9:15] = rng.uniform(size=(nz, 3, 6))
    dy, dx = 2, 1
    xs = np.roll(np.roll(x, n * dy, axis=1), n * dx, axis=2)
    a = oracle.forward(psf, x)
    b = oracle.forward(psf, xs)
    np.testing.assert_allclose(b[n * dy:, n * dx:], a[:h - n * dy, :w - n * dx], rtol=1e-14, atol=1e-14)


def test_sampled_forms_match_full_forms():
    n, k, nz, h, w = 3, 7, 2, 12, 15
    psf = random_psf(nz, n, k, seed=12)
    rng = np.random.default_rng(13)
    x = rng.uniform(size=(nz, h, w))
    y = rng.uniform(size=(h, w))
    full_f = oracle.forward(psf, x)
    full_b = oracle.backward(psf, y)
    rr, ss = rng.integers(0, h, 40), rng.integers(0, w, 40)
    jj = rng.integers(0, nz, 40)
    np.testing.assert_allclose(oracle.forward_at(psf, x, rr, ss), full_f[rr, ss], rtol=1e-13)
    np.testing.assert_allclose(oracle.backward_at(psf, y, jj, rr, ss), full_b[jj, rr, ss], rtol=1e-13)


def test_unit_sum_psf_conserves_flux_in_the_interior():
    n, k, nz = 5, 25, 5
    psf = gaussian_psf(n, nz, k, seed=11)
    h = w = 5 * 14
    x = np.zeros((nz, h, w))
    x[:, 30:40, 30:40] = 1.0
    img = oracle.forward(psf, x)
    assert img.sum() == pytest.approx(x.sum(), rel=1e-6)  # float32 taps: unit sum to ~1e-7


def test_sum_rule_matches_sensitivity():
    n, k, nz, h, w = 3, 7, 2, 9, 12
    psf = random_psf(nz, n, k, seed=14)
    rng = np.random.default_rng(15)
    x = rng.uniform(size=(nz, h, w))
    c = oracle.sensitivity(psf, h, w)
    assert oracle.forward(psf, x).sum() == pytest.approx(np.sum(c * x), rel=1e-12)


def test_psf_normalisation():
    """Every kernel sums to 1 after normalisation (float32 rounding of each tap
    bounds the error), a scaled copy normalises to the same taps, and a kernel
    with no positive weight is kept unchanged."""
    rng = np.random.default_rng(41)
    psf = rng.uniform(0.0, 1.0, size=(2, 3, 3, 7, 7)).astype(np.float32)
    psf *= rng.uniform(0.1, 50.0, size=(2, 3, 3, 1, 1)).astype(np.float32)
    psf[1, 2, 0] = 0.0
    out = oracle.normalize_psf(psf)
    sums = out.astype(np.float64).sum(axis=(-2, -1))
    live = np.ones((2, 3, 3), dtype=bool)
    live[1, 2, 0] = False
    np.testing.assert_allclose(sums[live], 1.0, atol=49 * 2 ** -24)
    np.testing.assert_array_equal(out[1, 2, 0], 0.0)
    again = oracle.normalize_psf(out * np.float32(4.0))
    np.testing.assert_array_equal(again[live], out[live])


@pytest.mark.parametrize("win", [(0, 9, 0, 12), (5, 17, 8, 20), (-4, 3, 25, 40), (10, 30, -2, 6),
                                 (0, 24, 0, 30), (3, 3, 0, 5)])
def test_window_form_matches_full_form(win):
    """The windowed forward projection is the full projection cropped to the
    window (zero where the window leaves the image), for windows inside, on
    the border of and partly outside the image, and an empty one; the delta
    pins above fix the full form."""
    n, k, nz = 3, 9, 3
    h, w = 24, 30
    psf = random_psf(nz, n, k, seed=31)
    x = np.random.default_rng(32).uniform(0.0, 1.0, size=(nz, h, w))
    x[1, 5:9, :] = 0.0  # zero voxels are skipped by the scatter form
    full = oracle.forward(psf, x)
    r0, r1, s0, s1 = win
    want = np.zeros((r1 - r0, s1 - s0))
    rr = np.arange(r0, r1)[:, None]
    ss = np.arange(s0, s1)[None, :]
    inside = (rr >= 0) & (rr < h) & (ss >= 0) & (ss < w)
    want[inside] = full[np.clip(rr, 0, h - 1), np.clip(ss, 0, w - 1)][inside]
    got = oracle.forward_window(psf, x, r0, r1, s0, s1)
    np.testing.assert_allclose(got, want, rtol=1e-13, atol=1e-13)
