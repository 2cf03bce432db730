"""The seeded input generators: reproducible, unit-sum PSFs, sparse beads."""
import hashlib

import numpy as np
import pytest

import lfrl_synth as S


def digest(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def test_gaussian_psf_reproducible_and_unit_sum():
    a = S.gaussian_psf(5, 5, 25, seed=11)
    b = S.gaussian_psf(5, 5, 25, seed=11)
    assert a.shape == (5, 5, 5, 25, 25) and a.dtype == np.float32
    assert digest(a) == digest(b)
    assert digest(a) != digest(S.gaussian_psf(5, 5, 25, seed=12))
    sums = a.astype(np.float64).sum(axis=(-2, -1))
    np.testing.assert_allclose(sums, 1.0, atol=1e-6)
    assert (a >= 0).all()


def test_gaussian_psf_parallax_moves_the_centroid():
    p = S.gaussian_psf(5, 5, 25, seed=1, jitter=0.0).astype(np.float64)
    u = np.arange(25)
    cent = (p.sum(axis=-1) * u).sum(axis=-1)     # row centroid [j][a][b]
    # plane j=4 is z=+2: row phase a=4 is shifted by 0.5*(4-2)*2 = +2 pixels
    assert cent[4, 4, 0] == pytest.approx(12 + 2.0, abs=0.01)  # truncation at the support edge biases it slightly
    assert cent[0, 4, 0] == pytest.approx(12 - 2.0, abs=0.01)  # truncation at the support edge biases it slightly
    assert cent[2, 4, 0] == pytest.approx(12.0, abs=0.01)  # truncation at the support edge biases it slightly


def test_disk_psf_small():
    p = S.disk_psf(3, 3, 31, seed=2, r0=2.0, r_slope=2.0)
    assert p.shape == (3, 3, 3, 31, 31)
    np.testing.assert_allclose(p.astype(np.float64).sum(axis=(-2, -1)), 1.0, atol=1e-6)
    # the in-focus plane is more compact than the defocused ones
    assert p[1].max() > p[0].max()


def test_bead_volume_sparse_and_reproducible():
    v = S.bead_volume(5, 55, 55, 20, seed=12)
    assert v.shape == (5, 55, 55)
    assert digest(v) == digest(S.bead_volume(5, 55, 55, 20, seed=12))
    assert (v >= 0).all() and v.max() <= 20
    assert (v == 0).mean() > 0.5


def test_filaments_add_signal():
    v = S.bead_volume(4, 40, 40, 0, seed=1)
    f = S.add_filaments(v, 2, seed=3)
    assert f.sum() > 0 and (f >= 0).all()


def test_measure_counts():
    clean = np.random.default_rng(0).uniform(0.0, 1.0, size=(30, 30))
    y = S.measure(clean, 1000.0, 10.0, seed=13)
    assert y.dtype == np.float32
    assert np.all(y >= 10.0)
    assert np.all(np.mod(y - 10.0, 1.0) == 0)      # integer counts on the background
    assert digest(y) == digest(S.measure(clean, 1000.0, 10.0, seed=13))


def test_bead_splats_rebuild_the_bead_volume():
    import numpy as np
    import lfrl_synth as S
    for args in [(5, 40, 50, 30, 3), (3, 9, 12, 40, 4)]:
        v = S.bead_volume(*args, as_float64=True)
        idx, val = S.bead_splats(*args)
        z = np.zeros(v.size)
        np.add.at(z, idx, val)
        assert np.array_equal(z.reshape(v.shape), v)


def test_serving_request_specs():
    import lfrl_synth as S
    a = S.serving_requests(200)
    assert a == S.serving_requests(200)
    seen = set()
    for r in a:
        n, nz = S.SERVING["sets"][r["set"]][:2]
        assert (r["nnum"], r["nz"]) == (n, nz)
        assert r["h"] == r["w"] == n * r["lenslets"]
        assert 363 <= r["h"] <= 900
        seen.add(r["set"])
    assert seen == {0, 1, 2, 3}
    t = S.poisson_arrivals(1000, 50.0)
    assert (t[1:] > t[:-1]).all()
    assert abs(t[-1] / 1000 - 1 / 50.0) < 0.2 / 50.0
