"""PSF set readers (MAT and TIFF; the PSF sources of Fig. 1) on the CPU."""
import numpy as np
import pytest

from paper_2208_11422_amd import psf_io


def _psf(nz=3, n=4, k=5, seed=0):
    rng = np.random.default_rng(seed)
    return rng.random((nz, n, n, k, k)).astype(np.float32)


@pytest.mark.parametrize("axes", ["uvabz", "zabuv", "abzvu"])
def test_mat_round_trip(tmp_path, axes):
    psf = _psf()
    p = str(tmp_path / "psf.mat")
    psf_io.save_psf_mat(p, psf, axes=axes)
    got = psf_io.load_psf_mat(p, axes=axes)
    assert got.dtype == np.float32 and got.flags.c_contiguous
    np.testing.assert_array_equal(got, psf)


def test_mat_matlab_layout(tmp_path):
    """A file written the way MATLAB toolboxes store H(u, v, a, b, z): element
    (u, v, a, b, z) of the stored array lands at psf[z][a][b][u][v]."""
    from scipy import io as sio

    nz, n, k = 2, 3, 5
    stored = np.zeros((k, k, n, n, nz))
    for idx in np.ndindex(stored.shape):
        u, v, a, b, z = idx
        stored[idx] = u + 10 * v + 100 * a + 1000 * b + 10000 * z
    p = str(tmp_path / "h.mat")
    sio.savemat(p, {"H": stored, "Ht": stored[..., :1]})
    got = psf_io.load_psf_mat(p, var="H")
    z, a, b, u, v = np.indices(got.shape)
    np.testing.assert_array_equal(got, u + 10 * v + 100 * a + 1000 * b + 10000 * z)


def test_mat_variable_choice(tmp_path):
    from scipy import io as sio

    p = str(tmp_path / "two.mat")
    sio.savemat(p, {"H": np.ones((3, 3, 2, 2, 1)), "G": np.ones((3, 3, 2, 2, 1))})
    with pytest.raises(ValueError, match="name the PSF variable"):
        psf_io.load_psf_mat(p)
    assert psf_io.load_psf_mat(p, var="G").shape == (1, 2, 2, 3, 3)
    with pytest.raises(KeyError):
        psf_io.load_psf_mat(p, var="X")


def test_mat_rejects_hdf5(tmp_path):
    p = tmp_path / "v73.mat"
    p.write_bytes(b"\x89HDF\r\n\x1a\n" + bytes(200))
    with pytest.raises(ValueError, match="7.3"):
        psf_io.load_psf_mat(str(p))


@pytest.mark.parametrize("order", ["zab", "abz", "bza"])
def test_tiff_round_trip(tmp_path, order):
    psf = _psf(nz=2, n=3, k=7, seed=1)
    p = str(tmp_path / "psf.tif")
    psf_io.save_psf_tiff(p, psf, page_order=order)
    got = psf_io.load_psf_tiff(p, nnum=3, nz=2, page_order=order)
    np.testing.assert_array_equal(got, psf)


def test_tiff_page_meaning(tmp_path):
    """Page i of a 'zab' stack is psf[z][a][b] with i = (z * n + a) * n + b."""
    from PIL import Image

    nz, n, k = 2, 2, 3
    pages = [Image.fromarray(np.full((k, k), float(i), np.float32), mode="F")
             for i in range(nz * n * n)]
    p = str(tmp_path / "pages.tif")
    pages[0].save(p, save_all=True, append_images=pages[1:])
    got = psf_io.load_psf_tiff(p, nnum=n, nz=nz)
    for z in range(nz):
        for a in range(n):
            for b in range(n):
                assert np.all(got[z, a, b] == (z * n + a) * n + b)


def test_tiff_page_count_checked(tmp_path):
    psf = _psf(nz=2, n=2, k=3)
    p = str(tmp_path / "psf.tif")
    psf_io.save_psf_tiff(p, psf)
    with pytest.raises(ValueError, match="pages"):
        psf_io.load_psf_tiff(p, nnum=2, nz=3)


def test_check_psf_rejects():
    with pytest.raises(ValueError):
        psf_io.check_psf(np.ones((2, 2, 2, 4, 4)))      # even K
    with pytest.raises(ValueError):
        psf_io.check_psf(np.ones((2, 2, 3, 5, 5)))      # unequal phases
    with pytest.raises(ValueError):
        psf_io.check_psf(np.ones((2, 2, 5, 5)))         # rank
    bad = np.ones((1, 1, 1, 3, 3))
    bad[0, 0, 0, 1, 1] = np.nan
    with pytest.raises(ValueError):
        psf_io.check_psf(bad)
