"""Pins of the wave-optics PSF oracle (oracle/optics.py) against what
mathematics and optics fix independently of it: closed forms of the Debye
integral, the paraxial Airy and defocus laws, the Gaussian-beam solution of
Fresnel propagation, energy conservation, the focus of a square lens, the
lenslet geometry built from scratch in global coordinates, and the symmetries
of the light-field PSF.  Everything else about the end-to-end PSF values is
parity unpinned: the paper prints no PSF equations or values."""
import numpy as np
import pytest
from scipy import optimize, special

from oracle import optics as O


def small_optics(**kw):
    base = dict(wavelength=0.52, na=0.5, n_medium=1.0, mag=20.0, d_ml=50.0, f_ml=1000.0,
                nnum=5, ksize=25, osr=3, nquad=256)
    base.update(kw)
    return O.Optics(**base)


def test_nice_size():
    assert [O.nice_size(n) for n in (1, 7, 75, 765, 1275, 1785)] == [1, 8, 75, 768, 1280, 1800]


def test_debye_on_axis_in_focus_closed_form():
    """At r = 0, z = 0 the integral is int_0^alpha sqrt(cos t) sin t dt
    = (2/3) (1 - cos^(3/2) alpha), at any aperture."""
    for na, n in ((0.5, 1.0), (0.95, 1.0), (1.2, 1.33)):
        o = small_optics(na=na, n_medium=n, nquad=64)
        alpha = np.arcsin(na / n)
        want = 2.0 / 3.0 * (1.0 - np.cos(alpha) ** 1.5)
        got = O.debye_nip(np.array([0.0]), 0.0, o)[0]
        assert abs(got - want) <= 1e-13 * want


def test_debye_low_na_airy_pattern():
    """Small aperture, in focus: U(r) / U(0) = 2 J1(q) / q with q = k NA r / M
    (the Airy amplitude; its first zero at 0.61 lambda / NA in object space,
    the Airy unit of Eq. 11)."""
    o = small_optics(na=0.02, n_medium=1.0, mag=10.0, nquad=128)
    k = 2 * np.pi / o.wavelength
    q = np.linspace(0.25, 12.0, 48)
    r = q * o.mag / (k * o.na)
    u = O.debye_nip(r, 0.0, o) / O.debye_nip(np.array([0.0]), 0.0, o)[0]
    airy = 2 * special.j1(q) / q
    assert np.max(np.abs(u - airy)) < 1e-3
    # first zero of the amplitude, in object space
    f = lambda rr: O.debye_nip(np.array([rr]), 0.0, o)[0].real
    r0 = optimize.brentq(f, 0.5 * r[0] * 8, 2.0 * 3.8317 * o.mag / (k * o.na) * 0.75)
    assert r0 / o.mag == pytest.approx(0.6098 * o.wavelength / o.na, rel=2e-3)


def test_debye_low_na_axial_defocus():
    """Small aperture, on axis: |U(0, z)| / |U(0, 0)| = |sin(u/4) / (u/4)| with
    u = 4 k n z sin^2(alpha / 2) (paraxial defocus law)."""
    o = small_optics(na=0.05, n_medium=1.0, nquad=256)
    k = 2 * np.pi / o.wavelength
    alpha = np.arcsin(o.na)
    u0 = O.debye_nip(np.array([0.0]), 0.0, o)[0]
    for z in np.linspace(-4000.0, 4000.0, 17):
        u = 4 * k * z * np.sin(alpha / 2) ** 2
        want = abs(np.sinc(u / (4 * np.pi)))
        got = abs(O.debye_nip(np.array([0.0]), z, o)[0] / u0)
        assert abs(got - want) < 2e-3, (z, got, want)


def test_debye_depth_sign_is_conjugation():
    o = small_optics(nquad=200)
    r = np.linspace(0.0, 300.0, 37)
    np.testing.assert_allclose(O.debye_nip(r, -3.0, o), np.conj(O.debye_nip(r, 3.0, o)),
                               rtol=0, atol=1e-15)


def test_fresnel_gaussian_beam():
    """A Gaussian exp(-|x|^2 / w0^2) propagated over d is
    exp(-|x|^2 / (w0^2 (1 + i d / zR))) / (1 + i d / zR), zR = pi w0^2 / lambda
    (exact for the paraxial transfer function)."""
    n, delta, lam, w0, d = 256, 1.0, 0.5, 8.0, 200.0
    x = (np.arange(n) - n // 2) * delta
    r2 = x[:, None] ** 2 + x[None, :] ** 2
    u0 = np.exp(-r2 / w0 ** 2)
    got = O.fresnel_propagate(u0, delta, lam, d)
    q = 1 + 1j * d / (np.pi * w0 ** 2 / lam)
    want = np.exp(-r2 / (w0 ** 2 * q)) / q
    assert np.linalg.norm(got - want) <= 1e-10 * np.linalg.norm(want)


def test_fresnel_conserves_energy_and_reverses():
    rng = np.random.default_rng(3)
    f = rng.normal(size=(60, 60)) + 1j * rng.normal(size=(60, 60))
    g = O.fresnel_propagate(f, 2.0, 0.5, 700.0)
    assert np.sum(np.abs(g) ** 2) == pytest.approx(np.sum(np.abs(f) ** 2), rel=1e-12)
    back = O.fresnel_propagate(g, 2.0, 0.5, -700.0)
    assert np.max(np.abs(back - f)) < 1e-12


def test_square_lens_focus():
    """A unit plane wave through one square lenslet of side d, propagated over
    its focal length f: the intensity at the focus is (d^2 / (lambda f))^2 and the
    first zero along an axis is lambda f / d away (Fraunhofer pattern).  With
    the opposite lens sign the light would not focus."""
    o = small_optics(nnum=15, d_ml=150.0, f_ml=3000.0, osr=3, ksize=1)
    delta, lam, f, d = o.delta, o.wavelength, o.f_ml, o.d_ml
    n = 1200
    x = (np.arange(n) - n // 2) * delta
    inside = np.abs(x) < d / 2
    ap = (inside[:, None] & inside[None, :]).astype(float)
    lens = np.exp(-1j * np.pi * (x[:, None] ** 2 + x[None, :] ** 2) / (lam * f))
    out = O.fresnel_propagate(ap * lens, delta, lam, f)
    ifocus = np.abs(out[n // 2, n // 2]) ** 2
    want = (ap.sum() * delta ** 2 / (lam * f)) ** 2
    assert ifocus == pytest.approx(want, rel=0.03)
    row = np.abs(out[n // 2, n // 2:]) ** 2
    first_min = np.argmax(np.diff(row) > 0) * delta
    assert first_min == pytest.approx(lam * f / d, abs=delta)
    wrong = O.fresnel_propagate(ap * np.conj(lens), delta, lam, f)
    assert np.abs(wrong[n // 2, n // 2]) ** 2 < 0.01 * ifocus


def test_fresnel_matches_numpy_direct_sum_small():
    """On a tiny periodic grid the FFT transfer function equals the direct sum
    over the periodic impulse response sum_f H(f) exp(2 pi i f x) / N^2."""
    n, delta, lam, d = 12, 3.0, 0.5, 200.0
    rng = np.random.default_rng(9)
    f0 = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    fr = np.fft.fftfreq(n, d=delta)
    h = np.exp(-1j * np.pi * lam * d * (fr[:, None] ** 2 + fr[None, :] ** 2))
    idx = np.arange(n)
    ph = np.exp(2j * np.pi * np.outer(idx, idx) / n)   # [x][f]
    kern = ph @ h @ ph.T / n ** 2                        # periodic impulse response
    want = np.zeros_like(f0)
    for y in range(n):
        for x in range(n):
            want[y, x] = sum(f0[p, q] * kern[(y - p) % n, (x - q) % n]
                             for p in range(n) for q in range(n))
    got = O.fresnel_propagate(f0, delta, lam, d)
    assert np.max(np.abs(got - want)) < 1e-11


def test_lenslet_phase_against_global_grid():
    """The window's lenslet phases equal a lenslet array built in global
    coordinates (lenslet l covers pixels l*N .. l*N + N - 1, centre at
    l*N + (N - 1)/2) sampled around a source pixel, for every phase."""
    for nnum, osr in ((5, 3), (4, 1), (3, 5)):
        o = small_optics(nnum=nnum, d_ml=10.0 * nnum, osr=osr, ksize=11)
        g, _, _ = O.grid_sizes(o)
        hh = (g - 1) // 2
        for a in range(nnum):
            for b in range(nnum):
                r0, s0 = 7 * nnum + a, 9 * nnum + b          # a source pixel with phases (a, b)
                m = np.arange(-hh, hh + 1) / osr
                ys, xs = r0 + m, s0 + m                       # global pixel coordinates
                cy = np.floor((ys + 0.5) / nnum) * nnum + (nnum - 1) / 2
                cx = np.floor((xs + 0.5) / nnum) * nnum + (nnum - 1) / 2
                d2 = ((ys - cy)[:, None] ** 2 + (xs - cx)[None, :] ** 2) * o.pixel ** 2
                want = np.exp(-1j * np.pi * d2 / (o.wavelength * o.f_ml))
                np.testing.assert_allclose(O.lenslet_phase(a, b, o), want, rtol=0, atol=1e-12)


@pytest.fixture(scope="module")
def small_set():
    o = small_optics()
    z = [-4.0, 0.0, 3.0]
    return o, z, O.lf_psf(o, z)


def test_psf_symmetries(small_set):
    """Mirror and transpose symmetry of the light-field PSF: a source mirrored
    about its lenslet's centre column (phase b -> N - 1 - b) images mirrored,
    and swapping the axes swaps the phases."""
    o, z, psf = small_set
    n = o.nnum
    for j in range(len(z)):
        for a in range(n):
            for b in range(n):
                p = psf[j, a, b]
                scale = np.abs(p).max()
                assert np.max(np.abs(psf[j, a, n - 1 - b] - p[:, ::-1])) <= 1e-12 * scale
                assert np.max(np.abs(psf[j, n - 1 - a, b] - p[::-1, :])) <= 1e-12 * scale
                assert np.max(np.abs(psf[j, b, a] - p.T)) <= 1e-12 * scale


def test_psf_one_lenslet_shift(small_set):
    """A source one lenslet further along a row sees the same lenslet array
    around it, so its image is the same pattern shifted by nnum pixels."""
    o, z, psf = small_set
    nip = O.nip_window(z[0], o)
    for a, b in ((0, 0), (1, 3), (4, 2)):
        shifted = O.bin_pixels(O.sensor_field(nip, a + o.nnum, b - o.nnum, o), o)
        np.testing.assert_allclose(shifted, psf[0, a, b], rtol=1e-12, atol=0)


def test_psf_energy_and_positivity(small_set):
    """Energy through the array: the sensor grid holds exactly the energy of
    the native-image-plane window (Parseval, |lens| = 1), and intensities are
    non-negative."""
    o, z, psf = small_set
    assert np.all(psf >= 0)
    g, gf, off = O.grid_sizes(o)
    for j in range(len(z)):
        nip = O.nip_window(z[j], o)
        fld = O.sensor_field(nip, 2, 1, o)
        assert np.sum(np.abs(fld) ** 2) == pytest.approx(np.sum(np.abs(nip) ** 2), rel=1e-12)


def test_psf_unit_sum_and_field_selection(small_set):
    o, z, psf = small_set
    sel = [(1, 0, 4), (2, 3, 3)]
    part = O.lf_psf(o, z, unit_sum=True, fields=sel)
    for j, a, b in sel:
        assert part[j, a, b].sum() == pytest.approx(1.0, abs=1e-13)
        np.testing.assert_allclose(part[j, a, b], psf[j, a, b] / psf[j, a, b].sum(), rtol=1e-13)
    mask = np.ones(part.shape[:3], bool)
    for j, a, b in sel:
        mask[j, a, b] = False
    assert not part[mask].any()


def test_psf_in_focus_light_stays_under_its_lenslet(small_set):
    """Physics sanity (not exact): a source in focus at the centre of its
    lenslet sends most of its light to that lenslet's N x N pixels."""
    o, z, psf = small_set
    n, c0 = o.nnum, (o.ksize - 1) // 2
    p = psf[1, n // 2, n // 2]
    h = n // 2
    assert p[c0 - h:c0 + h + 1, c0 - h:c0 + h + 1].sum() > 0.8 * p.sum()
