"""CPU float64 oracle: the light-field PSF computed from optical parameters.

TEST INFRASTRUCTURE ONLY: the test suite and the CPU-baseline leg of the
benchmark use it; the product never imports it, and it imports nothing of the
product.

The paper moves the PSF computation of the light-field deconvolution to the
GPU (sec. 2.1; Fig. 1 makes "computing by specific parameters" the default PSF
source) and integrates the functions of the MATLAB program of Prevedel et al.
2014 (sec. 1), but prints no PSF equations.  The model written out here is the
scalar wave-optics light-field PSF of that line of work (Broxton et al. 2013),
in four steps, each plain and slow:

1. Field of a point source at depth z on the native image plane, from the
   Debye integral of a sine-condition objective (apodisation sqrt(cos t)):
       U(r, z) = int_0^alpha sqrt(cos t) sin t exp(i k n z (1 - cos t))
                             J0(k n r sin t / M) dt,
   alpha = asin(NA / n), k = 2 pi / lambda, r the radius in the image plane
   (object radius times M).  Constant prefactors and the depth-only global
   phase are dropped (they cancel in the unit-sum PSF and in every intensity
   ratio).  The integral is evaluated by Gauss-Legendre quadrature with nquad
   nodes on [0, alpha].
2. The microlens array: every lenslet multiplies the field by the thin-lens
   phase exp(-i pi |x - c|^2 / (lambda f_ml)) about its centre c.
3. Fresnel propagation over f_ml to the sensor with the transfer function
   exp(-i pi lambda f_ml (fx^2 + fy^2)) on a periodic grid (FFT).
4. Intensity |U|^2 summed over the osr x osr samples of every sensor pixel.

Discretisation (the same on both sides of any parity test, and stated in the
design notes): sensor pixel pitch p = d_ml / nnum, sample spacing
delta = p / osr (osr odd); the window is K x K pixels (K odd) centred on the
source pixel, G = K * osr samples per side with the source on the centre
sample; the FFT grid has Gf >= G samples (the smallest 2^a 3^b 5^c), the window
placed at offset (Gf - G) // 2, zero outside it.  The lenslet grid starts at
pixel 0 (pixel row r has phase r mod nnum): a source of row phase a sits a
pixels from its lenslet's first row, so lenslet centres lie at pixel offsets
nnum * l + (nnum - 1) / 2 - a from the source pixel.

Output layout: psf[j][a][b][u][v], tap (u, v) at pixel offset (u - c0, v - c0)
from the source pixel, c0 = (K - 1) / 2 - the layout every projection takes.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
from scipy import special


@dataclass(frozen=True)
class Optics:
    wavelength: float  # emission wavelength (one length unit throughout)
    na: float          # numerical aperture
    n_medium: float    # refractive index of the immersion medium (> na)
    mag: float         # objective magnification
    d_ml: float        # microlens pitch (sensor side)
    f_ml: float        # microlens focal length = microlens-to-sensor distance
    nnum: int          # sensor pixels per lenslet per axis
    ksize: int         # PSF window K (odd), in pixels
    osr: int = 3       # field samples per pixel per axis (odd)
    nquad: int = 1024  # Gauss-Legendre nodes of the Debye integral

    @property
    def pixel(self) -> float:
        return self.d_ml / self.nnum

    @property
    def delta(self) -> float:
        return self.pixel / self.osr


def nice_size(n: int) -> int:
    """Smallest m >= n whose prime factors are 2, 3 and 5."""
    m = max(1, int(n))
    while True:
        q = m
        for p in (2, 3, 5):
            while q % p == 0:
                q //= p
        if q == 1:
            return m
        m += 1


def grid_sizes(o: Optics):
    """(G, Gf, off): window samples per side, FFT grid side, window offset."""
    g = o.ksize * o.osr
    gf = nice_size(g)
    return g, gf, (gf - g) // 2


def gauss_legendre(nq: int, lo: float, hi: float):
    """Gauss-Legendre nodes and weights on [lo, hi] (library routine on [-1, 1])."""
    x, w = np.polynomial.legendre.leggauss(nq)
    half = 0.5 * (hi - lo)
    return lo + half * (x + 1.0), half * w


def debye_nip(r, z: float, o: Optics) -> np.ndarray:
    """Step 1: native-image-plane field of an on-axis point source at depth z,
    at image-plane radii r (array), by nquad-node Gauss-Legendre quadrature."""
    r = np.asarray(r, dtype=np.float64)
    alpha = np.arcsin(o.na / o.n_medium)
    k = 2.0 * np.pi / o.wavelength
    t, w = gauss_legendre(o.nquad, 0.0, alpha)
    # quadrature weight, apodisation, Jacobian and defocus phase per node
    e = w * np.sqrt(np.cos(t)) * np.sin(t) * np.exp(1j * k * o.n_medium * z * (1.0 - np.cos(t)))
    flat = r.reshape(-1)
    out = np.empty(flat.shape, dtype=np.complex128)
    step = 4096
    for s in range(0, flat.size, step):
        rr = flat[s:s + step]
        jm = special.j0(np.outer(k * o.n_medium * np.sin(t) / o.mag, rr))  # [node][radius]
        out[s:s + step] = e @ jm
    return out.reshape(r.shape)


def nip_window(z: float, o: Optics) -> np.ndarray:
    """Step 1 on the window grid: G x G samples, source on the centre sample."""
    g, _, _ = grid_sizes(o)
    hh = (g - 1) // 2
    m = np.arange(-hh, hh + 1, dtype=np.float64)
    rad = o.delta * np.sqrt(m[:, None] ** 2 + m[None, :] ** 2)
    # evaluate once per distinct radius
    uniq, inv = np.unique(rad, return_inverse=True)
    return debye_nip(uniq, z, o)[inv].reshape(g, g)


def lenslet_phase(a: int, b: int, o: Optics) -> np.ndarray:
    """Step 2: the microlens-array transmittance on the window grid for a
    source of row phase a and column phase b."""
    g, _, _ = grid_sizes(o)
    hh = (g - 1) // 2
    n, osr = o.nnum, o.osr
    m = np.arange(-hh, hh + 1)

    def centre_offset(idx, phase):
        # sample idx lies at pixel offset idx / osr from the source pixel centre;
        # the source's lenslet spans pixel offsets [-phase - 1/2, n - phase - 1/2)
        pix = idx / osr + phase + 0.5
        lens = np.floor(pix / n)
        centre = n * lens + (n - 1) / 2.0 - phase     # pixel offset of the lenslet centre
        return idx / osr - centre                     # in pixels

    dy = centre_offset(m, a) * o.pixel
    dx = centre_offset(m, b) * o.pixel
    d2 = dy[:, None] ** 2 + dx[None, :] ** 2
    return np.exp(-1j * np.pi * d2 / (o.wavelength * o.f_ml))


def fresnel_propagate(field: np.ndarray, delta: float, wavelength: float, dist: float):
    """Step 3: Fresnel propagation over `dist` of a periodic sampled field with
    the transfer function exp(-i pi lambda dist (fx^2 + fy^2))."""
    ny, nx = field.shape
    fy = np.fft.fftfreq(ny, d=delta)
    fx = np.fft.fftfreq(nx, d=delta)
    tf = np.exp(-1j * np.pi * wavelength * dist * (fy[:, None] ** 2 + fx[None, :] ** 2))
    return np.fft.ifft2(np.fft.fft2(field) * tf)


def sensor_field(nip: np.ndarray, a: int, b: int, o: Optics) -> np.ndarray:
    """Steps 2-3 for one source: the field on the whole Gf x Gf sensor grid."""
    g, gf, off = grid_sizes(o)
    full = np.zeros((gf, gf), dtype=np.complex128)
    full[off:off + g, off:off + g] = nip * lenslet_phase(a, b, o)
    return fresnel_propagate(full, o.delta, o.wavelength, o.f_ml)


def bin_pixels(field: np.ndarray, o: Optics) -> np.ndarray:
    """Step 4: |U|^2 summed over each pixel's osr x osr samples of the window."""
    g, _, off = grid_sizes(o)
    inten = np.abs(field[off:off + g, off:off + g]) ** 2
    k, s = o.ksize, o.osr
    return inten.reshape(k, s, k, s).sum(axis=(1, 3))


def lf_psf(o: Optics, depths, unit_sum: bool = False, fields=None) -> np.ndarray:
    """The PSF set psf[j][a][b][u][v] for the depths z_j (float64).  `fields`
    (optional) lists the (j, a, b) to compute; the others stay zero.  With
    unit_sum every computed (j, a, b) kernel is scaled to sum 1 (a kernel whose
    sum is not positive is kept as it is)."""
    depths = [float(z) for z in depths]
    n, k = o.nnum, o.ksize
    out = np.zeros((len(depths), n, n, k, k))
    want = fields if fields is not None else [(j, a, b) for j in range(len(depths))
                                               for a in range(n) for b in range(n)]
    by_depth = {}
    for j, a, b in want:
        by_depth.setdefault(j, []).append((a, b))
    for j, ab in by_depth.items():
        nip = nip_window(depths[j], o)
        for a, b in ab:
            img = bin_pixels(sensor_field(nip, a, b, o), o)
            if unit_sum:
                s = img.sum()
                if s > 0:
                    img = img / s
            out[j, a, b] = img
    return out
