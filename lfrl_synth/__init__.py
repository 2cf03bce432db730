"""Seeded synthetic inputs for light-field Richardson-Lucy deconvolution.

This module is the only code shared by the CPU oracle's tests and the HIP path's
tests and benchmark.  It makes inputs and nothing else: PSF sets, bead/filament
volumes and Poisson measurement noise.  It holds none of the method's arithmetic
(no projection, no update, no metric); where a clean light-field image is needed,
the caller projects the volume with its own implementation and hands the result
to :func:`measure`.

The paper measures on real data (C. elegans, fluorescence beads, MCF10A cells)
that is not available here; these generators stand in for it with the shapes,
value ranges and structure of light-field workloads (sec. 1, sec. 3.2).

Conventions shared with the library and the oracle:

* PSF array ``h[j][a][b][u][v]`` (float32, C order): depth j, lenslet-relative
  row phase a and column phase b of the source voxel, row tap u and column tap v.
  Tap (u, v) is the intensity at displacement (u - c0, v - c0) from the source
  pixel, with c0 = (K - 1) / 2 and K odd.
* Volume ``x[j][r][s]`` (float32), image ``y[r][s]`` (float32); the lenslet grid
  starts at pixel (0, 0), so the phase of pixel r is r mod Nnum.
* Physical depth of plane j is ``z_j = j - (Nz - 1) / 2``.

All randomness comes from ``numpy.random.default_rng(seed)`` (PCG64); arrays are
built in float64 and rounded to float32 once.
"""
from __future__ import annotations

import dataclasses
import math
import os

import numpy as np

__all__ = [
    "Geometry",
    "gaussian_psf",
    "disk_psf",
    "bead_volume",
    "add_filaments",
    "measure",
    "preset",
    "PRESETS",
]


@dataclasses.dataclass(frozen=True)
class Geometry:
    nnum: int          # pixels per lenslet along each axis (N)
    lenslets: int      # lenslets per side (square images)
    nz: int            # depth planes
    ksize: int         # PSF support per side (odd)

    @property
    def h(self) -> int:
        return self.nnum * self.lenslets

    @property
    def w(self) -> int:
        return self.nnum * self.lenslets

    @property
    def c0(self) -> int:
        return (self.ksize - 1) // 2


def _depths(nz: int) -> np.ndarray:
    return np.arange(nz, dtype=np.float64) - (nz - 1) / 2.0


def _unit_sum_f32(k: np.ndarray) -> np.ndarray:
    s = k.sum(axis=(-2, -1), keepdims=True)
    return (k / s).astype(np.float32)


def gaussian_psf(nnum: int, nz: int, ksize: int, seed: int, *,
                 shift_scale: float | None = 0.5, jitter: float = 0.25,
                 sigma0: float = 1.0) -> np.ndarray:
    """Gaussian-spot PSF set: sigma = sigma0 + |z|, centre shifted by
    ``shift_scale * (a - (N-1)/2, b - (N-1)/2) * z`` plus a per-(j,a,b) uniform
    jitter in [-jitter, jitter]^2 (the jitter breaks mirror symmetry so that a
    missing kernel flip cannot hide).  Truncated to K x K, unit sum in float64,
    then rounded to float32.

    ``shift_scale=None`` picks ``min(0.5, (K-1) / (4 * ((N-1)/2) * z_max))`` so the
    largest parallax shift stays inside the support."""
    if ksize % 2 != 1:
        raise ValueError("ksize must be odd")
    rng = np.random.default_rng(seed)
    z = _depths(nz)
    c0 = (ksize - 1) / 2.0
    ph = np.arange(nnum, dtype=np.float64) - (nnum - 1) / 2.0
    if shift_scale is None:
        zmax = max(abs(z[0]), 1e-9)
        half = max((nnum - 1) / 2.0, 1e-9)
        shift_scale = min(0.5, (ksize - 1) / (4.0 * half * zmax))
    jit = rng.uniform(-jitter, jitter, size=(nz, nnum, nnum, 2))
    u = np.arange(ksize, dtype=np.float64)
    out = np.empty((nz, nnum, nnum, ksize, ksize), dtype=np.float32)

    def plane(j: int) -> None:
        sig = sigma0 + abs(z[j])
        cu = c0 + shift_scale * ph[:, None] * z[j] + jit[j, :, :, 0]   # [a][b]
        cv = c0 + shift_scale * ph[None, :] * z[j] + jit[j, :, :, 1]
        gu = np.exp(-(u[None, None, :] - cu[..., None]) ** 2 / (2 * sig * sig))
        gv = np.exp(-(u[None, None, :] - cv[..., None]) ** 2 / (2 * sig * sig))
        k = gu[..., :, None] * gv[..., None, :]
        out[j] = _unit_sum_f32(k)

    _each_plane(plane, nz)
    return out


def _each_plane(fn, nz: int) -> None:
    """Run fn(j) for every plane on a thread pool (the planes are independent
    and numpy releases the GIL in the heavy calls)."""
    if nz <= 1:
        fn(0)
        return
    from concurrent.futures import ThreadPoolExecutor
    workers = max(1, min(16, os.cpu_count() or 1, nz))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        list(ex.map(fn, range(nz)))


def _disk_blur_profile(radius: float, blur: float, rmax: float,
                       step: float = 1.0 / 64.0) -> tuple[np.ndarray, np.ndarray]:
    """Radial profile of a uniform disk of ``radius`` convolved with an isotropic
    Gaussian of std ``blur``: P(|r + blur*n| <= radius), n ~ N(0, I2), which is the
    non-central chi-square CDF with 2 degrees of freedom."""
    from scipy.stats import ncx2
    r = np.arange(0.0, rmax + 2 * step, step)
    prof = ncx2.cdf((radius / blur) ** 2, 2, (r / blur) ** 2)
    return r, prof


def disk_psf(nnum: int, nz: int, ksize: int, seed: int, *,
             shift_scale: float = 0.5, jitter: float = 0.25,
             r0: float = 2.0, r_slope: float = 4.0, blur: float = 1.5,
             depth_rescale: float | None = None) -> np.ndarray:
    """Defocus-disk PSF set: a uniform disk of radius ``r0 + r_slope*|z|``
    convolved with a Gaussian of std ``blur``, centre shifted by
    ``shift_scale * (a - (N-1)/2, b - (N-1)/2) * z`` plus jitter, unit sum.

    ``depth_rescale=D`` replaces z by ``D * z / z_max`` so that sets with more
    planes keep the same largest disk and shift."""
    if ksize % 2 != 1:
        raise ValueError("ksize must be odd")
    rng = np.random.default_rng(seed)
    z = _depths(nz)
    if depth_rescale is not None and nz > 1:
        z = depth_rescale * z / abs(z[0])
    c0 = (ksize - 1) / 2.0
    ph = np.arange(nnum, dtype=np.float64) - (nnum - 1) / 2.0
    jit = rng.uniform(-jitter, jitter, size=(nz, nnum, nnum, 2))
    u = np.arange(ksize, dtype=np.float64)
    rmax = math.sqrt(2.0) * ksize + 4.0
    out = np.empty((nz, nnum, nnum, ksize, ksize), dtype=np.float32)
    cache: dict[float, tuple[np.ndarray, np.ndarray]] = {}
    for j in range(nz):
        key = round(r0 + r_slope * abs(z[j]), 12)
        if key not in cache:
            cache[key] = _disk_blur_profile(key, blur, rmax)

    def plane(j: int) -> None:
        rgrid, prof = cache[round(r0 + r_slope * abs(z[j]), 12)]
        cu = c0 + shift_scale * ph[:, None] * z[j] + jit[j, :, :, 0]
        cv = c0 + shift_scale * ph[None, :] * z[j] + jit[j, :, :, 1]
        du = (u[None, None, :] - cu[..., None]) ** 2          # [a][b][u]
        dv = (u[None, None, :] - cv[..., None]) ** 2          # [a][b][v]
        for a in range(nnum):
            d = np.sqrt(du[a][:, :, None] + dv[a][:, None, :])  # [b][u][v]
            k = np.interp(d, rgrid, prof)
            out[j, a] = _unit_sum_f32(k)

    _each_plane(plane, nz)
    return out


def _splat(vol: np.ndarray, centre, sigma: float, amp: float, trunc: float) -> None:
    """Add amp*exp(-|p-centre|^2/(2 sigma^2)) for voxels within trunc*sigma."""
    nz, h, w = vol.shape
    rad = trunc * sigma
    lo = [max(0, int(math.floor(c - rad))) for c in centre]
    hi = [min(n - 1, int(math.ceil(c + rad))) for c, n in zip(centre, (nz, h, w))]
    if any(l > u for l, u in zip(lo, hi)):
        return
    jz = np.arange(lo[0], hi[0] + 1, dtype=np.float64) - centre[0]
    jr = np.arange(lo[1], hi[1] + 1, dtype=np.float64) - centre[1]
    js = np.arange(lo[2], hi[2] + 1, dtype=np.float64) - centre[2]
    d2 = jz[:, None, None] ** 2 + jr[None, :, None] ** 2 + js[None, None, :] ** 2
    g = amp * np.exp(-d2 / (2 * sigma * sigma))
    g[d2 > rad * rad] = 0.0
    vol[lo[0]:hi[0] + 1, lo[1]:hi[1] + 1, lo[2]:hi[2] + 1] += g


def bead_volume(nz: int, h: int, w: int, n_beads: int, seed: int, *,
                sigma: float = 1.0, amp: float = 1.0, trunc: float = 4.0,
                as_float64: bool = False) -> np.ndarray:
    """Isotropic Gaussian beads with continuous-uniform centres; each bead is cut
    to zero beyond ``trunc*sigma`` so the volume is sparse."""
    rng = np.random.default_rng(seed)
    vol = np.zeros((nz, h, w), dtype=np.float64)
    cz = rng.uniform(0, nz, n_beads)
    cr = rng.uniform(0, h, n_beads)
    cs = rng.uniform(0, w, n_beads)
    for i in range(n_beads):
        _splat(vol, (cz[i], cr[i], cs[i]), sigma, amp, trunc)
    return vol if as_float64 else vol.astype(np.float32)


def bead_splats(nz: int, h: int, w: int, n_beads: int, seed: int, *,
                sigma: float = 1.0, amp: float = 1.0,
                trunc: float = 4.0) -> tuple[np.ndarray, np.ndarray]:
    """The beads of ``bead_volume`` (same draws, same values) as flat voxel
    indices and float64 values, in bead order: adding the values at the
    indices, in order, onto a zero volume gives ``bead_volume(...,
    as_float64=True)``.  Lets a large sparse volume be built where it is
    used instead of being shipped whole."""
    rng = np.random.default_rng(seed)
    c = np.stack([rng.uniform(0, nz, n_beads), rng.uniform(0, h, n_beads),
                  rng.uniform(0, w, n_beads)], axis=1)               # [bead][axis]
    rad = trunc * sigma
    dims = np.array([nz, h, w])
    lo = np.maximum(np.floor(c - rad).astype(np.int64), 0)
    hi = np.minimum(np.ceil(c + rad).astype(np.int64), dims - 1)
    m = int(2 * math.ceil(rad) + 2)                                  # widest box side
    ax = lo[:, :, None] + np.arange(m)[None, None, :]               # [bead][axis][m]
    inside = ax <= hi[:, :, None]
    dz = (ax[:, 0] - c[:, 0:1]) ** 2
    dr = (ax[:, 1] - c[:, 1:2]) ** 2
    ds = (ax[:, 2] - c[:, 2:3]) ** 2
    d2 = dz[:, :, None, None] + dr[:, None, :, None] + ds[:, None, None, :]
    g = amp * np.exp(-d2 / (2 * sigma * sigma))
    g[d2 > rad * rad] = 0.0
    keep = (inside[:, 0][:, :, None, None] & inside[:, 1][:, None, :, None]
            & inside[:, 2][:, None, None, :])
    flat = ((ax[:, 0][:, :, None, None] * h + ax[:, 1][:, None, :, None]) * w
            + ax[:, 2][:, None, None, :])
    return flat[keep].astype(np.int64), g[keep]


def add_filaments(vol: np.ndarray, n: int, seed: int, *, step: float = 0.25,
                  sigma: float = 1.0, amp: float = 0.25,
                  trunc: float = 4.0) -> np.ndarray:
    """Add ``n`` tubular filaments: cubic Bezier curves with control points drawn
    uniformly in the volume, sampled every ``step`` voxels of arc length, each
    sample an isotropic Gaussian of std ``sigma`` and amplitude ``amp``."""
    rng = np.random.default_rng(seed)
    nz, h, w = vol.shape
    out = vol.astype(np.float64, copy=True)
    box = np.array([nz, h, w], dtype=np.float64)
    for _ in range(n):
        p = rng.uniform(0, 1, size=(4, 3)) * box
        t = np.linspace(0.0, 1.0, 20001)[:, None]
        curve = ((1 - t) ** 3 * p[0] + 3 * (1 - t) ** 2 * t * p[1]
                 + 3 * (1 - t) * t ** 2 * p[2] + t ** 3 * p[3])
        seg = np.sqrt(((curve[1:] - curve[:-1]) ** 2).sum(axis=1))
        arc = np.concatenate([[0.0], np.cumsum(seg)])
        targets = np.arange(0.0, arc[-1], step)
        idx = np.searchsorted(arc, targets).clip(0, len(arc) - 1)
        for c in curve[idx]:
            _splat(out, tuple(c), sigma, amp, trunc)
    return out.astype(vol.dtype)


def measure(clean: np.ndarray, peak: float, background: float, seed: int) -> np.ndarray:
    """Noisy light-field measurement from a clean projected image: scale so the
    brightest pixel has ``peak`` expected counts, draw Poisson counts, add a
    constant ``background``.  Returns float32."""
    clean = np.asarray(clean, dtype=np.float64)
    m = clean.max()
    if not m > 0:
        raise ValueError("clean image has no positive pixel")
    rng = np.random.default_rng(seed)
    lam = clean * (peak / m)
    y = rng.poisson(np.maximum(lam, 0.0)).astype(np.float64) + background
    return y.astype(np.float32)


# Workload presets (sizes and seeds of the light-field configurations).
PRESETS = {
    # Nnum 5, 11x11 lenslets -> 55x55, 5 planes, 25x25 Gaussian PSF, 20 beads.
    "small": dict(geometry=Geometry(5, 11, 5, 25), psf="gaussian", psf_seed=11,
                  beads=20, vol_seed=12, filaments=0, peak=1000.0, background=10.0,
                  noise_seed=13, iters=5, spot_radius=1.0),
    # Nnum 15, 40x40 lenslets -> 600x600, 31 planes, 255x255 defocus-disk PSF,
    # 500 beads + 3 filaments.
    "large": dict(geometry=Geometry(15, 40, 31, 255), psf="disk", psf_seed=21,
                  beads=500, vol_seed=22, filaments=3, peak=2000.0, background=10.0,
                  noise_seed=23, iters=8, spot_radius=2.0),
}


# Serving workload: four resident PSF sets (Nnum, planes, seed), K = 255, built
# with the defocus-disk generator and depths rescaled so every set has the
# largest disk and shift of the 31-plane set; requests pick a set uniformly
# and a square size uniformly among the lenslet counts L with
# min_side <= Nnum * L <= max_side.
SERVING = dict(sets=((11, 21, 501), (13, 31, 502), (15, 31, 503), (15, 51, 504)),
               ksize=255, depth_rescale=15.0, requests=2000, arrival_seed=51,
               request_seed0=5000, beads=200, peak=1000.0, background=10.0,
               min_side=363, max_side=900, max_iters=50, spot_radius=2.0)


def serving_psf(k: int, ksize: int | None = None) -> np.ndarray:
    """PSF set k of the serving workload."""
    n, nz, seed = SERVING["sets"][k]
    return disk_psf(n, nz, ksize or SERVING["ksize"], seed,
                    depth_rescale=SERVING["depth_rescale"])


def serving_requests(count: int, *, seed0: int | None = None,
                     sets=None, min_side: int | None = None,
                     max_side: int | None = None) -> list[dict]:
    """Seeded request specs: PSF set index, Nnum, planes, lenslets per side,
    image size and the seed of the request's bead volume and noise."""
    sets = sets or SERVING["sets"]
    seed0 = SERVING["request_seed0"] if seed0 is None else seed0
    lo_side = min_side or SERVING["min_side"]
    hi_side = max_side or SERVING["max_side"]
    out = []
    for i in range(count):
        rng = np.random.default_rng(seed0 + i)
        k = int(rng.integers(len(sets)))
        n, nz = sets[k][0], sets[k][1]
        lo = -(-lo_side // n)
        hi = hi_side // n
        L = int(rng.integers(lo, hi + 1))
        out.append(dict(rid=i, set=k, nnum=n, nz=nz, lenslets=L, h=n * L, w=n * L,
                        seed=seed0 + i))
    return out


# Batched workload: independent frames, each with its own Nnum, planes, size
# and Gaussian PSF set (K = min(255, 8 Nnum + 1), shift scale kept inside the
# support), 200 beads, peak 1000 counts, background 10, 8 iterations.
BATCHED = dict(frames=16, seed0=300, nnums=(11, 13, 15), nzs=(21, 31, 41), min_lenslets=33,
               max_side=900, beads=200, peak=1000.0, background=10.0, iters=8,
               spot_radius=1.0)


def batched_frames(count: int | None = None) -> list[dict]:
    """Seeded specs of the batched workload's frames."""
    cfg = BATCHED
    out = []
    for f in range(cfg["frames"] if count is None else count):
        seed = cfg["seed0"] + f
        rng = np.random.default_rng(seed)
        n = int(rng.choice(cfg["nnums"]))
        L = int(rng.integers(cfg["min_lenslets"], cfg["max_side"] // n + 1))
        nz = int(rng.choice(cfg["nzs"]))
        k = min(255, 8 * n + 1)
        out.append(dict(frame=f, seed=seed, nnum=n, lenslets=L, h=n * L, w=n * L, nz=nz,
                        ksize=k))
    return out


def batched_psf(spec: dict) -> np.ndarray:
    return gaussian_psf(spec["nnum"], spec["nz"], spec["ksize"], spec["seed"], shift_scale=None)


def poisson_arrivals(count: int, rate: float, seed: int | None = None) -> np.ndarray:
    """Arrival times (s) of an open-loop Poisson process of `rate` per second."""
    rng = np.random.default_rng(SERVING["arrival_seed"] if seed is None else seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=count))


def _cached(key: str, make, cache_dir: str | None):
    """Load a generated array from ``cache_dir/key.npy`` or make and store it."""
    if not cache_dir:
        return make()
    import os
    os.makedirs(cache_dir, exist_ok=True)
    path = os.path.join(cache_dir, key + ".npy")
    if os.path.exists(path):
        return np.load(path, allow_pickle=False)
    arr = make()
    tmp = f"{path}.{os.getpid()}.tmp.npy"
    np.save(tmp, arr)
    os.replace(tmp, path)
    return arr


def preset(name: str, *, with_psf: bool = True, cache_dir: str | None = None) -> dict:
    """Build the seeded inputs of a named workload: ``psf_array``, ``x_true`` and
    the metadata needed to make the measurement (``peak``, ``background``,
    ``noise_seed``).  The clean image itself must be projected by the caller.
    ``cache_dir`` keeps generated PSF sets on disk between processes."""
    p = dict(PRESETS[name])
    g: Geometry = p["geometry"]
    if with_psf:
        key = f"psf_{p['psf']}_{g.nnum}_{g.nz}_{g.ksize}_{p['psf_seed']}"
        if p["psf"] == "gaussian":
            p["psf_array"] = _cached(key, lambda: gaussian_psf(g.nnum, g.nz, g.ksize,
                                                               p["psf_seed"]), cache_dir)
        else:
            p["psf_array"] = _cached(key, lambda: disk_psf(g.nnum, g.nz, g.ksize,
                                                           p["psf_seed"]), cache_dir)
    x = bead_volume(g.nz, g.h, g.w, p["beads"], p["vol_seed"])
    if p["filaments"]:
        x = add_filaments(x, p["filaments"], p["vol_seed"] + 1000)
    p["x_true"] = x
    return p
