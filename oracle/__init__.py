"""CPU float64 oracle for light-field Richardson-Lucy deconvolution with the
DCT-entropy stopping metric.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark use it.  The product (the HIP library and its binding)
never imports it, and it never imports the product.

Plain and slow on purpose.  The projections are direct spatial loops in C
(``lfrl_oracle.c``); the Richardson-Lucy loop, the metric and the stop rule are
written below in numpy, step by step, in the order the method states them.

Passages followed (section / equation of the paper):

* Richardson-Lucy deconvolution of the light-field image into a volume of axial
  layers: sec. 1 (the method is named and attributed to Prevedel et al. 2014)
  and sec. 2.1 (all iterations on the device, only the final volume returned).
* The metric input is the maximum projection of each iterate along z: sec. 2.2
  and the caption of Fig. 2(a).
* Orthonormal 2-D DCT-II: Eqs. (1)-(4).
* Shannon entropy over a region: Eq. (5); triangular region and its size:
  Eq. (6); cutoff geometry: Eqs. (7), (9)-(11); DCT entropy: Eq. (12) with the
  2-norm taken over the coefficient matrix.
* Stopping: iterate until the DCT entropy starts to decrease and keep the
  iterate at the maximum (sec. 2.2, after Eq. (12); Fig. 2(d)).

Readings where the text is silent or garbled (each also listed in the design
notes):

* RL update: x <- x * A^T(y / A x) / A^T 1, with y/Ax := 0 where Ax <= 0 and
  x := 0 where A^T 1 <= 0; ones initialisation.
* Variants (the paper names none of them; they widen the method): a known
  constant background b in the image model (A x + b), the ISRA update
  x <- x * A^T y / A^T(A x + b), and the back projection A^T y as x^0.
* Metric variants: the rectangle that Eq. (12)'s summation limits state, the
  whole coefficient matrix (the overall entropy of Fig. 2(c)), each with the
  prefactor 1 / area; the 2-norm over the region only instead of the whole
  matrix, or its spectral norm.  A "decreasing trend" (sec. 2.2) may be read
  from window means.
* Transposed PSF = exact adjoint of the forward projection.
* DCT axes: Eq. (1) pairs u with the width and v with the height (X_S is the
  width of the region, Eq. (6)); F is stored as F[v][u] (row frequency first).
* "L2 of a matrix" = Frobenius norm of the whole DCT coefficient matrix.
* "abslog2" = log2 of the absolute value, with 0 * log 0 = 0.
* The prefactor of Eq. (12) = 1 / G_S = 2 / (X_S * Y_S).
* Region S = {(u, v): u / X_S + v / Y_S < 1} (the upper-left triangle of Fig.
  2(c)), with real-valued legs X_S, Y_S.
* Eq. (8) is inverted relative to Eqs. (9)-(10); Eqs. (9)-(10) are used.

The PSF computed from optical parameters (sec. 2.1, Fig. 1) has its own
oracle module, ``oracle.optics``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lfrl_oracle.c")
_LIB = os.path.join(_HERE, "liblfrl_oracle.so")
_lock = threading.Lock()
_lib = None


def _compile(out: str, flags) -> None:
    tmp = out + ".tmp"
    # ISO C mode and no contraction: every product and sum rounds on its own
    cmd = (["gcc"] + list(flags) + ["-ffp-contract=off", "-fopenmp", "-shared", "-fPIC",
                                    "-std=c11", "-Wall", "-Wextra", "-o", tmp, _SRC])
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)


def build(force: bool = True) -> str:
    """Compile the C part of the oracle (gcc, OpenMP, generic x86-64)."""
    if force or not os.path.exists(_LIB):
        _compile(_LIB, ["-O2"])
    return _LIB


def use_native_build(directory: str) -> str:
    """Compile the same C source with -O3 -march=native for the host this runs
    on, into `directory`, and use it from now on in this process (for timing
    the oracle on the machine it runs on; the arithmetic is the same, each
    operation rounded on its own).  Returns the compiler flags."""
    global _lib
    path = os.path.join(directory, "liblfrl_oracle_native.so")
    flags = ["-O3", "-march=native"]
    _compile(path, flags)
    with _lock:
        _lib = _bind(ctypes.CDLL(path))
    return " ".join(flags + ["-ffp-contract=off", "-fopenmp"])


def _bind(lib):
    i, l = ctypes.c_int, ctypes.c_long
    fp = ctypes.POINTER(ctypes.c_float)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    lib.oracle_forward.argtypes = [i, i, i, i, i, fp, dp, dp]
    lib.oracle_backward.argtypes = [i, i, i, i, i, fp, dp, dp]
    lib.oracle_forward_at.argtypes = [i, i, i, i, i, fp, dp, l, ip, ip, dp]
    lib.oracle_forward_window.argtypes = [i, i, i, i, i, fp, dp, i, i, i, i, dp]
    lib.oracle_backward_at.argtypes = [i, i, i, i, i, fp, dp, l, ip, ip, ip, dp]
    for f in (lib.oracle_forward, lib.oracle_backward, lib.oracle_forward_at,
              lib.oracle_backward_at, lib.oracle_forward_window):
        f.restype = ctypes.c_int
    lib.oracle_threads.restype = ctypes.c_int
    return lib


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
            _lib = _bind(ctypes.CDLL(_LIB))
    return _lib


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _geom(psf: np.ndarray):
    if psf.ndim != 5 or psf.shape[1] != psf.shape[2] or psf.shape[3] != psf.shape[4]:
        raise ValueError("psf must be [nz][N][N][K][K]")
    nz, n, _, k, _ = psf.shape
    if k % 2 != 1:
        raise ValueError("PSF support must be odd")
    return nz, n, k


def _f32(psf) -> np.ndarray:
    return np.ascontiguousarray(psf, dtype=np.float32)


def threads() -> int:
    """OpenMP threads the C routines use."""
    return int(_load().oracle_threads())


def forward(psf, vol) -> np.ndarray:
    """Light-field forward projection A x of a volume [nz][H][W] (float64)."""
    psf = _f32(psf)
    nz, n, k = _geom(psf)
    vol = np.ascontiguousarray(vol, dtype=np.float64)
    if vol.ndim != 3 or vol.shape[0] != nz:
        raise ValueError("volume must be [nz][H][W]")
    h, w = vol.shape[1:]
    img = np.empty((h, w), dtype=np.float64)
    rc = _load().oracle_forward(n, nz, k, h, w, _ptr(psf, ctypes.c_float),
                                _ptr(vol, ctypes.c_double), _ptr(img, ctypes.c_double))
    if rc != 0:
        raise RuntimeError(f"oracle_forward failed ({rc})")
    return img


def backward(psf, img) -> np.ndarray:
    """Back projection A^T y (exact adjoint of :func:`forward`)."""
    psf = _f32(psf)
    nz, n, k = _geom(psf)
    img = np.ascontiguousarray(img, dtype=np.float64)
    h, w = img.shape
    vol = np.empty((nz, h, w), dtype=np.float64)
    rc = _load().oracle_backward(n, nz, k, h, w, _ptr(psf, ctypes.c_float),
                                 _ptr(img, ctypes.c_double), _ptr(vol, ctypes.c_double))
    if rc != 0:
        raise RuntimeError(f"oracle_backward failed ({rc})")
    return vol


def forward_at(psf, vol, rows, cols) -> np.ndarray:
    """A x evaluated only at pixels (rows[i], cols[i])."""
    psf = _f32(psf)
    nz, n, k = _geom(psf)
    vol = np.ascontiguousarray(vol, dtype=np.float64)
    h, w = vol.shape[1:]
    rows = np.ascontiguousarray(rows, dtype=np.int32)
    cols = np.ascontiguousarray(cols, dtype=np.int32)
    if rows.shape != cols.shape or rows.ndim != 1:
        raise ValueError("rows/cols must be 1-D of equal length")
    if rows.size and (rows.min() < 0 or rows.max() >= h or cols.min() < 0 or cols.max() >= w):
        raise ValueError("pixel index out of range")
    out = np.empty(rows.size, dtype=np.float64)
    rc = _load().oracle_forward_at(n, nz, k, h, w, _ptr(psf, ctypes.c_float),
                                   _ptr(vol, ctypes.c_double), rows.size,
                                   _ptr(rows, ctypes.c_int), _ptr(cols, ctypes.c_int),
                                   _ptr(out, ctypes.c_double))
    if rc != 0:
        raise RuntimeError(f"oracle_forward_at failed ({rc})")
    return out


def forward_window(psf, vol, r0: int, r1: int, s0: int, s1: int) -> np.ndarray:
    """A x on the pixel window rows [r0, r1) x columns [s0, s1): the same sums
    as :func:`forward`, evaluated only there (pixels outside the image are 0).
    Each output row is summed in a fixed order, whatever the thread count."""
    psf = _f32(psf)
    nz, n, k = _geom(psf)
    vol = np.ascontiguousarray(vol, dtype=np.float64)
    if vol.ndim != 3 or vol.shape[0] != nz:
        raise ValueError("volume must be [nz][H][W]")
    h, w = vol.shape[1:]
    if r1 < r0 or s1 < s0:
        raise ValueError("empty or inverted window")
    out = np.empty((r1 - r0, s1 - s0), dtype=np.float64)
    rc = _load().oracle_forward_window(n, nz, k, h, w, _ptr(psf, ctypes.c_float),
                                       _ptr(vol, ctypes.c_double), r0, r1, s0, s1,
                                       _ptr(out, ctypes.c_double))
    if rc != 0:
        raise RuntimeError(f"oracle_forward_window failed ({rc})")
    return out


def backward_at(psf, img, planes, rows, cols) -> np.ndarray:
    """A^T y evaluated only at voxels (planes[i], rows[i], cols[i])."""
    psf = _f32(psf)
    nz, n, k = _geom(psf)
    img = np.ascontiguousarray(img, dtype=np.float64)
    h, w = img.shape
    jj = np.ascontiguousarray(planes, dtype=np.int32)
    rr = np.ascontiguousarray(rows, dtype=np.int32)
    ss = np.ascontiguousarray(cols, dtype=np.int32)
    if not (jj.shape == rr.shape == ss.shape) or jj.ndim != 1:
        raise ValueError("index arrays must be 1-D of equal length")
    if jj.size and (jj.min() < 0 or jj.max() >= nz or rr.min() < 0 or rr.max() >= h
                    or ss.min() < 0 or ss.max() >= w):
        raise ValueError("voxel index out of range")
    out = np.empty(jj.size, dtype=np.float64)
    rc = _load().oracle_backward_at(n, nz, k, h, w, _ptr(psf, ctypes.c_float),
                                    _ptr(img, ctypes.c_double), jj.size,
                                    _ptr(jj, ctypes.c_int), _ptr(rr, ctypes.c_int),
                                    _ptr(ss, ctypes.c_int), _ptr(out, ctypes.c_double))
    if rc != 0:
        raise RuntimeError(f"oracle_backward_at failed ({rc})")
    return out


def sensitivity(psf, h: int, w: int) -> np.ndarray:
    """c = A^T 1: the total weight each voxel sends into the image."""
    return backward(psf, np.ones((h, w), dtype=np.float64))


def normalize_psf(psf) -> np.ndarray:
    """Scale every (j, a, b) kernel of a float32 PSF set to unit sum, the sums
    taken in float64, the result rounded back to float32.  A kernel whose sum
    is not positive has no unit-sum scaling and is kept as it is."""
    p = np.asarray(psf, dtype=np.float32).astype(np.float64)
    s = p.sum(axis=(-2, -1), keepdims=True)
    ok = s > 0
    return np.where(ok, p / np.where(ok, s, 1.0), p).astype(np.float32)


# --------------------------------------------------------------------------
# Richardson-Lucy (sec. 1, sec. 2.1)
# --------------------------------------------------------------------------
def rl_step(psf, y, x, c, background: float = 0.0):
    """One Richardson-Lucy iteration with a known constant background b >= 0 in
    the image model (b = 0: the plain update):

        m = A x + b,   x_new = x * A^T(y / m) / c,

    y / m := 0 where m <= 0 and x_new := 0 where c <= 0.  Returns (x_new, m)."""
    yhat = forward(psf, x) + background
    ratio = np.zeros_like(yhat)
    pos = yhat > 0
    ratio[pos] = y[pos] / yhat[pos]
    b = backward(psf, ratio)
    x_new = np.zeros_like(x)
    ok = c > 0
    x_new[ok] = x[ok] * b[ok] / c[ok]
    return x_new, yhat


def isra_step(psf, y, x, d, background: float = 0.0):
    """One ISRA iteration (the least-squares counterpart of the update, used
    under the Richardson-Lucy name in light-field work):

        m = A x + b,   x_new = x * d / A^T m,   d = A^T y,

    x_new := 0 where A^T m <= 0.  Returns (x_new, m)."""
    yhat = forward(psf, x) + background
    den = backward(psf, yhat)
    x_new = np.zeros_like(x)
    ok = den > 0
    x_new[ok] = x[ok] * d[ok] / den[ok]
    return x_new, yhat


def initial_volume(psf, y, init: str = "ones", x0=None) -> np.ndarray:
    """x^0: 'ones', 'given' (a copy of x0) or 'backprojection' (A^T y)."""
    nz = np.asarray(psf).shape[0]
    h, w = np.asarray(y).shape
    if init == "ones":
        return np.ones((nz, h, w))
    if init == "given":
        return np.array(x0, dtype=np.float64)
    if init == "backprojection":
        return backward(psf, np.asarray(y, dtype=np.float64))
    raise ValueError(f"unknown init {init!r}")


def rl(psf, y, iters: int, x0=None, keep_all: bool = False, *, update: str = "rl",
       background: float = 0.0, init: str = None):
    """Run ``iters`` iterations of the update ('rl' or 'isra') from x^0: ``x0``
    when given, else ones (or ``init``, see initial_volume).

    Returns the final iterate, or the list [x^0, x^1, ..., x^iters] when
    ``keep_all``."""
    y = np.asarray(y, dtype=np.float64)
    h, w = y.shape
    if init is None:
        init = "ones" if x0 is None else "given"
    x = initial_volume(psf, y, init, x0)
    if update == "rl":
        c = sensitivity(psf, h, w)
        step = lambda x: rl_step(psf, y, x, c, background)[0]  # noqa: E731
    elif update == "isra":
        d = backward(psf, y)
        step = lambda x: isra_step(psf, y, x, d, background)[0]  # noqa: E731
    else:
        raise ValueError(f"unknown update {update!r}")
    out = [x]
    for _ in range(iters):
        x = step(x)
        out.append(x)
    return out if keep_all else x


def rl_window(psf, y, iters: int, r0: int, r1: int, s0: int, s1: int,
              background: float = 0.0):
    """Richardson-Lucy iterates x^1 .. x^iters (ones start, the update of
    :func:`rl_step`) on the voxel window rows [r0, r1) x columns [s0, s1) of
    every plane, without whole-volume iterations.

    A back-projected voxel reads only pixels within c0 = (K - 1) / 2 of it and
    a projected pixel only voxels within c0, so x^k on the window needs the
    ratio of iteration k on the window grown by c0, x^{k-1} on the window
    grown by 2 c0, and so on: each iterate is computed exactly on the window
    the next step reads (clipped to the image), with the same sums as
    :func:`forward` and :func:`backward`.

    Returns (xs, c): xs[m] = x^{m+1} on the window as [nz][r1-r0][s1-s0], and
    c = A^T 1 there."""
    psf = _f32(psf)
    nz, n, k = _geom(psf)
    y = np.asarray(y, dtype=np.float64)
    h, w = y.shape
    c0 = (k - 1) // 2

    def grow(m):
        return (max(0, r0 - m * c0), min(h, r1 + m * c0), max(0, s0 - m * c0),
                min(w, s1 + m * c0))

    ones_img = np.ones((h, w))
    x = np.ones((nz, h, w))
    out = []
    c_win = None
    for it in range(1, iters + 1):
        pr0, pr1, ps0, ps1 = grow(2 * (iters - it) + 1)   # pixels of this ratio
        vr0, vr1, vs0, vs1 = grow(2 * (iters - it))       # voxels of this iterate
        yhat = forward_window(psf, x, pr0, pr1, ps0, ps1) + background
        rho = np.zeros((h, w))
        pos = yhat > 0
        rho[pr0:pr1, ps0:ps1][pos] = y[pr0:pr1, ps0:ps1][pos] / yhat[pos]
        jj, rr, ss = np.meshgrid(np.arange(nz), np.arange(vr0, vr1), np.arange(vs0, vs1),
                                 indexing="ij")
        jj, rr, ss = jj.ravel(), rr.ravel(), ss.ravel()
        c = backward_at(psf, ones_img, jj, rr, ss)
        b = backward_at(psf, rho, jj, rr, ss)
        old = x[jj, rr, ss]
        ok = c > 0
        new = np.zeros_like(c)
        new[ok] = old[ok] * b[ok] / c[ok]
        x = np.zeros((nz, h, w))
        x[jj, rr, ss] = new
        shape = (nz, vr1 - vr0, vs1 - vs0)
        win = (slice(None), slice(r0 - vr0, r1 - vr0), slice(s0 - vs0, s1 - vs0))
        out.append(new.reshape(shape)[win].copy())
        c_win = c.reshape(shape)[win].copy()
    return out, c_win


def poisson_loglik(y, yhat) -> float:
    """sum(y log yhat - yhat) over pixels with yhat > 0 (the objective RL ascends)."""
    y = np.asarray(y, dtype=np.float64)
    pos = yhat > 0
    return float(np.sum(y[pos] * np.log(yhat[pos]) - yhat[pos]))


# --------------------------------------------------------------------------
# DCT-entropy metric (sec. 2.2, Eqs. 1-12)
# --------------------------------------------------------------------------
def mip(vol) -> np.ndarray:
    """Maximum projection along z (sec. 2.2; Fig. 2(a))."""
    return np.asarray(vol, dtype=np.float64).max(axis=0)


def dct_basis(n: int) -> np.ndarray:
    """C[k][x] = c(k, n) cos((2x + 1) pi k / (2n)), c = sqrt(1/n) for k = 0 and
    sqrt(2/n) otherwise (Eqs. 2-4)."""
    k = np.arange(n, dtype=np.float64)[:, None]
    x = np.arange(n, dtype=np.float64)[None, :]
    c = np.full((n, 1), np.sqrt(2.0 / n))
    c[0, 0] = np.sqrt(1.0 / n)
    return c * np.cos((2 * x + 1) * np.pi * k / (2 * n))


def dct2(img) -> np.ndarray:
    """F[v][u] = sum_{y,x} f[y][x] C_v(y, M) C_u(x, N) (Eq. 1): v is the row
    (height) frequency, u the column (width) frequency."""
    img = np.asarray(img, dtype=np.float64)
    m, n = img.shape
    return dct_basis(m) @ img @ dct_basis(n).T


def triangle_mask(h: int, w: int, xs: float, ys: float) -> np.ndarray:
    """Region S of Eq. (6): mask[v][u] = u / X_S + v / Y_S < 1."""
    if not (xs > 0 and ys > 0):
        raise ValueError("triangle legs must be positive")
    v = np.arange(h, dtype=np.float64)[:, None]
    u = np.arange(w, dtype=np.float64)[None, :]
    return (u / xs + v / ys) < 1.0


REGIONS = ("triangle", "rectangle", "whole")


def region_mask(h: int, w: int, xs: float, ys: float, region: str = "triangle") -> np.ndarray:
    """Coefficients the entropy sums over: the triangle of Eq. (6), the
    rectangle u < X_S, v < Y_S that the summation limits of Eq. (12) literally
    state, or the whole matrix (the overall entropy of Fig. 2(c))."""
    if region == "triangle":
        return triangle_mask(h, w, xs, ys)
    if region == "rectangle":
        if not (xs > 0 and ys > 0):
            raise ValueError("rectangle sides must be positive")
        v = np.arange(h, dtype=np.float64)[:, None]
        u = np.arange(w, dtype=np.float64)[None, :]
        return (u < xs) & (v < ys)
    if region == "whole":
        return np.ones((h, w), dtype=bool)
    raise ValueError(f"unknown region {region!r}")


def region_area(h: int, w: int, xs: float, ys: float, region: str = "triangle") -> float:
    """Area G of the region (the entropy's prefactor is 1 / G): X_S Y_S / 2 for
    the triangle (Eq. 6), X_S Y_S for the rectangle, W H for the whole matrix."""
    return {"triangle": xs * ys / 2.0, "rectangle": xs * ys, "whole": float(h * w)}[region]


def dct_entropy(img, xs: float, ys: float, region: str = "triangle", norm: str = "full") -> float:
    """DCT entropy of a 2-D image (Eq. 12): with F the DCT of the image and n
    its 2-norm, p = |F| / n over the region S and
    e = -(1 / G) * sum_S p log2 p (0 log 0 = 0), G the area of S.

    n is the Frobenius norm of the whole coefficient matrix (norm='full'), of
    the coefficients inside S only (norm='region'), or the spectral norm (the
    largest singular value) of the whole coefficient matrix (norm='spectral').
    The default region is the triangle of Eq. (6) (G = X_S Y_S / 2).  Returns
    0 when n = 0."""
    f = dct2(img)
    h, w = f.shape
    mask = region_mask(h, w, xs, ys, region)
    if norm == "full":
        n = np.sqrt(np.sum(f * f))
    elif norm == "region":
        n = np.sqrt(np.sum(f[mask] ** 2))
    elif norm == "spectral":
        n = float(np.linalg.norm(f, 2))
    else:
        raise ValueError(f"unknown norm {norm!r}")
    if n == 0:
        return 0.0
    p = np.abs(f[mask]) / n
    p = p[p > 0]
    return float(-(1.0 / region_area(h, w, xs, ys, region)) * np.sum(p * np.log2(p)))


def metric(vol, xs: float, ys: float, region: str = "triangle", norm: str = "full") -> float:
    """Per-iterate quality metric: DCT entropy of the z maximum projection."""
    return dct_entropy(mip(vol), xs, ys, region, norm)


def stop_decision(trace, patience: int = 1, window: int = 1):
    """Apply the stopping rule to metric values trace[0] = e_1, trace[1] = e_2, ...

    The trend is read from the means of the last ``window`` values,
    s_k = mean(e_{k-window+1}, ..., e_k), defined from k = window on (window 1:
    the values themselves).  Stops at the first iteration k at which the last
    ``patience`` steps of s were all strict decreases (s_i < s_{i-1}); ties are
    not decreases.  The iterate kept is the one with the largest metric e seen
    so far (ties go to the later iterate).

    Returns (stopped, k_stop, best): ``stopped`` is False if the trace ran out
    first (k_stop is then len(trace)); ``best`` is the 1-based iteration kept."""
    if patience < 1:
        raise ValueError("patience must be >= 1")
    if window < 1:
        raise ValueError("window must be >= 1")
    best, best_e, run = 0, -np.inf, 0
    smooth = []
    for i, e in enumerate(trace):
        k = i + 1
        if k >= window:
            smooth.append(float(np.mean(trace[k - window:k])))
            if len(smooth) > 1:
                run = run + 1 if smooth[-1] < smooth[-2] else 0
        if e >= best_e:
            best, best_e = k, e
        if run >= patience:
            return True, k, best
    return False, len(trace), best


def cutoff(d_ml: float, mag: float, nnum: int, wavelength: float, na: float,
           h: int, w: int):
    """Triangle legs from the optics: pixel size P_u = d_ML / (Q Nnum) (Eq. 7),
    resolution limit d_psf = 1.22 lambda Nnum / NA (Eq. 11), X_S = P_u W / d_psf
    (Eq. 9) and Y_S = P_u H / d_psf (Eq. 10).  Lengths in one unit."""
    pu = d_ml / (mag * nnum)
    dpsf = 1.22 * wavelength * nnum / na
    return pu * w / dpsf, pu * h / dpsf


def synthetic_cutoff(nnum: int, spot_radius: float, h: int, w: int):
    """Triangle legs for synthetic PSFs given in pixel units: P_u = 1 and the
    resolution limit is Nnum times the in-focus spot diameter (Eq. 11 with the
    Airy unit replaced by the synthetic spot's diameter)."""
    dpsf = nnum * 2.0 * spot_radius
    return w / dpsf, h / dpsf


def deconvolve(psf, y, max_iters: int, xs: float, ys: float, *, stop: bool = True,
               patience: int = 1, x0=None, update: str = "rl", background: float = 0.0,
               init: str = None, region: str = "triangle", norm: str = "full",
               window: int = 1):
    """Iterations of ``update`` ('rl' or 'isra', with the constant background
    ``background``) from x^0 (``init``, see initial_volume), with the metric
    (``region``, ``norm``) evaluated on every iterate and the stopping rule
    (``patience``, ``window``) applied.  Returns (x_best, best_iter, iters_run,
    trace)."""
    y = np.asarray(y, dtype=np.float64)
    h, w = y.shape
    if init is None:
        init = "ones" if x0 is None else "given"
    x = initial_volume(psf, y, init, x0)
    if update == "rl":
        c = sensitivity(psf, h, w)
        step = lambda x: rl_step(psf, y, x, c, background)[0]  # noqa: E731
    elif update == "isra":
        d = backward(psf, y)
        step = lambda x: isra_step(psf, y, x, d, background)[0]  # noqa: E731
    else:
        raise ValueError(f"unknown update {update!r}")
    trace, iterates = [], {}
    best_x = x
    for k in range(1, max_iters + 1):
        x = step(x)
        trace.append(metric(x, xs, ys, region, norm))
        iterates[k] = x
        stopped, _, best = stop_decision(trace, patience, window)
        best_x = iterates[best]
        for kk in list(iterates):
            if kk != best and kk != k:
                del iterates[kk]
        if stop and stopped:
            return best_x, best, k, trace
    _, _, best = stop_decision(trace, patience, window)
    return iterates[best], best, max_iters, trace
