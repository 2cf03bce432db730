"""PSF sets from files: MAT and TIFF readers (and writers for round trips).

Fig. 1 of the paper names three sources for the PSF set a reconstruction
uses: computed from the optical parameters, read from a MAT file, or read from
a TIFF file.  These readers turn the two file forms into the layout every
entry point of the library takes, ``psf[nz][nnum][nnum][K][K]`` float32
(depth plane j, row phase a, column phase b, row tap u, column tap v; tap
(c0, c0) with c0 = (K - 1) / 2 lies on the source pixel).  They only move and
reorder numbers; nothing of the method is computed here.

Axis names used by ``axes`` / ``page_order``:
  ``z`` depth plane, ``a`` row phase, ``b`` column phase, ``u`` row tap,
  ``v`` column tap.

MAT files: MATLAB level 5 (v5/v6/v7) through :func:`scipy.io.loadmat`.
MATLAB light-field toolboxes usually store the set as ``H(u, v, a, b, z)``,
which scipy hands over with the same dimension order, hence the default
``axes="uvabz"``.  Level 7.3 files are HDF5 containers, which this reader does
not open (re-save them with ``-v7``).

TIFF files: a multi-page float32 stack (PIL mode ``F``), one K x K page per
(z, a, b), pages in ``page_order`` (default depth slowest, then the row phase,
then the column phase).
"""
from __future__ import annotations

from typing import Optional

import numpy as np

__all__ = ["load_psf_mat", "save_psf_mat", "load_psf_tiff", "save_psf_tiff", "check_psf"]

_CANON = "zabuv"


def check_psf(psf: np.ndarray) -> np.ndarray:
    """Validate a PSF set in the library layout and return it as contiguous
    float32.  Raises ValueError for a wrong rank, unequal phase or tap extents,
    an even support or non-finite values."""
    psf = np.asarray(psf)
    if psf.ndim != 5:
        raise ValueError(f"PSF set must have 5 axes (z, a, b, u, v), got shape {psf.shape}")
    nz, na, nb, ku, kv = psf.shape
    if nz < 1 or na < 1:
        raise ValueError(f"empty PSF set {psf.shape}")
    if na != nb:
        raise ValueError(f"row and column phase counts differ: {na} vs {nb}")
    if ku != kv or ku % 2 == 0:
        raise ValueError(f"taps must be K x K with K odd, got {ku} x {kv}")
    out = np.ascontiguousarray(psf, dtype=np.float32)
    if not np.all(np.isfinite(out)):
        raise ValueError("PSF set holds non-finite values")
    return out


def _perm(axes: str) -> tuple:
    if sorted(axes) != sorted(_CANON) or len(axes) != 5:
        raise ValueError(f"axes must be a permutation of {_CANON!r}, got {axes!r}")
    return tuple(axes.index(c) for c in _CANON)


def load_psf_mat(path: str, var: Optional[str] = None, axes: str = "uvabz") -> np.ndarray:
    """Read a PSF set from a MATLAB level-5 MAT file.

    ``var`` names the variable; when omitted the file must hold exactly one
    5-D numeric array.  ``axes`` gives the meaning of the stored array's axes
    in order (default ``"uvabz"``: ``H(u, v, a, b, z)``)."""
    from scipy import io as sio

    with open(path, "rb") as f:
        head = f.read(128)
    if b"MATLAB 7.3" in head[:116] or head[:8] == b"\x89HDF\r\n\x1a\n":
        raise ValueError(f"{path}: MAT 7.3 (HDF5) files are not read; save with -v7")
    data = sio.loadmat(path)
    if var is None:
        cands = [k for k, v in data.items()
                 if not k.startswith("__") and isinstance(v, np.ndarray) and v.ndim == 5]
        if len(cands) != 1:
            raise ValueError(f"{path}: name the PSF variable (5-D arrays found: {cands})")
        var = cands[0]
    if var not in data:
        raise KeyError(f"{path}: no variable {var!r}")
    arr = np.asarray(data[var])
    if arr.ndim != 5:
        raise ValueError(f"{path}: {var} has shape {arr.shape}, need 5 axes")
    if not np.issubdtype(arr.dtype, np.floating) and not np.issubdtype(arr.dtype, np.integer):
        raise ValueError(f"{path}: {var} is not real numeric ({arr.dtype})")
    return check_psf(np.transpose(arr, _perm(axes)))


def save_psf_mat(path: str, psf: np.ndarray, var: str = "H", axes: str = "uvabz") -> None:
    """Write a PSF set (library layout) to a MAT file with its axes in ``axes``
    order (the inverse of :func:`load_psf_mat`)."""
    from scipy import io as sio

    psf = check_psf(psf)
    inv = tuple(_CANON.index(c) for c in axes)
    sio.savemat(path, {var: np.transpose(psf, inv)}, do_compression=False)


def _page_perm(page_order: str) -> tuple:
    if sorted(page_order) != ["a", "b", "z"]:
        raise ValueError(f"page_order must be a permutation of 'zab', got {page_order!r}")
    return tuple(page_order.index(c) for c in "zab")


def load_psf_tiff(path: str, nnum: int, nz: int, page_order: str = "zab") -> np.ndarray:
    """Read a PSF set from a multi-page TIFF of nz * nnum^2 float K x K pages."""
    from PIL import Image

    pages = []
    with Image.open(path) as im:
        n = getattr(im, "n_frames", 1)
        if n != nz * nnum * nnum:
            raise ValueError(f"{path}: {n} pages, expected nz * nnum^2 = {nz * nnum * nnum}")
        for i in range(n):
            im.seek(i)
            pages.append(np.array(im, dtype=np.float64))
    shapes = {p.shape for p in pages}
    if len(shapes) != 1:
        raise ValueError(f"{path}: pages of different sizes {sorted(shapes)}")
    k = pages[0].shape
    dims = {"z": nz, "a": nnum, "b": nnum}
    stored = np.stack(pages).reshape(tuple(dims[c] for c in page_order) + k)
    return check_psf(np.transpose(stored, _page_perm(page_order) + (3, 4)))


def save_psf_tiff(path: str, psf: np.ndarray, page_order: str = "zab") -> None:
    """Write a PSF set (library layout) as a multi-page float32 TIFF, one
    K x K page per (z, a, b) in ``page_order``."""
    from PIL import Image

    psf = check_psf(psf)
    inv = tuple("zab".index(c) for c in page_order) + (3, 4)
    stored = np.transpose(psf, inv)
    k = psf.shape[3]
    flat = stored.reshape(-1, k, k)
    imgs = [Image.fromarray(np.ascontiguousarray(p, dtype=np.float32), mode="F") for p in flat]
    imgs[0].save(path, save_all=True, append_images=imgs[1:])
