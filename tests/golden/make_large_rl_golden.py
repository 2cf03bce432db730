"""Write tests/golden/large_rl_iterates.json: Richardson-Lucy iterates of the
full-size light-field workload at sampled voxels, computed by the CPU oracle
alone.

Workload: Nnum 15, 40 x 40 lenslets (600 x 600 image), 31 planes, the seeded
255 x 255 defocus-disk PSF set of the large preset, and a seeded uniform image
y ~ U(10, 2000) (float32).  Update (sec. 1, the Richardson-Lucy iteration of
the light-field model):

    x^0 = 1,   c = A^T 1,   x^k = x^{k-1} * A^T( y / A x^{k-1} ) / c,

with y / A x := 0 where A x <= 0 and x := 0 where c <= 0.

The oracle cannot run whole iterations at this size, so the iterates are
evaluated only where they are needed, window by window.  A back-projected
voxel reads pixels up to c0 = 127 away and a projected pixel reads voxels up
to c0 away, so x^2 on the corner window rows/cols [0, 16) needs
    rho^1 = y / A x^1  on pixels  [0, 16 + 127),
    x^1               on voxels  [0, 16 + 2*127)  (every plane),
    rho^0 = y / A 1    on pixels  [0, 16 + 3*127).
Each quantity is computed exactly on its window; values outside a window
are never read by the next step.

Stored: for the corner window (every voxel of five planes, including the
first and last, plus every weakly observed voxel of the other planes:
A^T 1 below 1e-2 of the largest) c, x^1 and x^2; for an interior window
(300 random voxels of rows/cols [292, 308), all planes) x^1.

Runs for several minutes on 8 cores; it calls only the oracle and the input
generators:  python tests/golden/make_large_rl_golden.py
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import lfrl_synth as S  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(HERE, "large_rl_iterates.json")
CACHE = "/tmp/lfrl_synth_cache"
IMAGE_SEED = 4101
WIN = 16
CORNER_PLANES = (0, 1, 15, 29, 30)
WEAK_REL = 1e-2


def image(h: int, w: int) -> np.ndarray:
    return np.random.default_rng(IMAGE_SEED).uniform(10.0, 2000.0, size=(h, w)).astype(np.float32)


def psf_checksum(psf: np.ndarray) -> list[float]:
    p = psf.astype(np.float64)
    return [float(p.sum()), float((p * p).sum())]


def log(msg: str) -> None:
    print(msg, flush=True)


def voxel_grid(nz_list, r0, r1, s0, s1):
    jj, rr, ss = np.meshgrid(np.asarray(nz_list), np.arange(r0, r1), np.arange(s0, s1),
                             indexing="ij")
    return jj.ravel(), rr.ravel(), ss.ravel()


def main() -> int:
    p = S.preset("large", cache_dir=CACHE)
    psf = p["psf_array"]
    g = p["geometry"]
    nz, h, w = g.nz, g.h, g.w
    c0 = (g.ksize - 1) // 2
    y = image(h, w).astype(np.float64)
    ones_img = np.ones((h, w))
    ones_vol = np.ones((nz, h, w))
    t_all = time.time()

    # ---- corner window: x^1 and x^2 -------------------------------------
    p1 = min(h, WIN + c0)          # pixels of rho^1
    v1 = min(h, WIN + 2 * c0)      # voxels of x^1
    p0 = min(h, WIN + 3 * c0)      # pixels of rho^0
    t = time.time()
    a1 = oracle.forward_window(psf, ones_vol, 0, p0, 0, p0)
    log(f"A 1 on [0,{p0})^2: {time.time() - t:.1f} s")
    rho0 = np.zeros((h, w))
    pos = a1 > 0
    rho0[:p0, :p0][pos] = y[:p0, :p0][pos] / a1[pos]
    t = time.time()
    jj, rr, ss = voxel_grid(range(nz), 0, v1, 0, v1)
    c_v1 = oracle.backward_at(psf, ones_img, jj, rr, ss)
    b_v1 = oracle.backward_at(psf, rho0, jj, rr, ss)
    x1_v1 = np.where(c_v1 > 0, b_v1 / np.where(c_v1 > 0, c_v1, 1.0), 0.0)
    log(f"x^1 on {nz} x [0,{v1})^2: {time.time() - t:.1f} s")
    x1 = np.zeros((nz, h, w))
    x1[:, :v1, :v1] = x1_v1.reshape(nz, v1, v1)
    c_full = np.zeros((nz, h, w))
    c_full[:, :v1, :v1] = c_v1.reshape(nz, v1, v1)
    t = time.time()
    ax1 = oracle.forward_window(psf, x1, 0, p1, 0, p1)
    log(f"A x^1 on [0,{p1})^2: {time.time() - t:.1f} s")
    rho1 = np.zeros((h, w))
    pos = ax1 > 0
    rho1[:p1, :p1][pos] = y[:p1, :p1][pos] / ax1[pos]
    # the voxels kept: five whole planes and the weak voxels of the others
    cmax = float(c_v1.max())
    keep = []
    for j in range(nz):
        for r in range(WIN):
            for s in range(WIN):
                if j in CORNER_PLANES or c_full[j, r, s] < WEAK_REL * cmax:
                    keep.append((j, r, s))
    kj, kr, ks = (np.array(v) for v in zip(*keep))
    b2 = oracle.backward_at(psf, rho1, kj, kr, ks)
    ck = c_full[kj, kr, ks]
    x1k = x1[kj, kr, ks]
    x2k = np.where(ck > 0, x1k * b2 / np.where(ck > 0, ck, 1.0), 0.0)
    corner = {"name": "corner", "rows": [0, WIN], "cols": [0, WIN],
              "planes_whole": list(CORNER_PLANES), "c_max": cmax,
              "voxels": [[int(a), int(b), int(c)] for a, b, c in keep],
              "c": ck.tolist(), "x1": x1k.tolist(), "x2": x2k.tolist()}
    log(f"corner: {len(keep)} voxels, {int((ck < WEAK_REL * cmax).sum())} weak")

    # ---- interior window: x^1 --------------------------------------------
    r0, r1 = 292, 292 + WIN
    t = time.time()
    lo, hi = r0 - c0, r1 + c0
    a1i = oracle.forward_window(psf, ones_vol, lo, hi, lo, hi)
    log(f"A 1 on [{lo},{hi})^2: {time.time() - t:.1f} s")
    rhoi = np.zeros((h, w))
    pos = a1i > 0
    rhoi[lo:hi, lo:hi][pos] = y[lo:hi, lo:hi][pos] / a1i[pos]
    rng = np.random.default_rng(4102)
    n = 300
    ij = rng.integers(0, nz, n)
    ir = rng.integers(r0, r1, n)
    is_ = rng.integers(r0, r1, n)
    ci = oracle.backward_at(psf, ones_img, ij, ir, is_)
    bi = oracle.backward_at(psf, rhoi, ij, ir, is_)
    x1i = np.where(ci > 0, bi / np.where(ci > 0, ci, 1.0), 0.0)
    interior = {"name": "interior", "rows": [r0, r1], "cols": [r0, r1],
                "voxels": [[int(a), int(b), int(c)] for a, b, c in zip(ij, ir, is_)],
                "c": ci.tolist(), "x1": x1i.tolist()}

    out = {
        "_source": "Written by tests/golden/make_large_rl_golden.py from the CPU oracle "
                   "(float64 direct sums) alone. Richardson-Lucy update of sec. 1: "
                   "x^k = x^{k-1} * A^T(y / A x^{k-1}) / A^T 1, ones start; values at "
                   "sampled voxels (plane, row, column).",
        "workload": {"preset": "large", "nnum": g.nnum, "h": h, "w": w, "nz": nz,
                     "ksize": g.ksize, "psf_checksum": psf_checksum(psf)},
        "image": {"generator": "numpy default_rng(seed).uniform(10, 2000, (h, w)) as float32",
                  "seed": IMAGE_SEED},
        "windows": [corner, interior],
    }
    with open(OUT, "w") as f:
        json.dump(out, f, indent=0)
        f.write("\n")
    log(f"wrote {OUT} in {time.time() - t_all:.0f} s")
    return 0


if __name__ == "__main__":
    sys.exit(main())
