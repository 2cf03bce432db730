"""The C ABI library without a GPU: it loads, exports every symbol the header
declares, and answers the host-only calls (memory estimate, optics cutoff,
argument checks that happen before any device work)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lfrl.h")
LIB = os.path.join(ROOT, "paper_2208_11422_amd", "liblfrl.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lfrl_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("liblfrl.so is not built; run __graft_entry__.build()")
    import torch  # noqa: F401  (HIP runtime shared with PyTorch)
    return ctypes.CDLL(LIB)


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert "lfrl_plan" in names and "lfrl_deconvolve" in names and "lfrl_metric" in names
    for n in names:
        assert hasattr(lib, n), n


def test_footprint_and_cutoff_without_gpu():
    import paper_2208_11422_amd as lf
    d = lf.PlanDesc(nnum=15, nz=31, ksize=255, max_h=600, max_w=600, precision=0,
                    tile_q=28, flags=0)
    res, ws = lf.lfrl_plan_footprint(d)
    nf = 28 * 15
    kk = 225 * 31
    # both layouts in MFMA fragment order, each over the 224 matrix-core indices of
    # c (forward [kk padded to 6976][c], adjoint [c][kk padded to 6976]), plus
    # the column / row of the lone index c = 224 (summed on the vector ALU)
    spec = nf * 6976 * 224 * 8 + nf * 224 * 6976 * 8 + 2 * nf * 6976 * 8
    psf_copy = 31 * 225 * 255 * 255 * 4     # the PSF kept for exact weak-voxel sums
    assert spec + psf_copy <= res < spec + psf_copy + 4096
    assert ws > nf * 16 * 225 * 31 * 8      # tile spectra of the volume
    # monotone in image size
    d2 = lf.PlanDesc(nnum=15, nz=31, ksize=255, max_h=900, max_w=900, precision=0,
                     tile_q=28, flags=0)
    assert lf.lfrl_plan_footprint(d2)[1] > ws
    # batch capacity scales the tile workspace; autotuning reports the largest candidate
    d3 = lf.PlanDesc(nnum=15, nz=31, ksize=255, max_h=600, max_w=600, precision=0,
                     tile_q=28, flags=0, max_batch=4)
    assert lf.lfrl_plan_footprint(d3)[1] > ws + 3 * nf * 16 * 225 * 31 * 8
    d4 = lf.PlanDesc(nnum=15, nz=31, ksize=255, max_h=600, max_w=600, precision=0,
                     tile_q=0, flags=0)
    d5 = lf.PlanDesc(nnum=15, nz=31, ksize=255, max_h=600, max_w=600, precision=0,
                     tile_q=0, flags=lf.PLAN_AUTOTUNE)
    r4, w4 = lf.lfrl_plan_footprint(d4)
    r5, w5 = lf.lfrl_plan_footprint(d5)
    assert r5 >= r4 and w5 >= w4
    # normalising the PSF copy costs no extra memory
    d6 = lf.PlanDesc(nnum=15, nz=31, ksize=255, max_h=600, max_w=600, precision=0,
                     tile_q=28, flags=lf.NORMALIZE_PSF)
    assert lf.lfrl_plan_footprint(d6) == (res, ws)
    xs, ys = lf.lfrl_metric_cutoff(150.0, 40.0, 15, 0.525, 0.95, 450, 600)
    assert xs == pytest.approx(0.25 * 600 / (1.22 * 0.525 * 15 / 0.95), rel=1e-12)
    assert ys == pytest.approx(0.25 * 450 / (1.22 * 0.525 * 15 / 0.95), rel=1e-12)


@pytest.mark.parametrize("field,value", [("ksize", 24), ("nnum", 0), ("max_h", 601),
                                         ("precision", 7), ("flags", 4), ("tile_q", 3),
                                         ("max_batch", 17), ("max_batch", -1)])
def test_footprint_rejects_bad_descriptions(field, value):
    import paper_2208_11422_amd as lf
    d = lf.PlanDesc(nnum=15, nz=31, ksize=255, max_h=600, max_w=600, precision=0,
                    tile_q=28, flags=0)
    setattr(d, field, value)
    with pytest.raises(lf.LfrlError):
        lf.lfrl_plan_footprint(d)


def test_null_arguments_rejected_before_device_work(lib):
    import paper_2208_11422_amd as lf
    assert lib.lfrl_forward(None, 15, 15, None, None, None) == -1
    assert lib.lfrl_backward(None, 15, 15, None, None, None) == -1
    h = ctypes.c_void_p()
    d = lf.PlanDesc(nnum=3, nz=2, ksize=5, max_h=12, max_w=12, precision=0, tile_q=0, flags=0)
    assert lf._load().lfrl_plan(ctypes.byref(h), ctypes.byref(d), None, None) == -1
    assert "psf" in lf.lfrl_last_error()
    assert lib.lfrl_plan_destroy(None) == 0


@pytest.mark.parametrize("region,norm,xs,msg", [
    (3, 0, 4.0, "region"),
    (-1, 0, 4.0, "region"),
    (0, 3, 4.0, "norm"),
    (0, 0, 0.0, "legs"),
    (1, 0, 300.0, "legs"),
])
def test_metric_variant_arguments_rejected_before_device_work(region, norm, xs, msg):
    """Unknown regions and norms, and legs the triangle or rectangle cannot
    take, are argument errors raised before any device work."""
    import paper_2208_11422_amd as lf
    lib = lf._load()
    fake = ctypes.c_void_p(0x1000)
    rc = lib.lfrl_metric_ex(1, 16, 16, fake, xs, 4.0, region, norm, fake, None)
    assert rc in (-1, -4)
    assert msg in lf.lfrl_last_error()


def test_rl_opts_layout_and_defaults():
    """The option struct keeps the header's field order (a zero-filled tail is
    the method as the paper states it), and the keyword helper fills it."""
    import paper_2208_11422_amd as lf
    names = [f for f, _ in lf.RlOpts._fields_]
    text = open(HEADER).read()
    body = text[text.index("typedef struct {\n    int32_t max_iters;"):]
    body = body[:body.index("} lfrl_rl_opts;")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    declared = re.findall(r"\b(?:int32_t|double)\s+([a-z_, ]+);", body)
    flat = [n.strip() for grp in declared for n in grp.split(",")]
    assert names == flat
    o = lf.RlOpts(max_iters=3)
    assert (o.update, o.region, o.norm, o.window, o.background) == (0, 0, 0, 0, 0.0)
    o = lf.rl_opts(5, lf.STOP_METRIC, 2, 3.0, 4.0, update=lf.UPDATE_ISRA, background=2.5,
                   backproject_start=True, region=lf.REGION_WHOLE, norm=lf.NORM_REGION, window=3)
    assert (o.init, o.update, o.region, o.norm, o.window, o.background) == (2, 1, 2, 1, 3, 2.5)
    with pytest.raises(lf.LfrlError):
        lf.rl_opts(5, given_start=True, backproject_start=True)


@pytest.mark.parametrize("field,value,code", [
    ("ksize", 24, -1), ("osr", 2, -1), ("na", 1.1, -1), ("wavelength", 0.0, -1),
    ("f_ml", float("nan"), -1), ("nnum", 0, -1), ("nquad", -3, -1),
    ("ksize", 1025, -4),   # ksize * osr above the largest field grid
])
def test_psf_optics_arguments_rejected_before_device_work(field, value, code):
    """Optical parameters are checked on the host before anything touches the
    device (the psf pointer is never dereferenced here)."""
    import paper_2208_11422_amd as lf
    o = lf.Optics(wavelength=0.52, na=0.5, n_medium=1.0, mag=20.0, d_ml=150.0, f_ml=3000.0,
                  nnum=15, nz=2, ksize=255, osr=3, nquad=0, flags=0)
    setattr(o, field, value)
    z = (ctypes.c_double * 2)(-1.0, 1.0)
    rc = lf._load().lfrl_psf_compute(ctypes.byref(o), z, ctypes.c_void_p(0x1000), None)
    assert rc == code, lf.lfrl_last_error()
    bad = (ctypes.c_double * 2)(0.0, float("inf"))
    o2 = lf.Optics(wavelength=0.52, na=0.5, n_medium=1.0, mag=20.0, d_ml=150.0, f_ml=3000.0,
                   nnum=15, nz=2, ksize=255, osr=3, nquad=0, flags=0)
    assert lf._load().lfrl_psf_compute(ctypes.byref(o2), bad, ctypes.c_void_p(0x1000), None) == -1
    assert "depth" in lf.lfrl_last_error()
