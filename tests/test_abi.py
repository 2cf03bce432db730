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
    # both layouts in MFMA fragment order: forward [kk padded to 6976][c padded to 240],
    # adjoint [c padded to 232][kk padded to 6976]
    spec = nf * 6976 * 240 * 8 + nf * 232 * 6976 * 8
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
    xs, ys = lf.lfrl_metric_cutoff(150.0, 40.0, 15, 0.525, 0.95, 450, 600)
    assert xs == pytest.approx(0.25 * 600 / (1.22 * 0.525 * 15 / 0.95), rel=1e-12)
    assert ys == pytest.approx(0.25 * 450 / (1.22 * 0.525 * 15 / 0.95), rel=1e-12)


@pytest.mark.parametrize("field,value", [("ksize", 24), ("nnum", 0), ("max_h", 601),
                                         ("precision", 7), ("flags", 2), ("tile_q", 3),
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
