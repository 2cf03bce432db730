"""The allocation-free metric entry point (lfrl_metric_noalloc) against the
allocating one (lfrl_metric_ex) through the C ABI (needs an MI355X).

Both run the same kernels, the first on the library's fixed per-GPU scratch
array, the second on its growable buffer, so their results must agree bit for
bit.  Two calls in a row, the second on a smaller input, check that leftovers
of the first call in the shared array do not leak into the second."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lf():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import os

    import paper_2208_11422_amd as lf
    assert os.path.exists(lf.library_path()), "liblfrl.so missing: build first"
    return lf


def _vol(nz, h, w, seed):
    rng = np.random.default_rng(seed)
    vol = rng.uniform(0.0, 1.0, size=(nz, h, w)).astype(np.float32)
    vol[:, h // 3:h // 2, w // 4:w // 2] += 3.0
    return vol


def _both(lf, vol, xs, ys, region, norm):
    import torch
    dev = torch.device("cuda:0")
    nz, h, w = vol.shape
    img = torch.from_numpy(vol).to(dev)
    a = torch.full((1,), -7.0, dtype=torch.float64, device=dev)
    b = torch.full((1,), -9.0, dtype=torch.float64, device=dev)
    lf.lfrl_metric_noalloc(nz, h, w, img, xs, ys, region, norm, a)
    lf.lfrl_metric_ex(nz, h, w, img, xs, ys, region, norm, b)
    torch.cuda.synchronize()
    return float(a.item()), float(b.item())


@pytest.mark.parametrize("first,second", [
    # large path (projection, row chunks, coefficients, final) then the one-block path
    ((31, 600, 600, 10.0, 10.0, 0, 0), (5, 55, 55, 5.5, 5.5, 0, 0)),
    # largest image served, rectangle with the region norm, then a smaller triangle
    ((3, 1024, 1024, 256.0, 200.0, 1, 1), (2, 300, 200, 40.0, 30.0, 0, 0)),
    # spectral norm, then a smaller image with the Frobenius norm
    ((1, 400, 500, 12.0, 9.0, 0, 2), (4, 128, 96, 6.0, 6.0, 1, 0)),
])
def test_noalloc_matches_allocating_metric(lf, first, second):
    region_names = {0: "triangle", 1: "rectangle"}
    norm_names = {0: "full", 1: "region", 2: "spectral"}
    for i, (nz, h, w, xs, ys, region, norm) in enumerate((first, second)):
        vol = _vol(nz, h, w, seed=h * w + nz + i)
        print(f"case nz={nz} {h}x{w} legs=({xs},{ys}) region={region} norm={norm}", flush=True)
        got, ref = _both(lf, vol, xs, ys, region, norm)
        assert got == ref, (got, ref)
        if h * w <= 300 * 200:
            want = oracle.metric(vol.astype(np.float64), xs, ys, region_names[region],
                                 norm_names[norm])
            assert got == pytest.approx(want, rel=1e-9)


def test_noalloc_refuses_beyond_its_limits(lf):
    import torch
    dev = torch.device("cuda:0")
    out = torch.zeros(1, dtype=torch.float64, device=dev)
    big = torch.zeros((1, 1025, 64), dtype=torch.float32, device=dev)
    with pytest.raises(lf.LfrlError) as e:
        lf.lfrl_metric_noalloc(1, 1025, 64, big, 5.0, 5.0, 0, 0, out)
    assert e.value.code == -4
    img = torch.zeros((1, 64, 64), dtype=torch.float32, device=dev)
    with pytest.raises(lf.LfrlError) as e:
        lf.lfrl_metric_noalloc(1, 64, 64, img, 5.0, 5.0, 2, 0, out)
    assert e.value.code == -4
    with pytest.raises(lf.LfrlError) as e:
        lf.lfrl_metric_noalloc(1, 64, 64, img, 300.0, 5.0, 0, 0, out)
    assert e.value.code == -4
