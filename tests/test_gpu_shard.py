"""Depth-sharding algebra on one GPU (needs an MI355X).

Spread over several GPUs, each would hold the spectra of a group of depth
planes: its forward projection is a partial image that an all-reduce sums,
and its back projection is its own planes of the full one.  Emulated here
with one plan per depth group (uneven groups, as 31 planes over 8 GPUs are)."""
import numpy as np
import pytest

import lfrl_synth as S
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lf():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2208_11422_amd as lf
    return lf


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to("cuda:0")


def rel_l2(got, want):
    got = np.asarray(got, np.float64)
    want = np.asarray(want, np.float64)
    return float(np.linalg.norm(got - want) / np.linalg.norm(want))


@pytest.mark.parametrize("precision", [0, 1], ids=["fp32", "split-fp16"])
def test_depth_groups_sum_to_the_full_projection(lf, precision):
    nz, n, k = 7, 5, 25
    psf = S.gaussian_psf(n, nz, k, seed=71, shift_scale=None)
    h, w = 55, 60
    rng = np.random.default_rng(72)
    x = rng.uniform(0.0, 1.0, size=(nz, h, w)).astype(np.float32)
    y = rng.uniform(0.0, 1.0, size=(h, w)).astype(np.float32)
    full = lf.Plan(to_dev(psf), h, w, precision=precision)
    q = full.info["tile_q"]
    groups = [(0, 2), (2, 4), (4, 6), (6, 7)]
    plans = [lf.Plan(to_dev(psf[a:b]), h, w, tile_q=q, precision=precision) for a, b in groups]
    try:
        f_full = full.forward(to_dev(x)).cpu().numpy()
        b_full = full.backward(to_dev(y)).cpu().numpy()
        partial = [p.forward(to_dev(x[a:b])).cpu().numpy() for p, (a, b) in zip(plans, groups)]
        summed = np.zeros((h, w), np.float32)
        for part in partial:                  # the all-reduce, in rank order
            summed += part
        tol = 1e-6 if precision == 0 else 1e-4
        assert rel_l2(summed, f_full) <= tol
        assert rel_l2(summed, oracle.forward(psf, x)) <= (1e-5 if precision == 0 else 1e-3)
        for p, (a, b) in zip(plans, groups):
            part = p.backward(to_dev(y)).cpu().numpy()
            if precision == 0:
                assert np.array_equal(part, b_full[a:b])
            else:
                # FP16 spectra scales are per frequency over the plan's planes
                assert rel_l2(part, b_full[a:b]) <= 1e-3
    finally:
        full.close()
        for p in plans:
            p.close()
