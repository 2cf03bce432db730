"""Split precision modes against the float64 oracle (needs an MI355X).

16-bit PSF spectra (FP16 or BF16, per-frequency power-of-two scale) and
hi/lo-split 16-bit tile spectra on matrix cores with FP32 accumulation.  Bar:
relative L2 error <= 1e-3 against the oracle, for single projections and for
every iterate of a 30-iteration deconvolution of the Nnum 5, 55 x 55,
5-plane workload."""
import numpy as np
import pytest

import lfrl_synth as S
import oracle

pytestmark = pytest.mark.gpu

TOL = 1e-3


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


PRECS = [pytest.param(1, id="fp16"), pytest.param(2, id="bf16")]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("n,ly,lx,nz,k,q", [(5, 11, 11, 5, 25, 0), (5, 11, 11, 5, 25, 10),
                                            (3, 7, 9, 3, 11, 0), (15, 4, 4, 2, 31, 0),
                                            (7, 5, 6, 3, 21, 0), (9, 4, 5, 2, 27, 0),
                                            (1, 20, 17, 3, 7, 0)])
def test_projections_split(lf, n, ly, lx, nz, k, q, prec):
    psf = S.gaussian_psf(n, nz, k, seed=40 + n, shift_scale=None)
    h, w = n * ly, n * lx
    rng = np.random.default_rng(41)
    x = rng.uniform(0.0, 1.0, size=(nz, h, w)).astype(np.float32)
    y = rng.uniform(0.0, 1.0, size=(h, w)).astype(np.float32)
    plan = lf.Plan(to_dev(psf), h, w, tile_q=q, precision=prec)
    try:
        ef = rel_l2(plan.forward(to_dev(x)).cpu().numpy(), oracle.forward(psf, x))
        eb = rel_l2(plan.backward(to_dev(y)).cpu().numpy(), oracle.backward(psf, y))
        print(f"split {'BF16' if prec == 2 else 'FP16'} N={n} {h}x{w} nz={nz} K={k} Q={plan.info['tile_q']}: "
              f"forward {ef:.2e}, backward {eb:.2e}", flush=True)
        assert ef <= TOL and eb <= TOL
    finally:
        plan.close()


@pytest.fixture(scope="module")
def small_run():
    """The small workload's image and the oracle's iterates x^0 .. x^50."""
    p = S.preset("small")
    psf = p["psf_array"]
    y = S.measure(oracle.forward(psf, p["x_true"]), p["peak"], p["background"], p["noise_seed"])
    return p, y, oracle.rl(psf, y, 50, keep_all=True)


def split_errors(lf, small_run, prec, iters):
    """Relative L2 error of every iterate 1..iters against the oracle (one
    fixed-length deconvolution per count, so each is the returned volume)."""
    import torch
    p, y, ref = small_run
    g = p["geometry"]
    plan = lf.Plan(to_dev(p["psf_array"]), g.h, g.w, precision=prec)
    errs = []
    try:
        y_d = to_dev(y)
        for it in range(1, iters + 1):
            vol, _ = plan.deconvolve(y_d, it, stop=lf.STOP_NONE)
            torch.cuda.synchronize()
            errs.append(rel_l2(vol.cpu().numpy(), ref[it]))
    finally:
        plan.close()
    name = "BF16" if prec == 2 else "FP16"
    print(f"split {name} per-iteration rel L2:",
          " ".join(f"{i + 1}:{e:.2e}" for i, e in enumerate(errs)), flush=True)
    return errs


@pytest.mark.parametrize("prec", PRECS)
def test_rl_30_iterations_split(lf, small_run, prec):
    """Relative L2 error vs the oracle at every one of 30 iterates."""
    errs = split_errors(lf, small_run, prec, 30)
    assert max(errs) <= TOL


def test_rl_50_iterations_split_fp16(lf, small_run):
    """Split FP16 stays within the bar at every iterate up to the serving cap
    of 50 iterations."""
    errs = split_errors(lf, small_run, 1, 50)
    assert max(errs) <= TOL


def test_split_footprint_is_half(lf):
    d32 = lf.PlanDesc(nnum=15, nz=31, ksize=255, max_h=600, max_w=600, precision=lf.FP32,
                      tile_q=28, flags=0)
    d16 = lf.PlanDesc(nnum=15, nz=31, ksize=255, max_h=600, max_w=600, precision=lf.SPLIT_FP16,
                      tile_q=28, flags=0)
    psf_copy = 31 * 225 * 255 * 255 * 4
    r32 = lf.lfrl_plan_footprint(d32)[0] - psf_copy
    r16 = lf.lfrl_plan_footprint(d16)[0] - psf_copy
    assert 0.45 < r16 / r32 < 0.55
