"""Parity of the variants of the update, the start volume, the metric and the
stop rule with the CPU oracle (needs an MI355X).

Workload: the Nnum 5, 55 x 55, 5-plane synthetic problem whose measurement
carries a constant background of 10 counts, so the background term of the
image model has something to model.  Every call goes through the C ABI.
Floating-point bar as for the plain method: relative L2 <= 1e-5 (FP32 path),
<= 1e-3 (split precision); metric values relative 1e-9 on float32 inputs."""
import numpy as np
import pytest

import lfrl_synth as S
import oracle

pytestmark = pytest.mark.gpu

TOL = 1e-5
TOL_SPLIT = 1e-3


@pytest.fixture(scope="module")
def lf():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2208_11422_amd as lf
    import os
    assert os.path.exists(lf.library_path()), "liblfrl.so missing: build first"
    return lf


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to("cuda:0")


def rel_l2(got, want):
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    return float(np.linalg.norm(got - want) / np.linalg.norm(want))


def small_problem():
    p = S.preset("small")
    g = p["geometry"]
    psf = p["psf_array"]
    y = S.measure(oracle.forward(psf, p["x_true"]), p["peak"], p["background"], p["noise_seed"])
    xs, ys = oracle.synthetic_cutoff(g.nnum, p["spot_radius"], g.h, g.w)
    return p, psf, y, xs, ys


@pytest.fixture(scope="module")
def problem(lf):
    p, psf, y, xs, ys = small_problem()
    g = p["geometry"]
    plan = lf.Plan(to_dev(psf), g.h, g.w)
    yield p, psf, y, xs, ys, plan
    plan.close()


@pytest.mark.parametrize("update,init", [("rl", "ones"), ("isra", "ones"),
                                         ("rl", "backprojection"), ("isra", "backprojection")])
def test_update_variants_match_oracle(lf, problem, update, init):
    import torch
    p, psf, y, xs, ys, plan = problem
    b = float(p["background"])
    ref = oracle.rl(psf, y, 5, keep_all=True, update=update, background=b, init=init)
    kw = dict(update=lf.UPDATE_ISRA if update == "isra" else lf.UPDATE_RL, background=b,
              backproject_start=init == "backprojection")
    for k in (1, 2, 5):
        print(f"case {update} start={init} b={b} iters={k}", flush=True)
        vol, rep = plan.deconvolve(to_dev(y), k, **kw)
        torch.cuda.synchronize()
        assert rep["iters_run"] == k
        err = rel_l2(vol.cpu().numpy(), ref[k])
        print(f"  rel L2 {err:.2e}", flush=True)
        assert err <= TOL


def test_background_changes_the_result(lf, problem):
    """The background enters the model: b = 0 and b = 10 give different
    iterates, each matching its own oracle run."""
    import torch
    p, psf, y, xs, ys, plan = problem
    for b in (0.0, 10.0):
        vol, _ = plan.deconvolve(to_dev(y), 3, background=b)
        torch.cuda.synchronize()
        assert rel_l2(vol.cpu().numpy(), oracle.rl(psf, y, 3, background=b)) <= TOL
    v0, _ = plan.deconvolve(to_dev(y), 3, background=0.0)
    v1, _ = plan.deconvolve(to_dev(y), 3, background=10.0)
    torch.cuda.synchronize()
    assert rel_l2(v0.cpu().numpy(), v1.cpu().numpy()) > 1e-3


def test_isra_weakly_observed_voxels(lf):
    """Corner voxels that send ~1e-6 of their light into the image: the ISRA
    numerator A^T y and denominator A^T(A x + b) there are window sums in
    float64, so those voxels match the oracle too."""
    import torch
    n, ly, nz, k = 3, 10, 3, 41
    psf = S.gaussian_psf(n, nz, k, seed=21, shift_scale=6.0)
    h = w = n * ly
    c = oracle.sensitivity(psf, h, w)
    assert (c < 1e-4 * c.max()).sum() >= 4
    rng = np.random.default_rng(23)
    y = rng.uniform(10.0, 100.0, size=(h, w)).astype(np.float32)
    ref = oracle.rl(psf, y, 4, keep_all=True, update="isra", background=2.0,
                    init="backprojection")
    plan = lf.Plan(to_dev(psf), h, w)
    try:
        for it in (1, 4):
            vol, rep = plan.deconvolve(to_dev(y), it, update=lf.UPDATE_ISRA, background=2.0,
                                       backproject_start=True)
            torch.cuda.synchronize()
            assert rep["weak_voxels"] > 0
            got = vol.cpu().numpy()
            err = rel_l2(got, ref[it])
            print(f"iter {it}: rel L2 {err:.2e}", flush=True)
            assert err <= TOL
            weak = c < 1e-2 * c.max()
            np.testing.assert_allclose(got[weak], ref[it][weak], rtol=1e-5,
                                       atol=1e-6 * np.abs(ref[it]).max())
    finally:
        plan.close()


@pytest.mark.parametrize("precision", ["fp16", "bf16"])
def test_isra_split_precision(lf, precision):
    import torch
    p, psf, y, xs, ys = small_problem()
    g = p["geometry"]
    prec = lf.SPLIT_FP16 if precision == "fp16" else lf.SPLIT_BF16
    ref = oracle.rl(psf, y, 3, update="isra", background=float(p["background"]))
    plan = lf.Plan(to_dev(psf), g.h, g.w, precision=prec)
    try:
        vol, _ = plan.deconvolve(to_dev(y), 3, update=lf.UPDATE_ISRA,
                                 background=float(p["background"]))
        torch.cuda.synchronize()
        err = rel_l2(vol.cpu().numpy(), ref)
        print(f"{precision}: rel L2 {err:.2e}", flush=True)
        assert err <= TOL_SPLIT
    finally:
        plan.close()


@pytest.mark.parametrize("region", ["triangle", "rectangle", "whole"])
@pytest.mark.parametrize("norm", ["full", "region", "spectral"])
@pytest.mark.parametrize("nz,h,w,xs,ys", [(1, 55, 55, 5.5, 5.5), (3, 40, 64, 7.3, 3.9),
                                         (1, 600, 600, 10.0, 10.0), (2, 300, 420, 230.0, 180.0)])
def test_metric_variants_match_oracle(lf, region, norm, nz, h, w, xs, ys):
    rng = np.random.default_rng(h * w + nz)
    vol = rng.uniform(0.0, 1.0, size=(nz, h, w)).astype(np.float32)
    vol[:, h // 3:h // 2, w // 4:w // 2] += 3.0
    img = vol[0] if nz == 1 else vol
    reg = {"triangle": lf.REGION_TRIANGLE, "rectangle": lf.REGION_RECTANGLE,
           "whole": lf.REGION_WHOLE}[region]
    nrm = {"full": lf.NORM_MATRIX, "region": lf.NORM_REGION, "spectral": lf.NORM_SPECTRAL}[norm]
    got = lf.metric(to_dev(img), xs, ys, region=reg, norm=nrm)
    want = oracle.metric(vol, xs, ys, region, norm)
    assert got == pytest.approx(want, rel=1e-9)


def test_window_stop_and_metric_variants_in_the_loop(lf, problem):
    """Metric trace on the rectangle with the region norm, and the window-mean
    stop rule, over 30 iterations of RL with the background term."""
    import torch
    p, psf, y, xs, ys, plan = problem
    b = float(p["background"])
    iters, window = 30, 3
    _, _, _, ref_trace = oracle.deconvolve(psf, y, iters, xs, ys, stop=False, background=b,
                                           region="rectangle", norm="region", window=window)
    kw = dict(background=b, region=lf.REGION_RECTANGLE, norm=lf.NORM_REGION, window=window)
    vol, rep = plan.deconvolve(to_dev(y), iters, stop=lf.STOP_TRACK, xs=xs, ys=ys, **kw)
    torch.cuda.synchronize()
    tr = np.array(rep["metric_trace"])
    np.testing.assert_allclose(tr, ref_trace, rtol=TOL)
    stopped, k_stop, best = oracle.stop_decision(list(ref_trace), 1, window)
    assert rep["best_iter"] == oracle.stop_decision(list(ref_trace), 10 ** 6, window)[2]
    vol2, rep2 = plan.deconvolve(to_dev(y), iters, stop=lf.STOP_METRIC, xs=xs, ys=ys, **kw)
    torch.cuda.synchronize()
    print(f"oracle: stopped={stopped} k={k_stop} best={best}; "
          f"gpu: stopped={rep2['stopped']} k={rep2['iters_run']} best={rep2['best_iter']}",
          flush=True)
    assert (rep2["stopped"] == 1) == stopped
    assert rep2["iters_run"] == k_stop
    assert rep2["best_iter"] == best
    ref_best = oracle.rl(psf, y, best, background=b)
    assert rel_l2(vol2.cpu().numpy(), ref_best) <= TOL


def test_spectral_norm_in_the_loop(lf, problem):
    """The spectral-norm reading tracked over the iterations of RL with the
    background term."""
    import torch
    p, psf, y, xs, ys, plan = problem
    b = float(p["background"])
    _, best, _, ref_trace = oracle.deconvolve(psf, y, 8, xs, ys, stop=False, background=b,
                                              norm="spectral")
    _, rep = plan.deconvolve(to_dev(y), 8, stop=lf.STOP_TRACK, xs=xs, ys=ys, background=b,
                             norm=lf.NORM_SPECTRAL)
    torch.cuda.synchronize()
    np.testing.assert_allclose(np.array(rep["metric_trace"]), ref_trace, rtol=TOL)
    assert rep["best_iter"] == best


@pytest.mark.parametrize("size", ["small", "large"])
@pytest.mark.parametrize("case", ["equal_top_pair", "rank_one", "tall", "wide", "zero"])
def test_spectral_norm_hard_spectra(lf, case, size):
    """The Lanczos spectral norm where the iteration is stressed: two equal
    largest singular values, a rank-one image (the Krylov space closes after
    one step), tall and wide images, and zero.  Small images run the one-block
    kernel, large ones (16384 pixels and up) the multi-block one."""
    rng = np.random.default_rng(7)
    big = size == "large"
    if case == "equal_top_pair":
        n = 240 if big else 120
        img = np.zeros((n, n))
        a, b = n // 12, n // 3
        img[a:b, a:b] = 5.0
        img[n - b:n - a, n - b:n - a] = 5.0       # block-diagonal: sigma_1 = sigma_2
        img += 1e-3 * rng.uniform(size=img.shape)
    elif case == "rank_one":
        img = np.outer(rng.uniform(1, 2, 300 if big else 90), rng.uniform(1, 2, 250 if big else 70))
    elif case == "tall":
        img = rng.uniform(0, 1, (500, 40) if big else (200, 30))
    elif case == "wide":
        img = rng.uniform(0, 1, (30, 700) if big else (20, 300))
    else:
        img = np.zeros((200, 160) if big else (64, 48))
    assert (img.size >= 16384) == big
    img = img.astype(np.float32)
    got = lf.metric(to_dev(img), 4.0, 3.0, region=lf.REGION_TRIANGLE, norm=lf.NORM_SPECTRAL)
    want = oracle.metric(img[None], 4.0, 3.0, "triangle", "spectral")
    assert got == pytest.approx(want, rel=1e-9, abs=1e-300)


def test_spectral_norm_size_limit(lf):
    """The one-block Lanczos iteration holds h + w values: larger images are
    refused before any device work."""
    import torch
    out = torch.empty(1, dtype=torch.float64, device="cuda:0")
    img = torch.zeros((8, 6200), dtype=torch.float32, device="cuda:0")
    with pytest.raises(lf.LfrlError):
        lf.lfrl_metric_ex(1, 8, 6200, img, 2.0, 2.0, lf.REGION_TRIANGLE, lf.NORM_SPECTRAL, out)


def test_whole_region_in_the_loop(lf, problem):
    """The overall entropy of Fig. 2(c) tracked over the iterations."""
    import torch
    p, psf, y, xs, ys, plan = problem
    _, _, _, ref_trace = oracle.deconvolve(psf, y, 6, xs, ys, stop=False, region="whole")
    _, rep = plan.deconvolve(to_dev(y), 6, stop=lf.STOP_TRACK, xs=xs, ys=ys,
                             region=lf.REGION_WHOLE)
    torch.cuda.synchronize()
    np.testing.assert_allclose(np.array(rep["metric_trace"]), ref_trace, rtol=TOL)


def test_mixed_update_jobs_share_launches(lf, problem):
    """An RL job and an ISRA job (different backgrounds) on one plan, stepped
    together: each equals its own run alone, bit for bit, and its oracle."""
    import torch
    p, psf, y, xs, ys, plan = problem
    yd = to_dev(y)
    specs = [dict(update=lf.UPDATE_RL, background=10.0),
             dict(update=lf.UPDATE_ISRA, background=4.0, backproject_start=True)]
    alone = []
    for kw in specs:
        j = lf.Job(plan, yd, 4, **kw)
        while lf.Job.step([j]):
            pass
        alone.append(j.result()[0].clone())
        j.close()
    jobs = [lf.Job(plan, yd, 4, **kw) for kw in specs]
    while lf.Job.step(jobs):
        pass
    together = [j.result()[0] for j in jobs]
    for j in jobs:
        j.close()
    torch.cuda.synchronize()
    for a, t in zip(alone, together):
        assert torch.equal(a, t)
    assert rel_l2(together[0].cpu().numpy(), oracle.rl(psf, y, 4, background=10.0)) <= TOL
    want = oracle.rl(psf, y, 4, update="isra", background=4.0, init="backprojection")
    assert rel_l2(together[1].cpu().numpy(), want) <= TOL


def test_graph_replay_keys_on_the_variants(lf, problem):
    """Fixed-length runs replay a captured graph; changing a variant option
    must capture a new one, not replay the old."""
    import torch
    p, psf, y, xs, ys, plan = problem
    yd = to_dev(y)
    out = torch.empty((psf.shape[0],) + y.shape, dtype=torch.float32, device="cuda:0")
    for kw, ref in [
        (dict(update=lf.UPDATE_ISRA, background=10.0), ("isra", 10.0)),
        (dict(update=lf.UPDATE_ISRA, background=10.0), ("isra", 10.0)),   # replay
        (dict(update=lf.UPDATE_ISRA, background=2.0), ("isra", 2.0)),
        (dict(update=lf.UPDATE_RL, background=2.0), ("rl", 2.0)),
    ]:
        _, rep = plan.deconvolve(yd, 3, stop=lf.STOP_TRACK, xs=xs, ys=ys, out=out, **kw)
        torch.cuda.synchronize()
        _, best, _, trace = oracle.deconvolve(psf, y, 3, xs, ys, stop=False, update=ref[0],
                                              background=ref[1])
        np.testing.assert_allclose(np.array(rep["metric_trace"]), trace, rtol=TOL)
        assert rep["best_iter"] == best     # the tracked run returns the best iterate
        want = oracle.rl(psf, y, best, update=ref[0], background=ref[1])
        assert rel_l2(out.cpu().numpy(), want) <= TOL


def test_variant_argument_errors(lf, problem):
    p, psf, y, xs, ys, plan = problem
    yd = to_dev(y)
    bad = [dict(update=2), dict(background=-1.0), dict(background=float("nan")),
           dict(stop=lf.STOP_TRACK, region=3), dict(stop=lf.STOP_TRACK, norm=3),
           dict(stop=lf.STOP_TRACK, window=-1)]
    for kw in bad:
        stop = kw.pop("stop", lf.STOP_NONE)
        with pytest.raises(lf.LfrlError):
            plan.deconvolve(yd, 2, stop=stop, xs=xs, ys=ys, **kw)


def test_batch_entry_point_with_per_frame_variants(lf):
    """lfrl_deconvolve_batch with a different update, background, start and
    metric per frame (frames of one plan share launches): each frame matches
    its oracle run."""
    import torch
    psf = S.gaussian_psf(3, 3, 13, seed=71, shift_scale=None)
    plan = lf.Plan(to_dev(psf), 36, 36, max_batch=3)
    try:
        specs = [
            (11, 12, dict(update="rl", background=10.0, init="ones"),
             lf.rl_opts(5, lf.STOP_NONE, background=10.0)),
            (12, 10, dict(update="isra", background=4.0, init="backprojection"),
             lf.rl_opts(5, lf.STOP_NONE, update=lf.UPDATE_ISRA, background=4.0,
                        backproject_start=True)),
            (9, 12, dict(update="isra", background=0.0, init="ones"),
             lf.rl_opts(5, lf.STOP_TRACK, 1, 2.0, 2.5, update=lf.UPDATE_ISRA,
                        region=lf.REGION_WHOLE, norm=lf.NORM_REGION, window=2)),
        ]
        imgs, vols, opts, refs = [], [], [], []
        for i, (ly, lx, okw, o) in enumerate(specs):
            h, w = 3 * ly, 3 * lx
            x = S.bead_volume(3, h, w, 10, 1200 + i)
            y = S.measure(oracle.forward(psf, x), 500.0, 10.0, 1300 + i)
            imgs.append(to_dev(y))
            vols.append(torch.empty((3, h, w), device="cuda:0"))
            opts.append(o)
            if o.stop == lf.STOP_NONE:
                refs.append((oracle.rl(psf, y, 5, **okw), None))
            else:
                xb, best, _, trace = oracle.deconvolve(psf, y, 5, 2.0, 2.5, stop=False,
                                                       region="whole", norm="region",
                                                       window=2, **okw)
                refs.append((xb, trace))
        reps = lf.lfrl_deconvolve_batch([plan.handle] * 3, [3 * s[0] for s in specs],
                                        [3 * s[1] for s in specs], imgs, vols, opts)
        torch.cuda.synchronize()
        for i, (want, trace) in enumerate(refs):
            err = rel_l2(vols[i].cpu().numpy(), want)
            print(f"frame {i}: rel L2 {err:.2e}", flush=True)
            assert err <= TOL
            if trace is not None:
                np.testing.assert_allclose(np.array(reps[i]["metric_trace"]), trace, rtol=TOL)
    finally:
        plan.close()
