"""Batched and served deconvolution through the job API (needs an MI355X).

Frames that share a plan are stepped together: their tiles share every
projection launch.  Each frame's iterates must be bitwise the ones it gets
when deconvolved alone (every tile's arithmetic is independent of the other
tiles in a launch), its reports identical, and a batched frame must match the
float64 oracle like a single one.  Also: a frame whose image holds NaN is
refused at creation without disturbing the others, and batches larger than a
plan's tile capacity are split over several launches."""
import numpy as np
import pytest

import lfrl_synth as S
import oracle

pytestmark = pytest.mark.gpu

TOL = 1e-5


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


def frame(psf, n, ly, lx, seed, beads=12):
    nz = psf.shape[0]
    h, w = n * ly, n * lx
    x = S.bead_volume(nz, h, w, beads, seed)
    return S.measure(oracle.forward(psf, x), 500.0, 10.0, seed + 1)


def alone(plan, y, iters, stop, xs, ys, patience=1):
    vol, rep = plan.deconvolve(to_dev(y), iters, stop=stop, xs=xs, ys=ys, patience=patience)
    return vol.cpu().numpy(), rep


def run_jobs(lf, jobs):
    import torch
    steps = 0
    while lf.Job.step(jobs) > 0:
        steps += 1
        assert steps <= 1000
    torch.cuda.synchronize()
    return [j.result() for j in jobs]


def assert_same(got, rep_got, want, rep_want):
    assert rep_got["iters_run"] == rep_want["iters_run"]
    assert rep_got["best_iter"] == rep_want["best_iter"]
    assert rep_got["stopped"] == rep_want["stopped"]
    assert rep_got["weak_voxels"] == rep_want["weak_voxels"]
    if "metric_trace" in rep_want:
        assert rep_got["metric_trace"] == rep_want["metric_trace"]
    assert np.array_equal(got, want)


@pytest.mark.parametrize("precision", [0, 1], ids=["fp32", "split-fp16"])
def test_alone_vs_mix(lf, precision):
    """Frames of two plans, uneven sizes and stop modes, stepped together."""
    psf_a = S.gaussian_psf(5, 5, 25, seed=61, shift_scale=None)
    psf_b = S.gaussian_psf(3, 3, 15, seed=62, shift_scale=None)
    plan_a = lf.Plan(to_dev(psf_a), 65, 65, precision=precision, max_batch=3)
    plan_b = lf.Plan(to_dev(psf_b), 36, 45, precision=precision, max_batch=2)
    specs = [  # (plan, psf, n, ly, lx, iters, stop, patience)
        (plan_a, psf_a, 5, 11, 11, 12, lf.STOP_METRIC, 1),
        (plan_a, psf_a, 5, 13, 8, 7, lf.STOP_TRACK, 1),
        (plan_b, psf_b, 3, 12, 15, 9, lf.STOP_NONE, 1),
        (plan_a, psf_a, 5, 5, 13, 10, lf.STOP_METRIC, 2),
        (plan_b, psf_b, 3, 7, 7, 6, lf.STOP_METRIC, 1),
        (plan_a, psf_a, 5, 12, 12, 5, lf.STOP_NONE, 1),
    ]
    try:
        ys_, wants, jobs = [], [], []
        for i, (plan, psf, n, ly, lx, iters, stop, pat) in enumerate(specs):
            y = frame(psf, n, ly, lx, seed=600 + 10 * i)
            xs, ysl = oracle.synthetic_cutoff(n, 2.0, n * ly, n * lx)
            ys_.append((y, xs, ysl))
            print(f"frame {i}: N={n} {n*ly}x{n*lx} iters={iters} stop={stop}", flush=True)
            wants.append(alone(plan, y, iters, stop, xs, ysl, pat))
        for i, (plan, psf, n, ly, lx, iters, stop, pat) in enumerate(specs):
            y, xs, ysl = ys_[i]
            jobs.append(lf.Job(plan, to_dev(y), iters, stop=stop, patience=pat, xs=xs, ys=ysl))
        got = run_jobs(lf, jobs)
        for i in range(len(specs)):
            vol, rep = got[i]
            assert_same(vol.cpu().numpy(), rep, *wants[i])
        for j in jobs:
            j.close()
    finally:
        plan_a.close()
        plan_b.close()


def test_over_capacity_is_split(lf):
    """Four largest-size frames on a plan whose launches hold one frame."""
    psf = S.gaussian_psf(5, 3, 21, seed=63, shift_scale=None)
    plan = lf.Plan(to_dev(psf), 50, 60, max_batch=1)
    try:
        frames = [frame(psf, 5, 10, 12, seed=700 + i) for i in range(4)]
        wants = [alone(plan, y, 4, lf.STOP_NONE, 1.0, 1.0) for y in frames]
        jobs = [lf.Job(plan, to_dev(y), 4) for y in frames]
        got = run_jobs(lf, jobs)
        for (vol, rep), want in zip(got, wants):
            assert_same(vol.cpu().numpy(), rep, *want)
        for j in jobs:
            j.close()
    finally:
        plan.close()


def test_batched_frames_match_oracle(lf):
    """lfrl_deconvolve_batch over frames of two plans against oracle.rl."""
    import torch
    psf_a = S.gaussian_psf(5, 4, 25, seed=64, shift_scale=None)
    psf_b = S.gaussian_psf(3, 2, 11, seed=65, shift_scale=None)
    plan_a = lf.Plan(to_dev(psf_a), 60, 60, max_batch=2)
    plan_b = lf.Plan(to_dev(psf_b), 30, 30)
    try:
        cases = [(plan_a, psf_a, 5, 12, 9), (plan_b, psf_b, 3, 10, 10), (plan_a, psf_a, 5, 7, 12)]
        imgs, vols, opts, refs = [], [], [], []
        for i, (plan, psf, n, ly, lx) in enumerate(cases):
            y = frame(psf, n, ly, lx, seed=800 + 10 * i)
            imgs.append(to_dev(y))
            vols.append(torch.empty((psf.shape[0], n * ly, n * lx), device="cuda:0"))
            opts.append(lf.RlOpts(max_iters=6, stop=lf.STOP_NONE, patience=1, init=0,
                                  xs=1.0, ys=1.0))
            refs.append(oracle.rl(psf, y, 6))
        reps = lf.lfrl_deconvolve_batch([c[0].handle for c in cases],
                                        [c[2] * c[3] for c in cases],
                                        [c[2] * c[4] for c in cases], imgs, vols, opts,
                                        want_flux=True)
        torch.cuda.synchronize()
        for i in range(len(cases)):
            err = rel_l2(vols[i].cpu().numpy(), refs[i])
            print(f"batched frame {i}: rel L2 {err:.2e}", flush=True)
            assert err <= TOL
            assert reps[i]["iters_run"] == 6
            assert np.max(np.abs(reps[i]["flux_trace"])) <= 1e-4
    finally:
        plan_a.close()
        plan_b.close()


def test_nan_frame_is_refused(lf):
    psf = S.gaussian_psf(3, 2, 11, seed=66, shift_scale=None)
    plan = lf.Plan(to_dev(psf), 30, 30, max_batch=2)
    try:
        good = frame(psf, 3, 10, 10, seed=900)
        bad = good.copy()
        bad[4, 7] = np.nan
        want = alone(plan, good, 5, lf.STOP_NONE, 1.0, 1.0)
        j_good = lf.Job(plan, to_dev(good), 5)
        with pytest.raises(lf.LfrlError) as ei:
            lf.Job(plan, to_dev(bad), 5)
        assert ei.value.code == -5
        neg = good.copy()
        neg[0, 0] = -1.0
        with pytest.raises(lf.LfrlError):
            lf.Job(plan, to_dev(neg), 5)
        (vol, rep), = run_jobs(lf, [j_good])
        assert_same(vol.cpu().numpy(), rep, *want)
        j_good.close()
    finally:
        plan.close()


def test_job_argument_errors(lf):
    psf = S.gaussian_psf(3, 2, 11, seed=67, shift_scale=None)
    plan = lf.Plan(to_dev(psf), 30, 30)
    try:
        y = to_dev(np.ones((33, 30), np.float32))
        with pytest.raises(lf.LfrlError):
            lf.Job(plan, y, 5)                       # above the plan maximum
        y = to_dev(np.ones((30, 30), np.float32))
        with pytest.raises(lf.LfrlError):
            lf.Job(plan, y, 0)                       # no iterations
        with pytest.raises(lf.LfrlError):
            lf.lfrl_job_create(plan.handle, 30, 30, y,
                               lf.RlOpts(max_iters=3, stop=0, patience=1, init=1, xs=1, ys=1))
        assert lf.lfrl_job_footprint(plan.handle, 30, 30) > 4 * 2 * 30 * 30 * 4
    finally:
        plan.close()
