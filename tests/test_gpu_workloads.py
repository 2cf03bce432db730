"""Full-size parity at the batched and serving workloads (needs an MI355X).

Plans are built as bench.py builds them: the batched frames on autotuned FP32
plans, the largest serving PSF set (Nnum 15, 51 planes, K = 255, 900 x 900)
on a split-FP16 plan with room for four frames per launch.  The oracle
computes sampled outputs one by one; whole runs are checked through
invariants that hold at any size."""
import numpy as np
import pytest

import lfrl_synth as S
import oracle

pytestmark = pytest.mark.gpu

CACHE = "/tmp/lfrl_synth_cache"


@pytest.fixture(scope="module")
def lf():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2208_11422_amd as lf
    return lf


def sample_pixels(h, w, n, seed):
    rng = np.random.default_rng(seed)
    rr = np.concatenate([rng.integers(0, h, n), [0, 0, h - 1, h - 1, 5, h - 6]])
    cc = np.concatenate([rng.integers(0, w, n), [0, w - 1, 0, w - 1, w - 7, 2]])
    return rr, cc


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def check_projections(lf, plan, psf, h, w, tol, seed, npix=60, nvox=800):
    import torch
    nz = psf.shape[0]
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, 1.0, size=(nz, h, w)).astype(np.float32)
    img = plan.forward(torch.from_numpy(x).cuda()).cpu().numpy()
    rr, cc = sample_pixels(h, w, npix, seed + 1)
    ef = rel_l2(img[rr, cc], oracle.forward_at(psf, x, rr, cc))
    del x
    y = rng.uniform(10.0, 1000.0, size=(h, w)).astype(np.float32)
    vol = plan.backward(torch.from_numpy(y).cuda()).cpu().numpy()
    rr, cc = sample_pixels(h, w, nvox, seed + 2)
    jj = rng.integers(0, nz, rr.size)
    jj[-6:] = [0, nz - 1, 0, nz - 1, nz // 2, 1]
    eb = rel_l2(vol[jj, rr, cc], oracle.backward_at(psf, y, jj, rr, cc))
    return ef, eb


@pytest.mark.parametrize("frame", [14, 6])
def test_batched_frame_projections_full_size(lf, frame):
    """A frame of the batched workload on its autotuned FP32 plan."""
    import torch
    sp = S.batched_frames()[frame]
    psf = S.batched_psf(sp)
    print(f"batched frame {frame}: {sp}", flush=True)
    plan = lf.Plan(torch.from_numpy(psf).cuda(), sp["h"], sp["w"], autotune=True)
    try:
        print(f"plan Q={plan.info['tile_q']} tuned over {plan.info['tune_candidates']}",
              flush=True)
        ef, eb = check_projections(lf, plan, psf, sp["h"], sp["w"], 1e-5, 300 + frame)
        print(f"forward {ef:.2e} backward {eb:.2e}", flush=True)
        assert ef <= 1e-5 and eb <= 1e-5
    finally:
        plan.close()


def test_batched_jobs_full_size_invariants(lf):
    """Two batched frames stepped together for 3 iterations: flux
    <A^T 1, x^k> = sum(y) where every predicted pixel is positive, and
    non-negative iterates."""
    import torch
    specs = [S.batched_frames()[i] for i in (6, 9)]
    plans, jobs = [], []
    try:
        for sp in specs:
            psf = S.batched_psf(sp)
            plans.append(lf.Plan(torch.from_numpy(psf).cuda(), sp["h"], sp["w"], autotune=True))
            rng = np.random.default_rng(sp["seed"])
            y = rng.uniform(50.0, 1000.0, size=(sp["h"], sp["w"])).astype(np.float32)
            jobs.append(lf.Job(plans[-1], torch.from_numpy(y).cuda(), 3, want_flux=True))
        while lf.Job.step(jobs) > 0:
            pass
        for j in jobs:
            vol, rep = j.result()
            v = vol.cpu().numpy()
            print(f"job {vol.shape}: flux {rep['flux_trace']}, weak {rep['weak_voxels']}",
                  flush=True)
            assert rep["iters_run"] == 3
            assert np.max(np.abs(rep["flux_trace"])) <= 1e-4
            assert v.min() >= -1e-6 * v.max()
            j.close()
    finally:
        for p in plans:
            p.close()


def test_serving_set_projections_full_size(lf):
    """The largest serving PSF set on its split-FP16 plan (bar 1e-3)."""
    import torch
    cfg = S.SERVING
    k = 3
    n, nz, seed = cfg["sets"][k]
    psf = S._cached(f"psf_serving_{n}_{nz}_{cfg['ksize']}_{seed}", lambda: S.serving_psf(k),
                    CACHE)
    side = cfg["max_side"] // n * n
    plan = lf.Plan(torch.from_numpy(psf).cuda(), side, side, precision=lf.SPLIT_FP16,
                   max_batch=4)
    try:
        print(f"serving set {k}: N={n} nz={nz} {side}x{side} Q={plan.info['tile_q']}",
              flush=True)
        ef, eb = check_projections(lf, plan, psf, side, side, 1e-3, 77, npix=40, nvox=600)
        print(f"split forward {ef:.2e} backward {eb:.2e}", flush=True)
        assert ef <= 1e-3 and eb <= 1e-3
    finally:
        plan.close()


def test_batched_frame_iterates_full_size(lf):
    """x^1 and x^2 of a batched-workload frame (Nnum 15, 720 x 720, 41
    planes, K = 121) on its autotuned FP32 plan, against the oracle's
    windowed iterates (oracle.rl_window) in the top-left corner window, where
    the weakly observed voxels sit, and in an interior window.  Bar: relative
    L2 1e-5 per window and iterate; every weakly observed voxel to rtol 1e-5."""
    import torch
    sp = S.batched_frames()[4]
    psf = S.batched_psf(sp)
    h, w, nz = sp["h"], sp["w"], sp["nz"]
    print(f"batched frame 4: {sp}", flush=True)
    y = np.random.default_rng(sp["seed"] + 7).uniform(10.0, 1000.0, size=(h, w)).astype(np.float32)
    plan = lf.Plan(torch.from_numpy(psf).cuda(), h, w, autotune=True)
    try:
        print(f"plan Q={plan.info['tile_q']} tuned over {plan.info['tune_candidates']}",
              flush=True)
        y_d = torch.from_numpy(y).cuda()
        got = {k: plan.deconvolve(y_d, k, stop=lf.STOP_NONE)[0].cpu().numpy() for k in (1, 2)}
    finally:
        plan.close()
    for name, (r0, r1, s0, s1), iters in (("corner", (0, 16, 0, 16), 2),
                                          ("interior", (352, 368, 352, 368), 1)):
        xs, c = oracle.rl_window(psf, y, iters, r0, r1, s0, s1)
        weak = c < 1e-2 * c.max()
        for m in range(iters):
            g = got[m + 1][:, r0:r1, s0:s1].astype(np.float64)
            err = rel_l2(g, xs[m])
            print(f"{name} x^{m + 1}: rel L2 {err:.2e}, {int(weak.sum())} weak voxels", flush=True)
            assert err <= 1e-5
            if weak.any():
                np.testing.assert_allclose(g[weak], xs[m][weak], rtol=1e-5, atol=0)
        if name == "corner":
            assert weak.sum() > 0
