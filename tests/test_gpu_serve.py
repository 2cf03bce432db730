"""The serving loop on the GPU: open-loop arrivals over two resident PSF sets,
jobs admitted under a memory budget and stepped together (needs an MI355X).
Every served result must be bitwise the volume the same request gets when
deconvolved alone; a request with a NaN pixel fails alone."""
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


def test_served_results_equal_alone(lf):
    import torch
    from paper_2208_11422_amd.serve import JobExecutor, Request, Scheduler, latency_stats
    sets = [(5, 4, 25, 81), (3, 3, 15, 82)]
    psfs = [S.gaussian_psf(n, nz, k, seed=s, shift_scale=None) for n, nz, k, s in sets]
    plans = [lf.Plan(torch.from_numpy(p).cuda(), 75, 75, precision=prec, max_batch=2)
             for p, prec in zip(psfs, (0, 1))]
    try:
        specs = S.serving_requests(14, seed0=8100, sets=[(5, 4), (3, 3)], min_side=30,
                                   max_side=75)
        imgs, legs = [], {}
        for sp in specs:
            x = S.bead_volume(sp["nz"], sp["h"], sp["w"], 15, sp["seed"])
            y = S.measure(oracle.forward(psfs[sp["set"]], x), 800.0, 10.0, sp["seed"] + 1)
            imgs.append(torch.from_numpy(y).pin_memory())
            legs[sp["rid"]] = (sp["w"] / (sp["nnum"] * 4.0), sp["h"] / (sp["nnum"] * 4.0))
        imgs[5] = imgs[5].clone()
        imgs[5][3, 3] = float("nan")
        arrivals = S.poisson_arrivals(len(specs), 400.0, seed=8)

        def opts_for(req):
            xs, ys = legs[req.rid]
            return dict(iters=12, stop=lf.STOP_METRIC, patience=1, xs=xs, ys=ys)

        reqs = [Request(rid=sp["rid"], plan=sp["set"], h=sp["h"], w=sp["w"], image=img,
                        arrival=float(a)) for sp, img, a in zip(specs, imgs, arrivals)]
        ex = JobExecutor(plans, opts_for, keep=range(len(specs)))
        budget = 6 * lf.lfrl_job_footprint(plans[0].handle, 75, 75)
        sched = Scheduler(ex, budget, max_active=8)
        sched.run(reqs)
        print(f"served: {latency_stats(reqs)}; peak active {sched.peak_active}, "
              f"rounds {sched.rounds}", flush=True)
        assert reqs[5].status == "failed"
        assert sched.peak_bytes <= budget
        assert max(sched.batch_sizes) >= 2
        for q in reqs:
            if q.rid == 5:
                continue
            assert q.status == "done", q.error
            xs, ys = legs[q.rid]
            alone, rep = plans[q.plan].deconvolve(imgs[q.rid].cuda(), 12, stop=lf.STOP_METRIC,
                                                  xs=xs, ys=ys)
            assert q.iters == rep["iters_run"] and q.best_iter == rep["best_iter"]
            assert torch.equal(alone.cpu(), q.result), q.rid
    finally:
        for p in plans:
            p.close()
