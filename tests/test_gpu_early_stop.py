"""Early stop (sec. 2.2: stop once the DCT entropy decreases) with iterations
queued in chunks ahead of the host's look at the stop rule (needs an MI355X).

Iterations queued past the stop must change nothing: every check compares the
early-stop run with a fixed-length tracked run of as many iterations as the
rule allows (same kernels, so bit for bit) and the rule itself with the
oracle's stop_decision on the tracked trace.  Stops are placed before, at and
after the chunk edges (chunks of 4 iterations), with graphs replayed (twice,
the second time from the cached chunk graphs) and with direct launches."""
import numpy as np
import pytest

import lfrl_synth as S
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


@pytest.fixture(scope="module")
def problem(lf):
    import torch
    p = S.preset("small")
    g = p["geometry"]
    psf = p["psf_array"]
    y = S.measure(oracle.forward(psf, p["x_true"]), p["peak"], p["background"], p["noise_seed"])
    xs, ys = oracle.synthetic_cutoff(g.nnum, p["spot_radius"], g.h, g.w)
    dev = torch.device("cuda:0")
    plan = lf.Plan(torch.from_numpy(psf).to(dev), g.h, g.w)
    yield plan, torch.from_numpy(y).to(dev), xs, ys
    plan.close()


def run(lf, problem, iters, stop, **kw):
    import torch
    plan, y, xs, ys = problem
    vol, rep = plan.deconvolve(y, iters, stop=stop, xs=xs, ys=ys, **kw)
    torch.cuda.synchronize()
    return vol.cpu().numpy(), rep


@pytest.mark.parametrize("patience,window", [(1, 1), (2, 1), (3, 1), (4, 1), (6, 1), (2, 3)])
def test_early_stop_equals_tracked_prefix(lf, problem, patience, window):
    cap = 24
    _, track = run(lf, problem, cap, lf.STOP_TRACK, patience=patience, window=window)
    stopped, k_stop, best = oracle.stop_decision(list(track["metric_trace"]), patience, window)
    print(f"patience {patience} window {window}: stop at {k_stop} (best {best})", flush=True)
    assert stopped
    vol_e, rep_e = run(lf, problem, cap, lf.STOP_METRIC, patience=patience, window=window)
    assert rep_e["stopped"] == 1 and rep_e["iters_run"] == k_stop and rep_e["best_iter"] == best
    assert list(rep_e["metric_trace"]) == list(track["metric_trace"][:k_stop])
    vol_t, rep_t = run(lf, problem, k_stop, lf.STOP_TRACK, patience=patience, window=window)
    assert rep_t["best_iter"] == best
    assert np.array_equal(vol_e, vol_t)
    # replayed from the cached chunk graphs
    vol_r, rep_r = run(lf, problem, cap, lf.STOP_METRIC, patience=patience, window=window)
    assert rep_r["iters_run"] == k_stop and np.array_equal(vol_r, vol_e)


def test_early_stop_direct_launches(lf, problem, monkeypatch):
    vol_g, rep_g = run(lf, problem, 24, lf.STOP_METRIC, patience=3)
    monkeypatch.setenv("LFRL_GRAPH", "0")
    vol_d, rep_d = run(lf, problem, 24, lf.STOP_METRIC, patience=3)
    assert rep_d["iters_run"] == rep_g["iters_run"] and rep_d["best_iter"] == rep_g["best_iter"]
    assert list(rep_d["metric_trace"]) == list(rep_g["metric_trace"])
    assert np.array_equal(vol_d, vol_g)


@pytest.mark.parametrize("cap", [1, 4, 7])
def test_early_stop_reaching_the_cap(lf, problem, cap):
    """A rule that cannot fire within the cap runs every iteration and keeps
    the best, like the tracked run."""
    vol_e, rep_e = run(lf, problem, cap, lf.STOP_METRIC, patience=30)
    vol_t, rep_t = run(lf, problem, cap, lf.STOP_TRACK, patience=30)
    assert rep_e["stopped"] == 0 and rep_e["iters_run"] == cap
    assert rep_e["best_iter"] == rep_t["best_iter"]
    assert list(rep_e["metric_trace"]) == list(rep_t["metric_trace"])
    assert np.array_equal(vol_e, vol_t)
