"""Parity of the HIP path with the CPU oracle (needs an MI355X).

Every call goes through the C ABI (the ctypes binding only marshals
arguments).  Sizes span several DFT tiles with a ragged last tile, several
tile groups in the contraction, non-square images, images smaller than the
plan maximum, Nnum = 1 and Nnum = 15.  Floating-point bar: relative L2 error
<= 1e-5 against the float64 oracle on the same float32 inputs."""
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
    import os
    assert os.path.exists(lf.library_path()), "liblfrl.so missing: build first"
    return lf


def dev():
    import torch
    return torch.device("cuda:0")


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev())


def rel_l2(got, want):
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    return float(np.linalg.norm(got - want) / np.linalg.norm(want))


def random_psf(nz, n, k, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 1.0, size=(nz, n, n, k, k)).astype(np.float32)


# (name, nnum, lenslets_y, lenslets_x, nz, ksize, psf kind, tile_q list)
GEOMS = [
    ("small-N5", 5, 11, 11, 5, 25, "gauss", [0, 10, 7]),
    ("nonsquare-N3", 3, 5, 8, 2, 9, "rand", [0, 6]),
    ("nnum1", 1, 20, 17, 3, 7, "rand", [0, 9]),
    ("N15", 15, 4, 4, 2, 31, "gauss", [0]),
    # Nnum^2 = 1 mod 16: the last lenslet position is contracted apart
    ("N7", 7, 5, 6, 3, 21, "rand", [0, 9]),
    ("N9", 9, 4, 5, 2, 27, "gauss", [0]),
    ("delta-N2", 2, 6, 7, 1, 1, "rand", [0, 3]),
]


def make_psf(n, nz, k, kind, seed):
    if kind == "gauss":
        return S.gaussian_psf(n, nz, k, seed=seed, shift_scale=None)
    return random_psf(nz, n, k, seed)


def cases():
    for name, n, ly, lx, nz, k, kind, qs in GEOMS:
        for q in qs:
            yield pytest.param(n, ly, lx, nz, k, kind, q, id=f"{name}-Q{q}")


@pytest.mark.parametrize("n,ly,lx,nz,k,kind,q", list(cases()))
def test_forward_backward_parity(lf, n, ly, lx, nz, k, kind, q):
    import torch
    psf = make_psf(n, nz, k, kind, seed=100 + n)
    h, w = n * ly, n * lx
    rng = np.random.default_rng(7)
    x = rng.uniform(0.0, 1.0, size=(nz, h, w)).astype(np.float32)
    y = rng.uniform(0.0, 1.0, size=(h, w)).astype(np.float32)
    print(f"case N={n} {h}x{w} nz={nz} K={k} Q={q}", flush=True)
    # plan sized for a larger image than the one used
    plan = lf.Plan(to_dev(psf), h + 2 * n, w + n, tile_q=q)
    try:
        fx = plan.forward(to_dev(x))
        by = plan.backward(to_dev(y))
        torch.cuda.synchronize()
        assert rel_l2(fx.cpu().numpy(), oracle.forward(psf, x)) <= TOL
        assert rel_l2(by.cpu().numpy(), oracle.backward(psf, y)) <= TOL
    finally:
        plan.close()


def test_adjointness_on_gpu(lf):
    import torch
    n, ly, lx, nz, k = 3, 9, 7, 3, 11
    psf = random_psf(nz, n, k, seed=3)
    h, w = n * ly, n * lx
    rng = np.random.default_rng(4)
    x = rng.normal(size=(nz, h, w)).astype(np.float32)
    y = rng.normal(size=(h, w)).astype(np.float32)
    plan = lf.Plan(to_dev(psf), h, w, tile_q=7)
    try:
        ax = plan.forward(to_dev(x)).cpu().numpy().astype(np.float64)
        aty = plan.backward(to_dev(y)).cpu().numpy().astype(np.float64)
    finally:
        plan.close()
    lhs = np.sum(ax * y.astype(np.float64))
    rhs = np.sum(x.astype(np.float64) * aty)
    assert abs(lhs - rhs) <= 1e-5 * np.sqrt(np.sum(ax ** 2) * np.sum(y.astype(np.float64) ** 2))


def test_delta_voxel_reproduces_psf(lf):
    import torch
    n, ly, nz, k = 5, 9, 3, 13
    psf = random_psf(nz, n, k, seed=5)
    h = w = n * ly
    c0 = (k - 1) // 2
    plan = lf.Plan(to_dev(psf), h, w, tile_q=9)
    try:
        for (j, r, s) in [(1, 22, 21), (2, 20, 24), (0, 23, 19)]:
            x = np.zeros((nz, h, w), dtype=np.float32)
            x[j, r, s] = 1.0
            img = plan.forward(to_dev(x)).cpu().numpy()
            want = np.zeros((h, w))
            want[r - c0:r + c0 + 1, s - c0:s + c0 + 1] = psf[j, r % n, s % n]
            assert np.max(np.abs(img - want)) <= 1e-6 * psf.max()
    finally:
        plan.close()


def small_problem():
    p = S.preset("small")
    g = p["geometry"]
    psf = p["psf_array"]
    y = S.measure(oracle.forward(psf, p["x_true"]), p["peak"], p["background"], p["noise_seed"])
    xs, ys = oracle.synthetic_cutoff(g.nnum, p["spot_radius"], g.h, g.w)
    return p, psf, y, xs, ys


def test_rl_iterates_match_oracle(lf):
    """Each of the first 5 iterates of the Nnum 5, 55 x 55, 5-plane workload."""
    import torch
    p, psf, y, xs, ys = small_problem()
    g = p["geometry"]
    ref = oracle.rl(psf, y, p["iters"], keep_all=True)
    plan = lf.Plan(to_dev(psf), g.h, g.w)
    try:
        for k in range(1, p["iters"] + 1):
            vol, rep = plan.deconvolve(to_dev(y), k, stop=lf.STOP_NONE)
            torch.cuda.synchronize()
            assert rep["iters_run"] == k
            err = rel_l2(vol.cpu().numpy(), ref[k])
            print(f"iter {k}: rel L2 {err:.2e}", flush=True)
            assert err <= TOL
    finally:
        plan.close()


@pytest.mark.parametrize("n,ly,nz,k", [(5, 11, 5, 25), (15, 4, 2, 31)])
def test_staged_epilogue_inputs_bitwise(lf, monkeypatch, n, ly, nz, k):
    """The inverse tile DFT takes its epilogue inputs either staged in LDS by
    direct loads (where the LDS admits it) or by batched register loads: the
    same values bit for bit in every epilogue (store with a background, ratio,
    RL update, ISRA), and both match the oracle's first RL iterate."""
    import torch
    psf = S.gaussian_psf(n, nz, k, seed=31 + n)
    h = w = n * ly
    rng = np.random.default_rng(8)
    x = rng.uniform(0.0, 1.0, size=(nz, h, w)).astype(np.float32)
    y = rng.uniform(0.5, 1.5, size=(h, w)).astype(np.float32)
    outs = []
    for stage in ("0", "1"):
        monkeypatch.setenv("LFRL_C2R_STAGE", stage)
        plan = lf.Plan(to_dev(psf), h, w)
        try:
            fx = plan.forward(to_dev(x))
            v_rl, _ = plan.deconvolve(to_dev(y), 3, stop=lf.STOP_NONE, background=0.25)
            v_isra, _ = plan.deconvolve(to_dev(y), 3, stop=lf.STOP_NONE, update=lf.UPDATE_ISRA)
            v1, _ = plan.deconvolve(to_dev(y), 1, stop=lf.STOP_NONE)
            torch.cuda.synchronize()
            outs.append([t.cpu().numpy() for t in (fx, v_rl, v_isra, v1)])
        finally:
            plan.close()
    monkeypatch.delenv("LFRL_C2R_STAGE")
    for a, b in zip(outs[0], outs[1]):
        assert np.array_equal(a, b)
    assert rel_l2(outs[1][0], oracle.forward(psf, x)) <= TOL
    assert rel_l2(outs[1][3], oracle.rl(psf, y, 1)) <= TOL


def test_rl_with_metric_matches_oracle(lf):
    """Metric trace, best iterate and stop decision over 30 iterations."""
    import torch
    p, psf, y, xs, ys = small_problem()
    g = p["geometry"]
    iters = 30
    ref_x, ref_best, ref_run, ref_trace = oracle.deconvolve(psf, y, iters, xs, ys, stop=False)
    plan = lf.Plan(to_dev(psf), g.h, g.w)
    try:
        vol, rep = plan.deconvolve(to_dev(y), iters, stop=lf.STOP_TRACK, xs=xs, ys=ys,
                                   want_flux=True)
        torch.cuda.synchronize()
        tr = np.array(rep["metric_trace"])
        np.testing.assert_allclose(tr, ref_trace, rtol=TOL)
        assert rep["best_iter"] == ref_best
        assert rel_l2(vol.cpu().numpy(), ref_x) <= TOL
        # flux invariant <A^T 1, x^k> = sum(y) (every predicted pixel is positive here)
        assert np.max(np.abs(rep["flux_trace"])) <= 1e-5
        # early stop: same stop iteration as the oracle's rule on the same trace
        stopped, k_stop, best = oracle.stop_decision(list(ref_trace), 1)
        vol2, rep2 = plan.deconvolve(to_dev(y), iters, stop=lf.STOP_METRIC, xs=xs, ys=ys)
        torch.cuda.synchronize()
        assert rep2["stopped"] == stopped
        assert rep2["iters_run"] == k_stop
        assert rep2["best_iter"] == best
        ref_best_x = oracle.rl(psf, y, best)
        assert rel_l2(vol2.cpu().numpy(), ref_best_x) <= TOL
    finally:
        plan.close()


def test_rl_weakly_observed_voxels(lf):
    """PSFs shifted so far that some corner voxels send only ~1e-6 of their
    light into the image: those voxels' updates divide two tiny window sums and
    must still match the oracle (the library evaluates them exactly)."""
    import torch
    n, ly, nz, k = 3, 10, 3, 41
    psf = S.gaussian_psf(n, nz, k, seed=21, shift_scale=6.0)
    h = w = n * ly
    c = oracle.sensitivity(psf, h, w)
    assert (c < 1e-4 * c.max()).sum() >= 4          # the case really has weak voxels
    rng = np.random.default_rng(22)
    y = rng.uniform(10.0, 100.0, size=(h, w)).astype(np.float32)
    ref = oracle.rl(psf, y, 5, keep_all=True)
    plan = lf.Plan(to_dev(psf), h, w)
    try:
        for it in (1, 5):
            vol, rep = plan.deconvolve(to_dev(y), it, stop=lf.STOP_NONE)
            torch.cuda.synchronize()
            assert rep["weak_voxels"] > 0
            got = vol.cpu().numpy()
            err = rel_l2(got, ref[it])
            print(f"iter {it}: rel L2 {err:.2e}, weak voxels {rep['weak_voxels']}", flush=True)
            assert err <= TOL
            weak = c < 1e-2 * c.max()
            np.testing.assert_allclose(got[weak], ref[it][weak], rtol=1e-5, atol=1e-6)
    finally:
        plan.close()


def test_weak_voxel_list_overflow_is_refused(lf, monkeypatch):
    """A depth plane whose PSF is all zero has A^T 1 = 0 on every voxel, below
    any threshold.  With the weak-voxel list shortened to 64 entries
    (LFRL_WEAK_CAP) its 900 voxels cannot all be listed, and the call is
    refused instead of leaving an arbitrary subset on the inexact path.  With
    the normal list the same frame matches the oracle, the empty plane at 0."""
    import torch
    n, ly, nz, k = 3, 10, 3, 11
    psf = S.gaussian_psf(n, nz, k, seed=5)
    psf[1] = 0.0
    h = w = n * ly
    y = np.random.default_rng(6).uniform(10.0, 100.0, size=(h, w)).astype(np.float32)
    monkeypatch.setenv("LFRL_WEAK_CAP", "64")
    plan = lf.Plan(to_dev(psf), h, w)
    try:
        with pytest.raises(lf.LfrlError) as e:
            plan.deconvolve(to_dev(y), 1, stop=lf.STOP_NONE)
        assert e.value.code == -4
        print(f"refused: {e.value}", flush=True)
    finally:
        plan.close()
    monkeypatch.delenv("LFRL_WEAK_CAP")
    plan = lf.Plan(to_dev(psf), h, w)
    try:
        vol, rep = plan.deconvolve(to_dev(y), 2, stop=lf.STOP_NONE)
        torch.cuda.synchronize()
        got = vol.cpu().numpy()
    finally:
        plan.close()
    assert rep["weak_voxels"] >= h * w
    assert not got[1].any()
    ref = oracle.rl(psf, y, 2, keep_all=True)[2]
    assert rel_l2(got, ref) <= TOL


@pytest.mark.parametrize("nz,h,w,xs,ys", [(1, 55, 55, 5.5, 5.5), (3, 40, 64, 7.3, 3.9),
                                         (1, 600, 600, 10.0, 10.0), (5, 31, 17, 2.0, 30.0)])
def test_metric_matches_oracle(lf, nz, h, w, xs, ys):
    rng = np.random.default_rng(h * w + nz)
    vol = rng.uniform(0.0, 1.0, size=(nz, h, w)).astype(np.float32)
    vol[:, h // 3:h // 2, w // 4:w // 2] += 3.0
    img = vol[0] if nz == 1 else vol
    got = lf.metric(to_dev(img), xs, ys)
    want = oracle.metric(vol, xs, ys)
    assert got == pytest.approx(want, rel=1e-9)


def test_metric_zero_image(lf):
    assert lf.metric(to_dev(np.zeros((15, 20))), 3.0, 3.0) == 0.0


def test_deterministic(lf):
    import torch
    p, psf, y, xs, ys = small_problem()
    g = p["geometry"]
    plan = lf.Plan(to_dev(psf), g.h, g.w, tile_q=10)
    try:
        a, _ = plan.deconvolve(to_dev(y), 3, stop=lf.STOP_TRACK, xs=xs, ys=ys)
        b, _ = plan.deconvolve(to_dev(y), 3, stop=lf.STOP_TRACK, xs=xs, ys=ys)
        torch.cuda.synchronize()
        assert torch.equal(a, b)
    finally:
        plan.close()


def test_argument_errors(lf):
    import torch
    psf = random_psf(2, 3, 5, seed=1)
    plan = lf.Plan(to_dev(psf), 12, 12)
    try:
        with pytest.raises(lf.LfrlError):
            plan.forward(to_dev(np.zeros((2, 15, 12))))      # exceeds max_h
        with pytest.raises(lf.LfrlError):
            plan.forward(to_dev(np.zeros((2, 10, 12))))      # not a multiple of nnum
        with pytest.raises(lf.LfrlError):
            plan.deconvolve(to_dev(np.ones((12, 12))), 0)    # max_iters < 1
        with pytest.raises(lf.LfrlError):
            plan.deconvolve(to_dev(np.ones((12, 12))), 2, stop=lf.STOP_METRIC, xs=-1.0)
    finally:
        plan.close()
    with pytest.raises(lf.LfrlError):
        lf.Plan(to_dev(random_psf(2, 3, 4, seed=1)), 12, 12)  # even support


def test_autotuned_plan(lf):
    """The tuner times a few tile sides and keeps one; the plan then behaves
    exactly like a plan built with that side."""
    import torch
    n, ly, nz, k = 5, 14, 4, 25
    psf = S.gaussian_psf(n, nz, k, seed=91, shift_scale=None)
    h = w = n * ly
    rng = np.random.default_rng(92)
    x = rng.uniform(0.0, 1.0, size=(nz, h, w)).astype(np.float32)
    y = rng.uniform(0.0, 1.0, size=(h, w)).astype(np.float32)
    tuned = lf.Plan(to_dev(psf), h, w, autotune=True, max_batch=2)
    try:
        info = tuned.info
        print(f"autotune: Q={info['tile_q']} over {info['tune_candidates']} sides, "
              f"{info['tune_ms']:.3f} ms", flush=True)
        assert info["tune_candidates"] >= 2 and info["tune_ms"] > 0
        fixed = lf.Plan(to_dev(psf), h, w, tile_q=info["tile_q"], max_batch=2)
        try:
            assert fixed.info["tune_candidates"] == 0
            assert torch.equal(tuned.forward(to_dev(x)), fixed.forward(to_dev(x)))
            assert torch.equal(tuned.backward(to_dev(y)), fixed.backward(to_dev(y)))
        finally:
            fixed.close()
        assert rel_l2(tuned.forward(to_dev(x)).cpu().numpy(), oracle.forward(psf, x)) <= TOL
    finally:
        tuned.close()


def test_plans_of_one_tile_side_keep_their_lds(lf):
    """Two plans with the same tile side and different Nnum need different
    amounts of LDS in the same tile-DFT kernels; building the smaller one
    after the larger must not lower what the larger launches with (here above
    64 KiB)."""
    import torch
    q = 36
    psf_a = random_psf(2, 15, 31, seed=41)          # 36 x 19 x 15 complex: 82 KB
    ha = 15 * 4
    rng = np.random.default_rng(43)
    x = rng.uniform(0.0, 1.0, size=(2, ha, ha)).astype(np.float32)
    y = rng.uniform(0.0, 1.0, size=(ha, ha)).astype(np.float32)
    a = lf.Plan(to_dev(psf_a), ha, ha, tile_q=q)
    try:
        fa, ba = a.forward(to_dev(x)), a.backward(to_dev(y))
        psf_b = random_psf(1, 3, 9, seed=42)
        b = lf.Plan(to_dev(psf_b), 27, 27, tile_q=q)
        try:
            xb = rng.uniform(0.0, 1.0, size=(1, 27, 27)).astype(np.float32)
            fb = b.forward(to_dev(xb))
            torch.cuda.synchronize()
            assert rel_l2(fb.cpu().numpy(), oracle.forward(psf_b, xb)) <= TOL
        finally:
            b.close()
        fa2, ba2 = a.forward(to_dev(x)), a.backward(to_dev(y))
        torch.cuda.synchronize()
        assert torch.equal(fa, fa2) and torch.equal(ba, ba2)
        assert rel_l2(fa.cpu().numpy(), oracle.forward(psf_a, x)) <= TOL
        assert rel_l2(ba.cpu().numpy(), oracle.backward(psf_a, y)) <= TOL
    finally:
        a.close()


def test_graph_replays_match_direct_launches(lf, monkeypatch):
    """Fixed-length runs replay a captured graph; every replay, with other
    work and synchronisations in between, equals the run with graphs off."""
    import torch
    p, psf, y, xs, ys = small_problem()
    g = p["geometry"]
    plan = lf.Plan(to_dev(psf), g.h, g.w)
    try:
        yd = to_dev(y)
        monkeypatch.setenv("LFRL_GRAPH", "0")
        want, rep_w = plan.deconvolve(yd, 7, stop=lf.STOP_TRACK, xs=xs, ys=ys, want_flux=True)
        want = want.clone()
        monkeypatch.setenv("LFRL_GRAPH", "1")
        out = torch.empty_like(want)
        for rep in range(4):
            plan.forward(want)                      # eager work between replays
            torch.cuda.synchronize()
            got, rep_g = plan.deconvolve(yd, 7, stop=lf.STOP_TRACK, xs=xs, ys=ys, out=out,
                                         want_flux=True)
            torch.cuda.synchronize()
            assert torch.equal(got, want), rep
            assert rep_g["metric_trace"] == rep_w["metric_trace"]
            assert rep_g["flux_trace"] == rep_w["flux_trace"]
            assert rep_g["best_iter"] == rep_w["best_iter"]
        # other legs between replays must not leak into the graph's tables
        monkeypatch.setenv("LFRL_GRAPH", "0")
        plan.deconvolve(yd, 3, stop=lf.STOP_METRIC, xs=xs * 0.5, ys=ys * 0.7)
        monkeypatch.setenv("LFRL_GRAPH", "1")
        got, rep_g = plan.deconvolve(yd, 7, stop=lf.STOP_TRACK, xs=xs, ys=ys, out=out,
                                     want_flux=True)
        torch.cuda.synchronize()
        assert torch.equal(got, want)
        assert rep_g["metric_trace"] == rep_w["metric_trace"]
        assert rel_l2(got.cpu().numpy(), oracle.deconvolve(psf, y, 7, xs, ys, stop=False)[0]) <= TOL
    finally:
        plan.close()


def test_normalized_psf_plan(lf):
    """A plan built with LFRL_NORMALIZE_PSF from kernels of arbitrary scale (one
    of them all zero) projects and deconvolves like the oracle on
    oracle.normalize_psf of the same taps; the caller's PSF array is unchanged."""
    import torch
    n, ly, lx, nz, k = 3, 8, 7, 2, 9
    rng = np.random.default_rng(78)
    psf = random_psf(nz, n, k, seed=77)
    psf *= rng.uniform(0.05, 40.0, size=(nz, n, n, 1, 1)).astype(np.float32)
    psf[1, 0, 2] = 0.0
    want_psf = oracle.normalize_psf(psf)
    h, w = n * ly, n * lx
    x = rng.uniform(0.0, 1.0, size=(nz, h, w)).astype(np.float32)
    y = rng.uniform(1.0, 5.0, size=(h, w)).astype(np.float32)
    d_psf = to_dev(psf)
    plan = lf.Plan(d_psf, h, w, normalize_psf=True)
    try:
        fx = plan.forward(to_dev(x))
        by = plan.backward(to_dev(y))
        vol, _ = plan.deconvolve(to_dev(y), 3)
        torch.cuda.synchronize()
        assert rel_l2(fx.cpu().numpy(), oracle.forward(want_psf, x)) <= TOL
        assert rel_l2(by.cpu().numpy(), oracle.backward(want_psf, y)) <= TOL
        assert rel_l2(vol.cpu().numpy(), oracle.rl(want_psf, y, 3)) <= TOL
        assert torch.equal(d_psf.cpu(), torch.from_numpy(psf))
    finally:
        plan.close()
