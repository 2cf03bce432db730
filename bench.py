"""Benchmark: light-field Richardson-Lucy iterations per second on one MI355X.

Workload: Nnum 15, 40 x 40 lenslets (600 x 600 image), 31 depth planes,
255 x 255 synthetic defocus-disk PSF per (plane, phase), 500 beads + 3
filaments, Poisson noise at peak 2000 counts.  One step = one full RL
iteration: forward projection, ratio, back projection, multiplicative update
and the DCT-entropy metric with best-iterate tracking.

Prints one JSON line.  Inputs are resident in HBM before the timed region;
plan construction (PSF -> spectra) is outside it.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "LF-RL iters/s at 600²×31 (FP32 vs split-FP16); p50/p99 job latency"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
F16_PEAK_TFLOPS = 2500.0   # dense FP16 / BF16 matrix peak
CACHE = os.environ.get("LFRL_SYNTH_CACHE", "/tmp/lfrl_synth_cache")


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def contraction_bytes(info: dict, g, nt: int, kernel: str) -> float:
    """Algorithmic HBM bytes of one launch of a spectral contraction kernel:
    the PSF spectra it must stream once plus its tile-spectrum input and
    output (complex float32, 8 bytes per coefficient), at the unique
    frequencies of the Hermitian half spectrum (the ones the kernels visit)."""
    nf, nn, kk = info["nfreq_unique"], g.nnum ** 2, g.nnum ** 2 * g.nz
    spectra = nf * nn * kk * 8.0
    if kernel == "contract_fwd":
        return spectra + nf * nt * kk * 8.0 + info["split_k"] * nf * nt * nn * 8.0
    return spectra + nf * nt * nn * 8.0 + nf * nt * kk * 8.0


def contraction_flops(info: dict, g, nt: int) -> float:
    return 8.0 * info["nfreq_unique"] * g.nnum ** 2 * (g.nnum ** 2 * g.nz) * nt


def iteration_model(info: dict, g, h: int, w: int, nt: int, ms_measured: float,
                    precision: str = "fp32") -> dict:
    """Roofline model of one whole iteration at the plan's tile shape.

    Bytes: both PSF spectra passes (8 bytes per complex coefficient in float32,
    4 in the split modes' 16-bit words), the tile spectra written and read
    around each contraction, the volume reads of the tile gather (overlap
    included), the update's volume traffic and the image-sized buffers.
    Compute: the two contractions on their own units (float32 matrix cores at
    157.3 TFLOP/s; the split modes do two 16-bit products, hi and lo, per real
    product on the FP16/BF16 matrix cores at 2.5 PFLOP/s) plus the tile DFTs
    in float32 vector arithmetic.  The floor is the PSF read once per
    projection, whatever the shape."""
    n, nz, k = g.nnum, g.nz, g.ksize
    q, t, r, nf = info["tile_q"], info["tile_out"], info["taps"], info["nfreq_unique"]
    split = precision != "fp32"
    s_g = n ** 4 * nz * nf * (4.0 if split else 8.0)
    s_x = n ** 2 * nz * nt * nf * 8.0
    b = (2 * s_g + 4 * s_x + 4.0 * w * h * nz * (((t + r - 1) / t) ** 2 + 3) + 24.0 * w * h)
    f_contract = 16.0 * n ** 4 * nz * nf * nt
    f_dft = 2.0 * (n * n * nz + n * n) * nt * 5 * q * q * math.log2(q * q)
    t_hbm = b / (HBM_PEAK_GBS * 1e9) * 1e3
    if split:
        t_contract = 2.0 * f_contract / (F16_PEAK_TFLOPS * 1e12) * 1e3
    else:
        t_contract = f_contract / (FP32_PEAK_TFLOPS * 1e12) * 1e3
    t_dft = f_dft / (FP32_PEAK_TFLOPS * 1e12) * 1e3
    t_compute = t_contract + t_dft
    floor = 2.0 * n * n * nz * k * k * 4 / (HBM_PEAK_GBS * 1e9) * 1e3
    bound = max(t_hbm, t_compute)
    return {"precision": precision, "bytes_per_iter": b,
            "flops_per_iter": f_contract * (2.0 if split else 1.0) + f_dft,
            "t_hbm_ms": t_hbm, "t_contract_ms": t_contract, "t_dft_ms": t_dft,
            "t_compute_ms": t_compute, "bound": "hbm" if t_hbm >= t_compute else "compute",
            "t_bound_ms": bound, "frac_of_bound": bound / ms_measured,
            "floor_ms": floor, "floor_frac": floor / ms_measured}


def source_digest() -> str:
    """sha256 over the kernel sources (every file under the package's csrc)."""
    d = os.path.join(ROOT, "paper_2208_11422_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(d)):
        with open(os.path.join(d, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def measured_traffic(kernel: str, bytes_alg: float):
    """HBM traffic per launch from the committed counter summary, if it was
    taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "contract_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    k = d.get("kernels", {}).get(kernel)
    if not k or d.get("source_sha256") != source_digest():
        return None
    return k.get("hbm_bytes_per_launch")


def cpu_baseline(psf, x, y, xs, ys, budget_s: float = 8.0) -> dict:
    """Time the oracle on a bounded sample of one iteration and scale up:
    forward projection at random pixels, back projection at random voxels
    (each sized to take ~budget_s), plus one full-size metric evaluation."""
    import numpy as np
    import oracle
    nz, h, w = x.shape
    rng = np.random.default_rng(0)
    xd = x.astype(np.float64)
    yd = y.astype(np.float64)

    def timed(fn, n):
        t = time.perf_counter()
        fn(n)
        return time.perf_counter() - t

    def fwd(n):
        oracle.forward_at(psf, xd, rng.integers(0, h, n), rng.integers(0, w, n))

    def bwd(n):
        oracle.backward_at(psf, yd, rng.integers(0, nz, n), rng.integers(0, h, n),
                           rng.integers(0, w, n))

    legs = {}
    for name, fn, total in (("forward", fwd, h * w), ("backward", bwd, nz * h * w)):
        n = 64
        t = timed(fn, n)
        while t < 0.5 and n < total:
            n = min(total, n * 4)
            t = timed(fn, n)
        n2 = int(min(total, max(n, n * budget_s / max(t, 1e-9))))
        t2 = timed(fn, n2)
        legs[name] = (n2, t2, t2 * total / n2)
    t = time.perf_counter()
    oracle.metric(xd, xs, ys)
    t_metric = time.perf_counter() - t
    t_iter = legs["forward"][2] + legs["backward"][2] + t_metric
    sample = (f"oracle forward at {legs['forward'][0]} random pixels ({legs['forward'][1]:.1f} s) "
              f"and back projection at {legs['backward'][0]} random voxels "
              f"({legs['backward'][1]:.1f} s), scaled to all {h * w} pixels and "
              f"{nz * h * w} voxels, plus one full metric ({t_metric:.2f} s); "
              f"estimated {t_iter:.0f} s per iteration")
    return {"value": 1.0 / t_iter, "unit": "iters/s", "cores": oracle.threads(),
            "kind": "oracle", "sample": sample}


GOLDEN_LARGE = os.path.join(ROOT, "tests", "golden", "large_rl_iterates.json")


def large_samples(lf, plan, g, dev) -> dict:
    """x^1 and x^2 of `plan` (fixed iteration counts, ones start) on the seeded
    image of the golden file of full-size iterates, at that file's sampled
    voxels: {window: {"x1": values, "x2": values}}.  The file holds the
    oracle's values at the same voxels (written by its own script from the
    oracle alone); the CPU leg compares the two."""
    import numpy as np
    import torch
    with open(GOLDEN_LARGE) as f:
        gold = json.load(f)
    seed = gold["image"]["seed"]
    y = np.random.default_rng(seed).uniform(10.0, 2000.0, size=(g.h, g.w)).astype(np.float32)
    y_d = torch.from_numpy(y).to(dev)
    out = {}
    for k in (1, 2):
        vol, _ = plan.deconvolve(y_d, k, stop=lf.STOP_NONE)
        v = vol.cpu().numpy()
        for win in gold["windows"]:
            if f"x{k}" in win:
                idx = np.asarray(win["voxels"])
                out.setdefault(win["name"], {})[f"x{k}"] = v[idx[:, 0], idx[:, 1], idx[:, 2]]
    return out


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def rel_l2(a, b) -> float:
    import numpy as np
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def accuracy_vs_oracle(samples: dict, dev) -> dict:
    """Relative L2 error against the float64 oracle, per workload:

    * small (Nnum 5, 55 x 55, 5 planes, K = 25) and its precision variant:
      every iterate x^1 .. x^30 of FP32, split FP16 and split BF16 (BF16 on to
      x^50, the serving cap), each the result of a fixed-length run, against
      the oracle's iterates on the same seeded input (the image projected by
      the oracle, Poisson noise from the generators);
    * large (600 x 600 x 31, K = 255): x^1 and x^2 at the golden file's
      sampled voxels (corner window with weakly observed voxels, interior
      window), per precision, against the oracle's stored values."""
    import numpy as np
    import torch

    import lfrl_synth as S
    import oracle
    import paper_2208_11422_amd as lf
    out = {}
    p = S.preset("small")
    g = p["geometry"]
    psf = p["psf_array"]
    y = S.measure(oracle.forward(psf, p["x_true"]), p["peak"], p["background"], p["noise_seed"])
    t = time.perf_counter()
    ref = oracle.rl(psf, y, 50, keep_all=True)
    log(f"accuracy: oracle 50 iterates of the small workload in {time.perf_counter() - t:.1f} s")
    y_d = torch.from_numpy(y).to(dev)
    psf_d = torch.from_numpy(psf).to(dev)
    for name, prec, iters in (("fp32", lf.FP32, 30), ("split_fp16", lf.SPLIT_FP16, 30),
                              ("split_bf16", lf.SPLIT_BF16, 50)):
        plan = lf.Plan(psf_d, g.h, g.w, precision=prec)
        errs = []
        for k in range(1, iters + 1):
            vol, _ = plan.deconvolve(y_d, k, stop=lf.STOP_NONE)
            errs.append(rel_l2(vol.cpu().numpy(), ref[k]))
        plan.close()
        tol = 1e-5 if prec == lf.FP32 else 1e-3
        within = next((k for k, e in enumerate(errs, 1) if e > tol), None)
        out[f"small_{name}"] = {"rel_l2_by_iter": errs, "max": max(errs),
                                "max_first_5": max(errs[:5]), "tol": tol,
                                "first_iter_above_tol": within}
    # large workload, sampled
    with open(GOLDEN_LARGE) as f:
        gold = json.load(f)
    for name, smp in samples.items():
        res = {}
        for win in gold["windows"]:
            for key in ("x1", "x2"):
                if key in win and key in smp.get(win["name"], {}):
                    want = np.asarray(win[key])
                    got = smp[win["name"]][key]
                    res[f"{win['name']}_{key}_rel_l2"] = rel_l2(got, want)
                    if win["name"] == "corner":
                        c = np.asarray(win["c"])
                        weak = c < 1e-2 * win["c_max"]
                        res[f"corner_{key}_weak_max_rel"] = float(
                            np.max(np.abs(got[weak] - want[weak]) / np.abs(want[weak])))
                        res["corner_weak_voxels"] = int(weak.sum())
        out[f"large_{name}"] = res
    log(f"accuracy: {json.dumps({k: {kk: vv for kk, vv in v.items() if kk != 'rel_l2_by_iter'} for k, v in out.items()})}")
    return out


def synth_measurement(plan, nz, h, w, seed, beads, peak, background, dev):
    """Measured image of a bead volume, made on the device: the bead splats of
    `seed` scattered into a volume, projected with `plan`, scaled to `peak`
    expected counts, Poisson counts from a device generator seeded with
    `seed`, plus `background`."""
    import numpy as np
    import torch

    import lfrl_synth as S
    idx, val = S.bead_splats(nz, h, w, beads, seed)
    uidx, inv = np.unique(idx, return_inverse=True)
    uval = np.zeros(uidx.size)
    np.add.at(uval, inv, val)                       # overlaps summed in bead order
    vol = torch.zeros(nz * h * w, dtype=torch.float32, device=dev)
    vol[torch.from_numpy(uidx).to(dev)] = torch.from_numpy(uval.astype(np.float32)).to(dev)
    lam = plan.forward(vol.view(nz, h, w))
    lam = torch.clamp_min(lam * (peak / lam.max()), 0.0)
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    return torch.poisson(lam, generator=gen) + background


def request_images(specs, plans, cfg, dev):
    """Serving request images (see synth_measurement), as pinned host tensors:
    a request's image arrives from the host."""
    import torch
    out = []
    for sp in specs:
        y = synth_measurement(plans[sp["set"]], sp["nz"], sp["h"], sp["w"], sp["seed"],
                              cfg["beads"], cfg["peak"], cfg["background"], dev)
        host = torch.empty(y.shape, dtype=torch.float32, pin_memory=True)
        host.copy_(y)
        out.append(host)
    torch.cuda.synchronize()
    return out


def small_leg(args, dev) -> dict:
    """The small workload (Nnum 5, 55 x 55, 5 planes, K = 25), which is bound
    by launch latency rather than bandwidth: calls of lfrl_deconvolve with its
    5 iterations, with the run replayed from a captured graph and with direct
    launches.  (Its accuracy against the oracle, per iterate and precision,
    is measured in the CPU leg.)"""
    import torch

    import lfrl_synth as S
    import paper_2208_11422_amd as lf
    p = S.preset("small")
    g = p["geometry"]
    psf_d = torch.from_numpy(p["psf_array"]).to(dev)
    plan = lf.Plan(psf_d, g.h, g.w)
    clean = plan.forward(torch.from_numpy(p["x_true"]).to(dev)).cpu().numpy()
    y = torch.from_numpy(S.measure(clean, p["peak"], p["background"], p["noise_seed"])).to(dev)
    xs = ys = g.w / (g.nnum * 2.0 * p["spot_radius"])
    vol = torch.empty((g.nz, g.h, g.w), dtype=torch.float32, device=dev)
    opts = lf.RlOpts(max_iters=p["iters"], stop=lf.STOP_TRACK, patience=1, init=0, xs=xs, ys=ys)
    out = {"workload": "Nnum 5, 11x11 lenslets (55x55), 5 planes, K=25, 5 iterations per call",
           "iters_per_call": p["iters"]}
    for mode in ("graph", "direct"):
        os.environ["LFRL_GRAPH"] = "1" if mode == "graph" else "0"
        for _ in range(5):
            lf.lfrl_deconvolve(plan.handle, g.h, g.w, y, vol, opts, want_metric=False)
        torch.cuda.synchronize()
        calls = args.small_calls
        t0 = time.perf_counter()
        for _ in range(calls):
            lf.lfrl_deconvolve(plan.handle, g.h, g.w, y, vol, opts, want_metric=False)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / calls
        out[mode] = {"ms_per_call": ms, "iters_per_s": p["iters"] * 1e3 / ms}
    os.environ.pop("LFRL_GRAPH", None)
    out["graph_speedup"] = out["direct"]["ms_per_call"] / out["graph"]["ms_per_call"]
    plan.close()
    log(f"small: {json.dumps(out)}")
    return out


def batched_leg(args, dev) -> dict:
    """Independent frames of uneven sizes, each with its own FP32 plan (tile
    side chosen by the autotuner): the frames one after another through
    lfrl_deconvolve, then all together as jobs stepped in lock-step (plans run
    side by side on internal streams).  A^T 1 of each frame is formed before
    the timed regions, like the plans."""
    import torch

    import lfrl_synth as S
    import paper_2208_11422_amd as lf
    cfg = S.BATCHED
    t_all = time.perf_counter()
    specs = S.batched_frames(args.batched_frames)
    plans, imgs, opts = [], [], []
    for sp in specs:
        t = time.perf_counter()
        psf_d = torch.from_numpy(S.batched_psf(sp)).to(dev)
        plans.append(lf.Plan(psf_d, sp["h"], sp["w"], autotune=True))
        del psf_d
        imgs.append(synth_measurement(plans[-1], sp["nz"], sp["h"], sp["w"], sp["seed"],
                                      cfg["beads"], cfg["peak"], cfg["background"], dev))
        xs = sp["w"] / (sp["nnum"] * 2.0 * cfg["spot_radius"])
        ys = sp["h"] / (sp["nnum"] * 2.0 * cfg["spot_radius"])
        opts.append(lf.RlOpts(max_iters=cfg["iters"], stop=lf.STOP_TRACK, patience=1, init=0,
                              xs=xs, ys=ys))
        info = plans[-1].info
        log(f"batched: frame {sp['frame']} N={sp['nnum']} {sp['h']}x{sp['w']}x{sp['nz']} "
            f"K={sp['ksize']} Q={info['tile_q']} (tuned over {info['tune_candidates']}, "
            f"{info['tune_ms']:.2f} ms) {time.perf_counter() - t:.1f} s")
    vols_seq = [torch.empty((sp["nz"], sp["h"], sp["w"]), device=dev) for sp in specs]
    vols_bat = [torch.empty_like(v) for v in vols_seq]
    for pl, sp, y, o, v in zip(plans, specs, imgs, opts, vols_seq):   # warm-up, A^T 1
        o1 = lf.RlOpts(max_iters=1, stop=o.stop, patience=1, init=0, xs=o.xs, ys=o.ys)
        lf.lfrl_deconvolve(pl.handle, sp["h"], sp["w"], y, v, o1, want_metric=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for pl, sp, y, o, v in zip(plans, specs, imgs, opts, vols_seq):
        lf.lfrl_deconvolve(pl.handle, sp["h"], sp["w"], y, v, o, want_metric=False)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    jobs = [lf.Job(pl, y, cfg["iters"], stop=lf.STOP_TRACK, xs=o.xs, ys=o.ys)
            for pl, y, o in zip(plans, imgs, opts)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while lf.Job.step(jobs) > 0:
        pass
    for j, v in zip(jobs, vols_bat):
        j.result(out=v)
    torch.cuda.synchronize()
    t_bat = time.perf_counter() - t0
    same = all(bool(torch.equal(a, b)) for a, b in zip(vols_seq, vols_bat))
    for j in jobs:
        j.close()
    n_it = len(specs) * cfg["iters"]
    vox = sum(sp["nz"] * sp["h"] * sp["w"] for sp in specs) * cfg["iters"]
    out = {"frames": len(specs), "iters_per_frame": cfg["iters"], "precision": "fp32",
           "stop": "metric tracked, best kept",
           "batched": {"seconds": t_bat, "frames_per_s": len(specs) / t_bat,
                       "iters_per_s": n_it / t_bat, "voxel_updates_per_s": vox / t_bat},
           "sequential": {"seconds": t_seq, "frames_per_s": len(specs) / t_seq,
                          "iters_per_s": n_it / t_seq, "voxel_updates_per_s": vox / t_seq},
           "speedup": t_seq / t_bat, "batched_equals_sequential": same,
           "tile_q": [pl.info["tile_q"] for pl in plans]}
    for pl in plans:
        pl.close()
    torch.cuda.empty_cache()
    out["leg_seconds"] = time.perf_counter() - t_all
    log(f"batched: {json.dumps(out)}")
    return out


def serving_leg(args, dev) -> dict:
    """Served deconvolution requests for four resident split-FP16 PSF sets:
    saturation rate from a closed loop (every request queued at t = 0), then
    open-loop Poisson arrivals at 0.8 and 0.5 of it; latency is arrival to
    result volume in host memory."""
    import torch

    import lfrl_synth as S
    import paper_2208_11422_amd as lf
    from paper_2208_11422_amd.serve import JobExecutor, Request, Scheduler, latency_stats
    cfg = S.SERVING
    t_all = time.perf_counter()
    plans = []
    for k, (n, nz, seed) in enumerate(cfg["sets"]):
        t = time.perf_counter()
        psf = S._cached(f"psf_serving_{n}_{nz}_{cfg['ksize']}_{seed}",
                        lambda: S.serving_psf(k), CACHE)
        t_gen = time.perf_counter() - t
        psf_d = torch.from_numpy(psf).to(dev)
        del psf
        side = cfg["max_side"] // n * n
        plans.append(lf.Plan(psf_d, side, side, precision=lf.SPLIT_FP16,
                             max_batch=args.serving_batch, autotune=args.serving_autotune))
        del psf_d
        torch.cuda.synchronize()
        info = plans[-1].info
        log(f"serving: set {k} (N={n}, nz={nz}) PSF {t_gen:.1f} s, plan Q={info['tile_q']} "
            f"spectra {info['resident_bytes'] / 1e9:.2f} GB, workspace "
            f"{info['workspace_bytes'] / 1e9:.2f} GB, {time.perf_counter() - t:.1f} s")
    specs = S.serving_requests(args.serving_requests)
    t = time.perf_counter()
    images = request_images(specs, plans, cfg, dev)
    log(f"serving: {len(specs)} request images in {time.perf_counter() - t:.1f} s")
    r = cfg["spot_radius"]
    legs = {sp["rid"]: (sp["w"] / (sp["nnum"] * 2.0 * r), sp["h"] / (sp["nnum"] * 2.0 * r))
            for sp in specs}

    def opts_for(req):
        xs, ys = legs[req.rid]
        return dict(iters=cfg["max_iters"], stop=lf.STOP_METRIC, patience=1, xs=xs, ys=ys)

    check = [sp["rid"] for sp in specs[:3]]
    budget = int(args.serving_budget_gb * 1e9)

    def run(arrivals, keep=()):
        reqs = [Request(rid=sp["rid"], plan=sp["set"], h=sp["h"], w=sp["w"], image=img,
                        arrival=float(a)) for sp, img, a in zip(specs, images, arrivals)]
        ex = JobExecutor(plans, opts_for, keep=keep)
        sched = Scheduler(ex, budget, max_active=args.serving_active)
        t0 = time.perf_counter()
        sched.run(reqs)
        span = time.perf_counter() - t0
        st = latency_stats(reqs, span)
        st.update(span_s=span, rounds=sched.rounds, peak_active=sched.peak_active,
                  peak_job_gb=sched.peak_bytes / 1e9,
                  mean_batch=sum(sched.batch_sizes) / max(len(sched.batch_sizes), 1),
                  mean_iters=sum(q.iters for q in reqs) / len(reqs),
                  op_seconds={k: round(v, 4) for k, v in sched.op_seconds.items()})
        return st, reqs

    closed, reqs = run([0.0] * len(specs), keep=check)
    mu = closed["frames_per_s"]
    log(f"serving: closed loop {json.dumps(closed)}")
    # a served result is the volume the same request gets alone
    same = True
    for q in reqs:
        if q.rid in check:
            sp = specs[q.rid]
            xs, ys = legs[q.rid]
            alone, _ = plans[sp["set"]].deconvolve(images[q.rid].to(dev), cfg["max_iters"],
                                                   stop=lf.STOP_METRIC, xs=xs, ys=ys)
            same &= bool(torch.equal(alone.cpu(), q.result))
    out = {"requests": len(specs), "psf_sets": [list(s[:2]) for s in cfg["sets"]],
           "ksize": cfg["ksize"], "precision": "split-fp16", "stop": "metric, cap 50",
           "budget_gb": args.serving_budget_gb, "saturation_frames_per_s": mu,
           "closed_loop": closed, "alone_vs_mix_equal": same}
    for frac in (0.8, 0.5):
        arr = S.poisson_arrivals(len(specs), frac * mu)
        st, _ = run(arr)
        log(f"serving: open loop at {frac} x saturation {json.dumps(st)}")
        out[f"open_loop_{frac}"] = st
    for p in plans:
        p.close()
    torch.cuda.empty_cache()
    out["leg_seconds"] = time.perf_counter() - t_all
    return out


def variants_leg(args, lf, plan, y_d, vol, h, w, xs, ys, background, ms_rl) -> dict:
    """The variants on the headline workload: ISRA with the background term from
    the back projection start, RL with the background and the window stop on
    the rectangle with the region norm, and the whole-matrix metric alone."""
    import torch
    out = {}
    steps = max(args.steps, 1)
    runs = {
        "isra_background_backproject": dict(update=lf.UPDATE_ISRA, background=background,
                                            backproject_start=True),
        "rl_background_rectangle_window3": dict(background=background,
                                                region=lf.REGION_RECTANGLE,
                                                norm=lf.NORM_REGION, window=3),
    }
    for name, kw in runs.items():
        opts = lf.rl_opts(max(args.warmup, 1), lf.STOP_TRACK, 1, xs, ys, **kw)
        lf.lfrl_deconvolve(plan.handle, h, w, y_d, vol, opts)
        torch.cuda.synchronize()
        opts.max_iters = steps
        t0 = time.perf_counter()
        rep = lf.lfrl_deconvolve(plan.handle, h, w, y_d, vol, opts)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1000.0 / steps
        out[name] = {"value": 1000.0 / ms, "unit": "iters/s", "ms_per_step": ms,
                     "vs_rl": ms_rl / ms, "best_iter": rep["best_iter"]}
        log(f"bench: variant {name}: {ms:.3f} ms/iter ({1000.0 / ms:.1f} it/s)")
    out["isra_background_backproject"]["note"] = "includes the one back projection A^T y"
    res = torch.empty(1, dtype=torch.float64, device=vol.device)
    for name, region, norm in (("triangle", lf.REGION_TRIANGLE, lf.NORM_MATRIX),
                               ("whole", lf.REGION_WHOLE, lf.NORM_MATRIX),
                               ("triangle_spectral", lf.REGION_TRIANGLE, lf.NORM_SPECTRAL)):
        nz = vol.shape[0]
        lf.lfrl_metric_ex(nz, h, w, vol, xs, ys, region, norm, res)
        torch.cuda.synchronize()
        calls = 20
        t0 = time.perf_counter()
        for _ in range(calls):
            lf.lfrl_metric_ex(nz, h, w, vol, xs, ys, region, norm, res)
        torch.cuda.synchronize()
        out[f"metric_{name}_ms"] = (time.perf_counter() - t0) * 1000.0 / calls
        log(f"bench: metric {name}: {out[f'metric_{name}_ms']:.3f} ms per call")
    return out


PSF_OPTICS = dict(wavelength=0.52, na=0.5, n_medium=1.0, mag=20.0, d_ml=150.0, f_ml=3000.0,
                  nnum=15, ksize=255, osr=3, nquad=1024)
PSF_DEPTHS = [2.0 * (j - 15) for j in range(31)]


def psf_optics_leg(args, lf, dev) -> dict:
    """The PSF set from optical parameters (a 20x / 0.5 objective, 150 um
    lenslets of f/20, Nnum 15, 255 x 255 pixels at 3 samples per pixel, 31
    depths 2 um apart): time per full set on the GPU."""
    import numpy as np
    import torch
    log("bench: psf from optics")
    out = torch.empty((len(PSF_DEPTHS), 15, 15, 255, 255), dtype=torch.float32, device=dev)
    o = lf.Optics(nz=len(PSF_DEPTHS), flags=lf.PSF_UNIT_SUM, **PSF_OPTICS)
    lf.lfrl_psf_compute(o, PSF_DEPTHS, out)   # warm-up (first launches, allocations)
    times = []
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lf.lfrl_psf_compute(o, PSF_DEPTHS, out)
        times.append(time.perf_counter() - t0)
    res = {"optics": dict(PSF_OPTICS), "depths": [PSF_DEPTHS[0], PSF_DEPTHS[-1], len(PSF_DEPTHS)],
           "kernels": len(PSF_DEPTHS) * 15 * 15, "seconds_per_set": float(np.median(times)),
           "grid": 768}
    del out
    log(f"bench: psf from optics {res['seconds_per_set']:.3f} s per set")
    return res


def psf_optics_cpu(res: dict) -> dict:
    """The oracle on one depth's Debye field and one kernel's propagation,
    scaled to the whole set (31 depths, 225 kernels each)."""
    from oracle import optics as O
    o = O.Optics(**PSF_OPTICS)
    t0 = time.perf_counter()
    nip = O.nip_window(PSF_DEPTHS[0], o)
    t1 = time.perf_counter()
    for a, b in ((0, 0), (7, 7)):
        O.bin_pixels(O.sensor_field(nip, a, b, o), o)
    t2 = time.perf_counter()
    per_depth = t1 - t0
    per_kernel = (t2 - t1) / 2
    total = len(PSF_DEPTHS) * (per_depth + 225 * per_kernel)
    return {"seconds_per_set_est": total, "sample": "one depth's Debye field "
            f"({per_depth:.1f} s) and two kernels' propagation ({per_kernel:.2f} s each), "
            "scaled to 31 depths x 225 kernels", "speedup_gpu_vs_oracle":
            total / res["seconds_per_set"]}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--tile-q", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-split", action="store_true",
                    help="skip the split-FP16 measurement")
    ap.add_argument("--small-calls", type=int, default=200,
                    help="timed calls of the small-workload leg (0 skips it)")
    ap.add_argument("--batched-frames", type=int, default=16,
                    help="frames of the batched uneven-size leg (0 skips it)")
    ap.add_argument("--serving-requests", type=int, default=2000,
                    help="requests of the serving leg (0 skips it; the full workload is 2000)")
    ap.add_argument("--serving-batch", type=int, default=4,
                    help="largest frames one projection launch of a PSF set covers")
    ap.add_argument("--serving-active", type=int, default=32, help="jobs in flight at most")
    ap.add_argument("--serving-autotune", action="store_true",
                    help="measured tile side for the serving PSF sets (default: the model's)")
    ap.add_argument("--serving-budget-gb", type=float, default=96.0,
                    help="device memory admitted jobs may hold")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the update / metric variant leg")
    ap.add_argument("--no-psf-optics", action="store_true",
                    help="skip the PSF-from-optics leg")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run one 1 GiB device-to-device copy (reference kernel of known "
                         "size for hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the z-sharded "
              "multi-GPU path is designed but not implemented", file=sys.stderr)
        return 2
    if os.environ.get("WORLD_SIZE", "1") != "1":
        print("bench.py is single-process; WORLD_SIZE must be 1", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import lfrl_synth as S
    import paper_2208_11422_amd as lf

    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    t_setup = time.perf_counter()
    p = S.preset("large", cache_dir=CACHE)
    g = p["geometry"]
    h, w = g.h, g.w
    log(f"bench: inputs ready in {time.perf_counter() - t_setup:.1f} s")
    psf_d = torch.from_numpy(p["psf_array"]).to(dev)
    x_true = torch.from_numpy(p["x_true"]).to(dev)
    t = time.perf_counter()
    plan = lf.Plan(psf_d, h, w, tile_q=args.tile_q)
    torch.cuda.synchronize()
    info = plan.info
    log(f"bench: plan Q={info['tile_q']} T={info['tile_out']} R={info['taps']} "
        f"tiles={info['max_tiles']} split={info['split_k']} "
        f"spectra {info['resident_bytes'] / 1e9:.2f} GB, built in {time.perf_counter() - t:.2f} s")
    del psf_d
    clean = plan.forward(x_true).cpu().numpy()
    y = S.measure(clean, p["peak"], p["background"], p["noise_seed"])
    y_d = torch.from_numpy(y).to(dev)
    xs, ys = 2 * [w / (g.nnum * 2.0 * p["spot_radius"])]
    vol = torch.empty((g.nz, h, w), dtype=torch.float32, device=dev)

    def run(iters: int):
        opts = lf.RlOpts(max_iters=iters, stop=lf.STOP_TRACK, patience=1, init=0, xs=xs, ys=ys)
        return lf.lfrl_deconvolve(plan.handle, h, w, y_d, vol, opts)

    log(f"bench: warmup {args.warmup}")
    if args.warmup > 0:
        run(args.warmup)
    torch.cuda.synchronize()
    lf.lfrl_profile_enable(plan.handle, True)
    log(f"bench: timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rep = run(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = {k: lf.lfrl_profile_read(plan.handle, k) for k in ("contract_fwd", "contract_adj")}
    lf.lfrl_profile_enable(plan.handle, False)
    ms_per_step = (t1 - t0) * 1000.0 / args.steps
    value = 1000.0 / ms_per_step
    nt = info["max_tiles"]
    dom = max(prof, key=lambda k: prof[k][0])
    tot_ms, launches = prof[dom]
    avg_ms = tot_ms / max(launches, 1)
    b_alg = contraction_bytes(info, g, nt, dom)
    achieved = b_alg / (avg_ms * 1e-3) / 1e9
    traffic = measured_traffic(dom, b_alg)
    kern = {k: {"avg_ms": v[0] / max(v[1], 1), "launches": v[1],
                "gbs": contraction_bytes(info, g, nt, k) / (v[0] / max(v[1], 1) * 1e-3) / 1e9,
                "tflops": contraction_flops(info, g, nt) / (v[0] / max(v[1], 1) * 1e-3) / 1e12}
            for k, v in prof.items()}
    log(f"bench: {ms_per_step:.3f} ms/iter, {value:.1f} it/s; kernels {json.dumps(kern)}")
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "light-field RL, Nnum 15, 40x40 lenslets (600x600 image), 31 planes, "
                        "255x255 defocus-disk PSF, 500 beads + 3 filaments, Poisson peak 2000, "
                        "DCT-entropy metric every iteration (best iterate kept)",
            "nnum": g.nnum, "h": h, "w": w, "nz": g.nz, "ksize": g.ksize,
            "precision": "fp32", "tile_q": info["tile_q"], "tiles": nt,
            "metric_legs": [xs, ys],
        },
        "voxel_updates_per_s": value * g.nz * h * w,
        "best_iter": rep["best_iter"],
        "roofline": {
            "kernel": dom,
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "bytes_per_launch": b_alg,
            "avg_ms": avg_ms,
            "launches": launches,
            "flops_frac_fp32": contraction_flops(info, g, nt) / (avg_ms * 1e-3) / 1e12
            / FP32_PEAK_TFLOPS,
        },
        "kernels": kern,
        "model": iteration_model(info, g, h, w, nt, ms_per_step, precision="fp32"),
    }
    # x^steps of a fixed-length run (no stop rule), which the split paths are
    # compared with; and x^1, x^2 at the golden file's sampled voxels of its
    # seeded image, compared with the oracle's values in the CPU leg
    vol32, _ = plan.deconvolve(y_d, args.steps, stop=lf.STOP_NONE)
    samples = {"fp32": large_samples(lf, plan, g, dev)}
    if not args.no_variants:
        out["variants"] = variants_leg(args, lf, plan, y_d, vol, h, w, xs, ys,
                                       float(p["background"]), ms_per_step)
    if not args.no_split:
        for name, prec in (("split_fp16", lf.SPLIT_FP16), ("split_bf16", lf.SPLIT_BF16)):
            plan.close()
            torch.cuda.empty_cache()
            psf_d = torch.from_numpy(p["psf_array"]).to(dev)
            plan = lf.Plan(psf_d, h, w, tile_q=args.tile_q, precision=prec)
            del psf_d
            torch.cuda.synchronize()
            opts16 = lf.RlOpts(max_iters=args.warmup if args.warmup > 0 else 1,
                               stop=lf.STOP_TRACK, patience=1, init=0, xs=xs, ys=ys)
            lf.lfrl_deconvolve(plan.handle, h, w, y_d, vol, opts16)
            lf.lfrl_profile_enable(plan.handle, True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            opts16.max_iters = args.steps
            lf.lfrl_deconvolve(plan.handle, h, w, y_d, vol, opts16)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            prof16 = {k: lf.lfrl_profile_read(plan.handle, k)
                      for k in ("contract_fwd", "contract_adj")}
            lf.lfrl_profile_enable(plan.handle, False)
            ms16 = (t1 - t0) * 1000.0 / args.steps
            x16, _ = plan.deconvolve(y_d, args.steps, stop=lf.STOP_NONE)
            diff = float(torch.linalg.vector_norm(x16 - vol32) / torch.linalg.vector_norm(vol32))
            del x16
            samples[name] = large_samples(lf, plan, g, dev)
            word = "f16" if prec == lf.SPLIT_FP16 else "bf16"
            out[name] = {
                "value": 1000.0 / ms16, "unit": "iters/s", "ms_per_step": ms16,
                "model": iteration_model(plan.info, g, h, w, plan.info["max_tiles"], ms16,
                                         precision=name.replace("_", "-")),
                "dtype": f"{word} spectra, hi/lo {word} tile spectra, f32 accumulate",
                "rel_l2_vs_fp32": {"iterate": args.steps, "stop": "none", "value": diff},
                "speedup_vs_fp32": ms_per_step / ms16,
                "kernels": {k: {"avg_ms": v[0] / max(v[1], 1), "launches": v[1]}
                            for k, v in prof16.items()},
            }
            log(f"bench: {name} {ms16:.3f} ms/iter ({1000.0 / ms16:.1f} it/s), "
                f"x^{args.steps} rel L2 vs FP32 {diff:.2e}")
    if args.small_calls > 0 or args.batched_frames > 0 or args.serving_requests > 0:
        plan.close()
        plan = None
        torch.cuda.empty_cache()
    if not args.no_psf_optics:
        out["psf_optics"] = psf_optics_leg(args, lf, dev)
        torch.cuda.empty_cache()
    if args.small_calls > 0:
        out["small"] = small_leg(args, dev)
    if args.batched_frames > 0:
        out["batched"] = batched_leg(args, dev)
    if args.serving_requests > 0:
        out["serving"] = serving_leg(args, dev)
        out["p50_ms"] = out["serving"]["open_loop_0.8"]["p50_ms"]
        out["p99_ms"] = out["serving"]["open_loop_0.8"]["p99_ms"]
    if not args.no_cpu_baseline:
        import tempfile

        import oracle
        log("bench: cpu baseline (oracle, bounded sample)")
        with tempfile.TemporaryDirectory() as tmp:
            flags = oracle.use_native_build(tmp)
        # oracle inputs come from the generators, never from the GPU path; the
        # oracle's cost does not depend on the values
        x_dense = p["x_true"] + np.float32(1.0)
        y_syn = np.random.default_rng(1).uniform(10.0, 2000.0, size=(h, w)).astype(np.float32)
        out["cpu_baseline"] = cpu_baseline(p["psf_array"], x_dense, y_syn, xs, ys)
        out["cpu_baseline"].update(cpu_model=cpu_model(), build=f"gcc {flags}",
                                   method="sampled outputs, time scaled to the whole iteration",
                                   host_cpus=os.cpu_count())
        log(f"bench: cpu baseline {json.dumps(out['cpu_baseline'])}")
        out["accuracy_vs_oracle"] = accuracy_vs_oracle(samples, dev)
        if "psf_optics" in out:
            out["psf_optics"]["cpu_oracle"] = psf_optics_cpu(out["psf_optics"])
            log(f"bench: psf oracle {json.dumps(out['psf_optics']['cpu_oracle'])}")
    if plan is not None:
        plan.close()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
