"""Host-side bookkeeping of bench.py (no GPU): the algorithmic bytes of the
contraction launches at the 600 x 600 x 31 workload, the roofline model's
bound, the rule that counter traffic is reported only for the kernel
sources it was taken on, and the one-GPU guard."""
import importlib.util
import json
import os
import subprocess
import sys
import types

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_host", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


# Nnum 15, 31 planes, 255 x 255 PSF, Q = 28 (T = 10, R = 19), 16 tiles,
# 394 unique frequencies of 420, 5 forward reduction chunks
G = types.SimpleNamespace(nnum=15, nz=31, ksize=255)
INFO = {"nfreq_unique": 394, "split_k": 5, "tile_q": 28, "tile_out": 10, "taps": 19}


def test_contraction_bytes_by_hand(bench):
    nf, nn, kk, nt = 394, 225, 225 * 31, 16
    spectra = nf * nn * kk * 8            # the PSF spectra, once
    x = nf * nt * kk * 8                  # volume tile spectra
    yp = 5 * nf * nt * nn * 8             # forward partial images
    r = nf * nt * nn * 8                  # image tile spectra
    assert bench.contraction_bytes(INFO, G, nt, "contract_fwd") == spectra + x + yp
    assert bench.contraction_bytes(INFO, G, nt, "contract_adj") == spectra + r + x
    assert spectra + x + yp == 5_355_169_200


def test_iteration_model_bounds(bench):
    m32 = bench.iteration_model(INFO, G, 600, 600, 16, 2.43, "fp32")
    m16 = bench.iteration_model(INFO, G, 600, 600, 16, 1.62, "split-fp16")
    # both are bound by memory; the split modes stream half the PSF bytes and
    # their contraction flops run on the 16-bit matrix cores
    assert m32["bound"] == "hbm" and m16["bound"] == "hbm"
    assert m16["bytes_per_iter"] < m32["bytes_per_iter"]
    assert m16["t_contract_ms"] < 0.2 < m32["t_contract_ms"]
    assert m32["frac_of_bound"] == pytest.approx(m32["t_bound_ms"] / 2.43)
    # floor: the PSF (31 x 225 kernels of 255^2 float32) read once per projection
    assert m32["floor_ms"] == pytest.approx(2 * 31 * 225 * 255 * 255 * 4 / 8e12 * 1e3)


def test_traffic_only_for_matching_sources(bench, monkeypatch, tmp_path):
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "contract_traffic.json").write_text(json.dumps(
        {"source_sha256": "abc", "kernels": {"contract_fwd": {"hbm_bytes_per_launch": 123.0}}}))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "source_digest", lambda: "abc")
    assert bench.measured_traffic("contract_fwd", 1.0) == 123.0
    assert bench.measured_traffic("contract_adj", 1.0) is None
    monkeypatch.setattr(bench, "source_digest", lambda: "changed")
    assert bench.measured_traffic("contract_fwd", 1.0) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""
