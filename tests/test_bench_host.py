"""Host logic of bench.py (CPU): the one-GPU contract, the algorithmic work per
unit that the roofline divides by, the bound and peak it picks, and the rule
that a counter summary gives `traffic` only when it was taken on the current
kernel sources."""
import hashlib
import importlib.util
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_host", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_work_per_unit_of_the_metric_kernels(bench):
    N, Nt, r = 15, 2 ** 14, 45
    Np = N * (N + 1) // 2
    c = bench.work_per_eval("contract", N, Nt, "bf16x3", rank=r)
    # C = U Y' then the mode projection: 2 Np r Nt useful flops; Y' (hi/lo, 4 bytes per value) in, A in, NL out
    assert c["compute"] == "mfma"
    assert c["flops"] == 2.0 * Np * r * Nt == 176_947_200
    assert c["bytes"] == r * Nt * 4 + 2 * N * Nt * 8 == 6_881_280
    p = bench.work_per_eval("project", N, Nt, "bf16x3", rank=r)
    assert p["flops"] == 2.0 * r * Np * Nt and p["bytes"] == N * Nt * 8 + r * Nt * 4
    k = bench.work_per_eval("pairs_raman", N, Nt, "bf16x3", rank=r)
    assert k["bytes"] == 2 * r * Nt * 4           # Y in, Y' out
    # FP64 doubles every stored value
    assert bench.work_per_eval("contract", N, Nt, "fp64", rank=r)["bytes"] == r * Nt * 8 + 2 * N * Nt * 16


def test_roofline_bound_peak_and_fraction(bench):
    N, Nt, r = 15, 2 ** 14, 45
    wk = bench.work_per_eval("contract", N, Nt, "bf16x3", rank=r)
    launches, evals, us = 150, 1550, 27.0
    prof = {"contract": (launches * us * 1e-3, launches), "pairs_raman": (1.0, launches)}
    line = bench.roofline(prof, {"evaluations": evals}, N, Nt, "bf16x3", "no_such_workload", rank=r)
    assert line["kernel"] == "contract"            # the kind with the most total time
    sec = launches * us * 1e-6
    hbm = wk["bytes"] * evals / sec / 1e9
    assert line["bound"] == "hbm" and line["unit"] == "GB/s" and line["peak"] == 8000.0
    assert line["achieved"] == pytest.approx(hbm, rel=1e-3)
    assert line["frac"] == pytest.approx(hbm / 8000.0, abs=1e-4)
    # four bf16 products per useful multiply-add on the rank-r contraction: a quarter of 2.5 PFLOP/s
    assert line["compute_frac"] == pytest.approx(wk["flops"] * evals / sec / 1e12 / 625.0, abs=1e-4)
    assert line["traffic"] is None                 # no counter summary for this workload name
    assert line["units_per_launch"] == pytest.approx(evals / launches, rel=1e-3)
    # the general route keeps three products
    g = bench.roofline({"contract": (1.0, 10)}, {"evaluations": 100}, N, Nt, "bf16x3", "x", rank=0,
                       route="general")
    wg = bench.work_per_eval("contract", N, Nt, "bf16x3", route="general")
    assert g["compute_frac"] == pytest.approx(wg["flops"] * 100 / 1e-3 / 1e12 / (2500.0 / 3.0), abs=1e-4)


def test_traffic_only_from_a_summary_of_the_current_sources(bench, tmp_path, monkeypatch):
    h = hashlib.sha256()
    src = os.path.join(ROOT, "paper_1708_05324_amd", "csrc")
    for f in sorted(os.listdir(src)):
        h.update(open(os.path.join(src, f), "rb").read())
    sha = h.hexdigest()[:16]
    fake = tmp_path / "repo"
    (fake / "profiles").mkdir(parents=True)
    os.symlink(os.path.join(ROOT, "paper_1708_05324_amd"), fake / "paper_1708_05324_amd")
    monkeypatch.setattr(bench, "ROOT", str(fake))
    path = fake / "profiles" / "counters_contract_wl_bf16x3.md"
    path.write_text(f"kernel_sources_sha: {sha}\nhbm_bytes_per_launch: 7.25e+07\n")
    assert bench.read_traffic("contract", "wl", "bf16x3") == 7.25e7
    path.write_text("kernel_sources_sha: 0000000000000000\nhbm_bytes_per_launch: 7.25e+07\n")
    assert bench.read_traffic("contract", "wl", "bf16x3") is None
    assert bench.read_traffic("project", "wl", "bf16x3") is None
