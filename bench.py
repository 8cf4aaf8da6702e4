#!/usr/bin/env python3
"""Benchmark of the massively parallel GMMNLSE propagation step on one MI355X.

Workload: parabolic GRIN fibre, 15 modes (Hermite-Gauss groups 0-4), Nt = 2^14
samples over 40 ps, Kerr + Raman (fR = 0.18) + self-steepening, 200 fs
Gaussian of 100 nJ spread evenly over the modes with seeded phases, M = 10
small steps per large step, dz = min(z_NL/200, z_IM/5) = 9.13 um.

One benchmark step is one MPA large step (M small steps dz, iterated to the
tolerance).  The metric is converged small steps dz per second.  Prints one
JSON line.  Use --gpus 1 only: the library runs on one GPU.
"""
from __future__ import annotations

import argparse
import glob
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAKS = {  # MI355X published dense peaks
    "hbm_GBps": 8000.0,
    "mfma_fp32_TFLOPs": 157.3,
    "mfma_fp64_TFLOPs": 78.6,
    "mfma_bf16_TFLOPs": 2500.0,
    # three bf16 products per useful multiply-add: useful-work peak of the split contraction
    "mfma_bf16x3_TFLOPs": 2500.0 / 3.0,
    # four on the packed and rank-r routes' contraction and projection (a third plane of the fixed matrix)
    "mfma_bf16x4_TFLOPs": 2500.0 / 4.0,
    # vector ALU with packed FP32 disabled: 256 CU x 64 lanes x 2 (FMA) x 2.4 GHz
    "alu_fp32_TFLOPs": 78.6,
    "alu_fp64_TFLOPs": 78.6,
}
TOL = {"fp64": 1e-12, "fp32": 1e-6, "bf16x3": 1e-5}
DTYPE = {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3+f32"}


def work_per_eval(kind: str, N: int, Nt: int, prec: str, rank: int = 0, route: str = "packed") -> dict:
    """Algorithmic work of one kernel kind for one sub-step integrand: flops
    (of the unit named in "compute") and HBM bytes.

    rank > 0: the plan contracts through the factor S^ = U V (U: Np x r), so the
    Raman convolution acts on r rows and the products are 2 r Np Nt each.
    bf16x3 executes three bf16 products per useful multiply-add (four in the
    packed and rank-r contraction and projection, whose fixed matrix has a
    third plane);
    the useful count is what is reported (against the matching useful-work peak).  The
    sub-step transforms and the spectral output also read the phase table
    (one complex per element)."""
    Np = N * (N + 1) // 2
    rs = 8 if prec == "fp64" else 4        # bytes per real (a bf16 hi/lo pair is 4 bytes too)
    cs = 2 * rs
    fft = 5.0 * Nt * math.log2(Nt)
    if route == "general":   # 4 real rows per pair; real GEMM 2 N^2 x 4 Np; one complex transform pair per pair
        if kind == "contract":
            return {"compute": "mfma", "flops": 2.0 * (2 * N * N) * (4 * Np) * Nt,
                    "bytes": 4 * Np * Nt * rs + 2 * N * Nt * cs}
        if kind == "pairs_raman":
            return {"compute": "alu", "flops": Np * 2 * fft, "bytes": N * Nt * cs + 4 * Np * Nt * rs}
    if kind == "contract":
        k = rank if rank else Np
        return {"compute": "mfma", "flops": 2.0 * Np * k * Nt, "bytes": k * Nt * rs + 2 * N * Nt * cs}
    if kind == "project":
        return {"compute": "mfma", "flops": 2.0 * rank * Np * Nt, "bytes": N * Nt * cs + rank * Nt * rs}
    if kind == "pairs_raman":
        if rank:   # convolution of the r rows of Y: read Y, write Y'
            return {"compute": "alu", "flops": math.ceil(rank / 2) * 2 * fft, "bytes": 2 * rank * Nt * rs}
        return {"compute": "alu", "flops": math.ceil(Np / 2) * 2 * fft, "bytes": N * Nt * cs + Np * Nt * rs}
    if kind in ("phase_to_time", "spectral_out"):
        return {"compute": "alu", "flops": N * fft, "bytes": 3 * N * Nt * cs}
    if kind == "trapz":
        return {"compute": "alu", "flops": 0.0, "bytes": 3 * N * Nt * cs}
    return {"compute": "alu", "flops": 0.0, "bytes": 0.0}


def read_traffic(kind: str, workload: str, prec: str):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if it
    was taken on the current kernel sources (else None)."""
    import hashlib
    src = os.path.join(ROOT, "paper_1708_05324_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(src, "*"))):
        h.update(open(f, "rb").read())
    sha = h.hexdigest()[:16]
    path = os.path.join(ROOT, "profiles", f"counters_{kind}_{workload}_{prec}.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_sha = re.search(r"kernel_sources_sha:\s*([0-9a-f]+)", text)
    m_b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not (m_sha and m_b) or m_sha.group(1) != sha:
        return None
    return float(m_b.group(1))


def run_gpu(prec: str, w, steps: int, warmup: int, latency_solves: int, profile: bool, make_plan=None,
            repeats: int = 5, chain: bool = True):
    """Time `repeats` windows of `steps` large steps each (no per-kernel events
    inside them) and report the median window.  With `profile`, the warm-up
    times every kernel kind (per-kernel breakdown), and one more window of
    `steps` large steps after the timed ones brackets each launch of the
    dominant kind with HIP events on the plan's stream (roofline).  chain: each
    propagation starts from the previous one's output (else from the launch
    field, for workloads whose field grows without bound, like a random complex
    coupling tensor)."""
    import torch
    from paper_1708_05324_amd import gmmpa
    plan = (make_plan(prec) if make_plan else
            gmmpa.plan_from_workload(w, precision=prec, tol=TOL[prec], max_iter=30))
    rank = plan.rank()
    dtype = torch.complex128 if prec == "fp64" else torch.complex64
    A0 = torch.from_numpy(w.A0).to(device="cuda", dtype=dtype)
    A = A0
    Ls = w.M * w.dz
    breakdown, dominant = None, None
    if warmup > 0:                    # first large step: code loading, allocation, cold caches
        A = plan.propagate(A, Ls, w.dz, w.M).field
    if warmup > 1:                    # rest of the warm-up with every kernel kind timed: per-kernel breakdown
        if profile:
            plan.profile(True)
        wres = plan.propagate(A if chain else A0, (warmup - 1) * Ls, w.dz, w.M)
        A = wres.field
        if profile:
            breakdown = {k: (v[0] / wres.stats["large_steps"], v[1]) for k, v in plan.profile_read().items()}
            dominant = max(breakdown, key=lambda k: breakdown[k][0])
        plan.profile(False)
    windows = []
    for _ in range(max(1, repeats)):  # timed windows: only propagate between the two synchronisations
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = plan.propagate(A if chain else A0, steps * Ls, w.dz, w.M)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        A = res.field
        st = res.stats
        windows.append({"seconds": t1 - t0, "stats": st})
    order = sorted(range(len(windows)), key=lambda i: windows[i]["seconds"])
    med = windows[order[len(order) // 2]]
    prof, prof_window = None, None
    if dominant:                      # roofline window: events around each launch of the dominant kind
        plan.profile([dominant])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pres = plan.propagate(A if chain else A0, steps * Ls, w.dz, w.M)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        prof = {dominant: plan.profile_read()[dominant]}
        prof_window = {"seconds": t1 - t0, "stats": pres.stats}
        plan.profile(False)
        A = pres.field
    lat = []
    solve_L = 11 * Ls                      # one "solve": 110 small steps (about 1 mm)
    B = A
    for _ in range(latency_solves):
        torch.cuda.synchronize()
        a = time.perf_counter()
        B = plan.propagate(B, solve_L, w.dz, w.M).field
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - a) * 1e3)
    st = med["stats"]
    sec = med["seconds"]
    out = {
        "seconds": sec,
        "small_steps_per_s": st["small_steps"] / sec,
        "ms_per_large_step": sec / st["large_steps"] * 1e3,
        "iterations_per_large_step": st["iterations"] / st["large_steps"],
        "evaluations_per_s": st["evaluations"] / sec,
        "nonconverged_steps": st["nonconverged_steps"],
        "windows_small_steps_per_s": [round(x["stats"]["small_steps"] / x["seconds"], 1) for x in windows],
        "stats": st,
        "prof": prof,
        "prof_stats": prof_window["stats"] if prof_window else None,
        "prof_window_small_steps_per_s": (prof_window["stats"]["small_steps"] / prof_window["seconds"]
                                          if prof_window else None),
        "breakdown": breakdown,
        "rank": rank,
        "device_bytes": plan.device_bytes(),
    }
    if lat:
        lat.sort()
        out["latency_ms_p50"] = lat[len(lat) // 2]
        out["latency_ms_p99"] = lat[min(len(lat) - 1, int(math.ceil(0.99 * len(lat))) - 1)]
        out["latency_small_steps"] = int(round(solve_L / w.dz))
        out["latency_solves"] = len(lat)
    plan.close()
    return out


GOLDEN = os.path.join(ROOT, "tests", "golden", "metric_22_large_steps.npz")


def field_error_vs_oracle(prec: str, w, make_plan=None):
    """Max field error, normalised by the peak, after the oracle golden's
    propagation (22 large steps of the metric workload, about 2 mm) run in the
    benchmark's own mode (tolerance per precision), against the FP64 oracle's
    stored result (tests/golden, written by a script that calls only the oracle)."""
    import numpy as np
    import torch
    from paper_1708_05324_amd import gmmpa
    if not os.path.exists(GOLDEN):
        return None
    g = np.load(GOLDEN)
    plan = (make_plan(prec) if make_plan else
            gmmpa.plan_from_workload(w, precision=prec, tol=TOL[prec], max_iter=30))
    dtype = torch.complex128 if prec == "fp64" else torch.complex64
    A = torch.from_numpy(w.A0).to(device="cuda", dtype=dtype)
    res = plan.propagate(A, float(g["L"]), float(g["dz"]), int(g["M"]))
    got = res.field.cpu().numpy()
    plan.close()
    ref = g["A_ref"]
    return {"field_error": float(np.max(np.abs(got - ref)) / np.max(np.abs(ref))),
            "length_small_steps": int(res.stats["small_steps"]), "reference": "FP64 oracle, tol 1e-12",
            "iterations": int(res.stats["iterations"])}


def run_rk4ip(prec: str, w, n_steps: int, h: float | None = None) -> float:
    """Steps of h per second (h = the workload's dz unless given) of the serial
    RK4IP baseline over n_steps steps."""
    import torch
    from paper_1708_05324_amd import gmmpa
    h = w.dz if h is None else h
    plan = gmmpa.plan_from_workload(w, precision=prec)
    A = torch.from_numpy(w.A0).to(device="cuda", dtype=torch.complex128 if prec == "fp64" else torch.complex64)
    A = plan.propagate_rk4ip(A, 4 * h, h).field
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = plan.propagate_rk4ip(A, n_steps * h, h)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    plan.close()
    return res.stats["small_steps"] / sec


def sweep_accuracy(w, n_steps: int = 40) -> dict:
    """FP64 field errors after n_steps small steps (length n_steps dz) against
    RK4IP at dz/4: the MPA (converged to 1e-12; M = 1, 10, 40) and RK4IP at dz;
    then the largest RK4IP step h = L/n whose error does not exceed the MPA's
    (the step at which the two reach the same accuracy)."""
    import numpy as np
    import torch
    from paper_1708_05324_amd import gmmpa
    L = n_steps * w.dz
    plan = gmmpa.plan_from_workload(w, precision="fp64", tol=1e-12, max_iter=40)
    A0 = torch.from_numpy(w.A0).to(device="cuda", dtype=torch.complex128)
    ref = plan.propagate_rk4ip(A0, L, w.dz / 4).field.cpu().numpy()

    def err(x):
        return float(np.max(np.abs(x - ref)) / np.max(np.abs(ref)))
    out = {"length_small_steps": n_steps, "reference": "RK4IP at dz/4",
           "rk4ip": err(plan.propagate_rk4ip(A0, L, w.dz).field.cpu().numpy())}
    for M in (1, 10, 40):
        out[f"mpa_M{M}"] = err(plan.propagate(A0, L, w.dz, M).field.cpu().numpy())
    target = out["mpa_M10"]
    best = 1
    for n in range(n_steps, 0, -1):            # coarser and coarser RK4IP steps
        e = err(plan.propagate_rk4ip(A0, L, L / n).field.cpu().numpy())
        if e <= target:
            best, best_err = n, e
        else:
            break
    out["rk4ip_equal_accuracy"] = {"steps": best, "h_over_dz": round(n_steps / best, 3), "error": best_err}
    plan.close()
    return out


def roofline(prof: dict, stats: dict, N: int, Nt: int, prec: str, workload: str, rank: int = 0,
             route: str = "packed"):
    """Roofline entry of the kernel kind with the largest total time.  The bound
    is the ceiling that takes longer for the kernel's algorithmic work: its
    flops at the compute peak (MFMA, or vector ALU for the transforms) or its
    bytes at the HBM peak; both fractions are reported."""
    kind = max(prof, key=lambda k: prof[k][0])
    total_ms, launches = prof[kind]
    evals = stats["evaluations"]          # sub-step integrands = units processed by all counted launches
    wk = work_per_eval(kind, N, Nt, prec, rank, route)
    sec = total_ms * 1e-3
    if wk["compute"] == "mfma":
        split = ("mfma_bf16x4_TFLOPs" if route != "general" and kind in ("contract", "project")
                 else "mfma_bf16x3_TFLOPs")
        cpeak = PEAKS["mfma_fp64_TFLOPs" if prec == "fp64" else split if prec == "bf16x3" else "mfma_fp32_TFLOPs"]
    else:
        cpeak = PEAKS["alu_fp64_TFLOPs" if prec == "fp64" else "alu_fp32_TFLOPs"]
    t_compute = wk["flops"] / (cpeak * 1e12)
    t_hbm = wk["bytes"] / (PEAKS["hbm_GBps"] * 1e9)
    c_ach = wk["flops"] * evals / sec / 1e12
    m_ach = wk["bytes"] * evals / sec / 1e9
    if t_compute >= t_hbm:
        bound, achieved, peak, unit = wk["compute"], c_ach, cpeak, "TFLOP/s"
    else:
        bound, achieved, peak, unit = "hbm", m_ach, PEAKS["hbm_GBps"], "GB/s"
    return {
        "kernel": kind,
        "bound": bound,
        "achieved": round(achieved, 3),
        "peak": peak,
        "unit": unit,
        "frac": round(achieved / peak, 4),
        "traffic": read_traffic(kind, workload, prec),
        "compute_frac": round(c_ach / cpeak, 4),
        "hbm_frac": round(m_ach / PEAKS["hbm_GBps"], 4),
        "avg_launch_us": round(total_ms / launches * 1e3, 2) if launches else None,
        "launches": launches,
        "units_per_launch": round(evals / launches, 3) if launches else None,
    }


def bench_batch(length_scale: float) -> dict:
    """The batched workload: one FP32 plan per shape class (modes, samples), its
    contraction launch autotuned for the batch's rows, each on its own stream;
    every propagation of a class goes into one batch of that class, and the
    rounds of all classes are queued together.  Baseline: the same plans
    propagating the same problems one after another.  The outputs of the two
    are compared bit for bit."""
    import numpy as np
    import torch
    from paper_1708_05324_amd import gmmpa, synth
    probs = synth.batch_problems(length_scale=length_scale)
    classes = sorted({p.extra["class"] for p in probs})
    plans, batches, tune = {}, {}, {}
    for cl in classes:
        w = next(p for p in probs if p.extra["class"] == cl)
        n_in = sum(1 for p in probs if p.extra["class"] == cl)
        plan = gmmpa.plan_from_workload(w, precision="fp32", tol=TOL["fp32"], max_iter=30,
                                        stream=torch.cuda.Stream())
        choice, us = plan.autotune(n_in * (w.M + 1))
        tune[f"{cl[0]}x{cl[1]}"] = {"chosen": choice, "us_per_launch": [round(x, 2) for x in us],
                                    "route": "rank-r" if plan.rank() else "packed"}
        plans[cl] = plan
        batches[cl] = gmmpa.Batch(plan, slots=n_in, M=w.M)
    order = {cl: i for i, cl in enumerate(classes)}
    inputs = [torch.from_numpy(p.A0).to(device="cuda", dtype=torch.complex64) for p in probs]
    torch.cuda.synchronize()
    small = sum(int(round(p.L / p.dz)) for p in probs)
    # warm-up: one short propagation per class through its batch and alone
    for cl in classes:
        p = next(q for q in probs if q.extra["class"] == cl)
        A = torch.from_numpy(p.A0).to(device="cuda", dtype=torch.complex64)
        torch.cuda.synchronize()
        gmmpa.run_batches([batches[cl]], [(0, A, 2 * p.M * p.dz, p.dz, -1)])
        plans[cl].propagate(A, 2 * p.M * p.dz, p.dz, p.M)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = gmmpa.run_batches([batches[cl] for cl in classes],
                            [(order[p.extra["class"]], inputs[i], p.L, p.dz, i) for i, p in enumerate(probs)])
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    seq = []
    t0 = time.perf_counter()
    for i, p in enumerate(probs):
        seq.append(plans[p.extra["class"]].propagate(inputs[i], p.L, p.dz, p.M))
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    equal = all(np.array_equal(res[i][2].cpu().numpy(), seq[i].field.cpu().numpy()) and
                res[i][1]["iterations"] == seq[i].stats["iterations"] for i in range(len(probs)))
    evals = sum(r.stats["evaluations"] for r in seq)
    out = {"metric": "batched MPA propagations: small steps/s over 64 problems of uneven modes and samples",
           "unit": "small steps/s", "value": round(small / t_batch, 1), "dtype": "f32",
           "config": {"workload": "grin_batch64", "problems": len(probs), "classes": len(classes),
                      "modes": [3, 6, 10, 15], "nt": [4096, 8192, 16384], "lengths_m": [0.1 * length_scale,
                                                                                       1.0 * length_scale],
                      "energy_nJ": [1, 200], "chirp": [-5, 5], "M": 10, "tol": TOL["fp32"]},
           "small_steps": small, "evaluations": evals, "seconds_batched": round(t_batch, 3),
           "sequential": {"small_steps_per_s": round(small / t_seq, 1), "seconds": round(t_seq, 3)},
           "speedup_vs_sequential": round(t_seq / t_batch, 3), "problems_per_s": round(len(probs) / t_batch, 2),
           "bitwise_equal_to_sequential": bool(equal), "autotune": tune,
           "batch_device_bytes": sum(b.device_bytes() for b in batches.values())}
    for b in batches.values():
        b.close()
    for pl in plans.values():
        pl.close()
    return out


def bench_serve(args) -> dict:
    """Serve the seeded Poisson stream at the offered rate, then at 0.7 times
    the capacity measured in that run (served requests per second; a second
    stream of the same draws with the arrival times stretched)."""
    from paper_1708_05324_amd import serve, synth
    reqs = synth.request_stream(count=args.requests, rate=args.rate, max_groups=args.max_groups,
                                length_scale=args.serve_length_scale)
    warm = synth.request_stream(seed=6, count=12, rate=1e4, max_groups=args.max_groups, length_scale=1e-4)
    srv = serve.Server(precision="bf16x3")
    srv.prepare(reqs)
    srv.run(warm, realtime=False)                        # code loading, first batches of several classes
    _, first = srv.run(reqs, realtime=True)
    capacity = first["served_requests_per_s"]
    slow = [synth.Request(r.idx, r.arrival * args.rate / (0.7 * capacity), r.groups, r.nt, r.L, r.A0, r.energy,
                          r.chirp) for r in reqs]
    _, second = srv.run(slow, realtime=True)
    srv.close()
    return {"metric": "served GRIN propagations: p50/p99 latency and throughput under a Poisson stream",
            "unit": "ms", "value": first["latency_ms_p50"], "dtype": "bf16x3+f32 (FP64 norm)",
            "config": {"workload": "grin_serve", "requests": args.requests, "rate_per_s": args.rate,
                       "groups": [1, args.max_groups], "modes_max": args.max_groups * (args.max_groups + 1) // 2,
                       "nt": [4096, 32768],
                       "lengths_m": [0.1 * args.serve_length_scale, 2.0 * args.serve_length_scale],
                       "energy_nJ": [1, 200], "chirp": [-5, 5], "M": 10, "slots_per_batch": srv.slots,
                       "budget_GiB": srv.budget_bytes / 2 ** 30},
            "at_offered_rate": first, "at_0.7x_capacity": dict(second, offered_rate_per_s=round(0.7 * capacity, 3))}


def bench_configs() -> dict:
    """The two small configurations run as stated.  Config 1 (3 modes, Kerr only,
    dz = 1 mm) over its full 0.5 m in FP64: the energy invariant, and the field
    against the oracle's RK4IP over the same 0.5 m at the same step.  Config 2
    (6 modes, Raman, 1 m): once at its stated dz = 2 mm (M dz gamma P0 = 3.2, far
    outside the regime L << z_NL the method needs) with the status the library
    returns, then over the full 1 m at the step rule, FP64 and FP32."""
    import numpy as np
    import torch
    from oracle import gmmnlse as O
    from paper_1708_05324_amd import gmmpa, synth

    def run(w, prec, L, dz, M, tol):
        plan = gmmpa.plan_from_workload(w, precision=prec, tol=tol, max_iter=30)
        dtype = torch.complex128 if prec == "fp64" else torch.complex64
        A = torch.from_numpy(w.A0).to(device="cuda", dtype=dtype)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        try:
            res = plan.propagate(A, L, dz, M)
            rc, st, field = res.status, res.stats, res.field.cpu().numpy()
        except gmmpa.GmmError as e:
            rc, st, field = e.code, None, None
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        plan.close()
        out = {"status": {0: "ok", 1: "not converged (max_iter reached in some large steps)",
                          -6: "diverged (non-finite relative change)"}.get(rc, str(rc)), "seconds": round(sec, 3)}
        if st:
            out.update({"large_steps": st["large_steps"], "small_steps": st["small_steps"],
                        "nonconverged_steps": st["nonconverged_steps"], "iterations": st["iterations"],
                        "small_steps_per_s": round(st["small_steps"] / sec, 1),
                        "energy_rel_change": float(st["energy_out"] / st["energy_in"] - 1.0),
                        "photon_number_rel_change": float(st["photons_out"] / st["photons_in"] - 1.0)})
        return out, field

    out = {"metric": "configurations 1 and 2 as stated", "unit": "-"}
    w1 = synth.config1()
    r1, f1 = run(w1, "fp64", w1.L, w1.dz, w1.M, TOL["fp64"])
    ref = O.rk4ip_propagate(w1.A0, O.model_from_workload(w1), w1.L, w1.dz)
    r1["field_vs_oracle_rk4ip_same_dz"] = float(np.max(np.abs(f1 - ref)) / np.max(np.abs(ref)))
    out["config1_fp64_full_0.5m"] = dict(r1, dz_m=w1.dz, L_m=w1.L, M=w1.M)
    w2s = synth.config2(dz=2e-3)
    out["config2_stated_dz_2mm"] = {p: run(w2s, p, w2s.L, w2s.dz, w2s.M, TOL[p])[0] for p in ("fp64", "fp32")}
    w2 = synth.config2()
    out["config2_rule_dz_full_1m"] = {p: dict(run(w2, p, w2.L, w2.dz, w2.M, TOL[p])[0], dz_um=round(w2.dz * 1e6, 3))
                                      for p in ("fp64", "fp32")}
    return out


def bench_full_length() -> dict:
    """The metric workload over its full 1 m (about 110 000 small steps) in FP64
    (tol 1e-12), and FP32 and BF16X3 over a range of stopping tolerances (the
    defaults first): each run's field error at 1 m against the FP64 run (whose
    first 2 mm match the oracle to 1.3e-14), and
    the conditioning at 1 m: the FP64 run again from the launch field perturbed
    by 1e-12 relative (seeded), kappa = (change at 1 m) / 1e-12."""
    import numpy as np
    import torch
    from paper_1708_05324_amd import gmmpa, synth
    w = synth.config3()

    def run(prec, A0, tol=None):
        plan = gmmpa.plan_from_workload(w, precision=prec, tol=TOL[prec] if tol is None else tol, max_iter=30)
        dtype = torch.complex128 if prec == "fp64" else torch.complex64
        A = torch.from_numpy(A0).to(device="cuda", dtype=dtype)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = plan.propagate(A, w.L, w.dz, w.M)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        plan.close()
        st = res.stats
        return res.field.cpu().numpy().astype(np.complex128), {
            "seconds": round(sec, 2), "small_steps": st["small_steps"], "small_steps_per_s": round(st["small_steps"] / sec, 1),
            "iterations_per_large_step": round(st["iterations"] / st["large_steps"], 3),
            "nonconverged_steps": st["nonconverged_steps"],
            "photon_number_rel_change": float(st["photons_out"] / st["photons_in"] - 1.0)}

    ref, r64 = run("fp64", w.A0)
    out = {"metric": "metric workload over the full 1 m: field error per precision against FP64", "unit": "-",
           "config": {"workload": "grin15_raman_nt16384", "L_m": w.L, "dz_um": round(w.dz * 1e6, 4), "M": w.M},
           "fp64": r64}
    peak = float(np.max(np.abs(ref)))
    for prec, tols in (("fp32", (1e-6, 1e-7, 3e-8)), ("bf16x3", (3e-5, 1e-5, 3e-6, 1e-6, 1e-7))):
        out[prec] = []
        for tol in tols:
            f, r = run(prec, w.A0, tol)
            r["tol"] = tol
            r["field_error_vs_fp64"] = float(np.max(np.abs(f - ref)) / peak)
            out[prec].append(r)
            print(json.dumps({prec: r}), file=sys.stderr, flush=True)
    eta = np.random.default_rng(synth.SEED_BASE + 7000).standard_normal(w.A0.shape)
    fp, _ = run("fp64", w.A0 * (1.0 + 1e-12 * eta))
    out["kappa_1m_fp64"] = float(np.max(np.abs(fp - ref)) / peak / 1e-12)
    return out


def cpu_baseline(w, min_seconds: float = 10.0, max_large_steps: int = 6):
    """The FP64 oracle on the host: large steps (M small steps each) of the same
    workload from its launch field, until at least min_seconds of work.  The
    oracle's transforms are numpy.fft (one thread); its matrix products use the
    BLAS thread pool.  `cores` is the average number of busy threads over the
    sample (process CPU time / wall time), the pool size is stated beside it."""
    from oracle import gmmnlse as O
    try:
        from threadpoolctl import threadpool_info
        pool = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        pool = os.cpu_count() or 1
    m = O.model_from_workload(w)
    A = w.A0
    n_large, iters, evals = 0, 0, 0
    c0 = time.process_time()
    t0 = time.perf_counter()
    while n_large < max_large_steps and (n_large == 0 or time.perf_counter() - t0 < min_seconds):
        A, st = O.mpa_propagate(A, m, w.M * w.dz, w.dz, w.M, tol=TOL["fp64"], max_iter=30, return_stats=True)
        n_large += 1
        iters += sum(st.iterations)
        evals += st.evaluations
    sec = time.perf_counter() - t0
    busy = (time.process_time() - c0) / sec
    return {"value": round(n_large * w.M / sec, 4), "unit": "small steps/s", "cores": max(1, int(round(busy))),
            "kind": "oracle",
            "sample": f"{n_large} large steps ({n_large * w.M} small steps of {w.dz * 1e6:.2f} um) of the same "
                      f"workload from its launch field, FP64, tol 1e-12 ({iters} iterations, {evals} evaluations) "
                      f"in {sec:.1f} s; {busy:.1f} threads busy on average (numpy.fft single-threaded, BLAS "
                      f"pool of {pool} threads for the products), {os.cpu_count()} host CPUs"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50, help="timed large steps (per window)")
    ap.add_argument("--warmup", type=int, default=4, help="untimed large steps (per-kernel breakdown taken here)")
    ap.add_argument("--precision", default="bf16x3", choices=["bf16x3", "fp32", "fp64"])
    ap.add_argument("--no-compare", action="store_true", help="skip the comparison runs in the other precisions")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--latency-solves", type=int, default=100)
    ap.add_argument("--repeats", type=int, default=5, help="timed windows of --steps large steps (median reported)")
    ap.add_argument("--no-profile", action="store_true", help="no per-kernel events in the timed region")
    ap.add_argument("--sweep-M", action="store_true",
                    help="only run the parallel-extent sweep M = 1..40 (M = 1 is the serial trapezoid) and the "
                         "serial RK4IP baseline on the 10-mode 2^14 workload with z_NL/dz = 200, and print its "
                         "own JSON line")
    ap.add_argument("--general", action="store_true",
                    help="only time the general-tensor route (complex S^K != S^R without index symmetry, as "
                         "polarised modes give) on the 15-mode 2^14 workload, 3 iterations per large step, and "
                         "print its own JSON line")
    ap.add_argument("--wide", action="store_true",
                    help="only time the wide rank-r route on 55 modes (ten Hermite-Gauss groups, rank 190) at "
                         "Nt = 2^15 and 2^14 in the chosen precision (tolerance mode), and print its own JSON line")
    ap.add_argument("--full-length", action="store_true",
                    help="only run the metric workload over its full 1 m in FP64, FP32 and BF16X3 (field errors "
                         "against FP64, conditioning probe at 1 m) and print their JSON line")
    ap.add_argument("--configs", action="store_true",
                    help="only run configurations 1 and 2 as stated (config 1 over 0.5 m in FP64 against the "
                         "oracle's RK4IP; config 2 at its stated dz = 2 mm and at the step rule over 1 m) and "
                         "print their JSON line")
    ap.add_argument("--coupling-exact", action="store_true",
                    help="only time the metric workload with a Hermitian linear coupling matrix placed in the "
                         "linear operator (per-frequency eigenbasis, mode mixing around the transforms)")
    ap.add_argument("--gain-coupling", action="store_true",
                    help="only time the metric workload with the terms of Sec. III.F on (saturating gain, "
                         "g = 2/m per mode, I_sat = 2 S_0000 E_pulse; linear coupling, a random symmetric Q of "
                         "20/m entries) and print its own JSON line")
    ap.add_argument("--batch", action="store_true",
                    help="only run the batched workload (64 GRIN propagations of 3-15 modes and 2^12-2^14 samples, "
                         "FP32, autotuned contraction): batched rounds against the same propagations one after "
                         "another, and print its own JSON line")
    ap.add_argument("--length-scale", type=float, default=0.05,
                    help="batched workload: fibre lengths are uniform in [0.1, 1] m times this factor")
    ap.add_argument("--serve", action="store_true",
                    help="only run the serving workload (seeded Poisson stream of GRIN requests of 1-55 modes and "
                         "2^12-2^15 samples, BF16X3 with the FP64 norm) at the offered rate and at 0.7x the "
                         "measured capacity, and print its own JSON line")
    ap.add_argument("--requests", type=int, default=200, help="serving: requests per stream")
    ap.add_argument("--max-groups", type=int, default=10,
                    help="serving: Hermite-Gauss groups drawn uniformly in 1..this (10 groups = 55 modes)")
    ap.add_argument("--rate", type=float, default=200.0, help="serving: offered requests per second")
    ap.add_argument("--serve-length-scale", type=float, default=0.001,
                    help="serving: lengths are uniform in [0.1, 2] m times this factor")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 256 MiB device-to-device copy three times (counter calibration)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(the sub-step split of one large step is how it would shard).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1708_05324_amd import gmmpa, synth
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(3)
    if args.sweep_M:
        w = synth.fig3_workload()
        out = {"sweep": "parallel extent M", "workload": w.name, "n_modes": w.n_modes, "nt": w.nt,
               "dz_um": round(w.dz * 1e6, 4), "precision": args.precision, "tol": TOL[args.precision], "points": []}
        for M in (1, 2, 5, 10, 20, 40):
            w.M = M
            n_large = max(4, 200 // M)            # about the same fibre length for every M
            r = run_gpu(args.precision, w, n_large, 2, 0, False, repeats=3)
            out["points"].append({"M": M, "small_steps_per_s": round(r["small_steps_per_s"], 1),
                                  "iterations_per_large_step": round(r["iterations_per_large_step"], 3),
                                  "evaluations_per_s": round(r["evaluations_per_s"], 1)})
            print(f"M={M}: {out['points'][-1]}", file=sys.stderr, flush=True)
        base = out["points"][0]["small_steps_per_s"]
        rk = run_rk4ip(args.precision, w, 200)
        out["rk4ip"] = {"small_steps_per_s": round(rk, 1), "evaluations_per_step": 4}
        acc = sweep_accuracy(w)
        out["accuracy_fp64"] = acc
        # RK4IP at the step where its FP64 error equals the MPA's: fibre length per second in units of dz
        ratio = acc["rk4ip_equal_accuracy"]["h_over_dz"]
        rk_eq = run_rk4ip(args.precision, w, max(20, int(200 / ratio)), h=ratio * w.dz) * ratio
        out["rk4ip_equal_accuracy"] = {"h_over_dz": ratio, "dz_equivalents_per_s": round(rk_eq, 1)}
        for pt in out["points"]:
            pt["speedup_vs_serial"] = round(pt["small_steps_per_s"] / base, 3)
            pt["speedup_vs_rk4ip_equal_dz"] = round(pt["small_steps_per_s"] / rk, 3)
            pt["speedup_vs_rk4ip_equal_accuracy"] = round(pt["small_steps_per_s"] / rk_eq, 3)
        print(json.dumps(out), flush=True)
        return
    if args.coupling_exact:
        w = synth.config3()
        rng = np.random.default_rng(synth.SEED_BASE + 5001)
        Qh = (rng.standard_normal((w.n_modes, w.n_modes)) + 1j * rng.standard_normal((w.n_modes, w.n_modes))) * 10.0
        Q = Qh + Qh.conj().T
        setup = []

        def make_exact(p):
            plan = gmmpa.plan_from_workload(w, precision=p, tol=TOL[p], max_iter=30)
            t0 = time.perf_counter()
            plan.set_coupling_exact(Q)
            setup.append(time.perf_counter() - t0)
            return plan
        r = run_gpu(args.precision, w, max(8, args.steps // 2), max(2, args.warmup), 0, not args.no_profile,
                    make_exact)
        out = {"metric": "MPA steps/s with linear mode coupling in the linear operator", "unit": "small steps/s",
               "value": round(r["small_steps_per_s"], 2), "dtype": DTYPE[args.precision],
               "config": {"workload": "grin15_raman_nt16384_coupling_exact", "n_modes": w.n_modes, "nt": w.nt,
                          "M": w.M, "Q": "complex Hermitian, entries of rms 20/m", "coupling_rank": r["rank"]},
               "eigen_setup_s": round(setup[0], 3),
               "iterations_per_large_step": round(r["iterations_per_large_step"], 3),
               "evaluations_per_s": round(r["evaluations_per_s"], 2),
               "ms_per_large_step": round(r["ms_per_large_step"], 4)}
        if r["breakdown"]:
            out["kernel_ms_per_large_step_warmup"] = {k: round(v[0], 4) for k, v in r["breakdown"].items()}
        print(json.dumps(out), flush=True)
        return
    if args.gain_coupling:
        w = synth.config3()
        g = np.full(w.n_modes, 2.0)
        I_sat = 2.0 * float(w.S[0, 0, 0, 0]) * float(np.sum(np.abs(w.A0) ** 2) * w.dt)
        Qr = np.random.default_rng(synth.SEED_BASE + 5000).standard_normal((w.n_modes, w.n_modes)) * 20.0
        Q = Qr + Qr.T

        def make_gain(p):
            plan = gmmpa.plan_from_workload(w, precision=p, tol=TOL[p], max_iter=30)
            plan.set_gain(g, I_sat)
            plan.set_coupling(Q)
            return plan
        r = run_gpu(args.precision, w, max(8, args.steps // 2), max(2, args.warmup), 0, not args.no_profile,
                    make_gain)
        out = {"metric": "MPA steps/s with saturating gain and linear mode coupling", "unit": "small steps/s",
               "value": round(r["small_steps_per_s"], 2), "dtype": DTYPE[args.precision],
               "config": {"workload": "grin15_raman_nt16384_gain_coupling", "n_modes": w.n_modes, "nt": w.nt,
                          "M": w.M, "gain_per_m": 2.0, "I_sat_J_per_m2": I_sat, "Q_rms_per_m": 20.0 * math.sqrt(2),
                          "coupling_rank": r["rank"]},
               "iterations_per_large_step": round(r["iterations_per_large_step"], 3),
               "evaluations_per_s": round(r["evaluations_per_s"], 2),
               "ms_per_large_step": round(r["ms_per_large_step"], 4)}
        if r["breakdown"]:
            out["kernel_ms_per_large_step_warmup"] = {k: round(v[0], 4) for k, v in r["breakdown"].items()}
        print(json.dumps(out), flush=True)
        return
    if args.wide:
        prec = "bf16x3" if args.precision == "fp64" else args.precision
        lines = {}
        for nt in (2 ** 15, 2 ** 14):
            w = synth.wide_workload(nt)
            r = run_gpu(prec, w, max(3, args.steps // 10), 2, 0, not args.no_profile, repeats=3)
            lines[f"nt{nt}"] = {"small_steps_per_s": round(r["small_steps_per_s"], 2),
                                "ms_per_large_step": round(r["ms_per_large_step"], 3),
                                "iterations_per_large_step": round(r["iterations_per_large_step"], 3),
                                "evaluations_per_s": round(r["evaluations_per_s"], 2), "rank": r["rank"],
                                "dz_um": round(w.dz * 1e6, 4), "plan_device_GiB": round(r["device_bytes"] / 2 ** 30, 3)}
            if r["breakdown"]:
                lines[f"nt{nt}"]["kernel_ms_per_large_step_warmup"] = {k: round(v[0], 4)
                                                                       for k, v in r["breakdown"].items()}
        out = {"metric": "MPA steps/s, wide rank-r route at 55 modes", "unit": "small steps/s",
               "value": lines["nt32768"]["small_steps_per_s"], "dtype": DTYPE[prec],
               "config": {"workload": "grin55_raman_nt32768", "n_modes": 55, "M": 10, "tol": TOL[prec],
                          "route": "wide rank-r (pair kernel, rocBLAS GEMMs V B and U Y', fold kernel)"},
               "by_nt": lines}
        print(json.dumps(out), flush=True)
        return
    if args.general:
        w = synth.config3()
        scale = float(w.S[0, 0, 0, 0])
        SK = synth.random_general_tensor(0, w.n_modes) * scale
        SR = synth.random_general_tensor(1, w.n_modes) * scale
        prec = args.precision

        def make(p):
            return gmmpa.Plan(w.betas, SK, w.hR, nt=w.nt, dt=w.dt, omega0=w.omega0, n2=w.n2, fR=w.fR,
                              self_steepening=w.self_steepening, precision=p, SR=SR, fixed_iters=3)
        # the random complex tensor is not conservative: the field grows along the fibre and becomes non-finite
        # within about 12 large steps (in FP64 too), so every timed run is 5 large steps from the launch field
        r = run_gpu(prec, w, 5, max(2, args.warmup), 0, not args.no_profile, make, chain=False)
        out = {"metric": "MPA steps/s, general-tensor route (complex S^K != S^R)", "unit": "small steps/s",
               "value": round(r["small_steps_per_s"], 2), "dtype": DTYPE[prec],
               "config": {"workload": "grin15_raman_nt16384_general_tensor", "n_modes": w.n_modes, "nt": w.nt,
                          "M": w.M, "iterations_per_large_step": 3, "gemm_rows": 2 * w.n_modes ** 2,
                          "gemm_k": 2 * w.n_modes * (w.n_modes + 1)},
               "evaluations_per_s": round(r["evaluations_per_s"], 2),
               "ms_per_large_step": round(r["ms_per_large_step"], 4)}
        if r["prof"]:
            out["roofline"] = roofline(r["prof"], r["stats"], w.n_modes, w.nt, prec,
                                       "grin15_raman_nt16384_general", 0, "general")
        if r["breakdown"]:
            out["kernel_ms_per_large_step_warmup"] = {k: round(v[0], 4) for k, v in r["breakdown"].items()}
        print(json.dumps(out), flush=True)
        return
    if args.serve:
        print(json.dumps(bench_serve(args)), flush=True)
        return
    if args.configs:
        print(json.dumps(bench_configs()), flush=True)
        return
    if args.full_length:
        print(json.dumps(bench_full_length()), flush=True)
        return
    if args.batch:
        print(json.dumps(bench_batch(args.length_scale)), flush=True)
        return
    if args.copy_probe:
        n = 256 * 2 ** 20 // 4
        src = torch.ones(n, device="cuda", dtype=torch.float32)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": 4 * n, "copy_probe_bytes_written": 4 * n}), flush=True)
        return
    gmmpa.load_library()
    w = synth.config3()
    N, Nt = w.n_modes, w.nt
    workload = "grin15_raman_nt16384"

    main_run = run_gpu(args.precision, w, args.steps, args.warmup, args.latency_solves, not args.no_profile,
                       repeats=args.repeats)
    main_acc = field_error_vs_oracle(args.precision, w)
    extra = {}
    if not args.no_compare:
        for other in ("bf16x3", "fp32", "fp64"):
            if other == args.precision:
                continue
            o = run_gpu(other, w, args.steps, 1, 0, False, repeats=args.repeats)
            extra[other] = {"small_steps_per_s": round(o["small_steps_per_s"], 2),
                            "evaluations_per_s": round(o["evaluations_per_s"], 2),
                            "iterations_per_large_step": round(o["iterations_per_large_step"], 3),
                            "ms_per_large_step": round(o["ms_per_large_step"], 4), "tol": TOL[other],
                            "accuracy_2mm": field_error_vs_oracle(other, w)}
        # the same stopping rule in both complex64 precisions: FP32 at the BF16X3 tolerance
        if args.precision == "bf16x3":
            t_b = TOL["bf16x3"]
            o = run_gpu("fp32", w, args.steps, 1, 0, False, repeats=args.repeats,
                        make_plan=lambda p: gmmpa.plan_from_workload(w, precision=p, tol=t_b, max_iter=30))
            extra["fp32_at_bf16x3_tol"] = {"small_steps_per_s": round(o["small_steps_per_s"], 2),
                                           "evaluations_per_s": round(o["evaluations_per_s"], 2),
                                           "iterations_per_large_step": round(o["iterations_per_large_step"], 3),
                                           "ms_per_large_step": round(o["ms_per_large_step"], 4), "tol": t_b,
                                           "accuracy_2mm": field_error_vs_oracle(
                                               "fp32", w, make_plan=lambda p: gmmpa.plan_from_workload(
                                                   w, precision=p, tol=t_b, max_iter=30))}
        # the packed contraction route (the full-rank form an Eq. (2) tensor of a mode solver would take)
        o = run_gpu(args.precision, w, args.steps, 1, 0, False, repeats=args.repeats,
                    make_plan=lambda p: gmmpa.plan_from_workload(w, precision=p, tol=TOL[p], max_iter=30,
                                                                 factor_policy=1))
        extra[f"{args.precision}_packed_route"] = {
            "small_steps_per_s": round(o["small_steps_per_s"], 2),
            "evaluations_per_s": round(o["evaluations_per_s"], 2),
            "iterations_per_large_step": round(o["iterations_per_large_step"], 3),
            "ms_per_large_step": round(o["ms_per_large_step"], 4), "tol": TOL[args.precision],
            "route": "packed matrix S^ (120 x 120), no rank factor"}
    line = {
        "metric": "MPA steps/s at N=15 modes, Nt=2^14 (BF16/FP32 vs FP64); p50/p99 solve latency",
        "value": round(main_run["small_steps_per_s"], 2),
        "unit": "small steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_run["ms_per_large_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.precision],
        "data": "synthetic",
        "config": {"workload": workload, "n_modes": N, "nt": Nt, "window_ps": round(Nt * w.dt * 1e12, 3),
                   "M": w.M, "coupling_rank": main_run["rank"], "dz_um": round(w.dz * 1e6, 4), "tol": TOL[args.precision], "fR": w.fR,
                   "self_steepening": w.self_steepening, "step": "one MPA large step (M small steps)",
                   "parallelism": "single GPU"},
        "iterations_per_large_step": round(main_run["iterations_per_large_step"], 3),
        "evaluations_per_s": round(main_run["evaluations_per_s"], 2),
        "timed_windows_small_steps_per_s": main_run["windows_small_steps_per_s"],
        "accuracy_2mm": main_acc,
        "latency_ms_p50": round(main_run.get("latency_ms_p50", float("nan")), 3),
        "latency_ms_p99": round(main_run.get("latency_ms_p99", float("nan")), 3),
        "latency_solve": (f"{main_run.get('latency_solves')} back-to-back solves of "
                          f"{main_run.get('latency_small_steps')} small steps on one warm plan (solve latency, "
                          f"not a served latency)"),
        "compare": extra,
    }
    if main_run["prof"]:
        line["roofline"] = roofline(main_run["prof"], main_run["prof_stats"], N, Nt, args.precision, workload,
                                    main_run["rank"])
        line["roofline"]["window_small_steps_per_s"] = round(main_run["prof_window_small_steps_per_s"], 1)
    if main_run["breakdown"]:
        line["kernel_ms_per_large_step_warmup"] = {k: round(v[0], 4) for k, v in main_run["breakdown"].items()}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
