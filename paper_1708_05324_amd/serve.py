"""Serving loop: continuous batching of GRIN propagation requests on one GPU.

Requests arrive over time (see synth.request_stream).  Each belongs to a shape
class (Hermite-Gauss groups 1..10, so 1 to 55 modes; samples); a class is served by batches
(gmm_batch_*, one plan and one HIP stream each) of a few slots.  Admission is
by device-memory footprint: a request whose class has a free slot is admitted
at once; otherwise a new batch of its class is created if the bytes it needs
fit the budget next to the batches alive, after idle batches of other
classes are released; otherwise it waits.  Every round queues one MPA
iteration of every running propagation of every batch before waiting for any,
so work of different classes overlaps on the device, and requests admitted
while others run join them at the next round.  Fields stay on the device: the
launch field is copied in at admission, the result is a device tensor.

The server is host-side scheduling only; every step of a propagation runs in
the library's kernels.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time
from dataclasses import dataclass, field

import numpy as np

from . import gmmpa, synth

TOL = {"fp64": 1e-12, "fp32": 1e-6, "bf16x3": 1e-5}


def step_for(req, template) -> float:
    """dz = min(z_NL/200, z_IM/5) from the request's peak power (all of it in the
    fundamental mode, the conservative choice) and the class's largest
    propagation-constant offset."""
    P0 = float(np.max(np.sum(np.abs(req.A0) ** 2, axis=0)))
    return synth.step_rule(template.extra["gamma0000"] * P0, float(np.max(np.abs(template.betas[:, 0]))))


@dataclass
class _Engine:
    cls: tuple
    plan: gmmpa.Plan
    batch: gmmpa.Batch
    stream: object
    slots: int
    bytes: int
    running: int = 0
    last_used: float = 0.0


@dataclass
class Served:
    """What the server reports for one request."""
    idx: int
    arrival: float
    admitted: float
    completed: float
    status: int
    stats: dict
    field: object = None

    @property
    def latency(self) -> float:
        return self.completed - self.arrival


@dataclass
class Server:
    precision: str = "bf16x3"
    budget_bytes: int = 64 << 30
    slots: int = 4
    M: int = 10
    keep_fields: bool = False
    templates: dict = field(default_factory=dict)
    engines: list = field(default_factory=list)
    bytes_per_class: dict = field(default_factory=dict)
    peak_bytes: int = 0
    peak_engines: int = 0

    def template(self, cls):
        """Fibre data of a class: GRIN modes of `groups` groups, Nt samples of
        2.441 fs (the coupling tensor is computed once per group count)."""
        if cls not in self.templates:
            groups, nt = cls
            same = next((w for (g, _), w in self.templates.items() if g == groups), None)
            if same is None:
                w = synth.grin_workload(5, groups, nt, synth.DT_FINE, "gaussian", 200e-15, peak_power=1.0,
                                        fR=0.18, self_steepening=1, M=self.M, L=1.0, dz=1.0,
                                        name=f"serve_g{groups}_nt{nt}")
            else:
                w = dataclasses.replace(same, nt=nt, hR=synth.raman_hR(nt, synth.DT_FINE),
                                        A0=np.zeros((same.n_modes, nt), np.complex128),
                                        name=f"serve_g{groups}_nt{nt}")
            self.templates[cls] = w
        return self.templates[cls]

    def prepare(self, requests):
        """Build the fibre data of every class the requests use (host work kept
        out of the served time)."""
        for r in requests:
            self.template((r.groups, r.nt))

    def _alive_bytes(self):
        return sum(e.bytes for e in self.engines)

    def _estimate(self, cls) -> int:
        if cls in self.bytes_per_class:
            return self.bytes_per_class[cls]
        # per slot: psi_0, I_0, M iterates, M + 1 phase rows and M + 1 work rows of N Nt complex values (single
        # precision: and the FP64 factor that ends a large step, two more such rows).  Per row
        # (sub-step of a round): at most 512 Nt bytes of pair rows and 256 Nt of rank-r rows on the routes up to
        # 15 modes, 64 MiB for the plan's constants; on the wide rank-r route (more modes) 4 (Np + 2 RQ) Nt bytes
        # (pair rows / C, Y', Y; RQ = the rank G (2 G - 1) rounded up to 16) and 256 MiB for the constants and
        # the GEMM library's workspace
        groups, nt = cls
        N = synth.n_modes_for_groups(groups)
        c = 16 if self.precision == "fp64" else 8
        rows = self.slots * (self.M + 1)
        fields = self.slots * (3 * self.M + 4 + (0 if c == 16 else 2)) * N * nt * c
        if N <= 15:
            return int(fields + rows * (512 + 256) * nt + (64 << 20))
        Np, rq = N * (N + 1) // 2, -(-groups * (2 * groups - 1) // 16) * 16
        return int(fields + rows * 4 * (Np + 2 * rq) * nt + (256 << 20))

    def _new_engine(self, cls):
        import torch
        stream = torch.cuda.Stream()
        w = self.template(cls)
        plan = gmmpa.plan_from_workload(w, precision=self.precision, tol=TOL[self.precision], max_iter=30,
                                        stream=stream)
        batch = gmmpa.Batch(plan, slots=self.slots, M=self.M)
        e = _Engine(cls, plan, batch, stream, self.slots, plan.device_bytes() + batch.device_bytes())
        self.bytes_per_class[cls] = e.bytes
        self.engines.append(e)
        self.peak_bytes = max(self.peak_bytes, self._alive_bytes())
        self.peak_engines = max(self.peak_engines, len(self.engines))
        return e

    def _release_idle(self, need: int, keep_cls) -> bool:
        """Release idle batches (least recently used first) until `need` more bytes fit."""
        idle = sorted((e for e in self.engines if e.running == 0 and e.cls != keep_cls), key=lambda e: e.last_used)
        for e in idle:
            if self._alive_bytes() + need <= self.budget_bytes:
                break
            e.batch.close()
            e.plan.close()
            self.engines.remove(e)
        return self._alive_bytes() + need <= self.budget_bytes

    def _admit(self, req, now):
        """Admit one request if its class has a free slot or a new batch fits; returns the engine or None."""
        import torch
        cls = (req.groups, req.nt)
        eng = next((e for e in self.engines if e.cls == cls and e.running < e.slots), None)
        if eng is None:
            need = self._estimate(cls)
            if self._alive_bytes() + need > self.budget_bytes and not self._release_idle(need, cls):
                return None
            eng = self._new_engine(cls)
        dt = torch.complex128 if self.precision == "fp64" else torch.complex64
        with torch.cuda.stream(eng.stream):           # copy in on the batch's stream: ordered before its use
            A0 = torch.from_numpy(req.A0).to(device="cuda", dtype=dt)
        slot = eng.batch.submit(A0, req.L, step_for(req, self.template(cls)), req.idx)
        if slot is None:
            return None
        eng.running += 1
        eng.last_used = now
        return eng

    def run(self, requests, realtime: bool = True, max_seconds: float = 600.0) -> dict:
        """Serve the requests (arrival times relative to the start); returns
        {idx: Served} and a summary."""
        by_idx = {r.idx: r for r in requests}
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        waiting = collections.deque()
        admitted_at = {}
        out = {}
        t0 = time.perf_counter()
        rounds = 0
        while pending or waiting or any(e.running for e in self.engines):
            now = time.perf_counter() - t0
            if now > max_seconds:
                raise RuntimeError("serving did not finish within max_seconds")
            while pending and (not realtime or pending[0].arrival <= now):
                waiting.append(pending.popleft())
            for _ in range(len(waiting)):              # admit what fits, keep the rest in arrival order
                req = waiting.popleft()
                if self._admit(req, now) is None:
                    waiting.append(req)
                else:
                    admitted_at[req.idx] = now
            active = [e for e in self.engines if e.running]
            if not active:
                if waiting and not pending:
                    raise RuntimeError("a request does not fit the memory budget")
                if pending:
                    time.sleep(max(0.0, min(pending[0].arrival - (time.perf_counter() - t0), 0.01)))
                continue
            for e in active:
                e.batch.launch()
            rounds += 1
            for e in active:
                running, done = e.batch.wait()
                e.running = running
                t_done = time.perf_counter() - t0
                for tag, rc, st, fld in done:
                    req = by_idx[tag]
                    out[tag] = Served(tag, req.arrival, admitted_at[tag], t_done, rc, st,
                                      fld if self.keep_fields else None)
        makespan = time.perf_counter() - t0
        return out, self._summary(requests, out, makespan, rounds)

    def _summary(self, requests, out, makespan, rounds):
        lat = np.array(sorted(s.latency for s in out.values()))
        waitq = np.array([s.admitted - s.arrival for s in out.values()])
        steps = sum(s.stats["small_steps"] for s in out.values())
        span = max(r.arrival for r in requests) - min(r.arrival for r in requests)
        pct = lambda q: float(lat[min(len(lat) - 1, int(math.ceil(q * len(lat))) - 1)])  # noqa: E731
        return {"requests": len(out), "makespan_s": round(makespan, 4), "rounds": rounds,
                "served_requests_per_s": round(len(out) / makespan, 3),
                "served_small_steps_per_s": round(steps / makespan, 1),
                "offered_requests_per_s": round((len(requests) - 1) / span, 3) if span > 0 else None,
                "latency_ms_p50": round(1e3 * pct(0.50), 3), "latency_ms_p90": round(1e3 * pct(0.90), 3),
                "latency_ms_p99": round(1e3 * pct(0.99), 3), "latency_ms_max": round(1e3 * float(lat[-1]), 3),
                "queue_wait_ms_mean": round(1e3 * float(np.mean(waitq)), 3),
                "small_steps": steps, "not_ok": sum(1 for s in out.values() if s.status != gmmpa.GMM_OK),
                "peak_device_bytes": self.peak_bytes, "peak_batches": self.peak_engines}

    def close(self):
        for e in self.engines:
            e.batch.close()
            e.plan.close()
        self.engines.clear()

