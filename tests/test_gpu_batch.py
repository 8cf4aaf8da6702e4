"""Batched propagations with continuous admission (gmm_batch_*) against
gmm_propagate through the C ABI: every propagation of a batch, admitted while
others run and of its own length, step and launch field, gives bit for bit the
field and statistics of the same propagation run alone on the same plan (the
kernels compute each slot's rows exactly as the single-propagation path does).
Several batches on their own streams run together the same way."""
import numpy as np
import pytest

from paper_1708_05324_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1708_05324_amd import gmmpa
    gmmpa.load_library()
    return torch


def problems(w, count, seed):
    """Launch fields of different energy and chirp, lengths of 1 to 4.5 large
    steps (ragged last steps) and steps between 0.7 and 1.3 dz."""
    rng = np.random.default_rng(synth.SEED_BASE + 8000 + seed)
    t = synth.time_grid(w.nt, w.dt)
    out = []
    for i in range(count):
        scale = np.sqrt(rng.uniform(0.3, 1.5))
        chirp = np.exp(1j * rng.uniform(-2, 2) * (t / (20 * w.dt * 50)) ** 2)
        A0 = w.A0 * scale * chirp[None, :]
        dz = w.dz * rng.uniform(0.7, 1.3)
        L = dz * int(rng.integers(w.M, 4 * w.M + 6))
        out.append((A0, L, dz))
    return out


def to_dev(torch, x, prec):
    dt = torch.complex128 if prec == "fp64" else torch.complex64
    return torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda", dtype=dt)


def solo(plan, torch, prec, A0, L, dz, M):
    r = plan.propagate(to_dev(torch, A0, prec), L, dz, M)
    return r.field.cpu().numpy(), r.stats, r.status


KEYS = ("large_steps", "small_steps", "iterations", "evaluations", "max_iters_seen", "nonconverged_steps",
        "last_eps", "dz_used", "energy_in", "energy_out", "photons_in", "photons_out")


@pytest.mark.parametrize("prec,fixed,tuned", [("fp64", 0, False), ("fp32", 0, False), ("bf16x3", 0, False),
                                              ("fp32", 3, False), ("fp32", 0, True)])
def test_batch_equals_solo_bitwise(torch_gpu, prec, fixed, tuned):
    from paper_1708_05324_amd import gmmpa
    torch = torch_gpu
    w = synth.config2()                                 # 6 modes, 2^13 samples, packed route, Raman + shock
    tol = {"fp64": 1e-12, "fp32": 1e-6, "bf16x3": 1e-5}[prec]
    plan = gmmpa.plan_from_workload(w, precision=prec, tol=tol, max_iter=30, fixed_iters=fixed)
    if tuned:                                           # the tuned launch is the plan's: batch and solo share it
        choice, us = plan.autotune(3 * (w.M + 1))
        print(f"[autotune] chose {choice} of {[round(x, 1) for x in us]} us", flush=True)
    jobs = problems(w, 7, 0)
    batch = gmmpa.Batch(plan, slots=3, M=w.M)           # 7 propagations through 3 slots: admission mid-flight
    inputs = [(0, to_dev(torch, A0, prec), L, dz, i) for i, (A0, L, dz) in enumerate(jobs)]
    torch.cuda.synchronize()
    res = gmmpa.run_batches([batch], inputs)
    assert sorted(res) == list(range(len(jobs)))
    for i, (A0, L, dz) in enumerate(jobs):
        rc, st, out = res[i]
        ref, rst, rrc = solo(plan, torch, prec, A0, L, dz, w.M)
        got = out.cpu().numpy()
        print(f"[{prec} fixed={fixed} job {i}] steps {st['small_steps']} iters {st['iterations']} "
              f"max|diff| {np.max(np.abs(got - ref)):.3e}", flush=True)
        assert rc == rrc
        assert np.array_equal(got, ref)
        for k in KEYS:
            assert st[k] == rst[k], k
    batch.close()
    plan.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_batch_equals_solo_bitwise_rank_route(torch_gpu, prec):
    """The 15-mode rank-45 route at 2^13 samples (Y = V B, overlap-save
    convolution of the 45 rows, column-owner contraction): batch and single
    propagation agree bit for bit, and the single propagation agrees with the
    oracle over one large step."""
    from oracle import gmmnlse as O
    from paper_1708_05324_amd import gmmpa
    torch = torch_gpu
    w = synth.grin_workload(3, 5, 2 ** 13, synth.DT_FINE, "gaussian", 200e-15, energy=100e-9, fR=0.18,
                            self_steepening=1, M=10, L=1.0)
    tol = {"fp32": 1e-6, "bf16x3": 1e-5}[prec]
    plan = gmmpa.plan_from_workload(w, precision=prec, tol=tol, max_iter=30)
    assert plan.rank() == 45
    ref = O.mpa_propagate(w.A0, O.model_from_workload(w), w.M * w.dz, w.dz, w.M, fixed_iters=3)
    fixed = gmmpa.plan_from_workload(w, precision=prec, fixed_iters=3)
    got = fixed.propagate(to_dev(torch, w.A0, prec), w.M * w.dz, w.dz, w.M).field.cpu().numpy()
    err = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
    print(f"[{prec} rank-45 2^13] one large step vs oracle {err:.3e}", flush=True)
    assert err < {"fp32": 1e-5, "bf16x3": 1e-4}[prec]
    fixed.close()
    jobs = problems(w, 5, 3)
    batch = gmmpa.Batch(plan, slots=2, M=w.M)
    inputs = [(0, to_dev(torch, A0, prec), L, dz, i) for i, (A0, L, dz) in enumerate(jobs)]
    torch.cuda.synchronize()
    res = gmmpa.run_batches([batch], inputs)
    for i, (A0, L, dz) in enumerate(jobs):
        rc, st, out = res[i]
        refi, rst, rrc = solo(plan, torch, prec, A0, L, dz, w.M)
        assert rc == rrc
        assert np.array_equal(out.cpu().numpy(), refi), i
        for k in KEYS:
            assert st[k] == rst[k], k
    batch.close()
    plan.close()


def test_batches_on_two_streams_equal_solo(torch_gpu):
    """Two plans of different shape (3 modes / 2^10 samples, Kerr; 6 modes /
    2^13, Raman) on their own streams, their rounds queued together."""
    from paper_1708_05324_amd import gmmpa
    torch = torch_gpu
    ws = [synth.config1(), synth.config2()]
    plans = [gmmpa.plan_from_workload(w, precision="fp32", tol=1e-6, max_iter=30, stream=torch.cuda.Stream())
             for w in ws]
    batches = [gmmpa.Batch(p, slots=2, M=w.M) for p, w in zip(plans, ws)]
    jobs, meta = [], {}
    for b, w in enumerate(ws):
        for i, (A0, L, dz) in enumerate(problems(w, 4, 10 + b)):
            tag = 100 * b + i
            jobs.append((b, to_dev(torch, A0, "fp32"), L, dz, tag))
            meta[tag] = (b, A0, L, dz)
    torch.cuda.synchronize()                            # inputs written before the plan streams read them
    res = gmmpa.run_batches(batches, jobs)
    torch.cuda.synchronize()
    for tag, (b, A0, L, dz) in meta.items():
        rc, st, out = res[tag]
        with torch.cuda.stream(plans[b].stream):
            ref, rst, _ = solo(plans[b], torch, "fp32", A0, L, dz, ws[b].M)
        assert np.array_equal(out.cpu().numpy(), ref), tag
        assert st["iterations"] == rst["iterations"]
    for x in batches + plans:
        x.close()


def test_batch_slot_errors_and_divergence(torch_gpu):
    """A full batch refuses a submission (GMM_ERR_BUSY), a second launch before
    the wait is refused, and a non-finite launch field fails its own slot only
    (GMM_ERR_DIVERGED) while the other propagation completes unchanged."""
    from paper_1708_05324_amd import gmmpa
    torch = torch_gpu
    w = synth.config2()
    plan = gmmpa.plan_from_workload(w, precision="fp32", tol=1e-6, max_iter=30)
    batch = gmmpa.Batch(plan, slots=2, M=w.M)
    good = to_dev(torch, w.A0, "fp32")
    bad_np = w.A0.copy()
    bad_np[0, w.nt // 3] = np.nan
    bad = to_dev(torch, bad_np, "fp32")
    torch.cuda.synchronize()
    L = 2 * w.M * w.dz
    assert batch.submit(good, L, w.dz, 1) is not None
    assert batch.submit(bad, L, w.dz, 2) is not None
    assert batch.submit(good, L, w.dz, 3) is None               # both slots taken
    batch.launch()
    with pytest.raises(gmmpa.GmmError) as e:
        batch.launch()
    assert e.value.code == gmmpa.GMM_ERR_ARG
    results = {}
    running, done = batch.wait()
    while True:
        for tag, rc, st, out in done:
            results[tag] = (rc, out)
        if running == 0:
            break
        batch.launch()
        running, done = batch.wait()
    assert results[2][0] == gmmpa.GMM_ERR_DIVERGED
    assert results[1][0] == gmmpa.GMM_OK
    ref = plan.propagate(good, L, w.dz, w.M).field.cpu().numpy()
    assert np.array_equal(results[1][1].cpu().numpy(), ref)
    batch.close()
    plan.set_gain(np.ones(w.n_modes), float("inf"))
    with pytest.raises(gmmpa.GmmError) as e:
        gmmpa.Batch(plan, slots=1, M=w.M)
    assert e.value.code == gmmpa.GMM_ERR_UNSUPPORTED
    plan.close()


def test_autotune_candidates_match_the_oracle(torch_gpu):
    """Every contraction launch the autotuner can choose, on the FP32 rank-r
    route (15 modes) and the FP32 packed route (6 modes), evaluates the
    oracle's nonlinear operator; the autotuner times all of them and keeps one."""
    from oracle import gmmnlse as O
    from paper_1708_05324_amd import gmmpa
    torch = torch_gpu
    for groups, rank in ((5, 45), (3, 0)):
        w = synth.grin_workload(12, groups, 2 ** 11, 10e-15, "sech", 200e-15, peak_power=2e5, fR=0.18,
                                self_steepening=1, M=5, L=0.01)
        plan = gmmpa.plan_from_workload(w, precision="fp32")
        assert plan.rank() == rank
        ops = O._Ops(O.model_from_workload(w), w.nt)
        fields = [w.A0 * np.exp(0.4j * c) + 0.2 * synth.random_fields(c, w.n_modes, w.nt, scale=300.0)
                  for c in range(3)]
        At = np.stack([O.to_spectrum(a) for a in fields])
        ref = np.stack([ops.N(a) for a in At])
        dev = torch.from_numpy(At).to(device="cuda", dtype=torch.complex64)
        choice, us = plan.autotune(3)
        assert 0 <= choice < len(us) and all(x > 0 for x in us)
        for c in range(len(us)):
            plan.set_contraction(c)
            got = plan.nonlinear(dev).cpu().numpy()
            err = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
            print(f"[{w.n_modes} modes candidate {c}] {us[c]:.1f} us, operator error {err:.3e}", flush=True)
            assert err < 2e-5
        with pytest.raises(gmmpa.GmmError):
            plan.set_contraction(len(us))
        plan.close()
