"""Thin ctypes binding of libgmmpa.so (C ABI declared in include/gmmpa.h).

Argument marshalling only: every step of the propagation runs in the HIP
kernels of the library.  PyTorch provides device memory and the HIP stream.
Loading fails loudly when the library has not been built; there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgmmpa.so")

GMM_OK = 0
GMM_NOT_CONVERGED = 1
GMM_ERR_ARG = -1
GMM_ERR_NOMEM = -2
GMM_ERR_TENSOR = -3
GMM_ERR_HIP = -4
GMM_ERR_UNSUPPORTED = -5
GMM_ERR_DIVERGED = -6
GMM_ERR_BUSY = -7
GMM_FP64 = 0
GMM_FP32 = 1
GMM_BF16X3 = 2

EXPORTS = ("gmm_plan_create", "gmm_propagate", "gmm_propagate_rk4ip", "gmm_plan_set_gain",
           "gmm_plan_set_coupling", "gmm_plan_set_coupling_exact", "gmm_nonlinear", "gmm_nonlinear_noalloc",
           "gmm_plan_destroy", "gmm_last_error", "gmm_plan_device_bytes", "gmm_plan_rank", "gmm_profile_enable",
           "gmm_profile_read", "gmm_plan_autotune", "gmm_plan_set_contraction", "gmm_batch_create", "gmm_batch_submit", "gmm_batch_launch", "gmm_batch_wait",
           "gmm_batch_destroy", "gmm_batch_device_bytes")
PROFILE_KINDS = ("phase_to_time", "pairs_raman", "contract", "spectral_out", "trapz", "norm", "close", "project",
                 "gain")


class gmm_params(ctypes.Structure):
    _fields_ = [("n_modes", ctypes.c_int), ("nt", ctypes.c_int), ("n_beta", ctypes.c_int),
                ("dt", ctypes.c_double), ("omega0", ctypes.c_double), ("n2", ctypes.c_double),
                ("fR", ctypes.c_double), ("self_steepening", ctypes.c_int), ("precision", ctypes.c_int),
                ("tol", ctypes.c_double), ("max_iter", ctypes.c_int), ("fixed_iters", ctypes.c_int),
                ("factor_policy", ctypes.c_int), ("s_complex", ctypes.c_int)]


class gmm_stats(ctypes.Structure):
    _fields_ = [("large_steps", ctypes.c_int), ("small_steps", ctypes.c_int),
                ("iterations", ctypes.c_longlong), ("evaluations", ctypes.c_longlong),
                ("max_iters_seen", ctypes.c_int), ("nonconverged_steps", ctypes.c_int),
                ("last_eps", ctypes.c_double), ("dz_used", ctypes.c_double),
                ("energy_in", ctypes.c_double), ("energy_out", ctypes.c_double),
                ("photons_in", ctypes.c_double), ("photons_out", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libgmmpa.so and declare its signatures (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run `python -m paper_1708_05324_amd.build`")
    lib = ctypes.CDLL(path)
    vp, dbl, ci = ctypes.c_void_p, ctypes.c_double, ctypes.c_int
    lib.gmm_plan_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(gmm_params), vp, vp, vp, vp, vp]
    lib.gmm_plan_create.restype = ci
    lib.gmm_propagate.argtypes = [vp, vp, dbl, dbl, ci, vp, ctypes.POINTER(gmm_stats)]
    lib.gmm_propagate.restype = ci
    lib.gmm_propagate_rk4ip.argtypes = [vp, vp, dbl, dbl, vp, ctypes.POINTER(gmm_stats)]
    lib.gmm_propagate_rk4ip.restype = ci
    lib.gmm_plan_set_gain.argtypes = [vp, vp, dbl]
    lib.gmm_plan_set_gain.restype = ci
    lib.gmm_plan_set_coupling.argtypes = [vp, vp, ci]
    lib.gmm_plan_set_coupling.restype = ci
    lib.gmm_plan_set_coupling_exact.argtypes = [vp, vp, ci]
    lib.gmm_plan_set_coupling_exact.restype = ci
    lib.gmm_nonlinear.argtypes = [vp, vp, ci, vp]
    lib.gmm_nonlinear.restype = ci
    lib.gmm_nonlinear_noalloc.argtypes = [vp, vp, ci, vp]
    lib.gmm_nonlinear_noalloc.restype = ci
    lib.gmm_plan_destroy.argtypes = [vp]
    lib.gmm_plan_destroy.restype = ci
    lib.gmm_plan_autotune.argtypes = [vp, ci, ctypes.POINTER(ci), ctypes.POINTER(dbl), ci]
    lib.gmm_plan_autotune.restype = ci
    lib.gmm_plan_set_contraction.argtypes = [vp, ci]
    lib.gmm_plan_set_contraction.restype = ci
    lib.gmm_batch_create.argtypes = [ctypes.POINTER(vp), vp, ci, ci]
    lib.gmm_batch_create.restype = ci
    lib.gmm_batch_submit.argtypes = [vp, vp, dbl, dbl, vp, ctypes.c_longlong]
    lib.gmm_batch_submit.restype = ci
    lib.gmm_batch_launch.argtypes = [vp]
    lib.gmm_batch_launch.restype = ci
    lib.gmm_batch_wait.argtypes = [vp, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ci),
                                   ctypes.POINTER(gmm_stats), ci, ctypes.POINTER(ci)]
    lib.gmm_batch_wait.restype = ci
    lib.gmm_batch_destroy.argtypes = [vp]
    lib.gmm_batch_destroy.restype = ci
    lib.gmm_batch_device_bytes.argtypes = [vp]
    lib.gmm_batch_device_bytes.restype = ctypes.c_longlong
    lib.gmm_last_error.argtypes = []
    lib.gmm_last_error.restype = ctypes.c_char_p
    lib.gmm_plan_device_bytes.argtypes = [vp]
    lib.gmm_plan_device_bytes.restype = ctypes.c_longlong
    lib.gmm_plan_rank.argtypes = [vp]
    lib.gmm_plan_rank.restype = ci
    lib.gmm_profile_enable.argtypes = [vp, ci]
    lib.gmm_profile_enable.restype = ci
    lib.gmm_profile_read.argtypes = [vp, ctypes.POINTER(dbl), ctypes.POINTER(ctypes.c_longlong), ci]
    lib.gmm_profile_read.restype = ci
    _lib = lib
    return lib


class GmmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"gmmpa error {code}: {msg}")
        self.code = code


def _check(code: int, allow=(GMM_OK,)) -> int:
    if code not in allow:
        raise GmmError(code, load_library().gmm_last_error().decode())
    return code


def _host_ptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class Result:
    field: object          # torch tensor [N][Nt] on the device
    status: int
    stats: dict


class Plan:
    """A propagation plan: the inputs of Eq. (1) bound to one GPU stream.

    precision: "fp64" (complex128 fields), "fp32" (complex64 fields) or "bf16x3"
    (complex64 fields, BF16 hi/lo split contraction with FP32 accumulation).
    SK, SR: real or complex [N]*4 tensors (SR None: S^R = S^K); factor_policy
    0..3 picks the contraction route as documented in include/gmmpa.h.
    """

    def __init__(self, betas, SK, hR=None, *, nt: int, dt: float, omega0: float, n2: float, fR: float,
                 self_steepening: int = 1, precision: str = "fp64", tol: float = 1e-12, max_iter: int = 20,
                 fixed_iters: int = 0, factor_policy: int = 0, SR=None, stream=None):
        import torch
        self.lib = load_library()
        betas = np.ascontiguousarray(np.atleast_2d(np.asarray(betas, dtype=np.float64)))
        self.n_modes = betas.shape[0]
        s_complex = int(np.iscomplexobj(SK) or (SR is not None and np.iscomplexobj(SR)))
        sdt = np.complex128 if s_complex else np.float64
        SK = np.ascontiguousarray(np.asarray(SK, dtype=sdt))
        if SK.size != self.n_modes ** 4:
            raise ValueError("SK must hold N^4 values")
        SR = None if SR is None else np.ascontiguousarray(np.asarray(SR, dtype=sdt))
        if SR is not None and SR.size != self.n_modes ** 4:
            raise ValueError("SR must hold N^4 values")
        hR = None if hR is None else np.ascontiguousarray(np.asarray(hR, dtype=np.float64))
        if hR is not None and hR.size != nt:
            raise ValueError("hR must hold nt samples")
        self.precision = precision
        self.nt = nt
        self.dtype = torch.complex128 if precision == "fp64" else torch.complex64
        prec = {"fp64": GMM_FP64, "fp32": GMM_FP32, "bf16x3": GMM_BF16X3}[precision]
        self.params = gmm_params(self.n_modes, nt, betas.shape[1], dt, omega0, n2, fR, int(self_steepening),
                                 prec, tol, max_iter, fixed_iters, factor_policy, s_complex)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        handle = ctypes.c_void_p()
        self._keep = (betas, SK, SR, hR)
        _check(self.lib.gmm_plan_create(ctypes.byref(handle), ctypes.byref(self.params), _host_ptr(betas),
                                        _host_ptr(SK), _host_ptr(SR), _host_ptr(hR),
                                        ctypes.c_void_p(stream.cuda_stream)))
        self.handle = handle

    def _check_field(self, A):
        import torch
        if not isinstance(A, torch.Tensor) or not A.is_cuda:
            raise TypeError("fields must be torch tensors on the GPU")
        if A.dtype != self.dtype or not A.is_contiguous():
            raise TypeError(f"fields must be contiguous {self.dtype}")

    def propagate(self, A0, L: float, dz: float, M: int, out=None) -> Result:
        import torch
        self._check_field(A0)
        if tuple(A0.shape) != (self.n_modes, self.nt):
            raise ValueError("A0 must be [N][Nt]")
        if out is None:
            out = torch.empty_like(A0)
        st = gmm_stats()
        rc = self.lib.gmm_propagate(self.handle, ctypes.c_void_p(A0.data_ptr()), float(L), float(dz), int(M),
                                    ctypes.c_void_p(out.data_ptr()), ctypes.byref(st))
        _check(rc, allow=(GMM_OK, GMM_NOT_CONVERGED))
        return Result(out, rc, st.as_dict())

    def propagate_rk4ip(self, A0, L: float, dz: float, out=None) -> Result:
        """Serial RK4IP baseline over L with steps of dz (four dependent evaluations per step)."""
        import torch
        self._check_field(A0)
        if tuple(A0.shape) != (self.n_modes, self.nt):
            raise ValueError("A0 must be [N][Nt]")
        if out is None:
            out = torch.empty_like(A0)
        st = gmm_stats()
        rc = self.lib.gmm_propagate_rk4ip(self.handle, ctypes.c_void_p(A0.data_ptr()), float(L), float(dz),
                                          ctypes.c_void_p(out.data_ptr()), ctypes.byref(st))
        _check(rc)
        return Result(out, rc, st.as_dict())

    def set_gain(self, g=None, I_sat: float = float("inf")):
        """Saturating gain of Sec. III.F: g [N] small-signal field gain (1/m), or None to turn it off;
        I_sat the saturation fluence (J/m^2)."""
        if g is None:
            _check(self.lib.gmm_plan_set_gain(self.handle, None, float(I_sat)))
            return
        g = np.ascontiguousarray(np.asarray(g, dtype=np.float64).reshape(self.n_modes))
        self._gain = g
        _check(self.lib.gmm_plan_set_gain(self.handle, _host_ptr(g), float(I_sat)))

    def set_coupling(self, Q=None):
        """Linear mode coupling of Sec. III.F, C_p = i sum_n Q[n, p] A_n (Q [N][N] in 1/m, real or
        complex), or None to turn it off."""
        if Q is None:
            _check(self.lib.gmm_plan_set_coupling(self.handle, None, 0))
            return
        cplx_q = int(np.iscomplexobj(Q))
        Q = np.ascontiguousarray(np.asarray(Q, dtype=np.complex128 if cplx_q else np.float64)
                                 .reshape(self.n_modes, self.n_modes))
        self._coupling = Q
        _check(self.lib.gmm_plan_set_coupling(self.handle, _host_ptr(Q), cplx_q))

    def set_coupling_exact(self, Q=None):
        """The same coupling placed in the linear operator (exact for any step): Q [N][N] Hermitian,
        Q[n, p] = conj(Q[p, n]), or None to turn it off."""
        if Q is None:
            _check(self.lib.gmm_plan_set_coupling_exact(self.handle, None, 0))
            return
        cplx_q = int(np.iscomplexobj(Q))
        Q = np.ascontiguousarray(np.asarray(Q, dtype=np.complex128 if cplx_q else np.float64)
                                 .reshape(self.n_modes, self.n_modes))
        self._coupling = Q
        _check(self.lib.gmm_plan_set_coupling_exact(self.handle, _host_ptr(Q), cplx_q))

    def nonlinear(self, At, out=None):
        """Integrand factor of Eq. (MPA_eq) for spectra At [count][N][Nt]."""
        import torch
        self._check_field(At)
        if At.dim() == 2:
            At = At.unsqueeze(0)
        if tuple(At.shape[1:]) != (self.n_modes, self.nt):
            raise ValueError("At must be [count][N][Nt]")
        if out is None:
            out = torch.empty_like(At)
        _check(self.lib.gmm_nonlinear(self.handle, ctypes.c_void_p(At.data_ptr()), int(At.shape[0]),
                                      ctypes.c_void_p(out.data_ptr())))
        return out

    def nonlinear_noalloc(self, At, out):
        """The same evaluation through gmm_nonlinear_noalloc: the library
        allocates nothing (its workspace is the static device scratch); the
        caller passes the output buffer."""
        self._check_field(At)
        self._check_field(out)
        if At.dim() == 2:
            At = At.unsqueeze(0)
        if tuple(At.shape[1:]) != (self.n_modes, self.nt) or out.numel() != At.numel():
            raise ValueError("At and out must be [count][N][Nt]")
        _check(self.lib.gmm_nonlinear_noalloc(self.handle, ctypes.c_void_p(At.data_ptr()), int(At.shape[0]),
                                              ctypes.c_void_p(out.data_ptr())))
        return out

    def autotune(self, count: int):
        """Time the contraction launch candidates for `count` rows per launch and
        keep the fastest: returns (chosen index, [microseconds per launch])."""
        n = ctypes.c_int()
        us = (ctypes.c_double * 16)()
        rc = self.lib.gmm_plan_autotune(self.handle, int(count), ctypes.byref(n), us, 16)
        if rc < 0:
            _check(rc)
        return rc, [us[i] for i in range(n.value)]

    def set_contraction(self, candidate: int):
        """Use contraction launch candidate `candidate` (numbered as by autotune)."""
        _check(self.lib.gmm_plan_set_contraction(self.handle, int(candidate)))

    def profile(self, kinds=True):
        """Start (and zero) per-kernel HIP-event timing inside the library for the
        given kernel kinds (names from PROFILE_KINDS; True = all), or stop it (False)."""
        if kinds is True:
            mask = (1 << len(PROFILE_KINDS)) - 1
        elif not kinds:
            mask = 0
        else:
            mask = 0
            for k in ([kinds] if isinstance(kinds, str) else kinds):
                mask |= 1 << PROFILE_KINDS.index(k)
        _check(self.lib.gmm_profile_enable(self.handle, mask))

    def profile_read(self) -> dict:
        """{kernel kind: (total ms, launches)} for launches that did work."""
        k = len(PROFILE_KINDS)
        ms = (ctypes.c_double * k)()
        n = (ctypes.c_longlong * k)()
        _check(self.lib.gmm_profile_read(self.handle, ms, n, k))
        return {name: (ms[i], n[i]) for i, name in enumerate(PROFILE_KINDS)}

    def rank(self) -> int:
        """Rank of the coupling factor used (0: packed matrix)."""
        return int(self.lib.gmm_plan_rank(self.handle))

    def device_bytes(self) -> int:
        return int(self.lib.gmm_plan_device_bytes(self.handle))

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            self.lib.gmm_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def plan_from_workload(w, precision: str = "fp64", **kw) -> Plan:
    """Plan for a synthetic workload object (see paper_1708_05324_amd.synth)."""
    return Plan(w.betas, w.S, w.hR, nt=w.nt, dt=w.dt, omega0=w.omega0, n2=w.n2, fR=w.fR,
                self_steepening=w.self_steepening, precision=precision, **kw)


class Batch:
    """Batched propagations of one plan with continuous admission
    (gmm_batch_*): up to `slots` propagations advance together in rounds; a
    completed one frees its slot for the next submission."""

    def __init__(self, plan: Plan, slots: int, M: int):
        self.plan = plan
        self.lib = plan.lib
        self.slots = int(slots)
        self.M = int(M)
        handle = ctypes.c_void_p()
        _check(self.lib.gmm_batch_create(ctypes.byref(handle), plan.handle, self.slots, self.M))
        self.handle = handle
        self._keep = {}            # tag -> (A0, out): device buffers referenced by queued work
        self._tags = (ctypes.c_longlong * self.slots)()
        self._status = (ctypes.c_int * self.slots)()
        self._stats = (gmm_stats * self.slots)()

    def submit(self, A0, L: float, dz: float, tag: int, out=None):
        """Admit one propagation; returns (slot, out), or None when every slot is taken."""
        import torch
        self.plan._check_field(A0)
        if tuple(A0.shape) != (self.plan.n_modes, self.plan.nt):
            raise ValueError("A0 must be [N][Nt]")
        if out is None:
            out = torch.empty_like(A0)
        rc = self.lib.gmm_batch_submit(self.handle, ctypes.c_void_p(A0.data_ptr()), float(L), float(dz),
                                       ctypes.c_void_p(out.data_ptr()), int(tag))
        if rc == GMM_ERR_BUSY:
            return None
        if rc < 0:
            _check(rc)
        self._keep[int(tag)] = (A0, out)
        return rc, out

    def launch(self):
        _check(self.lib.gmm_batch_launch(self.handle))

    def wait(self):
        """Wait for the queued round: (propagations still running, completed
        [(tag, return code, stats dict, output tensor)])."""
        n = ctypes.c_int()
        rc = self.lib.gmm_batch_wait(self.handle, self._tags, self._status, self._stats, self.slots,
                                     ctypes.byref(n))
        if rc < 0:
            _check(rc)
        done = []
        for i in range(n.value):
            tag = int(self._tags[i])
            _, out = self._keep.pop(tag)
            done.append((tag, int(self._status[i]), self._stats[i].as_dict(), out))
        return rc, done

    def device_bytes(self) -> int:
        return int(self.lib.gmm_batch_device_bytes(self.handle))

    def close(self):
        if getattr(self, "handle", None) is not None:
            self.lib.gmm_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run_batches(batches, jobs):
    """Drive several batches (each with its own plan, ideally on its own stream)
    until every job is done, keeping their slots full: jobs is a list of
    (batch index, A0, L, dz, tag).  Rounds of all batches are queued before
    any is waited for, so their work overlaps on the device.  Returns
    {tag: (return code, stats, output)}."""
    pending = [list() for _ in batches]
    for j in jobs:
        pending[j[0]].append(j)
    for q in pending:
        q.reverse()
    results = {}
    active = [0] * len(batches)
    while True:
        any_work = False
        for b, batch in enumerate(batches):
            while pending[b]:
                _, A0, L, dz, tag = pending[b][-1]
                if batch.submit(A0, L, dz, tag) is None:
                    break
                pending[b].pop()
                active[b] += 1
            if active[b] > 0:
                batch.launch()
                any_work = True
        if not any_work:
            break
        for b, batch in enumerate(batches):
            if active[b] > 0:
                running, done = batch.wait()
                active[b] = running
                for tag, rc, st, out in done:
                    results[tag] = (rc, st, out)
    return results
