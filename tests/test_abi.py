"""The C ABI library: it loads, exports every declared entry point, and its host
validation rejects bad input with the documented codes (no GPU work involved:
every case below fails before the library touches a device)."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_1708_05324_amd import gmmpa, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(gmmpa.LIB_PATH):
        from paper_1708_05324_amd import build
        build.build(verbose=False)
    return gmmpa.load_library()


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "gmmpa.h")).read()
    return sorted(set(re.findall(r"\b(gmm_[a-z0-9_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert declared_symbols() == sorted(gmmpa.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    for name in declared_symbols():
        assert hasattr(lib, name), name


def test_struct_layouts_match_the_header(tmp_path):
    """Sizes and field offsets of the ctypes mirrors equal what a C compiler
    makes of include/gmmpa.h."""
    src = tmp_path / "layout.c"
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "gmmpa.h"', "int main(void) {"]
    for st in (gmmpa.gmm_params, gmmpa.gmm_stats):
        lines.append(f'printf("{st.__name__} %zu\\n", sizeof({st.__name__}));')
        for f, _ in st._fields_:
            lines.append(f'printf("{st.__name__}.{f} %zu\\n", offsetof({st.__name__}, {f}));')
    lines += ["return 0;", "}"]
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                  check=True).stdout.splitlines())
    for st in (gmmpa.gmm_params, gmmpa.gmm_stats):
        assert int(out[st.__name__]) == ctypes.sizeof(st)
        for f, _ in st._fields_:
            assert int(out[f"{st.__name__}.{f}"]) == getattr(st, f).offset, f


def _params(**kw):
    base = dict(n_modes=3, nt=256, n_beta=3, dt=10e-15, omega0=synth.GrinFiber().omega0, n2=2.3e-20,
                fR=0.0, self_steepening=0, precision=0, tol=1e-12, max_iter=20, fixed_iters=0, factor_policy=0,
                s_complex=0)
    base.update(kw)
    return gmmpa.gmm_params(**base)


def _create(lib, prm, S=None, hR=None, SR=None, betas=None):
    N = prm.n_modes
    S = synth.random_symmetric_tensor(0, N) if S is None else S
    betas = np.zeros((N, prm.n_beta)) if betas is None else betas
    h = ctypes.c_void_p()
    rc = lib.gmm_plan_create(ctypes.byref(h), ctypes.byref(prm), gmmpa._host_ptr(np.ascontiguousarray(betas)),
                             gmmpa._host_ptr(np.ascontiguousarray(S)),
                             None if SR is None else gmmpa._host_ptr(np.ascontiguousarray(SR)),
                             None if hR is None else gmmpa._host_ptr(np.ascontiguousarray(hR)), None)
    return rc, h


@pytest.mark.parametrize("kw,code", [
    (dict(nt=100), gmmpa.GMM_ERR_ARG),                      # not a power of two
    (dict(nt=128), gmmpa.GMM_ERR_ARG),                      # below 2^8
    (dict(nt=2 ** 16), gmmpa.GMM_ERR_UNSUPPORTED),          # above 2^15
    (dict(nt=2 ** 15, precision=0), gmmpa.GMM_ERR_UNSUPPORTED),   # FP64 stops at 2^14
    (dict(precision=7), gmmpa.GMM_ERR_ARG),
    (dict(n_modes=0), gmmpa.GMM_ERR_ARG),
    (dict(dt=0.0), gmmpa.GMM_ERR_ARG),
    (dict(fR=1.5), gmmpa.GMM_ERR_ARG),
    (dict(max_iter=0), gmmpa.GMM_ERR_ARG),
    (dict(factor_policy=3), gmmpa.GMM_ERR_ARG),
    (dict(s_complex=2), gmmpa.GMM_ERR_ARG),
    (dict(fR=0.18), gmmpa.GMM_ERR_ARG),                     # Raman without h_R
    (dict(self_steepening=1, dt=0.5e-15), gmmpa.GMM_ERR_ARG),   # 1 + w/w0 <= 0 on the grid
    (dict(n_modes=23, nt=256), gmmpa.GMM_ERR_UNSUPPORTED),  # beyond 256 packed rows
    (dict(n_modes=16, precision=2), gmmpa.GMM_ERR_UNSUPPORTED),   # BF16 split: up to 15 modes
])
def test_invalid_plans_are_rejected(lib, kw, code):
    rc, h = _create(lib, _params(**kw))
    assert rc == code
    assert h.value is None
    assert lib.gmm_last_error().decode() != ""


def test_packed_route_rejects_tensors_without_its_symmetries(lib):
    """factor_policy 1 insists on the packed matrix: a tensor without
    S_plmn = S_plnm, or with S^R != S^K, is reported (no GPU work involved)."""
    S = synth.random_symmetric_tensor(1, 3)
    S[0, 1, 2, 0] += 1.0                                     # breaks S_plmn = S_plnm
    rc, _ = _create(lib, _params(factor_policy=1), S=S)
    assert rc == gmmpa.GMM_ERR_TENSOR
    S = synth.random_symmetric_tensor(1, 3)
    rc, _ = _create(lib, _params(factor_policy=1), S=S, SR=2.0 * S)
    assert rc == gmmpa.GMM_ERR_TENSOR


def test_null_arguments(lib):
    assert lib.gmm_propagate(None, None, 1.0, 1.0, 1, None, None) == gmmpa.GMM_ERR_ARG
    assert lib.gmm_propagate_rk4ip(None, None, 1.0, 1.0, None, None) == gmmpa.GMM_ERR_ARG
    assert lib.gmm_plan_set_gain(None, None, 1.0) == gmmpa.GMM_ERR_ARG
    assert lib.gmm_plan_set_coupling(None, None, 0) == gmmpa.GMM_ERR_ARG
    assert lib.gmm_plan_set_coupling_exact(None, None, 0) == gmmpa.GMM_ERR_ARG
    assert lib.gmm_nonlinear(None, None, 1, None) == gmmpa.GMM_ERR_ARG
    assert lib.gmm_plan_destroy(None) == 0
    assert lib.gmm_plan_device_bytes(None) == 0
    assert lib.gmm_plan_rank(None) == 0
