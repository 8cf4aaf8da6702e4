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
    (dict(factor_policy=4), gmmpa.GMM_ERR_ARG),
    (dict(factor_policy=3), gmmpa.GMM_ERR_UNSUPPORTED),     # the wide rank-r route needs complex64 fields
    (dict(s_complex=2), gmmpa.GMM_ERR_ARG),
    (dict(fR=0.18), gmmpa.GMM_ERR_ARG),                     # Raman without h_R
    (dict(self_steepening=1, dt=0.5e-15), gmmpa.GMM_ERR_ARG),   # 1 + w/w0 <= 0 on the grid
    (dict(n_modes=23, nt=256), gmmpa.GMM_ERR_UNSUPPORTED),  # FP64 beyond 256 packed rows
])
def test_invalid_plans_are_rejected(lib, kw, code):
    rc, h = _create(lib, _params(**kw))
    assert rc == code
    assert h.value is None


@pytest.mark.parametrize("prec", [1, 2])
def test_more_than_55_modes_is_rejected(lib, prec):
    rc, h = _create(lib, _params(n_modes=56, precision=prec), S=np.zeros(56 ** 4))
    assert rc == gmmpa.GMM_ERR_UNSUPPORTED
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


DRIVER_C = r"""
#include <stdio.h>
#include <string.h>
#include "gmmpa.h"
static double S[81], B[9], H[256];
static int expect(int got, int want, const char* what) {
  if (got != want) { printf("FAIL %s: %d != %d (%s)\n", what, got, want, gmm_last_error()); return 1; }
  if (got < 0 && strlen(gmm_last_error()) == 0) { printf("FAIL %s: no message\n", what); return 1; }
  return 0;
}
int main(void) {
  int bad = 0;
  gmm_params p; memset(&p, 0, sizeof p);
  p.n_modes = 3; p.nt = 256; p.n_beta = 3; p.dt = 1e-14; p.omega0 = 1.8e15; p.n2 = 2.3e-20; p.fR = 0.0;
  p.precision = GMM_FP32; p.tol = 1e-6; p.max_iter = 20;
  for (int i = 0; i < 81; ++i) S[i] = 1.0;
  gmm_plan h = 0;
  gmm_params q = p; q.nt = 100;  bad += expect(gmm_plan_create(&h, &q, B, S, 0, 0, 0), GMM_ERR_ARG, "nt");
  /* refused before the tensor is read (S holds 3^4 values only) */
  q = p; q.n_modes = 56;         bad += expect(gmm_plan_create(&h, &q, B, S, 0, 0, 0), GMM_ERR_UNSUPPORTED, "modes");
  q = p; q.n_modes = 23; q.precision = GMM_FP64;
  bad += expect(gmm_plan_create(&h, &q, B, S, 0, 0, 0), GMM_ERR_UNSUPPORTED, "fp64 modes");
  q = p; q.fR = 0.18;            bad += expect(gmm_plan_create(&h, &q, B, S, 0, 0, 0), GMM_ERR_ARG, "hR");
  q = p; q.factor_policy = 1; S[1] = 2.0;
  bad += expect(gmm_plan_create(&h, &q, B, S, 0, 0, 0), GMM_ERR_TENSOR, "symmetry");
  S[1] = 1.0;
  q = p; q.fR = 0.18; for (int i = 0; i < 256; ++i) H[i] = 0.0;
  bad += expect(gmm_plan_create(&h, &q, B, S, 0, H, 0) < 0, 1, "zero h_R or no device");
  bad += expect(gmm_plan_create(0, &p, B, S, 0, 0, 0), GMM_ERR_ARG, "null out");
  bad += expect(gmm_propagate(0, 0, 1.0, 1.0, 1, 0, 0), GMM_ERR_ARG, "propagate null");
  bad += expect(gmm_propagate_rk4ip(0, 0, 1.0, 1.0, 0, 0), GMM_ERR_ARG, "rk4ip null");
  bad += expect(gmm_nonlinear(0, 0, 1, 0), GMM_ERR_ARG, "nonlinear null");
  bad += expect(gmm_nonlinear_noalloc(0, 0, 1, 0), GMM_ERR_ARG, "noalloc null");
  bad += expect(gmm_plan_autotune(0, 1, 0, 0, 0), GMM_ERR_ARG, "autotune null");
  bad += expect(gmm_plan_set_contraction(0, 0), GMM_ERR_ARG, "set_contraction null");
  gmm_batch b = 0;
  bad += expect(gmm_batch_create(&b, 0, 1, 10), GMM_ERR_ARG, "batch null plan");
  bad += expect(gmm_batch_launch(0), GMM_ERR_ARG, "batch launch null");
  int n = 0; long long tags[1];
  bad += expect(gmm_batch_wait(0, tags, 0, 0, 1, &n), GMM_ERR_ARG, "batch wait null");
  bad += expect(gmm_batch_destroy(0), GMM_OK, "batch destroy null");
  bad += expect(gmm_plan_destroy(0), GMM_OK, "plan destroy null");
  printf(bad ? "driver: %d failures\n" : "driver: ok\n", bad);
  return bad != 0;
}
"""


@pytest.mark.slow
def test_host_code_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    """The driver's host code (argument validation, tensor checks, the failure
    and clean-up paths of plan creation) built with AddressSanitizer and
    UndefinedBehaviorSanitizer on the host side only, linked with the library's
    kernel objects and run by a small C program that calls through the C ABI
    (no GPU needed: every call fails before device work, or at the first HIP
    call when there is no device)."""
    from paper_1708_05324_amd import build
    hipcc = build.HIPCC
    objs = [os.path.join(build.BUILD, f.replace(".hip", ".o")) for f in build.SOURCES if f != "gmmpa.hip"]
    if not all(os.path.exists(o) for o in objs):
        build.build(verbose=False)
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", "-g"]
    drv_obj = tmp_path / "gmmpa_san.o"
    subprocess.run([hipcc, *build.CFLAGS, *san, "-c", os.path.join(build.CSRC, "gmmpa.hip"), "-o", str(drv_obj)],
                   check=True, capture_output=True)
    lib = tmp_path / "libgmmpa_san.so"
    subprocess.run([hipcc, "-shared", "-fPIC", f"--offload-arch={build.ARCH}", "-fsanitize=address,undefined",
                    str(drv_obj), *objs, *build.LDFLAGS, "-o", str(lib)], check=True, capture_output=True)
    src = tmp_path / "driver.c"
    src.write_text(DRIVER_C)
    exe = tmp_path / "driver"
    subprocess.run(["/opt/rocm/llvm/bin/clang", "-fsanitize=address,undefined", "-g", "-I",
                    os.path.join(ROOT, "include"), str(src), str(lib), "-Wl,-rpath," + str(tmp_path), "-o", str(exe)],
                   check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1",
               HIP_VISIBLE_DEVICES="")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=120)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert r.returncode == 0
    assert "driver: ok" in r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
