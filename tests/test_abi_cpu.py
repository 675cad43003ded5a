"""Host-side checks of libfdas that need no GPU.

The library must load, export every symbol include/fdas.h declares, reject
bad arguments before touching a device, and its host FP64 arithmetic (its own
Gauss-Legendre templates and Erlang thresholds) must agree with the oracle's
independent closed forms.
"""

import ctypes
import os
import re

import numpy as np
import pytest

from blockref import closure_reference
from paper_1806_01556_amd import fdas

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _gpu_present():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(fdas.LIB_PATH):
        pytest.fail("libfdas.so is not built (run python -m paper_1806_01556_amd.build)")
    return fdas.lib()


def test_exports_every_declared_symbol(L):
    with open(os.path.join(ROOT, "include", "fdas.h")) as f:
        hdr = f.read()
    declared = set(re.findall(r"^\s*(?:[\w\s\*]+?)\b(fdas_\w+)\s*\(", hdr, flags=re.M))
    assert declared == set(fdas.EXPORTED), declared ^ set(fdas.EXPORTED)
    for name in declared:
        assert hasattr(L, name), name


def test_abi_version_and_struct_layout(L, tmp_path):
    assert fdas.abi_version() == 2
    d = fdas.plan_desc_default()
    assert d.struct_size == ctypes.sizeof(fdas.PlanDesc) == 64
    assert (d.z_max, d.n_harm, d.n_max, d.p_fa, d.top_k) == (42, 8, 1 << 22, 1e-6, 0)
    assert ctypes.sizeof(fdas.Cand) == 16
    # the binding's field offsets are the header's: compile a probe against it
    fields = [f for f, _ in fdas.PlanDesc._fields_]
    src = tmp_path / "layout.c"
    body = "".join(f'  printf("%s %zu\\n", "{f}", offsetof(fdas_plan_desc, {f}));\n' for f in fields)
    src.write_text("#include <stddef.h>\n#include <stdio.h>\n#include \"fdas.h\"\nint main(void) {\n" + body +
                   '  printf("size %zu\\n", sizeof(fdas_plan_desc));\n  return 0;\n}\n')
    exe = tmp_path / "layout"
    import subprocess
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = dict(line.split() for line in subprocess.run([str(exe)], check=True, capture_output=True,
                                                         text=True).stdout.splitlines())
    for f in fields:
        assert int(out[f]) == getattr(fdas.PlanDesc, f).offset, f
    assert int(out["size"]) == ctypes.sizeof(fdas.PlanDesc)


@pytest.mark.parametrize("n,blocks,n_harm", [
    (1 << 22, [0, 7, 100, 511, 1023], 8), (1 << 22, [], 8), (3 * (1 << 20) + 17, [3, 400, 767], 5),
    (5000, [0, 1], 8), (1 << 20, list(range(0, 256, 37)), 1), (1 << 20, [255], 2)])
def test_block_closure_matches_brute_force(L, n, blocks, n_harm):
    got = fdas.block_closure(blocks, n, n_harm)
    assert np.array_equal(got, closure_reference(blocks, n, n_harm))


def test_block_closure_errors(L):
    cnt = ctypes.c_int32(0)
    b = np.array([0, 5], dtype=np.int32)
    out = np.zeros(1, dtype=np.int32)
    assert L.fdas_block_closure(1 << 20, 8, b.ctypes.data, 2, out.ctypes.data, 1, ctypes.byref(cnt)) == \
        fdas.ERR_CAPACITY
    assert cnt.value == closure_reference([0, 5], 1 << 20, 8).size
    bad = np.array([256], dtype=np.int32)
    assert L.fdas_block_closure(1 << 20, 8, bad.ctypes.data, 1, out.ctypes.data, 1, ctypes.byref(cnt)) == \
        fdas.ERR_INVALID_ARG
    assert L.fdas_block_closure(1 << 20, 9, b.ctypes.data, 2, out.ctypes.data, 1, ctypes.byref(cnt)) == \
        fdas.ERR_INVALID_ARG


def test_prescreen_init_params(L):
    a = fdas.prescreen_init_params(3)
    assert a.size == fdas.Prescreen.param_count() and a.dtype == np.float32
    assert np.array_equal(a, fdas.prescreen_init_params(3))
    assert not np.array_equal(a, fdas.prescreen_init_params(4))
    o = 0
    for cin in (1, 32, 32, 32):
        w = a[o:o + 32 * cin * 9]
        lim = np.sqrt(6.0 / (cin * 9))
        assert np.all(np.abs(w) < lim) and abs(w.mean()) < 0.1 * lim and w.std() > 0.5 * lim / np.sqrt(3)
        o += 32 * cin * 9
        assert np.all(a[o:o + 32] == 0)
        o += 32
    assert np.all(np.abs(a[o:o + 32]) < 1 / np.sqrt(32)) and a[o + 32] == 0 and o + 33 == a.size


@pytest.mark.parametrize("z", list(range(-42, 43, 3)) + [42, -42, 64, -64, 1, -1])
def test_library_templates_match_oracle(L, z):
    from oracle import response
    d, h_ref = response.template(z)
    h = fdas.template_taps(z)
    assert h.shape == h_ref.shape
    assert np.max(np.abs(h - h_ref)) < 1e-12


def test_library_thresholds_match_oracle(L):
    from oracle import harmonic
    for p_fa in (1e-6, 1e-3, 0.1):
        t = fdas.thresholds(8, p_fa)
        ref = harmonic.thresholds(8, p_fa)
        assert np.max(np.abs(t / ref - 1.0)) < 1e-12


def test_bad_arguments_rejected_before_device(L):
    h = ctypes.c_void_p()
    assert L.fdas_plan_create(None, ctypes.byref(h)) == fdas.ERR_INVALID_ARG
    assert "NULL" in fdas.last_error()
    for field, val in [("struct_size", 8), ("z_max", -1), ("z_max", 65), ("n_harm", 0), ("n_harm", 9),
                       ("p_fa", 0.0), ("p_fa", 1.0), ("p_fa", float("nan")), ("n_max", 0),
                       ("cand_capacity", 0), ("top_k", -1), ("method", 7), ("n_max", 1 << 25)]:
        d = fdas.plan_desc_default(**{field: val})
        assert L.fdas_plan_create(ctypes.byref(d), ctypes.byref(h)) == fdas.ERR_INVALID_ARG, field
        assert h.value is None
        assert fdas.last_error()
    d = fdas.plan_desc_default(ols_chunk=1024)
    assert L.fdas_plan_create(ctypes.byref(d), ctypes.byref(h)) == fdas.ERR_UNSUPPORTED
    assert L.fdas_convolve(None, 16, 4, 16, 4, None) == fdas.ERR_INVALID_ARG
    assert L.fdas_harmonic_sum(None, 16, 4, 4, None, 16, 16, None) == fdas.ERR_INVALID_ARG
    n = ctypes.c_int64(5)
    assert L.fdas_candidates(None, 16, 16, None, 0, ctypes.byref(n), None, None) == fdas.ERR_INVALID_ARG
    assert L.fdas_plan_destroy(None) == fdas.OK
    assert L.fdas_template_taps(65, None, 0, None) == fdas.ERR_INVALID_ARG
    assert L.fdas_thresholds(9, 1e-6, None) == fdas.ERR_INVALID_ARG
    assert L.fdas_search_flagged(None, 16, 4, 16, 4, 16, 0.0, 16, 16, None) == fdas.ERR_INVALID_ARG
    assert L.fdas_prescreen_infer(None, 16, 4096, 1, 16, None) == fdas.ERR_INVALID_ARG
    assert "NULL" in fdas.last_error()


@pytest.mark.skipif(_gpu_present(), reason="checks the no-GPU path")
def test_plan_create_without_gpu_reports_no_device(L):
    h = ctypes.c_void_p()
    d = fdas.plan_desc_default()
    assert L.fdas_plan_create(ctypes.byref(d), ctypes.byref(h)) == fdas.ERR_NO_DEVICE
    assert h.value is None
    with pytest.raises(fdas.FdasError) as e:
        fdas.plan_create()
    assert e.value.status == fdas.ERR_NO_DEVICE
