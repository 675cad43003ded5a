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


def test_abi_version_and_struct_layout(L):
    assert fdas.abi_version() == 1
    d = fdas.plan_desc_default()
    assert d.struct_size == ctypes.sizeof(fdas.PlanDesc) == 56
    assert (d.z_max, d.n_harm, d.n_max, d.p_fa, d.top_k) == (42, 8, 1 << 22, 1e-6, 0)
    assert ctypes.sizeof(fdas.Cand) == 16


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
                       ("cand_capacity", 0), ("top_k", -1), ("method", 7)]:
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
