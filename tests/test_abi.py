"""The C-ABI library loads and exports every declared entry point; host-side argument
checks reject bad calls before any device work (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_1909_11873_amd import gwlike as gw

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gwlike.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gwl_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = gw.lib()
    names = declared_functions()
    assert len(names) >= 13
    for n in names:
        assert hasattr(L, n), f"{n} declared in include/gwlike.h but not exported"
    assert gw.version().startswith("gwlike")


def test_error_codes_without_device_work():
    L = gw.lib()
    vp = ctypes.c_void_p
    h = vp()
    dets = (gw.Detector * 1)(gw.Detector(0.8, -2.0, 2.2, 0.6))
    # null device pointers
    assert L.gwl_event_create(None, None, dets, 1, None, 100, 0.25, 0.0, 0, None, ctypes.byref(h)) == -1
    assert b"device pointers" in L.gwl_last_error()
    # bad sizes (checked before pointers are used)
    fake = vp(0x1000)
    assert L.gwl_event_create(fake, fake, dets, 0, fake, 100, 0.25, 0.0, 0, None, ctypes.byref(h)) == -2
    assert L.gwl_event_create(fake, fake, dets, 5, fake, 100, 0.25, 0.0, 0, None, ctypes.byref(h)) == -2
    assert L.gwl_event_create(fake, fake, dets, 1, fake, 0, 0.25, 0.0, 0, None, ctypes.byref(h)) == -2
    assert L.gwl_event_create(fake, fake, dets, 1, fake, 100, -1.0, 0.0, 0, None, ctypes.byref(h)) == -1
    assert L.gwl_event_create(fake, fake, dets, 1, fake, 100, float("nan"), 0.0, 0, None, ctypes.byref(h)) == -1
    assert L.gwl_event_create(fake, fake, dets, 1, fake, 100, 0.25, 0.0, 7, None, ctypes.byref(h)) == -5
    nan_det = (gw.Detector * 1)(gw.Detector(float("nan"), 0, 0, 0))
    assert L.gwl_event_create(fake, fake, nan_det, 1, fake, 100, 0.25, 0.0, 0, None, ctypes.byref(h)) == -1
    assert L.gwl_event_create(fake, fake, dets, 1, fake, 100, 0.25, 0.0, 0, None, None) == -1
    # calls on a null event
    assert L.gwl_logl_batch(None, fake, 10, 1, fake, None) == -1
    assert L.gwl_logl_grad(None, fake, 10, 0, fake, fake, None) == -1
    assert L.gwl_event_info(None, None, None, None) == -1
    assert L.gwl_autotune(None, None, 10, 1, 0) == -1
    assert L.gwl_event_destroy(None) == 0
    assert L.gwl_plan_destroy(None) == 0
    # waveform argument checks
    assert L.gwl_waveform(fake, -1, dets, 1, fake, 10, 0.0, fake, None) == -2
    assert L.gwl_waveform(fake, 1, dets, 0, fake, 10, 0.0, fake, None) == -2
    assert L.gwl_waveform(None, 1, dets, 1, fake, 10, 0.0, fake, None) == -1
    assert L.gwl_waveform(fake, 0, dets, 1, fake, 10, 0.0, fake, None) == 0  # empty batch: no-op
    assert L.gwl_autotune_load(b"/nonexistent/cache.json") == -1
    # multi-event plan calls without events or plan
    assert L.gwl_multi_autotune(None, None, 1, None, 1, 0) == -1
    assert L.gwl_plan_info(None, None, None, None) == -1
    assert L.gwl_launch_shape(None, 10, 1, 0, None, None) == -1
    assert L.gwl_multi_plan_create(None, 1, None, 1, 0, ctypes.byref(h)) == -1


def test_python_binding_rejects_cpu_tensors():
    import torch
    with pytest.raises(ValueError):
        gw.Event(torch.zeros(1, 10, dtype=torch.complex128), torch.ones(1, 10, dtype=torch.float64),
                 [(0.1, 0.2, 0.3, 0.4)], torch.ones(10, dtype=torch.float64), 0.25)
    with pytest.raises(ValueError):
        gw._prec("half")


def test_slice_entry_points_check_arguments_without_device_work():
    L = gw.lib()
    fake = ctypes.c_void_p(0x1000)
    ptrs9 = [fake] * 9
    assert L.gwl_slice_ends(0, 3, 4, *ptrs9, None) == -2
    assert L.gwl_slice_ends(10, 0, 4, *ptrs9, None) == -2
    assert L.gwl_slice_ends(10, 3, 0, *ptrs9, None) == -2
    assert L.gwl_slice_ends(10, 3, 4, None, *ptrs9[1:], None) == -1
    assert L.gwl_slice_ends_select(10, 3, 4, *([fake] * 6), None, None) == -1
    ptrs14 = [fake] * 14
    assert L.gwl_slice_draws(10, 3, 0, *ptrs14, None) == -2
    assert L.gwl_slice_draws(1 << 28, 3, 8, *ptrs14, None) == -2     # G n points beyond 2^30
    assert L.gwl_slice_draws(10, 3, 8, *([fake] * 12), None, None, None) == -1   # nact_next is required
    assert b"null pointer" in L.gwl_last_error()
    assert L.gwl_slice_select(10, 3, 8, *([fake] * 14), None, None) == -1
    assert b"null pointer" in L.gwl_last_error()
    # the next list (and its length) must differ from the current one
    assert L.gwl_slice_draws(10, 3, 8, *([fake] * 12), fake, None, None) == -1
    assert b"must not be" in L.gwl_last_error()
    assert L.gwl_slice_select(10, 3, 8, *([fake] * 15), None) == -1
    assert b"must not be" in L.gwl_last_error()
    assert L.gwl_slice_list_init(0, fake, fake, None) == -2
    assert L.gwl_slice_list_init(10, None, fake, None) == -1
    assert L.gwl_logl_batch_live(None, fake, 10, fake, 1, fake, None) == -1


def test_prior_transform_checks_arguments_without_device_work():
    L = gw.lib()
    fake = ctypes.c_void_p(0x1000)
    maps = (ctypes.c_int * 3)(0, 1, 7)
    coef = (ctypes.c_double * 3)(0.0, 1.0, 2.0)
    pm, pc = ctypes.cast(maps, ctypes.c_void_p), ctypes.cast(coef, ctypes.c_void_p)
    assert L.gwl_prior_transform(0, 3, pm, pc, pc, fake, fake, None) == -2
    assert L.gwl_prior_transform(10, 0, pm, pc, pc, fake, fake, None) == -2
    assert L.gwl_prior_transform(10, 65, pm, pc, pc, fake, fake, None) == -2
    assert L.gwl_prior_transform(10, 3, pm, pc, pc, None, fake, None) == -1
    assert L.gwl_prior_transform(10, 3, pm, pc, pc, fake, fake, None) == -1     # map code 7
    assert b"unknown map 7" in L.gwl_last_error()
    with pytest.raises(ValueError):
        gw.PriorColumns([0, 5], [0.0, 0.0], [1.0, 1.0])


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """Without the built library every entry into the binding raises; nothing falls back to
    a CPU implementation."""
    monkeypatch.setattr(gw, "_lib", None)
    monkeypatch.setattr(gw, "LIB_PATH", str(tmp_path / "libgwlike.so"))
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        gw.lib()
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        gw.version()
