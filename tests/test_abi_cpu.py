"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point include/mc.h declares, and rejects bad arguments before it
touches a device."""
import ctypes
import os
import re

import pytest

import paper_0812_2964_amd as mc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    hdr = open(os.path.join(ROOT, "include", "mc.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    return sorted(set(re.findall(r"\b(mc_[a-z_0-9]+)\s*\(", hdr)))


def test_library_exports_every_declared_symbol():
    if not os.path.exists(mc.LIB_PATH):
        pytest.skip("libmcgpu.so not built")
    L = mc.lib()
    names = _declared()
    assert "mc_run_chains" in names and "mc_join" in names and "mc_update_weights" in names
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(mc.EXPORTED)


def _create(sizes):
    L = mc.lib()
    arr = (mc._Size * len(sizes))(*[mc._Size(*s) for s in sizes])
    h = ctypes.c_void_p()
    st = L.mc_create(arr, len(sizes), None, ctypes.byref(h))
    return st, h


def test_argument_errors_before_device():
    if not os.path.exists(mc.LIB_PATH):
        pytest.skip("libmcgpu.so not built")
    for bad in [(7, 16, 1, 1), (2, 16, 1, 1), (258, 16, 1, 1), (8, 0, 1, 1), (8, 16, 1, 2), (8, 16, 1, -1)]:
        st, h = _create([bad])
        assert st == mc.MC_EINVAL, bad
        assert not h.value
        assert mc.lib().mc_last_error()
    st, _ = _create([])
    assert st == mc.MC_EINVAL
    L = mc.lib()
    assert L.mc_n_bins(None, 0) == -1
    assert L.mc_run_chains(None, 10, None, None) == mc.MC_EINVAL
    assert L.mc_join(None, 0, None, 10, None, None, 0) == mc.MC_EINVAL
    assert L.mc_update_weights(None, 0, None, None, None, None) == mc.MC_EINVAL
    assert L.mc_run_chains_part(None, 10, 0, 10, None, None) == mc.MC_EINVAL
    assert L.mc_get_stats(None, 0, None) == mc.MC_EINVAL
    assert L.mc_check_levels(None, 0, None) == mc.MC_EINVAL
    assert L.mc_destroy(None) == mc.MC_OK


def test_no_device_is_reported():
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    if not os.path.exists(mc.LIB_PATH):
        pytest.skip("libmcgpu.so not built")
    st, h = _create([(8, 16, 1, 1)])
    assert st == mc.MC_ENODEV
    assert not h.value
