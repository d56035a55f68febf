"""The C-ABI library loads and exports every entry point include/gsopt.h
declares (no GPU needed: nothing is called that touches the device)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "gsopt.h")).read()
    return sorted(set(re.findall(r"^(?:gs_status|const char\*)\s+(gs_\w+)\(", src, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ("gs_project", "gs_build_tile_lists", "gs_composite", "gs_backward", "gs_adam_step",
                 "gs_delta_extract", "gs_delta_reset_baseline", "gs_step_capture", "gs_step_launch"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2604_02851_amd import native
    if not os.path.exists(native.LIB_PATH):
        pytest.skip("libgsopt.so not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(native.LIB_PATH)
    for name in declared():
        assert hasattr(lib, name), name
    assert set(declared()) == set(native.EXPORTED)


def test_binding_structs_match_the_c_layout():
    from paper_2604_02851_amd import native, scenes
    assert ctypes.sizeof(native.GsParams) == 48
    assert ctypes.sizeof(native.GsRenderOpts) == 32
    assert ctypes.sizeof(native.GsAdamHparams) == 36
    assert ctypes.sizeof(native.GsCounters) == 32
    assert scenes.CAM_DTYPE.itemsize == 84
    assert ctypes.sizeof(native.GsStepArgs) == 376


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    from paper_2604_02851_amd import native
    monkeypatch.setattr(native, "LIB_PATH", str(tmp_path / "absent.so"))
    monkeypatch.setattr(native, "_lib", None)
    with pytest.raises(ImportError):
        native.lib()
