"""The C-ABI library loads and exports every entry point include/gsopt.h
declares (no GPU needed: nothing is called that touches the device)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "gsopt.h")).read()
    return sorted(set(re.findall(r"^(?:gs_status|const char\*|int64_t)\s+(gs_\w+)\(", src, flags=re.M)))


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


def test_binding_structs_match_the_c_layout(tmp_path):
    """Size and every field offset of each binding struct equal what the C
    compiler lays out from the header."""
    import subprocess
    from paper_2604_02851_amd import native, scenes
    structs = {"gs_params": native.GsParams, "gs_render_opts": native.GsRenderOpts,
               "gs_adam_hparams": native.GsAdamHparams, "gs_counters": native.GsCounters, "gs_grid": native.GsGrid, "gs_codec": native.GsCodec, "gs_transform": native.GsTransform,
               "gs_step_args": native.GsStepArgs}
    lines, expect = [], []
    for cname, cls in structs.items():
        lines.append(f'printf("%zu\\n", sizeof({cname}));')
        expect.append(ctypes.sizeof(cls))
        for f in cls._fields_:
            lines.append(f'printf("%zu\\n", offsetof({cname}, {f[0]}));')
            expect.append(getattr(cls, f[0]).offset)
    lines.append('printf("%zu\\n", sizeof(gs_camera));')
    expect.append(scenes.CAM_DTYPE.itemsize)
    src = tmp_path / "layout.c"
    src.write_text('#include <stdio.h>\n#include "gsopt.h"\nint main(void) {\n' + "\n".join(lines) +
                   "\nreturn 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
                           "-I", "/opt/rocm/include", "-o", str(exe), str(src)])
    got = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    assert got == expect


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    from paper_2604_02851_amd import native
    monkeypatch.setattr(native, "LIB_PATH", str(tmp_path / "absent.so"))
    monkeypatch.setattr(native, "_lib", None)
    with pytest.raises(ImportError):
        native.lib()
