"""Host-only checks of the C ABI: the library loads, exports every symbol that
include/rt.h declares, mirrors its structs, and rejects bad arguments before
touching a device."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rt.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:rt_status|const char\*)\s+(rt_\w+)\s*\(", text, flags=re.M)))


def test_library_exports_every_declared_symbol():
    from paper_2303_11103_amd import _lib
    names = _declared()
    assert len(names) >= 15
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if l.strip()}
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    # the binding declares exactly the header's functions
    assert sorted(_lib.SIGNATURES) == names


def test_struct_layouts_match_header(tmp_path):
    from paper_2303_11103_amd import _lib
    # sizes implied by the header (natural alignment, x86-64)
    assert ctypes.sizeof(_lib.rt_material) == 8
    assert ctypes.sizeof(_lib.rt_device) == 32
    assert ctypes.sizeof(_lib.rt_trace_params) == 56
    assert ctypes.sizeof(_lib.rt_grid) == 40
    assert ctypes.sizeof(_lib.rt_scene_info_t) == 40
    assert ctypes.sizeof(_lib.rt_mlp_config) == 88
    src = (
        "#include <stddef.h>\n#include <stdio.h>\n#include \"rt.h\"\n"
        "int main(){printf(\"%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n\", sizeof(rt_material), sizeof(rt_device),"
        " sizeof(rt_trace_params), sizeof(rt_grid), sizeof(rt_scene_info_t),"
        " offsetof(rt_trace_params, num_rays), offsetof(rt_grid, nx), sizeof(rt_mlp_config),"
        " offsetof(rt_mlp_config, ff_scale_cell), offsetof(rt_mlp_config, prior_freq_hz),"
        " offsetof(rt_mlp_config, ff_scale_rel)); return 0;}\n")
    c = tmp_path / "layout_check.c"
    exe = tmp_path / "layout_check"
    c.write_text(src)
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe)], check=True)
    vals = list(map(int, subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()))
    assert vals == [8, 32, 56, 40, 40, _lib.rt_trace_params.num_rays.offset, _lib.rt_grid.nx.offset, 88,
                    _lib.rt_mlp_config.ff_scale_cell.offset, _lib.rt_mlp_config.prior_freq_hz.offset,
                    _lib.rt_mlp_config.ff_scale_rel.offset]


def test_null_and_invalid_arguments_fail_on_host():
    from paper_2303_11103_amd import _lib
    lib = _lib.lib
    assert lib.rt_create(None, 0) == _lib.RT_ERR_ARG
    assert b"NULL" in lib.rt_last_error()
    p = _lib.rt_trace_params(3.5e9, 3, 16, 1000, 1e-4, 0, 1)
    assert lib.rt_coverage_map(None, None, ctypes.byref(p), None, None, None, None, None, None, None) == \
        _lib.RT_ERR_ARG
    assert lib.rt_set_stream(None, None) == _lib.RT_ERR_ARG
    assert lib.rt_scene_info(None, None) == _lib.RT_ERR_ARG
    assert lib.rt_profile_enable(None, 1) == _lib.RT_ERR_ARG
    for name in ("rt_compute_paths", "rt_compute_scattering", "rt_compute_diffraction", "rt_coverage_map_noalloc"):
        scalar = {ctypes.c_int32: 1, ctypes.c_int64: 1, ctypes.c_double: 3.5e9}
        args = [scalar.get(t) for t in _lib.SIGNATURES[name]]   # NULL for every pointer
        assert getattr(lib, name)(*args) == _lib.RT_ERR_ARG, name
        assert b"NULL" in lib.rt_last_error() or b"params" in lib.rt_last_error(), name
    # destroy functions accept NULL
    assert lib.rt_destroy(None) == _lib.RT_OK
    assert lib.rt_scene_destroy(None) == _lib.RT_OK
