"""The C ABI library builds, loads and exports every entry point include/snk.h declares (CPU)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "snk.h")


def declared_symbols():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:snk_status|const char \*)\s*(snk_\w+)\s*\(", txt, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_1804_06304_amd import snk
    if not os.path.exists(snk.LIB_PATH):
        from paper_1804_06304_amd import build
        build.build()
    return snk.load()


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for name in ("snk_create", "snk_set_params", "snk_set_directions", "snk_load_volume", "snk_load_seeds",
                 "snk_evolve", "snk_finalize", "snk_read", "snk_get_state", "snk_set_state", "snk_trace_step"):
        assert name in syms


def test_library_exports_every_declared_symbol(lib):
    from paper_1804_06304_amd import snk
    syms = declared_symbols()
    out = subprocess.check_output(["nm", "-D", "--defined-only", snk.LIB_PATH], text=True)
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    missing = [s for s in syms if s not in exported]
    assert not missing, missing
    assert set(snk.EXPORTS) == set(syms)
    for s in syms:
        assert hasattr(lib, s)


def test_no_torch_types_in_header():
    txt = open(HEADER).read()
    assert "torch" not in txt.lower().replace("torch.tensor.data_ptr", "")


def test_version_string(lib):
    from paper_1804_06304_amd import snk
    assert "gfx950" in snk.snk_version()


def test_params_struct_layout_matches_header(lib, tmp_path):
    """The binding's ctypes structs have the C compiler's size and field offsets."""
    from paper_1804_06304_amd import snk
    fields = [f for f, _ in snk.snk_params._fields_]
    tfields = [f for f, _ in snk.snk_timing._fields_]
    efields = [f for f, _ in snk.snk_engine_stats._fields_]
    src = tmp_path / "layout.c"
    body = "".join(f'printf("%zu ", offsetof(snk_params, {f}));' for f in fields)
    body += "".join(f'printf("%zu ", offsetof(snk_timing, {f}));' for f in tfields)
    body += "".join(f'printf("%zu ", offsetof(snk_engine_stats, {f}));' for f in efields)
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "snk.h"\nint main(void){' + body +
                   'printf("%zu %zu %zu", sizeof(snk_params), sizeof(snk_timing), sizeof(snk_engine_stats)); return 0;}')
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    vals = [int(v) for v in subprocess.check_output([str(exe)], text=True).split()]
    want = [getattr(snk.snk_params, f).offset for f in fields] + [getattr(snk.snk_timing, f).offset for f in tfields]
    want += [getattr(snk.snk_engine_stats, f).offset for f in efields]
    want += [ctypes.sizeof(snk.snk_params), ctypes.sizeof(snk.snk_timing), ctypes.sizeof(snk.snk_engine_stats)]
    assert vals == want


@pytest.mark.skipif(os.path.exists("/dev/kfd"), reason="checks the no-GPU error path")
def test_create_without_gpu_fails_cleanly(lib):
    from paper_1804_06304_amd import snk
    with pytest.raises(snk.SnkError) as e:
        snk.snk_create(0, None)
    assert e.value.code in (snk.SNK_EDEVICE, snk.SNK_EINVAL)
