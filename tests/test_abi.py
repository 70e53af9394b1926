"""The C-ABI library loads on a machine without a GPU and exports every
function include/kg.h declares; host-only entry points validate arguments."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kg.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(kg_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("kg_plan", "kg_step", "kg_energy", "kg_set_state", "kg_destroy"):
        assert required in names


def test_library_exports_every_declared_function():
    from paper_1501_04552_amd import kg
    lib = ctypes.CDLL(kg.LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(declared_functions()) <= set(kg.EXPORTS)


def test_host_side_validation():
    from paper_1501_04552_amd import kg
    assert kg.kg_status_str(kg.KG_BLOWUP) == "KG_BLOWUP"
    assert kg.kg_workspace_bytes(kg.make_params(64, 0.01)) > 0
    for good in (8, 24, 48, 96, 128, 384, 512):
        assert kg.kg_workspace_bytes(kg.make_params(good, 0.01)) > 0
    for bad in (kg.make_params(40, 0.01), kg.make_params(1024, 0.01), kg.make_params(100, 0.01),
                kg.make_params(12, 0.01), kg.make_params(36, 0.01), kg.make_params(768, 0.01),
                kg.make_params(64, 0.0), kg.make_params(64, -1.0),
                kg.make_params(64, 0.01, precision=7)):
        assert kg.kg_workspace_bytes(bad) == 0
    # FP32 is accepted and needs about half the FP64 workspace
    b64 = kg.kg_workspace_bytes(kg.make_params(256, 0.01))
    b32 = kg.kg_workspace_bytes(kg.make_params(256, 0.01, precision=kg.KG_FP32))
    assert 0.45 * b64 < b32 < 0.6 * b64
    # sizes of the stored fields: 3 complex fields of n*n*pitch plus small buffers
    b512 = kg.kg_workspace_bytes(kg.make_params(512, 0.005))
    assert 3 * 512 * 512 * 257 * 16 < b512 < 3.2 * 512 * 512 * 264 * 16
    with pytest.raises(kg.KGError) as e:
        kg.kg_plan(kg.make_params(40, 0.01))
    assert e.value.status == kg.KG_E_UNSUPPORTED_SIZE
    with pytest.raises(kg.KGError) as e:
        kg.kg_plan(kg.make_params(64, 0.0))
    assert e.value.status == kg.KG_E_INVALID
    # a borrowed workspace smaller than kg_workspace_bytes is refused before
    # the plan touches it (the pointer is never dereferenced)
    need = kg.kg_workspace_bytes(kg.make_params(32, 0.01))
    with pytest.raises(kg.KGError) as e:
        kg.kg_plan(kg.make_params(32, 0.01), 0x10000, need - 1)
    assert e.value.status == kg.KG_E_NOMEM


def test_plan_setup_runs_on_the_host():
    """kg_plan's host-side set-up (layout, launchers, slab choice) runs for
    every size and precision before any device work; without a GPU the
    allocation then fails cleanly."""
    import torch
    from paper_1501_04552_amd import kg
    if torch.cuda.is_available():
        pytest.skip("needs a machine without a GPU (the allocation must fail)")
    for n in (8, 24, 48, 64, 96, 128, 192, 256, 384, 512):
        for prec in (kg.KG_FP64, kg.KG_FP32):
            with pytest.raises(kg.KGError) as e:
                kg.kg_plan(kg.make_params(n, 0.01, precision=prec))
            assert e.value.status in (kg.KG_E_NOMEM, kg.KG_E_HIP)


def test_ctypes_structs_match_the_header(tmp_path):
    """The binding's ctypes mirrors of the header's structs have the C field
    offsets and sizes (a C program built against include/kg.h prints them)."""
    import json
    import subprocess
    from paper_1501_04552_amd import kg
    structs = {"kg_params": kg.kg_params, "kg_run_desc": kg.kg_run_desc,
               "kg_run_result": kg.kg_run_result, "kg_batch_opts": kg.kg_batch_opts}
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "kg.h"', "int main(void) {",
             '  printf("{");']
    first = True
    for name, cls in structs.items():
        for field, _ in cls._fields_:
            sep = "" if first else ","
            first = False
            lines.append(f'  printf("{sep}\\"{name}.{field}\\": %zu", offsetof({name}, {field}));')
        lines.append(f'  printf(",\\"{name}\\": %zu", sizeof({name}));')
    lines += ['  printf("}\\n");', "  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    c = json.loads(subprocess.run([str(exe)], check=True, capture_output=True,
                                  text=True).stdout)
    for name, cls in structs.items():
        assert c[name] == ctypes.sizeof(cls), name
        for field, _ in cls._fields_:
            assert c[f"{name}.{field}"] == getattr(cls, field).offset, (name, field)


def test_complex_field_workspace():
    """A complex field holds the full spectrum, n columns against the real
    field's n/2 + 1 padded to whole tiles (136 in FP64, 144 in FP32 at 256^3):
    1.7 to 2 times the real workspace."""
    from paper_1501_04552_amd import kg
    for prec in (kg.KG_FP64, kg.KG_FP32):
        br = kg.kg_workspace_bytes(kg.make_params(256, 0.01, precision=prec))
        bc = kg.kg_workspace_bytes(kg.make_params(256, 0.01, precision=prec, complex_field=True))
        assert 1.7 * br < bc < 2.05 * br
        bd = kg.kg_workspace_bytes(kg.make_params(256, 0.01, precision=prec, dealias=True))
        assert bd == br
