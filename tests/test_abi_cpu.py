"""CPU checks of the C-ABI library: it loads, exports every symbol that
include/pic.h declares, the ctypes structs match the C layout, and
configuration errors come back as codes (host-only calls, no device)."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pic.h")


@pytest.fixture(scope="module")
def P():
    from paper_2310_04957_amd.build import LIB, build
    if not os.path.exists(LIB):
        build()
    import paper_2310_04957_amd.pic as P
    return P


def test_every_declared_symbol_is_exported(P):
    decl = set(re.findall(r"^\w[\w\s\*]*?\b(pic_\w+)\s*\(", open(HEADER).read(), re.M))
    assert len(decl) >= 15
    lib = P.lib()
    for name in sorted(decl):
        assert hasattr(lib, name), name


def test_struct_layouts_match_the_header(P, tmp_path):
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include "pic.h"\n#include <stddef.h>\nint main(){'
                   'printf("%zu %zu %zu %zu\\n", sizeof(pic_config), sizeof(pic_diag_out), '
                   'offsetof(pic_config, solver), offsetof(pic_diag_out, error));}')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I" + os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    a = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    assert a == [C.sizeof(P.Config), C.sizeof(P.Diag), P.Config.solver.offset, P.Diag.error.offset]


def test_workspace_size_and_config_errors(P):
    from pic_inputs import workload
    cfg = P.make_config(workload("pp32x24"))
    assert P.workspace_bytes(cfg) > 0
    bad = P.make_config(workload("pp32x24"))
    bad.geom.nr = 31                  # odd cell count
    with pytest.raises(P.PicError) as e:
        P.workspace_bytes(bad)
    assert e.value.code == -1
    bad = P.make_config(workload("pp32x24"))
    bad.geom.nr, bad.geom.nz = 4096, 4096    # 256 x 256 tiles: more than 16-bit tile keys hold
    with pytest.raises(P.PicError) as e:
        P.workspace_bytes(bad)
    assert e.value.code == -1
    bad.geom.nz = 4064                        # 256 x 254 tiles
    assert P.workspace_bytes(bad) > 0
    bad = P.make_config(workload("pp32x24"))
    bad.abi_version = 99
    with pytest.raises(P.PicError):
        P.workspace_bytes(bad)
    assert P.lib().pic_strerror(-2) == b"particle capacity exceeded by births"


def test_pic_init_without_gpu_fails_loudly(P):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from pic_inputs import workload
    with pytest.raises(RuntimeError):
        P.Pic(workload("pp32x24"))
