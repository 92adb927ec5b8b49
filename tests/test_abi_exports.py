"""The C-ABI library loads and exports every function include/sgtp.h declares (no GPU needed)."""

import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sgtp.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sgtp_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_the_planning_calls():
    names = declared_functions()
    for required in ("sgtp_rollout_cost", "sgtp_ibr_sweep", "sgtp_plan_step", "sgtp_ctx_create",
                     "sgtp_ctx_destroy", "sgtp_track_upload", "sgtp_last_error", "sgtp_advance"):
        assert required in names


def test_library_exports_every_declared_symbol():
    import paper_2607_25388_amd.sgtp as sg
    if not os.path.exists(sg.LIB_PATH):
        pytest.skip("libsgtp.so not built")
    lib = C.CDLL(sg.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    lib.sgtp_abi_version.restype = C.c_int
    assert lib.sgtp_abi_version() == 1


def test_struct_sizes_match_the_header():
    """ctypes mirrors of the ABI structs have the C layout (checked with the host compiler)."""
    import shutil
    import subprocess
    import tempfile
    import paper_2607_25388_amd.sgtp as sg
    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("no host compiler")
    src = '#include <stdio.h>\n#include "sgtp.h"\nint main(){printf("%zu %zu %zu\\n", sizeof(sgtp_params), ' \
          'sizeof(sgtp_race), sizeof(sgtp_choice)); return 0;}\n'
    with tempfile.TemporaryDirectory() as td:
        open(os.path.join(td, "s.c"), "w").write(src)
        subprocess.check_call([cc, "-I", os.path.join(ROOT, "include"), "-o", os.path.join(td, "s"),
                               os.path.join(td, "s.c")])
        out = subprocess.check_output([os.path.join(td, "s")]).decode().split()
    assert [int(v) for v in out] == [C.sizeof(sg.Params), C.sizeof(sg.Race), C.sizeof(sg.Choice)]


def test_context_creation_fails_cleanly_without_a_gpu():
    import torch
    import paper_2607_25388_amd.sgtp as sg
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    lib = sg.load()
    ctx = C.c_void_p()
    rc = lib.sgtp_ctx_create(C.byref(ctx), 4, 20, 1, 1000, 1024)
    assert rc == -4 and not ctx.value
    with pytest.raises(RuntimeError):
        sg.Planner()
