"""The C-ABI library loads on the CPU and exports every function include/*.h declares
(no compute calls: there is no GPU here)."""
import ctypes
import glob
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s+\**\s*(dg_[a-z0-9_]+)\s*\(",
                             text, flags=re.M):
            names.add(m.group(1))
    return names


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("dg_mesh_create", "dg_rhs", "dg_limit", "dg_step", "dg_cfl_dt", "dg_check"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1305_5536_amd import capi
    lib = capi.lib()
    missing = [n for n in sorted(declared_functions()) if not hasattr(lib, n)]
    assert not missing, missing
    # the binding declares exactly the header's functions
    assert {s[0] for s in capi.SYMBOLS} == declared_functions()


def test_error_path_without_gpu():
    """Validation happens before any device call: NULL arguments are rejected."""
    from paper_1305_5536_amd import capi
    lib = capi.lib()
    assert lib.dg_rhs(None, None, None, None) == capi.DG_EINVAL
    assert b"NULL" in lib.dg_last_error()
    assert lib.dg_state_len(None) == -1
    out = ctypes.c_void_p()
    assert lib.dg_mesh_create(None, None, ctypes.byref(out)) == capi.DG_EINVAL
    cfg = capi.dg_config(capi.DG_EULER, capi.DG_FP64, capi.DG_FLUX_HLLD, 1, 1.4)
    d = capi.dg_mesh_desc()
    d.dim, d.kind = 2, 0
    assert lib.dg_mesh_create(ctypes.byref(d), ctypes.byref(cfg), ctypes.byref(out)) == \
        capi.DG_EUNSUPPORTED
