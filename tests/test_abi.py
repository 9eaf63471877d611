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


BOUNDARY = (
    # mesh handles and the per-stage operators
    "dg_mesh_create", "dg_mesh_destroy", "dg_state_len", "dg_rhs", "dg_limit", "dg_cfl_dt",
    "dg_step", "dg_adjoint_step", "dg_check", "dg_last_error",
    # batch handles
    "dg_batch_create", "dg_batch_offset", "dg_batch_run", "dg_batch_adjoint_step",
    "dg_batch_destroy",
)


def test_header_declares_the_boundary():
    names = declared_functions()
    missing = [n for n in BOUNDARY if n not in names]
    assert not missing, missing


def test_batch_calls_validate_without_gpu():
    from paper_1305_5536_amd import capi
    lib = capi.lib()
    out = ctypes.c_void_p(1)
    assert lib.dg_batch_create(None, 1, None, ctypes.byref(out)) == capi.DG_EINVAL
    assert not out.value
    assert lib.dg_batch_offset(None, 0) == -1
    assert lib.dg_batch_mesh(None) is None
    assert lib.dg_batch_run(None, None, 0.3, None, 1, None) == capi.DG_EINVAL
    assert lib.dg_batch_adjoint_step(None, None, None, None, None, None) == capi.DG_EINVAL
    lib.dg_batch_destroy(None)


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


def test_oversized_meshes_rejected_before_any_device_call():
    """Meshes whose coefficient offsets would overflow the kernels' 32-bit
    indexing are refused with DG_EINVAL during validation (no allocation, no
    launch): a 512^3 MHD box (31 arrays of 134M cells) and a face list with
    more faces than its slot tables can address."""
    from paper_1305_5536_amd import capi
    lib = capi.lib()
    out = ctypes.c_void_p()
    cfg = capi.dg_config(capi.DG_MHD, capi.DG_FP64, capi.DG_FLUX_HLLD, 1, 5.0 / 3.0)
    d = capi.dg_mesh_desc()
    d.dim, d.kind = 3, 0
    for k in range(3):
        d.n[k], d.lo[k], d.hi[k] = 512, 0.0, 1.0
    assert lib.dg_mesh_create(ctypes.byref(d), ctypes.byref(cfg), ctypes.byref(out)) == \
        capi.DG_EINVAL
    assert b"32-bit" in lib.dg_last_error()
    assert not out.value
    cfg = capi.dg_config(capi.DG_EULER, capi.DG_FP64, capi.DG_FLUX_HLL, 1, 5.0 / 3.0)
    d = capi.dg_mesh_desc()
    d.dim, d.kind = 2, 1
    d.ncells, d.nfaces = 40_000_000, 120_000_000
    assert lib.dg_mesh_create(ctypes.byref(d), ctypes.byref(cfg), ctypes.byref(out)) == \
        capi.DG_EINVAL
    assert b"32-bit" in lib.dg_last_error()
    d.ncells, d.nfaces = 200_000_000, 3
    assert lib.dg_mesh_create(ctypes.byref(d), ctypes.byref(cfg), ctypes.byref(out)) == \
        capi.DG_EINVAL


def test_empty_meshes_rejected_before_any_device_call():
    """Empty inputs of every mesh kind are refused with DG_EINVAL during
    validation (no allocation, no launch): a Cartesian axis of zero cells, a
    face list without cells or faces, a batch without instances or with an
    empty instance, a moving mesh without generators."""
    import numpy as np

    from paper_1305_5536_amd import capi
    lib = capi.lib()
    out = ctypes.c_void_p()
    euler = capi.dg_config(capi.DG_EULER, capi.DG_FP64, capi.DG_FLUX_HLL, 1, 1.4)
    mhd = capi.dg_config(capi.DG_MHD, capi.DG_FP64, capi.DG_FLUX_HLLD, 1, 5.0 / 3.0)

    def refused(d, cfg):
        out.value = None
        st = lib.dg_mesh_create(ctypes.byref(d), ctypes.byref(cfg), ctypes.byref(out))
        return st == capi.DG_EINVAL and not out.value

    for dim, cfg in ((2, euler), (2, mhd), (3, mhd)):
        for empty_axis in range(dim):
            d = capi.dg_mesh_desc()
            d.dim, d.kind = dim, 0
            for k in range(dim):
                d.n[k], d.lo[k], d.hi[k] = (0 if k == empty_axis else 8), 0.0, 1.0
            assert refused(d, cfg), (dim, empty_axis)
            assert b"cell count" in lib.dg_last_error()
    for ncells, nfaces in ((0, 0), (0, 4), (4, 0)):
        d = capi.dg_mesh_desc()
        d.dim, d.kind = 2, 1
        d.ncells, d.nfaces = ncells, nfaces
        d.box[0] = d.box[1] = 1.0
        assert refused(d, euler), (ncells, nfaces)
    n = np.array([16, 8, 0, 4], np.int32)
    box = np.tile([0.0, 0.0, 1.0, 1.0], 2)
    for ninst, sizes in ((0, n), (2, n)):
        d = capi.dg_mesh_desc()
        d.dim, d.kind, d.ninst = 2, 2, ninst
        d.inst_n = sizes.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        d.inst_box = box.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        assert refused(d, euler), ninst
    d = capi.dg_mesh_desc()
    d.dim, d.kind = 2, 3
    d.box[0] = d.box[1] = 1.0
    assert refused(d, euler)


def test_facelist_cell_without_faces_rejected():
    """A face list in which a cell has no faces (no tessellation has one) is
    refused with DG_EINVAL during validation, before any device call: the
    kernels take every cell's incidence list as non-empty."""
    import numpy as np

    from paper_1305_5536_amd import capi
    from workloads.voronoi import periodic_voronoi
    lib = capi.lib()
    m = periodic_voronoi(30, seed=11, lloyd=1)
    nc = len(m["cell_volume"])
    arrs = {
        "cell_volume": np.append(np.asarray(m["cell_volume"], np.float64), 1e-3),
        "cell_centroid": np.append(np.asarray(m["cell_centroid"], np.float64).reshape(-1),
                                   [0.5, 0.5]),
        "cell_moments": np.append(np.asarray(m["cell_moments"], np.float64).reshape(-1),
                                  [1e-7, 0.0, 1e-7]),
        "face_area": np.ascontiguousarray(m["face_area"], np.float64),
        "face_normal": np.ascontiguousarray(m["face_normal"], np.float64),
        "face_centroid": np.ascontiguousarray(m["face_centroid"], np.float64),
    }
    fc = np.ascontiguousarray(m["face_cells"], np.int32)
    fs = np.ascontiguousarray(m["face_shift"], np.int8)
    d = capi.dg_mesh_desc()
    d.dim, d.kind = 2, 1
    for k, a in arrs.items():
        setattr(d, k, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    d.face_cells = fc.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    d.face_shift = fs.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))
    d.ncells, d.nfaces = nc + 1, len(arrs["face_area"])
    d.box[0], d.box[1] = float(m["box"][0]), float(m["box"][1])
    cfg = capi.dg_config(capi.DG_EULER, capi.DG_FP64, capi.DG_FLUX_HLL, 1, 1.4)
    out = ctypes.c_void_p()
    assert lib.dg_mesh_create(ctypes.byref(d), ctypes.byref(cfg), ctypes.byref(out)) == \
        capi.DG_EINVAL
    assert f"cell {nc} has no faces".encode() in lib.dg_last_error()
    assert not out.value
