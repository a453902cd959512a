"""C-ABI checks that need no GPU: the library loads, exports every declared symbol, and
rejects bad arguments before its first HIP call (so fake non-NULL pointers are safe)."""
import ctypes
import os
import re

import pytest
import torch  # noqa: F401  (loads the HIP runtime libdwg links against)

from paper_2405_13839_amd import dwg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dwg.h")

pytestmark = pytest.mark.skipif(not os.path.exists(dwg.LIB_PATH), reason="libdwg.so not built")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dwg_[a-z_0-9]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    lib = dwg.load()
    names = declared_functions()
    assert len(names) >= 14
    for nm in names:
        assert hasattr(lib, nm), nm
    assert set(dwg.EXPORTED) == set(names)


def test_version_and_status_strings():
    lib = dwg.load()
    assert "gfx950" in dwg.version()
    assert lib.dwg_status_string(-2) == b"DWG_E_WORKSPACE"
    assert lib.dwg_status_string(1) == b"DWG_NOT_CONVERGED"


def test_workspace_bytes():
    assert dwg.workspace_bytes(0, 10) == 0
    a = dwg.workspace_bytes(1000, 1000)
    b = dwg.workspace_bytes(100_000, 100_000)
    assert 0 < a < b
    # O(n) bytes: the all-pairs split partial sums are held to 512 MiB (or 16 splits), the
    # rest is a few hundred bytes per point
    assert b < (512 << 20) + 1000 * 100_000
    assert dwg.workspace_bytes(4_000_000, 4_000_000) < 16 * 28 * 4_000_000 + 2000 * 4_000_000
    # invalid kernel parameters make it report 0
    assert dwg.workspace_bytes(1000, 1000, dwg.Params(lam=-1.0)) == 0


FAKE = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails before any device access


def _call_grad(n=10, m=10, kp=None, ws=FAKE, ws_bytes=1 << 40, P=FAKE, g=FAKE):
    lib = dwg.load()
    kp = kp or dwg.Params().c()
    return lib.dwg_gwn_grad(P, FAKE, FAKE, None, n, FAKE, m, ctypes.byref(kp), None, g, None, ws, ws_bytes, None)


def test_invalid_arguments_rejected_before_device():
    assert _call_grad(P=None) == dwg.DWG_E_INVALID
    assert _call_grad(g=None) == dwg.DWG_E_INVALID
    assert _call_grad(n=0) == dwg.DWG_E_INVALID
    assert _call_grad(m=-3) == dwg.DWG_E_INVALID
    assert _call_grad(n=1 << 31) == dwg.DWG_E_INVALID  # int32 point indices
    assert _call_grad(m=1 << 31) == dwg.DWG_E_INVALID
    for bad in [dwg.Params(lam=-1), dwg.Params(lam=float("nan")), dwg.Params(eps=-1e-3), dwg.Params(split=65),
                dwg.Params(beta=0.5), dwg.Params(beta=float("inf")), dwg.Params(beta=2.3, leaf=-1),
                dwg.Params(beta=2.3, leaf=2000)]:
        assert _call_grad(kp=bad.c()) == dwg.DWG_E_INVALID
    kp = dwg.Params().c()
    kp.reserved[1] = 1
    assert _call_grad(kp=kp) == dwg.DWG_E_INVALID
    assert b"reserved" in dwg.load().dwg_last_error()


def test_workspace_too_small():
    assert _call_grad(ws_bytes=64) == dwg.DWG_E_WORKSPACE
    assert _call_grad(ws=None, ws_bytes=0) == dwg.DWG_E_WORKSPACE
    assert b"workspace" in dwg.load().dwg_last_error()


def test_iterate_parameter_validation():
    lib = dwg.load()
    kp = dwg.Params().c()
    for ip in [dwg.IterateParams(0, 0, 0.1, 0.01), dwg.IterateParams(5, 0, -1.0, 0.01),
               dwg.IterateParams(5, 0, 0.1, 0.0), dwg.IterateParams(5, 0, 0.1, 1.5), dwg.IterateParams(5, 2, 0.1, 0.01)]:
        done = ctypes.c_int(7)
        st = lib.dwg_iterate(FAKE, FAKE, None, 100, FAKE, ctypes.byref(kp), ctypes.byref(ip), None, ctypes.byref(done),
                             FAKE, 1 << 40, None)
        assert st == dwg.DWG_E_INVALID
        assert done.value == 0


def test_knn_and_mlp_validation():
    lib = dwg.load()
    assert lib.dwg_knn(FAKE, 100, FAKE, 100, 0, 17, FAKE, None, FAKE, 1 << 40, None) == dwg.DWG_E_INVALID
    assert lib.dwg_knn(FAKE, 5, FAKE, 100, 1, 5, FAKE, None, FAKE, 1 << 40, None) == dwg.DWG_E_INVALID
    assert lib.dwg_delta_knn_mean(FAKE, 100, 10, 0.0, FAKE, FAKE, 1 << 40, None) == dwg.DWG_E_INVALID
    assert lib.dwg_mlp_train_step(FAKE, FAKE, FAKE, 0, 1e-3, FAKE, FAKE, None, 10, None, None, FAKE, 1 << 40,
                                  None) == dwg.DWG_E_INVALID
    assert lib.dwg_init_normals(7, 0, None, 10, None, FAKE, None, 0, None) == dwg.DWG_E_INVALID
    assert dwg.mlp_param_count() == 128 * 48 + 128 + 128 * 128 + 128 + 3 * 128 + 3
    assert dwg.mlp_blob_bytes() == 4 * dwg.mlp_param_count()


def test_octree_area_and_level_set_validation():
    lib = dwg.load()
    cnt = ctypes.c_int64(5)
    assert lib.dwg_octree(FAKE, 0, 0, FAKE, FAKE, 10, ctypes.byref(cnt), FAKE, 1 << 40, None) == dwg.DWG_E_INVALID
    assert cnt.value == 0
    assert lib.dwg_octree(FAKE, 100, 2000, FAKE, FAKE, 10, ctypes.byref(cnt), FAKE, 1 << 40, None) == dwg.DWG_E_INVALID
    assert lib.dwg_octree(FAKE, 100, 0, FAKE, FAKE, 200, ctypes.byref(cnt), FAKE, 64, None) == dwg.DWG_E_WORKSPACE
    assert lib.dwg_voronoi_area(FAKE, 100, 2, FAKE, FAKE, 1 << 40, None) == dwg.DWG_E_INVALID
    assert lib.dwg_voronoi_area(FAKE, 10, 15, FAKE, FAKE, 1 << 40, None) == dwg.DWG_E_INVALID
    assert lib.dwg_delta_knn_window(FAKE, 100, 10, 0.5, 0.1, FAKE, FAKE, 1 << 40, None) == dwg.DWG_E_INVALID
    assert lib.dwg_init_normals(dwg.INIT_PCA, 0, FAKE, 16, None, FAKE, FAKE, 1 << 40, None) == dwg.DWG_E_INVALID
    assert lib.dwg_init_normals(dwg.INIT_GAUSS, 0, None, 16, None, FAKE, None, 0, None) == dwg.DWG_E_INVALID
    kp = dwg.Params().c()
    ip = dwg.IterateParams(5, 0, 0.1, 0.01)
    for mp in [dwg.McParams(0, 1, 10, 0), dwg.McParams(17, 1, 10, 0), dwg.McParams(8, 3, 10, 0),
               dwg.McParams(8, 1, 0, 0), dwg.McParams(8, 1, 17, 0), dwg.McParams(8, 1, 10, 2),
               dwg.McParams(8, 1, 10, 0, 2), dwg.McParams(8, 1, 10, 0, -1)]:
        assert lib.dwg_mc_workspace_bytes(1000, ctypes.byref(kp), ctypes.byref(mp), 0) == 0
        done = ctypes.c_int(3)
        assert lib.dwg_iterate_mc(FAKE, FAKE, None, 1000, FAKE, ctypes.byref(kp), ctypes.byref(ip), ctypes.byref(mp),
                                  None, ctypes.byref(done), FAKE, 1 << 40, None) == dwg.DWG_E_INVALID
        assert done.value == 0
    good = dwg.McParams(8, 1, 10, 0)
    g = lib.dwg_mc_workspace_bytes(1000, ctypes.byref(kp), ctypes.byref(good), 0)
    assert g > 0 and lib.dwg_mc_workspace_bytes(1000, ctypes.byref(kp), ctypes.byref(good), 500) > g
    # marching tetrahedra keeps room for 12 faces per cell, Marching Cubes for 5
    tets = dwg.McParams(8, 1, 10, 0, 1)
    assert (lib.dwg_mc_workspace_bytes(1000, ctypes.byref(kp), ctypes.byref(tets), 500)
            > lib.dwg_mc_workspace_bytes(1000, ctypes.byref(kp), ctypes.byref(good), 500))
    cells = ctypes.c_int64(9)
    assert lib.dwg_mc_cells(FAKE, 1000, ctypes.byref(good), ctypes.byref(cells), FAKE, 64, None) == dwg.DWG_E_WORKSPACE
    assert cells.value == 0
    ntri, iso = ctypes.c_int64(4), ctypes.c_double(0.0)
    assert lib.dwg_level_set(FAKE, FAKE, FAKE, None, 1000, ctypes.byref(kp), ctypes.byref(good), FAKE, 0,
                             ctypes.byref(ntri), ctypes.byref(iso), FAKE, 1 << 40, None) == dwg.DWG_E_INVALID
    assert ntri.value == 0


def test_static_scratch_entry_validates_before_the_device():
    """dwg_gwn_grad_static rejects NULLs and sizes whose scratch exceeds its static array
    before any HIP call (so on a machine without a GPU too)."""
    lib = dwg.load()
    kp = dwg.Params(lam=10.0).c()
    assert lib.dwg_gwn_grad_static(None, FAKE, FAKE, None, 10, FAKE, 10, ctypes.byref(kp), None, FAKE, None,
                                   None) == dwg.DWG_E_INVALID
    assert lib.dwg_gwn_grad_static(FAKE, FAKE, FAKE, None, 10, FAKE, 10, ctypes.byref(kp), None, None, None,
                                   None) == dwg.DWG_E_INVALID
    assert lib.dwg_gwn_grad_static(FAKE, FAKE, FAKE, None, 700_000, FAKE, 700_000, ctypes.byref(kp), None, FAKE,
                                   None, None) == dwg.DWG_E_INVALID
    assert "static scratch" in lib.dwg_last_error().decode()


def test_single_hip_runtime_in_process():
    """libdwg must bind to the HIP runtime torch already loaded (one libamdhip64 mapped)."""
    dwg.load()
    maps = open("/proc/self/maps").read()
    paths = {line.split()[-1] for line in maps.splitlines() if "libamdhip64" in line}
    assert len(paths) == 1, paths
