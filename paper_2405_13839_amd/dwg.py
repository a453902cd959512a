"""Python binding of libdwg (include/dwg.h): argument marshalling only.

Every function takes and returns torch tensors on a ROCm device; the arithmetic runs in
the library's HIP kernels on the tensor's device and on torch's current stream. The library
must have been built (python -m paper_2405_13839_amd.build); importing this module on a
machine without it raises ImportError -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdwg.so")

DWG_OK, DWG_NOT_CONVERGED = 0, 1
DWG_E_INVALID, DWG_E_WORKSPACE, DWG_E_DEVICE, DWG_E_NONFINITE, DWG_E_UNSUPPORTED = -1, -2, -3, -4, -5
INIT_RANDOM, INIT_MLP, INIT_PCA, INIT_GAUSS = 0, 1, 2, 3
MLP_IN, MLP_HID, MLP_OUT, FEAT_K = 48, 128, 3, 16


class DwgError(RuntimeError):
    def __init__(self, status: int, name: str, detail: str):
        super().__init__(f"{name}: {detail}")
        self.status = status


class KernelParams(ctypes.Structure):
    _fields_ = [("lam", ctypes.c_float), ("eps", ctypes.c_float), ("compensated", ctypes.c_int),
                ("split", ctypes.c_int), ("tree_beta", ctypes.c_float), ("tree_leaf", ctypes.c_int),
                ("reserved", ctypes.c_int * 2)]


class IterateParams(ctypes.Structure):
    _fields_ = [("max_iters", ctypes.c_int), ("fixed_iters", ctypes.c_int), ("eps_deg", ctypes.c_double),
                ("top_frac", ctypes.c_double)]


class McParams(ctypes.Structure):
    _fields_ = [("depth", ctypes.c_int), ("dilate", ctypes.c_int), ("k", ctypes.c_int), ("iso", ctypes.c_int),
                ("surface", ctypes.c_int)]


class IterStat(ctypes.Structure):
    _fields_ = [("wmean", ctypes.c_double), ("top_mean_deg", ctypes.c_double), ("mean_chord", ctypes.c_double),
                ("gwn_ms", ctypes.c_double)]


_lib = None


def load():
    """Load libdwg.so (after torch, so that both share torch's HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2405_13839_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, sz, f32, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_size_t, ctypes.c_float, ctypes.c_int
    kpp = ctypes.POINTER(KernelParams)
    lib.dwg_version.restype = ctypes.c_char_p
    lib.dwg_status_string.restype = ctypes.c_char_p
    lib.dwg_status_string.argtypes = [i32]
    lib.dwg_last_error.restype = ctypes.c_char_p
    lib.dwg_workspace_bytes.restype = sz
    lib.dwg_workspace_bytes.argtypes = [i64, i64, kpp]
    lib.dwg_gwn_eval.argtypes = [vp, vp, vp, vp, i64, vp, i64, kpp, vp, vp, vp, sz, vp]
    lib.dwg_gwn_grad.argtypes = [vp, vp, vp, vp, i64, vp, i64, kpp, vp, vp, vp, vp, sz, vp]
    lib.dwg_gwn_grad_static.argtypes = [vp, vp, vp, vp, i64, vp, i64, kpp, vp, vp, vp, vp]
    lib.dwg_octree_work.argtypes = [vp, vp, vp, i64, vp, i64, kpp, ctypes.POINTER(i64), vp, sz, vp]
    lib.dwg_iterate.argtypes = [vp, vp, vp, i64, vp, kpp, ctypes.POINTER(IterateParams),
                                ctypes.POINTER(IterStat), ctypes.POINTER(ctypes.c_int), vp, sz, vp]
    lib.dwg_init_normals.argtypes = [i32, ctypes.c_uint64, vp, i64, vp, vp, vp, sz, vp]
    lib.dwg_knn.argtypes = [vp, i64, vp, i64, i32, i32, vp, vp, vp, sz, vp]
    lib.dwg_delta_knn_mean.argtypes = [vp, i64, i32, f32, vp, vp, sz, vp]
    lib.dwg_delta_anchor_mean.argtypes = [vp, i64, i32, i64, f32, vp, vp, sz, vp]
    lib.dwg_mlp_param_count.restype = i64
    lib.dwg_mlp_blob_bytes.restype = sz
    lib.dwg_octree.argtypes = [vp, i64, i32, vp, vp, i64, ctypes.POINTER(i64), vp, sz, vp]
    lib.dwg_delta_knn_window.argtypes = [vp, i64, i32, f32, f32, vp, vp, sz, vp]
    mcpp = ctypes.POINTER(McParams)
    lib.dwg_mc_workspace_bytes.restype = sz
    lib.dwg_mc_workspace_bytes.argtypes = [i64, kpp, mcpp, i64]
    lib.dwg_mc_cells.argtypes = [vp, i64, mcpp, ctypes.POINTER(i64), vp, sz, vp]
    lib.dwg_iterate_mc.argtypes = [vp, vp, vp, i64, vp, kpp, ctypes.POINTER(IterateParams), mcpp,
                                   ctypes.POINTER(IterStat), ctypes.POINTER(ctypes.c_int), vp, sz, vp]
    lib.dwg_level_set.argtypes = [vp, vp, vp, vp, i64, kpp, mcpp, vp, i64, ctypes.POINTER(i64),
                                  ctypes.POINTER(ctypes.c_double), vp, sz, vp]
    lib.dwg_voronoi_area.argtypes = [vp, i64, i32, vp, vp, sz, vp]
    lib.dwg_features.argtypes = [vp, i64, i64, vp, vp, sz, vp]
    lib.dwg_mlp_infer.argtypes = [vp, vp, i64, vp, vp, sz, vp]
    lib.dwg_mlp_train_step.argtypes = [vp, vp, vp, i64, f32, vp, vp, vp, i64, vp, vp, vp, sz, vp]
    for name in ["dwg_gwn_eval", "dwg_gwn_grad", "dwg_gwn_grad_static", "dwg_iterate", "dwg_init_normals", "dwg_knn",
                 "dwg_delta_knn_mean", "dwg_delta_anchor_mean", "dwg_features", "dwg_mlp_infer",
                 "dwg_mlp_train_step", "dwg_octree", "dwg_octree_work", "dwg_delta_knn_window", "dwg_voronoi_area",
                 "dwg_mc_cells", "dwg_iterate_mc", "dwg_level_set"]:
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


EXPORTED = ["dwg_version", "dwg_status_string", "dwg_last_error", "dwg_workspace_bytes", "dwg_gwn_eval",
            "dwg_gwn_grad", "dwg_gwn_grad_static", "dwg_iterate", "dwg_init_normals", "dwg_knn", "dwg_delta_knn_mean",
            "dwg_delta_anchor_mean", "dwg_mlp_param_count", "dwg_mlp_blob_bytes", "dwg_features", "dwg_mlp_infer",
            "dwg_mlp_train_step", "dwg_octree", "dwg_octree_work", "dwg_delta_knn_window", "dwg_voronoi_area",
            "dwg_mc_workspace_bytes", "dwg_mc_cells", "dwg_iterate_mc", "dwg_level_set"]


def version() -> str:
    return load().dwg_version().decode()


def _check(status: int, ok=(DWG_OK,)):
    if status not in ok:
        lib = load()
        raise DwgError(status, lib.dwg_status_string(status).decode(), lib.dwg_last_error().decode())
    return status


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dev(t, name, dtype=torch.float32, shape=None, device=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on a ROCm device (got {t.device})")
    if device is not None and t.device != device:
        raise ValueError(f"{name} must be on {device} like the points (got {t.device})")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype} (got {t.dtype})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)} (got {tuple(t.shape)})")
    return t


def _pts(t, name, device=None):
    """A planar [3, n] float32 point array (x, y, z rows), n >= 1."""
    t = _dev(t, name, device=device)
    if t.dim() != 2 or t.shape[0] != 3 or t.shape[1] < 1:
        raise ValueError(f"{name} must have shape (3, n) with n >= 1 (got {tuple(t.shape)})")
    return t


def _run(device, fn, *args):
    """Calls the C entry point with `device` current: the library launches on the current
    HIP device, the tensors' device."""
    with torch.cuda.device(device):
        return fn(*args)


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


@dataclass
class Params:
    lam: float = 0.0
    eps: float = 0.0
    compensated: bool = True
    split: int = 0
    beta: float = 0.0  # 0 = exact all-pairs sum; >= 1 = octree traversal (paper: 2.3)
    leaf: int = 0      # octree leaf capacity (0 = 32)

    def c(self):
        return KernelParams(float(self.lam), float(self.eps), int(bool(self.compensated)), int(self.split),
                            float(self.beta), int(self.leaf), (ctypes.c_int * 2)(0, 0))


def workspace_bytes(n_src: int, n_qry: int, params: Params | None = None) -> int:
    kp = (params or Params()).c()
    return int(load().dwg_workspace_bytes(int(n_src), int(n_qry), ctypes.byref(kp)))


def workspace(n_src: int, n_qry: int, device, params: Params | None = None, *more: Params) -> torch.Tensor:
    """A workspace for calls with any of the given parameter sets (the largest size)."""
    size = max(workspace_bytes(n_src, n_qry, p) for p in (params, *more))
    return torch.empty(max(1, size), dtype=torch.uint8, device=device)


def gwn(P, N, area, delta, Q, params: Params | None = None, grad=True, ws=None, want_wmean=False):
    """w [m] and (if grad) grad w [3, m] of the (screened) GWN of the oriented cloud at Q."""
    lib = load()
    params = params or Params()
    P = _pts(P, "P")
    n = P.shape[1]
    dev = P.device
    _dev(N, "N", shape=(3, n), device=dev)
    _dev(area, "area", shape=(n,), device=dev)
    if delta is not None:
        _dev(delta, "delta", shape=(n,), device=dev)
    Q = _pts(Q, "Q", device=dev)
    m = Q.shape[1]
    if ws is None:
        ws = workspace(n, m, dev, params)
    _dev(ws, "ws", dtype=torch.uint8, device=dev)
    w = torch.empty(m, dtype=torch.float32, device=dev)
    wm = torch.empty(1, dtype=torch.float64, device=dev) if want_wmean else None
    kp = params.c()
    if grad:
        g = torch.empty((3, m), dtype=torch.float32, device=dev)
        _check(_run(dev, lib.dwg_gwn_grad, _ptr(P), _ptr(N), _ptr(area), _ptr(delta), n, _ptr(Q), m, ctypes.byref(kp),
            _ptr(w), _ptr(g), _ptr(wm), _ptr(ws), ws.numel(), _stream(dev)))
        return (w, g, wm) if want_wmean else (w, g)
    _check(_run(dev, lib.dwg_gwn_eval, _ptr(P), _ptr(N), _ptr(area), _ptr(delta), n, _ptr(Q), m, ctypes.byref(kp),
        _ptr(w), _ptr(wm), _ptr(ws), ws.numel(), _stream(dev)))
    return (w, wm) if want_wmean else w


def gwn_static(P, N, area, delta, Q, params: Params | None = None, want_wmean=False):
    """w [m] and grad w [3, m] through dwg_gwn_grad_static (no workspace: the library's
    static scratch; sizes whose scratch exceeds it raise)."""
    lib = load()
    params = params or Params()
    P = _pts(P, "P")
    n = P.shape[1]
    dev = P.device
    _dev(N, "N", shape=(3, n), device=dev)
    _dev(area, "area", shape=(n,), device=dev)
    if delta is not None:
        _dev(delta, "delta", shape=(n,), device=dev)
    Q = _pts(Q, "Q", device=dev)
    m = Q.shape[1]
    w = torch.empty(m, dtype=torch.float32, device=dev)
    g = torch.empty((3, m), dtype=torch.float32, device=dev)
    wm = torch.empty(1, dtype=torch.float64, device=dev) if want_wmean else None
    kp = params.c()
    _check(_run(dev, lib.dwg_gwn_grad_static, _ptr(P), _ptr(N), _ptr(area), _ptr(delta), n, _ptr(Q), m,
                ctypes.byref(kp), _ptr(w), _ptr(g), _ptr(wm), _stream(dev)))
    return (w, g, wm) if want_wmean else (w, g)


def iterate(P, area, delta, N, params: Params | None = None, max_iters=50, fixed_iters=False, eps_deg=0.1,
            top_frac=0.01, ws=None):
    """Run Algorithm 1 in place on N ([3, n] float32). Returns (status, stats float64 [T, 4]):
    per iteration wmean, top-1% mean angle change (deg), mean chord, all-pairs kernel ms."""
    lib = load()
    params = params or Params()
    P = _pts(P, "P")
    n = P.shape[1]
    _dev(area, "area", shape=(n,), device=P.device)
    if delta is not None:
        _dev(delta, "delta", shape=(n,), device=P.device)
    _dev(N, "N", shape=(3, n), device=P.device)
    dev = P.device
    if ws is None:
        ws = workspace(n, n, dev, params)
    _dev(ws, "ws", dtype=torch.uint8, device=dev)
    kp = params.c()
    ip = IterateParams(int(max_iters), int(bool(fixed_iters)), float(eps_deg), float(top_frac))
    stats = (IterStat * int(max_iters))()
    done = ctypes.c_int(0)
    st = _run(dev, lib.dwg_iterate, _ptr(P), _ptr(area), _ptr(delta), n, _ptr(N), ctypes.byref(kp), ctypes.byref(ip),
        stats, ctypes.byref(done), _ptr(ws), ws.numel(), _stream(dev))
    _check(st, ok=(DWG_OK, DWG_NOT_CONVERGED))
    out = torch.tensor([[s.wmean, s.top_mean_deg, s.mean_chord, s.gwn_ms] for s in stats[: done.value]],
                       dtype=torch.float64).reshape(-1, 4)
    return st, out


def mc_workspace(P, params: Params | None = None, depth: int = 8, dilate: int = 1, k: int = 10,
                 iso: str = "points", surface: str = "cubes") -> torch.Tensor:
    """Workspace for iterate_mc / level_set on P: sized for the actual number of grid cells."""
    lib = load()
    P = _pts(P, "P")
    n = P.shape[1]
    kp = (params or Params()).c()
    mp = McParams(int(depth), int(dilate), int(k), _iso(iso), _surface(surface))
    g = int(lib.dwg_mc_workspace_bytes(n, ctypes.byref(kp), ctypes.byref(mp), 0))
    if g == 0:
        raise DwgError(DWG_E_INVALID, "DWG_E_INVALID", "invalid level-set parameters")
    gws = torch.empty(g, dtype=torch.uint8, device=P.device)
    cells = ctypes.c_int64(0)
    _check(_run(P.device, lib.dwg_mc_cells, _ptr(P), n, ctypes.byref(mp), ctypes.byref(cells), _ptr(gws), gws.numel(),
        _stream(P.device)))
    del gws
    total = int(lib.dwg_mc_workspace_bytes(n, ctypes.byref(kp), ctypes.byref(mp), cells.value))
    return torch.empty(total, dtype=torch.uint8, device=P.device)


def _surface(surface: str) -> int:
    """'cubes' = Marching Cubes (the paper's extraction), 'tets' = marching tetrahedra."""
    if surface not in ("cubes", "tets"):
        raise ValueError("surface must be 'cubes' or 'tets'")
    return 0 if surface == "cubes" else 1


def _iso(iso: str) -> int:
    if iso not in ("points", "corners"):
        raise ValueError("iso must be 'points' or 'corners'")
    return 0 if iso == "points" else 1


def iterate_mc(P, area, delta, N, params: Params | None = None, depth=8, dilate=1, k=10, max_iters=50,
               fixed_iters=False, eps_deg=0.1, top_frac=0.01, ws=None, iso: str = "points", surface: str = "cubes"):
    """Algorithm 1 with the paper's level-set update, in place on N. Returns (status, stats
    float64 [T, 4]): per iteration w_bar (over the points, or the grid corners with
    iso='corners'), top-1% mean angle change, mean chord, evaluation ms."""
    lib = load()
    params = params or Params()
    P = _pts(P, "P")
    n = P.shape[1]
    _dev(area, "area", shape=(n,), device=P.device)
    if delta is not None:
        _dev(delta, "delta", shape=(n,), device=P.device)
    _dev(N, "N", shape=(3, n), device=P.device)
    if ws is None:
        ws = mc_workspace(P, params, depth, dilate, k, iso, surface)
    _dev(ws, "ws", dtype=torch.uint8, device=P.device)
    kp = params.c()
    mp = McParams(int(depth), int(dilate), int(k), _iso(iso), _surface(surface))
    ip = IterateParams(int(max_iters), int(bool(fixed_iters)), float(eps_deg), float(top_frac))
    stats = (IterStat * int(max_iters))()
    done = ctypes.c_int(0)
    st = _run(P.device, lib.dwg_iterate_mc, _ptr(P), _ptr(area), _ptr(delta), n, _ptr(N), ctypes.byref(kp),
        ctypes.byref(ip), ctypes.byref(mp), stats, ctypes.byref(done), _ptr(ws), ws.numel(), _stream(P.device))
    _check(st, ok=(DWG_OK, DWG_NOT_CONVERGED))
    out = torch.tensor([[s.wmean, s.top_mean_deg, s.mean_chord, s.gwn_ms] for s in stats[: done.value]],
                       dtype=torch.float64).reshape(-1, 4)
    return st, out


def level_set(P, N, area, delta, params: Params | None = None, depth=8, dilate=1, ws=None, iso: str = "points",
              surface: str = "cubes"):
    """The w_bar level set: (triangles float32 [F, 3, 3] wound outwards, w_bar)."""
    lib = load()
    params = params or Params()
    P = _pts(P, "P")
    n = P.shape[1]
    if ws is None:
        ws = mc_workspace(P, params, depth, dilate, 10, iso, surface)
    _dev(ws, "ws", dtype=torch.uint8, device=P.device)
    kp = params.c()
    mp = McParams(int(depth), int(dilate), 10, _iso(iso), _surface(surface))
    ntri = ctypes.c_int64(0)
    iso = ctypes.c_double(0.0)
    tri = torch.empty((1, 9), dtype=torch.float32, device=P.device)
    args = lambda t: (_ptr(P), _ptr(N), _ptr(area), _ptr(delta), n, ctypes.byref(kp), ctypes.byref(mp), _ptr(t),
                      t.shape[0], ctypes.byref(ntri), ctypes.byref(iso), _ptr(ws), ws.numel(), _stream(P.device))
    st = _run(P.device, lib.dwg_level_set, *args(tri))
    if st == DWG_E_INVALID and ntri.value > 1:
        tri = torch.empty((ntri.value, 9), dtype=torch.float32, device=P.device)
        st = _run(P.device, lib.dwg_level_set, *args(tri))
    _check(st)
    return tri[: ntri.value].reshape(-1, 3, 3), iso.value


def random_normals(n: int, seed: int, device) -> torch.Tensor:
    lib = load()
    N = torch.empty((3, n), dtype=torch.float32, device=device)
    _check(_run(N.device, lib.dwg_init_normals, INIT_RANDOM, ctypes.c_uint64(seed), None, n, None, _ptr(N), None, 0,
        _stream(N.device)))
    return N


def voronoi_area(P, m: int = 15, ws=None) -> torch.Tensor:
    """Tangent-plane Voronoi area weights [n] (Sec. 5.1)."""
    lib = load()
    P = _pts(P, "P")
    n = P.shape[1]
    if ws is None:
        ws = workspace(n, n, P.device)
    _dev(ws, "ws", dtype=torch.uint8, device=P.device)
    out = torch.empty(n, dtype=torch.float32, device=P.device)
    _check(_run(P.device, lib.dwg_voronoi_area, _ptr(P), n, int(m), _ptr(out), _ptr(ws), ws.numel(), _stream(P.device)))
    return out


def delta_knn_window(P, k: int = 10, vmin: float = 0.0015, vmax: float = 0.015, ws=None) -> torch.Tensor:
    """The paper's windowed k-NN kernel radius [n] (Sec. 5.2)."""
    lib = load()
    P = _pts(P, "P")
    n = P.shape[1]
    if ws is None:
        ws = workspace(n, n, P.device)
    _dev(ws, "ws", dtype=torch.uint8, device=P.device)
    out = torch.empty(n, dtype=torch.float32, device=P.device)
    _check(_run(P.device, lib.dwg_delta_knn_window, _ptr(P), n, int(k), ctypes.c_float(vmin), ctypes.c_float(vmax),
        _ptr(out), _ptr(ws), ws.numel(), _stream(P.device)))
    return out


def octree(P, leaf: int = 0, ws=None):
    """Octree of the octree mode: (perm int32 [n], nodes int32 [count, 4] = (start, end,
    level, skip) in depth-first pre-order), both on P's device."""
    lib = load()
    P = _pts(P, "P")
    n = P.shape[1]
    if ws is None:
        ws = workspace(n, n, P.device, Params(beta=2.3, leaf=leaf))
    _dev(ws, "ws", dtype=torch.uint8, device=P.device)
    perm = torch.empty(n, dtype=torch.int32, device=P.device)
    cap = 2 * n
    nodes = torch.empty((cap, 4), dtype=torch.int32, device=P.device)
    cnt = ctypes.c_int64(0)
    _check(_run(P.device, lib.dwg_octree, _ptr(P), n, int(leaf), _ptr(perm), _ptr(nodes), cap, ctypes.byref(cnt),
        _ptr(ws), ws.numel(), _stream(P.device)))
    return perm, nodes[:cnt.value]


@dataclass(frozen=True)
class OctreeWork:
    """Work of one octree evaluation, totalled over the queries (dwg_octree_work)."""
    far: int         # (query, node) pairs taken as one dipole
    pairs: int       # (query, source) pairs summed at leaves
    far_steps: int   # wavefront steps with at least one query taking the node as a dipole
    leaf_steps: int  # source iterations of the wavefronts' leaf loops

    @property
    def far_lanes(self) -> float:
        """Fraction of the lanes of the far steps that add a dipole."""
        return self.far / (64 * self.far_steps) if self.far_steps else 0.0

    @property
    def leaf_lanes(self) -> float:
        """Fraction of the lanes of the leaf-loop iterations that add a pair."""
        return self.pairs / (64 * self.leaf_steps) if self.leaf_steps else 0.0


def octree_work(P, area, delta, Q, params: Params, ws=None) -> OctreeWork:
    """Work of the octree traversal for the queries Q (decisions only, no arithmetic)."""
    lib = load()
    P = _pts(P, "P")
    n = P.shape[1]
    _dev(area, "area", shape=(n,), device=P.device)
    if delta is not None:
        _dev(delta, "delta", shape=(n,), device=P.device)
    Q = _pts(Q, "Q", device=P.device)
    m = Q.shape[1]
    if ws is None:
        ws = workspace(n, m, P.device, params)
    _dev(ws, "ws", dtype=torch.uint8, device=P.device)
    kp = params.c()
    work = (ctypes.c_int64 * 4)()
    _check(_run(P.device, lib.dwg_octree_work, _ptr(P), _ptr(area), _ptr(delta), n, _ptr(Q), m, ctypes.byref(kp),
                work, _ptr(ws), ws.numel(), _stream(P.device)))
    return OctreeWork(*(int(v) for v in work))


def pca_normals(P, ws=None) -> torch.Tensor:
    """Smallest-eigenvalue eigenvector of each point's 16-NN covariance, [3, n]."""
    lib = load()
    P = _pts(P, "P")
    n = P.shape[1]
    if ws is None:
        ws = workspace(n, n, P.device)
    _dev(ws, "ws", dtype=torch.uint8, device=P.device)
    N = torch.empty((3, n), dtype=torch.float32, device=P.device)
    _check(_run(P.device, lib.dwg_init_normals, INIT_PCA, ctypes.c_uint64(0), _ptr(P), n, None, _ptr(N), _ptr(ws),
        ws.numel(), _stream(P.device)))
    return N


def gauss_normals(P) -> torch.Tensor:
    """Gauss map p / |p|, [3, n]."""
    lib = load()
    P = _pts(P, "P")
    n = P.shape[1]
    N = torch.empty((3, n), dtype=torch.float32, device=P.device)
    _check(_run(P.device, lib.dwg_init_normals, INIT_GAUSS, ctypes.c_uint64(0), _ptr(P), n, None, _ptr(N), None, 0,
        _stream(P.device)))
    return N


def mlp_normals(P, mlp_params, ws=None) -> torch.Tensor:
    lib = load()
    P = _pts(P, "P")
    n = P.shape[1]
    _dev(mlp_params, "mlp_params", shape=(mlp_param_count(),), device=P.device)
    if ws is None:
        ws = workspace(n, n, P.device)
    _dev(ws, "ws", dtype=torch.uint8, device=P.device)
    N = torch.empty((3, n), dtype=torch.float32, device=P.device)
    _check(_run(P.device, lib.dwg_init_normals, INIT_MLP, ctypes.c_uint64(0), _ptr(P), n, _ptr(mlp_params), _ptr(N),
        _ptr(ws), ws.numel(), _stream(P.device)))
    return N


def knn(R, Q, k: int, self_skip: bool = False, ws=None, want_dist=True):
    """(idx int32 [m, k], dist float32 [m, k]) of the k nearest points of R for each query."""
    lib = load()
    R = _pts(R, "R")
    Q = _pts(Q, "Q", device=R.device)
    nr, m = R.shape[1], Q.shape[1]
    if ws is None:
        ws = workspace(nr, m, R.device)
    _dev(ws, "ws", dtype=torch.uint8, device=R.device)
    idx = torch.empty((m, k), dtype=torch.int32, device=R.device)
    dist = torch.empty((m, k), dtype=torch.float32, device=R.device) if want_dist else None
    _check(_run(R.device, lib.dwg_knn, _ptr(R), nr, _ptr(Q), m, int(bool(self_skip)), int(k), _ptr(idx), _ptr(dist),
        _ptr(ws), ws.numel(), _stream(R.device)))
    return idx, dist


def delta_knn_mean(P, k: int = 10, scale: float = 1.0, ws=None) -> torch.Tensor:
    lib = load()
    P = _pts(P, "P")
    n = P.shape[1]
    if ws is None:
        ws = workspace(n, n, P.device)
    _dev(ws, "ws", dtype=torch.uint8, device=P.device)
    out = torch.empty(n, dtype=torch.float32, device=P.device)
    _check(_run(P.device, lib.dwg_delta_knn_mean, _ptr(P), n, int(k), float(scale), _ptr(out), _ptr(ws), ws.numel(),
        _stream(P.device)))
    return out


def delta_anchor_mean(P, k: int = 10, n_anchor: int = 4096, scale: float = 1.0, ws=None) -> torch.Tensor:
    """scale x mean distance to the k nearest of ~n_anchor anchor points, [n]."""
    lib = load()
    P = _pts(P, "P")
    n = P.shape[1]
    if ws is None:
        ws = workspace(n, n, P.device)
    _dev(ws, "ws", dtype=torch.uint8, device=P.device)
    out = torch.empty(n, dtype=torch.float32, device=P.device)
    _check(_run(P.device, lib.dwg_delta_anchor_mean, _ptr(P), n, int(k), int(n_anchor), float(scale), _ptr(out),
        _ptr(ws), ws.numel(), _stream(P.device)))
    return out


def mlp_param_count() -> int:
    return int(load().dwg_mlp_param_count())


def mlp_blob_bytes() -> int:
    return int(load().dwg_mlp_blob_bytes())


def features(P, n_anchor: int = 4096, ws=None) -> torch.Tensor:
    lib = load()
    P = _pts(P, "P")
    n = P.shape[1]
    if ws is None:
        ws = workspace(n, n, P.device)
    _dev(ws, "ws", dtype=torch.uint8, device=P.device)
    out = torch.empty((n, MLP_IN), dtype=torch.float32, device=P.device)
    _check(_run(P.device, lib.dwg_features, _ptr(P), n, int(n_anchor), _ptr(out), _ptr(ws), ws.numel(),
        _stream(P.device)))
    return out


def mlp_infer(params, X, ws=None) -> torch.Tensor:
    lib = load()
    X = _dev(X, "X")
    B = X.shape[0]
    _dev(params, "params", shape=(mlp_param_count(),), device=X.device)
    if ws is None:
        ws = workspace(B, B, X.device)
    _dev(ws, "ws", dtype=torch.uint8, device=X.device)
    Y = torch.empty((B, MLP_OUT), dtype=torch.float32, device=X.device)
    _check(_run(X.device, lib.dwg_mlp_infer, _ptr(params), _ptr(X), B, _ptr(Y), _ptr(ws), ws.numel(),
        _stream(X.device)))
    return Y


def mlp_train_step(params, adam_m, adam_v, step: int, lr: float, X, T, mask=None, ws=None, want_grad=False):
    """One Adam step in place on params / adam_m / adam_v. Returns (loss tensor [1], grad or None)."""
    lib = load()
    X = _dev(X, "X")
    B = X.shape[0]
    npar = mlp_param_count()
    for t, nm in [(params, "params"), (adam_m, "adam_m"), (adam_v, "adam_v")]:
        _dev(t, nm, shape=(npar,), device=X.device)
    _dev(T, "T", shape=(B, 3), device=X.device)
    if mask is not None:
        _dev(mask, "mask", dtype=torch.uint8, shape=(B,), device=X.device)
    if ws is None:
        ws = workspace(B, B, X.device)
    _dev(ws, "ws", dtype=torch.uint8, device=X.device)
    loss = torch.empty(1, dtype=torch.float32, device=X.device)
    grad = torch.empty(npar, dtype=torch.float32, device=X.device) if want_grad else None
    _check(_run(X.device, lib.dwg_mlp_train_step, _ptr(params), _ptr(adam_m), _ptr(adam_v), int(step), float(lr),
        _ptr(X), _ptr(T), _ptr(mask), B, _ptr(grad), _ptr(loss), _ptr(ws), ws.numel(), _stream(X.device)))
    return loss, grad


def top_count(n: int, top_frac: float = 0.01) -> int:
    """Number of largest normal changes the convergence statistic averages."""
    return max(1, min(n, int(math.ceil(top_frac * n))))
