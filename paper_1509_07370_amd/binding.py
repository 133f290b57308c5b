"""Thin ctypes binding of libbh.so (C ABI in include/bh.h).

Functions keep the C names and only marshal arguments: torch tensors are
passed by device pointer, the HIP stream is torch's current stream, results
stay in caller-owned tensors.  Every step of the method runs in the HIP
kernels of the library; if the library is missing this module raises on
import -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# BH_LIBRARY selects another build of the same library (e.g. a tuning variant)
LIB_PATH = os.environ.get("BH_LIBRARY") or os.path.join(HERE, "libbh.so")

BH_OK, BH_EINVAL, BH_ENOMEM, BH_EDEVICE, BH_ECAPACITY, BH_ESTATE = 0, -1, -2, -3, -4, -5
BH_FP64, BH_FP32 = 0, 1
_CODES = {BH_EINVAL: "BH_EINVAL", BH_ENOMEM: "BH_ENOMEM", BH_EDEVICE: "BH_EDEVICE", BH_ECAPACITY: "BH_ECAPACITY",
          BH_ESTATE: "BH_ESTATE"}

if not os.path.exists(LIB_PATH):
    raise ImportError("libbh.so is not built (run `python -m paper_1509_07370_amd.build`); "
                      "the Barnes-Hut path has no CPU fallback")

_lib = ctypes.CDLL(LIB_PATH)
P = ctypes.c_void_p
PP = ctypes.POINTER(ctypes.c_void_p)
i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double


class GridInfo(ctypes.Structure):
    _fields_ = [("n_nodes", i64), ("n_leaf", i64), ("n_cells", i64), ("n_groups", i64), ("group_cells", i32),
                ("nbase", i32), ("max_depth", i32), ("n_levels", i32)]


class BatchConfig(ctypes.Structure):
    _fields_ = [("order", i32), ("workgroups_per_cu", i32), ("waves_per_simd", i32), ("stack_limit", i32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class BatchTiming(ctypes.Structure):
    _fields_ = [("config", BatchConfig), ("ms", ctypes.c_float)]


_SIGS = {
    "bh_ctx_create": (ctypes.c_int, [PP, ctypes.c_int, P]),
    "bh_ctx_set_stream": (ctypes.c_int, [P, P]),
    "bh_ctx_destroy": (ctypes.c_int, [P]),
    "bh_last_error": (ctypes.c_char_p, [P]),
    "bh_create_error": (ctypes.c_char_p, []),
    "bh_grid_create": (ctypes.c_int, [P, PP, ctypes.c_int, ctypes.c_int, P, P, P, P, P, P, f64, ctypes.c_int]),
    "bh_grid_destroy": (ctypes.c_int, [P]),
    "bh_grid_info": (ctypes.c_int, [P, ctypes.POINTER(GridInfo)]),
    "bh_grid_node_keys": (ctypes.c_int, [P, P]),
    "bh_build_moments": (ctypes.c_int, [P, P, P, PP]),
    "bh_moments_check": (ctypes.c_int, [P, P]),
    "bh_moments_export": (ctypes.c_int, [P, P, P, P, P, P]),
    "bh_moments_destroy": (ctypes.c_int, [P]),
    "bh_walk": (ctypes.c_int, [P, P, P, f64, P, ctypes.c_int, PP]),
    "bh_lists_info": (ctypes.c_int, [P, ctypes.POINTER(i64), ctypes.POINTER(i64)]),
    "bh_lists_export": (ctypes.c_int, [P, P, P, P, P, P]),
    "bh_lists_destroy": (ctypes.c_int, [P]),
    "bh_potential": (ctypes.c_int, [P, P, P, P, f64, ctypes.c_int, P]),
    "bh_walk_potential": (ctypes.c_int, [P, P, P, f64, P, ctypes.c_int, f64, P, P]),
    "bh_potential_static": (ctypes.c_int, [P, P, P, f64, P, ctypes.c_int, f64, P, P, P]),
    "bh_walk_potential_ex": (ctypes.c_int, [P, P, P, f64, P, ctypes.c_int, f64, P, P, P]),
    "bh_walk_accel": (ctypes.c_int, [P, P, P, f64, P, ctypes.c_int, f64, P, P, P]),
    "bh_direct_accel": (ctypes.c_int, [P, P, P, P, i64, f64, P]),
    "bh_direct": (ctypes.c_int, [P, P, P, P, i64, f64, P]),
    "bh_ewald_create": (ctypes.c_int, [P, f64, ctypes.c_int, PP]),
    "bh_ewald_destroy": (ctypes.c_int, [P]),
    "bh_ewald_export": (ctypes.c_int, [P, P, P]),
    "bh_ewald_near_series": (ctypes.c_int, [P, P, P, P, P]),
    "bh_ewald_set_local_budget": (ctypes.c_int, [P, P, f64, P]),
    "bh_moments_export_trace": (ctypes.c_int, [P, P, P]),
    "bh_walk_potential_periodic": (ctypes.c_int, [P, P, P, P, f64, P, ctypes.c_int, f64, P, P]),
    "bh_direct_periodic": (ctypes.c_int, [P, P, P, P, P, i64, f64, P]),
    "bh_batch_create": (ctypes.c_int, [P, PP, ctypes.c_int, P]),
    "bh_batch_destroy": (ctypes.c_int, [P]),
    "bh_batch_info": (ctypes.c_int, [P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(i64)]),
    "bh_batch_solve": (ctypes.c_int, [P, P, P, P, f64, P, ctypes.c_int, f64]),
    "bh_batch_solve_periodic": (ctypes.c_int, [P, P, P, P, P, f64, P, ctypes.c_int, f64]),
    "bh_batch_capture": (ctypes.c_int, [P, P, P, P, f64, P, ctypes.c_int, f64]),
    "bh_batch_replay": (ctypes.c_int, [P, P]),
    "bh_batch_check": (ctypes.c_int, [P, P]),
    "bh_batch_counts": (ctypes.c_int, [P, P, P]),
    "bh_batch_schedule": (ctypes.c_int, [P, P, ctypes.c_int]),
    "bh_batch_set_launch": (ctypes.c_int, [P, P, ctypes.c_int]),
    "bh_batch_configure": (ctypes.c_int, [P, P, P]),
    "bh_batch_get_config": (ctypes.c_int, [P, P]),
    "bh_batch_autotune": (ctypes.c_int, [P, P, P, P, f64, P, ctypes.c_int, f64, ctypes.c_int, P, P, P,
                                         ctypes.c_int, P]),
    "bh_group_features": (ctypes.c_int, [P, P, P, P]),
    "bh_group_rms_error": (ctypes.c_int, [P, P, P, P, P]),
    "bh_mlp_create": (ctypes.c_int, [P, PP, P, P, P]),
    "bh_mlp_set_params": (ctypes.c_int, [P, P, P]),
    "bh_mlp_set_theta_floor": (ctypes.c_int, [P, P, ctypes.c_float]),
    "bh_mlp_get_params": (ctypes.c_int, [P, P, P]),
    "bh_mlp_forward": (ctypes.c_int, [P, P, P, i64, ctypes.c_int, ctypes.c_float, P]),
    "bh_mlp_grad": (ctypes.c_int, [P, P, P, P, i64, P, P]),
    "bh_learned_walk_potential": (ctypes.c_int, [P, P, P, P, ctypes.c_float, ctypes.c_int, f64, P, P, P]),
    "bh_theta_infer": (ctypes.c_int, [P, P, P, P, ctypes.c_float, P]),
    "bh_mlp_adam_step": (ctypes.c_int, [P, P, P, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float]),
    "bh_mlp_destroy": (ctypes.c_int, [P]),
}
MLP_INPUTS, MLP_HIDDEN, MLP_PARAMS = 12, 64, 5057
BH_ORDER_NATURAL, BH_ORDER_COST = 0, 1
BH_MAC_CELLS, BH_MAC_GROUP_BOX = 0, 1
for _name, (_res, _args) in _SIGS.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args

EXPORTED = tuple(_SIGS)


class BHError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (_CODES.get(code, code), msg))
        self.code = code


def _check(rc, ctx):
    if rc != BH_OK:
        msg = _lib.bh_last_error(ctx).decode() if ctx else _lib.bh_create_error().decode()
        raise BHError(rc, msg)


def _np(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _dev(t, dtype_name):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    if str(t.dtype) != "torch." + dtype_name:
        raise TypeError("tensor must be %s, got %s" % (dtype_name, t.dtype))
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _current_stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


# ------------------------------------------------------------------ context

def bh_ctx_create(device: int = 0, stream=None):
    """device -1 gives a host-only context (topology only)."""
    h = ctypes.c_void_p()
    if stream is None and device >= 0:
        import torch
        torch.cuda.set_device(device)
        stream = _current_stream()
    _check(_lib.bh_ctx_create(ctypes.byref(h), int(device), stream), None)
    return h


def bh_ctx_set_stream(ctx, stream=None):
    _check(_lib.bh_ctx_set_stream(ctx, _current_stream() if stream is None else stream), ctx)


def bh_ctx_destroy(ctx):
    _lib.bh_ctx_destroy(ctx)


def bh_last_error(ctx) -> str:
    return _lib.bh_last_error(ctx).decode()


# ------------------------------------------------------------------ grid

def bh_grid_create(ctx, level, lo, parent, child, is_leaf, box_lo, box_size, group_cells=64, nb=8):
    arrs = [_np(level, np.int32), _np(lo, np.float64), _np(parent, np.int32), _np(child, np.int32),
            _np(is_leaf, np.uint8), _np(box_lo, np.float64)]
    h = ctypes.c_void_p()
    _check(_lib.bh_grid_create(ctx, ctypes.byref(h), int(arrs[0].size), int(nb), *[_ptr(a) for a in arrs],
                               float(box_size), int(group_cells)), ctx)
    return h


def bh_grid_create_from(ctx, grid, group_cells=64):
    """bh_grid_create from an object with level/lo/parent/child/is_leaf/box_lo/box_size attributes."""
    return bh_grid_create(ctx, grid.level, grid.lo, grid.parent, grid.child, grid.is_leaf, grid.box_lo,
                          grid.box_size, group_cells)


def bh_grid_destroy(grid):
    _lib.bh_grid_destroy(grid)


def bh_grid_info(grid) -> dict:
    info = GridInfo()
    _check(_lib.bh_grid_info(grid, ctypes.byref(info)), None)
    return {name: getattr(info, name) for name, _ in GridInfo._fields_}


def bh_grid_node_keys(grid) -> np.ndarray:
    n = bh_grid_info(grid)["n_nodes"]
    keys = np.empty(n, np.uint64)
    _check(_lib.bh_grid_node_keys(grid, _ptr(keys)), None)
    return keys


# ------------------------------------------------------------------ moments

def bh_build_moments(ctx, grid, rho, m=None):
    """rho: float64 CUDA tensor [n_leaf, 8, 8, 8].  Returns the moments handle."""
    h = m if m is not None else ctypes.c_void_p()
    _check(_lib.bh_build_moments(ctx, grid, _dev(rho, "float64"), ctypes.byref(h)), ctx)
    return h


def bh_moments_check(ctx, m):
    _check(_lib.bh_moments_check(ctx, m), ctx)


def bh_moments_export(ctx, m, n_nodes):
    M = np.empty(n_nodes)
    X = np.empty((n_nodes, 3))
    Q = np.empty((n_nodes, 6))
    d = np.empty(n_nodes)
    _check(_lib.bh_moments_export(ctx, m, _ptr(M), _ptr(X), _ptr(Q), _ptr(d)), ctx)
    return dict(M=M, X=X, Q=Q, delta=d)


def bh_moments_destroy(m):
    _lib.bh_moments_destroy(m)


# ------------------------------------------------------------------ walk

def bh_walk(ctx, grid, m, theta=0.5, theta_group=None, precision=BH_FP32, lists=None):
    h = lists if lists is not None else ctypes.c_void_p()
    tg = _dev(theta_group, "float32") if theta_group is not None else None
    _check(_lib.bh_walk(ctx, grid, m, float(theta), tg, int(precision), ctypes.byref(h)), ctx)
    return h


def bh_lists_info(lists):
    a, b = i64(), i64()
    _check(_lib.bh_lists_info(lists, ctypes.byref(a), ctypes.byref(b)), None)
    return a.value, b.value


def bh_lists_export(ctx, lists, n_groups):
    nf, nn = bh_lists_info(lists)
    fo = np.empty(n_groups + 1, np.int64)
    no = np.empty(n_groups + 1, np.int64)
    fa = np.empty(max(nf, 1), np.int32)
    na = np.empty(max(nn, 1), np.int32)
    _check(_lib.bh_lists_export(ctx, lists, _ptr(fo), _ptr(fa), _ptr(no), _ptr(na)), ctx)
    return dict(far_off=fo, far_node=fa[:nf], near_off=no, near_node=na[:nn])


def bh_lists_destroy(lists):
    _lib.bh_lists_destroy(lists)


# ------------------------------------------------------------------ sums

def bh_potential(ctx, grid, m, lists, G, precision, phi):
    _check(_lib.bh_potential(ctx, grid, m, lists, float(G), int(precision), _dev(phi, "float64")), ctx)
    return phi


def bh_walk_potential(ctx, grid, m, theta, theta_group, precision, G, phi, counts=None):
    tg = _dev(theta_group, "float32") if theta_group is not None else None
    cn = _dev(counts, "int32") if counts is not None else None
    _check(_lib.bh_walk_potential(ctx, grid, m, float(theta), tg, int(precision), float(G), _dev(phi, "float64"), cn),
           ctx)
    return phi


def bh_potential_static(ctx, grid, rho, theta, theta_group, precision, G, phi, counts=None, status=None):
    tg = _dev(theta_group, "float32") if theta_group is not None else None
    cn = _dev(counts, "int32") if counts is not None else None
    st = _dev(status, "int32") if status is not None else None
    _check(_lib.bh_potential_static(ctx, grid, _dev(rho, "float64"), float(theta), tg, int(precision), float(G),
                                    _dev(phi, "float64"), cn, st), ctx)
    return phi


class WalkOptions(ctypes.Structure):
    _fields_ = [("mac", i32), ("order", i32)]


def bh_walk_potential_ex(ctx, grid, m, theta, theta_group, precision, G, phi, counts=None, mac=BH_MAC_CELLS,
                         order=2):
    tg = _dev(theta_group, "float32") if theta_group is not None else None
    cn = _dev(counts, "int32") if counts is not None else None
    opts = WalkOptions(int(mac), int(order))
    _check(_lib.bh_walk_potential_ex(ctx, grid, m, float(theta), tg, int(precision), float(G), _dev(phi, "float64"),
                                     cn, ctypes.byref(opts)), ctx)
    return phi


def bh_walk_accel(ctx, grid, m, theta, theta_group, precision, G, phi, acc, counts=None):
    """acc: float64 CUDA tensor [n_leaf, 8, 8, 8, 3]; phi: None or [n_leaf, 8, 8, 8]."""
    tg = _dev(theta_group, "float32") if theta_group is not None else None
    ph = _dev(phi, "float64") if phi is not None else None
    c = _dev(counts, "int32") if counts is not None else None
    _check(_lib.bh_walk_accel(ctx, grid, m, float(theta), tg, int(precision), float(G), ph, _dev(acc, "float64"), c),
           ctx)
    return acc


def bh_direct_accel(ctx, grid, m, targets, G, acc):
    n = int(targets.numel())
    _check(_lib.bh_direct_accel(ctx, grid, m, _dev(targets, "int64"), n, float(G), _dev(acc, "float64")), ctx)
    return acc


def bh_direct(ctx, grid, m, targets, G, phi):
    n = int(targets.numel())
    _check(_lib.bh_direct(ctx, grid, m, _dev(targets, "int64"), n, float(G), _dev(phi, "float64")), ctx)
    return phi


# ------------------------------------------------------------------ periodic boxes

EWALD_VALUES = 20


def bh_ewald_create(ctx, box_size, n_points=33):
    h = ctypes.c_void_p()
    _check(_lib.bh_ewald_create(ctx, float(box_size), int(n_points), ctypes.byref(h)), ctx)
    return h


def bh_ewald_destroy(table):
    _lib.bh_ewald_destroy(table)


def bh_ewald_export(ctx, table, n_points):
    """fp64 table [n, n, n, 20] indexed [k][j][i] (z, y, x)."""
    v = np.empty((n_points, n_points, n_points, EWALD_VALUES))
    _check(_lib.bh_ewald_export(ctx, table, _ptr(v)), ctx)
    return v


EWALD_NEAR_TERMS = 11
EWALD_LOCAL_BUDGET = 5e-5


def bh_ewald_set_local_budget(ctx, table, budget):
    """Error budget of the group-centre cubic of the fp32 periodic walks (0: off); returns the largest cell side
    whose groups take it."""
    h = ctypes.c_double()
    _check(_lib.bh_ewald_set_local_budget(ctx, table, float(budget), ctypes.byref(h)), ctx)
    return h.value


def bh_ewald_near_series(ctx, table):
    """(coefficients c0..c10, radius in units of L (0: unused), largest error at the check points)."""
    c = np.empty(EWALD_NEAR_TERMS)
    r = ctypes.c_double()
    e = ctypes.c_double()
    _check(_lib.bh_ewald_near_series(ctx, table, _ptr(c), ctypes.byref(r), ctypes.byref(e)), ctx)
    return c, r.value, e.value


def bh_moments_export_trace(ctx, m, n_nodes):
    S = np.empty(n_nodes)
    _check(_lib.bh_moments_export_trace(ctx, m, _ptr(S)), ctx)
    return S


def bh_walk_potential_periodic(ctx, grid, m, table, theta, theta_group, precision, G, phi, counts=None):
    tg = _dev(theta_group, "float32") if theta_group is not None else None
    cn = _dev(counts, "int32") if counts is not None else None
    _check(_lib.bh_walk_potential_periodic(ctx, grid, m, table, float(theta), tg, int(precision), float(G),
                                           _dev(phi, "float64"), cn), ctx)
    return phi


def bh_direct_periodic(ctx, grid, m, table, targets, G, phi):
    n = int(targets.numel())
    _check(_lib.bh_direct_periodic(ctx, grid, m, table, _dev(targets, "int64"), n, float(G), _dev(phi, "float64")),
           ctx)
    return phi


# ------------------------------------------------------------------ learned theta

def bh_group_features(ctx, grid, m, feat):
    """feat: float32 CUDA tensor [n_groups, 12]."""
    _check(_lib.bh_group_features(ctx, grid, m, _dev(feat, "float32")), ctx)
    return feat


def bh_group_rms_error(ctx, grid, phi, ref, rms):
    _check(_lib.bh_group_rms_error(ctx, grid, _dev(phi, "float64"), _dev(ref, "float64"), _dev(rms, "float32")), ctx)
    return rms


def bh_mlp_create(ctx, params, mean, scale):
    h = ctypes.c_void_p()
    p = _np(params, np.float32)
    mu = _np(mean, np.float32)
    sc = _np(scale, np.float32)
    assert p.size == MLP_PARAMS and mu.size == MLP_INPUTS and sc.size == MLP_INPUTS
    _check(_lib.bh_mlp_create(ctx, ctypes.byref(h), _ptr(p), _ptr(mu), _ptr(sc)), ctx)
    return h


def bh_mlp_set_params(ctx, net, params):
    p = _np(params, np.float32)
    assert p.size == MLP_PARAMS
    _check(_lib.bh_mlp_set_params(ctx, net, _ptr(p)), ctx)


def bh_mlp_get_params(ctx, net):
    p = np.empty(MLP_PARAMS, np.float32)
    _check(_lib.bh_mlp_get_params(ctx, net, _ptr(p)), ctx)
    return p


def bh_mlp_forward(ctx, net, feat, theta, bf16=True, shift=0.0):
    n = int(feat.shape[0])
    _check(_lib.bh_mlp_forward(ctx, net, _dev(feat, "float32"), n, int(bool(bf16)), float(shift),
                               _dev(theta, "float32")), ctx)
    return theta


def bh_mlp_set_theta_floor(ctx, net, theta_floor):
    _check(_lib.bh_mlp_set_theta_floor(ctx, net, float(theta_floor)), ctx)


def bh_learned_walk_potential(ctx, grid, m, net, shift, precision, G, phi, theta=None, counts=None):
    th = _dev(theta, "float32") if theta is not None else None
    c = _dev(counts, "int32") if counts is not None else None
    _check(_lib.bh_learned_walk_potential(ctx, grid, m, net, float(shift), int(precision), float(G),
                                          _dev(phi, "float64"), th, c), ctx)
    return phi


def bh_theta_infer(ctx, grid, m, net, theta, shift=0.0):
    _check(_lib.bh_theta_infer(ctx, grid, m, net, float(shift), _dev(theta, "float32")), ctx)
    return theta


def bh_mlp_grad(ctx, net, feat, label, grad, loss=None):
    n = int(feat.shape[0])
    _check(_lib.bh_mlp_grad(ctx, net, _dev(feat, "float32"), _dev(label, "float32"), n, _dev(grad, "float32"),
                            _dev(loss, "float32") if loss is not None else None), ctx)
    return grad


def bh_mlp_adam_step(ctx, net, grad, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    _check(_lib.bh_mlp_adam_step(ctx, net, _dev(grad, "float32"), float(lr), float(beta1), float(beta2), float(eps)),
           ctx)


def bh_mlp_destroy(net):
    _lib.bh_mlp_destroy(net)


# ------------------------------------------------------------------ batches

def _ptr_array(tensors, dtype_name, allow_none=False):
    arr = (ctypes.c_void_p * len(tensors))()
    for k, t in enumerate(tensors):
        arr[k] = None if (t is None and allow_none) else _dev(t, dtype_name).value
    return arr


def bh_batch_create(ctx, grids):
    h = ctypes.c_void_p()
    arr = (ctypes.c_void_p * len(grids))(*[g.value for g in grids])
    _check(_lib.bh_batch_create(ctx, ctypes.byref(h), len(grids), arr), ctx)
    return h


def bh_batch_destroy(batch):
    _lib.bh_batch_destroy(batch)


def bh_batch_info(batch):
    n, t = ctypes.c_int(), i64()
    _check(_lib.bh_batch_info(batch, ctypes.byref(n), ctypes.byref(t)), None)
    return n.value, t.value


def _batch_args(rho, phi, theta_group):
    r = _ptr_array(rho, "float64")
    p = _ptr_array(phi, "float64")
    tg = _ptr_array(theta_group, "float32", allow_none=True) if theta_group is not None else None
    return r, p, tg


def bh_batch_solve(ctx, batch, rho, phi, theta=0.5, theta_group=None, precision=BH_FP32, G=1.0):
    r, p, tg = _batch_args(rho, phi, theta_group)
    _check(_lib.bh_batch_solve(ctx, batch, r, p, float(theta), tg, int(precision), float(G)), ctx)


def bh_batch_solve_periodic(ctx, batch, table, rho, phi, theta=0.5, theta_group=None, precision=BH_FP32, G=1.0):
    r, p, tg = _batch_args(rho, phi, theta_group)
    _check(_lib.bh_batch_solve_periodic(ctx, batch, table, r, p, float(theta), tg, int(precision), float(G)), ctx)


def bh_batch_capture(ctx, batch, rho, phi, theta=0.5, theta_group=None, precision=BH_FP32, G=1.0):
    r, p, tg = _batch_args(rho, phi, theta_group)
    _check(_lib.bh_batch_capture(ctx, batch, r, p, float(theta), tg, int(precision), float(G)), ctx)


def bh_batch_replay(ctx, batch):
    _check(_lib.bh_batch_replay(ctx, batch), ctx)


def bh_batch_check(ctx, batch):
    _check(_lib.bh_batch_check(ctx, batch), ctx)


def bh_batch_counts(ctx, batch):
    _, total = bh_batch_info(batch)
    c = np.empty((total, 2), np.int32)
    _check(_lib.bh_batch_counts(ctx, batch, _ptr(c)), ctx)
    return c


def bh_batch_schedule(ctx, batch, mode):
    _check(_lib.bh_batch_schedule(ctx, batch, int(mode)), ctx)


def bh_batch_set_launch(ctx, batch, workgroups_per_cu):
    _check(_lib.bh_batch_set_launch(ctx, batch, int(workgroups_per_cu)), ctx)


def bh_batch_configure(ctx, batch, order=BH_ORDER_NATURAL, workgroups_per_cu=0, waves_per_simd=0, stack_limit=0):
    cfg = BatchConfig(int(order), int(workgroups_per_cu), int(waves_per_simd), int(stack_limit))
    _check(_lib.bh_batch_configure(ctx, batch, ctypes.byref(cfg)), ctx)


def bh_batch_get_config(batch):
    cfg = BatchConfig()
    _check(_lib.bh_batch_get_config(batch, ctypes.byref(cfg)), None)
    return cfg.as_dict()


def bh_batch_autotune(ctx, batch, rho, phi, theta=0.5, theta_group=None, precision=BH_FP32, G=1.0, reps=3):
    """Returns (best config dict, best median ms, [(config dict, ms), ...])."""
    r, p, tg = _batch_args(rho, phi, theta_group)
    best, best_ms, n = BatchConfig(), ctypes.c_float(), ctypes.c_int()
    cap = 128
    table = (BatchTiming * cap)()
    _check(_lib.bh_batch_autotune(ctx, batch, r, p, float(theta), tg, int(precision), float(G), int(reps),
                                  ctypes.byref(best), ctypes.byref(best_ms), table, cap, ctypes.byref(n)), ctx)
    rows = [(table[i].config.as_dict(), float(table[i].ms)) for i in range(min(n.value, cap))]
    return best.as_dict(), float(best_ms.value), rows
