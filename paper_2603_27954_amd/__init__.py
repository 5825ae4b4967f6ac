"""Python binding of liblbmtree (C ABI in include/lbmtree.h).

Argument marshalling only: every step of the solver runs in the HIP kernels of
the shared library.  Importing this package fails loudly when the library has
not been built (``python -m paper_2603_27954_amd.build`` or
``__graft_entry__.build()``); there is no fallback path.
"""
import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbmtree.so")

LBM_OK, LBM_E_INVALID, LBM_E_NOMEM, LBM_E_DEVICE, LBM_E_UNSTABLE, LBM_E_STATE = 0, -1, -2, -3, -4, -5
LBM_FP32, LBM_FP16_DEV, LBM_BF16_DEV = 0, 1, 2
LBM_F_NO_GALILEAN, LBM_F_GRAPH, LBM_F_PERSISTENT, LBM_F_AUTOTUNE, LBM_F_FRICTION = 1, 2, 4, 8, 16
STORAGE = {"fp32": LBM_FP32, "fp16": LBM_FP16_DEV, "bf16": LBM_BF16_DEV}
MAX_LEVELS = 8  # LBM_MAX_LEVELS

_STATUS_NAMES = {0: "LBM_OK", -1: "LBM_E_INVALID", -2: "LBM_E_NOMEM", -3: "LBM_E_DEVICE",
                 -4: "LBM_E_UNSTABLE", -5: "LBM_E_STATE"}


class LbmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Branch(C.Structure):
    _fields_ = [("p0", C.c_double * 3), ("p1", C.c_double * 3), ("diameter", C.c_double),
                ("generation", C.c_int32), ("parent", C.c_int32), ("id", C.c_int32)]


class TreeParams(C.Structure):
    _fields_ = [("m", C.c_int32), ("order", C.c_int32), ("s0", C.c_double), ("w0", C.c_double),
                ("len_ratio", C.c_double * 4), ("wid_ratio", C.c_double * 4),
                ("pre_roll", C.c_double * 4), ("pitch", C.c_double * 4),
                ("post_roll", C.c_double * 4), ("jitter", C.c_double), ("seed", C.c_uint64)]


class GridDesc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("block_edge", C.c_int32),
                ("levels", C.c_int32), ("u_in", C.c_double), ("re_h", C.c_double), ("nu", C.c_double),
                ("storage", C.c_int32), ("periodic_yz", C.c_int32), ("turb_intensity", C.c_double),
                ("turb_length", C.c_double), ("turb_seed", C.c_uint64), ("turb_modes", C.c_int32),
                ("drag_every", C.c_int32), ("flags", C.c_uint32), ("device", C.c_int32),
                ("stream", C.c_void_p)]


class RefineDesc(C.Structure):
    _fields_ = [("band", C.c_int32 * MAX_LEVELS), ("wake", C.c_int32 * MAX_LEVELS)]


class Plan(C.Structure):
    _fields_ = [("levels", C.c_int32), ("block_edge", C.c_int32), ("lattice", (C.c_int32 * 3) * MAX_LEVELS),
                ("blocks", C.c_int64 * MAX_LEVELS), ("leaf_cells", C.c_int64 * MAX_LEVELS), ("collided_cells", C.c_int64 * MAX_LEVELS),
                ("updated_cells", C.c_int64 * MAX_LEVELS), ("work_blocks", C.c_int64 * MAX_LEVELS), ("work_tiles", C.c_int64 * MAX_LEVELS),
                ("links", C.c_int64), ("solid_cells", C.c_int64),
                ("pop_bytes", C.c_int64)]


class PhaseInfo(C.Structure):
    _fields_ = [("kind", C.c_int32), ("step", C.c_int32), ("items", C.c_int32), ("chunk", C.c_int32),
                ("chunks", C.c_int32)]


class PersistModelResult(C.Structure):
    _fields_ = [("chunks_run", C.c_int64), ("chunks_missed", C.c_int64), ("chunks_repeated", C.c_int64),
                ("order_violations", C.c_int64), ("waits_given_up", C.c_int64), ("abandoned", C.c_int32),
                ("counters_zero", C.c_int32), ("seconds", C.c_double)]


class DragResult(C.Structure):
    _fields_ = [("force", C.c_double * 3), ("cd", C.c_double), ("area_x", C.c_double),
                ("height", C.c_double), ("mass", C.c_double), ("samples", C.c_int64), ("step", C.c_int64),
                ("friction", C.c_double * 3), ("cf", C.c_double), ("cp", C.c_double)]


class Info(C.Structure):
    _fields_ = [("levels", C.c_int32), ("block_edge", C.c_int32), ("storage", C.c_int32),
                ("blocks", C.c_int64 * MAX_LEVELS), ("active_cells", C.c_int64 * MAX_LEVELS),
                ("updated_cells", C.c_int64 * MAX_LEVELS), ("links", C.c_int64), ("branches", C.c_int32),
                ("omega1", C.c_double * MAX_LEVELS), ("height", C.c_double), ("area_x", C.c_double),
                ("nu_finest", C.c_double), ("device_bytes", C.c_size_t), ("tile_cells", C.c_int32),
                ("threads", C.c_int32), ("occ_even", C.c_int32), ("occ_odd", C.c_int32),
                ("persist_wgs", C.c_int32), ("persist_graph", C.c_int32), ("collided_cells", C.c_int64 * MAX_LEVELS),
                ("xcd_group", C.c_int32), ("wall_clock_khz", C.c_int32), ("persist_wait_ticks", C.c_uint64)]


_lib = None
_P = C.c_void_p
_dp = C.POINTER(C.c_double)


def lib():
    """Loads liblbmtree.so; raises when it is missing (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run python -m paper_2603_27954_amd.build")
    L = C.CDLL(LIB_PATH)
    sigs = {
        "lbm_create_grid": [C.POINTER(GridDesc), C.POINTER(_P)],
        "lbm_set_geometry": [_P, C.POINTER(Branch), C.c_int32, C.POINTER(RefineDesc), C.POINTER(C.c_size_t)],
        "lbm_step": [_P, C.c_int32],
        "lbm_drag": [_P, C.POINTER(DragResult), _dp],
        "lbm_drag_series": [_P, _dp, C.c_int64, C.POINTER(C.c_int64)],
        "lbm_get_info": [_P, C.POINTER(Info)],
        "lbm_tree_generate": [C.POINTER(TreeParams), C.POINTER(Branch), C.c_int32, C.POINTER(C.c_int32)],
        "lbm_tree_place": [C.POINTER(Branch), C.c_int32, C.c_double, _dp, _dp],
        "lbm_get_populations": [_P, C.c_int32, _dp],
        "lbm_set_populations": [_P, C.c_int32, _dp],
        "lbm_get_fields": [_P, C.c_int32, _dp, _dp],
        "lbm_get_solid": [_P, C.POINTER(C.c_uint8)],
        "lbm_get_links": [_P, C.c_int64, C.POINTER(C.c_int64), C.POINTER(C.c_int8), _dp,
                          C.POINTER(C.c_int32), C.POINTER(C.c_int64)],
        "lbm_get_block_map": [_P, C.c_int32, C.POINTER(C.c_int8)],
        "lbm_get_cells": [_P, C.c_int32, C.c_int64, C.POINTER(C.c_int64), _dp],
        "lbm_mlp_create": [C.c_uint64, C.c_int32, _P, C.POINTER(_P)],
        "lbm_mlp_get_params": [_P, C.POINTER(C.c_float)],
        "lbm_mlp_set_params": [_P, C.POINTER(C.c_float)],
        "lbm_mlp_set_scaling": [_P, C.POINTER(C.c_float), C.POINTER(C.c_float), C.c_float, C.c_float],
        "lbm_mlp_grad": [_P, _P, _P, C.c_int64, C.POINTER(C.c_float), C.POINTER(C.c_float)],
        "lbm_mlp_grad_noalloc": [_P, _P, _P, C.c_int64, _P, _P],
        "lbm_mlp_adam_step": [_P, C.POINTER(C.c_float), C.c_float],
        "lbm_mlp_train": [_P, _P, _P, C.c_int64, C.c_int32, C.c_int32, C.c_float, C.c_uint64,
                          C.POINTER(C.c_float)],
        "lbm_mlp_predict": [_P, _P, C.c_int64, _P],
        "lbm_tree_batch": [C.c_void_p, C.c_uint64, C.c_int32, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p],
        "lbm_frontal_area": [_P, _P, C.c_int32, C.c_double, _P, _P],
        "lbm_surrogate_sweep": [_P, _P],
        "lbm_analytic_sweep": [_P, _P],
        "lbm_analytic_split": [_P, _P, _P, _P, _P],
        "lbm_branch_features": [C.POINTER(Branch), C.c_int32, C.c_double, C.c_double, C.POINTER(C.c_float), _dp],
        "lbm_inflow_modes": [C.c_uint64, C.c_int32, C.c_double, C.c_double, C.c_double, C.c_double, _dp, _dp],
        "lbm_plan_levels": [C.POINTER(GridDesc), C.POINTER(Branch), C.c_int32, C.POINTER(RefineDesc),
                            C.POINTER(Plan), C.POINTER(C.POINTER(C.c_int8))],
        "lbm_mass": [_P, _dp],
        "lbm_drag_split": [_P, C.POINTER(DragResult), _dp, _dp],
        "lbm_bind_memory": [_P, _P, C.c_size_t],
        "lbm_plan_phases": [C.POINTER(GridDesc), C.POINTER(Branch), C.c_int32, C.POINTER(RefineDesc), C.c_int32,
                            C.c_int32, C.POINTER(PhaseInfo), C.c_int32, C.POINTER(C.c_int32)],
        "lbm_persist_model": [C.POINTER(C.c_int32), C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_uint32),
                              C.POINTER(C.c_uint32), C.c_double, C.c_int32, C.POINTER(PersistModelResult)],
        "lbm_autotune": [_P, C.c_char_p],
        "lbm_save": [_P, C.c_char_p],
        "lbm_load": [_P, C.c_char_p],
        "lbm_collide_cell_host": [_dp, _dp, C.c_double, C.c_double, C.c_int],
        "lbm_timing_enable": [_P, C.c_int32],
        "lbm_timing_read": [_P, _dp, C.POINTER(C.c_int64), _dp, C.POINTER(C.c_int64)],
        "lbm_geometry_build": [C.POINTER(Branch), C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                               C.POINTER(C.c_uint8), C.c_int64, C.POINTER(C.c_int64), C.POINTER(C.c_int8),
                               _dp, C.POINTER(C.c_int32), C.POINTER(C.c_int64), _dp],
    }
    for name, args in sigs.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = C.c_int
    L.lbm_destroy_grid.argtypes = [_P]
    L.lbm_destroy_grid.restype = None
    L.lbm_mlp_destroy.argtypes = [_P]
    L.lbm_mlp_destroy.restype = None
    L.lbm_last_error.argtypes = [_P]
    L.lbm_last_error.restype = C.c_char_p
    _lib = L
    return L


def _check(st, handle=None):
    if st != LBM_OK:
        msg = lib().lbm_last_error(handle)
        raise LbmError(st, msg.decode() if msg else "")


def _dptr(a):
    return a.ctypes.data_as(_dp)


# ---- geometry helpers --------------------------------------------------------

def tree_params(m, order, s0, w0, len_ratio, wid_ratio, pre_roll, pitch, post_roll, jitter=0.0, seed=0):
    p = TreeParams()
    p.m, p.order, p.s0, p.w0 = m, order, s0, w0
    for name, vals in (("len_ratio", len_ratio), ("wid_ratio", wid_ratio), ("pre_roll", pre_roll),
                       ("pitch", pitch), ("post_roll", post_roll)):
        arr = getattr(p, name)
        for j in range(4):
            arr[j] = vals[j] if j < len(vals) else 0.0
    p.jitter = jitter
    p.seed = seed & 0xFFFFFFFFFFFFFFFF
    return p


def tree_generate(p: TreeParams):
    n = C.c_int32(0)
    _check(lib().lbm_tree_generate(C.byref(p), None, 0, C.byref(n)))
    arr = (Branch * n.value)()
    _check(lib().lbm_tree_generate(C.byref(p), arr, n.value, C.byref(n)))
    return arr


def tree_place(arr, target_h: float, com: Sequence[float]):
    c = np.ascontiguousarray(com, dtype=np.float64)
    h = C.c_double(0.0)
    _check(lib().lbm_tree_place(arr, len(arr), target_h, _dptr(c), C.byref(h)))
    return h.value


def branches_to_numpy(arr) -> np.ndarray:
    out = np.zeros((len(arr), 10))
    for i, b in enumerate(arr):
        out[i, 0:3] = list(b.p0)
        out[i, 3:6] = list(b.p1)
        out[i, 6] = b.diameter
        out[i, 7:10] = (b.generation, b.parent, b.id)
    return out


def branches_from_numpy(a: np.ndarray):
    arr = (Branch * len(a))()
    for i, r in enumerate(a):
        for k in range(3):
            arr[i].p0[k] = r[k]
            arr[i].p1[k] = r[3 + k]
        arr[i].diameter = r[6]
        arr[i].generation, arr[i].parent, arr[i].id = int(r[7]), int(r[8]), int(r[9])
    return arr


def geometry_build(branches, nx, ny, nz):
    """Host-side solid mask, links and frontal area of a uniform box."""
    if isinstance(branches, np.ndarray):
        branches = branches_from_numpy(branches)
    n = C.c_int64(0)
    ax = C.c_double(0.0)
    solid = np.zeros(nx * ny * nz, np.uint8)
    _check(lib().lbm_geometry_build(branches, len(branches), nx, ny, nz,
                                    solid.ctypes.data_as(C.POINTER(C.c_uint8)), 0, None, None, None, None,
                                    C.byref(n), C.byref(ax)))
    m = n.value
    cell = np.zeros(m, np.int64)
    d = np.zeros(m, np.int8)
    q = np.zeros(m)
    br = np.zeros(m, np.int32)
    _check(lib().lbm_geometry_build(branches, len(branches), nx, ny, nz, None, m,
                                    cell.ctypes.data_as(C.POINTER(C.c_int64)), d.ctypes.data_as(C.POINTER(C.c_int8)),
                                    _dptr(q), br.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(n), None))
    return solid, {"cell": cell, "dir": d, "q": q, "branch": br}, ax.value


def collide_cell_host(f, omega1, omega2=1.0, galilean=True):
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.empty(27)
    _check(lib().lbm_collide_cell_host(_dptr(f), _dptr(out), omega1, omega2, int(galilean)))
    return out


# ---- grid --------------------------------------------------------------------

def _make_desc(nx, ny, nz, u_in=0.05, re_h=0.0, nu=0.0, block_edge=16, levels=1, storage="fp32", drag_every=1,
               flags=0, device=0, stream=None, turb_intensity=0.0, turb_length=0.0, turb_seed=0, turb_modes=0,
               periodic_yz=1):
    d = GridDesc()
    d.nx, d.ny, d.nz = nx, ny, nz
    d.block_edge, d.levels = block_edge, levels
    d.u_in, d.re_h, d.nu = u_in, re_h, nu
    d.storage = STORAGE[storage] if isinstance(storage, str) else storage
    d.periodic_yz = int(periodic_yz)
    d.turb_intensity, d.turb_length, d.turb_seed, d.turb_modes = turb_intensity, turb_length, turb_seed, turb_modes
    d.drag_every, d.flags, d.device = drag_every, flags, device
    d.stream = stream
    return d


def _refine_desc(refine):
    if refine is None:
        return None
    r = RefineDesc()
    for k, v in enumerate(refine.get("band", [])):
        r.band[k] = v
    for k, v in enumerate(refine.get("wake", [])):
        r.wake[k] = v
    return r


def _fptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_float))


class SweepDesc(C.Structure):
    _fields_ = [("rec", _P), ("tree_start", _P), ("n_trees", C.c_int32), ("re_h", _dp), ("n_re", C.c_int32),
                ("intensity", C.c_double), ("re_d_lo", C.c_double), ("re_d_hi", C.c_double), ("area", _P),
                ("cd", _P)]


class CfTable(C.Structure):
    _fields_ = [("lg_re", _dp), ("cf", _dp), ("n", C.c_int32)]


def tree_batch(params, seed0, orders):
    """Branch records (n_branches, 10) float32 and offsets (n_trees + 1) int64
    of seeded trees (lbm_tree_batch)."""
    orders = np.ascontiguousarray(orders, dtype=np.int32)
    n = len(orders)
    start = np.empty(n + 1, np.int64)
    _check(lib().lbm_tree_batch(C.byref(params), seed0, n, orders.ctypes.data, 0, None, start.ctypes.data))
    rec = np.empty((int(start[-1]), 10), np.float32)
    _check(lib().lbm_tree_batch(C.byref(params), seed0, n, orders.ctypes.data, rec.shape[0], rec.ctypes.data,
                                start.ctypes.data))
    return rec, start


def _dptr_t(a):
    assert a.is_cuda and a.is_contiguous()
    return C.c_void_p(a.data_ptr())


def frontal_area(rec, start, h, area, stream=None):
    """A_x / H^2 per tree into the torch tensor area (device arrays)."""
    _check(lib().lbm_frontal_area(_dptr_t(rec), _dptr_t(start), start.shape[0] - 1, float(h), _dptr_t(area), stream))
    return area


def _sweep_desc(rec, start, area, cd, re_h, intensity, re_d_range):
    re_h = np.ascontiguousarray(re_h, dtype=np.float64)
    d = SweepDesc()
    d.rec, d.tree_start, d.n_trees = _dptr_t(rec), _dptr_t(start), start.shape[0] - 1
    d.re_h, d.n_re = _dptr(re_h), len(re_h)
    d.intensity = intensity
    d.re_d_lo, d.re_d_hi = re_d_range
    d.area, d.cd = _dptr_t(area), _dptr_t(cd)
    return d, re_h


def analytic_sweep(rec, start, area, cd, re_h, intensity=0.0, stream=None):
    d, keep = _sweep_desc(rec, start, area, cd, re_h, intensity, (1.0, 1.0))
    _check(lib().lbm_analytic_sweep(C.byref(d), stream))
    return cd


def analytic_split(rec, start, area, cd, cf, re_h, table, intensity=0.0, cp=None, stream=None):
    """C_D-est into cd, C_F-est into cf and (when given) C_P-est into cp, all
    torch device tensors (n_trees, n_re); table = (log10 Re_D nodes, C_f)."""
    d, keep = _sweep_desc(rec, start, area, cd, re_h, intensity, (1.0, 1.0))
    need = (start.shape[0] - 1) * len(keep)
    for t in (cd, cf) + ((cp,) if cp is not None else ()):
        if t.element_size() != 4 or t.numel() < need:
            raise ValueError(f"outputs: float32 device tensors of n_trees x n_re = {need} values")
    lg = np.ascontiguousarray(table[0], dtype=np.float64)
    cv = np.ascontiguousarray(table[1], dtype=np.float64)
    if lg.shape != cv.shape:
        raise ValueError("table: as many C_f values as nodes")
    t = CfTable(_dptr(lg), _dptr(cv), len(lg))
    _check(lib().lbm_analytic_split(C.byref(d), C.byref(t), _dptr_t(cf), _dptr_t(cp) if cp is not None else None,
                                    stream))
    return cd, cf, cp


class Mlp:
    """Owns one lbm_mlp handle (the per-branch drag surrogate network).  Device
    arrays are torch CUDA tensors (float32, contiguous); the library computes on
    them in place of copies."""

    N_PARAM = 4609

    def __init__(self, seed=0, device=0, stream=None):
        self.h = _P()
        _check(lib().lbm_mlp_create(seed, device, stream, C.byref(self.h)))

    def close(self):
        if self.h:
            lib().lbm_mlp_destroy(self.h)
            self.h = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self):
        p = np.empty(self.N_PARAM, np.float32)
        _check(lib().lbm_mlp_get_params(self.h, _fptr(p)))
        return p

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        _check(lib().lbm_mlp_set_params(self.h, _fptr(p)))

    def set_scaling(self, x_mean, x_std, y_mean, y_std):
        xm = np.ascontiguousarray(x_mean, dtype=np.float32)
        xs = np.ascontiguousarray(x_std, dtype=np.float32)
        _check(lib().lbm_mlp_set_scaling(self.h, _fptr(xm), _fptr(xs), float(y_mean), float(y_std)))

    @staticmethod
    def _dev(a):
        assert a.is_cuda and a.dtype.is_floating_point and a.is_contiguous()
        return C.c_void_p(a.data_ptr())

    def grad(self, x, t):
        g = np.empty(self.N_PARAM, np.float32)
        loss = C.c_float(0.0)
        _check(lib().lbm_mlp_grad(self.h, self._dev(x), self._dev(t), x.shape[0], _fptr(g), C.byref(loss)))
        return g, loss.value

    def grad_noalloc(self, x, t, grad, loss=None):
        """lbm_mlp_grad_noalloc: gradient (4609) and loss (1) into the device
        tensors grad and loss, enqueued on the handle's stream (no sync)."""
        _check(lib().lbm_mlp_grad_noalloc(self.h, self._dev(x), self._dev(t), x.shape[0], self._dev(grad),
                                          self._dev(loss) if loss is not None else None))
        return grad

    def adam_step(self, grad, lr):
        g = np.ascontiguousarray(grad, dtype=np.float32)
        _check(lib().lbm_mlp_adam_step(self.h, _fptr(g), float(lr)))

    def train(self, x, t, epochs, batch=256, lr=1e-3, seed=0):
        losses = np.empty(epochs, np.float32)
        _check(lib().lbm_mlp_train(self.h, self._dev(x), self._dev(t), x.shape[0], epochs, batch, float(lr), seed,
                                   _fptr(losses)))
        return losses

    def sweep(self, rec, start, area, cd, re_h, intensity=0.0, re_d_range=(1.0, 1e3)):
        d, keep = _sweep_desc(rec, start, area, cd, re_h, intensity, re_d_range)
        _check(lib().lbm_surrogate_sweep(self.h, C.byref(d)))
        return cd

    def predict(self, x, out):
        _check(lib().lbm_mlp_predict(self.h, self._dev(x), x.shape[0], self._dev(out)))
        return out


def branch_features(branches, re_h, intensity=0.0):
    """(features (n, 5) float32, L D (n,) float64) of a tree's branches
    (lbm_branch_features)."""
    if isinstance(branches, np.ndarray):
        branches = branches_from_numpy(branches)
    n = len(branches)
    feat = np.empty((n, 5), np.float32)
    ld = np.empty(n)
    _check(lib().lbm_branch_features(branches, n, float(re_h), float(intensity), _fptr(feat), _dptr(ld)))
    return feat, ld


def inflow_modes(seed, n_modes, intensity, length, u_in, dx):
    """Host-built mode set of the synthetic turbulent inflow (lbm_inflow_modes):
    dict of arrays kvec (n, 3), sigma (n, 3), psi, amp and the float k_e."""
    out = np.empty(8 * n_modes)
    ke = C.c_double(0.0)
    _check(lib().lbm_inflow_modes(seed, n_modes, intensity, length, u_in, dx, _dptr(out), C.byref(ke)))
    o = out.reshape(8, n_modes)
    return {"kvec": o[0:3].T.copy(), "sigma": o[3:6].T.copy(), "psi": o[6].copy(), "amp": o[7].copy(),
            "k_e": ke.value}


def plan_levels(branches, refine=None, maps=False, **desc):
    """Host-only plan of a grid (lbm_plan_levels): per-level lattice, block
    and cell counts, link and solid counts, population bytes, and optionally
    the block map of every level.  desc takes the Grid arguments."""
    if isinstance(branches, np.ndarray):
        branches = branches_from_numpy(branches)
    d = _make_desc(**desc)
    r = _refine_desc(refine)
    out = Plan()
    L = d.levels
    arrs = []
    ptrs = None
    if maps:
        s = d.block_edge << (L - 1)
        for l in range(L):
            f = 1 << l
            arrs.append(np.zeros((d.nx // s) * f * (d.ny // s) * f * (d.nz // s) * f, np.int8))
        ptrs = (C.POINTER(C.c_int8) * MAX_LEVELS)(*[a.ctypes.data_as(C.POINTER(C.c_int8)) for a in arrs])
    _check(lib().lbm_plan_levels(C.byref(d), branches, len(branches), C.byref(r) if r else None, C.byref(out),
                                 ptrs))
    res = {"levels": out.levels, "block_edge": out.block_edge,
           "lattice": [tuple(out.lattice[l]) for l in range(L)], "blocks": list(out.blocks[:L]),
           "leaf_cells": list(out.leaf_cells[:L]), "collided_cells": list(out.collided_cells[:L]),
           "updated_cells": list(out.updated_cells[:L]), "work_blocks": list(out.work_blocks[:L]),
           "work_tiles": list(out.work_tiles[:L]),
           "links": out.links, "solid_cells": out.solid_cells, "pop_bytes": out.pop_bytes}
    if maps:
        res["maps"] = arrs
    return res


def plan_phases(branches, groups, coarse_steps=1, refine=None, **desc):
    """Host-only phase lists of the persistent coarse step (lbm_plan_phases):
    list of dicts kind, step, items, chunk, chunks."""
    if isinstance(branches, np.ndarray):
        branches = branches_from_numpy(branches)
    d = _make_desc(**desc)
    r = _refine_desc(refine)
    n = C.c_int32(0)
    _check(lib().lbm_plan_phases(C.byref(d), branches, len(branches), C.byref(r) if r else None, groups,
                                 coarse_steps, None, 0, C.byref(n)))
    out = (PhaseInfo * max(n.value, 1))()
    _check(lib().lbm_plan_phases(C.byref(d), branches, len(branches), C.byref(r) if r else None, groups,
                                 coarse_steps, out, n.value, C.byref(n)))
    return [{"kind": p.kind, "step": p.step, "items": p.items, "chunk": p.chunk, "chunks": p.chunks}
            for p in out[:n.value]]


def persist_model(chunks, groups, threads, ctr=None, abort=0, wait_s=0.5, stuck_phase=-1):
    """One launch of the persistent protocol on host threads
    (lbm_persist_model).  ctr: the 2n + 1 counters at the start (None: zero),
    updated in place when given as a uint32 array.  Returns (result dict,
    counters, abort flag)."""
    ch = np.ascontiguousarray(chunks, dtype=np.int32)
    n = len(ch)
    c = np.zeros(2 * n + 1, np.uint32) if ctr is None else ctr
    assert c.dtype == np.uint32 and c.flags["C_CONTIGUOUS"] and len(c) == 2 * n + 1
    ab = C.c_uint32(abort)
    r = PersistModelResult()
    _check(lib().lbm_persist_model(ch.ctypes.data_as(C.POINTER(C.c_int32)), n, groups, threads,
                                   c.ctypes.data_as(C.POINTER(C.c_uint32)), C.byref(ab), float(wait_s),
                                   stuck_phase, C.byref(r)))
    res = {k: getattr(r, k) for k, _ in PersistModelResult._fields_}
    return res, c, ab.value


class Grid:
    """Owns one lbm_grid handle."""

    def __init__(self, nx, ny, nz, u_in=0.05, re_h=0.0, nu=0.0, block_edge=16, levels=1,
                 storage="fp32", drag_every=1, flags=0, device=0, stream=None,
                 turb_intensity=0.0, turb_length=0.0, turb_seed=0, turb_modes=0, periodic_yz=1):
        d = _make_desc(nx, ny, nz, u_in, re_h, nu, block_edge, levels, storage, drag_every, flags, device, stream,
                       turb_intensity, turb_length, turb_seed, turb_modes, periodic_yz)
        self.desc = d
        self.h = _P()
        _check(lib().lbm_create_grid(C.byref(d), C.byref(self.h)))
        self.n_branch = 0

    def close(self):
        if self.h:
            lib().lbm_destroy_grid(self.h)
            self.h = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def level_shape(self, level):
        s = self.desc.levels - 1 - level
        return self.desc.nx >> s, self.desc.ny >> s, self.desc.nz >> s

    def bind_memory(self, tensor):
        """Populations in the caller's device tensor (lbm_bind_memory); the
        tensor must outlive the grid."""
        assert tensor.is_cuda and tensor.is_contiguous()
        self._bound = tensor
        _check(lib().lbm_bind_memory(self.h, C.c_void_p(tensor.data_ptr()), tensor.numel() * tensor.element_size()),
               self.h)

    def set_geometry(self, branches, refine: Optional[dict] = None):
        if isinstance(branches, np.ndarray):
            branches = branches_from_numpy(branches)
        r = _refine_desc(refine)
        nbytes = C.c_size_t(0)
        _check(lib().lbm_set_geometry(self.h, branches, len(branches), C.byref(r) if r else None,
                                      C.byref(nbytes)), self.h)
        self.n_branch = len(branches)
        return nbytes.value

    def step(self, n=1):
        _check(lib().lbm_step(self.h, n), self.h)

    def drag(self, per_branch=False, per_branch_friction=False):
        r = DragResult()
        pb = np.zeros(3 * max(self.n_branch, 1)) if per_branch else None
        pf = np.zeros(3 * max(self.n_branch, 1)) if per_branch_friction else None
        _check(lib().lbm_drag_split(self.h, C.byref(r), _dptr(pb) if pb is not None else None,
                                    _dptr(pf) if pf is not None else None), self.h)
        out = {"force": np.array(r.force), "cd": r.cd, "area_x": r.area_x, "height": r.height,
               "mass": r.mass, "samples": r.samples, "step": r.step, "friction": np.array(r.friction),
               "cf": r.cf, "cp": r.cp}
        if per_branch:
            out["per_branch"] = pb.reshape(-1, 3)[: self.n_branch]
        if per_branch_friction:
            out["per_branch_friction"] = pf.reshape(-1, 3)[: self.n_branch]
        return out

    def drag_series(self, cap=65536):
        out = np.zeros(3 * cap)
        n = C.c_int64(0)
        _check(lib().lbm_drag_series(self.h, _dptr(out), cap, C.byref(n)), self.h)
        return out[: 3 * n.value].reshape(-1, 3)

    def info(self):
        i = Info()
        _check(lib().lbm_get_info(self.h, C.byref(i)), self.h)
        return {"levels": i.levels, "block_edge": i.block_edge, "storage": i.storage,
                "blocks": list(i.blocks), "active_cells": list(i.active_cells),
                "updated_cells": list(i.updated_cells), "links": i.links, "branches": i.branches,
                "omega1": list(i.omega1), "height": i.height, "area_x": i.area_x,
                "nu_finest": i.nu_finest, "device_bytes": i.device_bytes, "tile_cells": i.tile_cells,
                "threads": i.threads, "occ_even": i.occ_even, "occ_odd": i.occ_odd,
                "persist_wgs": i.persist_wgs, "persist_graph": i.persist_graph,
                "collided_cells": list(i.collided_cells), "xcd_group": i.xcd_group,
                "wall_clock_khz": i.wall_clock_khz, "persist_wait_ticks": i.persist_wait_ticks}

    def get_populations(self, level=0):
        nx, ny, nz = self.level_shape(level)
        f = np.empty((27, nx * ny * nz))
        _check(lib().lbm_get_populations(self.h, level, _dptr(f)), self.h)
        return f

    def get_cells(self, cells, level=0):
        """FP64 populations (27, n) of the listed cells (indices over the
        level's box); NaN where the level holds no cell."""
        c = np.ascontiguousarray(cells, dtype=np.int64)
        f = np.empty((27, len(c)))
        _check(lib().lbm_get_cells(self.h, level, len(c), c.ctypes.data_as(C.POINTER(C.c_int64)), _dptr(f)),
               self.h)
        return f

    def set_populations(self, f, level=0):
        f = np.ascontiguousarray(f, dtype=np.float64)
        _check(lib().lbm_set_populations(self.h, level, _dptr(f)), self.h)

    def fields(self, level=0):
        nx, ny, nz = self.level_shape(level)
        N = nx * ny * nz
        rho = np.empty(N)
        u = np.empty((N, 3))
        _check(lib().lbm_get_fields(self.h, level, _dptr(rho), _dptr(u)), self.h)
        return rho, u

    def solid(self):
        s = np.empty(self.desc.nx * self.desc.ny * self.desc.nz, np.uint8)
        _check(lib().lbm_get_solid(self.h, s.ctypes.data_as(C.POINTER(C.c_uint8))), self.h)
        return s

    def links(self):
        n = C.c_int64(0)
        _check(lib().lbm_get_links(self.h, 0, None, None, None, None, C.byref(n)), self.h)
        m = n.value
        cell = np.zeros(m, np.int64)
        d = np.zeros(m, np.int8)
        q = np.zeros(m)
        br = np.zeros(m, np.int32)
        _check(lib().lbm_get_links(self.h, m, cell.ctypes.data_as(C.POINTER(C.c_int64)),
                                   d.ctypes.data_as(C.POINTER(C.c_int8)), _dptr(q),
                                   br.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(n)), self.h)
        return {"cell": cell, "dir": d, "q": q, "branch": br}

    def block_map(self, level):
        B = self.desc.block_edge
        nx, ny, nz = self.level_shape(level)
        m = np.zeros((nx // B) * (ny // B) * (nz // B), np.int8)
        _check(lib().lbm_get_block_map(self.h, level, m.ctypes.data_as(C.POINTER(C.c_int8))), self.h)
        return m

    def mass(self):
        m = C.c_double(0.0)
        _check(lib().lbm_mass(self.h, C.byref(m)), self.h)
        return m.value

    def timing(self, enable: bool):
        _check(lib().lbm_timing_enable(self.h, int(enable)), self.h)

    def timing_read(self):
        cm, lm = C.c_double(0), C.c_double(0)
        cn, ln = C.c_int64(0), C.c_int64(0)
        _check(lib().lbm_timing_read(self.h, C.byref(cm), C.byref(cn), C.byref(lm), C.byref(ln)), self.h)
        return {"collide_ms": cm.value, "collide_launches": cn.value, "links_ms": lm.value,
                "links_launches": ln.value}

    def autotune(self, cache_path=None):
        _check(lib().lbm_autotune(self.h, cache_path.encode() if cache_path else None), self.h)

    def save(self, path):
        _check(lib().lbm_save(self.h, path.encode()), self.h)

    def load(self, path):
        _check(lib().lbm_load(self.h, path.encode()), self.h)
