"""FP64 CPU reference ("oracle") of the D3Q27 cumulant LBM hot path.

TEST INFRASTRUCTURE ONLY.  Only the tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` import this package.  The product library and
its Python binding never import it; it shares no code with them.  Every
function here is a thin ctypes wrapper around the plain C in this directory
(``lbm_oracle.c``, ``geom_oracle.c``, ``amr_oracle.c``) or plain numpy
(``turb_oracle.py`` for the inflow turbulence).

Population layout: ``f[i, cell]`` with ``i = (cx+1) + 3(cy+1) + 9(cz+1)`` and
``cell = x + nx*(y + ny*z)``.
"""
import ctypes as C
import os
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None

Q = 27
CX = np.array([i % 3 - 1 for i in range(Q)])
CY = np.array([(i // 3) % 3 - 1 for i in range(Q)])
CZ = np.array([i // 9 - 1 for i in range(Q)])
CVEC = np.stack([CX, CY, CZ], axis=1)
OPP = np.array([Q - 1 - i for i in range(Q)])

_dp = C.POINTER(C.c_double)
_u8p = C.POINTER(C.c_uint8)
_i64p = C.POINTER(C.c_int64)
_i8p = C.POINTER(C.c_int8)
_i32p = C.POINTER(C.c_int32)


def _ptr(a, t=_dp):
    return a.ctypes.data_as(t) if a is not None else None


class _TreeParams(C.Structure):
    _fields_ = [("m", C.c_int), ("order", C.c_int), ("s0", C.c_double), ("w0", C.c_double),
                ("len_ratio", C.c_double * 4), ("wid_ratio", C.c_double * 4),
                ("pre_roll", C.c_double * 4), ("pitch", C.c_double * 4),
                ("post_roll", C.c_double * 4), ("jitter", C.c_double), ("seed", C.c_uint64)]


class _Params(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("periodic_x", C.c_int),
                ("omega1", C.c_double), ("omega2", C.c_double), ("omega_high", C.c_double),
                ("galilean", C.c_int), ("u_in", C.c_double), ("force", C.c_double * 3),
                ("inlet_u", _dp), ("lateral_inflow", C.c_int)]


def lib():
    global _lib
    if _lib is None:
        path = os.path.join(_HERE, "liblbm_oracle.so")
        srcs = [os.path.join(_HERE, s) for s in _build.SOURCES if os.path.exists(os.path.join(_HERE, s))]
        if not os.path.exists(path) or any(os.path.getmtime(s) > os.path.getmtime(path) for s in srcs):
            _build.build()
        L = C.CDLL(path)
        L.or_weight.restype = C.c_double
        L.or_weight.argtypes = [C.c_int]
        L.or_equilibrium.argtypes = [C.c_double, _dp, _dp]
        for n in ("or_central_moments_direct", "or_chimera_forward", "or_chimera_inverse"):
            getattr(L, n).argtypes = [_dp, _dp, _dp]
        L.or_cumulants_from_central.argtypes = [_dp, _dp]
        L.or_central_from_cumulants.argtypes = [_dp, _dp]
        L.or_relax_cumulants.argtypes = [_dp, _dp, C.c_double, C.c_double, C.c_double, C.c_int]
        L.or_collide.argtypes = [_dp, _dp, C.c_double, C.c_double, C.c_double, C.c_int, _dp]
        L.or_step.restype = C.c_int
        L.or_step.argtypes = [C.POINTER(_Params), _dp, _dp, _u8p, C.c_int, _i64p, _i8p, _dp, _i32p,
                              C.c_int, _dp, _dp]
        L.or_fields.argtypes = [_dp, C.c_int64, _dp, _dp, _dp]
        L.or_init.argtypes = [C.c_int64, _u8p, C.c_double, _dp]
        L.or_splitmix_uniform.restype = C.c_double
        L.or_splitmix_uniform.argtypes = [C.POINTER(C.c_uint64)]
        L.or_tree_generate.restype = C.c_int
        L.or_tree_generate.argtypes = [C.POINTER(_TreeParams), _dp, C.c_int]
        L.or_tree_height.restype = C.c_double
        L.or_tree_height.argtypes = [_dp, C.c_int]
        L.or_tree_place.argtypes = [_dp, C.c_int, C.c_double, _dp]
        L.or_voxelize.argtypes = [_dp, C.c_int, C.c_int, C.c_int, C.c_int, _u8p]
        L.or_links.restype = C.c_int64
        L.or_links.argtypes = [_dp, C.c_int, C.c_int, C.c_int, C.c_int, _u8p, C.c_int64, _i64p, _i8p,
                               _dp, _i32p]
        L.or_set_threads.argtypes = [C.c_int]
        L.or_area_x.restype = C.c_int64
        L.or_area_x.argtypes = [_u8p, C.c_int, C.c_int, C.c_int]
        _lib = L
        _bind_extra(L)
    return _lib


def _bind_extra(L):
    """Argument types of the AMR and inflow references (added when present)."""
    try:
        from . import _amr_bind  # noqa: F401
        _amr_bind.bind(L)
    except ImportError:
        pass


# --------------------------------------------------------------------------
# lattice and single-cell collision
# --------------------------------------------------------------------------

def weights() -> np.ndarray:
    return np.array([lib().or_weight(i) for i in range(Q)])


def equilibrium(rho: float, u) -> np.ndarray:
    u = np.ascontiguousarray(u, dtype=np.float64)
    f = np.empty(Q)
    lib().or_equilibrium(rho, _ptr(u), _ptr(f))
    return f


def _unary(name, a, u):
    a = np.ascontiguousarray(a, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.empty(Q)
    getattr(lib(), name)(_ptr(a), _ptr(u), _ptr(out))
    return out


def central_moments_direct(f, u):
    return _unary("or_central_moments_direct", f, u)


def chimera_forward(f, u):
    return _unary("or_chimera_forward", f, u)


def chimera_inverse(k, u):
    return _unary("or_chimera_inverse", k, u)


def cumulants_from_central(k):
    k = np.ascontiguousarray(k, dtype=np.float64)
    c = np.empty(Q)
    lib().or_cumulants_from_central(_ptr(k), _ptr(c))
    return c


def central_from_cumulants(c):
    c = np.ascontiguousarray(c, dtype=np.float64)
    k = np.empty(Q)
    lib().or_central_from_cumulants(_ptr(c), _ptr(k))
    return k


def collide(f, omega1, omega2=1.0, omega_high=1.0, galilean=True, force=None):
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.empty(Q)
    fr = None if force is None else np.ascontiguousarray(force, dtype=np.float64)
    lib().or_collide(_ptr(f), _ptr(out), omega1, omega2, omega_high, int(galilean), _ptr(fr))
    return out


def set_threads(n: int) -> None:
    """Threads of the oracle's OpenMP loops."""
    lib().or_set_threads(int(n))


def omega_from_nu(nu: float) -> float:
    """Shear relaxation rate of a lattice viscosity nu = (1/omega - 1/2)/3."""
    return 1.0 / (3.0 * nu + 0.5)


# --------------------------------------------------------------------------
# geometry
# --------------------------------------------------------------------------

@dataclass
class TreeParams:
    m: int
    order: int
    s0: float
    w0: float
    len_ratio: List[float]
    wid_ratio: List[float]
    pre_roll: List[float]
    pitch: List[float]
    post_roll: List[float]
    jitter: float = 0.0
    seed: int = 0

    def to_c(self) -> _TreeParams:
        p = _TreeParams()
        p.m, p.order, p.s0, p.w0 = self.m, self.order, self.s0, self.w0
        for name in ("len_ratio", "wid_ratio", "pre_roll", "pitch", "post_roll"):
            arr = getattr(p, name)
            vals = getattr(self, name)
            for j in range(4):
                arr[j] = vals[j] if j < len(vals) else 0.0
        p.jitter = self.jitter
        p.seed = self.seed & 0xFFFFFFFFFFFFFFFF
        return p


def tree_generate(params: TreeParams) -> np.ndarray:
    p = params.to_c()
    n = lib().or_tree_generate(C.byref(p), None, 0)
    out = np.zeros((n, 10))
    lib().or_tree_generate(C.byref(p), _ptr(out), n)
    return out


def tree_height(b: np.ndarray) -> float:
    b = np.ascontiguousarray(b, dtype=np.float64)
    return lib().or_tree_height(_ptr(b), b.shape[0])


def tree_place(b: np.ndarray, target_h: float, com) -> np.ndarray:
    b = np.ascontiguousarray(b, dtype=np.float64).copy()
    com = np.ascontiguousarray(com, dtype=np.float64)
    lib().or_tree_place(_ptr(b), b.shape[0], target_h, _ptr(com))
    return b


def voxelize(b, nx, ny, nz) -> np.ndarray:
    b = np.ascontiguousarray(b, dtype=np.float64)
    s = np.zeros(nx * ny * nz, dtype=np.uint8)
    lib().or_voxelize(_ptr(b), b.shape[0], nx, ny, nz, _ptr(s, _u8p))
    return s


def links(b, solid, nx, ny, nz):
    b = np.ascontiguousarray(b, dtype=np.float64)
    solid = np.ascontiguousarray(solid, dtype=np.uint8)
    n = lib().or_links(_ptr(b), b.shape[0], nx, ny, nz, _ptr(solid, _u8p), 0, None, None, None, None)
    cell = np.zeros(n, np.int64)
    d = np.zeros(n, np.int8)
    q = np.zeros(n)
    br = np.zeros(n, np.int32)
    lib().or_links(_ptr(b), b.shape[0], nx, ny, nz, _ptr(solid, _u8p), n, _ptr(cell, _i64p),
                   _ptr(d, _i8p), _ptr(q), _ptr(br, _i32p))
    return {"cell": cell, "dir": d, "q": q, "branch": br}


def area_x(solid, nx, ny, nz) -> int:
    solid = np.ascontiguousarray(solid, dtype=np.uint8)
    return int(lib().or_area_x(_ptr(solid, _u8p), nx, ny, nz))


# --------------------------------------------------------------------------
# uniform-grid simulation
# --------------------------------------------------------------------------

class UniformSim:
    """Two-array FP64 stepping of the whole box (collide, then pull-stream)."""

    def __init__(self, nx, ny, nz, omega1, u_in=0.0, solid=None, link=None, n_branch=0,
                 omega2=1.0, omega_high=1.0, galilean=True, periodic_x=False, force=(0.0, 0.0, 0.0),
                 lateral_inflow=False):
        self.nx, self.ny, self.nz = nx, ny, nz
        self.N = nx * ny * nz
        self.p = _Params()
        self.p.nx, self.p.ny, self.p.nz = nx, ny, nz
        self.p.periodic_x = int(periodic_x)
        self.p.omega1, self.p.omega2, self.p.omega_high = omega1, omega2, omega_high
        self.p.galilean = int(galilean)
        self.p.u_in = u_in
        for a in range(3):
            self.p.force[a] = force[a]
        self.p.inlet_u = None
        self.p.lateral_inflow = int(lateral_inflow)
        self.force = np.array(force, dtype=np.float64)
        self.solid = None if solid is None else np.ascontiguousarray(solid, dtype=np.uint8)
        if link is None:
            link = {"cell": np.zeros(0, np.int64), "dir": np.zeros(0, np.int8), "q": np.zeros(0),
                    "branch": np.zeros(0, np.int32)}
        self.link = {k: np.ascontiguousarray(v) for k, v in link.items()}
        self.n_branch = n_branch
        self.f = np.empty((Q, self.N))
        lib().or_init(self.N, _ptr(self.solid, _u8p), u_in, _ptr(self.f))
        self._g = np.empty_like(self.f)
        self.steps = 0
        self.missing = 0
        self.last_force = np.zeros(3)
        self.last_branch_force = np.zeros((max(n_branch, 1), 3))
        self._inlet = None

    def set_inlet_fluctuation(self, du: Optional[np.ndarray]):
        """du: (nz, ny, 3) velocity added to the inlet ghost plane, or None."""
        if du is None:
            self._inlet = None
            self.p.inlet_u = None
        else:
            self._inlet = np.ascontiguousarray(du, dtype=np.float64)
            self.p.inlet_u = _ptr(self._inlet)

    def step(self, n=1, record=None):
        L = self.link
        fb = np.zeros(3 * max(self.n_branch, 1))
        for _ in range(n):
            ft = np.zeros(3)
            m = lib().or_step(C.byref(self.p), _ptr(self.f), _ptr(self._g), _ptr(self.solid, _u8p),
                              len(L["cell"]), _ptr(L["cell"], _i64p), _ptr(L["dir"], _i8p), _ptr(L["q"]),
                              _ptr(L["branch"], _i32p), self.n_branch, _ptr(ft),
                              _ptr(fb) if self.n_branch > 0 else None)
            self.missing += m
            self.f, self._g = self._g, self.f
            self.steps += 1
            self.last_force = ft
            if self.n_branch > 0:
                self.last_branch_force = fb.reshape(-1, 3).copy()
            if record is not None:
                record.append(ft.copy())
        return self

    def fields(self):
        rho = np.empty(self.N)
        u = np.empty((self.N, 3))
        fr = self.force if np.any(self.force != 0) else None
        lib().or_fields(_ptr(self.f), self.N, _ptr(fr), _ptr(rho), _ptr(u))
        return rho, u


# --------------------------------------------------------------------------
# multi-level (octree block) simulation
# --------------------------------------------------------------------------

CLS_NONE, CLS_ACTIVE, CLS_BAND, CLS_DEEP, CLS_GHOST = 0, 1, 2, 3, 4


class AmrSim:
    """FP64 multi-level stepping (coarse-first recursion, moment-space transfer)."""

    def __init__(self, L, B, nx, ny, nz, u_in, nu_f, branches, band, wake, solid=None, link=None,
                 n_branch=0, galilean=True, periodic_x=False):
        self.L, self.B = L, B
        b = np.ascontiguousarray(branches, dtype=np.float64)
        band = (C.c_int * 8)(*[int(v) for v in (list(band) + [0] * 8)[:8]])
        wake = (C.c_int * 8)(*[int(v) for v in (list(wake) + [0] * 8)[:8]])
        self.solid = None if solid is None else np.ascontiguousarray(solid, dtype=np.uint8)
        if link is None:
            link = {"cell": np.zeros(0, np.int64), "dir": np.zeros(0, np.int8), "q": np.zeros(0),
                    "branch": np.zeros(0, np.int32)}
        self.link = {k: np.ascontiguousarray(v) for k, v in link.items()}
        Lb = lib()
        self.h = Lb.or_amr_create(L, B, nx, ny, nz, u_in, nu_f, int(galilean), int(periodic_x), _ptr(b), len(b),
                                  band, wake, _ptr(self.solid, _u8p), len(self.link["cell"]),
                                  _ptr(self.link["cell"], _i64p), _ptr(self.link["dir"], _i8p),
                                  _ptr(self.link["q"]), _ptr(self.link["branch"], _i32p), n_branch)
        self.n_branch = n_branch
        if Lb.or_amr_error(self.h) == 2:
            Lb.or_amr_destroy(self.h)
            self.h = None
            raise ValueError("invalid refinement: a refined region comes too close to the box faces")

    def __del__(self):
        if getattr(self, "h", None):
            lib().or_amr_destroy(self.h)
            self.h = None

    def shape(self, l):
        out = (C.c_int * 6)()
        lib().or_amr_level_shape(self.h, l, out)
        return tuple(out)

    def block_map(self, l):
        s = self.shape(l)
        m = np.zeros(s[3] * s[4] * s[5], np.uint8)
        lib().or_amr_block_map(self.h, l, _ptr(m, _u8p))
        return m

    def classes(self, l):
        s = self.shape(l)
        m = np.zeros(s[0] * s[1] * s[2], np.uint8)
        lib().or_amr_classes(self.h, l, _ptr(m, _u8p))
        return m

    def get_f(self, l):
        s = self.shape(l)
        f = np.empty((Q, s[0] * s[1] * s[2]))
        lib().or_amr_get_f(self.h, l, _ptr(f))
        return f

    def set_f(self, l, f):
        f = np.ascontiguousarray(f, dtype=np.float64)
        lib().or_amr_set_f(self.h, l, _ptr(f))

    def set_inlet_series(self, planes):
        """planes: (n, nz0, ny0, 3) inlet ghost-plane fluctuations of level-0
        steps 0 .. n-1 (counted from the start of the run)."""
        self._inlet = np.ascontiguousarray(planes, dtype=np.float64)
        lib().or_amr_set_inlet(self.h, _ptr(self._inlet), len(self._inlet))

    def step(self, n=1):
        lib().or_amr_step(self.h, n)
        return self

    def force_log(self):
        n = lib().or_amr_force_log(self.h, None, 0)
        out = np.zeros(3 * max(n, 1))
        lib().or_amr_force_log(self.h, _ptr(out), n)
        return out[: 3 * n].reshape(-1, 3)

    def branch_force(self):
        out = np.zeros(3 * max(self.n_branch, 1))
        lib().or_amr_branch_force(self.h, _ptr(out))
        return out.reshape(-1, 3)[: self.n_branch]

    def prolong_only(self, l):
        """Ghost cells of level l + 1 rebuilt from level l's present state
        (the prolongation from time T alone, no stepping)."""
        lib().or_amr_prolong_only(self.h, l)

    def restrict_only(self, l):
        """Band cells of level l rebuilt from level l + 1's present state."""
        lib().or_amr_restrict_only(self.h, l)

    def fields(self, l):
        f = self.get_f(l)
        rho = f.sum(0)
        u = (f.T @ CVEC) / rho[:, None]
        return rho, u


def amr_maps(L, B, nx, ny, nz, branches, band, wake):
    """Block maps of every level (0 none, 1 leaf, 2 refined, 3 ghost storage;
    x fastest over each level's block lattice) from the refinement rule alone,
    without the dense state of AmrSim.  Raises ValueError when a refined region
    comes too close to the box faces."""
    b = np.ascontiguousarray(branches, dtype=np.float64).reshape(-1, 10)
    bd = (C.c_int * 8)(*[int(v) for v in (list(band) + [0] * 8)[:8]])
    wk = (C.c_int * 8)(*[int(v) for v in (list(wake) + [0] * 8)[:8]])
    maps = []
    for l in range(L):
        h = 1 << (L - 1 - l)
        maps.append(np.zeros((nx // h // B) * (ny // h // B) * (nz // h // B), np.uint8))
    ptrs = (C.c_void_p * 8)(*([m.ctypes.data for m in maps] + [None] * (8 - L)))
    if lib().or_amr_maps(L, B, nx, ny, nz, _ptr(b), len(b), bd, wk, ptrs) != 0:
        raise ValueError("invalid refinement: a refined region comes too close to the box faces")
    return maps


def cell_transfer(f, omega1, dt):
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.empty(10)
    lib().or_cell_transfer(_ptr(f), omega1, dt, _ptr(out))
    return out


def cell_rebuild(v, omega1, dt):
    v = np.ascontiguousarray(v, dtype=np.float64)
    out = np.empty(Q)
    lib().or_cell_rebuild(_ptr(v), omega1, dt, _ptr(out))
    return out


# --------------------------------------------------------------------------
# tree presets (parameter sets; the generator above does the arithmetic)
# --------------------------------------------------------------------------

def cfg1_tree_params() -> TreeParams:
    """Trunk 16 cells long, diameter 3; two children at +-30 deg, ratios 0.7."""
    return TreeParams(m=2, order=1, s0=16.0, w0=3.0, len_ratio=[0.7, 0.7], wid_ratio=[0.7, 0.7],
                      pre_roll=[0.0, 0.0], pitch=[30.0, -30.0], post_roll=[0.0, 0.0])


def seeded3_tree_params(order: int, seed: int) -> TreeParams:
    """Three children per node, pitch 35 +- 5 deg, 90 deg phyllotaxis, ratios 0.7,
    trunk diameter / length 0.3."""
    return TreeParams(m=3, order=order, s0=1.0, w0=0.3, len_ratio=[0.7] * 3, wid_ratio=[0.7] * 3,
                      pre_roll=[0.0, 120.0, 240.0], pitch=[35.0] * 3, post_roll=[90.0] * 3,
                      jitter=5.0, seed=seed)


def paper_tree_params(generations: int) -> TreeParams:
    """Binary family of the paper's Table 2 (r = 0.8, alpha = +-30, phi = 137,
    s0 = 100, w0 = 30, q = 0.5, e = 0.5)."""
    wq = 0.5 ** 0.5
    return TreeParams(m=2, order=generations, s0=100.0, w0=30.0, len_ratio=[0.8, 0.8],
                      wid_ratio=[wq, wq], pre_roll=[0.0, 0.0], pitch=[30.0, -30.0],
                      post_roll=[137.0, 137.0])


def build_tree(params: TreeParams, target_h: float, com) -> np.ndarray:
    return tree_place(tree_generate(params), target_h, com)
