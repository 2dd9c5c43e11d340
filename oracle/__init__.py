"""FP64 CPU oracle for the time-stepping method (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the HIP library
(``paper_2409_20380_amd``); it neither imports it nor is imported by it.

The arithmetic lives in ``oracle.c`` (plain C, FP64, optional OpenMP); this
module only marshals numpy arrays into it.  See ``oracle.c`` for the
definitions each function follows.  ``oracle.mlp`` (NumPy, FP64) holds the
oracle of the node-wise learned predictor.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (gcc, -O2, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None

d_p = C.POINTER(C.c_double)
i32_p = C.POINTER(C.c_int32)
i64_p = C.POINTER(C.c_int64)
u8_p = C.POINTER(C.c_uint8)


class SolveStats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("restarts", C.c_int32), ("res0", C.c_double),
                ("res_rec", C.c_double), ("res_true", C.c_double), ("fnorm", C.c_double),
                ("status", C.c_int32), ("pad", C.c_int32)]


class Params(C.Structure):
    _fields_ = [("dt", C.c_double), ("aR", C.c_double), ("bR", C.c_double), ("tol", C.c_double),
                ("drop", C.c_double), ("max_iter", C.c_int32), ("s", C.c_int32), ("kind", C.c_int32),
                ("want_ab_residual", C.c_int32), ("s_min", C.c_int32), ("guard", C.c_int32),
                ("skip_ratio", C.c_double), ("col_cost", C.c_double), ("probe_every", C.c_int32),
                ("probe_step", C.c_int32)]


class Window(C.Structure):
    _fields_ = [("win", C.c_int32), ("s_cap", C.c_int32), ("since", C.c_int32), ("grow_next", C.c_int32),
                ("rho_ab", C.c_double), ("rate", C.c_double)]


class StepStats(C.Structure):
    _fields_ = [("it", C.c_int32), ("s_eff", C.c_int32), ("iters", C.c_int32), ("status", C.c_int32),
                ("pick", C.c_int32), ("first", C.c_int32), ("skipped", C.c_int32), ("probe", C.c_int32),
                ("s_cap", C.c_int32), ("pad", C.c_int32),
                ("res_ab", C.c_double), ("res_map", C.c_double), ("res_probe", C.c_double), ("res0", C.c_double),
                ("res_rec", C.c_double), ("res_true", C.c_double), ("fnorm", C.c_double)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [C.c_int64, d_p, C.c_int64, i32_p, i32_p, C.c_int32, d_p, u8_p,
                                 C.c_double, C.c_double, C.POINTER(C.c_int)]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_nnzb.restype = C.c_int64
        L.orc_nnzb.argtypes = [C.c_void_p]
        L.orc_element_matrices.restype = C.c_double
        L.orc_element_matrices.argtypes = [d_p, C.c_double, C.c_double, C.c_double, d_p, d_p]
        L.orc_spmv.argtypes = [C.c_void_p, C.c_int, d_p, d_p]
        L.orc_precond.argtypes = [C.c_void_p, d_p, d_p]
        L.orc_copy_binv.argtypes = [C.c_void_p, d_p]
        L.orc_copy_bcsr.argtypes = [C.c_void_p, C.c_int, i64_p, i32_p, d_p]
        L.orc_pcg.restype = C.c_int
        L.orc_pcg.argtypes = [C.c_void_p, d_p, d_p, C.c_double, C.c_int, C.POINTER(SolveStats)]
        L.orc_rhs.argtypes = [C.c_void_p, d_p, d_p, d_p, d_p, d_p, C.c_double, C.c_double, C.c_double, d_p]
        L.orc_ab4.argtypes = [C.c_int64, C.c_double, d_p, d_p, d_p, d_p, d_p]
        L.orc_predict_regional.argtypes = [C.c_int64, i32_p, C.c_int32, C.c_int, C.POINTER(d_p),
                                           C.POINTER(d_p), d_p, C.c_double, d_p]
        L.orc_step.restype = C.c_int
        L.orc_step.argtypes = [C.c_void_p, C.POINTER(Params), i32_p, C.c_int32, d_p, d_p, d_p,
                               C.POINTER(d_p), C.POINTER(d_p), C.POINTER(C.c_int32), C.POINTER(Window),
                               d_p, d_p, d_p, d_p, C.POINTER(StepStats)]
        L.orc_num_threads.restype = C.c_int
        L.orc_set_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def _d(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(d_p)


def element_matrices(xv, lam, mu, rho):
    """(Ke, Me, V): 30x30 stiffness and consistent mass of a straight 10-node tet."""
    xv = np.ascontiguousarray(xv, dtype=np.float64).reshape(12)
    Ke = np.zeros((30, 30)); Me = np.zeros((30, 30))
    V = lib().orc_element_matrices(_d(xv), lam, mu, rho, _d(Ke), _d(Me))
    return Ke, Me, V


def num_threads() -> int:
    return lib().orc_num_threads()


def set_threads(n: int) -> None:
    """Thread count of the oracle's later parallel loops (timing only)."""
    lib().orc_set_threads(int(n))


class Model:
    """Assembled BCSR M, K, A = cM M + cK K (fixed dofs: identity) and B^{-1}."""

    def __init__(self, coords, conn, elem_mat, mat, fixed, cM, cK):
        self.coords = np.ascontiguousarray(coords, dtype=np.float64)
        self.conn = np.ascontiguousarray(conn, dtype=np.int32)
        self.elem_mat = np.ascontiguousarray(elem_mat, dtype=np.int32)
        self.mat = np.ascontiguousarray(mat, dtype=np.float64)
        self.fixed = np.ascontiguousarray(fixed, dtype=np.uint8)
        self.n = self.coords.shape[0]
        self.cM, self.cK = float(cM), float(cK)
        err = C.c_int(0)
        h = lib().orc_create(self.n, _d(self.coords), self.conn.shape[0],
                             self.conn.ctypes.data_as(i32_p), self.elem_mat.ctypes.data_as(i32_p),
                             self.mat.shape[0], _d(self.mat), self.fixed.ctypes.data_as(u8_p),
                             self.cM, self.cK, C.byref(err))
        if not h:
            raise ValueError(f"oracle model rejected the mesh (code {err.value})")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_destroy(h)
            self._h = None

    @property
    def n3(self):
        return 3 * self.n

    def spmv(self, which: str, p):
        p = np.ascontiguousarray(p, dtype=np.float64)
        y = np.empty(self.n3)
        lib().orc_spmv(self._h, {"M": 0, "K": 1, "A": 2}[which], _d(p), _d(y))
        return y

    def precond(self, r):
        r = np.ascontiguousarray(r, dtype=np.float64)
        z = np.empty(self.n3)
        lib().orc_precond(self._h, _d(r), _d(z))
        return z

    def binv(self):
        out = np.empty((self.n, 3, 3))
        lib().orc_copy_binv(self._h, _d(out))
        return out

    def bcsr(self, which: str):
        nnzb = lib().orc_nnzb(self._h)
        rowptr = np.empty(self.n + 1, dtype=np.int64)
        col = np.empty(nnzb, dtype=np.int32)
        val = np.empty((nnzb, 3, 3))
        lib().orc_copy_bcsr(self._h, {"M": 0, "K": 1, "A": 2}[which], rowptr.ctypes.data_as(i64_p),
                            col.ctypes.data_as(i32_p), _d(val))
        return rowptr, col, val

    def scipy(self, which: str):
        import scipy.sparse as sp
        rowptr, col, val = self.bcsr(which)
        return sp.bsr_matrix((val, col, rowptr), shape=(self.n3, self.n3)).tocsr()

    def pcg(self, b, x0, tol=1e-8, max_iter=10000):
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.array(x0, dtype=np.float64, copy=True)
        st = SolveStats()
        lib().orc_pcg(self._h, _d(b), _d(x), tol, max_iter, C.byref(st))
        return x, st

    def rhs(self, u, v, a, dt, aR, bR, g=None, f_add=None):
        b = np.empty(self.n3)
        gg = None if g is None else np.ascontiguousarray(g, dtype=np.float64)
        fa = None if f_add is None else np.ascontiguousarray(f_add, dtype=np.float64)
        lib().orc_rhs(self._h, _d(fa), _d(gg), _d(np.ascontiguousarray(u)), _d(np.ascontiguousarray(v)),
                      _d(np.ascontiguousarray(a)), dt, aR, bR, _d(b))
        return b


def ab4(dt, v1, v2, v3, v4):
    out = np.empty_like(v1)
    lib().orc_ab4(v1.size, dt, _d(v1), _d(v2), _d(v3), _d(v4), _d(out))
    return out


def predict_regional(region_of_node, X, Y, x, drop=1e-6):
    """Regional MGS predictor. X, Y: lists of s full-length vectors (oldest first)."""
    region_of_node = np.ascontiguousarray(region_of_node, dtype=np.int32)
    s = len(X)
    Xs = [np.ascontiguousarray(c, dtype=np.float64) for c in X]
    Ys = [np.ascontiguousarray(c, dtype=np.float64) for c in Y]
    Xp = (d_p * s)(*[_d(c) for c in Xs])
    Yp = (d_p * s)(*[_d(c) for c in Ys])
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    nreg = int(region_of_node.max()) + 1
    lib().orc_predict_regional(region_of_node.size, region_of_node.ctypes.data_as(i32_p), nreg, s, Xp, Yp,
                               _d(x), drop, _d(out))
    return out


@dataclass
class StepRecord:
    it: int
    s_eff: int
    iters: int
    status: int
    res_ab: float
    res0: float
    res_rec: float
    res_true: float
    pick: int = -1       # guard: 1 map kept, 0 AB4 kept (window restarted), -1 no comparison
    first: int = 0       # oldest AB error e^first in the window used (0: no map)
    res_map: float = 0.0
    skipped: int = 0     # guard: AB4 guess not evaluated (the map far ahead)
    probe: int = 0       # window length probed this step (0: none)
    s_cap: int = 0       # window length cap after the step
    res_probe: float = 0.0


class Stepper:
    """Time-stepping state and driver (u, v, a, AB velocity history, AB-error ring,
    start of the snapshot window).

    kind 2 uses the regional map once s_min column pairs are available and, with
    guard, keeps the AB4 guess when its initial residual is smaller and restarts
    the window, skips that comparison while the map is far ahead (skip_ratio) and
    probes shorter and longer windows (col_cost > 0) (``orc_step``)."""

    def __init__(self, model: Model, dt, aR, bR, s=16, kind=2, tol=1e-8, max_iter=10000, drop=1e-6,
                 regions=None, want_ab_residual=False, s_min=3, guard=True, skip_ratio=0.01, col_cost=0.08,
                 probe_every=16, probe_step=8):
        self.m = model
        n3 = model.n3
        self.P = Params(dt=dt, aR=aR, bR=bR, tol=tol, drop=drop, max_iter=max_iter, s=s, kind=kind,
                        want_ab_residual=int(want_ab_residual), s_min=int(s_min), guard=int(bool(guard)),
                        skip_ratio=float(skip_ratio), col_cost=float(col_cost), probe_every=int(probe_every),
                        probe_step=int(probe_step))
        self.regions = (np.zeros(model.n, dtype=np.int32) if regions is None
                        else np.ascontiguousarray(regions, dtype=np.int32))
        self.nreg = int(self.regions.max()) + 1
        self.u = np.zeros(n3); self.v = np.zeros(n3); self.a = np.zeros(n3)
        self.vh = [np.zeros(n3) for _ in range(4)]
        self.ring = [np.zeros(n3) for _ in range(max(s, 0) + 1)]
        self.it = C.c_int32(0)
        self.ws = Window(win=1, s_cap=0, since=0, grow_next=0, rho_ab=0.0, rate=0.0)
        self._vhp = (d_p * 4)(*[_d(c) for c in self.vh])
        self._rp = (d_p * len(self.ring))(*[_d(c) for c in self.ring])

    def step(self, g=None, f_add=None, want_du=False, want_guess=False):
        st = StepStats()
        gg = None if g is None else np.ascontiguousarray(g, dtype=np.float64)
        fa = None if f_add is None else np.ascontiguousarray(f_add, dtype=np.float64)
        du = np.empty(self.m.n3) if want_du else None
        gs = np.empty(self.m.n3) if want_guess else None
        lib().orc_step(self.m._h, C.byref(self.P), self.regions.ctypes.data_as(i32_p), self.nreg,
                       _d(self.u), _d(self.v), _d(self.a), self._vhp, self._rp, C.byref(self.it),
                       C.byref(self.ws), _d(gg), _d(fa), _d(du), _d(gs), C.byref(st))
        rec = StepRecord(st.it, st.s_eff, st.iters, st.status, st.res_ab, st.res0, st.res_rec, st.res_true,
                         st.pick, st.first, st.res_map, st.skipped, st.probe, st.s_cap, st.res_probe)
        return rec, du, gs

    @property
    def win(self):
        """First step whose AB error may enter the snapshot window."""
        return self.ws.win
