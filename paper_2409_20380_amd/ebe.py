"""Thin ctypes binding of the C ABI declared in ``include/ebe.h``.

Argument marshalling only: every numerical step runs in the gfx950 kernels of
``libebe.so``.  Device vectors are torch float64 CUDA tensors (contiguous,
length 3 * n_nodes, node-major xyz); PyTorch provides device memory and the
stream.  There is no CPU fallback: if the library is missing the import of
this module's ``lib()`` raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libebe.so")

OK, NOT_CONVERGED = 0, 1
E_INVALID_ARG, E_HIP, E_NO_MEMORY, E_BAD_STATE, E_NONFINITE = -1, -2, -3, -4, -5
PRED_ZERO, PRED_AB4, PRED_SNAPSHOT, PRED_LEARNED = 0, 1, 2, 3
MLP_IN, MLP_HIDDEN, MLP_OUT, MLP_PARAMS, MLP_SAMPLE, MLP_MAX_BATCH, MLP_SCALES = 15, 64, 3, 5379, 18, 8192, 4
PREC_FP64, PREC_FP32, PREC_BF16 = 0, 1, 2


class EbeError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ebe error {code}: {msg}")
        self.code = code


class Config(C.Structure):
    _fields_ = [("dt", C.c_double), ("rayleigh_alpha", C.c_double), ("rayleigh_beta", C.c_double),
                ("tol", C.c_double), ("drop_tol", C.c_double), ("inner_tol", C.c_double), ("max_iter", C.c_int32),
                ("s", C.c_int32), ("predictor", C.c_int32), ("region_nodes", C.c_int32),
                ("patch_elems", C.c_int32), ("chunk_iters", C.c_int32), ("precision", C.c_int32),
                ("inner_iters", C.c_int32), ("s_min", C.c_int32), ("fixed_window", C.c_int32),
                ("probe_every", C.c_int32), ("probe_step", C.c_int32), ("skip_ratio", C.c_double),
                ("col_cost", C.c_double), ("region_merge", C.c_int32), ("reserved", C.c_int32 * 3)]


class Window(C.Structure):
    """Snapshot-window state (ebe_window)."""
    _fields_ = [("start", C.c_int32), ("s_cap", C.c_int32), ("since", C.c_int32), ("grow_next", C.c_int32),
                ("rho_ab", C.c_double), ("rate", C.c_double)]


class SolveStats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("restarts", C.c_int32), ("status", C.c_int32), ("inner_iters", C.c_int32),
                ("res0", C.c_double), ("res_rec", C.c_double), ("res_true", C.c_double), ("bnorm", C.c_double)]


class StepStats(C.Structure):
    _fields_ = [("it", C.c_int32), ("s_eff", C.c_int32), ("iters", C.c_int32), ("restarts", C.c_int32),
                ("status", C.c_int32), ("inner_iters", C.c_int32), ("res0", C.c_double), ("res_rec", C.c_double),
                ("res_true", C.c_double), ("bnorm", C.c_double), ("learned", C.c_int32), ("first", C.c_int32),
                ("res0_snapshot", C.c_double), ("res0_learned", C.c_double), ("map_kept", C.c_int32),
                ("skipped", C.c_int32), ("res0_map", C.c_double), ("res0_ab", C.c_double), ("probe", C.c_int32),
                ("s_cap", C.c_int32), ("res0_probe", C.c_double)]


class PredStats(C.Structure):
    _fields_ = [("s_eff", C.c_int32), ("first", C.c_int32), ("map_kept", C.c_int32), ("learned", C.c_int32),
                ("res0", C.c_double), ("res0_map", C.c_double), ("res0_ab", C.c_double),
                ("res0_learned", C.c_double), ("bnorm", C.c_double)]


class BatchStats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("restarts", C.c_int32), ("status", C.c_int32), ("s_eff", C.c_int32),
                ("res0", C.c_double), ("res_true", C.c_double), ("bnorm", C.c_double), ("first", C.c_int32),
                ("map_kept", C.c_int32)]


# Every symbol include/ebe.h declares (checked by the CPU test suite).
EXPORTS = ("ebe_version", "ebe_create", "ebe_destroy", "ebe_last_error", "ebe_assemble", "ebe_get_regions",
           "ebe_apply", "ebe_apply_mk", "ebe_precond", "ebe_rhs", "ebe_predict", "ebe_refine", "ebe_step",
           "ebe_get_state", "ebe_set_state", "ebe_get_history", "ebe_set_history", "ebe_sync",
           "ebe_set_kernel_timing", "ebe_kernel_time", "ebe_sizes", "ebe_get_config", "ebe_set_predictor",
           "ebe_reset", "ebe_mlp_set", "ebe_mlp_get", "ebe_mlp_forward", "ebe_mlp_grad", "ebe_mlp_grad_noalloc", "ebe_mlp_adam",
           "ebe_collect", "ebe_samples", "ebe_mlp_fit_scales", "ebe_mlp_train", "ebe_batch_create",
           "ebe_batch_destroy", "ebe_batch_last_error", "ebe_batch_add_mesh", "ebe_batch_set_group_config",
           "ebe_batch_assemble", "ebe_batch_group_info", "ebe_batch_use_graph", "ebe_batch_reset", "ebe_batch_apply",
           "ebe_batch_step", "ebe_batch_get_state", "ebe_batch_sizes")

_lib = None
vp = C.c_void_p
d_p = C.POINTER(C.c_double)
i32_p = C.POINTER(C.c_int32)
i64_p = C.POINTER(C.c_int64)
u8_p = C.POINTER(C.c_uint8)


def lib():
    """Load libebe.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} not found: build it with `python -m paper_2409_20380_amd.build`")
    L = C.CDLL(LIB_PATH)
    L.ebe_version.restype = C.c_char_p
    L.ebe_last_error.restype = C.c_char_p
    L.ebe_last_error.argtypes = [vp]
    L.ebe_create.argtypes = [C.POINTER(Config), vp, C.POINTER(vp)]
    L.ebe_destroy.argtypes = [vp]
    L.ebe_assemble.argtypes = [vp, C.c_int64, d_p, C.c_int64, i32_p, i32_p, C.c_int32, d_p, u8_p, i32_p]
    L.ebe_get_regions.argtypes = [vp, i32_p, i32_p]
    L.ebe_apply.argtypes = [vp, vp, vp]
    L.ebe_apply_mk.argtypes = [vp, C.c_double, C.c_double, vp, vp]
    L.ebe_precond.argtypes = [vp, vp, vp]
    L.ebe_rhs.argtypes = [vp, vp, d_p, vp]
    L.ebe_predict.argtypes = [vp, vp, d_p, vp, vp]
    L.ebe_refine.argtypes = [vp, vp, vp, C.POINTER(SolveStats)]
    L.ebe_step.argtypes = [vp, vp, d_p, C.POINTER(StepStats)]
    L.ebe_get_state.argtypes = [vp, vp, vp, vp]
    L.ebe_set_state.argtypes = [vp, vp, vp, vp]
    L.ebe_get_history.argtypes = [vp, vp, vp, i32_p, C.POINTER(Window)]
    L.ebe_set_history.argtypes = [vp, vp, vp, C.c_int32, C.POINTER(Window)]
    L.ebe_sync.argtypes = [vp]
    L.ebe_set_kernel_timing.argtypes = [vp, C.c_int32]
    L.ebe_kernel_time.argtypes = [vp, i64_p, d_p]
    L.ebe_sizes.argtypes = [vp, i64_p, i64_p, i64_p, i64_p]
    L.ebe_get_config.argtypes = [vp, C.POINTER(Config)]
    f_p = C.POINTER(C.c_float)
    L.ebe_set_predictor.argtypes = [vp, C.c_int32]
    L.ebe_reset.argtypes = [vp]
    L.ebe_mlp_set.argtypes = [vp, f_p, f_p]
    L.ebe_mlp_get.argtypes = [vp, f_p, f_p]
    L.ebe_mlp_forward.argtypes = [vp, C.c_int64, vp, vp]
    L.ebe_mlp_grad.argtypes = [vp, C.c_int64, vp, vp, vp, d_p]
    L.ebe_mlp_grad_noalloc.argtypes = [vp, C.c_int64, vp, vp, vp, d_p]
    L.ebe_mlp_adam.argtypes = [vp, vp, C.c_float]
    L.ebe_collect.argtypes = [vp, C.c_int64, vp, C.c_int32]
    L.ebe_samples.argtypes = [vp, i64_p, vp]
    L.ebe_mlp_fit_scales.argtypes = [vp, f_p]
    L.ebe_mlp_train.argtypes = [vp, C.c_int32, C.c_int32, vp, C.c_float, d_p]
    L.ebe_batch_create.argtypes = [C.POINTER(Config), vp, C.POINTER(vp)]
    L.ebe_batch_destroy.argtypes = [vp]
    L.ebe_batch_last_error.argtypes = [vp]
    L.ebe_batch_last_error.restype = C.c_char_p
    L.ebe_batch_add_mesh.argtypes = [vp, C.c_int64, d_p, C.c_int64, i32_p, i32_p, C.c_int32, d_p, u8_p, i32_p,
                                     C.c_int32, i32_p]
    L.ebe_batch_set_group_config.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32]
    L.ebe_batch_assemble.argtypes = [vp, C.c_int32]
    L.ebe_batch_group_info.argtypes = [vp, C.c_int32, i32_p, i32_p, i64_p, i32_p, i32_p]
    L.ebe_batch_use_graph.argtypes = [vp, C.c_int32, C.c_int32]
    L.ebe_batch_reset.argtypes = [vp]
    L.ebe_batch_apply.argtypes = [vp, C.c_int32, vp, vp]
    L.ebe_batch_step.argtypes = [vp, d_p, C.POINTER(BatchStats)]
    L.ebe_batch_get_state.argtypes = [vp, C.c_int32, vp, vp, vp]
    L.ebe_batch_sizes.argtypes = [vp, i32_p, i32_p, i64_p]
    for name in EXPORTS:
        getattr(L, name).restype = getattr(L, name).restype or C.c_int
    L.ebe_version.restype = C.c_char_p
    L.ebe_last_error.restype = C.c_char_p
    L.ebe_batch_last_error.restype = C.c_char_p
    _lib = L
    return L


def _dev(t):
    """Device pointer of a contiguous float64 CUDA tensor (or None)."""
    if t is None:
        return None
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError("expected a contiguous float64 CUDA tensor")
    return C.c_void_p(t.data_ptr())


def _devt(t, dtype_name, n=None):
    """Device pointer of a contiguous CUDA tensor of the given dtype (and length)."""
    import torch
    dt = getattr(torch, dtype_name)
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dt and t.is_contiguous()):
        raise TypeError(f"expected a contiguous {dtype_name} CUDA tensor")
    if n is not None and t.numel() != n:
        raise ValueError(f"expected {n} elements, got {t.numel()}")
    return C.c_void_p(t.data_ptr())


def _host(a, dtype, ptr_t):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(ptr_t)


@dataclass
class Mesh:
    coords: np.ndarray
    conn: np.ndarray
    elem_mat: np.ndarray
    mat: np.ndarray
    fixed: np.ndarray
    regions: np.ndarray | None = None


class Solver:
    """One handle of the library: a mesh, its state and its history."""

    def __init__(self, dt, rayleigh_alpha=0.0, rayleigh_beta=0.0, tol=1e-8, s=16, predictor=PRED_SNAPSHOT,
                 max_iter=10000, drop_tol=0.0, region_nodes=512, patch_elems=256, chunk_iters=0, precision=PREC_FP64,
                 inner_iters=0, inner_tol=0.0, s_min=0, fixed_window=False, skip_ratio=0.0, col_cost=0.0,
                 probe_every=0, probe_step=0, region_merge=0, stream=None):
        import torch
        L = lib()
        cfg = Config(dt=dt, rayleigh_alpha=rayleigh_alpha, rayleigh_beta=rayleigh_beta, tol=tol,
                     drop_tol=drop_tol, max_iter=max_iter, s=s, predictor=predictor, region_nodes=region_nodes,
                     patch_elems=patch_elems, chunk_iters=chunk_iters, precision=precision,
                     inner_iters=inner_iters, inner_tol=inner_tol, s_min=s_min, fixed_window=int(bool(fixed_window)),
                     skip_ratio=skip_ratio, col_cost=col_cost, probe_every=probe_every, probe_step=probe_step,
                     region_merge=region_merge)
        self.cfg = cfg
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = C.c_void_p()
        rc = L.ebe_create(C.byref(cfg), C.c_void_p(stream.cuda_stream), C.byref(h))
        if rc != OK:
            raise EbeError(rc, L.ebe_last_error(None).decode())
        self._h = h
        self.n_nodes = 0

    def close(self):
        if getattr(self, "_h", None):
            lib().ebe_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, allow_not_converged=False):
        if rc == OK or (allow_not_converged and rc == NOT_CONVERGED):
            return rc
        raise EbeError(rc, lib().ebe_last_error(self._h).decode())

    @property
    def n3(self):
        return 3 * self.n_nodes

    def assemble(self, coords, conn, elem_mat, mat, fixed, regions=None):
        L = lib()
        coords, cp = _host(coords, np.float64, d_p)
        conn, np_ = _host(conn, np.int32, i32_p)
        elem_mat, ep = _host(elem_mat, np.int32, i32_p)
        mat, mp = _host(mat, np.float64, d_p)
        fixed, fp = _host(fixed, np.uint8, u8_p)
        rp = None
        if regions is not None:
            regions, rp = _host(regions, np.int32, i32_p)
        self._check(L.ebe_assemble(self._h, coords.shape[0], cp, conn.shape[0], np_, ep, mat.shape[0], mp, fp, rp))
        self.n_nodes = coords.shape[0]

    def regions(self):
        out = np.empty(self.n_nodes, dtype=np.int32)
        n = C.c_int32()
        self._check(lib().ebe_get_regions(self._h, out.ctypes.data_as(i32_p), C.byref(n)))
        return out, n.value

    def _out(self, out):
        import torch
        return torch.empty(self.n3, dtype=torch.float64, device="cuda") if out is None else out

    def apply(self, p, out=None):
        q = self._out(out)
        self._check(lib().ebe_apply(self._h, _dev(p), _dev(q)))
        return q

    def apply_mk(self, cm, ck, p, out=None):
        q = self._out(out)
        self._check(lib().ebe_apply_mk(self._h, cm, ck, _dev(p), _dev(q)))
        return q

    def precond(self, r, out=None):
        z = self._out(out)
        self._check(lib().ebe_precond(self._h, _dev(r), _dev(z)))
        return z

    def rhs(self, f_ext=None, base_acc=None, out=None):
        b = self._out(out)
        g = None if base_acc is None else (C.c_double * 3)(*[float(x) for x in base_acc])
        self._check(lib().ebe_rhs(self._h, _dev(f_ext), g, _dev(b)))
        return b

    def predict(self, f_next=None, base_acc=None, out=None, stats=True):
        """Guess of the next step's increment; returns (x, PredStats or None)."""
        x = self._out(out)
        st = PredStats() if stats else None
        g = None if base_acc is None else (C.c_double * 3)(*[float(v) for v in base_acc])
        self._check(lib().ebe_predict(self._h, _dev(f_next), g, _dev(x), C.byref(st) if stats else None))
        return x, st

    def refine(self, b, x):
        st = SolveStats()
        rc = lib().ebe_refine(self._h, _dev(b), _dev(x), C.byref(st))
        self._check(rc, allow_not_converged=True)
        return st

    def step(self, f_ext=None, base_acc=None, stats=True):
        st = StepStats() if stats else None
        g = None if base_acc is None else (C.c_double * 3)(*[float(x) for x in base_acc])
        rc = lib().ebe_step(self._h, _dev(f_ext), g, C.byref(st) if stats else None)
        self._check(rc, allow_not_converged=True)
        return st

    def get_state(self):
        import torch
        u, v, a = (torch.empty(self.n3, dtype=torch.float64, device="cuda") for _ in range(3))
        self._check(lib().ebe_get_state(self._h, _dev(u), _dev(v), _dev(a)))
        return u, v, a

    def set_state(self, u=None, v=None, a=None):
        self._check(lib().ebe_set_state(self._h, _dev(u), _dev(v), _dev(a)))

    def get_history(self):
        import torch
        vh = torch.empty(4 * self.n3, dtype=torch.float64, device="cuda")
        ring = torch.empty((self.cfg.s + 1) * self.n3, dtype=torch.float64, device="cuda")
        it = C.c_int32()
        win = Window()
        self._check(lib().ebe_get_history(self._h, _dev(vh), _dev(ring), C.byref(it), C.byref(win)))
        return vh.view(4, self.n3), ring.view(self.cfg.s + 1, self.n3), it.value, win

    def set_history(self, vhist, ring, it, win=None):
        """win: a Window, an int (window start; length s, no probe history) or None (start 1)."""
        if isinstance(win, int):
            win = Window(start=win, s_cap=0, since=0, grow_next=0, rho_ab=0.0, rate=0.0)
        self._check(lib().ebe_set_history(self._h, _dev(vhist.contiguous().view(-1)),
                                          _dev(ring.contiguous().view(-1)), int(it),
                                          C.byref(win) if win is not None else None))

    def sync(self):
        self._check(lib().ebe_sync(self._h))

    def set_kernel_timing(self, every_n):
        self._check(lib().ebe_set_kernel_timing(self._h, int(every_n)))

    def kernel_time(self):
        n = C.c_int64()
        ms = C.c_double()
        self._check(lib().ebe_kernel_time(self._h, C.byref(n), C.byref(ms)))
        return n.value, ms.value

    def effective_config(self):
        """The configuration the library uses (defaults filled in)."""
        c = Config()
        self._check(lib().ebe_get_config(self._h, C.byref(c)))
        return c

    # ---- learned predictor
    def set_predictor(self, kind):
        self._check(lib().ebe_set_predictor(self._h, int(kind)))
        self.cfg.predictor = int(kind)

    def reset(self):
        self._check(lib().ebe_reset(self._h))

    def mlp_set(self, params, scales):
        p, pp = _host(params, np.float32, C.POINTER(C.c_float))
        s, sp = _host(scales, np.float32, C.POINTER(C.c_float))
        if p.size != MLP_PARAMS or s.size != MLP_SCALES:
            raise ValueError(f"need {MLP_PARAMS} parameters and {MLP_SCALES} scales")
        self._check(lib().ebe_mlp_set(self._h, pp, sp))

    def mlp_get(self):
        p = np.empty(MLP_PARAMS, dtype=np.float32)
        s = np.empty(MLP_SCALES, dtype=np.float32)
        self._check(lib().ebe_mlp_get(self._h, p.ctypes.data_as(C.POINTER(C.c_float)),
                                      s.ctypes.data_as(C.POINTER(C.c_float))))
        return p, s

    def mlp_forward(self, x):
        """x: float32 CUDA tensor [n][15] (scaled inputs) -> outputs [n][3]."""
        import torch
        n = x.shape[0]
        y = torch.empty((n, MLP_OUT), dtype=torch.float32, device="cuda")
        self._check(lib().ebe_mlp_forward(self._h, n, _devt(x, "float32", n * MLP_IN), _devt(y, "float32")))
        return y

    def mlp_grad(self, x, t):
        import torch
        n = x.shape[0]
        g = torch.empty(MLP_PARAMS, dtype=torch.float32, device="cuda")
        loss = C.c_double()
        self._check(lib().ebe_mlp_grad(self._h, n, _devt(x, "float32", n * MLP_IN), _devt(t, "float32", n * MLP_OUT),
                                       _devt(g, "float32"), C.byref(loss)))
        return g, loss.value

    def mlp_grad_noalloc(self, x, t, out=None, want_loss=True):
        """ebe_mlp_grad_noalloc: the library allocates nothing during the call (out: the caller's
        float32 [5379] device tensor, or one allocated here before the call)."""
        import torch
        n = x.shape[0]
        g = torch.empty(MLP_PARAMS, dtype=torch.float32, device="cuda") if out is None else out
        loss = C.c_double()
        self._check(lib().ebe_mlp_grad_noalloc(self._h, n, _devt(x, "float32", n * MLP_IN),
                                               _devt(t, "float32", n * MLP_OUT), _devt(g, "float32", MLP_PARAMS),
                                               C.byref(loss) if want_loss else None))
        return g, (loss.value if want_loss else None)

    def mlp_adam(self, grad, lr):
        self._check(lib().ebe_mlp_adam(self._h, _devt(grad, "float32", MLP_PARAMS), float(lr)))

    def collect(self, capacity, nodes=None):
        """Collect samples at the listed nodes (int32 CUDA tensor of node ids) during later steps."""
        if nodes is None:
            self._check(lib().ebe_collect(self._h, int(capacity), None, 0))
        else:
            self._check(lib().ebe_collect(self._h, int(capacity), _devt(nodes, "int32"), int(nodes.numel())))

    def samples(self):
        import torch
        n = C.c_int64()
        self._check(lib().ebe_samples(self._h, C.byref(n), None))
        out = torch.empty((n.value, MLP_SAMPLE), dtype=torch.float32, device="cuda")
        if n.value:
            self._check(lib().ebe_samples(self._h, C.byref(n), _devt(out, "float32")))
        return out

    def mlp_fit_scales(self):
        s = np.empty(MLP_SCALES, dtype=np.float32)
        self._check(lib().ebe_mlp_fit_scales(self._h, s.ctypes.data_as(C.POINTER(C.c_float))))
        return s

    def mlp_train(self, idx, lr):
        """Adam steps over minibatches idx (int64 CUDA tensor [steps][batch]); returns the losses."""
        steps, batch = idx.shape
        loss = np.empty(steps, dtype=np.float64)
        self._check(lib().ebe_mlp_train(self._h, int(steps), int(batch), _devt(idx, "int64"), float(lr),
                                        loss.ctypes.data_as(d_p)))
        return loss

    def sizes(self):
        v = [C.c_int64() for _ in range(4)]
        self._check(lib().ebe_sizes(self._h, *[C.byref(x) for x in v]))
        return dict(n_nodes=v[0].value, n_elems=v[1].value, n_patch_nodes=v[2].value, n_patches=v[3].value)


class Batch:
    """A batched ensemble: cases (each with its own base acceleration) on one
    or more meshes, advanced one time step together."""

    def __init__(self, dt, rayleigh_alpha=0.0, rayleigh_beta=0.0, tol=1e-8, s=16, predictor=PRED_SNAPSHOT,
                 max_iter=10000, drop_tol=1e-6, region_nodes=512, s_min=0, fixed_window=False, region_merge=0,
                 stream=None):
        import torch
        L = lib()
        cfg = Config(dt=dt, rayleigh_alpha=rayleigh_alpha, rayleigh_beta=rayleigh_beta, tol=tol, drop_tol=drop_tol,
                     max_iter=max_iter, s=s, predictor=predictor, region_nodes=region_nodes, s_min=s_min,
                     fixed_window=int(bool(fixed_window)), region_merge=region_merge)
        self.cfg = cfg
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p()
        rc = L.ebe_batch_create(C.byref(cfg), C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if rc != OK:
            raise EbeError(rc, L.ebe_batch_last_error(None).decode())
        self._h = h
        self.groups = []     # (n_nodes, n_cases) per group

    def close(self):
        if getattr(self, "_h", None):
            lib().ebe_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, allow_not_converged=False):
        if rc == OK or (allow_not_converged and rc == NOT_CONVERGED):
            return rc
        raise EbeError(rc, lib().ebe_batch_last_error(self._h).decode())

    def add_mesh(self, coords, conn, elem_mat, mat, fixed, regions=None, n_cases=1):
        coords, cp = _host(coords, np.float64, d_p)
        conn, np_ = _host(conn, np.int32, i32_p)
        elem_mat, ep = _host(elem_mat, np.int32, i32_p)
        mat, mp = _host(mat, np.float64, d_p)
        fixed, fp = _host(fixed, np.uint8, u8_p)
        rp = None
        if regions is not None:
            regions, rp = _host(regions, np.int32, i32_p)
        g = C.c_int32()
        self._check(lib().ebe_batch_add_mesh(self._h, coords.shape[0], cp, conn.shape[0], np_, ep, mat.shape[0], mp,
                                             fp, rp, int(n_cases), C.byref(g)))
        self.groups.append((coords.shape[0], int(n_cases)))
        return g.value

    def set_group_config(self, group, case_tile, chunks):
        self._check(lib().ebe_batch_set_group_config(self._h, int(group), int(case_tile), int(chunks)))

    def assemble(self, tune=True):
        self._check(lib().ebe_batch_assemble(self._h, 1 if tune else 0))

    def group_info(self, group):
        v = [C.c_int32(), C.c_int32(), C.c_int64(), C.c_int32(), C.c_int32()]
        self._check(lib().ebe_batch_group_info(self._h, int(group), *[C.byref(x) for x in v]))
        return dict(first_case=v[0].value, n_cases=v[1].value, n_nodes=v[2].value, case_tile=v[3].value,
                    chunks=v[4].value)

    def use_graph(self, on=True, trips=8):
        self._check(lib().ebe_batch_use_graph(self._h, 1 if on else 0, int(trips)))

    def reset(self):
        self._check(lib().ebe_batch_reset(self._h))

    @property
    def n_cases(self):
        return sum(r for _, r in self.groups)

    def apply(self, group, p):
        import torch
        q = torch.empty_like(p)
        self._check(lib().ebe_batch_apply(self._h, int(group), _dev(p), _dev(q)))
        return q

    def step(self, base_acc):
        g, gp = _host(np.asarray(base_acc, dtype=np.float64).reshape(-1, 3), np.float64, d_p)
        if g.shape[0] != self.n_cases:
            raise ValueError(f"need {self.n_cases} base accelerations")
        st = (BatchStats * self.n_cases)()
        rc = lib().ebe_batch_step(self._h, gp, st)
        self._check(rc, allow_not_converged=True)
        return list(st)

    def get_state(self, case):
        import torch
        n = None
        c = int(case)
        for nodes, r in self.groups:
            if c < r:
                n = nodes
                break
            c -= r
        if n is None:
            raise ValueError("no such case")
        u, v, a = (torch.empty(3 * n, dtype=torch.float64, device="cuda") for _ in range(3))
        self._check(lib().ebe_batch_get_state(self._h, int(case), _dev(u), _dev(v), _dev(a)))
        return u, v, a
