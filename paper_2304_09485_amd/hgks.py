"""Python binding of libhgks (argument marshalling only).

Every step of the residual / Jv / implicit step runs in the HIP kernels of
`libhgks.so`; this module converts numpy arrays (host) or torch tensors
(device) to pointers and checks status codes.  If the library has not been
built, importing the binding raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhgks.so")

WENO, HWENO, KFVS1 = 0, 1, 2
EULER, NS = 0, 1
FP64, FP32_INNER = 0, 1
JV_FD, JV_APPROX = 0, 1
SOLVER_GMRES, SOLVER_LUSGS = 0, 1
SUBS_FACES, SUBS_HEX_WENO = 0, 1
WEIGHTS_NONLINEAR, WEIGHTS_LINEAR = 0, 1
FARFIELD, SLIP_WALL, NOSLIP_ADIABATIC, SUP_IN, SUP_OUT = 0, 1, 2, 3, 4

STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EMESH", -4: "ESTATE", -5: "ENOCONV", -6: "EDEVICE"}

# exported symbols declared in include/hgks.h
SYMBOLS = ["hgks_default_options", "hgks_create", "hgks_load_mesh", "hgks_load_hex_mesh", "hgks_set_freestream", "hgks_set_bc",
           "hgks_set_state", "hgks_get_state", "hgks_residual", "hgks_time_step", "hgks_jv", "hgks_precond",
           "hgks_implicit_step", "hgks_solve_steady", "hgks_residual_dev", "hgks_residual_dev_static",
           "hgks_residual_static_bytes", "hgks_jv_dev", "hgks_n_cells", "hgks_steps_done",
           "hgks_n_faces", "hgks_kernel_times", "hgks_last_error", "hgks_destroy", "hgks_estimate_bytes",
           "hgks_checkpoint", "hgks_restore",
           "hgks_server_create", "hgks_server_submit", "hgks_server_poll", "hgks_server_wait",
           "hgks_server_get_state", "hgks_server_release", "hgks_server_stats", "hgks_server_destroy"]


class HgksError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Options(ctypes.Structure):
    _fields_ = [("scheme", ctypes.c_int32), ("physics", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("weights", ctypes.c_int32), ("krylov_dim", ctypes.c_int32), ("restarts", ctypes.c_int32),
                ("jacobi_sweeps", ctypes.c_int32), ("jv_mode", ctypes.c_int32), ("solver", ctypes.c_int32),
                ("compact_subs", ctypes.c_int32), ("gamma", ctypes.c_double), ("cfl", ctypes.c_double), ("tau_eps", ctypes.c_double),
                ("tau_C", ctypes.c_double), ("gamma_lin", ctypes.c_double), ("weno_eps", ctypes.c_double),
                ("mu", ctypes.c_double), ("prandtl", ctypes.c_double), ("fd_sigma", ctypes.c_double),
                ("cfl_flux", ctypes.c_double), ("cfl_start", ctypes.c_double), ("cfl_growth", ctypes.c_double),
                ("max_update", ctypes.c_double), ("grad_relax", ctypes.c_double),
                ("stream", ctypes.c_void_p), ("dev_alloc", ctypes.c_void_p), ("dev_free", ctypes.c_void_p),
                ("alloc_user", ctypes.c_void_p)]


# Device allocator hook: PyTorch's caching allocator, so that the library's
# device buffers count in torch's memory statistics and reuse its pool.
_ALLOC_T = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_T = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


def _torch_alloc(nbytes, user):
    try:
        import torch
        return torch.cuda.caching_allocator_alloc(int(nbytes))
    except Exception:  # out of memory or torch torn down: NULL -> HGKS_ENOMEM
        return None


def _torch_free(ptr, user):
    try:
        import torch
        torch.cuda.caching_allocator_delete(ptr)
    except Exception:
        pass


_TORCH_HOOK = (_ALLOC_T(_torch_alloc), _FREE_T(_torch_free))  # kept alive for the process


def torch_allocator_hook():
    """(dev_alloc, dev_free) function pointers of PyTorch's caching allocator."""
    return (ctypes.cast(_TORCH_HOOK[0], ctypes.c_void_p).value, ctypes.cast(_TORCH_HOOK[1], ctypes.c_void_p).value)


class StepInfo(ctypes.Structure):
    _fields_ = [("res", ctypes.c_double), ("res_rel", ctypes.c_double), ("gmres_rel", ctypes.c_double),
                ("n_resid_evals", ctypes.c_int64), ("n_fallbacks", ctypes.c_int64), ("n_limited", ctypes.c_int64),
                ("t_ms", ctypes.c_double)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int32), ("converged", ctypes.c_int32), ("res0", ctypes.c_double),
                ("res_final", ctypes.c_double), ("drop", ctypes.c_double), ("n_resid_evals", ctypes.c_int64),
                ("t_ms", ctypes.c_double)]


class Request(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int64), ("xyz", ctypes.c_void_p), ("n_tets", ctypes.c_int64),
                ("tet2node", ctypes.c_void_p), ("n_bfaces", ctypes.c_int64), ("bface2node", ctypes.c_void_p),
                ("bface_tag", ctypes.c_void_p), ("n_bc", ctypes.c_int32), ("bc_tag", ctypes.c_void_p),
                ("bc_kind", ctypes.c_void_p), ("prim_inf", ctypes.c_double * 5), ("opts", Options),
                ("drop", ctypes.c_double), ("max_steps", ctypes.c_int32)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("steps", ctypes.c_int32), ("res0", ctypes.c_double),
                ("res_final", ctypes.c_double), ("n_cells", ctypes.c_int64), ("n_resid_evals", ctypes.c_int64),
                ("t_queue_ms", ctypes.c_double), ("t_solve_ms", ctypes.c_double), ("t_total_ms", ctypes.c_double),
                ("footprint_bytes", ctypes.c_size_t)]


class ServerStats(ctypes.Structure):
    _fields_ = [("queued", ctypes.c_int32), ("active", ctypes.c_int32), ("done", ctypes.c_int32),
                ("bytes_in_use", ctypes.c_size_t), ("budget", ctypes.c_size_t),
                ("cell_resid_evals", ctypes.c_int64), ("steps_done", ctypes.c_int64)]


_lib = None


def load_library():
    """Load libhgks.so; raises if it is missing (build it with
    `python -m paper_2304_09485_amd.build`)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} not built: run `python -m paper_2304_09485_amd.build`")
    # bind the process to PyTorch's HIP runtime first, so that the library and
    # torch tensors share one runtime (same soname, libamdhip64.so.7)
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "hgks_default_options": (None, [ctypes.POINTER(Options)]),
        "hgks_create": (i32, [ctypes.POINTER(Options), ctypes.POINTER(vp)]),
        "hgks_load_mesh": (i32, [vp, i64, vp, i64, vp, i64, vp, vp]),
        "hgks_load_hex_mesh": (i32, [vp, i64, vp, i64, vp, i64, vp, vp]),
        "hgks_set_freestream": (i32, [vp, vp]),
        "hgks_set_bc": (i32, [vp, i32, i32, vp]),
        "hgks_set_state": (i32, [vp, vp, vp]),
        "hgks_get_state": (i32, [vp, vp, vp]),
        "hgks_checkpoint": (i32, [vp, ctypes.c_char_p]),
        "hgks_restore": (i32, [vp, ctypes.c_char_p]),
        "hgks_residual": (i32, [vp, vp, vp, vp, vp]),
        "hgks_time_step": (i32, [vp, vp, vp]),
        "hgks_jv": (i32, [vp, vp, d, vp, vp]),
        "hgks_precond": (i32, [vp, vp, vp]),
        "hgks_implicit_step": (i32, [vp, ctypes.POINTER(StepInfo)]),
        "hgks_solve_steady": (i32, [vp, d, i32, ctypes.POINTER(SolveInfo)]),
        "hgks_residual_dev": (i32, [vp, vp, vp, vp]),
        "hgks_residual_dev_static": (i32, [vp, vp, vp, vp]),
        "hgks_residual_static_bytes": (ctypes.c_size_t, [vp]),
        "hgks_jv_dev": (i32, [vp, vp, d, vp, vp]),
        "hgks_n_cells": (i64, [vp]),
        "hgks_steps_done": (i64, [vp]),
        "hgks_n_faces": (i64, [vp]),
        "hgks_kernel_times": (i32, [vp, vp, vp, ctypes.POINTER(i32), i32]),
        "hgks_last_error": (ctypes.c_char_p, [vp]),
        "hgks_destroy": (None, [vp]),
        "hgks_estimate_bytes": (ctypes.c_size_t, [i64, i64, ctypes.POINTER(Options)]),
        "hgks_server_create": (i32, [ctypes.c_size_t, i32, ctypes.POINTER(vp)]),
        "hgks_server_submit": (i32, [vp, ctypes.POINTER(Request), ctypes.POINTER(i64)]),
        "hgks_server_poll": (i32, [vp, i64, ctypes.POINTER(i32), ctypes.POINTER(Result)]),
        "hgks_server_wait": (i32, [vp, i64, ctypes.POINTER(Result)]),
        "hgks_server_get_state": (i32, [vp, i64, vp]),
        "hgks_server_release": (i32, [vp, i64]),
        "hgks_server_stats": (i32, [vp, ctypes.POINTER(ServerStats)]),
        "hgks_server_destroy": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def default_options(allocator="torch", **kw) -> Options:
    """The library's defaults with kw applied.  allocator="torch" (default)
    routes the context's device memory through PyTorch's caching allocator,
    None through hipMalloc."""
    o = Options()
    load_library().hgks_default_options(ctypes.byref(o))
    if allocator == "torch":
        o.dev_alloc, o.dev_free = torch_allocator_hook()
    elif allocator is not None:
        raise ValueError(f"allocator must be 'torch' or None, not {allocator!r}")
    for k, v in kw.items():
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


class Solver:
    """One steady problem: mesh, boundary kinds, free stream and state."""

    def __init__(self, mesh, kinds: dict, prim, **opts):
        self._L = load_library()
        self.opts = default_options(**opts)
        h = ctypes.c_void_p()
        self._check(self._L.hgks_create(ctypes.byref(self.opts), ctypes.byref(h)), None)
        self.h = h
        xyz, cells, bf, bt = mesh.arrays()
        # 8 nodes per cell: a hexahedral mesh
        load = self._L.hgks_load_hex_mesh if cells.shape[1] == 8 else self._L.hgks_load_mesh
        self._check(load(self.h, len(xyz), _ptr(xyz), len(cells), _ptr(cells), len(bf), _ptr(bf), _ptr(bt)))
        p = _f64(prim)
        self._check(self._L.hgks_set_freestream(self.h, _ptr(p)))
        for tag, kind in kinds.items():
            self._check(self._L.hgks_set_bc(self.h, int(tag), int(kind), None))
        self.N = int(self._L.hgks_n_cells(self.h))
        self.F = int(self._L.hgks_n_faces(self.h))

    def _check(self, st, h="self"):
        if st != 0:
            msg = self._L.hgks_last_error(self.h if h == "self" else None)
            raise HgksError(st, msg.decode() if msg else "")

    def close(self):
        if getattr(self, "h", None):
            self._L.hgks_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # --- host-array interface -------------------------------------------------
    def set_state(self, Q, G=None):
        Q = _f64(Q)
        G = None if G is None else _f64(G)
        self._check(self._L.hgks_set_state(self.h, _ptr(Q), _ptr(G)))

    def get_state(self, want_grad=False):
        Q = np.zeros((5, self.N))
        G = np.zeros((15, self.N)) if want_grad else None
        self._check(self._L.hgks_get_state(self.h, _ptr(Q), _ptr(G)))
        return (Q, G) if want_grad else Q

    def residual(self, Q=None, G=None, want_grad=False, allow_bad_state=False):
        Q = None if Q is None else _f64(Q)
        G = None if G is None else _f64(G)
        R = np.zeros((5, self.N))
        Gn = np.zeros((15, self.N)) if want_grad else None
        st = self._L.hgks_residual(self.h, _ptr(Q), _ptr(G), _ptr(R), _ptr(Gn))
        if not (allow_bad_state and st == -4):
            self._check(st)
        return (R, Gn) if want_grad else R

    def time_step(self, Q=None):
        Q = None if Q is None else _f64(Q)
        dt = np.zeros(self.N)
        self._check(self._L.hgks_time_step(self.h, _ptr(Q), _ptr(dt)))
        return dt

    def jv(self, v, sigma=0.0):
        v = _f64(v)
        Av = np.zeros((5, self.N))
        s = ctypes.c_double()
        self._check(self._L.hgks_jv(self.h, _ptr(v), float(sigma), _ptr(Av), ctypes.byref(s)))
        return Av, s.value

    def precond(self, r):
        r = _f64(r)
        out = np.zeros((5, self.N))
        self._check(self._L.hgks_precond(self.h, _ptr(r), _ptr(out)))
        return out

    def implicit_step(self):
        info = StepInfo()
        self._check(self._L.hgks_implicit_step(self.h, ctypes.byref(info)))
        return info

    def solve_steady(self, drop=1e-8, max_steps=1000, raise_on_noconv=False):
        info = SolveInfo()
        st = self._L.hgks_solve_steady(self.h, float(drop), int(max_steps), ctypes.byref(info))
        if st != 0 and (st != -5 or raise_on_noconv):
            self._check(st)
        return info

    def checkpoint(self, path):
        self._check(self._L.hgks_checkpoint(self.h, os.fsencode(path)))

    def restore(self, path):
        self._check(self._L.hgks_restore(self.h, os.fsencode(path)))

    # --- device interface (torch tensors, caller's stream) ---------------------
    def residual_dev(self, Q, R, stream=None):
        self._check(self._L.hgks_residual_dev(self.h, ctypes.c_void_p(Q.data_ptr()), ctypes.c_void_p(R.data_ptr()),
                                              ctypes.c_void_p(stream)))

    def residual_dev_static(self, Q, R, stream=None):
        """hgks_residual_dev with the work space in the library's static device
        buffer (no allocation in the call)."""
        self._check(self._L.hgks_residual_dev_static(self.h, ctypes.c_void_p(Q.data_ptr()),
                                                     ctypes.c_void_p(R.data_ptr()), ctypes.c_void_p(stream)))

    def residual_static_bytes(self):
        return int(self._L.hgks_residual_static_bytes(self.h))

    def jv_dev(self, v, Av, sigma=0.0, stream=None):
        self._check(self._L.hgks_jv_dev(self.h, ctypes.c_void_p(v.data_ptr()), float(sigma),
                                        ctypes.c_void_p(Av.data_ptr()), ctypes.c_void_p(stream)))

    def kernel_times(self):
        names = (ctypes.c_char_p * 8)()
        ms = (ctypes.c_double * 8)()
        n = ctypes.c_int32()
        self._check(self._L.hgks_kernel_times(self.h, names, ms, ctypes.byref(n), 8))
        return {names[k].decode(): ms[k] for k in range(n.value)}


def estimate_bytes(n_tets, n_bfaces, **opts):
    return int(load_library().hgks_estimate_bytes(int(n_tets), int(n_bfaces), ctypes.byref(default_options(**opts))))


class Server:
    """Continuous-batching server of steady solves (see include/hgks.h)."""

    def __init__(self, hbm_budget_bytes, max_slots):
        self._L = load_library()
        h = ctypes.c_void_p()
        st = self._L.hgks_server_create(int(hbm_budget_bytes), int(max_slots), ctypes.byref(h))
        if st != 0:
            raise HgksError(st, "server create failed")
        self.h = h
        self._keep = {}

    def submit(self, mesh, kinds: dict, prim, drop=1e-8, max_steps=1000, **opts):
        xyz, tets, bf, bt = mesh.arrays()
        if tets.shape[1] != 4:
            raise ValueError("the server takes tetrahedral meshes")
        tags = np.array(sorted(kinds), dtype=np.int32)
        knd = np.array([kinds[t] for t in sorted(kinds)], dtype=np.int32)
        r = Request()
        r.n_nodes, r.xyz, r.n_tets, r.tet2node = len(xyz), xyz.ctypes.data, len(tets), tets.ctypes.data
        r.n_bfaces, r.bface2node, r.bface_tag = len(bf), bf.ctypes.data, bt.ctypes.data
        r.n_bc, r.bc_tag, r.bc_kind = len(tags), tags.ctypes.data, knd.ctypes.data
        for k in range(5):
            r.prim_inf[k] = float(prim[k])
        r.opts = default_options(**opts)
        r.drop, r.max_steps = float(drop), int(max_steps)
        t = ctypes.c_int64()
        st = self._L.hgks_server_submit(self.h, ctypes.byref(r), ctypes.byref(t))
        if st != 0:
            raise HgksError(st, "submit failed")
        self._keep[t.value] = len(tets)
        return t.value

    def poll(self, ticket):
        done = ctypes.c_int32()
        res = Result()
        st = self._L.hgks_server_poll(self.h, int(ticket), ctypes.byref(done), ctypes.byref(res))
        if st != 0:
            raise HgksError(st, "poll failed")
        return res if done.value else None

    def wait(self, ticket):
        res = Result()
        st = self._L.hgks_server_wait(self.h, int(ticket), ctypes.byref(res))
        if st != 0:
            raise HgksError(st, "wait failed")
        return res

    def state(self, ticket):
        Q = np.zeros((5, self._keep[ticket]))
        st = self._L.hgks_server_get_state(self.h, int(ticket), ctypes.c_void_p(Q.ctypes.data))
        if st != 0:
            raise HgksError(st, "no state")
        return Q

    def release(self, ticket):
        self._L.hgks_server_release(self.h, int(ticket))
        self._keep.pop(ticket, None)

    def stats(self):
        s = ServerStats()
        self._L.hgks_server_stats(self.h, ctypes.byref(s))
        return s

    def close(self):
        if getattr(self, "h", None):
            self._L.hgks_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
