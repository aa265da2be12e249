"""ctypes binding of libsfcngb (include/sfcngb.h).

Argument marshalling only: every step of the neighbour search runs in the
HIP library.  Device memory and streams come from PyTorch.  Importing this
module does not need a GPU; creating a Context does, and fails loudly when
the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libsfcngb.so")

SFC_OK, SFC_EINVAL, SFC_EWORKSPACE, SFC_EHIP, SFC_EOVERFLOW, SFC_EORDER = 0, -1, -2, -3, -4, -5
POLICY_COUNT, POLICY_PAPER, POLICY_TREE = 0, 1, 2
KERNEL_CUBIC, KERNEL_WC6 = 0, 1
ACCUM_F32, ACCUM_F64 = 0, 1
HYDRO_STANDARD, HYDRO_PRODUCTION = 0, 1
SORT_STATIC_MAX_N = 262144
ST_LIST_OVERFLOW, ST_NODE_OVERFLOW, ST_BAD_INPUT, ST_GUARD, ST_REUSE_ACTIVE = 1, 2, 4, 8, 16

EXPORTS = [
    "sfc_ctx_create", "sfc_ctx_destroy", "sfc_ctx_set_stream", "sfc_ctx_set_trace",
    "sfc_ctx_last_error",
    "sfc_ctx_cu_count", "sfc_workspace_bytes", "sfc_workspace_bind", "sfc_sort",
    "sfc_sort_static", "tree_build",
    "tree_refit_hmax", "tree_refit", "group_ngb_search", "density", "hydro_force", "sfc_status_read",
    "sfc_status_clear", "sfc_get_views", "sfc_graph_begin", "sfc_graph_end",
    "sfc_graph_launch", "sfc_graph_destroy",
]

_P = C.c_void_p


class SfcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"sfcngb error {code}: {msg}")
        self.code = code


class Dims(C.Structure):
    _fields_ = [("n", C.c_int64), ("n_boxes", C.c_int32), ("n_leaf_min", C.c_int32),
                ("t_cand_max", C.c_int32), ("cand_per_particle", C.c_int32),
                ("keep_supersets", C.c_int32)]


class CParticles(C.Structure):
    _fields_ = [("n", C.c_int64), ("n_boxes", C.c_int32), ("box_off_host", _P),
                ("box_off", _P), ("box_L", _P), ("x", _P), ("y", _P), ("z", _P), ("h", _P),
                ("m", _P), ("vx", _P), ("vy", _P), ("vz", _P), ("u", _P), ("rho", _P),
                ("fgrad", _P), ("active", _P), ("orig", _P)]


class GroupParams(C.Structure):
    _fields_ = [("policy", C.c_int32), ("n_group_max", C.c_int32), ("f", C.c_double),
                ("level", C.c_int32), ("t_cand", C.c_int32)]


class Verify(C.Structure):
    _fields_ = [("mode", C.c_int32), ("count", _P), ("fingerprint", _P), ("list_off", _P),
                ("list", _P), ("list_cap", C.c_int64)]


class DensityParams(C.Structure):
    _fields_ = [("kernel", C.c_int32), ("n_ngb", C.c_int32), ("dn", C.c_int32),
                ("max_iter", C.c_int32), ("fixed_h", C.c_int32), ("accum", C.c_int32),
                ("skin", C.c_double), ("t_cand", C.c_int32), ("reuse", C.c_int32)]


class DensityOut(C.Structure):
    _fields_ = [("drhodh", _P), ("nngb", _P), ("iters", _P), ("converged", _P),
                ("rho64", _P), ("drhodh64", _P), ("fgrad64", _P)]


class HydroParams(C.Structure):
    _fields_ = [("kernel", C.c_int32), ("gamma", C.c_double), ("alpha", C.c_double),
                ("accum", C.c_int32), ("t_cand", C.c_int32), ("skin", C.c_double),
                ("reuse", C.c_int32), ("physics", C.c_int32), ("alpha_i", _P),
                ("alpha_u", C.c_double), ("alpha_min", C.c_double), ("alpha_max", C.c_double),
                ("ell", C.c_double)]

    def __init__(self, *args, **kw):
        if len(args) < 6:  # skin defaults to 1 (a group ball of R_g + max h)
            kw.setdefault("skin", 1.0)
        super().__init__(*args, **kw)


class HydroOut(C.Structure):
    _fields_ = [("ax", _P), ("ay", _P), ("az", _P), ("dudt", _P), ("vsigmax", _P),
                ("ax64", _P), ("ay64", _P), ("az64", _P), ("dudt64", _P),
                ("divv", _P), ("dalphadt", _P)]


class Status(C.Structure):
    _fields_ = [("flags", C.c_uint32), ("n_nodes", C.c_int32), ("n_active", C.c_int32),
                ("n_groups", C.c_int32), ("n_deferred", C.c_int64), ("n_overflow", C.c_int64),
                ("n_not_converged", C.c_int64), ("sum_cand", C.c_int64),
                ("n_walks", C.c_int64), ("sum_iters", C.c_int64), ("sum_tests", C.c_int64),
                ("sum_pairs", C.c_int64), ("sched_units", C.c_int64 * 2),
                ("sched_span_us", C.c_double * 2), ("sched_tail_us", C.c_double * 2)]

    def as_dict(self):
        return {k: (list(getattr(self, k)) if k.startswith("sched") else getattr(self, k))
                for k, _ in self._fields_}


class Views(C.Structure):
    _fields_ = [("capacity", C.c_int32), ("n_nodes", _P), ("info", _P), ("lo", _P),
                ("hi", _P), ("box_root", _P), ("act", _P), ("n_act", _P), ("goff", _P),
                ("n_groups", _P)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libsfcngb.so and declare its signatures (no GPU needed)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with "
                          f"`python -m paper_1810_09898_amd.build` (hipcc, gfx950)")
    L = C.CDLL(path)
    I, PP = C.c_int, C.POINTER
    L.sfc_ctx_create.argtypes = [PP(_P), _P]
    L.sfc_ctx_create.restype = I
    L.sfc_ctx_destroy.argtypes = [_P]
    L.sfc_ctx_destroy.restype = None
    L.sfc_ctx_set_stream.argtypes = [_P, _P]
    L.sfc_ctx_set_stream.restype = I
    L.sfc_ctx_set_trace.argtypes = [_P, I]
    L.sfc_ctx_set_trace.restype = I
    L.sfc_ctx_last_error.argtypes = [_P]
    L.sfc_ctx_last_error.restype = C.c_char_p
    L.sfc_ctx_cu_count.argtypes = [_P]
    L.sfc_ctx_cu_count.restype = C.c_int32
    L.sfc_workspace_bytes.argtypes = [PP(Dims)]
    L.sfc_workspace_bytes.restype = C.c_size_t
    L.sfc_workspace_bind.argtypes = [_P, PP(Dims), _P, C.c_size_t]
    L.sfc_workspace_bind.restype = I
    L.sfc_sort.argtypes = [_P, PP(CParticles), PP(CParticles), _P, _P]
    L.sfc_sort.restype = I
    L.sfc_sort_static.argtypes = [_P, PP(CParticles), PP(CParticles), _P, _P]
    L.sfc_sort_static.restype = I
    L.tree_build.argtypes = [_P, PP(CParticles), _P, C.c_int32]
    L.tree_build.restype = I
    L.tree_refit_hmax.argtypes = [_P, PP(CParticles)]
    L.tree_refit_hmax.restype = I
    L.tree_refit.argtypes = [_P, PP(CParticles)]
    L.tree_refit.restype = I
    L.group_ngb_search.argtypes = [_P, PP(CParticles), PP(GroupParams), _P, PP(Verify),
                                   C.c_int32]
    L.group_ngb_search.restype = I
    L.density.argtypes = [_P, PP(CParticles), PP(DensityParams), PP(DensityOut)]
    L.density.restype = I
    L.hydro_force.argtypes = [_P, PP(CParticles), PP(HydroParams), PP(HydroOut)]
    L.hydro_force.restype = I
    L.sfc_status_read.argtypes = [_P, PP(Status)]
    L.sfc_status_read.restype = I
    L.sfc_status_clear.argtypes = [_P]
    L.sfc_status_clear.restype = I
    L.sfc_get_views.argtypes = [_P, PP(Views)]
    L.sfc_get_views.restype = I
    L.sfc_graph_begin.argtypes = [_P]
    L.sfc_graph_begin.restype = I
    L.sfc_graph_end.argtypes = [_P, PP(_P)]
    L.sfc_graph_end.restype = I
    L.sfc_graph_launch.argtypes = [_P, _P]
    L.sfc_graph_launch.restype = I
    L.sfc_graph_destroy.argtypes = [_P]
    L.sfc_graph_destroy.restype = None
    _lib = L
    return L


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


# --------------------------------------------------------------------------
# particles on the device
# --------------------------------------------------------------------------
F64 = ("x", "y", "z", "h")
F32 = ("m", "vx", "vy", "vz", "u", "rho", "fgrad")


class Particles:
    """Per-particle device arrays (torch tensors) plus the box layout."""

    def __init__(self, tensors: dict, box_off: np.ndarray, box_L: np.ndarray, device):
        import torch
        self.t = tensors
        self.box_off_host = np.ascontiguousarray(box_off, np.int64)
        self.box_off = torch.as_tensor(self.box_off_host, device=device)
        self.box_L = torch.as_tensor(np.ascontiguousarray(box_L, np.float64), device=device)
        self.n = int(self.box_off_host[-1])
        self.n_boxes = len(box_L)
        self.device = device

    @staticmethod
    def from_state(state: dict, box_off, box_L, device="cuda", hydro=True):
        import torch
        t = {}
        for k in F64:
            t[k] = torch.as_tensor(np.ascontiguousarray(state[k], np.float64), device=device)
        for k in F32:
            if k in ("vx", "vy", "vz", "u") and not hydro:
                continue
            t[k] = torch.as_tensor(np.ascontiguousarray(state[k], np.float32), device=device)
        t["active"] = torch.as_tensor(np.ascontiguousarray(state["active"], np.uint8),
                                      device=device)
        t["orig"] = torch.as_tensor(np.ascontiguousarray(state["orig"], np.uint32).view(np.int32),
                                    device=device)
        return Particles(t, box_off, box_L, device)

    def empty_like(self):
        import torch
        return Particles({k: torch.empty_like(v) for k, v in self.t.items()}, self.box_off_host,
                         self.box_L.cpu().numpy(), self.device)

    def c(self) -> CParticles:
        s = CParticles()
        s.n = self.n
        s.n_boxes = self.n_boxes
        s.box_off_host = self.box_off_host.ctypes.data_as(_P)
        s.box_off = _ptr(self.box_off)
        s.box_L = _ptr(self.box_L)
        for k in F64 + F32 + ("active", "orig"):
            setattr(s, k, _ptr(self.t.get(k)))
        return s

    def numpy(self, key):
        a = self.t[key].cpu().numpy()
        return a.view(np.uint32) if key == "orig" else a


# --------------------------------------------------------------------------
# context
# --------------------------------------------------------------------------
class Context:
    """A library context bound to a torch stream and a device workspace."""

    def __init__(self, n: int, n_boxes: int = 1, n_leaf_min: int = 8, t_cand_max: int = 4096,
                 stream=None, cand_per_particle: int = 0, keep_supersets: bool = False):
        import torch
        self.L = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("sfcngb needs a GPU (torch.cuda is not available)")
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = _P()
        self._check(self.L.sfc_ctx_create(C.byref(h), _P(self.stream.cuda_stream)), None)
        self.h = h
        self.dims = Dims(n, n_boxes, n_leaf_min, t_cand_max, cand_per_particle, int(keep_supersets))
        nbytes = self.L.sfc_workspace_bytes(C.byref(self.dims))
        if nbytes == 0:
            raise SfcError(SFC_EINVAL, f"invalid workspace dims {n}, {n_boxes}")
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        self.ws_off = (-self.ws.data_ptr()) % 256
        self.ws_base = self.ws.data_ptr() + self.ws_off
        self._check(self.L.sfc_workspace_bind(self.h, C.byref(self.dims), _P(self.ws_base),
                                              nbytes))
        self.nbytes = nbytes

    def _check(self, code, h=0):
        if code != SFC_OK:
            msg = ""
            hh = self.h if h == 0 else h
            if hh is not None:
                msg = self.L.sfc_ctx_last_error(hh).decode()
            raise SfcError(code, msg)

    def close(self):
        if getattr(self, "h", None):
            self.L.sfc_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def cu_count(self) -> int:
        return int(self.L.sfc_ctx_cu_count(self.h))

    # ---- the five calls of the boundary
    def sfc_sort(self, pin: Particles, pout: Particles, keys, perm=None):
        a, b = pin.c(), pout.c()
        self._check(self.L.sfc_sort(self.h, C.byref(a), C.byref(b), _ptr(keys), _ptr(perm)))

    def sfc_sort_static(self, pin: Particles, pout: Particles, keys, perm=None):
        """sfc_sort in the library's static device scratch (no allocation,
        no workspace needed; n <= SORT_STATIC_MAX_N)."""
        a, b = pin.c(), pout.c()
        self._check(self.L.sfc_sort_static(self.h, C.byref(a), C.byref(b), _ptr(keys),
                                           _ptr(perm)))

    def tree_build(self, p: Particles, keys, n_leaf: int):
        a = p.c()
        self._check(self.L.tree_build(self.h, C.byref(a), _ptr(keys), n_leaf))

    def tree_refit_hmax(self, p: Particles):
        a = p.c()
        self._check(self.L.tree_refit_hmax(self.h, C.byref(a)))

    def tree_refit(self, p: Particles):
        a = p.c()
        self._check(self.L.tree_refit(self.h, C.byref(a)))

    def group_ngb_search(self, p: Particles, policy=POLICY_PAPER, n_group_max=32, f=0.5,
                         gp_box=None, verify: Verify | None = None, t_cand=1024, level=0):
        a = p.c()
        gp = GroupParams(policy, n_group_max, f, level)
        self._check(self.L.group_ngb_search(
            self.h, C.byref(a), None if gp_box is not None else C.byref(gp), _ptr(gp_box),
            C.byref(verify) if verify is not None else None, t_cand))

    def density(self, p: Particles, params: DensityParams, out: DensityOut | None = None):
        a = p.c()
        self._check(self.L.density(self.h, C.byref(a), C.byref(params),
                                   C.byref(out) if out is not None else None))

    def hydro_force(self, p: Particles, params: HydroParams, out: HydroOut):
        a = p.c()
        self._check(self.L.hydro_force(self.h, C.byref(a), C.byref(params), C.byref(out)))

    # ---- status, views, graphs
    def status(self, raise_on_overflow=True) -> dict:
        s = Status()
        code = self.L.sfc_status_read(self.h, C.byref(s))
        if code != SFC_OK and (raise_on_overflow or code != SFC_EOVERFLOW):
            self._check(code)
        return s.as_dict()

    def status_clear(self):
        self._check(self.L.sfc_status_clear(self.h))

    def set_trace(self, on: bool):
        """Schedule statistics of the group and member kernels (status()'s
        sched_* fields); off by default."""
        self._check(self.L.sfc_ctx_set_trace(self.h, 1 if on else 0))

    def views(self) -> Views:
        v = Views()
        self._check(self.L.sfc_get_views(self.h, C.byref(v)))
        return v

    def ws_view(self, ptr, count, dtype):
        """A torch view of `count` elements of the workspace at device address ptr."""
        import torch
        addr = ptr if isinstance(ptr, int) else ptr.value if hasattr(ptr, "value") else int(ptr)
        off = addr - self.ws.data_ptr()
        nbytes = count * torch.empty((), dtype=dtype).element_size()
        assert 0 <= off and off + nbytes <= self.ws.numel(), "view outside the workspace"
        return self.ws[off:off + nbytes].view(dtype)

    def graph_begin(self):
        self._check(self.L.sfc_graph_begin(self.h))

    def graph_end(self):
        g = _P()
        self._check(self.L.sfc_graph_end(self.h, C.byref(g)))
        return g

    def graph_launch(self, g):
        self._check(self.L.sfc_graph_launch(self.h, g))

    def graph_destroy(self, g):
        self.L.sfc_graph_destroy(g)
