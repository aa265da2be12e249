"""Oracle for the grouped SPH neighbour search.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It is a plain,
slow, FP64 implementation of what the GPU path computes (brute-force
neighbour sets, the greedy grouping, the smoothing-length loop, density and
hydro sums), written from the paper (Ragagnin et al., "Exploiting the Space
Filling Curve Ordering of Particles in the Neighbour Search of Gadget3") and
sharing no code with the GPU library.  The arithmetic lives in
``sph_oracle.c``; this module marshals numpy arrays and performs the one
library step the definition allows (a stable sort).

Every function documents the passage of the paper it follows.  Readings of
the paper (where it is silent) are stated in ``sph_oracle.c``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sph_oracle.c")
_SO = os.path.join(_HERE, "_build", "liboracle.so")

KEY_BITS = 21  # bits per axis of the Hilbert key

_lib_handle = None


def build(force: bool = True) -> str:
    """Compile sph_oracle.c into oracle/_build/liboracle.so (gcc, OpenMP)."""
    os.makedirs(os.path.dirname(_SO), exist_ok=True)
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC",
               "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _SO)
    return _SO


def _lib():
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(_SO):
            build(force=False)
        _lib_handle = C.CDLL(_SO)
        _declare(_lib_handle)
    return _lib_handle


_P = C.c_void_p
_I32, _I64, _D, _U32 = C.c_int32, C.c_int64, C.c_double, C.c_uint32


def _declare(L):
    L.orc_set_threads.restype = None
    L.orc_set_threads.argtypes = [_I32]
    L.orc_get_threads.restype = _I32
    L.orc_get_threads.argtypes = []
    L.orc_hilbert_key_cell.restype = C.c_uint64
    L.orc_hilbert_key_cell.argtypes = [_U32, _U32, _U32, _I32]
    L.orc_hilbert_keys.restype = None
    L.orc_hilbert_keys.argtypes = [_I64, _P, _P, _P, _P, _P, _I32, _P]
    L.orc_octree.restype = _I64
    L.orc_octree.argtypes = [_I64, _P, _I32, _P, _I32, _I32, _P, _P, _P, _P, _I64,
                             _P, _P, _P, _P, _P, _P, _P]
    L.orc_groups.restype = _I64
    L.orc_groups.argtypes = [_I64, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _I32, _P]
    L.orc_ngb_count.restype = None
    L.orc_ngb_count.argtypes = [_I32, _I64, _P, _P, _P, _P, _P, _I32, _P, _P, _I64, _P,
                                _I32, _P, _P]
    L.orc_ngb_fill.restype = None
    L.orc_ngb_fill.argtypes = [_I32, _I64, _P, _P, _P, _P, _I32, _P, _P, _I64, _P, _I32,
                               _P, _P]
    L.orc_kernel_norm.restype = _D
    L.orc_kernel_norm.argtypes = [_I32]
    L.orc_kernel_w.restype = None
    L.orc_kernel_w.argtypes = [_I32, _D, _P, _P]
    L.orc_h_step.restype = _D
    L.orc_h_step.argtypes = [_I32, _I32, _I32, _D, _P, _P]
    L.orc_density.restype = None
    L.orc_density.argtypes = [_I64, _P, _P, _P, _P, _P, _I32, _P, _P, _I64, _P, _I32,
                              _I32, _I32, _I32, _I32, _I32, _P, _P, _P, _P, _P, _P, _P,
                              _P]
    L.orc_hydro.restype = None
    L.orc_hydro.argtypes = [_I64, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _I32, _P,
                            _P, _I64, _P, _I32, _I32, _D, _D, _P, _P, _P, _P, _P, _P, _P]
    L.orc_hydro_prod.restype = None
    L.orc_hydro_prod.argtypes = [_I64, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _I32,
                                 _P, _P, _I64, _P, _I32, _I32, _D, _D, _D, _D, _D, _P, _P,
                                 _P, _P, _P, _P, _P, _P, _P, _P]
    L.orc_group_superset_size.restype = _I64
    L.orc_group_superset_size.argtypes = [_I64, _P, _P, _P, _P, _I32, _P, _P, _P, _I64,
                                          _I64, _D]


def set_threads(n: int) -> None:
    """Threads of the OpenMP loops over targets."""
    _lib().orc_set_threads(int(n))


def get_threads() -> int:
    return int(_lib().orc_get_threads())


def _c(a, dtype):
    """Contiguous array of the given dtype (copy only if needed)."""
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


@dataclass
class Boxes:
    """A concatenation of periodic boxes: box b owns particles
    [off[b], off[b+1]) and has side L[b]."""
    off: np.ndarray
    L: np.ndarray

    @staticmethod
    def single(n: int, L: float = 1.0) -> "Boxes":
        return Boxes(np.array([0, n], np.int64), np.array([L], np.float64))

    @property
    def nbox(self) -> int:
        return len(self.L)

    def box_of(self) -> np.ndarray:
        n = int(self.off[-1])
        b = np.zeros(n, np.int32)
        for k in range(self.nbox):
            b[self.off[k]:self.off[k + 1]] = k
        return b


# --------------------------------------------------------------------------
# Hilbert keys and sort (Peano-Hilbert ordering of the particles)
# --------------------------------------------------------------------------
def hilbert_key_cell(ix: int, iy: int, iz: int, bits: int = KEY_BITS) -> int:
    """Hilbert index of one integer cell (Skilling's transpose algorithm)."""
    return int(_lib().orc_hilbert_key_cell(ix, iy, iz, bits))


def hilbert_keys(x, y, z, boxes: Boxes, bits: int = KEY_BITS) -> np.ndarray:
    """Per-particle Hilbert key of cell floor(x/L * 2^bits) per axis."""
    x, y, z = (_c(a, np.float64) for a in (x, y, z))
    n = len(x)
    box = _c(boxes.box_of(), np.int32)
    L = _c(boxes.L, np.float64)
    out = np.empty(n, np.uint64)
    _lib().orc_hilbert_keys(n, _ptr(x), _ptr(y), _ptr(z), _ptr(box), _ptr(L), bits,
                            _ptr(out))
    return out


def sort_order(keys, boxes: Boxes) -> np.ndarray:
    """Stable order by (box, key): ties keep the original index.  A library
    sort is the step here (numpy lexsort is stable)."""
    box = boxes.box_of()
    return np.lexsort((np.asarray(keys, np.uint64), box)).astype(np.uint32)


# --------------------------------------------------------------------------
# Octree
# --------------------------------------------------------------------------
@dataclass
class Tree:
    first: np.ndarray
    count: np.ndarray
    level: np.ndarray
    leaf: np.ndarray
    skip: np.ndarray
    bbox: np.ndarray  # [n,6] lo xyz, hi xyz
    hmax: np.ndarray

    @property
    def n(self) -> int:
        return len(self.first)


def octree(keys_sorted, x, y, z, h, boxes: Boxes, n_leaf: int,
           bits: int = KEY_BITS) -> Tree:
    """Octree over particles already in (box, key) order; nodes in pre-order."""
    k = _c(keys_sorted, np.uint64)
    x, y, z, h = (_c(a, np.float64) for a in (x, y, z, h))
    off = _c(boxes.off, np.int64)
    L = _lib()
    nn = L.orc_octree(len(k), _ptr(k), boxes.nbox, _ptr(off), n_leaf, bits, _ptr(x),
                      _ptr(y), _ptr(z), _ptr(h), 0, None, None, None, None, None, None,
                      None)
    first = np.empty(nn, np.int32)
    count = np.empty(nn, np.int32)
    level = np.empty(nn, np.int32)
    leaf = np.empty(nn, np.int32)
    skip = np.empty(nn, np.int32)
    bbox = np.empty((nn, 6), np.float64)
    hmax = np.empty(nn, np.float64)
    L.orc_octree(len(k), _ptr(k), boxes.nbox, _ptr(off), n_leaf, bits, _ptr(x), _ptr(y),
                 _ptr(z), _ptr(h), nn, _ptr(first), _ptr(count), _ptr(level), _ptr(leaf),
                 _ptr(skip), _ptr(bbox), _ptr(hmax))
    return Tree(first, count, level, leaf, skip, bbox, hmax)


# --------------------------------------------------------------------------
# Grouping
# --------------------------------------------------------------------------
POLICY_COUNT = 0
POLICY_PAPER = 1
POLICY_TREE = 2


def _per_box(v, nbox, dtype):
    a = np.asarray(v, dtype)
    if a.ndim == 0:
        a = np.full(nbox, a, dtype)
    return _c(a, dtype)


def leaf_levels(tree: Tree, n: int) -> np.ndarray:
    """Depth of the leaf that holds each particle."""
    out = np.full(n, -1, np.int32)
    for k in np.nonzero(tree.leaf)[0]:
        out[tree.first[k]:tree.first[k] + tree.count[k]] = tree.level[k]
    return out


def groups(act, x, y, z, h, boxes: Boxes, policy, n_group_max, f, level=0,
           leaf_level=None) -> np.ndarray:
    """Group starts (positions in `act`, plus A at the end) of the greedy
    grouping along the curve, one pass over the whole active list (section
    "Implementation of Neighbour Recycling using a Space Filling Curve");
    policy/n_group_max/f/level scalar or per box.  The tree policy needs
    leaf_level (leaf_levels() of the octree)."""
    act = _c(act, np.int32)
    x, y, z, h = (_c(a, np.float64) for a in (x, y, z, h))
    box = _c(boxes.box_of(), np.int32)
    nb = boxes.nbox
    pol = _per_box(policy, nb, np.int32)
    cap = _per_box(n_group_max, nb, np.int32)
    ff = _per_box(f, nb, np.float64)
    lev = _per_box(level, nb, np.int32)
    if np.any(pol == POLICY_TREE) and leaf_level is None:
        raise ValueError("the tree policy needs leaf_level")
    ll = _c(leaf_level if leaf_level is not None else np.zeros(len(x)), np.int32)
    out = np.empty(len(act) + 1, np.int32)
    G = _lib().orc_groups(len(act), _ptr(act), _ptr(x), _ptr(y), _ptr(z), _ptr(h),
                          _ptr(box), _ptr(_c(boxes.L, np.float64)), _ptr(pol), _ptr(cap),
                          _ptr(ff), _ptr(lev), _ptr(ll), KEY_BITS, _ptr(out))
    return out[:G + 1].copy()


# --------------------------------------------------------------------------
# Neighbour sets
# --------------------------------------------------------------------------
MODE_DENSITY = 0
MODE_HYDRO = 1


def ngb_count(mode, x, y, z, h, boxes: Boxes, targets, orig=None, use_grid=False):
    """(counts, fingerprints) of N_i (mode 0) or H_i (mode 1) per target;
    fingerprint = sum_j splitmix64(orig_j) mod 2^64."""
    x, y, z, h = (_c(a, np.float64) for a in (x, y, z, h))
    t = _c(targets, np.int32)
    o = None if orig is None else _c(orig, np.uint32)
    cnt = np.empty(len(t), np.int32)
    fp = np.empty(len(t), np.uint64)
    _lib().orc_ngb_count(mode, len(x), _ptr(x), _ptr(y), _ptr(z), _ptr(h), _ptr(o),
                         boxes.nbox, _ptr(_c(boxes.off, np.int64)),
                         _ptr(_c(boxes.L, np.float64)), len(t), _ptr(t), int(use_grid),
                         _ptr(cnt), _ptr(fp))
    return cnt, fp


def ngb_lists(mode, x, y, z, h, boxes: Boxes, targets, use_grid=False):
    """CSR (offsets, indices) of the neighbour sets, ascending index."""
    x, y, z, h = (_c(a, np.float64) for a in (x, y, z, h))
    t = _c(targets, np.int32)
    cnt, _ = ngb_count(mode, x, y, z, h, boxes, t, None, use_grid)
    off = np.zeros(len(t) + 1, np.int64)
    np.cumsum(cnt, out=off[1:])
    out = np.empty(int(off[-1]), np.int32)
    _lib().orc_ngb_fill(mode, len(x), _ptr(x), _ptr(y), _ptr(z), _ptr(h), boxes.nbox,
                        _ptr(_c(boxes.off, np.int64)), _ptr(_c(boxes.L, np.float64)),
                        len(t), _ptr(t), int(use_grid), _ptr(off), _ptr(out))
    return off, out


# --------------------------------------------------------------------------
# Kernels, h loop, density, hydro
# --------------------------------------------------------------------------
KERNEL_CUBIC = 0
KERNEL_WC6 = 1


def kernel_norm(kernel: int) -> float:
    return float(_lib().orc_kernel_norm(kernel))


def kernel_w(kernel: int, q: float):
    w = C.c_double()
    dw = C.c_double()
    _lib().orc_kernel_w(kernel, q, C.byref(w), C.byref(dw))
    return w.value, dw.value


def h_step(n: int, n_ngb: int, dn: int, h: float, lo: float, hi: float):
    a = C.c_double(lo)
    b = C.c_double(hi)
    hn = _lib().orc_h_step(n, n_ngb, dn, h, C.byref(a), C.byref(b))
    return hn, a.value, b.value


@dataclass
class DensityResult:
    h: np.ndarray
    nngb: np.ndarray
    iters: np.ndarray
    converged: np.ndarray
    rho: np.ndarray
    drhodh: np.ndarray
    fgrad: np.ndarray
    abs_drhodh: np.ndarray


def density(x, y, z, h, m, boxes: Boxes, targets, kernel, n_ngb, dn, max_iter=64,
            fixed_h=False, use_grid=False) -> DensityResult:
    """Smoothing-length loop then density sums for each target."""
    x, y, z, h, m = (_c(a, np.float64) for a in (x, y, z, h, m))
    t = _c(targets, np.int32)
    nt = len(t)
    r = DensityResult(*(np.empty(nt, d) for d in (np.float64, np.int32, np.int32, np.int32,
                                                  np.float64, np.float64, np.float64,
                                                  np.float64)))
    _lib().orc_density(len(x), _ptr(x), _ptr(y), _ptr(z), _ptr(h), _ptr(m), boxes.nbox,
                       _ptr(_c(boxes.off, np.int64)), _ptr(_c(boxes.L, np.float64)), nt,
                       _ptr(t), int(use_grid), kernel, n_ngb, dn, max_iter, int(fixed_h),
                       _ptr(r.h), _ptr(r.nngb), _ptr(r.iters), _ptr(r.converged),
                       _ptr(r.rho), _ptr(r.drhodh), _ptr(r.fgrad), _ptr(r.abs_drhodh))
    return r


@dataclass
class HydroResult:
    ax: np.ndarray
    ay: np.ndarray
    az: np.ndarray
    dudt: np.ndarray
    vsigmax: np.ndarray
    abs_a: np.ndarray
    abs_du: np.ndarray


def hydro(x, y, z, h, m, vx, vy, vz, u, rho, fgrad, boxes: Boxes, targets, kernel,
          gamma=5.0 / 3.0, alpha=0.8, use_grid=False) -> HydroResult:
    """Hydro accelerations, du/dt and max signal speed for each target."""
    arrs = [_c(a, np.float64) for a in (x, y, z, h, m, vx, vy, vz, u, rho, fgrad)]
    t = _c(targets, np.int32)
    nt = len(t)
    r = HydroResult(*(np.empty(nt, np.float64) for _ in range(7)))
    _lib().orc_hydro(len(arrs[0]), *(_ptr(a) for a in arrs), boxes.nbox,
                     _ptr(_c(boxes.off, np.int64)), _ptr(_c(boxes.L, np.float64)), nt,
                     _ptr(t), int(use_grid), kernel, gamma, alpha, _ptr(r.ax), _ptr(r.ay),
                     _ptr(r.az), _ptr(r.dudt), _ptr(r.vsigmax), _ptr(r.abs_a),
                     _ptr(r.abs_du))
    return r


@dataclass
class HydroProdResult:
    ax: np.ndarray
    ay: np.ndarray
    az: np.ndarray
    dudt: np.ndarray
    vsigmax: np.ndarray
    divv: np.ndarray
    dalphadt: np.ndarray
    abs_a: np.ndarray
    abs_du: np.ndarray
    abs_divv: np.ndarray  # sum of the divergence terms' magnitudes over rho_i


def hydro_prod(x, y, z, h, m, vx, vy, vz, u, rho, fgrad, alpha, boxes: Boxes, targets, kernel,
               gamma=5.0 / 3.0, alpha_u=1.0, alpha_min=0.1, alpha_max=1.0, ell=0.1,
               use_grid=False) -> HydroProdResult:
    """Gadget3's production SPH (per-particle viscosity coefficient, artificial
    conduction, velocity divergence and the viscosity switch's rate) for
    each target; see orc_hydro_prod."""
    arrs = [_c(a, np.float64) for a in (x, y, z, h, m, vx, vy, vz, u, rho, fgrad, alpha)]
    t = _c(targets, np.int32)
    nt = len(t)
    r = HydroProdResult(*(np.empty(nt, np.float64) for _ in range(10)))
    _lib().orc_hydro_prod(len(arrs[0]), *(_ptr(a) for a in arrs), boxes.nbox,
                          _ptr(_c(boxes.off, np.int64)), _ptr(_c(boxes.L, np.float64)), nt,
                          _ptr(t), int(use_grid), kernel, gamma, alpha_u, alpha_min, alpha_max,
                          ell, _ptr(r.ax), _ptr(r.ay), _ptr(r.az), _ptr(r.dudt),
                          _ptr(r.vsigmax), _ptr(r.divv), _ptr(r.dalphadt), _ptr(r.abs_a),
                          _ptr(r.abs_du), _ptr(r.abs_divv))
    return r


def group_superset_size(x, y, z, h, boxes: Boxes, act, g0, g1, R_nominal=0.0) -> int:
    """|S_g|: particles closer than R + max(h_i) to the group's first member."""
    x, y, z, h = (_c(a, np.float64) for a in (x, y, z, h))
    act = _c(act, np.int32)
    return int(_lib().orc_group_superset_size(
        len(x), _ptr(x), _ptr(y), _ptr(z), _ptr(h), boxes.nbox,
        _ptr(_c(boxes.off, np.int64)), _ptr(_c(boxes.L, np.float64)), _ptr(act), g0, g1,
        R_nominal))


# --------------------------------------------------------------------------
# One whole pass, as the oracle computes it (used by tests and the baseline)
# --------------------------------------------------------------------------
def sorted_state(state: dict, boxes: Boxes):
    """Keys, stable (box,key) order, and every per-particle array permuted."""
    keys = hilbert_keys(state["x"], state["y"], state["z"], boxes)
    perm = sort_order(keys, boxes)
    out = {k: np.asarray(v)[perm] for k, v in state.items()}
    out["orig"] = perm.astype(np.uint32)
    return keys[perm], perm, out
