"""One pass of the hot path on the GPU through the C-ABI.

    sort (Hilbert keys + gather) -> octree -> active list + groups
        -> density (h loop, sums) -> hydro force

Every step is a call of libsfcngb; this module only allocates device arrays
(torch) and sequences the calls.  Each step reads the pristine unsorted
inputs, so repeated steps do identical work.
"""
from __future__ import annotations

import ctypes as C
import math
from dataclasses import dataclass, field, replace

import numpy as np

from . import sfcngb as S


@dataclass
class StepConfig:
    n_leaf: int = 16
    policy: int = S.POLICY_PAPER
    n_group_max: int = 32
    f: float = 0.5
    level: int = 5  # tree policy: depth of the grouping nodes
    t_cand: int = 2048
    hydro_t_cand: int = 2048
    skin: float = 1.0
    hydro_skin: float = 1.0
    keep_supersets: bool = False  # keep the supersets for reuse after a drift
    accum: int = S.ACCUM_F32
    max_iter: int = 64
    gamma: float = 5.0 / 3.0
    alpha: float = 0.8

    def with_(self, **kw):
        return replace(self, **kw)


class Pipeline:
    """Device state of one workload plus the calls of one step."""

    def __init__(self, w, cfg: StepConfig, hydro: bool | None = None, gp_box=None,
                 cand_per_particle: int | None = None):
        """cand_per_particle: capacity of the superset buffer per particle; by
        default 1.5 N_ngb per active particle (an ungrouped pass fits), times
        skin^3 for a skin wider than 1, at least 96."""
        import torch
        if cand_per_particle is None:
            grow = max(cfg.skin, cfg.hydro_skin) ** 3
            per_act = 1.5 * grow * w.n_ngb * float(np.count_nonzero(w.state["active"])) / max(w.n, 1)
            cand_per_particle = int(min(4096, max(96, math.ceil(per_act) + 16)))
        self.w = w
        self.cfg = cfg
        self.hydro = w.hydro if hydro is None else hydro
        self.pin = S.Particles.from_state(w.state, w.box_off, w.box_L, hydro=True)
        self.ps = self.pin.empty_like()
        n = w.n
        dev = "cuda"
        self.keys = torch.empty(n, dtype=torch.int64, device=dev)
        t_max = max(cfg.t_cand, cfg.hydro_t_cand)
        t_max = max(64, ((t_max + 63) // 64) * 64)
        self.ctx = S.Context(n, len(w.box_L), n_leaf_min=min(cfg.n_leaf, 8), t_cand_max=t_max,
                             cand_per_particle=cand_per_particle,
                             keep_supersets=cfg.keep_supersets)
        f32 = lambda: torch.zeros(n, dtype=torch.float32, device=dev)  # noqa: E731
        f64 = lambda: torch.zeros(n, dtype=torch.float64, device=dev)  # noqa: E731
        i32 = lambda: torch.zeros(n, dtype=torch.int32, device=dev)  # noqa: E731
        self.o = {"drhodh": f32(), "nngb": i32(), "iters": i32(),
                  "converged": torch.zeros(n, dtype=torch.uint8, device=dev)}
        if cfg.accum == S.ACCUM_F64:
            self.o.update(rho64=f64(), drhodh64=f64(), fgrad64=f64())
        if self.hydro:
            self.o.update(ax=f32(), ay=f32(), az=f32(), dudt=f32(), vsigmax=f32())
            if cfg.accum == S.ACCUM_F64:
                self.o.update(ax64=f64(), ay64=f64(), az64=f64(), dudt64=f64())
        self.gp_box = gp_box
        self._build_params()

    def _build_params(self):
        cfg, w, o = self.cfg, self.w, self.o
        self.dp = S.DensityParams(w.kernel, w.n_ngb, w.dn, cfg.max_iter, int(w.fixed_h),
                                  cfg.accum, cfg.skin, cfg.t_cand)
        p = lambda k: S._ptr(o.get(k))  # noqa: E731
        self.dout = S.DensityOut(p("drhodh"), p("nngb"), p("iters"), p("converged"),
                                 p("rho64"), p("drhodh64"), p("fgrad64"))
        if self.hydro:
            self.hp = S.HydroParams(w.kernel, cfg.gamma, cfg.alpha, cfg.accum, cfg.hydro_t_cand,
                                    cfg.hydro_skin)
            self.hout = S.HydroOut(p("ax"), p("ay"), p("az"), p("dudt"), p("vsigmax"),
                                   p("ax64"), p("ay64"), p("az64"), p("dudt64"))

    # ---- the step, call by call
    def sort(self):
        self.ctx.sfc_sort(self.pin, self.ps, self.keys)

    def tree(self):
        self.ctx.tree_build(self.ps, self.keys, self.cfg.n_leaf)

    def groups(self, verify=None, t_cand=None):
        c = self.cfg
        self.ctx.group_ngb_search(self.ps, c.policy, c.n_group_max, c.f,
                                  gp_box=self.gp_box, verify=verify,
                                  t_cand=t_cand or c.t_cand, level=c.level)

    def density(self, reuse=False):
        self.dp.reuse = int(reuse)
        self.ctx.density(self.ps, self.dp, self.dout)

    def hydro_force(self, reuse=False):
        self.hp.reuse = int(reuse)
        self.ctx.hydro_force(self.ps, self.hp, self.hout)

    def refit(self):
        """Node boxes and max h after the sorted particles moved in place."""
        self.ctx.tree_refit(self.ps)

    def reuse_step(self):
        """After the sorted particles moved: the step on the kept supersets
        (needs keep_supersets and a walking step since the last regrouping)."""
        self.refit()
        self.density(reuse=True)
        if self.hydro:
            self.hydro_force(reuse=True)

    def step(self):
        self.sort()
        self.tree()
        self.groups()
        self.density()
        if self.hydro:
            self.hydro_force()

    # ---- results
    def sorted_numpy(self, keys=("x", "y", "z", "h", "m", "rho", "fgrad", "active", "orig")):
        return {k: self.ps.numpy(k) for k in keys if k in self.ps.t}

    def outputs_numpy(self):
        return {k: v.cpu().numpy() for k, v in self.o.items()}

    def results_by_orig(self):
        """Per-particle results indexed by the caller's original particle id."""
        s = self.sorted_numpy()
        o = self.outputs_numpy()
        orig = s["orig"].astype(np.int64)
        n = len(orig)
        out = {}
        for k, v in list(s.items()) + list(o.items()):
            if k == "orig":
                continue
            a = np.empty(n, v.dtype)
            a[orig] = v
            out[k] = a
        return out
