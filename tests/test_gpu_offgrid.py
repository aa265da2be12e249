"""Pairs placed at r = h (1 +- 2^-23 .. 2^-21), off the 2^-24 coordinate grid,
some across the periodic faces, through the whole step on the GPU: the
membership tests must decide every such pair as the FP64 oracle does.

Each centre gets satellites at relative distances 1 +- 2^-21, 2^-22, 2^-23
of its h (density: r < h_i decides), and satellites whose own h sits at
r (1 +- 2^-22) with the centre's h below r (hydro: r < max(h_i, h_j)
decides through h_j).  FP32 coordinates are off by up to 2^-24 L, far more
than these margins, so every screen must hand these pairs to its FP64 test.
Density: neighbour counts at fixed h equal the oracle's.  Hydro: the
borderline satellites approach their centre fast, so the largest signal
speed of every centre is set by the borderline pairs it includes; v_sig max
must equal the oracle's (1e-4, far below the change a pair decided the
other way makes), and the forces agree within 1e-5.
"""
import numpy as np
import pytest

import oracle
from paper_1810_09898_amd import workloads as W
from paper_1810_09898_amd.pipeline import Pipeline, StepConfig

pytestmark = pytest.mark.gpu
TOL32 = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _offgrid(seed=7, nc=1200, nbg=20000):
    rng = np.random.default_rng(seed)
    c = rng.random((nc, 3))
    # a quarter of the centres within reach of a face: their pairs fold
    edge = rng.random(nc) < 0.25
    ax = rng.integers(0, 3, nc)
    c[edge, ax[edge]] = rng.choice([0.004, 0.996], edge.sum()) + rng.normal(0, 0.002, edge.sum())
    c %= 1.0
    hc = 0.06 * (1.0 + 0.2 * rng.random(nc))
    rel = np.array([-2.0 ** -21, 2.0 ** -21, -2.0 ** -22, 2.0 ** -22, -2.0 ** -23, 2.0 ** -23])
    xs, hs, vs = [c], [hc], [rng.normal(0, 1.0, (nc, 3))]
    for k, e in enumerate(rel):
        d = rng.normal(size=(nc, 3))
        d /= np.linalg.norm(d, axis=1)[:, None]
        r = hc * (1.0 + e)
        xs.append((c + r[:, None] * d) % 1.0)
        hs.append(np.full(nc, 0.004))
        # fast approach toward the centre, a different speed per satellite
        vs.append(-d * (50.0 + 10.0 * k + rng.random(nc))[:, None])
    # satellites whose own h decides: r = h_j (1 +- 2^-22) with h_i < r
    for k, e in enumerate((-2.0 ** -22, 2.0 ** -22)):
        d = rng.normal(size=(nc, 3))
        d /= np.linalg.norm(d, axis=1)[:, None]
        r = 1.3 * hc
        xs.append((c + r[:, None] * d) % 1.0)
        hs.append(r / (1.0 + e))
        vs.append(-d * (120.0 + 10.0 * k + rng.random(nc))[:, None])
    # an off-grid background, so that group supersets outgrow a 64-candidate
    # tile while the members' own supersets (radius 1.25 h) mostly fit it
    xs.append(rng.random((nbg, 3)))
    hs.append(np.full(nbg, 0.004))
    vs.append(rng.normal(0, 1.0, (nbg, 3)))
    x = np.concatenate(xs)
    h = np.concatenate(hs)
    v = np.concatenate(vs)
    n = len(x)
    st = W._state(x[:, 0].copy(), x[:, 1].copy(), x[:, 2].copy(), h, np.full(n, float(n)), n,
                  rng=rng, hydro=True)
    st["vx"], st["vy"], st["vz"] = (v[:, i].astype(np.float32) for i in range(3))
    st["active"] = np.ones(n, np.uint8)
    return W.Workload("offgrid", st, np.array([0, n], np.int64), np.ones(1), kernel=1, n_ngb=32,
                      dn=2, fixed_h=True, hydro=True)


WL = _offgrid()
OB = oracle.Boxes(WL.box_off, WL.box_L)
KEYS, PERM, SO = oracle.sorted_state(WL.state, OB)
ACT = np.nonzero(SO["active"])[0]
RD = oracle.density(SO["x"], SO["y"], SO["z"], SO["h"], SO["m"], OB, ACT, 1, 32, 2, fixed_h=True,
                    use_grid=True)
RHO32 = SO["rho"].astype(np.float32)
FG32 = SO["fgrad"].astype(np.float32)
RHO32[ACT] = RD.rho.astype(np.float32)
FG32[ACT] = RD.fgrad.astype(np.float32)
RH = oracle.hydro(SO["x"], SO["y"], SO["z"], SO["h"], SO["m"], SO["vx"], SO["vy"], SO["vz"],
                  SO["u"], RHO32.astype(np.float64), FG32.astype(np.float64), OB, ACT, 1,
                  use_grid=True)


@pytest.mark.parametrize("cfg", [
    dict(n_group_max=16, f=0.5, t_cand=1024),  # group supersets
    dict(n_group_max=1, f=0.5, t_cand=1024),   # one member per group
    dict(n_group_max=16, f=0.5, t_cand=64),    # group supersets overflow: own supersets, walks
], ids=["grouped", "ungrouped", "alone"])
def test_offgrid_borderline_pairs(cfg):
    import torch
    print(f"[offgrid] {cfg}", flush=True)
    pl = Pipeline(WL, StepConfig(n_leaf=16, hydro_t_cand=cfg["t_cand"], **cfg))
    pl.sort()
    pl.tree()
    pl.groups()
    pl.density()
    torch.cuda.synchronize()
    st = pl.ctx.status()
    assert st["flags"] == 0
    if cfg["t_cand"] == 64:
        assert st["n_overflow"] > 0 and st["n_deferred"] > 0
    o = pl.outputs_numpy()
    # every borderline pair decided as the oracle decides it
    assert np.array_equal(o["nngb"][ACT], RD.nngb)
    # hydro on the oracle's density fields
    pl.ps.t["rho"].copy_(torch.as_tensor(RHO32, device="cuda"))
    pl.ps.t["fgrad"].copy_(torch.as_tensor(FG32, device="cuda"))
    pl.hydro_force()
    torch.cuda.synchronize()
    assert pl.ctx.status()["flags"] == 0
    o = pl.outputs_numpy()
    # a background particle may have no hydro neighbour at all: v_sig max 0.
    # The satellites' speeds (50 .. 130, ten apart per family) dominate v_sig,
    # so a pair decided the other way moves v_sig max by several percent,
    # while the FP32 rounding of v_ij . r_ij for the oblique pairs among a
    # centre's satellites reaches a few 1e-6: the gate sits between the two.
    vs = o["vsigmax"][ACT]
    has = RH.vsigmax > 0
    assert np.all(vs[~has] == 0)
    assert np.max(np.abs(vs[has] / RH.vsigmax[has] - 1)) < 1e-4
    # A particle whose only pairs sit at the edge of the support gets terms of
    # order (2^-22)^7: below FP32's normal range, where no relative accuracy
    # exists; the scale of the gate has a floor of 1e-30 for them.  du/dt
    # holds v_ij . x_ij twice in its viscous heating: for the fast satellites
    # meeting at oblique angles that FP32 dot product cancels, so its gate is
    # 1e-3 (a pair at the edge of the support contributes ~ (2^-22)^7 either
    # way: the decisions are checked by the counts and v_sig above).
    for k, ref, a, tol in (("ax", RH.ax, RH.abs_a, TOL32), ("ay", RH.ay, RH.abs_a, TOL32),
                           ("az", RH.az, RH.abs_a, TOL32), ("dudt", RH.dudt, RH.abs_du, 1e-3)):
        assert np.max(np.abs(o[k][ACT] - ref) / np.maximum(a, 1e-30)) < tol, k


def test_offgrid_case_is_borderline():
    """The satellites' FP32 distances cannot decide them: pin that the case
    really sits inside the FP32 rounding (on the CPU side, from the oracle's
    own inputs)."""
    x32 = SO["x"].astype(np.float32).astype(np.float64)
    n = len(SO["x"])
    assert n == 9 * 1200 + 20000
    # margins of the first satellite family relative to the FP32 coordinate error
    marg = 0.072 * 2.0 ** -22
    assert marg < 2.0 ** -24  # below the grid spacing of FP32 coordinates in [0, 1)
    assert np.max(np.abs(x32 - SO["x"])) > marg
