"""Superset reuse after a drift (a Verlet skin on the group supersets),
through the C ABI, against the oracle at the drifted positions.

A walking step keeps its supersets; the sorted particles then move in place
(x += v dt, wrapped into the box), h, rho and f are set to values of the
oracle, and the step runs again on the kept supersets.  Members whose bound
no longer holds finish as members whose h outgrew the superset.  The
results must be those of the oracle, and bit for bit those of a walking
call on the same inputs (the neighbour lists, and their order, do not depend
on which superset they were filtered from)."""
import numpy as np
import pytest

import oracle
from paper_1810_09898_amd import sfcngb as S
from paper_1810_09898_amd import workloads as W
from paper_1810_09898_amd.pipeline import Pipeline, StepConfig

pytestmark = pytest.mark.gpu

TOL32 = 1e-5
# The pair displacement of the FP32 sums is the FP64 one rounded once, so
# the signal speed (w_ij = v_ij . r_ij / r) keeps FP32 accuracy also at the
# drifted positions, which are off the generator's 2^-24 grid.
TOL_VSIG = 1e-6


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    S.load_library()


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def logn():
    return W.lognormal_hydro(n=65536, grid=64, seed=3)


@pytest.fixture(scope="module")
def sorted_ref(logn):
    ob = oracle.Boxes(logn.box_off, logn.box_L)
    keys, perm, s = oracle.sorted_state(logn.state, ob)
    return ob, perm, s, np.nonzero(s["active"])[0]


def drifted(s, L, frac, ref="min"):
    """x + v dt wrapped into [0, L), dt such that the fastest particle moves
    frac times the smallest h (a global Courant-limited step: ref "min") or
    the median h."""
    v = np.sqrt(s["vx"].astype(np.float64) ** 2 + s["vy"].astype(np.float64) ** 2
                + s["vz"].astype(np.float64) ** 2)
    hr = float(np.min(s["h"])) if ref == "min" else float(np.median(s["h"]))
    dt = frac * hr / float(v.max())
    out = {}
    for c, vc in (("x", "vx"), ("y", "vy"), ("z", "vz")):
        a = np.mod(s[c] + dt * s[vc].astype(np.float64), L)
        a[a >= L] -= L
        out[c] = a
    return out


def upload(pl, **arrays):
    import torch
    for k, a in arrays.items():
        t = pl.ps.t[k]
        t.copy_(torch.from_numpy(np.ascontiguousarray(a, dtype=t.cpu().numpy().dtype)))


def outputs(pl, keys):
    import torch
    torch.cuda.synchronize()
    o = {**pl.sorted_numpy(("h", "rho", "fgrad")), **pl.outputs_numpy()}
    return {k: o[k].copy() for k in keys}


DKEYS = ("h", "rho", "fgrad", "drhodh", "nngb", "iters")
HKEYS = ("ax", "ay", "az", "dudt", "vsigmax")


@pytest.mark.parametrize("frac,ref,skin", [(0.1, "min", 1.25), (0.1, "min", 1.0),
                                          (1.0, "median", 1.25)])
def test_reuse_after_drift(frac, ref, skin, logn, sorted_ref):
    say(f"[reuse] drift {frac} {ref} h, skin {skin}")
    import torch
    ob, perm, s, act = sorted_ref
    w = logn
    L = float(w.box_L[0])
    cfg = StepConfig(n_leaf=128, n_group_max=32, t_cand=2048, hydro_t_cand=2048, skin=skin,
                     hydro_skin=skin, keep_supersets=True)
    pl = Pipeline(w, cfg)
    # the walking step that keeps its supersets
    pl.sort()
    pl.tree()
    pl.groups()
    pl.ctx.status_clear()
    pl.density()
    torch.cuda.synchronize()
    walks_fresh = pl.ctx.status()["n_walks"]
    pl.hydro_force()
    torch.cuda.synchronize()
    assert pl.ctx.status()["flags"] == 0
    assert np.array_equal(pl.sorted_numpy(("orig",))["orig"].astype(np.int64), perm)

    # drift; h from the oracle's step before (both sides iterate from it)
    h1 = s["h"].copy()
    h1[act] = oracle.density(s["x"], s["y"], s["z"], s["h"], s["m"], ob, act, w.kernel, w.n_ngb,
                             w.dn, use_grid=True).h
    d = drifted(s, L, frac, ref)
    r = oracle.density(d["x"], d["y"], d["z"], h1, s["m"], ob, act, w.kernel, w.n_ngb, w.dn,
                       use_grid=True)
    upload(pl, x=d["x"], y=d["y"], z=d["z"], h=h1)
    pl.ctx.status_clear()
    pl.refit()
    pl.density(reuse=True)
    dr = outputs(pl, DKEYS)
    st = pl.ctx.status()
    assert st["flags"] == 0
    say(f"  density walks: fresh {walks_fresh}, reuse {st['n_walks']}, deferred {st['n_deferred']}")
    if ref == "min":  # the kept supersets save walks
        assert st["n_walks"] < walks_fresh
    if ref == "median":
        assert st["n_deferred"] > 0
    assert np.array_equal(dr["h"][act], r.h)
    assert np.array_equal(dr["nngb"][act], r.nngb)
    assert np.max(np.abs(dr["rho"][act] / r.rho - 1)) < TOL32

    # the same density call walking: the same bits
    upload(pl, h=h1)
    pl.density(reuse=False)
    dw = outputs(pl, DKEYS)
    for k in DKEYS:
        assert np.array_equal(dr[k], dw[k]), k

    # hydro on the oracle's density fields
    h = h1.copy()
    rho = s["rho"].astype(np.float64)
    fg = s["fgrad"].astype(np.float64)
    h[act], rho[act], fg[act] = r.h, r.rho, r.fgrad
    hr = oracle.hydro(d["x"], d["y"], d["z"], h, s["m"], s["vx"], s["vy"], s["vz"], s["u"], rho, fg,
                      ob, act, w.kernel, use_grid=True)
    upload(pl, h=h, rho=rho, fgrad=fg)
    pl.ctx.status_clear()
    pl.hydro_force(reuse=True)
    hre = outputs(pl, HKEYS)
    st = pl.ctx.status()
    assert st["flags"] == 0
    say(f"  hydro reuse: walks {st['n_walks']}, deferred {st['n_deferred']}")
    for k, ref, A in (("ax", hr.ax, hr.abs_a), ("ay", hr.ay, hr.abs_a), ("az", hr.az, hr.abs_a),
                      ("dudt", hr.dudt, hr.abs_du)):
        assert np.max(np.abs(hre[k][act] - ref) / A) < TOL32, k
    assert np.max(np.abs(hre["vsigmax"][act] / hr.vsigmax - 1)) < TOL_VSIG
    pl.hydro_force(reuse=False)
    hw = outputs(pl, HKEYS)
    for k in HKEYS:
        assert np.array_equal(hre[k], hw[k]), k


def test_reuse_fp64_sums(logn, sorted_ref):
    """The FP64-accumulator kernels on kept supersets, skin 1 (many hydro
    members outgrow theirs and walk in the pass of their own): within 1e-12
    of the oracle."""
    say("[reuse] FP64 sums, skin 1.0")
    import torch
    ob, perm, s, act = sorted_ref
    w = logn
    L = float(w.box_L[0])
    pl = Pipeline(w, StepConfig(n_leaf=128, n_group_max=32, accum=S.ACCUM_F64, keep_supersets=True))
    pl.step()
    torch.cuda.synchronize()
    h1 = s["h"].copy()
    h1[act] = oracle.density(s["x"], s["y"], s["z"], s["h"], s["m"], ob, act, w.kernel, w.n_ngb,
                             w.dn, use_grid=True).h
    d = drifted(s, L, 0.1)
    r = oracle.density(d["x"], d["y"], d["z"], h1, s["m"], ob, act, w.kernel, w.n_ngb, w.dn,
                       use_grid=True)
    upload(pl, x=d["x"], y=d["y"], z=d["z"], h=h1)
    pl.refit()
    pl.density(reuse=True)
    o = outputs(pl, ("h", "rho64"))
    assert np.array_equal(o["h"][act], r.h)
    assert np.max(np.abs(o["rho64"][act] / r.rho - 1)) < 1e-12
    h = h1.copy()
    rho = s["rho"].astype(np.float64)
    fg = s["fgrad"].astype(np.float64)
    h[act], rho[act], fg[act] = r.h, r.rho, r.fgrad
    # rho and f enter the hydro pass as FP32 fields: both sides take the FP32 values
    rho32 = rho.astype(np.float32).astype(np.float64)
    fg32 = fg.astype(np.float32).astype(np.float64)
    hr = oracle.hydro(d["x"], d["y"], d["z"], h, s["m"], s["vx"], s["vy"], s["vz"], s["u"], rho32,
                      fg32, ob, act, w.kernel, use_grid=True)
    upload(pl, h=h, rho=rho32, fgrad=fg32)
    pl.ctx.status_clear()
    pl.hydro_force(reuse=True)
    ho = outputs(pl, ("ax64", "ay64", "az64", "dudt64"))
    st = pl.ctx.status()
    assert st["flags"] == 0
    say(f"  hydro deferred {st['n_deferred']} of {len(act)}")
    assert st["n_deferred"] > 0
    for k, ref, A in (("ax64", hr.ax, hr.abs_a), ("ay64", hr.ay, hr.abs_a), ("az64", hr.az, hr.abs_a),
                      ("dudt64", hr.dudt, hr.abs_du)):
        assert np.max(np.abs(ho[k][act] - ref) / A) < 1e-12, k


def test_reuse_twice_in_a_row(logn, sorted_ref):
    """Two drifts on the same kept supersets: the bound is taken from the
    snapshot of the walk, not from the previous reuse."""
    say("[reuse] two drifts")
    import torch
    ob, perm, s, act = sorted_ref
    w = logn
    L = float(w.box_L[0])
    pl = Pipeline(w, StepConfig(n_leaf=128, n_group_max=32, skin=1.25, hydro_skin=1.25,
                                keep_supersets=True))
    pl.sort()
    pl.tree()
    pl.groups()
    pl.density()
    for frac in (0.1, 0.3):
        d = drifted(s, L, frac)
        upload(pl, x=d["x"], y=d["y"], z=d["z"], h=s["h"])
        pl.refit()
        pl.density(reuse=True)
        torch.cuda.synchronize()
        assert pl.ctx.status()["flags"] == 0
    r = oracle.density(d["x"], d["y"], d["z"], s["h"], s["m"], ob, act, w.kernel, w.n_ngb, w.dn,
                       use_grid=True)
    dr = outputs(pl, DKEYS)
    assert np.array_equal(dr["h"][act], r.h)
    assert np.max(np.abs(dr["rho"][act] / r.rho - 1)) < TOL32


def test_reuse_finer_bin(logn, sorted_ref):
    """A finer timestep bin: after the drift only a subset of the grouped
    particles is active; the reuse call computes exactly those, against the
    oracle, and leaves the others alone.  An active particle outside every
    kept group is reported."""
    say("[reuse] finer bin (10% of the grouped particles)")
    import torch
    ob, perm, s, act = sorted_ref
    w = logn
    L = float(w.box_L[0])
    pl = Pipeline(w, StepConfig(n_leaf=128, n_group_max=32, skin=1.25, hydro_skin=1.25,
                                keep_supersets=True))
    pl.step()
    torch.cuda.synchronize()
    rng = np.random.default_rng(7)
    sub = np.sort(act[rng.random(len(act)) < 0.1])
    rest = np.setdiff1d(act, sub)
    a_now = np.zeros(w.n, np.uint8)
    a_now[sub] = 1
    d = drifted(s, L, 0.2)
    upload(pl, x=d["x"], y=d["y"], z=d["z"], h=s["h"], active=a_now)
    pl.ctx.status_clear()
    pl.refit()
    pl.density(reuse=True)
    dr = outputs(pl, DKEYS)
    assert pl.ctx.status()["flags"] == 0
    r = oracle.density(d["x"], d["y"], d["z"], s["h"], s["m"], ob, sub, w.kernel, w.n_ngb, w.dn,
                       use_grid=True)
    assert np.array_equal(dr["h"][sub], r.h)
    assert np.max(np.abs(dr["rho"][sub] / r.rho - 1)) < TOL32
    assert np.array_equal(dr["h"][rest], s["h"][rest])  # not computed
    h = s["h"].copy()
    rho = s["rho"].astype(np.float64)
    fg = s["fgrad"].astype(np.float64)
    h[sub], rho[sub], fg[sub] = r.h, r.rho, r.fgrad
    hr = oracle.hydro(d["x"], d["y"], d["z"], h, s["m"], s["vx"], s["vy"], s["vz"], s["u"], rho, fg,
                      ob, sub, w.kernel, use_grid=True)
    upload(pl, h=h, rho=rho, fgrad=fg)
    pl.hydro_force(reuse=True)
    hre = outputs(pl, HKEYS)
    assert pl.ctx.status()["flags"] == 0
    for k, ref, A in (("ax", hr.ax, hr.abs_a), ("ay", hr.ay, hr.abs_a), ("az", hr.az, hr.abs_a),
                      ("dudt", hr.dudt, hr.abs_du)):
        assert np.max(np.abs(hre[k][sub] - ref) / A) < TOL32, k
    # a particle that was not grouped, active now: reported
    outside = np.nonzero(s["active"] == 0)[0][:5]
    a_now[outside] = 1
    upload(pl, active=a_now)
    pl.density(reuse=True)
    torch.cuda.synchronize()
    assert pl.ctx.status()["flags"] & S.ST_REUSE_ACTIVE


def test_reuse_batch_of_boxes():
    """Six periodic boxes in one launch: the drift bound takes each
    particle's displacement in its own box (minimum image), and the reuse
    matches the oracle box by box."""
    say("[reuse] batch of 6 boxes")
    import torch
    w = W.plummer_batch(n_boxes=6, seed0=1000, n_range=(2000, 30000))
    ob = oracle.Boxes(w.box_off, w.box_L)
    keys, perm, s = oracle.sorted_state(w.state, ob)
    act = np.nonzero(s["active"])[0]
    # the step before has converged h (the oracle's), as in a running simulation
    h1 = s["h"].copy()
    h1[act] = oracle.density(s["x"], s["y"], s["z"], s["h"], s["m"], ob, act, w.kernel, w.n_ngb,
                             w.dn).h
    w.state["h"] = w.state["h"].copy()
    w.state["h"][perm] = h1
    pl = Pipeline(w, StepConfig(n_leaf=16, n_group_max=16, f=0.5, t_cand=1024, skin=1.1,
                                keep_supersets=True), cand_per_particle=256)
    pl.step()
    torch.cuda.synchronize()
    st = pl.ctx.status(raise_on_overflow=False)
    say(f"  walking step: overflow {st['n_overflow']}, deferred {st['n_deferred']}")
    assert st["flags"] == 0 and st["n_overflow"] == 0
    # random displacements, the largest 0.1 of the smallest h; every box has L = 1
    rng = np.random.default_rng(11)
    disp = rng.normal(size=(3, w.n))
    disp *= 0.1 * float(s["h"].min()) / float(np.sqrt((disp ** 2).sum(0)).max())
    d = {}
    for c, dc in zip("xyz", disp):
        a_ = np.mod(s[c] + dc, 1.0)
        a_[a_ >= 1.0] -= 1.0
        d[c] = a_
    r = oracle.density(d["x"], d["y"], d["z"], h1, s["m"], ob, act, w.kernel, w.n_ngb, w.dn)
    upload(pl, x=d["x"], y=d["y"], z=d["z"], h=h1)
    pl.ctx.status_clear()
    pl.reuse_step()
    dr = outputs(pl, DKEYS)
    st = pl.ctx.status()
    assert st["flags"] == 0
    say(f"  walks {st['n_walks']}, deferred {st['n_deferred']} of {len(act)}")
    assert st["n_deferred"] < len(act) // 10
    assert np.array_equal(dr["h"][act], r.h)
    assert np.array_equal(dr["nngb"][act], r.nngb)
    assert np.max(np.abs(dr["rho"][act] / r.rho - 1)) < TOL32


def test_reuse_step_in_a_graph(logn, sorted_ref):
    """The reuse step (refit, density, hydro on the kept supersets) captured
    as one HIP graph: every replay gives the eager bits."""
    say("[reuse] graph capture and replay")
    import torch
    ob, perm, s, act = sorted_ref
    L = float(logn.box_L[0])
    d = drifted(s, L, 0.1)
    st_ = torch.cuda.Stream()
    with torch.cuda.stream(st_):
        pl = Pipeline(logn, StepConfig(n_leaf=128, n_group_max=32, skin=1.1, hydro_skin=1.1,
                                       t_cand=4096, hydro_t_cand=4096, keep_supersets=True))
        pl.step()
        st_.synchronize()
        h1 = pl.ps.t["h"].clone()
        upload(pl, x=d["x"], y=d["y"], z=d["z"])
        pl.reuse_step()
        ref = outputs(pl, DKEYS + HKEYS)
        pl.ps.t["h"].copy_(h1)
        pl.ctx.graph_begin()
        pl.reuse_step()
        g = pl.ctx.graph_end()
        try:
            for rep in range(3):
                for t in pl.o.values():
                    t.zero_()
                pl.ps.t["h"].copy_(h1)
                pl.ctx.graph_launch(g)
                st_.synchronize()
                got = outputs(pl, DKEYS + HKEYS)
                for k in DKEYS + HKEYS:
                    assert np.array_equal(ref[k], got[k]), (rep, k)
        finally:
            pl.ctx.graph_destroy(g)
        assert pl.ctx.status()["flags"] == 0


def test_status_clear_keeps_the_tree(logn):
    """Clearing the status counters between the tree and the hydro pass
    keeps the node count that the refits read: the same bits either way."""
    say("[status] clear between tree and hydro")
    import torch
    outs = []
    for clear in (False, True):
        pl = Pipeline(logn, StepConfig(n_leaf=128, n_group_max=32))
        pl.sort()
        pl.tree()
        pl.groups()
        torch.cuda.synchronize()
        nodes = pl.ctx.status()["n_nodes"]
        if clear:
            pl.ctx.status_clear()
            st = pl.ctx.status()
            assert st["n_nodes"] == nodes and st["n_deferred"] == 0
        pl.density()
        pl.hydro_force()
        outs.append(outputs(pl, DKEYS + HKEYS))
    for k in DKEYS + HKEYS:
        assert np.array_equal(outs[0][k], outs[1][k]), k


def test_reuse_with_no_member_active(logn, sorted_ref):
    """A reuse call when no particle is active: nothing is computed, nothing
    flagged, every output untouched."""
    say("[reuse] no member active now")
    import torch
    ob, perm, s, act = sorted_ref
    pl = Pipeline(logn, StepConfig(n_leaf=128, n_group_max=32, skin=1.1, hydro_skin=1.1,
                                   keep_supersets=True))
    pl.step()
    torch.cuda.synchronize()
    before = outputs(pl, DKEYS + HKEYS)
    upload(pl, active=np.zeros(logn.n, np.uint8))
    pl.ctx.status_clear()
    pl.reuse_step()
    after = outputs(pl, DKEYS + HKEYS)
    st = pl.ctx.status()
    assert st["flags"] == 0 and st["n_walks"] == 0 and st["sum_pairs"] == 0
    for k in DKEYS + HKEYS:
        assert np.array_equal(before[k], after[k]), k


def test_reuse_errors(logn):
    """Reuse without kept supersets, after a new sort, or with another tile
    is refused on the host."""
    say("[reuse] host-side errors")
    pl = Pipeline(logn, StepConfig(n_group_max=32, t_cand=1024, keep_supersets=False))
    pl.sort()
    pl.tree()
    pl.groups()
    with pytest.raises(S.SfcError) as e:
        pl.density(reuse=True)
    assert e.value.code == S.SFC_EORDER
    pk = Pipeline(logn, StepConfig(n_group_max=32, t_cand=1024, keep_supersets=True))
    pk.step()
    pk.hp.skin = 0.5
    with pytest.raises(S.SfcError) as e:
        pk.hydro_force()
    assert e.value.code == S.SFC_EINVAL
    pk.hp.skin = 1.0
    pk.dp.t_cand = 512
    with pytest.raises(S.SfcError) as e:
        pk.density(reuse=True)
    assert e.value.code == S.SFC_EINVAL
    pk.dp.t_cand = 1024
    pk.sort()
    with pytest.raises(S.SfcError) as e:
        pk.density(reuse=True)
    assert e.value.code == S.SFC_EORDER
    with pytest.raises(S.SfcError) as e:
        pk.hydro_force(reuse=True)
    assert e.value.code == S.SFC_EORDER
