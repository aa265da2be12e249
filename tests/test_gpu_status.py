"""Status paths of the device side, through the C-ABI (the paper's analogue:
the export buffer that aborts a phase when it is full and the end of a
phase, section "Phases of Neighbour Search"): a neighbour-list buffer too
small for the lists is reported as an overflow and never written past its
end; a smoothing-length loop cut at one evaluation reports the particles
that did not converge, exactly those the oracle flags."""
import numpy as np
import pytest

import oracle
from paper_1810_09898_amd import sfcngb as S
from paper_1810_09898_amd import workloads as W
from paper_1810_09898_amd.pipeline import Pipeline, StepConfig

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    S.load_library()


@pytest.fixture(scope="module")
def plum():
    return W.plummer_clustered(n=30000, seed=2)


def _sync():
    import torch
    torch.cuda.synchronize()


def osorted(w):
    ob = oracle.Boxes(w.box_off, w.box_L)
    keys, perm, s = oracle.sorted_state(w.state, ob)
    return ob, keys, perm, s, np.nonzero(s["active"])[0]


@pytest.mark.parametrize("mode", [0, 1])
def test_list_overflow_is_reported_and_bounded(mode, plum):
    import torch
    print(f"[status] list overflow mode={mode}", flush=True)
    pl = Pipeline(plum, StepConfig(n_group_max=32))
    pl.sort()
    pl.tree()
    n = plum.n
    cnt = torch.zeros(n, dtype=torch.int32, device="cuda")
    v = S.Verify(mode, S._ptr(cnt), None, None, None, 0)
    pl.groups(verify=v, t_cand=2048)
    _sync()
    assert pl.ctx.status()["flags"] == 0
    ob, keys, perm, s, act = osorted(plum)
    c = cnt.cpu().numpy()
    per = np.zeros(n, np.int64)
    per[act] = c[act]
    off = np.zeros(n + 1, np.int64)
    np.cumsum(per, out=off[1:])
    total = int(off[-1])
    cap = total // 3
    pad = 4096
    lst = torch.full((total + pad,), -1, dtype=torch.int32, device="cuda")
    offd = torch.as_tensor(off, device="cuda")
    v = S.Verify(mode, S._ptr(cnt), None, S._ptr(offd), S._ptr(lst), cap)
    pl.ctx.status_clear()
    pl.groups(verify=v, t_cand=2048)
    _sync()
    st = pl.ctx.status(raise_on_overflow=False)
    assert st["flags"] & S.ST_LIST_OVERFLOW
    with pytest.raises(S.SfcError) as e:
        pl.ctx.status()
    assert e.value.code == S.SFC_EOVERFLOW
    out = lst.cpu().numpy()
    assert np.all(out[cap:] == -1), "written past the list capacity"
    # the lists that fit are complete and exact
    full = np.nonzero(off[act + 1] <= cap)[0]
    assert len(full) > 10
    ref_off, ref = oracle.ngb_lists(mode, s["x"], s["y"], s["z"], s["h"], ob, act[full])
    for t, i in enumerate(act[full][:200]):
        assert np.array_equal(out[off[i]:off[i + 1]], ref[ref_off[t]:ref_off[t + 1]])
    # a window one entry short for one particle: flagged as well
    off2 = off.copy()
    i0 = act[np.argmax(per[act])]
    off2[i0 + 1:] -= 1
    lst2 = torch.full((total + pad,), -1, dtype=torch.int32, device="cuda")
    v = S.Verify(mode, S._ptr(cnt), None, S._ptr(torch.as_tensor(off2, device="cuda")),
                 S._ptr(lst2), total)
    pl.ctx.status_clear()
    pl.groups(verify=v, t_cand=2048)
    _sync()
    assert pl.ctx.status(raise_on_overflow=False)["flags"] & S.ST_LIST_OVERFLOW


def test_unconverged_counts_match_the_oracle(plum):
    print("[status] max_iter=1", flush=True)
    pl = Pipeline(plum, StepConfig(n_group_max=32, max_iter=1))
    pl.sort()
    pl.tree()
    pl.groups()
    pl.ctx.status_clear()
    pl.density()
    _sync()
    st = pl.ctx.status()
    ob, keys, perm, s, act = osorted(plum)
    r = oracle.density(s["x"], s["y"], s["z"], s["h"], s["m"], ob, act, plum.kernel, plum.n_ngb,
                       plum.dn, max_iter=1)
    o = pl.outputs_numpy()
    sn = pl.sorted_numpy()
    assert (r.iters == 1).all() and np.array_equal(o["iters"][act], r.iters)
    assert np.array_equal(o["converged"][act], r.converged.astype(np.uint8))
    assert st["n_not_converged"] == int((r.converged == 0).sum()) > 0
    assert np.array_equal(sn["h"][act], r.h)
    assert np.array_equal(o["nngb"][act], r.nngb)


def test_schedule_statistics_follow_the_trace_switch():
    """With tracing on, the status reports every workgroup of the density
    group kernel and every wave of the hydro member kernel that ran, a span
    within the pass and a tail within the span; with tracing off, nothing,
    and the results are the same bits either way."""
    import torch
    w = W.lognormal_hydro(n=32768, grid=32, seed=5)
    cfg = StepConfig(n_leaf=32, n_group_max=24, f=0.5, t_cand=1024, hydro_t_cand=1024)
    pl = Pipeline(w, cfg)
    pl.step()
    _sync()
    st = pl.ctx.status()
    assert st["sched_units"] == [0, 0] and st["sched_span_us"] == [0.0, 0.0]
    ref = pl.outputs_numpy()
    pl.ctx.set_trace(True)
    pl.step()
    _sync()
    st = pl.ctx.status()
    pl.ctx.set_trace(False)
    for k in range(2):
        assert st["sched_units"][k] > 0
        assert 0.0 < st["sched_span_us"][k] < 1e6
        assert 0.0 <= st["sched_tail_us"][k] <= st["sched_span_us"][k]
    out = pl.outputs_numpy()
    for key in ("nngb", "iters", "ax", "ay", "az", "dudt", "vsigmax"):
        assert np.array_equal(out[key], ref[key]), key
    with pytest.raises(S.SfcError):
        pl.ctx._check(pl.ctx.L.sfc_ctx_set_trace(pl.ctx.h, 2))
