"""The sort entry point that allocates nothing (sfc_sort_static) against
sfc_sort, through the C-ABI: two calls in a row on the library's static
device scratch, the second with a smaller input, each bit-identical to the
workspace sort of the same input (keys, permutation, every gathered field).
"""
import numpy as np
import pytest

from paper_1810_09898_amd import sfcngb as S
from paper_1810_09898_amd import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ("x", "y", "z", "h", "m", "vx", "vy", "vz", "u", "rho", "fgrad", "active", "orig")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    S.load_library()


def _sorted_both(w):
    """(workspace sort, static sort) of workload w: keys, perm and fields."""
    import torch
    pin = S.Particles.from_state(w.state, w.box_off, w.box_L, hydro=True)
    ctx = S.Context(w.n, len(w.box_L))
    out = []
    for call in (ctx.sfc_sort, ctx.sfc_sort_static):
        ps = pin.empty_like()
        keys = torch.empty(w.n, dtype=torch.int64, device="cuda")
        perm = torch.empty(w.n, dtype=torch.int32, device="cuda")
        call(pin, ps, keys, perm)
        torch.cuda.synchronize()
        r = {k: ps.numpy(k) for k in FIELDS}
        r["keys"] = keys.cpu().numpy()
        r["perm"] = perm.cpu().numpy()
        out.append(r)
    ctx.close()
    return out


def _same(a, b):
    for k in a:
        assert np.array_equal(a[k], b[k]), k


def test_static_sort_equals_workspace_sort_twice():
    # first call: a batch of boxes near the limit; second: one smaller box
    big = W.plummer_batch(n_boxes=5, seed0=7100, n_range=(30000, 60000))
    assert big.n <= S.SORT_STATIC_MAX_N
    print(f"[no-alloc] call 1: n={big.n} boxes={len(big.box_L)}", flush=True)
    ref, got = _sorted_both(big)
    _same(ref, got)
    small = W.lognormal_hydro(n=20000, grid=32, seed=71)
    print(f"[no-alloc] call 2: n={small.n} boxes=1", flush=True)
    ref, got = _sorted_both(small)
    _same(ref, got)


def test_static_sort_rejects_sizes_beyond_its_scratch():
    import torch
    n = S.SORT_STATIC_MAX_N + 1
    st = {"x": np.full(n, 0.5), "y": np.full(n, 0.5), "z": np.full(n, 0.5), "h": np.full(n, 0.1),
          "m": np.ones(n, np.float32), "vx": np.zeros(n, np.float32),
          "vy": np.zeros(n, np.float32), "vz": np.zeros(n, np.float32),
          "u": np.ones(n, np.float32), "rho": np.ones(n, np.float32),
          "fgrad": np.ones(n, np.float32), "active": np.ones(n, np.uint8),
          "orig": np.arange(n, dtype=np.uint32)}
    off = np.array([0, n], np.int64)
    pin = S.Particles.from_state(st, off, np.ones(1))
    ps = pin.empty_like()
    keys = torch.empty(n, dtype=torch.int64, device="cuda")
    ctx = S.Context(1000)
    with pytest.raises(S.SfcError) as e:
        ctx.sfc_sort_static(pin, ps, keys)
    assert e.value.code == S.SFC_EINVAL
    ctx.close()
