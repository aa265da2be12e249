"""Production SPH variant of hydro_force (per-particle viscosity coefficient,
artificial conduction, velocity divergence, viscosity switch rate) on the
GPU through the C-ABI, against oracle.hydro_prod on the same inputs: the
density fields the oracle computes (rounded to FP32 as the GPU keeps them)
and seeded alpha_i, none of them from the HIP path.  FP32 sums: a and du/dt
within 1e-5 of the sum of term magnitudes, v_sig max within 1e-6, div v
within 1e-5 of the sum of its term magnitudes, the switch rate within 1e-5 of
its two parts' magnitudes; FP64 sums: 1e-12.  Grouped and ungrouped.
The paper prints none of these formulas: parity unpinned against the paper
(the oracle is pinned by conservation and closed forms)."""
import numpy as np
import pytest

import oracle
from paper_1810_09898_amd import sfcngb as S
from paper_1810_09898_amd import workloads as W
from paper_1810_09898_amd.pipeline import Pipeline, StepConfig

pytestmark = pytest.mark.gpu
AMIN, AMAX, ELL, AU = 0.1, 1.5, 0.2, 1.0


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def case():
    w = W.lognormal_hydro(n=32768, grid=32, seed=11)
    ob = oracle.Boxes(w.box_off, w.box_L)
    keys, perm, s = oracle.sorted_state(w.state, ob)
    act = np.nonzero(s["active"])[0]
    r = oracle.density(s["x"], s["y"], s["z"], s["h"], s["m"], ob, act, w.kernel, w.n_ngb, w.dn,
                       use_grid=True)
    h = s["h"].copy()
    rho32 = s["rho"].astype(np.float32)
    fg32 = s["fgrad"].astype(np.float32)
    h[act] = r.h
    rho32[act] = r.rho.astype(np.float32)
    fg32[act] = r.fgrad.astype(np.float32)
    alpha = np.random.default_rng(5).uniform(AMIN, AMAX, len(h)).astype(np.float32)
    ref = oracle.hydro_prod(s["x"], s["y"], s["z"], h, s["m"], s["vx"], s["vy"], s["vz"], s["u"],
                            rho32.astype(np.float64), fg32.astype(np.float64),
                            alpha.astype(np.float64), ob, act, w.kernel, alpha_u=AU,
                            alpha_min=AMIN, alpha_max=AMAX, ell=ELL, use_grid=True)
    return w, s, act, h, rho32, fg32, alpha, ref


@pytest.mark.parametrize("cap,accum", [(24, S.ACCUM_F32), (1, S.ACCUM_F32), (24, S.ACCUM_F64)],
                         ids=["grouped-f32", "ungrouped-f32", "grouped-f64"])
def test_production_hydro_matches_oracle(case, cap, accum):
    import torch
    w, s, act, h, rho32, fg32, alpha, ref = case
    print(f"[hydro-prod] cap {cap} accum {accum}", flush=True)
    pl = Pipeline(w, StepConfig(n_leaf=32, n_group_max=cap, f=0.5, t_cand=2048, hydro_t_cand=2048,
                                accum=accum))
    pl.sort()
    pl.tree()
    pl.groups()
    sn = pl.sorted_numpy()
    assert np.array_equal(sn["orig"], s["orig"])
    # the oracle's density fields, as the GPU keeps them
    pl.ps.t["h"].copy_(torch.as_tensor(h, device="cuda"))
    pl.ps.t["rho"].copy_(torch.as_tensor(rho32, device="cuda"))
    pl.ps.t["fgrad"].copy_(torch.as_tensor(fg32, device="cuda"))
    n = w.n
    al = torch.as_tensor(alpha, device="cuda")
    divv = torch.zeros(n, dtype=torch.float32, device="cuda")
    rate = torch.zeros(n, dtype=torch.float32, device="cuda")
    hp = S.HydroParams(w.kernel, 5.0 / 3.0, 0.8, accum, 2048, 1.0, 0, S.HYDRO_PRODUCTION,
                       S._ptr(al), AU, AMIN, AMAX, ELL)
    ho = pl.hout
    out = S.HydroOut(ho.ax, ho.ay, ho.az, ho.dudt, ho.vsigmax, ho.ax64, ho.ay64, ho.az64, ho.dudt64,
                     S._ptr(divv), S._ptr(rate))
    pl.ctx.hydro_force(pl.ps, hp, out)
    torch.cuda.synchronize()
    assert pl.ctx.status()["flags"] == 0
    o = pl.outputs_numpy()
    tol = 1e-5 if accum == S.ACCUM_F32 else 1e-12
    if accum == S.ACCUM_F32:
        got = {k: o[k][act] for k in ("ax", "ay", "az", "dudt")}
    else:
        got = {k: o[k + "64"][act] for k in ("ax", "ay", "az", "dudt")}
    for k, r_, a in (("ax", ref.ax, ref.abs_a), ("ay", ref.ay, ref.abs_a),
                     ("az", ref.az, ref.abs_a), ("dudt", ref.dudt, ref.abs_du)):
        assert np.max(np.abs(got[k] - r_) / a) < tol, k
    assert np.max(np.abs(o["vsigmax"][act] / ref.vsigmax - 1)) < 1e-6
    dv = divv.cpu().numpy()[act]
    assert np.max(np.abs(dv - ref.divv) / ref.abs_divv) < max(tol, 1e-6)
    c = np.sqrt(5.0 / 3.0 * (2.0 / 3.0) * s["u"][act])
    al64 = alpha[act].astype(np.float64)
    scale = np.abs(al64 - AMIN) * ELL * c / h[act] + ref.abs_divv * (AMAX - al64)
    rt = rate.cpu().numpy()[act]
    assert np.max(np.abs(rt - ref.dalphadt) / scale) < max(tol, 1e-6)


def test_standard_physics_ignores_the_production_fields(case):
    """physics = standard with the production fields set computes the
    standard force (the FP32 path's outputs equal a call without them)."""
    import torch
    w, s, act, h, rho32, fg32, alpha, ref = case
    pl = Pipeline(w, StepConfig(n_leaf=32, n_group_max=24, f=0.5, t_cand=2048, hydro_t_cand=2048))
    pl.sort()
    pl.tree()
    pl.groups()
    pl.ps.t["h"].copy_(torch.as_tensor(h, device="cuda"))
    pl.ps.t["rho"].copy_(torch.as_tensor(rho32, device="cuda"))
    pl.ps.t["fgrad"].copy_(torch.as_tensor(fg32, device="cuda"))
    pl.hydro_force()
    torch.cuda.synchronize()
    a0 = pl.outputs_numpy()["ax"].copy()
    al = torch.as_tensor(alpha, device="cuda")
    hp = S.HydroParams(w.kernel, 5.0 / 3.0, 0.8, S.ACCUM_F32, 2048, 1.0, 0, S.HYDRO_STANDARD,
                       S._ptr(al), AU, AMIN, AMAX, ELL)
    pl.ctx.hydro_force(pl.ps, hp, pl.hout)
    torch.cuda.synchronize()
    assert np.array_equal(pl.outputs_numpy()["ax"], a0)
