"""CPU-only checks of the C-ABI library: it builds, loads, exports every
declared entry point, its structs have the C layout the binding assumes, and
host-side argument checks reject bad calls without touching a GPU."""
import ctypes as C
import os
import re
import subprocess

import pytest

from paper_1810_09898_amd import sfcngb as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sfcngb.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(S.LIB_PATH):
        from paper_1810_09898_amd import build
        build.build()
    return S.load_library()


def _declared():
    txt = open(HEADER).read()
    return [n for n in re.findall(r"^SFC_API\s+[\w\s\*]*?\b(\w+)\s*\(", txt, re.M)]


def test_header_declares_the_boundary():
    names = set(_declared())
    for n in ("sfc_sort", "tree_build", "group_ngb_search", "density", "hydro_force"):
        assert n in names
    assert names == set(S.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", S.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if " T " in ln}
    missing = set(_declared()) - exported
    assert not missing, missing


def test_struct_layout_matches_c(tmp_path):
    src = tmp_path / "sz.c"
    names = ["sfc_dims", "sfc_particles", "sfc_group_params", "sfc_verify",
             "sfc_density_params", "sfc_density_out", "sfc_hydro_params", "sfc_hydro_out",
             "sfc_status", "sfc_views"]
    body = "".join(f'printf("%zu\\n", sizeof({n}));' for n in names)
    src.write_text('#include <stdio.h>\n#include "sfcngb.h"\nint main(){' + body + "return 0;}")
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    sizes = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                            check=True).stdout.split()]
    py = [S.Dims, S.CParticles, S.GroupParams, S.Verify, S.DensityParams, S.DensityOut,
          S.HydroParams, S.HydroOut, S.Status, S.Views]
    assert sizes == [C.sizeof(t) for t in py]


def test_workspace_sizes(lib):
    bad = [S.Dims(0, 1, 8, 1024), S.Dims(100, 0, 8, 1024), S.Dims(100, 1, 0, 1024),
           S.Dims(100, 1, 8, 100), S.Dims(100, 1, 8, 64 * 200), S.Dims(10, 11, 8, 1024)]
    for d in bad:
        assert lib.sfc_workspace_bytes(C.byref(d)) == 0
    sizes = [lib.sfc_workspace_bytes(C.byref(S.Dims(n, 1, 8, 1024))) for n in (1000, 10 ** 5, 10 ** 6)]
    assert 0 < sizes[0] < sizes[1] < sizes[2]
    # more boxes and smaller leaves never shrink the layout
    assert lib.sfc_workspace_bytes(C.byref(S.Dims(10 ** 5, 64, 8, 1024))) >= sizes[1]
    assert lib.sfc_workspace_bytes(C.byref(S.Dims(10 ** 5, 1, 1, 1024))) > sizes[1]
    # kept supersets: a second candidate buffer, group records and snapshots
    kept = lib.sfc_workspace_bytes(C.byref(S.Dims(10 ** 5, 1, 8, 1024, 0, 1)))
    assert kept > sizes[1] + 10 ** 5 * (96 * 4 + 2 * 32)
    assert lib.sfc_workspace_bytes(C.byref(S.Dims(10 ** 5, 1, 8, 1024, 0, 2))) == 0


def test_null_context_is_rejected(lib):
    p = S.CParticles()
    assert lib.sfc_sort(None, C.byref(p), C.byref(p), None, None) == S.SFC_EINVAL
    assert lib.tree_build(None, C.byref(p), None, 8) == S.SFC_EINVAL
    assert lib.tree_refit_hmax(None, C.byref(p)) == S.SFC_EINVAL
    assert lib.tree_refit(None, C.byref(p)) == S.SFC_EINVAL
    gp = S.GroupParams(1, 8, 0.5)
    assert lib.group_ngb_search(None, C.byref(p), C.byref(gp), None, None, 1024) == S.SFC_EINVAL
    assert lib.density(None, C.byref(p), C.byref(S.DensityParams()), None) == S.SFC_EINVAL
    assert lib.hydro_force(None, C.byref(p), C.byref(S.HydroParams()), C.byref(S.HydroOut())) == S.SFC_EINVAL
    assert lib.sfc_status_read(None, C.byref(S.Status())) == S.SFC_EINVAL
    assert lib.sfc_ctx_create(None, None) == S.SFC_EINVAL
    assert lib.sfc_get_views(None, C.byref(S.Views())) == S.SFC_EINVAL
    assert lib.sfc_graph_begin(None) == S.SFC_EINVAL
    assert lib.sfc_ctx_last_error(None) == b"no context"


def test_binding_imports_without_gpu():
    from paper_1810_09898_amd import pipeline  # noqa: F401
    assert S.POLICY_PAPER == 1 and S.KERNEL_WC6 == 1
    # the hydro skin defaults to 1 (a group ball of R_g + max h), positional or not
    assert S.HydroParams().skin == 1.0
    assert S.HydroParams(1, 5.0 / 3.0, 0.8, 0, 2048).skin == 1.0
    assert S.HydroParams(1, 5.0 / 3.0, 0.8, 0, 2048, 1.25).skin == 1.25


def test_step_parameters_marshalling():
    """The pipeline's parameter blocks carry the step configuration, the
    hydro skin and the reuse flags into the C structs (host logic only)."""
    from types import SimpleNamespace as NS
    from paper_1810_09898_amd.pipeline import Pipeline, StepConfig
    cfg = StepConfig(skin=1.1, hydro_skin=1.25, t_cand=1024, hydro_t_cand=4096,
                     keep_supersets=True)
    pl = NS(cfg=cfg, w=NS(kernel=1, n_ngb=295, dn=6, fixed_h=False), o={}, hydro=True)
    Pipeline._build_params(pl)
    assert (pl.dp.kernel, pl.dp.n_ngb, pl.dp.dn, pl.dp.t_cand) == (1, 295, 6, 1024)
    assert pl.dp.skin == 1.1 and pl.dp.reuse == 0
    assert pl.hp.skin == 1.25 and pl.hp.t_cand == 4096 and pl.hp.reuse == 0
    assert abs(pl.hp.gamma - 5.0 / 3.0) < 1e-15 and pl.hp.alpha == 0.8
