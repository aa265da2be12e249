"""Pins of the oracle's hydro force, grad-h factor and h step against facts
that do not come from its own formulas.

* a two-particle pair worked by hand (tests/golden/hydro_pair.txt), which
  fixes the magnitude of every term, the kernel-gradient scale and the
  viscosity coefficient alpha/2;
* the variational origin of the grad-h equations: with every h_j tied to its
  density by (4 pi / 3) h_j^3 rho_j = M, the pressure acceleration of
  particle i is -(1/m_i) dU/dx_i of the thermal energy U = sum_j m_j u_j(rho_j)
  at fixed entropies, and du_i/dt = P_i / rho_i^2 drho_i/dt along the flow;
  both derivatives are taken by central differences of the oracle's own
  densities, so a wrong gradient scale, a missing f or a swapped h_i/h_j
  fails;
* f_i as the ratio of the constrained to the fixed-h density change, and on
  a lattice from the integer-vector enumeration;
* the h step's growth factor against the library cube root.
"""
import math
import os

import numpy as np
import pytest

import oracle
from oracle import Boxes

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
GAMMA = 5.0 / 3.0


def _golden(name):
    vals = {}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.split("#")[0].strip()
            if line:
                k, v = line.split()
                vals[k] = float(v)
    return vals


# --------------------------------------------------------------------------
# the pair worked by hand
# --------------------------------------------------------------------------
def _pair(vi, vj):
    x = np.array([0.5, 0.5 + 1.0 / 16.0])
    y = z = np.full(2, 0.5)
    h = np.array([0.25, 0.125])
    m = np.array([1.0, 0.75])
    rho = np.array([2.0, 1.0])
    fg = np.array([0.5, 1.25])
    u = np.array([0.9, 3.6])
    v = np.array([vi, vj], dtype=np.float64)
    return oracle.hydro(x, y, z, h, m, v[:, 0], v[:, 1], v[:, 2], u, rho, fg, Boxes.single(2),
                        [0, 1], 0, gamma=GAMMA, alpha=0.8)


def test_hydro_pair_worked_by_hand():
    g = _golden("hydro_pair.txt")
    C = 8.0 / math.pi
    r = _pair((0.5, 0.0, 0.0), (-0.5, 0.25, 0.0))
    assert abs(r.ax[0] / C - g["approach_ax_i_over_C"]) < 1e-12 * abs(g["approach_ax_i_over_C"])
    assert abs(r.dudt[0] / C - g["approach_dudt_i_over_C"]) < 1e-12 * abs(g["approach_dudt_i_over_C"])
    assert abs(r.vsigmax[0] - g["approach_vsig_i"]) < 1e-12
    assert abs(r.ax[1] / C - g["approach_ax_j_over_C"]) < 1e-12 * abs(g["approach_ax_j_over_C"])
    assert abs(r.dudt[1] / C - g["approach_dudt_j_over_C"]) < 1e-12 * abs(g["approach_dudt_j_over_C"])
    assert r.ay[0] == 0.0 and r.az[0] == 0.0
    r = _pair((-0.5, 0.0, 0.0), (0.5, 0.25, 0.0))
    assert abs(r.ax[0] / C - g["recede_ax_i_over_C"]) < 1e-12 * abs(g["recede_ax_i_over_C"])
    assert abs(r.dudt[0] / C - g["recede_dudt_i_over_C"]) < 1e-12 * abs(g["recede_dudt_i_over_C"])
    assert abs(r.vsigmax[0] - g["recede_vsig_i"]) < 1e-12


# --------------------------------------------------------------------------
# variational pins: h tied to the density, derivatives by central differences
# --------------------------------------------------------------------------
N_VAR = 800
# mass inside the kernel sphere, (4 pi / 3) h^3 rho: above the self term of
# either kernel ((4 pi / 3) C w(0) m = 10.7 m cubic, 28.4 m Wendland C6)
NGB_MASS = 50.0 / N_VAR


def _var_state(seed):
    rng = np.random.default_rng(seed)
    x, y, z = (rng.random(N_VAR) for _ in range(3))
    m = rng.uniform(0.5, 1.5, N_VAR) / N_VAR
    A = rng.uniform(0.5, 2.0, N_VAR)  # entropies P = A rho^gamma
    v = rng.normal(0.0, 1.0, (3, N_VAR))
    return x, y, z, m, A, v


def _solve_h(x, y, z, m, kernel):
    """h_j with (4 pi/3) h_j^3 rho_j(h_j) = NGB_MASS for every j, by bisection
    to the last bit (rho_j h_j^3 grows with h_j); returns h and the oracle's
    density result at that h."""
    n = len(x)
    B = Boxes.single(n)
    tg = np.arange(n)
    lo = np.zeros(n)
    hi = np.full(n, 0.45)
    for _ in range(80):
        mid = 0.5 * (lo + hi)
        r = oracle.density(x, y, z, mid, m, B, tg, kernel, 1, 0, fixed_h=True)
        low = 4.0 / 3.0 * math.pi * mid ** 3 * r.rho < NGB_MASS
        lo = np.where(low, mid, lo)
        hi = np.where(low, hi, mid)
        if np.all((mid == lo) | (mid == hi)) and np.all(hi - lo <= np.spacing(hi)):
            break
    h = hi
    r = oracle.density(x, y, z, h, m, B, tg, kernel, 1, 0, fixed_h=True)
    assert h.max() < 0.4  # minimum image: every neighbour within half the box
    assert (r.nngb >= 2).all()  # a root with neighbours, not the self term alone
    assert np.allclose(4.0 / 3.0 * math.pi * h ** 3 * r.rho, NGB_MASS, rtol=1e-13)
    return h, r


def _energy(x, y, z, m, A, kernel):
    h, r = _solve_h(x, y, z, m, kernel)
    return np.sum(m * A * r.rho ** (GAMMA - 1.0) / (GAMMA - 1.0))


@pytest.mark.parametrize("kernel", [0, 1])
def test_pressure_force_is_the_energy_gradient(kernel):
    x, y, z, m, A, _ = _var_state(31 + kernel)
    h, r = _solve_h(x, y, z, m, kernel)
    u = A * r.rho ** (GAMMA - 1.0) / (GAMMA - 1.0)
    zero = np.zeros(N_VAR)
    targets = [3, 117, 250]
    hy = oracle.hydro(x, y, z, h, m, zero, zero, zero, u, r.rho, r.fgrad, Boxes.single(N_VAR),
                      targets, kernel, gamma=GAMMA, alpha=0.0)
    for t, i in enumerate(targets):
        for axis, a in ((0, hy.ax), (2, hy.az)):
            eps = 2e-6
            pos = [x.copy(), y.copy(), z.copy()]
            pos[axis][i] += eps
            up = _energy(*pos, m, A, kernel)
            pos[axis][i] -= 2 * eps
            um = _energy(*pos, m, A, kernel)
            fd = -(up - um) / (2 * eps) / m[i]
            assert abs(fd - a[t]) < 1e-5 * hy.abs_a[t], (i, axis, fd, a[t])


@pytest.mark.parametrize("kernel", [0, 1])
def test_dudt_is_adiabatic_compression(kernel):
    x, y, z, m, A, v = _var_state(41 + kernel)
    h, r = _solve_h(x, y, z, m, kernel)
    u = A * r.rho ** (GAMMA - 1.0) / (GAMMA - 1.0)
    targets = [5, 199, 321]
    hy = oracle.hydro(x, y, z, h, m, v[0], v[1], v[2], u, r.rho, r.fgrad, Boxes.single(N_VAR),
                      targets, kernel, gamma=GAMMA, alpha=0.0)
    eps = 1e-6
    _, rp = _solve_h(x + eps * v[0], y + eps * v[1], z + eps * v[2], m, kernel)
    _, rm = _solve_h(x - eps * v[0], y - eps * v[1], z - eps * v[2], m, kernel)
    for t, i in enumerate(targets):
        P = A[i] * r.rho[i] ** GAMMA
        fd = P / r.rho[i] ** 2 * (rp.rho[i] - rm.rho[i]) / (2 * eps)
        assert abs(fd - hy.dudt[t]) < 1e-5 * hy.abs_du[t], (i, fd, hy.dudt[t])


@pytest.mark.parametrize("kernel", [0, 1])
def test_fgrad_is_the_constrained_density_change(kernel):
    # along a displacement field: drho_i (h tied to rho) = f_i drho_i (h fixed)
    x, y, z, m, _, v = _var_state(51 + kernel)
    h, r = _solve_h(x, y, z, m, kernel)
    eps = 1e-6
    B = Boxes.single(N_VAR)
    tg = np.arange(N_VAR)
    _, rp = _solve_h(x + eps * v[0], y + eps * v[1], z + eps * v[2], m, kernel)
    _, rm = _solve_h(x - eps * v[0], y - eps * v[1], z - eps * v[2], m, kernel)
    fp = oracle.density(x + eps * v[0], y + eps * v[1], z + eps * v[2], h, m, B, tg, kernel, 1, 0,
                        fixed_h=True)
    fm = oracle.density(x - eps * v[0], y - eps * v[1], z - eps * v[2], h, m, B, tg, kernel, 1, 0,
                        fixed_h=True)
    total = rp.rho - rm.rho
    fixed = fp.rho - fm.rho
    ok = np.abs(fixed) > 1e-3 * np.abs(fixed).max()
    assert ok.sum() > N_VAR // 5
    ratio = total[ok] / fixed[ok]
    assert np.allclose(ratio, r.fgrad[ok], rtol=2e-5)
    # the factor is not 1 here: the pin sees it
    assert np.abs(r.fgrad - 1.0).max() > 0.05


def _lattice(n):
    a = 1.0 / n
    g = (np.arange(n) + 0.5) * a
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    return X.ravel(), Y.ravel(), Z.ravel(), a


@pytest.mark.parametrize("kernel,s2", [(0, 6.5), (1, 20.5)])
def test_lattice_fgrad_from_integer_vectors(kernel, s2):
    # rho and drho/dh of a lattice site as sums over integer vectors v with
    # |v|^2 < s2 (h = a sqrt(s2)); f from those sums
    n = 12
    x, y, z, a = _lattice(n)
    N = len(x)
    h = a * math.sqrt(s2)
    r = oracle.density(x, y, z, np.full(N, h), np.full(N, 1.0 / N), Boxes.single(N),
                       [0, 777], kernel, 64, 2, fixed_h=True)
    C = 8 / math.pi if kernel == 0 else 1365 / (64 * math.pi)
    k = int(math.isqrt(int(s2))) + 1
    sw = sd = 0.0
    for i in range(-k, k + 1):
        for j in range(-k, k + 1):
            for l in range(-k, k + 1):
                d2 = i * i + j * j + l * l
                if d2 < s2:
                    q = math.sqrt(d2 / s2)
                    if kernel == 0:
                        w = 1 - 6 * q * q + 6 * q ** 3 if q < 0.5 else 2 * (1 - q) ** 3
                        dw = -12 * q + 18 * q * q if q < 0.5 else -6 * (1 - q) ** 2
                    else:
                        w = (1 - q) ** 8 * (1 + 8 * q + 25 * q * q + 32 * q ** 3)
                        dw = -22 * q * (1 - q) ** 7 * (1 + 7 * q + 16 * q * q)
                    sw += w
                    sd += 3 * w + q * dw
    m = 1.0 / N
    rho = m * C * sw / h ** 3
    drho = -m * C * sd / h ** 4
    f = 1.0 / (1.0 + h / (3 * rho) * drho)
    assert np.allclose(r.fgrad, f, rtol=1e-12)
    assert abs(f - 1.0) > 1e-4


# --------------------------------------------------------------------------
# the h step's growth factor approximates (n_ngb / n)^(1/3)
# --------------------------------------------------------------------------
def test_h_step_factor_is_a_cube_root():
    n_ngb, dn = 295, 6
    for n in range(n_ngb // 2, 2 * n_ngb + 1):
        if abs(n - n_ngb) <= dn:  # inside the window the loop stops; no step
            continue
        hn, lo, hi = oracle.h_step(n, n_ngb, dn, 1.0, 0.0, math.inf)
        t = n_ngb / n
        # two Halley steps from 1: error of order |t - 1|^9
        assert abs(hn - t ** (1.0 / 3.0)) < 2e-3 * abs(t - 1) ** 9 + 1e-15, (n, hn)
