"""Pins of the oracle's production SPH variant (per-particle viscosity
coefficient, artificial conduction, velocity divergence, viscosity switch
rate; oracle.hydro_prod), written from the scheme the paper cites for
Gadget3's SPH.  The paper prints none of its formulas, so parity against
the paper is unpinned; these tests pin the oracle against facts that do not
come from its own formulas:

* with every alpha_i equal and no conduction it is exactly the standard
  hydro force (itself pinned by a pair worked by hand and by the energy
  gradient);
* momentum and total energy are conserved with unequal alpha_i and with
  conduction (a non-symmetric alpha_ij, a missing half of the viscous
  heating or a sign error in the conduction breaks this);
* conduction alone conserves the thermal energy, carries heat from the
  hotter particle to the colder one, and its two-particle value equals the
  kernel derivative taken by central differences of the (pinned) density;
* the divergence of a rigid rotation is zero, and of a uniform expansion
  v = H x on a lattice it is 3H up to the lattice's discretisation (the
  integration-by-parts identity -sum_j m_j r W'(r) = 3 sum_j m_j W(r) of a
  well-sampled kernel);
* the switch rate at its end points: no change at alpha_min without
  compression, pure decay at the rate ell c / h without it.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import Boxes

GAMMA = 5.0 / 3.0


def _state(n, seed):
    rng = np.random.default_rng(seed)
    c = rng.random((5, 3))
    p = (c[rng.integers(0, 5, n)] + rng.normal(0, 0.02, (n, 3))) % 1.0
    x, y, z = (np.floor(p[:, k] * 2 ** 24) * 2.0 ** -24 for k in range(3))
    B = Boxes.single(n)
    st = {"x": x, "y": y, "z": z, "h": rng.uniform(0.01, 0.05, n)}
    keys, perm, s = oracle.sorted_state(st, B)
    s["m"] = rng.uniform(0.5, 1.5, n) / n
    s["vx"], s["vy"], s["vz"] = rng.normal(0, 0.1, (3, n))
    s["u"] = rng.uniform(0.5, 2.0, n)
    s["rho"] = rng.uniform(0.5, 3.0, n)
    s["fgrad"] = rng.uniform(0.8, 1.2, n)
    s["alpha"] = rng.uniform(0.1, 1.0, n)
    return s, B


def _prod(s, B, tg, kernel, **kw):
    return oracle.hydro_prod(s["x"], s["y"], s["z"], s["h"], s["m"], s["vx"], s["vy"], s["vz"],
                             s["u"], s["rho"], s["fgrad"], s["alpha"], B, tg, kernel, **kw)


@pytest.mark.parametrize("kernel", [0, 1])
def test_reduces_to_the_standard_force(kernel):
    n = 2000
    s, B = _state(n, 3)
    tg = np.arange(0, n, 3)
    s["alpha"] = np.full(n, 0.8)
    p = _prod(s, B, tg, kernel, alpha_u=0.0)
    r = oracle.hydro(s["x"], s["y"], s["z"], s["h"], s["m"], s["vx"], s["vy"], s["vz"], s["u"],
                     s["rho"], s["fgrad"], B, tg, kernel, alpha=0.8)
    for a, b in ((p.ax, r.ax), (p.ay, r.ay), (p.az, r.az), (p.dudt, r.dudt),
                 (p.vsigmax, r.vsigmax)):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("kernel", [0, 1])
def test_conservation_with_alpha_i_and_conduction(kernel):
    n = 3000
    s, B = _state(n, 21)
    tg = np.arange(n)
    p = _prod(s, B, tg, kernel, alpha_u=1.0)
    m = s["m"]
    scale = (m * p.abs_a).sum()
    for a in (p.ax, p.ay, p.az):
        assert abs((m * a).sum()) < 1e-12 * scale
    dE = (m * (s["vx"] * p.ax + s["vy"] * p.ay + s["vz"] * p.az + p.dudt)).sum()
    escale = (m * (np.abs(s["vx"] * p.ax) + np.abs(s["vy"] * p.ay) + np.abs(s["vz"] * p.az)
                   + p.abs_du)).sum()
    assert abs(dE) < 1e-12 * escale
    # the conduction part alone: zero velocities leave only it in du/dt
    z0 = np.zeros(n)
    s0 = dict(s, vx=z0, vy=z0, vz=z0)
    q = _prod(s0, B, tg, kernel, alpha_u=1.0)
    assert np.abs(q.dudt).max() > 0
    assert abs((m * q.dudt).sum()) < 1e-12 * (m * q.abs_du).sum()
    q0 = _prod(s0, B, tg, kernel, alpha_u=0.0)
    assert np.abs(q0.dudt).max() == 0.0


@pytest.mark.parametrize("kernel", [0, 1])
def test_conduction_pair_by_central_differences(kernel):
    # two particles at rest, the hotter one at higher pressure
    r0, hh = 0.012, 0.03
    x = np.array([0.5, 0.5 + r0])
    y = z = np.full(2, 0.5)
    h = np.full(2, hh)
    m = np.array([1.0, 2.0])
    rho = np.array([1.5, 1.1])
    u = np.array([2.0, 0.7])
    one = np.ones(2)
    B = Boxes.single(2)
    s = {"x": x, "y": y, "z": z, "h": h, "m": m, "vx": 0 * one, "vy": 0 * one, "vz": 0 * one,
         "u": u, "rho": rho, "fgrad": one, "alpha": np.full(2, 0.5)}
    au = 0.7
    p = _prod(s, B, [0, 1], kernel, alpha_u=au)
    # heat flows from hot to cold, and the pair exchange is antisymmetric
    assert p.dudt[0] < 0 < p.dudt[1]
    assert abs(m[0] * p.dudt[0] + m[1] * p.dudt[1]) < 1e-15 * abs(m[0] * p.dudt[0])
    # the radial kernel derivative by central differences of the density a
    # single unit-mass neighbour puts on a particle at fixed h
    eps = 1e-6

    def w_at(r):
        xx = np.array([0.5, 0.5 + r])
        d = oracle.density(xx, y, z, h, np.array([0.0, 1.0]), B, [0], kernel, 2, 1, fixed_h=True)
        return d.rho[0]

    F = (w_at(r0 + eps) - w_at(r0 - eps)) / (2 * eps)
    P = (GAMMA - 1) * rho * u
    rb = 0.5 * (rho[0] + rho[1])
    expect = m[1] * au * math.sqrt(abs(P[0] - P[1]) / rb) * (u[0] - u[1]) * F / rb
    assert abs(p.dudt[0] / expect - 1) < 1e-6
    # linear in alpha_u
    p2 = _prod(s, B, [0, 1], kernel, alpha_u=2 * au)
    assert abs(p2.dudt[0] / (2 * p.dudt[0]) - 1) < 1e-14


def _lattice(n):
    a = 1.0 / n
    g = (np.arange(n) + 0.5) * a
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    return X.ravel(), Y.ravel(), Z.ravel(), a


@pytest.mark.parametrize("kernel,hfac", [(0, 2.5), (1, 3.0)])
def test_divergence_of_rotation_and_expansion(kernel, hfac):
    n = 20
    x, y, z, a = _lattice(n)
    N = len(x)
    one = np.ones(N)
    B = Boxes.single(N)
    h = np.full(N, hfac * a)
    # targets whose neighbourhoods do not reach the box faces
    c = np.abs(np.stack([x, y, z]) - 0.5).max(axis=0)
    tg = np.nonzero(c < 0.5 - hfac * a - a)[0]
    rho0 = 2.0  # the density the hydro call is given (the divergence divides by it)
    s = {"x": x, "y": y, "z": z, "h": h, "m": one / N, "u": one, "rho": rho0 * one,
         "fgrad": one, "alpha": np.full(N, 0.5)}
    om = 0.3
    s.update(vx=-om * (y - 0.5), vy=om * (x - 0.5), vz=0 * one)
    p = _prod(s, B, tg, kernel)
    assert np.abs(p.divv).max() < 1e-12
    H = 0.2
    s.update(vx=H * (x - 0.5), vy=H * (y - 0.5), vz=H * (z - 0.5))
    p = _prod(s, B, tg, kernel)
    # v_ij . x_ij = H r^2, so div v = -(H / rho) sum_j m_j r W'(r):
    # the lattice sum over integer vectors, W' by central differences of the
    # density one unit-mass neighbour puts on a particle (fixed h)
    H0 = hfac * a
    eps = 1e-7
    yy = zz = np.full(2, 0.5)
    B2 = Boxes.single(2)

    def w_at(r):
        d = oracle.density(np.array([0.5, 0.5 + r]), yy, zz, np.full(2, H0),
                           np.array([0.0, 1.0]), B2, [0], kernel, 2, 1, fixed_h=True)
        return d.rho[0]

    kmax = int(hfac) + 1
    mult = {}
    for i in range(-kmax, kmax + 1):
        for j in range(-kmax, kmax + 1):
            for k in range(-kmax, kmax + 1):
                q2 = i * i + j * j + k * k
                if 0 < q2 and q2 * a * a < H0 * H0:
                    mult[q2] = mult.get(q2, 0) + 1
    S = 0.0
    for q2, cnt in mult.items():
        r = math.sqrt(q2) * a
        S += cnt * (1.0 / N) * r * (w_at(r + eps) - w_at(r - eps)) / (2 * eps)
    assert np.abs(p.divv / (-H * S / rho0) - 1).max() < 1e-5
    # and the integration-by-parts identity holds to the lattice's sampling
    d = oracle.density(x, y, z, h, one / N, B, tg, kernel, 64, 1, fixed_h=True)
    assert np.abs(p.divv * rho0 / (3 * H * d.rho) - 1).max() < 2e-2


def test_switch_rate_end_points():
    n = 2000
    s, B = _state(n, 5)
    tg = np.arange(0, n, 7)
    amin, amax, ell = 0.1, 1.0, 0.1
    c = np.sqrt(GAMMA * (GAMMA - 1) * s["u"][tg])
    # without compression at alpha_min: no change; at alpha_max: decay only
    z0 = np.zeros(n)
    s0 = dict(s, vx=z0, vy=z0, vz=z0, alpha=np.full(n, amin))
    p = _prod(s0, B, tg, 1, alpha_min=amin, alpha_max=amax, ell=ell)
    assert np.all(p.divv == 0) and np.all(p.dalphadt == 0)
    s1 = dict(s0, alpha=np.full(n, amax))
    p = _prod(s1, B, tg, 1, alpha_min=amin, alpha_max=amax, ell=ell)
    assert np.allclose(p.dalphadt, -(amax - amin) * ell * c / s["h"][tg], rtol=1e-14, atol=0)
    # compression raises alpha below alpha_max
    s2 = dict(s, alpha=np.full(n, 0.5))
    p = _prod(s2, B, tg, 1, alpha_min=amin, alpha_max=amax, ell=ell)
    comp = p.divv < 0
    src = -p.divv[comp] * (amax - 0.5)
    dec = -(0.5 - amin) * ell * c[comp] / s["h"][tg][comp]
    assert np.allclose(p.dalphadt[comp], src + dec, rtol=1e-13, atol=0)
