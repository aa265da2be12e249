"""Seeded synthetic particle sets for the grouped neighbour search.

This module only draws inputs: positions, masses, velocities, internal
energies, initial smoothing lengths and active flags.  It contains none of
the method's arithmetic (no Hilbert keys, no tree, no SPH kernel): both the
GPU path and the oracle consume what it returns.

The paper's test case (Magneticum box5hr, 2*81^3 particles, <N_ngb> = 291,
section "The Test Case") is not available; these generators stand in for it
with the shapes and value distributions of the five workloads below.

Common rules
  * numpy Generator(PCG64(seed));
  * positions quantised to multiples of 2^-24 in the periodic unit box, so
    that every coordinate difference and squared distance is exact in FP64;
  * m = 1/N (FP32);  u = 1, v = 0 unless stated;
  * initial h: the distance to the N_ngb-th nearest particle (self counted
    first; scipy's periodic k-d tree), times (1 + U[-0.1, 0.1]), i.e. the
    smoothing length of a previous step perturbed by +-10%;
  * stored rho for inactive particles: N_ngb m / (4/3 pi h^3), f = 1;
  * active particles come in runs that are contiguous along any octree-based
    space-filling curve: whole cells of a level-l grid (with l chosen so that
    a cell holds about `run_mean` particles) are switched on, in random order,
    until the target fraction is reached.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

QUANT = 2.0 ** -24
# when set, the slow generation steps report their progress on stderr
VERBOSE = False


def _say(msg):
    if VERBOSE:
        import sys
        print(f"# {msg}", file=sys.stderr, flush=True)


@dataclass
class Workload:
    name: str
    state: dict            # per-particle arrays, concatenated over boxes
    box_off: np.ndarray    # int64 [B+1]
    box_L: np.ndarray      # float64 [B]
    kernel: int            # 0 cubic spline, 1 Wendland C6
    n_ngb: int
    dn: int
    fixed_h: bool
    hydro: bool
    n_group_max: int = 32
    f: float = 0.5
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.box_off[-1])

    @property
    def n_active(self) -> int:
        return int(self.state["active"].sum())


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def quantise(u):
    """Map [0,1) floats to multiples of 2^-24 in [0,1)."""
    q = np.floor(np.asarray(u, np.float64) * 2.0 ** 24)
    q = np.mod(q, 2.0 ** 24)
    return q * QUANT


def uniform_positions(rng, n):
    return [quantise(rng.random(n)) for _ in range(3)]


def plummer_mixture(rng, n, n_spheres=200, background=0.3, a_range=(0.005, 0.03)):
    """30% uniform background; the rest shared by Plummer spheres with equal
    weights (multinomial), log-uniform scale radii, centres U[0,1)^3,
    r = a (U^(-2/3) - 1)^(-1/2) truncated at 10a, isotropic, periodic wrap."""
    nb = int(round(background * n))
    ns = n - nb
    counts = rng.multinomial(ns, np.full(n_spheres, 1.0 / n_spheres))
    centres = rng.random((n_spheres, 3))
    a = np.exp(rng.uniform(np.log(a_range[0]), np.log(a_range[1]), n_spheres))
    pos = [rng.random((nb, 3))]
    for s in range(n_spheres):
        k = int(counts[s])
        r = np.empty(0)
        while len(r) < k:
            u = rng.random(2 * (k - len(r)) + 8)
            u = u[u > 0]
            rr = a[s] * (u ** (-2.0 / 3.0) - 1.0) ** -0.5
            r = np.concatenate([r, rr[rr <= 10 * a[s]]])
        r = r[:k]
        d = rng.normal(size=(k, 3))
        d /= np.linalg.norm(d, axis=1)[:, None]
        pos.append(centres[s] + d * r[:, None])
    p = np.concatenate(pos)
    p = np.mod(p, 1.0)
    perm = rng.permutation(n)
    p = p[perm]
    return [quantise(p[:, k]) for k in range(3)]


def lognormal_positions(rng, n, grid=256, sigma=1.5, slope=-2.0):
    """Gaussian random field on a grid^3 mesh with P(k) ~ k^slope (k=0 zeroed,
    up to the Nyquist frequency), scaled to sigma; rho ~ exp(delta -
    sigma^2/2); counts per cell multinomial(n, rho/sum rho); positions
    uniform inside each cell."""
    kf = np.fft.fftfreq(grid) * grid
    kz = np.fft.rfftfreq(grid) * grid
    k2 = kf[:, None, None] ** 2 + kf[None, :, None] ** 2 + kz[None, None, :] ** 2
    amp = np.zeros_like(k2)
    nz = k2 > 0
    amp[nz] = k2[nz] ** (slope / 4.0)  # sqrt(P) with P ~ k^slope
    del k2
    white = rng.normal(size=(grid, grid, grid)).astype(np.float64)
    wk = np.fft.rfftn(white)
    del white
    wk *= amp
    del amp
    delta = np.fft.irfftn(wk, s=(grid, grid, grid), axes=(0, 1, 2))
    del wk
    delta *= sigma / delta.std()
    rho = np.exp(delta - 0.5 * sigma * sigma).ravel()
    del delta
    counts = rng.multinomial(n, rho / rho.sum())
    del rho
    cell = np.repeat(np.arange(grid ** 3, dtype=np.int64), counts)
    cz = cell % grid
    cy = (cell // grid) % grid
    cx = cell // (grid * grid)
    del cell
    pos = []
    for c in (cx, cy, cz):
        pos.append(quantise((c + rng.random(n)) / grid))
    perm = rng.permutation(n)
    return [p[perm] for p in pos]


def initial_h(rng, x, y, z, n_ngb, perturb=0.1, chunk=1 << 18, thin=1):
    """h0 = d_(N_ngb) * (1 + U[-perturb, perturb]), d_k the distance to the
    k-th nearest particle counting the particle itself; nd = number density
    N_ngb / (4/3 pi h0^3).  With thin > 1 the distance is that to the
    (N_ngb/thin)-th nearest of a random 1/thin of the particles (the same
    radius in expectation, at a fraction of the cost for very large N)."""
    from scipy.spatial import cKDTree
    p = np.stack([x, y, z], axis=1)
    k = n_ngb
    if thin > 1:
        sub = rng.random(len(x)) < 1.0 / thin
        tree = cKDTree(p[sub], boxsize=1.0)
        k = max(2, int(round(n_ngb / thin)))
    else:
        tree = cKDTree(p, boxsize=1.0)
    d = np.empty(len(x))
    for s in range(0, len(x), chunk):
        d[s:s + chunk] = tree.query(p[s:s + chunk], k=[k], workers=-1)[0][:, 0]
        _say(f"initial h: {min(s + chunk, len(x))}/{len(x)}")
    del tree, p
    h = d * (1.0 + rng.uniform(-perturb, perturb, len(x)))
    nd = n_ngb / (4.0 / 3.0 * math.pi * h ** 3)
    return h, nd


def active_cells(rng, x, y, z, fraction, run_mean, within=None):
    """Switch on whole level-l cells in random order until `fraction` of the
    particles are active; l is chosen so a cell holds ~run_mean particles.
    With `within` (a 0/1 mask made by this function with the same run_mean),
    only cells lying wholly inside it are drawn, so the result is a subset."""
    n = len(x)
    if fraction >= 1.0:
        return np.ones(n, np.uint8) if within is None else within.astype(np.uint8)
    lev = max(1, int(round(math.log(max(n / run_mean, 1.0), 8))))
    g = 1 << lev
    ix = np.minimum((x * g).astype(np.int64), g - 1)
    iy = np.minimum((y * g).astype(np.int64), g - 1)
    iz = np.minimum((z * g).astype(np.int64), g - 1)
    cid = (ix * g + iy) * g + iz
    cnt = np.bincount(cid, minlength=g ** 3)
    pool = cnt > 0
    if within is not None:
        pool &= np.bincount(cid, weights=within, minlength=g ** 3) == cnt
    order = rng.permutation(np.nonzero(pool)[0])
    csum = np.cumsum(cnt[order])
    take = int(np.searchsorted(csum, fraction * n)) + 1
    on = np.zeros(g ** 3, bool)
    on[order[:take]] = True
    return on[cid].astype(np.uint8)


def _state(x, y, z, h, nd, n, rng=None, hydro=False):
    m = np.full(n, 1.0 / n, np.float32)
    st = {
        "x": x.astype(np.float64), "y": y.astype(np.float64), "z": z.astype(np.float64),
        "h": np.asarray(h, np.float64),
        "m": m,
        "vx": np.zeros(n, np.float32), "vy": np.zeros(n, np.float32),
        "vz": np.zeros(n, np.float32), "u": np.ones(n, np.float32),
        "rho": (np.asarray(nd, np.float64) / n).astype(np.float32),
        "fgrad": np.ones(n, np.float32),
        "orig": np.arange(n, dtype=np.uint32),
    }
    if hydro:
        st["u"] = rng.uniform(0.5, 2.0, n).astype(np.float32)
        v = rng.normal(0.0, 0.1, (3, n)).astype(np.float32)
        st["vx"], st["vy"], st["vz"] = v[0], v[1], v[2]
    return st


def _one_box(n):
    return np.array([0, n], np.int64), np.array([1.0], np.float64)


# --------------------------------------------------------------------------
# The five workloads
# --------------------------------------------------------------------------
def uniform_fixed_h(n=32768, seed=1, n_ngb=64):
    """N uniform particles, cubic spline, fixed h = (3 n_ngb / (4 pi N))^(1/3)
    (E[n_i] = 1 + (N-1) 4/3 pi h^3 ~ n_ngb + 1), all active, density only."""
    rng = _rng(seed)
    x, y, z = uniform_positions(rng, n)
    h0 = (3.0 * n_ngb / (4.0 * math.pi * n)) ** (1.0 / 3.0)
    st = _state(x, y, z, np.full(n, h0), np.full(n, float(n)), n)
    st["active"] = np.ones(n, np.uint8)
    off, L = _one_box(n)
    return Workload("uniform_fixed_h", st, off, L, kernel=0, n_ngb=n_ngb, dn=2,
                    fixed_h=True, hydro=False, n_group_max=1, f=0.5,
                    meta={"seed": seed, "h": h0})


def plummer_clustered(n=262144, seed=2, active=0.10, n_ngb=64, dn=2, run_mean=64):
    """30% uniform + 200 Plummer spheres, cubic N_ngb=64, 10% active runs."""
    rng = _rng(seed)
    x, y, z = plummer_mixture(rng, n)
    h, nd = initial_h(rng, x, y, z, n_ngb)
    st = _state(x, y, z, h, nd, n)
    st["active"] = active_cells(rng, x, y, z, active, run_mean)
    off, L = _one_box(n)
    return Workload("plummer_clustered", st, off, L, kernel=0, n_ngb=n_ngb, dn=dn,
                    fixed_h=False, hydro=False, n_group_max=16, f=0.5,
                    meta={"seed": seed})


def lognormal_hydro(n=2097152, seed=3, active=0.25, n_ngb=295, dn=6, grid=256,
                    sigma=1.5, run_mean=256):
    """Lognormal field (sigma_lnrho = 1.5, P(k) ~ k^-2), Wendland C6,
    N_ngb = 295, u ~ U[0.5,2], v ~ N(0, 0.1^2), 25% active runs; density then
    hydro."""
    rng = _rng(seed)
    x, y, z = lognormal_positions(rng, n, grid=grid, sigma=sigma)
    h, nd = initial_h(rng, x, y, z, n_ngb)
    st = _state(x, y, z, h, nd, n, rng=rng, hydro=True)
    st["active"] = active_cells(rng, x, y, z, active, run_mean)
    off, L = _one_box(n)
    return Workload("lognormal_hydro", st, off, L, kernel=1, n_ngb=n_ngb, dn=dn,
                    fixed_h=False, hydro=True, n_group_max=32, f=0.5,
                    meta={"seed": seed, "grid": grid, "sigma": sigma})


def plummer_batch(n_boxes=64, seed0=1000, n_range=(1e4, 5e5), n_ngb=64, dn=2,
                  run_mean=64):
    """Independent periodic unit boxes with log-uniform particle counts,
    config-2 Plummer recipe per box, active fraction U[0.01, 1] per box."""
    parts = []
    sizes = []
    for b in range(n_boxes):
        rng = _rng(seed0 + b)
        nb = int(round(math.exp(rng.uniform(math.log(n_range[0]), math.log(n_range[1])))))
        x, y, z = plummer_mixture(rng, nb)
        h, nd = initial_h(rng, x, y, z, n_ngb)
        _say(f"box {b + 1}/{n_boxes}: {nb} particles")
        st = _state(x, y, z, h, nd, nb)
        frac = rng.uniform(0.01, 1.0)
        st["active"] = active_cells(rng, x, y, z, frac, run_mean)
        parts.append(st)
        sizes.append(nb)
    off = np.zeros(n_boxes + 1, np.int64)
    np.cumsum(sizes, out=off[1:])
    st = {k: np.concatenate([p[k] for p in parts]) for k in parts[0]}
    st["orig"] = np.arange(int(off[-1]), dtype=np.uint32)
    return Workload("plummer_batch", st, off, np.ones(n_boxes), kernel=0, n_ngb=n_ngb,
                    dn=dn, fixed_h=False, hydro=False, n_group_max=16, f=0.5,
                    meta={"seed0": seed0, "sizes": sizes})


def lognormal_bins(n=16777216, seed=5, grid=256, sigma=1.82, n_ngb=295, dn=6,
                   run_mean=256):
    """Large lognormal box with three nested timestep bins (100%, 10%, 1%
    active); `state['bin']` holds the deepest bin of each particle.  sigma
    = 1.82 puts the 0.1 - 99.9 percentile ratio of the SPH density near 1e4
    (the oracle's converged density on 20 000 random particles: 1.4e3 at
    sigma 1.5, 8.5e3 at 1.8, 3.9e4 at 2.0).  The initial h comes from a 1/8
    subsample (initial_h(thin=8))."""
    rng = _rng(seed)
    x, y, z = lognormal_positions(rng, n, grid=grid, sigma=sigma)
    h, nd = initial_h(rng, x, y, z, n_ngb, thin=8 if n > (1 << 22) else 1)
    st = _state(x, y, z, h, nd, n, rng=rng, hydro=True)
    b1 = active_cells(rng, x, y, z, 0.10, run_mean)
    b2 = active_cells(rng, x, y, z, 0.01, run_mean, within=b1)
    st["bin"] = (b1.astype(np.uint8) + b2.astype(np.uint8))
    st["active"] = np.ones(n, np.uint8)
    off, L = _one_box(n)
    return Workload("lognormal_bins", st, off, L, kernel=1, n_ngb=n_ngb, dn=dn,
                    fixed_h=False, hydro=True, n_group_max=32, f=0.5,
                    meta={"seed": seed, "grid": grid, "sigma": sigma})


WORKLOADS = {
    "uniform_fixed_h": uniform_fixed_h,
    "plummer_clustered": plummer_clustered,
    "lognormal_hydro": lognormal_hydro,
    "plummer_batch": plummer_batch,
    "lognormal_bins": lognormal_bins,
}
