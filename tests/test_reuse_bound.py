"""The bound under which a kept group superset still holds every neighbour
of a member after the particles moved (the Verlet-skin reading of superset
reuse), checked by brute force on random periodic configurations.

At the walk: centre c (first member), R_g = largest member distance to c,
H = largest member h.  Density superset: every j with |x_j - c| <= R_g +
skin H.  Hydro superset: every j with |x_j - c| <= R_s + max(H, h_j),
R_s = R_g + (skin - 1) H.  Afterwards every particle moved by at most
delta and every h grew by at most dh.  A member passing

    density: h_i + |x_i - c| + delta <= R_g + skin H
    hydro:   h_i + |x_i - c| + delta <= R_s + H  and  |x_i - c| + delta + dh <= R_s

must find all its neighbours (density r < h_i, hydro r < max(h_i, h_j)) in
the kept superset.  Plain numpy, FP64, minimum image; no GPU."""
import numpy as np


def _dist(a, b, L=1.0):
    d = a - b
    d -= L * np.round(d / L)
    return np.sqrt((d * d).sum(-1))


def _trial(rng, skin, n=3000):
    x0 = rng.random((n, 3))
    h0 = rng.uniform(0.1, 0.2, n)
    # a group: the particles within f h_0 of a first member
    c_i = int(rng.integers(n))
    c = x0[c_i]
    mem = np.nonzero(_dist(x0, c) < 0.5 * h0[c_i])[0]
    R = _dist(x0[mem], c).max()
    H = h0[mem].max()
    cov_d = R + skin * H
    Rs = R + (skin - 1.0) * H
    dj = _dist(x0, c)
    keep_d = dj <= cov_d
    keep_h = (dj <= Rs + H) | (dj <= Rs + h0)
    # a drift of at most delta and an h change of at most +dh (some shrink)
    delta = rng.uniform(0.0, 0.03)
    v = rng.normal(size=(n, 3))
    v *= (delta * rng.random(n) / np.linalg.norm(v, axis=1))[:, None]
    x1 = np.mod(x0 + v, 1.0)
    dh = rng.uniform(0.0, 0.02)
    h1 = h0 * rng.uniform(0.9, 1.0, n) + dh * rng.random(n)
    h1 = np.minimum(h1, h0 + dh)
    checked = [0, 0]
    for i in mem:
        di = _dist(x1[i], c)
        r = _dist(x1, x1[i])
        if h1[i] + di + delta <= cov_d:
            checked[0] += 1
            nb = np.nonzero(r < h1[i])[0]
            assert keep_d[nb].all(), ("density", i)
        if h1[i] + di + delta <= Rs + H and di + delta + dh <= Rs:
            checked[1] += 1
            nb = np.nonzero((r < np.maximum(h1[i], h1)) & (np.arange(n) != i))[0]
            assert keep_h[nb].all(), ("hydro", i)
    return checked


def test_reuse_bound_keeps_every_neighbour():
    rng = np.random.default_rng(20)
    total = np.zeros(2, int)
    for t in range(150):
        total += _trial(rng, skin=(1.0, 1.1, 1.25)[t % 3])
    # the bound is not vacuous: many members pass it
    assert total[0] > 300 and total[1] > 100, total


def test_a_looser_bound_would_lose_neighbours():
    """Dropping the displacement term from the density bound (the mistake it
    guards against) admits members with a neighbour outside the superset."""
    rng = np.random.default_rng(21)
    lost = 0
    for _ in range(100):
        n = 3000
        x0 = rng.random((n, 3))
        h0 = rng.uniform(0.1, 0.2, n)
        c = x0[0]
        mem = np.nonzero(_dist(x0, c) < 0.5 * h0[0])[0]
        R = _dist(x0[mem], c).max()
        H = h0[mem].max()
        keep = _dist(x0, c) <= R + H
        v = rng.normal(size=(n, 3))
        v *= (0.03 / np.linalg.norm(v, axis=1))[:, None]
        x1 = np.mod(x0 + v, 1.0)
        for i in mem:
            if h0[i] + _dist(x1[i], c) <= R + H:  # no delta term
                nb = np.nonzero(_dist(x1, x1[i]) < h0[i])[0]
                lost += int((~keep[nb]).sum())
    assert lost > 0


def test_hydro_bound_needs_the_h_growth():
    """Dropping dh from the second hydro condition admits members that miss
    a neighbour j whose own h grew (a pair through h_j)."""
    rng = np.random.default_rng(22)
    lost = 0
    for _ in range(100):
        n = 3000
        x0 = rng.random((n, 3))
        h0 = rng.uniform(0.1, 0.2, n)
        c = x0[0]
        mem = np.nonzero(_dist(x0, c) < 0.5 * h0[0])[0]
        R = _dist(x0[mem], c).max()
        H = h0[mem].max()
        Rs = R + 0.1 * H
        dj = _dist(x0, c)
        keep = (dj <= Rs + H) | (dj <= Rs + h0)
        h1 = h0 + 0.05 * rng.random(n)  # no motion, h grows by up to 0.05
        for i in mem:
            di = _dist(x0[i], c)
            if h1[i] + di <= Rs + H and di <= Rs:  # dh term dropped
                r = _dist(x0, x0[i])
                nb = np.nonzero((r < np.maximum(h1[i], h1)) & (np.arange(n) != i))[0]
                lost += int((~keep[nb]).sum())
    assert lost > 0
