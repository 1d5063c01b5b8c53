"""Pins of the oracle's building blocks against things other than itself:
numpy's Philox4x64-10, 80-bit long-double trigonometry, geometry with a
known answer, brute force versus the oracle's BVH, and the invariants of the
paper's material model (Eqs. 1-3)."""
import math

import numpy as np
import pytest

import scenegen as sg


# ---------------------------------------------------------------- RNG (Philox)

def _numpy_philox(ctr, key):
    """numpy's Philox increments the 256-bit counter before each block."""
    v = sum(int(c) << (64 * i) for i, c in enumerate(ctr))
    v = (v - 1) % (1 << 256)
    cm = np.array([(v >> (64 * i)) & (2**64 - 1) for i in range(4)], dtype=np.uint64)
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=cm)
    return bg.random_raw(4)


def test_philox_matches_numpy(orc):
    rng = np.random.default_rng(123)
    cases = [((0, 0, 0, 0), (0, 0)), ((2**64 - 1,) * 4, (2**64 - 1,) * 2)]
    for _ in range(300):
        cases.append((tuple(int(x) for x in rng.integers(0, 2**63, 4)),
                      tuple(int(x) for x in rng.integers(0, 2**63, 2))))
    for ctr, key in cases:
        assert (orc.philox4x64(ctr, key) == _numpy_philox(ctr, key)).all(), (ctr, key)


def test_uniforms_chi2(orc):
    """53-bit uniforms from consecutive counters: chi^2 over 64 bins."""
    n = 20000
    u = np.array([(int(orc.philox4x64((i, 3, 1, 0), (7, 0))[0]) >> 11) * 2.0**-53
                  for i in range(n)])
    assert u.min() >= 0 and u.max() < 1
    h = np.bincount((u * 64).astype(int), minlength=64)
    chi2 = ((h - n / 64) ** 2 / (n / 64)).sum()
    assert chi2 < 120          # 63 dof: p ~ 1e-5


# ----------------------------------------------------------- trigonometry

def test_sincos_turn_vs_long_double(orc):
    rng = np.random.default_rng(5)
    us = np.concatenate([rng.uniform(-1, 1, 4000), np.linspace(-1, 1, 1025),
                         [0.0, 0.125, -0.125, 0.25, 0.5, 0.75, 1 - 2**-53]])
    two_pi = np.longdouble("6.28318530717958647692528676655900577")
    for u in us:
        s, c = orc.sincos_turn(u)
        a = two_pi * np.longdouble(u)
        assert abs(s - float(np.sin(a))) < 4.5e-16, u
        assert abs(c - float(np.cos(a))) < 4.5e-16, u
    assert orc.sincos_turn(0.0) == (0.0, 1.0)
    s, c = orc.sincos_turn(0.25)
    assert s == 1.0 and c == 0.0


# ------------------------------------------------------------- intersection

def _one_tri(v):
    v = np.asarray(v, dtype=np.float32).reshape(3, 3)
    return sg.Scene(v, np.array([[0, 1, 2]], np.int32), np.zeros(1, np.int32),
                    np.zeros(1, np.float32), np.zeros((1, 3))).checked()


def test_closest_hit_known_answers(orc):
    sc = _one_tri([[5, -1, -1], [5, 2, -1], [5, -1, 2]])
    h, t = orc.closest(sc, [0, 0, 0], [1, 0, 0])
    assert h == 0 and t == 5.0
    # the ray through a vertex and along an edge counts (closed triangle)
    h, t = orc.closest(sc, [0, -1, -1], [1, 0, 0])
    assert h == 0 and t == 5.0
    h, t = orc.closest(sc, [0, 0.5, 0.5], [1, 0, 0])       # u + v == 1 edge
    assert h == 0
    h, _ = orc.closest(sc, [0, 0.51, 0.5], [1, 0, 0])      # just outside
    assert h == -1
    h, _ = orc.closest(sc, [0, 0, 0], [-1, 0, 0])          # behind
    assert h == -1
    h, _ = orc.closest(sc, [0, 0, 0], [0, 1, 0])           # parallel
    assert h == -1
    h, _ = orc.closest(sc, [0, 0, 0], [1, 0, 0], skip=0)   # excluded
    assert h == -1
    h, _ = orc.closest(sc, [5 - 5e-7, 0, 0], [1, 0, 0])    # t below t_min
    assert h == -1
    # oblique ray: t from the plane equation
    d = np.array([1.0, 0.1, -0.05]); d /= np.linalg.norm(d)
    h, t = orc.closest(sc, [0, 0, 0], d)
    assert h == 0 and abs(t - 5.0 / d[0]) < 1e-13


def test_tie_lowest_id(orc):
    """Two copies of one triangle: the lower id wins; a nearer third wins."""
    v = np.array([[5, -1, -1], [5, 2, -1], [5, -1, 2]], np.float32)
    verts = np.concatenate([v, v, v - [1, 0, 0]])
    sc = sg.Scene(verts, np.arange(9, dtype=np.int32).reshape(3, 3), np.zeros(3, np.int32),
                  np.zeros(1, np.float32), np.zeros((1, 3))).checked()
    h, t = orc.closest(sc, [0, 0, 0], [1, 0, 0])
    assert h == 2 and t == 4.0
    sc2 = sg.Scene(verts[:6], np.arange(6, dtype=np.int32).reshape(2, 3), np.zeros(2, np.int32),
                   np.zeros(1, np.float32), np.zeros((1, 3))).checked()
    for bvh in (False, True):
        h, t = orc.closest(sc2, [0, 0, 0], [1, 0, 0], use_bvh=bvh)
        assert h == 0 and t == 5.0


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_bvh_equals_brute_force_soup(orc, seed):
    sc = sg.random_soup(600, seed)
    rng = np.random.default_rng(100 + seed)
    for _ in range(400):
        o = rng.uniform(0.5, 2.5, 3)
        d = rng.normal(size=3); d /= np.linalg.norm(d)
        skip = int(rng.integers(-1, 600))
        hb, tb = orc.closest(sc, o, d, skip, use_bvh=False)
        hv, tv = orc.closest(sc, o, d, skip, use_bvh=True)
        assert hb == hv and (tb == tv or (hb == -1 and math.isinf(tb) and math.isinf(tv)))


def test_bvh_equals_brute_force_trace(orc):
    """Whole-trace check on the tiny scene: hit lists and paths identical."""
    w = sg.workload_tiny()
    w.trace.n_rays = 5000
    h1, p1 = orc.trace(w.scene, w.array, w.trace, use_bvh=False)
    h2, p2 = orc.trace(w.scene, w.array, w.trace, use_bvh=True)
    assert (h1 == h2).all()
    assert p1.tobytes() == p2.tobytes()


# --------------------------------------------------------- material model

def _unit(x):
    x = np.asarray(x, dtype=np.float64)
    return x / np.linalg.norm(x)


def test_eq2_mirror_invariants(orc):
    """alpha = 0 is the law of reflection: unit length, m.n = -d.n, m in
    span(d, n), and reflecting the reflection gives d back."""
    rng = np.random.default_rng(9)
    for _ in range(500):
        n = _unit(rng.normal(size=3))
        d = _unit(rng.normal(size=3))
        if d @ n > 0:
            n = -n
        m = orc.bounce(d, n, 0.0, rng.random(), rng.random())
        assert abs(np.linalg.norm(m) - 1) < 1e-14
        assert abs(m @ n + d @ n) < 1e-14
        assert abs(np.linalg.det(np.stack([m, d, n]))) < 1e-14
        back = orc.bounce(m, -n, 0.0, 0.3, 0.7)
        assert np.allclose(back, d, atol=1e-14)


def test_eq1_lambert_density(orc):
    """alpha = 1 gives n + r with r uniform on the sphere: cos(theta) to the
    normal has density 2 cos(theta) on [0, 1], i.e. cos^2 is uniform; the
    azimuth about n is uniform."""
    rng = np.random.default_rng(4)
    n = _unit([0.3, -0.2, 0.9])
    d = _unit([0.1, 0.4, -1.0])
    cs = []
    for _ in range(20000):
        t = orc.bounce(d, n, 1.0, rng.random(), rng.random())
        assert abs(np.linalg.norm(t) - 1) < 1e-14
        cs.append(t @ n)
    c2 = np.sort(np.array(cs) ** 2)
    ks = np.max(np.abs(c2 - (np.arange(1, c2.size + 1) / c2.size)))
    assert ks < 1.63 / math.sqrt(c2.size) * 1.3
    assert min(cs) >= -1e-12


def test_eq3_blend(orc):
    """0 < alpha < 1: the result is the normalised blend of the alpha = 1 and
    alpha = 0 directions for the same random draw."""
    rng = np.random.default_rng(11)
    for _ in range(300):
        n = _unit(rng.normal(size=3))
        d = _unit(rng.normal(size=3))
        if d @ n > 0:
            n = -n
        u0, u1, a = rng.random(), rng.random(), rng.random()
        td = orc.bounce(d, n, 1.0, u0, u1)
        tm = orc.bounce(d, n, 0.0, u0, u1)
        tc = orc.bounce(d, n, a, u0, u1)
        ref = _unit(a * td + (1 - a) * tm)
        assert np.allclose(tc, ref, atol=1e-14)
