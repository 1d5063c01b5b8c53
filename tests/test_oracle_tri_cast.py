"""Pins of the oracle's per-triangle ray casting (Sec. III: rays are cast
towards every mesh triangle) against closed forms.  With a reception sphere
that takes every specular return, the summed path amplitude of a launch is p0
times the solid angle its counted rays cover (p0 = 1 / field-of-view solid
angle), so:
  * one triangle: p0 times the Van Oosterom-Strackee solid angle (pins the
    area-uniform point map, the A |cos| / d^2 weight and its factor 1/2);
  * a small triangle in front of a large one: p0 times the large one's solid
    angle, and no counted ray of the large one crosses the small one's
    silhouette (pins the first-hit rule: nothing counted twice);
  * the specular plate of the uniform-launch pin: p0 times the solid angle of
    the returning disc, 2 pi (1 - cos theta_max);
plus: every counted ray's first hit is its own triangle, weights scale as
1/g^2, rays outside the field of view are not traced, invalid grids raise."""
import math

import numpy as np
import pytest

import oracle
import scenegen as sg


def _scene(tris_xyz, alpha=0.0):
    v = np.asarray(tris_xyz, dtype=np.float32).reshape(-1, 3)
    n = v.shape[0] // 3
    return sg.Scene(v, np.arange(3 * n, dtype=np.int32).reshape(n, 3), np.zeros(n, np.int32),
                    np.array([alpha], np.float32), np.zeros((1, 3))).checked()


def _solid_angle(tri, o):
    a, b, c = (np.asarray(p, np.float64) - o for p in tri)
    la, lb, lc = (np.linalg.norm(x) for x in (a, b, c))
    num = abs(np.dot(a, np.cross(b, c)))
    den = la * lb * lc + np.dot(a, b) * lc + np.dot(a, c) * lb + np.dot(b, c) * la
    return 2.0 * math.atan2(num, den)


def _mono(r=1e3):
    o = np.zeros((1, 3))
    return sg.Array(o, o.copy(), r, sg.MODE_PER_TX)


def _tp(g, b=1, seed=1, **fov):
    return sg.TraceParams(n_rays=0, max_bounces=b, seed=seed, rays_per_tri=g * g, **fov)


def test_single_triangle_solid_angle():
    tri = [[5.0, -0.3, 0.2], [5.4, 0.9, -0.1], [4.8, 0.1, 1.1]]
    sc = _scene(tri)
    tri32 = sc.verts.astype(np.float64)
    omega_fov = math.pi * 2.0                      # the default hemisphere
    want = _solid_angle(tri32, np.zeros(3)) / omega_fov
    for g in (16, 64):
        hits, paths = oracle.trace(sc, _mono(), _tp(g))
        assert len(paths) == g * g                 # every ray is counted and returns
        assert (hits[:, 0] == 0).all()
        got = paths["amp"].sum()
        assert abs(got / want - 1) < (2e-3 if g == 16 else 2e-4), (g, got, want)
    # g = 1: a single ray, weight p0 A |cos| / d^2
    _, p1 = oracle.trace(sc, _mono(), _tp(1))
    assert len(p1) == 1 and abs(p1["amp"][0] / want - 1) < 0.2


def test_occluded_rays_not_counted_twice():
    big = [[6.0, -1.0, -1.0], [6.0, 1.5, -0.8], [6.0, -0.2, 1.4]]
    small = [[4.0, -0.2, -0.1], [4.0, 0.3, -0.1], [4.0, 0.0, 0.3]]   # inside big's silhouette
    sc = _scene(small + big)
    tri32 = sc.verts.astype(np.float64).reshape(2, 3, 3)
    want = _solid_angle(tri32[1], np.zeros(3)) / (2 * math.pi)
    g = 64
    hits, paths = oracle.trace(sc, _mono(), _tp(g))
    ray_tri = np.arange(hits.shape[0]) // (g * g)
    counted = hits[:, 0] >= 0
    assert (hits[counted, 0] == ray_tri[counted]).all()
    assert counted[: g * g].all()                  # the front triangle is never occluded
    blocked = ~counted[g * g:]
    assert 0 < blocked.mean() < 1
    # the big triangle's dropped share = the small one's solid angle over the big one's
    frac = _solid_angle(tri32[0], np.zeros(3)) / _solid_angle(tri32[1], np.zeros(3))
    w = np.zeros(hits.shape[0])
    w[paths["ray"]] = paths["amp"]
    assert abs(paths["amp"].sum() / want - 1) < 1e-3
    assert abs(w[g * g:][blocked].size / (g * g) - frac) < 0.05


def test_specular_plate_disc():
    R, r = 5.0, 0.25
    sc = sg.plate(R, 1.0, alpha=0.0)
    o = np.array([[0.0, 0.0, 0.5]])
    ar = sg.Array(o, o.copy(), r, sg.MODE_PER_TX)
    st = r / (2 * R)
    want = 1.0 - math.sqrt(1 - st * st)            # p0 * 2 pi (1 - cos theta_max), p0 = 1 / 2 pi
    _, paths = oracle.trace(sc, ar, _tp(256))
    assert abs(paths["amp"].sum() / want - 1) < 0.01
    assert np.allclose(paths["p"][:, 0, 0], R, atol=1e-12)


def test_weights_scale_and_field_of_view():
    tri = [[5.0, -0.3, 0.2], [5.4, 0.9, -0.1], [4.8, 0.1, 1.1]]
    sc = _scene(tri)
    a = oracle.trace(sc, _mono(), _tp(8))[1]["amp"].sum()
    b = oracle.trace(sc, _mono(), _tp(32))[1]["amp"].sum()
    assert abs(a / b - 1) < 0.02
    # a field of view that excludes the triangle: nothing is traced
    hits, paths = oracle.trace(sc, _mono(), _tp(8, az_min=-1.0, az_max=-0.5))
    assert len(paths) == 0 and (hits == -1).all()
    # a field of view that cuts it: fewer rays, the rest at the same points
    # with weights scaled by p0 = 1 / (d_az (sin el_max - sin el_min))
    h2, p2 = oracle.trace(sc, _mono(), _tp(8, az_min=-0.2, az_max=0.05))
    h1, p1 = oracle.trace(sc, _mono(), _tp(8))
    kept = np.isin(p1["ray"], p2["ray"])
    assert 0 < len(p2) < len(p1)
    assert np.array_equal(p1["p"][kept], p2["p"])
    assert np.allclose(p1["amp"][kept] * 2 * math.pi, p2["amp"] * 0.25 * 2, rtol=1e-13, atol=0)
    # p0 follows the field of view: twice the solid angle, half the weight
    h3, p3 = oracle.trace(sc, _mono(), _tp(8, el_min=-math.pi / 2, el_max=math.pi / 2,
                                            az_min=-math.pi / 2, az_max=math.pi / 2))
    assert np.array_equal(p3["amp"], p1["amp"])


def test_invalid_grids():
    sc = _scene([[5.0, 0, 0], [5.0, 1, 0], [5.0, 0, 1]])
    with pytest.raises(ValueError):
        oracle.trace(sc, _mono(), sg.TraceParams(n_rays=0, max_bounces=1, rays_per_tri=5))
    with pytest.raises(RuntimeError):
        oracle.trace(sc, _mono(), sg.TraceParams(n_rays=0, max_bounces=1, rays_per_tri=4,
                                                 az_min=-2.0, az_max=2.0))


# ---------------------------------------------------------------- subdivision
def _area(t):
    return 0.5 * np.linalg.norm(np.cross(t[1] - t[0], t[2] - t[0]))


def test_pieces_without_subdivision_are_the_triangles():
    sc = sg.scene_street(3, scale=0.05, n_cars=2, n_poles=2)
    v, par = oracle.pieces(sc, _mono(), 0.0, 8)
    assert np.array_equal(par, np.arange(sc.n_tris))
    assert np.array_equal(v, sc.verts.astype(np.float64)[sc.tris])


def test_one_level_midpoint_children():
    tri = np.array([[5.0, -0.3, 0.2], [5.4, 0.9, -0.1], [4.8, 0.1, 1.1]], np.float32)
    sc = _scene(tri)
    v, par = oracle.pieces(sc, _mono(), 1e-9, 1)
    a, b, c = tri.astype(np.float64)
    ab, bc, ca = (a + b) / 2, (b + c) / 2, (c + a) / 2
    want = np.array([[a, ab, ca], [ab, b, bc], [ca, bc, c], [ab, bc, ca]])
    assert np.array_equal(v, want) and (par == 0).all()


def test_pieces_tile_their_triangle():
    """Children cover the parent exactly once: areas and solid angles add up,
    every leaf is below the threshold unless at the depth limit, and every
    piece lies inside its parent."""
    sc = sg.plate(3.0, 1.0, alpha=0.0)
    o = np.array([[0.0, 0.0, 0.5]])
    ar = sg.Array(o, o.copy(), 0.25, sg.MODE_PER_TX)
    for om, dm in ((2e-2, 12), (1e-3, 3)):
        v, par = oracle.pieces(sc, ar, om, dm)
        tris = sc.verts.astype(np.float64)[sc.tris]
        assert len(v) > sc.n_tris and np.array_equal(np.unique(par), np.arange(sc.n_tris))
        assert np.all(np.diff(par) >= 0)           # upload order, depth first
        for f in range(sc.n_tris):
            kids = v[par == f]
            assert abs(sum(_area(k) for k in kids) / _area(tris[f]) - 1) < 1e-12
            om_kids = [_solid_angle(k, o[0]) for k in kids]
            assert abs(sum(om_kids) / _solid_angle(tris[f], o[0]) - 1) < 1e-10
            depth = np.round(np.log(_area(tris[f]) / np.array([_area(k) for k in kids])) /
                             np.log(4)).astype(int)
            assert ((np.array(om_kids) <= om) | (depth == dm)).all()
            # barycentric coordinates of each piece vertex in the parent
            e1, e2 = tris[f][1] - tris[f][0], tris[f][2] - tris[f][0]
            G = np.array([[e1 @ e1, e1 @ e2], [e1 @ e2, e2 @ e2]])
            rhs = np.stack([(kids - tris[f][0]) @ e1, (kids - tris[f][0]) @ e2], -1)
            uv = np.linalg.solve(G, rhs.reshape(-1, 2).T).T
            assert (uv > -1e-12).all() and (uv.sum(1) < 1 + 1e-12).all()
    with pytest.raises(RuntimeError):
        oracle.trace(sc, ar, sg.TraceParams(n_rays=0, max_bounces=1, rays_per_tri=1,
                                            tri_omega_max=1e-3, tri_depth_max=21))


def test_subdivided_launch_keeps_the_estimate():
    """Cutting the triangles leaves the estimate unbiased and sharpens it: the
    single triangle's and the specular disc's closed forms hold, with fewer
    rays per piece."""
    tri = [[5.0, -0.3, 0.2], [5.4, 0.9, -0.1], [4.8, 0.1, 1.1]]
    sc = _scene(tri)
    want = _solid_angle(sc.verts.astype(np.float64), np.zeros(3)) / (2 * math.pi)
    tp = sg.TraceParams(n_rays=0, max_bounces=1, seed=1, rays_per_tri=16, tri_omega_max=2e-3,
                        tri_depth_max=8)
    hits, paths = oracle.trace(sc, _mono(), tp)
    n_p = len(oracle.pieces(sc, _mono(), 2e-3, 8)[1])
    assert n_p == 16 and hits.shape[0] == 16 * n_p and (hits[:, 0] == 0).all()
    assert abs(paths["amp"].sum() / want - 1) < 2e-4
    # the disc: the near plate is cut where it fills the view
    R, r = 5.0, 0.25
    pl = sg.plate(R, 1.0, alpha=0.0)
    o = np.array([[0.0, 0.0, 0.5]])
    ar = sg.Array(o, o.copy(), r, sg.MODE_PER_TX)
    st = r / (2 * R)
    want = 1.0 - math.sqrt(1 - st * st)
    tp = sg.TraceParams(n_rays=0, max_bounces=1, seed=1, rays_per_tri=64, tri_omega_max=1e-3,
                        tri_depth_max=10)
    _, paths = oracle.trace(pl, ar, tp)
    assert abs(paths["amp"].sum() / want - 1) < 0.01
    assert np.allclose(paths["p"][:, 0, 0], R, atol=1e-12)


# ------------------------------------------------------------ field of view
def test_pieces_outside_the_view_are_dropped():
    """Triangles behind the array, or beyond an azimuth or elevation bound,
    take no ray indices; the launch's sum of weights is unchanged (p0 times
    the solid angle of what is in view); a triangle that straddles a bound
    is kept, and so is one that only another source of a per-element launch
    sees."""
    front = [[6.0, -1.0, -1.0], [6.0, 1.5, -0.8], [6.0, -0.2, 1.4]]
    behind = [[-5.0, -1.0, -1.0], [-5.0, 1.0, -1.0], [-5.0, 0.0, 1.0]]
    straddle = [[-0.5, 3.0, 0.0], [2.0, 3.0, 0.0], [1.0, 3.0, 1.0]]
    sc = _scene(front + behind + straddle)
    tris = sc.verts.astype(np.float64).reshape(3, 3, 3)
    fov = (-math.pi / 2, math.pi / 2, -math.pi / 2, math.pi / 2)
    v, par = oracle.pieces(sc, _mono(), 0.0, 8, fov)
    assert par.tolist() == [0, 2]
    assert len(oracle.pieces(sc, _mono(), 0.0, 8)[1]) == 3      # no culling asked
    hits, paths = oracle.trace(sc, _mono(), _tp(32, b=1))
    assert hits.shape[0] == 2 * 32 * 32
    # the straddling triangle's rays behind the array are not traced; the
    # front one returns its full solid angle (specular, normal incidence)
    front_amp = paths["amp"][paths["ray"] < 32 * 32].sum()
    assert abs(front_amp / (_solid_angle(tris[0], np.zeros(3)) / (2 * math.pi)) - 1) < 1e-3
    # elevation: a floor far below a +-10 degree band is dropped, and so is a
    # triangle beyond the azimuth bound of a narrow wedge
    deg = math.pi / 180
    floor = [[3.0, -1.0, -4.0], [6.0, 1.0, -4.0], [6.0, -1.0, -4.0]]
    side = [[3.0, 4.0, 0.0], [3.0, 5.0, 0.2], [4.0, 4.5, -0.2]]
    sc2 = _scene(front + floor + side)
    band = (-30 * deg, 30 * deg, -10 * deg, 10 * deg)
    assert oracle.pieces(sc2, _mono(), 0.0, 8, band)[1].tolist() == [0]
    # el_min > 0: the region below it is not convex, so the floor is kept
    # (conservative); the side triangle is still beyond the azimuth bound
    up = (-30 * deg, 30 * deg, 20 * deg, 60 * deg)
    assert oracle.pieces(sc2, _mono(), 0.0, 8, up)[1].tolist() == [0, 1]
    # per-element sources: seen at positive azimuth only from the Tx at y = -1
    tri = [[5.0, -0.6, -0.1], [5.0, -0.4, -0.1], [5.0, -0.5, 0.2]]
    sc3 = _scene(tri)
    tx = np.array([[0.0, 1.0, 0.0], [0.0, -1.0, 0.0]])
    right = (0.0, math.pi / 2, -math.pi / 2, math.pi / 2)
    per_el = sg.Array(tx, np.zeros((1, 3)), 1e3, sg.MODE_PER_TX)
    shared = sg.Array(tx, np.zeros((1, 3)), 1e3, sg.MODE_SHARED)
    assert oracle.pieces(sc3, per_el, 0.0, 8, right)[1].tolist() == [0]
    assert oracle.pieces(sc3, shared, 0.0, 8, right)[1].tolist() == []
