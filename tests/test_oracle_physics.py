"""Pins of the oracle's trace and synthesis against closed forms, invariants
and special cases: FMCW beat frequency 2RB/c and Doppler 2v/lambda of a point
reflector, array steering phases, specular-plate return, reciprocity, empty
scene, translation invariance, linearity, range reduction, separable = exact
for a single channel, and unbiasedness of importance-sampled launch."""
import math

import numpy as np
import pytest

import scenegen as sg

C0 = sg.C0


def _array(tx, rx, mode=sg.MODE_PER_TX, radius=0.25):
    return sg.Array(np.array(tx, float).reshape(-1, 3), np.array(rx, float).reshape(-1, 3),
                    radius, mode).checked()


def _tp(n, bounces=2, seed=0):
    return sg.TraceParams(n_rays=n, max_bounces=bounces, seed=seed)


# ------------------------------------------------------------------ launch

def test_launch_uniform_over_hemisphere(orc):
    """Uniform in solid angle over x > 0: the x component is uniform on [0, 1]
    (Archimedes) and the azimuth about +x is uniform."""
    sc = sg.point_only([[5.0, 0, 0.5]])
    ar = _array([0, 0, 0.5], [0, 0, 0.5])
    tp = _tp(1000)
    ds = np.array([orc.launch_dir(sc, ar, tp, i, 0)[:3] for i in range(20000)])
    assert np.allclose(np.linalg.norm(ds, axis=1), 1, atol=1e-15)
    x = np.sort(ds[:, 0])
    assert x.min() >= 0
    ks = np.max(np.abs(x - np.arange(1, x.size + 1) / x.size))
    assert ks < 1.63 / math.sqrt(x.size) * 1.3
    phi = np.sort((np.arctan2(ds[:, 2], ds[:, 1]) + np.pi) / (2 * np.pi))
    ks = np.max(np.abs(phi - np.arange(1, phi.size + 1) / phi.size))
    assert ks < 1.63 / math.sqrt(phi.size) * 1.3


# ------------------------------------------------------- specular plate

def test_specular_plate_monostatic(orc):
    """alpha = 0 plate normal to +x at distance R, Tx = Rx.  A ray at angle
    theta to the normal returns along the image line and passes the radar at
    distance 2R sin(theta), so it is received iff sin(theta) <= r/(2R); every
    received path has one hit inside the disc of radius R tan(theta_max) and
    length 2R/cos(theta).  The count is Binomial(N, 1 - cos(theta_max))."""
    R, r = 5.0, 0.25
    sc = sg.plate(R, 1.0, alpha=0.0)
    o = [0.0, 0.0, 0.5]
    ar = _array(o, o, radius=r)
    N = 1_000_000
    _, paths = orc.trace(sc, ar, _tp(N))
    st = r / (2 * R)
    ct = math.sqrt(1 - st * st)
    p = 1 - ct
    assert abs(len(paths) - N * p) < 4.5 * math.sqrt(N * p * (1 - p))
    assert (paths["K"] == 1).all() and set(paths["tri"][:, 0]) <= {0, 1}
    hit = paths["p"][:, 0, :]
    assert np.allclose(hit[:, 0], R, atol=1e-12)
    rad = np.hypot(hit[:, 1], hit[:, 2] - 0.5)
    assert rad.max() <= R * st / ct + 1e-9
    d = 2 * np.linalg.norm(hit - np.array(o), axis=1)
    assert d.min() >= 2 * R - 1e-12 and d.max() <= 2 * R / ct + 1e-12
    assert np.allclose(paths["amp"], 1.0 / N)


def test_specular_plate_bistatic_and_reciprocity(orc):
    """Bistatic: path lengths are bounded below by |tx - mirror(rx)| and come
    close to it; swapping Tx and Rx gives the same bound (reciprocity)."""
    R = 5.0
    sc = sg.plate(R, 2.0, alpha=0.0)
    a, b = [0.0, -0.1, 0.5], [0.0, 0.1, 0.5]
    for tx, rx in ((a, b), (b, a)):
        ar = _array(tx, rx, radius=0.2)
        _, paths = orc.trace(sc, ar, _tp(400_000))
        hit = paths["p"][:, 0, :]
        d = np.linalg.norm(hit - tx, axis=1) + np.linalg.norm(hit - rx, axis=1)
        mirror = np.array([2 * R - rx[0], rx[1], rx[2]])
        dmin = np.linalg.norm(mirror - tx)
        assert d.min() >= dmin - 1e-12
        assert d.min() - dmin < 2e-3


# ------------------------------------------------------- point reflectors

def test_empty_scene_points_only(orc):
    """No triangles: no traced paths; every point gives one K = 1 path with
    amplitude A / (|q - tx|^2 Omega_FOV)."""
    pts = [[10.0, 1.0, 0.5], [20.0, -3.0, 1.0]]
    sc = sg.point_only(pts, aperture=[0.01, 0.02])
    ar = _array([[0, -0.01, 0.5], [0, 0.01, 0.5]], [0, 0, 0.5])
    _, paths = orc.trace(sc, ar, _tp(1000))
    assert len(paths) == 4
    assert (paths["K"] == 1).all() and (paths["tri"][:, 0] == -1).all()
    omega = math.pi * 2.0
    for p in paths:
        q = np.array(pts[p["vid"][0] - sc.n_obj])
        tx = ar.tx[p["src"]]
        ap = [0.01, 0.02][p["vid"][0] - sc.n_obj]
        assert abs(p["amp"] - ap / (np.sum((q - tx) ** 2) * omega)) < 1e-18


def test_point_shadowed(orc):
    """A plate between radar and point blocks the point path."""
    sc = sg.plate(5.0, 1.0)
    sc.pt_pos = np.array([[10.0, 0.0, 0.5]])
    sc.pt_vel = np.zeros((1, 3))
    sc.pt_aperture = np.array([0.01])
    ar = _array([0, 0, 0.5], [0, 0, 0.5])
    tp = _tp(10)
    _, paths = orc.trace(sc, ar, tp)
    assert not (paths["tri"][:, 0] == -1).any()


def _point_cube(orc, R, v, chirp, tx=(0, 0, 0.5), rx=(0, 0, 0.5)):
    sc = sg.point_only([[R, 0, 0.5]], vel=[[v, 0, 0]], aperture=0.01)
    ar = _array(tx, rx)
    _, paths = orc.trace(sc, ar, _tp(10))
    assert len(paths) == 1
    return paths, sc, ar, orc.synth(paths, sc, ar, chirp)


def test_monostatic_point_closed_form(orc):
    """Tx = Rx, point at range R with radial speed v: d(m) = 2 (R + v m T_rep)
    and the cube is sigma exp(-j 2 pi f_k d(m) / c) exactly."""
    ch = sg.Chirp(n_samples=64, n_chirps=16)
    R, v = 12.3, 3.7
    paths, _, _, cube = _point_cube(orc, R, v, ch)
    sigma = paths["amp"][0]
    m = np.arange(16)[:, None]
    k = np.arange(64)[None, :]
    fk = ch.f0 + ch.bandwidth * k / 64
    ref = sigma * np.exp(-2j * np.pi * fk * 2 * (R + v * m * ch.t_rep) / C0)
    assert np.abs(cube[0] - ref).max() < 1e-9 * sigma


def test_beat_and_doppler_peaks(orc):
    """2-D FFT peak of a moving point: beat frequency 2 R S / c and Doppler
    2 v / lambda (negative frequencies under exp(-j...)), at the bins
    2 R B / c and 2 v f0 T_rep M / c."""
    ch = sg.Chirp(n_samples=64, n_chirps=16)
    rbin, dbin = 9, 2
    R = rbin * C0 / (2 * ch.bandwidth)
    v = dbin * C0 / (2 * ch.f0 * ch.t_rep * ch.n_chirps)
    _, _, _, cube = _point_cube(orc, R, v, ch)
    spec = np.abs(np.fft.fft2(cube[0]))
    mi, ki = np.unravel_index(np.argmax(spec), spec.shape)
    assert ki == (-rbin) % 64 and mi == (-dbin) % 16
    # beat frequency in Hz from the slope S = B / T_c
    S = ch.bandwidth / ch.t_chirp
    fb = 2 * R * S / C0
    assert abs(fb * ch.t_chirp - rbin) < 1e-9


def test_array_steering_phase(orc):
    """Far point at azimuth theta seen by a half-wavelength Rx ULA: the phase
    step between neighbouring channels at k = 0 is pi sin(theta)."""
    lam = sg.LAMBDA77
    th = math.radians(20.0)
    Rr = 2000.0
    q = [Rr * math.cos(th), Rr * math.sin(th), 0.5]
    sc = sg.point_only([q])
    rx = [[0, (r - 3.5) * lam / 2, 0.5] for r in range(8)]
    ar = _array([0, 0, 0.5], rx)
    ch = sg.Chirp(n_samples=8, n_chirps=1)
    _, paths = orc.trace(sc, ar, _tp(10))
    cube = orc.synth(paths, sc, ar, ch)
    ph = np.angle(cube[1:, 0, 0] / cube[:-1, 0, 0])
    assert np.allclose(ph, math.pi * math.sin(th), atol=2e-5)


def test_reciprocity_point(orc):
    """Swapping Tx and Rx leaves every phase unchanged for a point path."""
    ch = sg.Chirp(n_samples=32, n_chirps=4)
    a, b = (0, -0.2, 0.5), (0, 0.3, 0.7)
    _, _, _, c1 = _point_cube(orc, 8.0, 1.5, ch, a, b)
    _, _, _, c2 = _point_cube(orc, 8.0, 1.5, ch, b, a)
    ratio = c1 / c2
    assert np.abs(np.angle(ratio)).max() < 1e-9
    assert np.ptp(np.abs(ratio)) < 1e-9 * np.abs(ratio).max()


def test_range_reduction_quarter_cycle(orc):
    """Path length with f0 d / c = N + 1/4: the k = 0 entry is -j a."""
    ch = sg.Chirp(n_samples=4, n_chirps=1)
    d = (123456 + 0.25) * C0 / ch.f0
    R = d / 2
    paths, _, _, cube = _point_cube(orc, R, 0.0, ch)
    a = paths["amp"][0]
    assert abs(cube[0, 0, 0] - (-1j * a)) < 1e-8 * a


# -------------------------------------------------------- model / algebra

def test_separable_equals_exact_single_channel(orc):
    w = sg.workload_tiny()
    w.trace.n_rays = 20000
    ar = _array(w.array.tx[:1], w.array.rx[:1])
    _, paths = orc.trace(w.scene, ar, w.trace)
    assert len(paths) > 10
    e = orc.synth(paths, w.scene, ar, w.chirp, model=0)
    s = orc.synth(paths, w.scene, ar, w.chirp, model=1)
    assert np.array_equal(e, s)


def test_separable_reduces_to_exact(orc):
    """The separable model differs from the exact one only through the
    bandwidth-aperture term (f_k - f0) (dT + dR) and the motion of the channel
    offsets.  With zero bandwidth and no motion between chirps the two models
    agree to rounding for every channel; with 1 GHz the gap is small."""
    w = sg.workload_tiny()
    w.trace.n_rays = 20000
    _, paths = orc.trace(w.scene, w.array, w.trace)
    ch = sg.Chirp(bandwidth=0.0, t_rep=0.0, n_samples=8, n_chirps=2)
    e = orc.synth(paths, w.scene, w.array, ch, model=0)
    s = orc.synth(paths, w.scene, w.array, ch, model=1)
    assert np.linalg.norm(e - s) / np.linalg.norm(e) < 1e-9
    e = orc.synth(paths, w.scene, w.array, w.chirp, model=0)
    s = orc.synth(paths, w.scene, w.array, w.chirp, model=1)
    gap = np.linalg.norm(e - s) / np.linalg.norm(e)
    assert 1e-6 < gap < 1e-2


def test_linearity(orc):
    w = sg.workload_tiny()
    w.trace.n_rays = 20000
    _, paths = orc.trace(w.scene, w.array, w.trace)
    h = len(paths) // 2
    full = orc.synth(paths, w.scene, w.array, w.chirp)
    parts = orc.synth(paths[:h], w.scene, w.array, w.chirp) + \
        orc.synth(paths[h:], w.scene, w.array, w.chirp)
    assert np.abs(full - parts).max() < 1e-12 * np.abs(full).max()


def test_translation_invariance(orc):
    """Shift scene, array and points by a float32-exact offset: same hit
    lists, and the cube agrees to rounding."""
    w = sg.workload_tiny()
    w.trace.n_rays = 20000
    h1, p1 = orc.trace(w.scene, w.array, w.trace)
    c1 = orc.synth(p1, w.scene, w.array, w.chirp)
    off = np.array([16.0, -8.0, 4.0])
    sc = sg.Scene((w.scene.verts + off.astype(np.float32)).astype(np.float32), w.scene.tris,
                  w.scene.tri_obj, w.scene.obj_alpha, w.scene.obj_vel, w.scene.pt_pos + off,
                  w.scene.pt_vel, w.scene.pt_aperture).checked()
    ar = _array(w.array.tx + off, w.array.rx + off)
    h2, p2 = orc.trace(sc, ar, w.trace)
    c2 = orc.synth(p2, sc, ar, w.chirp)
    assert (h1 == h2).all()
    assert np.linalg.norm(c1 - c2) / np.linalg.norm(c1) < 1e-8


def test_sampled_entries_match_full_cube(orc):
    w = sg.workload_tiny()
    w.trace.n_rays = 5000
    _, paths = orc.trace(w.scene, w.array, w.trace)
    full = orc.synth(paths, w.scene, w.array, w.chirp)
    idx = np.random.default_rng(0).choice(full.size, 300, replace=False)
    assert np.array_equal(orc.synth(paths, w.scene, w.array, w.chirp, idx=idx),
                          full.reshape(-1)[idx])


# ------------------------------------------------------ importance sampling

def test_proposal_launch_unbiased(orc):
    """Binned proposal q with weight p0/q: the received amplitude mass of the
    specular plate still estimates 1 - cos(theta_max)."""
    R, r = 5.0, 0.25
    sc = sg.plate(R, 1.0)
    o = [0.0, 0.0, 0.5]
    ar = _array(o, o, radius=r)
    na, ne = 128, 64
    rng = np.random.default_rng(3)
    ia = np.arange(na)[None, :]
    ie = np.arange(ne)[:, None]
    # concentrate on boresight, with random texture and a floor everywhere
    q = np.exp(-((ia - 63.5) ** 2 + (ie - 31.5) ** 2) / 30.0) + 0.02 * rng.random((ne, na)) + 1e-3
    q = (q / q.sum()).reshape(-1)
    cdf = np.concatenate([[0.0], np.cumsum(q)])
    cdf[-1] = 1.0
    N = 200_000
    tp = _tp(N)
    _, paths = orc.trace(sc, ar, tp, cdf=cdf, n_az=na, n_el=ne)
    est = paths["amp"].sum()
    st = r / (2 * R)
    exact = 1 - math.sqrt(1 - st * st)
    sd = math.sqrt(np.sum(paths["amp"] ** 2))
    assert abs(est - exact) < 4.5 * sd + 1e-12
    # the proposal concentrates samples there: far more paths than uniform
    assert len(paths) > 20 * N * exact
    # weights are 1 / (nb q_b) of the sampled bin
    w = paths["amp"] * N
    assert np.all(w > 0) and w.max() < 1.0


# ------------------------------------------------- multi-bounce path lengths

_CORNER = np.array([6.0, -1.5, -1.0])   # trihedral corner; FP32-exact coordinates
_SIDE = 3.0


def _corner_scene(vel=((0.0, 0.0, 0.0),) * 3, alpha=0.0):
    """Three mutually perpendicular square plates meeting at _CORNER, opening
    towards the radar at the origin side: plate 0 in the plane x = 6, plate 1
    in y = -1.5, plate 2 in z = -1 (one object each, so that each may move
    with its own velocity).  Plate i's triangles are 2 i and 2 i + 1."""
    mb = sg._MeshBuilder()
    X, Y, Z = _CORNER
    a = _SIDE
    mb.grid_quad((X, Y, Z), (0, a, 0), (0, 0, a), 1, 1, 0)
    mb.grid_quad((X - a, Y, Z), (a, 0, 0), (0, 0, a), 1, 1, 1)
    mb.grid_quad((X - a, Y, Z), (a, 0, 0), (0, a, 0), 1, 1, 2)
    return mb.build([alpha] * 3, list(vel))


def _mirror(pt, plate):
    """Mirror image of a point through the plane of plate 0, 1 or 2."""
    q = np.array(pt, float).copy()
    q[plate] = 2.0 * _CORNER[plate] - q[plate]
    return q


def _corner_paths(orc, n_rays=600_000, seed=1, vel=((0.0, 0.0, 0.0),) * 3):
    S = [0.0, 0.0, 0.5]
    rx = [[0.0, -0.05, 0.5], [0.0, 0.0, 0.45], [0.0, 0.07, 0.52]]
    ar = _array(S, rx, radius=0.5)
    sc = _corner_scene(vel)
    _, paths = orc.trace(sc, ar, _tp(n_rays, bounces=3, seed=seed))
    return sc, ar, paths


def test_multibounce_lengths_method_of_images(orc):
    """Specular (alpha = 0) trihedral: a path that reflects off the planes of
    hits 1 .. K-1 travels, from the source to its last hit p_K, exactly the
    straight distance from the source's image through those planes (taken in
    hit order) to p_K (method of images).  So every K = 1, 2, 3 path's length
    L = |p_K - S_(K-1)|, every hit lies on its plate's plane, and the cube of a
    single path is a exp(-j 2 pi f_k (|p_K - S_(K-1)| + |rx - p_K|) / c) for every
    receiver: this fixes the multi-bounce inner length of Eq. 4's path length
    without reference to the oracle's own sum over hit points."""
    sc, ar, paths = _corner_paths(orc)
    Ks = np.bincount(paths["K"], minlength=4)
    assert Ks[2] > 200 and Ks[3] > 100, Ks
    S = ar.tx[0]
    ch = sg.Chirp(n_samples=8, n_chirps=1)
    fk = ch.f0 + ch.bandwidth * np.arange(8) / 8
    for p in paths:
        K = int(p["K"])
        plates = [int(p["tri"][j]) // 2 for j in range(K)]
        img = np.array(S, float)
        for j in range(K):
            assert abs(p["p"][j][plates[j]] - _CORNER[plates[j]]) < 1e-12
            if j < K - 1:
                img = _mirror(img, plates[j])
        pK = p["p"][K - 1]
        Lref = np.linalg.norm(pK - img)
        assert abs(p["L"] - Lref) < 1e-12 * Lref, (K, p["L"], Lref)
    # synthesis of single paths, every receiver (K >= 2 only: the inner sum)
    for p in paths[paths["K"] >= 2][::7]:
        K = int(p["K"])
        img = np.array(S, float)
        for j in range(K - 1):
            img = _mirror(img, int(p["tri"][j]) // 2)
        pK = p["p"][K - 1]
        d = np.linalg.norm(pK - img) + np.linalg.norm(ar.rx - pK, axis=1)
        ref = p["amp"] * np.exp(-2j * np.pi * fk[None, :] * d[:, None] / C0)
        cube = orc.synth(p[None], sc, ar, ch)[:, 0, :]
        assert np.abs(cube - ref).max() < 1e-9 * p["amp"], (K, np.abs(cube - ref).max())


def test_triple_bounce_retroreflects(orc):
    """Three perpendicular mirrors send a ray back antiparallel: a K = 3 path
    that meets all three plates leaves its last hit along -d0 (d0 = its launch
    direction), and its image source is the source inverted through the
    corner.  Checks the K = 3 geometry of Eq. 2 applied three times."""
    sc, ar, paths = _corner_paths(orc, n_rays=300_000)
    S = ar.tx[0]
    p3 = paths[(paths["K"] == 3)]
    n_all = 0
    for p in p3:
        plates = sorted(int(t) // 2 for t in p["tri"][:3])
        if plates != [0, 1, 2]:
            continue
        n_all += 1
        d0 = (p["p"][0] - S) / np.linalg.norm(p["p"][0] - S)
        img = 2.0 * _CORNER - S
        # the last segment continues the line from the triple image through p3
        u = (p["p"][2] - img) / np.linalg.norm(p["p"][2] - img)
        assert np.abs(u + d0).max() < 1e-12 or np.abs(u - (-d0)).max() < 1e-12
        assert abs(p["L"] - np.linalg.norm(p["p"][2] - img)) < 1e-12 * p["L"]
    assert n_all > 50


def test_motion_galilean_shift(orc):
    """Every object (plates and a point reflector) moving with one velocity v:
    in the exact model, the cube at chirp m equals the chirp-0 cube of the
    static scene with every Tx and Rx moved by -v m T_rep (only relative
    positions enter a path length).  Covers the motion of the first, inner and
    last hit points of K = 1, 2, 3 paths."""
    v = (2.5, -1.25, 0.75)
    sc, ar, paths = _corner_paths(orc, n_rays=200_000, vel=(v,) * 3)
    assert (paths["K"] >= 2).sum() > 50
    sc.pt_pos = np.array([[4.0, 1.0, 0.3]])
    sc.pt_vel = np.array([v])
    sc.pt_aperture = np.array([0.02])
    _, ppt = orc.trace(sc, ar, _tp(10))
    pts = ppt[ppt["tri"][:, 0] == -1]
    assert len(pts) == 1
    allp = np.concatenate([paths, pts])
    ch = sg.Chirp(n_samples=16, n_chirps=6)
    moving = orc.synth(allp, sc, ar, ch, model=0)
    static = sg.Scene(sc.verts, sc.tris, sc.tri_obj, sc.obj_alpha, np.zeros((3, 3)),
                      sc.pt_pos, np.zeros((1, 3)), sc.pt_aperture).checked()
    ch1 = sg.Chirp(n_samples=16, n_chirps=1)
    for m in range(6):
        sh = -np.array(v) * m * ch.t_rep
        ar_m = _array(ar.tx + sh, ar.rx + sh, radius=ar.rx_radius)
        ref = orc.synth(allp, static, ar_m, ch1, model=0)[:, 0, :]
        err = np.abs(moving[:, m, :] - ref).max() / np.abs(ref).max()
        assert err < 1e-9, (m, err)
    # and the motion is really there: chirp 5 differs from chirp 0
    assert np.abs(moving[:, 5, :] - moving[:, 0, :]).max() > 0.1 * np.abs(moving).max()


def test_motion_per_object_hit_points(orc):
    """Each plate moving with its own velocity (reading R17: a hit point moves
    with the object it lies on, the path's topology is frozen at chirp 0): the
    cube at chirp m equals the chirp-0 cube of a static scene whose path
    records have every hit point p_j advanced by v_obj(j) m T_rep.  The inner
    segments of K = 2, 3 paths then change length, so a hit point that is not
    moved, or moved with another hit's object, fails."""
    vel = ((3.0, 0.5, -0.25), (-1.0, 2.0, 0.5), (0.25, -0.75, 1.5))
    sc, ar, paths = _corner_paths(orc, n_rays=200_000, vel=vel)
    multi = paths[paths["K"] >= 2]
    mixed = [len({int(t) // 2 for t in p["tri"][:p["K"]]}) > 1 for p in multi]
    assert sum(mixed) > 50
    ch = sg.Chirp(n_samples=16, n_chirps=5)
    moving = orc.synth(paths, sc, ar, ch, model=0)
    static = sg.Scene(sc.verts, sc.tris, sc.tri_obj, sc.obj_alpha, np.zeros((3, 3))).checked()
    ch1 = sg.Chirp(n_samples=16, n_chirps=1)
    V = np.array(vel)
    for m in range(5):
        tau = m * ch.t_rep
        q = paths.copy()
        for j in range(3):
            live = q["K"] > j
            q["p"][live, j, :] += V[q["vid"][live, j]] * tau
        ref = orc.synth(q, static, ar, ch1, model=0)[:, 0, :]
        err = np.abs(moving[:, m, :] - ref).max() / np.abs(ref).max()
        assert err < 1e-9, (m, err)
    # a frozen inner point would change the answer: check the relation is sharp
    tau = 4 * ch.t_rep
    q = paths.copy()
    for j in (0,):
        q["p"][:, j, :] += V[q["vid"][:, j]] * tau
    last = q["K"] - 1
    sel = last > 0
    q["p"][sel, last[sel], :] += V[q["vid"][sel, last[sel]]] * tau
    wrong = orc.synth(q, static, ar, ch1, model=0)[:, 0, :]
    three = q["K"] == 3
    assert three.sum() > 0
    assert np.abs(moving[:, 4, :] - wrong).max() > 1e-3 * np.abs(wrong).max()


# ------------------------------------------------------- proposal scene code

def test_probe_code_closed_form(orc):
    """Scene code of the learned proposal: 16 azimuth sectors of 8 rays at
    elevation 0 from the Tx phase centre, ray i of sector s at azimuth
    az_min + (8 s + i + 1/2) / 128 (az_max - az_min); each ray scores
    exp(-t / 10 m) if its closest hit belongs to an object other than object 0,
    else 0.  Object 0 here is a wall covering the left half (y > 0) in front of
    a plate of object 1 at x = R, so rays that meet the wall score 0 and the
    others that meet the plate score exp(-R' / (10 cos az)), R' = R - x_radar."""
    R, R0, W = 12.0, 6.0, 30.0
    mb = sg._MeshBuilder()
    mb.grid_quad((R0, 0.0, -5.0), (0.0, W, 0.0), (0.0, 0.0, 10.0), 1, 1, 0)
    mb.grid_quad((R, -W, -5.0), (0.0, 2 * W, 0.0), (0.0, 0.0, 10.0), 1, 1, 1)
    sc = mb.build([0.5, 0.5], [[0, 0, 0], [0, 0, 0]])
    o = np.array([0.5, 0.25, 0.5])
    ar = _array([o - [0, 0.01, 0], o + [0, 0.01, 0]], [o, o], mode=sg.MODE_SHARED)
    for az_lo, az_hi in ((-math.pi / 2, math.pi / 2), (-1.0, 0.6)):
        tp = sg.TraceParams(n_rays=10, max_bounces=1, seed=0, az_min=az_lo, az_max=az_hi)
        code = orc.probe_code(sc, ar, tp)
        ref = np.zeros(16)
        for s in range(16):
            acc = 0.0
            for i in range(8):
                az = az_lo + (8 * s + i + 0.5) / 128 * (az_hi - az_lo)
                y0 = o[1] + (R0 - o[0]) * math.tan(az)
                if 0.0 <= y0 <= W:
                    continue                       # object 0 (the wall) is hit first
                y = o[1] + (R - o[0]) * math.tan(az)
                if -W <= y <= W:
                    acc += math.exp(-(R - o[0]) / (10.0 * math.cos(az)))
            ref[s] = acc / 8
        assert np.abs(code - ref).max() < 1e-12, (az_lo, np.abs(code - ref).max())
        assert (code > 0).any() and (code == 0).any()
