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
