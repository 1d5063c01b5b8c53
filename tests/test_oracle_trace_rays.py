"""Caller-supplied rays in the oracle (orc_trace_rays), pinned without
reference to itself: fed the uniform launch's own rays (Sec. III-A) it must
reproduce the pinned orc_trace bit for bit, in both launch modes; a mirror
(Eq. 2, alpha = 0) returns a normal-incidence ray to the receiver with the
closed-form hit point and length; malformed inputs are refused."""
import math

import numpy as np
import pytest

import oracle
import scenegen as sg


def _no_points(sc):
    return sg.Scene(sc.verts, sc.tris, sc.tri_obj, sc.obj_alpha, sc.obj_vel).checked()


def _centroid(p):
    # summed in index order, as the tracer does
    s = [0.0, 0.0, 0.0]
    for row in p:
        for a in range(3):
            s[a] += float(row[a])
    return np.array([x / len(p) for x in s])


def _launch_rays(scene, array, tp):
    """The rays the uniform launch draws: origin, direction, amplitude w / N_t
    and source of every launched ray, in virtual-ray order."""
    n_src = oracle.n_src(array)
    n_per = oracle.n_per_src(scene, array, tp)
    orig, dirs, amp, src = [], [], [], []
    for t in range(n_src):
        o = _centroid(array.tx) if array.mode == sg.MODE_SHARED else array.tx[t]
        for i in range(n_per):
            d = oracle.launch_dir(scene, array, tp, i, t)
            orig.append(o)
            dirs.append(d[:3])
            amp.append(d[3] / n_per)
            src.append(-1 if array.mode == sg.MODE_SHARED else t)
    return (np.array(orig), np.array(dirs), np.array(amp), np.array(src, dtype=np.int32))


@pytest.mark.parametrize("mode", [sg.MODE_PER_TX, sg.MODE_SHARED])
def test_launch_rays_reproduce_trace(mode):
    w = sg.workload_tiny(2)
    scene = _no_points(w.scene)
    array = sg.array_ula(3, 4, mode=mode)
    tp = sg.TraceParams(n_rays=3000, max_bounces=3, seed=9)
    hits, paths = oracle.trace(scene, array, tp)
    o, d, a, s = _launch_rays(scene, array, tp)
    hits2, paths2 = oracle.trace_rays(scene, array, o, d, a, s, tp.max_bounces, tp.seed)
    assert len(paths) > 50
    assert np.array_equal(hits, hits2)
    assert paths.tobytes() == paths2.tobytes()


def test_mirror_normal_incidence():
    dist = 7.25
    scene = sg.plate(dist, 1.0, alpha=0.0)
    array = sg.array_c1()
    oR = _centroid(array.rx)
    hits, paths = oracle.trace_rays(scene, array, oR[None, :], np.array([[2.0, 0.0, 0.0]]),
                                    np.array([0.125]), np.array([0], dtype=np.int32), 2, 1)
    assert hits[0, 0] >= 0 and hits[0, 1] == -1
    assert len(paths) == 1
    p = paths[0]
    assert p["K"] == 1 and p["src"] == 0 and p["ray"] == 0 and p["amp"] == 0.125
    assert p["L"] == pytest.approx(dist - oR[0], abs=1e-12)
    assert np.allclose(p["p"][0], [dist, oR[1], oR[2]], atol=1e-12)


def test_rejects_malformed_rays():
    scene = sg.plate(5.0, 1.0)
    per = sg.array_ula(2, 2)
    shared = sg.array_ula(2, 2, mode=sg.MODE_SHARED)
    o = np.zeros((2, 3))
    d = np.array([[1.0, 0, 0], [1.0, 0, 0]])
    a = np.ones(2)
    ok = np.array([0, 1], dtype=np.int32)
    oracle.trace_rays(scene, per, o, d, a, ok, 1, 0)
    for arr, src, dd, aa in [(per, np.array([1, 0], np.int32), d, a),      # not ascending
                             (per, np.array([0, 2], np.int32), d, a),      # no such Tx
                             (shared, ok, d, a),                           # shared needs -1
                             (per, ok, np.array([[1.0, 0, 0], [0, 0, 0]]), a),
                             (per, ok, np.array([[1.0, 0, 0], [math.nan, 0, 0]]), a),
                             (per, ok, d, np.array([1.0, math.inf]))]:
        with pytest.raises(ValueError):
            oracle.trace_rays(scene, arr, o, dd, aa, src, 1, 0)
