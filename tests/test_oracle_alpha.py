"""Pins of the oracle's per-face material mix (Eq. 3 with alpha per face
instead of per object), against facts that do not depend on how it reads the
override: a face override equal to every face's object value changes nothing
(a wrong index would pick another object's alpha on a scene whose objects
differ); giving a set of faces their own alpha is the same as moving them into
an object of that alpha; an all-specular override of a diffuse plate is the
specular plate; and the paper's sweep values."""
import numpy as np

import oracle
import scenegen as sg


def _tp(n=20_000, b=2, seed=3):
    return sg.TraceParams(n_rays=n, max_bounces=b, seed=seed)


def _same(a, b, skip=()):
    ha, pa = a
    hb, pb = b
    assert np.array_equal(ha, hb)
    assert len(pa) == len(pb)
    for f in pa.dtype.names:
        if f not in skip:
            assert np.array_equal(pa[f], pb[f]), f


def test_override_equal_to_objects_changes_nothing():
    w = sg.workload_tiny(0)
    sc = w.scene
    sc = sg.Scene(sc.verts, sc.tris, sc.tri_obj, np.array([0.15, 0.85], np.float32)[:sc.n_obj],
                  sc.obj_vel, sc.pt_pos, sc.pt_vel, sc.pt_aperture).checked()
    assert sc.n_obj == 2 and sc.obj_alpha[0] != sc.obj_alpha[1]
    ov = sg.Scene(sc.verts, sc.tris, sc.tri_obj, sc.obj_alpha, sc.obj_vel, sc.pt_pos, sc.pt_vel,
                  sc.pt_aperture, sc.obj_alpha[sc.tri_obj]).checked()
    ref = oracle.trace(sc, w.array, _tp())
    got = oracle.trace(ov, w.array, _tp())
    assert len(ref[1]) > 100
    _same(got, ref)
    # swapping the two objects' values in the override must change the result
    sw = sg.Scene(sc.verts, sc.tris, sc.tri_obj, sc.obj_alpha, sc.obj_vel, sc.pt_pos, sc.pt_vel,
                  sc.pt_aperture, sc.obj_alpha[1 - sc.tri_obj]).checked()
    other = oracle.trace(sw, w.array, _tp())
    assert not np.array_equal(other[0], ref[0])


def test_face_set_equals_own_object():
    """Faces of the box given alpha 0.9 by override = the box as an object of
    alpha 0.9 (paths equal except the recorded object ids)."""
    w = sg.workload_tiny(1)
    sc = w.scene
    box = sc.tri_obj == 1
    one = sg.Scene(sc.verts, sc.tris, np.zeros_like(sc.tri_obj), np.array([0.4], np.float32),
                   np.zeros((1, 3)), sc.pt_pos, sc.pt_vel, sc.pt_aperture,
                   np.where(box, 0.9, 0.4).astype(np.float32)).checked()
    two = sg.Scene(sc.verts, sc.tris, box.astype(np.int32), np.array([0.4, 0.9], np.float32),
                   np.zeros((2, 3)), sc.pt_pos, sc.pt_vel, sc.pt_aperture).checked()
    a = oracle.trace(one, w.array, _tp(seed=5))
    b = oracle.trace(two, w.array, _tp(seed=5))
    assert len(a[1]) > 100
    _same(a, b, skip=("vid",))


def test_specular_override_of_diffuse_plate():
    diffuse = sg.plate(5.0, 1.0, alpha=1.0)
    spec = sg.plate(5.0, 1.0, alpha=0.0)
    ov = sg.Scene(diffuse.verts, diffuse.tris, diffuse.tri_obj, diffuse.obj_alpha,
                  diffuse.obj_vel, tri_alpha=np.zeros(diffuse.n_tris, np.float32)).checked()
    arr = sg.Array(np.array([[0, 0, 0.5]]), np.array([[0, 0, 0.5]]), 0.25, sg.MODE_PER_TX)
    tp = sg.TraceParams(n_rays=50_000, max_bounces=1, seed=2)
    ref = oracle.trace(spec, arr, tp)
    _same(oracle.trace(ov, arr, tp), ref)
    assert len(ref[1]) > 10
    # the diffuse plate returns other rays
    dif = oracle.trace(diffuse, arr, tp)[1]
    assert set(dif["ray"].tolist()) != set(ref[1]["ray"].tolist())


def test_sweep_values_and_variation():
    v = sg.alpha_sweep()
    assert len(v) == 11 and v[0] == 0.0 and v[-1] == 1.0
    assert np.allclose(np.diff(v), 0.1, atol=1e-6)
    sc = sg.vary_alpha(sg.scene_hand_proxy(0, step=6e-3), seed=4, spread=0.2)
    assert sc.tri_alpha.shape == (sc.n_tris,)
    assert sc.tri_alpha.min() >= 0.1 - 1e-6 and sc.tri_alpha.max() <= 0.5 + 1e-6
    assert np.unique(sc.tri_alpha).size > sc.n_tris // 2
