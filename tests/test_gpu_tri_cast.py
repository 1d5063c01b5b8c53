"""Per-triangle ray casting on the GPU against the FP64 oracle: hit lists
(all -1 for rays that are outside the field of view or whose first hit is not
the aimed-at triangle) and path records bitwise, on the tiny scene (per-element
launch, several bounce counts), the hand proxy (shared launch, +-25 degree
field of view that cuts the mesh), an occluding pair of triangles and a reduced
street, also with the triangles cut into pieces by solid angle; the cube
synthesised from those paths against the oracle's; invalid grids and casting
parameters rejected."""
import math

import numpy as np
import pytest

import scenegen as sg
from helpers import assert_paths_equal, gpu_soa_np, oracle_to_soa, rel_err, traced_rows

pytestmark = pytest.mark.gpu


def _compare(gpu, orc, w):
    gpu.setup(w)
    n = gpu.trace_workload(w, record_hits=True)
    hits = gpu.hits().cpu().numpy()
    oh, op = orc.trace(w.scene, w.array, w.trace)
    oh = oh[traced_rows(orc, w.scene, w.array, w.trace)]
    assert hits.shape == oh.shape
    bad = np.argwhere((hits != oh).any(axis=1))
    assert bad.size == 0, f"{bad.size} rays differ, first {bad[:5].ravel().tolist()}"
    assert n == len(op)
    assert_paths_equal(gpu_soa_np(gpu), oracle_to_soa(op))
    return n, hits, op


def test_tiny_per_element(gpu, orc):
    for g, b in ((16, 2), (8, 1), (1, 3)):
        w = sg.workload_tiny(4)
        w.trace = sg.TraceParams(n_rays=0, max_bounces=b, seed=6, rays_per_tri=g * g)
        n, hits, _ = _compare(gpu, orc, w)
        assert (hits[:, 0] == -1).any()
    assert n > 0


def test_hand_shared_cut_fov(gpu, orc):
    deg = math.pi / 180
    w = sg.Workload("hand", sg.scene_hand_proxy(5, step=6e-3),
                    sg.array_square(n_side=5, pitch=3e-3, rx_radius=0.07), sg.chirp_sfcw(72e9, 82e9, 32),
                    sg.TraceParams(n_rays=0, max_bounces=2, seed=3, az_min=-8 * deg, az_max=12 * deg,
                                   el_min=-10 * deg, el_max=6 * deg, rays_per_tri=9))
    n, hits, op = _compare(gpu, orc, w)
    assert n > 20
    counted = hits[:, 0] >= 0
    assert 0.05 < counted.mean() < 0.95
    # the cube of these paths (exact model, direct engine)
    import paper_2307_15412_amd as rr
    cube = gpu.synthesize(model=rr.EXACT, engine=rr.DIRECT_FP32).cpu().numpy()
    ref = orc.synth(op, w.scene, w.array, w.chirp, model=0)
    assert rel_err(cube, ref) < 1e-4


def test_occluding_pair_and_street(gpu, orc):
    v = np.array([[4.0, -0.2, -0.1], [4.0, 0.3, -0.1], [4.0, 0.0, 0.3],
                  [6.0, -1.0, -1.0], [6.0, 1.5, -0.8], [6.0, -0.2, 1.4]], np.float32)
    sc = sg.Scene(v, np.arange(6, dtype=np.int32).reshape(2, 3), np.zeros(2, np.int32),
                  np.array([0.5], np.float32), np.zeros((1, 3))).checked()
    o = np.zeros((1, 3))
    w = sg.Workload("pair", sc, sg.Array(o, o.copy(), 1e3, sg.MODE_PER_TX), sg.Chirp(),
                    sg.TraceParams(n_rays=0, max_bounces=2, seed=2, rays_per_tri=32 * 32))
    n, hits, _ = _compare(gpu, orc, w)
    assert (hits[: 1024, 0] == 0).all() and (hits[1024:, 0] == -1).any()
    st = sg.Workload("street", sg.scene_street(3, scale=0.05, n_cars=5, n_poles=6),
                     sg.array_ula(2, 4, mode=sg.MODE_PER_TX), sg.Chirp(n_samples=64, n_chirps=8),
                     sg.TraceParams(n_rays=0, max_bounces=3, seed=8, rays_per_tri=16))
    assert st.scene.n_tris > 1000
    _compare(gpu, orc, st)


def test_subdivided_pieces(gpu, orc):
    """Triangles cut into pieces by solid angle, pieces out of view dropped:
    the piece count and every hit and path bitwise against the oracle, on the
    reduced street (its ground and facades fill most of the view) and on the
    occluding pair; changing the parameters, the field of view or the
    vertices rebuilds the pieces."""
    st = sg.Workload("street", sg.scene_street(3, scale=0.05, n_cars=5, n_poles=6),
                     sg.array_ula(2, 4, mode=sg.MODE_PER_TX), sg.Chirp(n_samples=64, n_chirps=8),
                     sg.TraceParams(n_rays=0, max_bounces=2, seed=8, rays_per_tri=4,
                                    tri_omega_max=2e-3, tri_depth_max=6))
    fov = orc.fov_of(st.trace)
    n_orc = len(orc.pieces(st.scene, st.array, 2e-3, 6, fov)[1])
    assert n_orc > st.scene.n_tris
    _compare(gpu, orc, st)
    assert gpu.casting_pieces(*fov) == n_orc
    gpu.set_casting(2e-3, 2)
    assert gpu.casting_pieces(*fov) == len(orc.pieces(st.scene, st.array, 2e-3, 2, fov)[1])
    gpu.set_casting(0.0, 8)
    assert gpu.casting_pieces(*fov) == len(orc.pieces(st.scene, st.array, 0.0, 8, fov)[1])
    # a narrower view drops more pieces; no culling keeps every triangle
    deg = math.pi / 180
    narrow = (-20 * deg, 35 * deg, -15 * deg, 10 * deg)
    assert (gpu.casting_pieces(*narrow) == len(orc.pieces(st.scene, st.array, 0.0, 8, narrow)[1])
            < len(orc.pieces(st.scene, st.array, 0.0, 8)[1]) == st.scene.n_tris)
    v = np.array([[4.0, -0.2, -0.1], [4.0, 0.3, -0.1], [4.0, 0.0, 0.3],
                  [6.0, -1.0, -1.0], [6.0, 1.5, -0.8], [6.0, -0.2, 1.4]], np.float32)
    sc = sg.Scene(v, np.arange(6, dtype=np.int32).reshape(2, 3), np.zeros(2, np.int32),
                  np.array([0.5], np.float32), np.zeros((1, 3))).checked()
    o = np.zeros((1, 3))
    w = sg.Workload("pair", sc, sg.Array(o, o.copy(), 1e3, sg.MODE_PER_TX), sg.Chirp(),
                    sg.TraceParams(n_rays=0, max_bounces=2, seed=2, rays_per_tri=16,
                                   tri_omega_max=5e-3, tri_depth_max=5))
    _compare(gpu, orc, w)
    n0 = gpu.casting_pieces()
    # moved vertices: the pieces follow
    v2 = v - np.array([1.5, 0.0, 0.0], np.float32)
    gpu.update_vertices(v2)
    w2 = sg.Workload("pair2", sg.with_verts(sc, v2), w.array, w.chirp, w.trace)
    assert gpu.casting_pieces() == len(orc.pieces(w2.scene, w2.array, 5e-3, 5,
                                                  orc.fov_of(w2.trace))[1]) != n0
    n = gpu.trace_workload(w2, record_hits=True)
    oh, op = orc.trace(w2.scene, w2.array, w2.trace)
    assert np.array_equal(gpu.hits().cpu().numpy(), oh[traced_rows(orc, w2.scene, w2.array,
                                                                   w2.trace)])
    assert n == len(op)
    assert_paths_equal(gpu_soa_np(gpu), oracle_to_soa(op))


def test_nothing_in_view(gpu, orc):
    """A field of view that holds no triangle: every piece is dropped, the
    launch traces nothing and returns no path, on both sides."""
    v = np.array([[4.0, -0.2, -0.1], [4.0, 0.3, -0.1], [4.0, 0.0, 0.3]], np.float32)
    sc = sg.Scene(v, np.arange(3, dtype=np.int32).reshape(1, 3), np.zeros(1, np.int32),
                  np.array([0.5], np.float32), np.zeros((1, 3))).checked()
    o = np.zeros((1, 3))
    w = sg.Workload("aside", sc, sg.Array(o, o.copy(), 1e3, sg.MODE_PER_TX), sg.Chirp(),
                    sg.TraceParams(n_rays=0, max_bounces=2, seed=1, az_min=-1.2, az_max=-0.6,
                                   rays_per_tri=16, tri_omega_max=1e-3, tri_depth_max=4))
    n, hits, _ = _compare(gpu, orc, w)
    assert n == 0 and hits.shape == (0, 3)
    assert gpu.casting_pieces(*orc.fov_of(w.trace)) == 0


def test_invalid_grids(gpu):
    import paper_2307_15412_amd as rr
    w = sg.workload_tiny()
    gpu.setup(w)
    for n, az in ((5, 1.0), (0, 1.0), (4, 1.7)):
        with pytest.raises(rr.RadrayError) as e:
            gpu.trace(n_rays=n, max_bounces=2, az_min=-az, az_max=az, sampler=rr.PER_TRIANGLE)
        assert e.value.code == rr.binding.RR_EINVAL
    for om, dm in ((-1.0, 4), (float("nan"), 4), (1e-3, 21), (1e-3, -1)):
        with pytest.raises(rr.RadrayError) as e:
            gpu.set_casting(om, dm)
        assert e.value.code == rr.binding.RR_EINVAL
