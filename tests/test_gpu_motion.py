"""Moving meshes (the paper's outlook: radar responses of hand movements):
the BVH refit on the GPU after rr_scene_update_vertices.  An unchanged mesh
refits to the bitwise identical tree (so the refit pads and rounds exactly as
the host build); after every frame of a hand motion, after large random
vertex jitter and for per-triangle casting, hit lists and path records are
bitwise equal to the oracle tracing the moved mesh from scratch; every
refit child box contains its subtree's triangles; invalid updates are
rejected."""
import math

import numpy as np
import pytest

import scenegen as sg
from helpers import assert_paths_equal, gpu_soa_np, oracle_to_soa, traced_rows

pytestmark = pytest.mark.gpu


def _hand_w(scene, n_rays=30_000, rays_per_tri=0):
    deg = math.pi / 180
    return sg.Workload("hand", scene, sg.array_square(n_side=5, pitch=3e-3, rx_radius=0.07),
                       sg.chirp_sfcw(72e9, 82e9, 32),
                       sg.TraceParams(n_rays=n_rays, max_bounces=2, seed=11, az_min=-25 * deg,
                                      az_max=25 * deg, el_min=-25 * deg, el_max=25 * deg,
                                      rays_per_tri=rays_per_tri))


def _compare(gpu, orc, w):
    n = gpu.trace_workload(w, record_hits=True)
    hits = gpu.hits().cpu().numpy()
    oh, op = orc.trace(w.scene, w.array, w.trace)
    oh = oh[traced_rows(orc, w.scene, w.array, w.trace)]
    bad = np.argwhere((hits != oh).any(axis=1))
    assert bad.size == 0, f"{bad.size} rays differ, first {bad[:5].ravel().tolist()}"
    assert n == len(op)
    assert_paths_equal(gpu_soa_np(gpu), oracle_to_soa(op))
    return n


def test_refit_unchanged_is_identical(gpu):
    for sc in (sg.scene_hand_proxy(2, step=3e-3), sg.scene_street(4, scale=0.05, n_cars=4, n_poles=4)):
        w = _hand_w(sc)
        gpu.setup(w)
        before = gpu.bvh_nodes()
        gpu.update_vertices(sc.verts)
        assert np.array_equal(gpu.bvh_nodes().view(np.uint32), before.view(np.uint32))


def test_motion_frames_bitwise(gpu, orc):
    sc, frames = sg.hand_motion(3, n_frames=6, step=4e-3)
    w = _hand_w(sc)
    gpu.setup(w)
    first = gpu.bvh_nodes()
    counts = []
    for f in range(1, len(frames)):
        gpu.update_vertices(frames[f])
        counts.append(_compare(gpu, orc, _hand_w(sg.with_verts(sc, frames[f]))))
    assert len(set(counts)) > 1
    # back to frame 0: the original tree again
    gpu.update_vertices(frames[0])
    assert np.array_equal(gpu.bvh_nodes().view(np.uint32), first.view(np.uint32))
    _compare(gpu, orc, w)


def test_large_jitter_and_per_triangle(gpu, orc):
    sc = sg.scene_hand_proxy(4, step=5e-3)
    w = _hand_w(sc)
    gpu.setup(w)
    rng = np.random.default_rng(0)
    moved = (sc.verts + rng.uniform(-0.05, 0.05, sc.verts.shape)).astype(np.float32)
    gpu.update_vertices(moved)
    sc2 = sg.with_verts(sc, moved)
    _compare(gpu, orc, _hand_w(sc2))
    _compare(gpu, orc, _hand_w(sc2, n_rays=0, rays_per_tri=4))
    # every moved triangle lies inside the root's two child boxes, and every
    # internal child box holds its child node's two boxes
    nodes = gpu.bvh_nodes()
    refs = nodes[:, 12:14].copy().view(np.int32)
    tri_lo = moved[sc.tris].min(axis=1)
    tri_hi = moved[sc.tris].max(axis=1)
    root_lo = np.minimum(nodes[0, 0:3], nodes[0, 6:9])
    root_hi = np.maximum(nodes[0, 3:6], nodes[0, 9:12])
    assert (tri_lo >= root_lo).all() and (tri_hi <= root_hi).all()
    stack = [0]
    while stack:
        n = stack.pop()
        for c in range(2):
            r = refs[n, c]
            if r >= 0:
                box = nodes[n, 6 * c: 6 * c + 6]
                for cc in range(2):
                    kid = nodes[r, 6 * cc: 6 * cc + 6]
                    assert (kid[:3] >= box[:3]).all() and (kid[3:] <= box[3:]).all()
                stack.append(r)


def test_invalid_updates(gpu):
    import paper_2307_15412_amd as rr
    sc = sg.scene_hand_proxy(0, step=6e-3)
    gpu.setup(_hand_w(sc))
    for v in (sc.verts[:-1], np.where(np.arange(sc.verts.size).reshape(sc.verts.shape) == 7,
                                      np.nan, sc.verts)):
        with pytest.raises(rr.RadrayError) as e:
            gpu.update_vertices(v)
        assert e.value.code == rr.binding.RR_EINVAL
