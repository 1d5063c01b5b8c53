"""GPU tracer parity with the FP64 oracle: per-ray hit lists (closest-hit
triangle ids of every segment) and the received path records must be
bitwise identical."""
import time

import numpy as np
import pytest

import scenegen as sg
from helpers import assert_paths_equal, gpu_soa_np, oracle_to_soa, traced_rows

pytestmark = pytest.mark.gpu


def _check_full(gpu, orc, w):
    gpu.setup(w)
    n = gpu.trace_workload(w, record_hits=True)
    hits = gpu.hits().cpu().numpy()
    oh, op = orc.trace(w.scene, w.array, w.trace)
    rows = traced_rows(orc, w.scene, w.array, w.trace)
    oh = oh[rows if len(rows) else slice(0, 0)]
    assert hits.shape == oh.shape
    bad = np.argwhere((hits != oh).any(axis=1))
    assert bad.size == 0, f"{bad.size} rays differ, first {bad[:5].ravel().tolist()}"
    assert n == len(op)
    assert_paths_equal(gpu_soa_np(gpu), oracle_to_soa(op))
    return n


def test_tiny_bit_exact(gpu, orc):
    """1e5 rays, 2 bounces, ground + moving box + 3 reflectors."""
    n = _check_full(gpu, orc, sg.workload_tiny())
    assert n > 1000


def test_tiny_other_seeds_and_bounces(gpu, orc):
    for seed, b in ((1, 1), (7, 3), (11, 4)):
        w = sg.workload_tiny(seed)
        w.trace.n_rays = 30_000
        w.trace.max_bounces = b
        _check_full(gpu, orc, w)


def test_ragged_and_empty(gpu, orc):
    """Ray counts that leave a partial block, a single ray, zero rays, and a
    scene without triangles (points only)."""
    w = sg.workload_tiny()
    for n in (1, 129, 1000):
        w.trace.n_rays = n
        _check_full(gpu, orc, w)
    w.trace.n_rays = 0
    _check_full(gpu, orc, w)
    pts = sg.point_only([[10.0, 1.0, 0.5], [20.0, -3.0, 1.0], [7.0, 0.0, 0.2]], aperture=0.02)
    wp = sg.Workload("pts", pts, sg.array_ula(3, 4), sg.Chirp(), sg.TraceParams(n_rays=999))
    assert _check_full(gpu, orc, wp) == 9


def test_specular_plate_and_shared_launch(gpu, orc):
    sc = sg.plate(5.0, 1.0, alpha=0.0)
    arr = sg.Array(np.array([[0, 0, 0.5]]), np.array([[0, 0, 0.5]]), 0.25, sg.MODE_PER_TX)
    w = sg.Workload("plate", sc, arr, sg.Chirp(), sg.TraceParams(n_rays=200_000, max_bounces=2))
    _check_full(gpu, orc, w)
    w2 = sg.workload_tiny()
    w2.array = sg.array_sparse_grid(8, 8, 3, mode=sg.MODE_SHARED)
    w2.trace.n_rays = 50_000
    _check_full(gpu, orc, w2)


def test_street_reduced_bit_exact(gpu, orc):
    """Street scene (5.1e5 triangles), 12 Tx x 16 Rx, 3 bounces, 1.2e5 rays:
    every ray against the oracle (its BVH is pinned to brute force)."""
    w = sg.workload_street(0, n_rays=120_000)
    n = _check_full(gpu, orc, w)
    assert n > 0


def test_street_full_size_sampled(gpu, orc):
    """Street at full size (1e7 rays) in the benchmarked launch: 3000 seeded
    rays traced one by one by the oracle, hit lists and paths bitwise."""
    w = sg.workload_street(0)
    gpu.setup(w)
    gpu.trace_workload(w, record_hits=True)
    hits = gpu.hits().cpu().numpy()
    gp = gpu_soa_np(gpu)
    rows = traced_rows(orc, w.scene, w.array, w.trace)
    rng = np.random.default_rng(42)
    pick = np.sort(rng.choice(len(rows), 3000, replace=False))
    # include the last ray of every source (ragged tails of the launch)
    per = orc.n_per_src(w.scene, w.array, w.trace)
    pick = np.unique(np.concatenate([pick, np.arange(1, orc.n_src(w.array) + 1) * per - 1]))
    vids = rows[pick]
    t0 = time.time()
    oh, op = orc.trace(w.scene, w.array, w.trace, vids=vids)
    assert time.time() - t0 < 300
    assert (hits[pick] == oh).all()
    sel = np.isin(gp["ray"], vids)
    g = {k: (v[..., sel]) for k, v in gp.items()}
    assert_paths_equal(g, oracle_to_soa(op))


def test_trace_without_host_count(gpu, orc):
    """rr_trace with no count pointer does not wait for the GPU: the path
    count is read back by the first call that needs it, and the paths, hit
    list and cube equal those of a trace that read it back at once."""
    import paper_2307_15412_amd as rr
    w = sg.workload_tiny(2)
    w.trace.n_rays = 40_000
    gpu.setup(w)
    n_sync = gpu.trace_workload(w, record_hits=True)
    ref_paths = gpu_soa_np(gpu)
    ref_hits = gpu.hits().cpu().numpy()
    ref_cube = gpu.synthesize(model=rr.EXACT, engine=rr.DIRECT_FP32).cpu().numpy()
    assert gpu.trace_workload(w, record_hits=True, sync=False) is None
    cube = gpu.synthesize(model=rr.EXACT, engine=rr.DIRECT_FP32).cpu().numpy()
    assert np.array_equal(cube, ref_cube)
    assert gpu.path_count() == n_sync
    assert_paths_equal(gpu_soa_np(gpu), ref_paths)
    assert np.array_equal(gpu.hits().cpu().numpy(), ref_hits)
    # and against the oracle, path cap included
    w.path_cap = n_sync // 3
    gpu.trace_workload(w, record_hits=False, sync=False)
    assert gpu.path_count() == n_sync // 3
    _, op = orc.trace(w.scene, w.array, w.trace)
    assert_paths_equal(gpu_soa_np(gpu), oracle_to_soa(op[: n_sync // 3]))


def test_trace_without_host_count_overflow(orc):
    """More paths than the temporary buffer holds, without a host count: the
    first call that needs the count reports RR_EOVERFLOW (the dropped records
    are never read), the buffer has grown, and the repeated trace is exact."""
    import paper_2307_15412_amd as rr
    ctx = rr.Context(0)
    try:
        sc = sg.plate(2.0, 50.0, alpha=1.0)
        arr = sg.Array(np.array([[0, 0, 0.5]]), np.array([[0, 0, 0.5]]), 60.0, sg.MODE_PER_TX)
        w = sg.Workload("plate", sc, arr, sg.Chirp(), sg.TraceParams(n_rays=400_000, max_bounces=2))
        ctx.setup(w)
        ctx.trace_workload(w, record_hits=False, sync=False)
        with pytest.raises(rr.RadrayError) as e:
            ctx.path_count()
        assert e.value.code == rr.binding.RR_EOVERFLOW
        with pytest.raises(rr.RadrayError):
            ctx.synthesize(model=rr.EXACT, engine=rr.DIRECT_FP32)
        ctx.trace_workload(w, record_hits=False, sync=False)
        n = ctx.path_count()
        _, op = orc.trace(w.scene, w.array, w.trace)
        assert n == len(op) > 65536
        assert_paths_equal(gpu_soa_np(ctx), oracle_to_soa(op))
    finally:
        ctx.close()
