"""Batched launch (a persistent trace kernel, the direct engine's persistent
synthesis kernel and the exact product engine's per-scene kernels captured
as one hipGraph): every scene's path count and cube must equal the
single-scene launch of the same workload on the same engine (bitwise with
the same tile shape, within float rounding after autotuning), replays must
reproduce the result, and sampled entries must match the FP64 oracle."""
import numpy as np
import pytest
import torch

import scenegen as sg
from helpers import rel_err

pytestmark = pytest.mark.gpu


def _workloads():
    w0 = sg.workload_tiny()
    w0.trace.n_rays = 50_000
    ws = [w0]
    ws += sg.workload_batch(n_scenes=4, seed0=2000, rays=200_000, tri_lo=1e4, tri_hi=1e5, ch_hi=256)
    ws.append(sg.workload_box_family(3, 30_000))
    ws.append(sg.Workload("street_small", sg.scene_street(1, scale=0.05, n_cars=5, n_poles=6),
                          sg.array_ula(4, 8), sg.Chirp(n_samples=96, n_chirps=32),
                          sg.TraceParams(n_rays=100_003, max_bounces=3, seed=5)))
    # no triangles: every ray misses, only the point reflectors return
    ws.append(sg.Workload("points", sg.point_only([[8.0, 1.0, 0.5], [15.0, -2.0, 0.6]],
                                                  vel=[[1.0, 0.0, 0.0], [-2.0, 0.5, 0.0]]),
                          sg.array_ula(2, 3), sg.Chirp(n_samples=64, n_chirps=8),
                          sg.TraceParams(n_rays=1000, max_bounces=2, seed=3)))
    return ws


def _single(gpu, w, engine=None):
    import paper_2307_15412_amd as rr
    gpu.setup(w)
    n = gpu.trace_workload(w, record_hits=False)
    eng = rr.DIRECT_FP32 if engine is None else engine
    return n, gpu.synthesize(model=rr.EXACT, engine=eng).clone()


def _sampled_oracle_err(orc, w, cube, seed, n=512):
    _, op = orc.trace(w.scene, w.array, w.trace, want_hits=False)
    flat = cube.reshape(-1)
    idx = np.random.default_rng(seed).choice(flat.numel(), n, replace=False)
    got = flat[torch.from_numpy(idx).to(flat.device)].cpu().numpy()
    return rel_err(got, orc.synth(op, w.scene, w.array, w.chirp, model=0, idx=idx))


def test_batch_matches_single_scene(gpu):
    import paper_2307_15412_amd as rr
    ws = _workloads()
    B = rr.Batch(gpu, len(ws))
    for i, w in enumerate(ws):
        B.set_workload(i, w)
        B.set_engine(i, rr.DIRECT_FP32)
    cubes = B.alloc_cubes()
    counts = B.launch(cubes)
    st = B.stats()
    assert st["paths"] == counts.sum() and st["ms_total"] > 0
    for i, w in enumerate(ws):
        n, ref = _single(gpu, w)
        assert counts[i] == n, (i, counts[i], n)
        assert torch.equal(cubes[i], ref), (i, rel_err(cubes[i].cpu().numpy(), ref.cpu().numpy()))
    # replay of the captured graph reproduces the result bitwise
    first = [c.clone() for c in cubes]
    for c in cubes:
        c.zero_()
    counts2 = B.launch(cubes)
    assert np.array_equal(counts, counts2)
    for a, b in zip(first, cubes):
        assert torch.equal(a, b)
    # new output buffers: only the device table changes
    other = B.alloc_cubes()
    B.launch(other)
    for a, b in zip(first, other):
        assert torch.equal(a, b)
    B.close()


def _exact_workloads():
    """Shared launches around the product tiles (16 to 96, and ragged), a
    moving street, a per-element launch and a points-only scene; the slots
    left at the least cost tile split their paths alike in the batch and in
    the single-scene launch (the batch sizes its splits by table capacity)."""
    def wl(name, scene, arr, K, M, rays, seed):
        return sg.Workload(name, scene, arr, sg.Chirp(n_samples=K, n_chirps=M),
                           sg.TraceParams(n_rays=rays, max_bounces=2, seed=seed))
    c1 = sg.scene_c1(4)
    street = sg.scene_street(2, scale=0.05, n_cars=5, n_poles=6)
    return [
        (wl("tiny33x70", c1, sg.array_sparse_grid(33, 70, 5), 64, 16, 60_000, 1), 0),
        (wl("street40", street, sg.array_sparse_grid(40, 40, 6), 96, 8, 120_000, 2), 64),
        (wl("tiny96", c1, sg.array_sparse_grid(96, 96, 7, grid=128), 16, 2, 40_000, 3), 96),
        (wl("street7x9", street, sg.array_sparse_grid(7, 9, 8), 128, 16, 100_000, 4), 32),
        (wl("tiny12", c1, sg.array_sparse_grid(12, 13, 10), 64, 8, 60_000, 6), 16),
        (wl("street42", street, sg.array_sparse_grid(42, 42, 12), 32, 4, 80_000, 7), 48),
        (wl("perel", c1, sg.array_ula(6, 8, mode=sg.MODE_PER_TX), 128, 128, 60_000, 5), 0),
        (wl("street12x16", street, sg.array_sparse_grid(12, 16, 13), 512, 16, 100_000, 8), 1),
        (sg.Workload("points", sg.point_only([[8.0, 1.0, 0.5], [15.0, -2.0, 0.6]],
                                             vel=[[1.0, 0.0, 0.0], [-2.0, 0.5, 0.0]]),
                     sg.array_sparse_grid(5, 6, 9), sg.Chirp(n_samples=64, n_chirps=8),
                     sg.TraceParams(n_rays=1000, max_bounces=2, seed=3)), 0),
    ]


def test_batch_exact_engine(gpu, orc):
    """Every slot pinned to the product engine (tiles 16 / 32 / 48 / 64 / 96
    or the per-channel sample split forced, or the layout of least modelled
    time): counts equal the single-scene launch; a slot at the least cost
    layout equals the single-scene product engine bit for bit (same layout,
    same path splits on both sides), forced layouts agree with it within the
    operands' rounding (2e-5); sampled entries within 1e-4 of the FP64
    oracle; replays, and a re-capture for new cube buffers, reproduce the
    cubes bit for bit."""
    import paper_2307_15412_amd as rr
    cases = _exact_workloads()
    B = rr.Batch(gpu, len(cases))
    for i, (w, tile) in enumerate(cases):
        B.set_workload(i, w)
        B.set_engine(i, rr.GEMM_EXACT, tile)
    eng, tiles = B.plan()
    assert (eng == rr.GEMM_EXACT).all()
    assert [int(t) for t in tiles[1:6]] == [64, 96, 32, 16, 48] and tiles[7] == 1
    cubes = B.alloc_cubes()
    counts = B.launch(cubes)
    for i, (w, tile) in enumerate(cases):
        n, ref = _single(gpu, w, rr.GEMM_EXACT)
        assert counts[i] == n, (i, counts[i], n)
        got = cubes[i]
        if tile == 0:
            assert torch.equal(got, ref), (i, rel_err(got.cpu().numpy(), ref.cpu().numpy()))
        else:
            # another layout rounds other split-bf16 operands (each product
            # term carries ~6e-6 relative rounding): agreement to 2e-5
            d = rel_err(got.cpu().numpy(), ref.cpu().numpy())
            assert d < 2e-5, (i, d)
        if n:
            assert _sampled_oracle_err(orc, w, got, 40 + i) < 1e-4, i
        else:
            assert not got.any()
    first = [c.clone() for c in cubes]
    for c in cubes:
        c.zero_()
    assert np.array_equal(B.launch(cubes), counts)
    for a, b in zip(first, cubes):
        assert torch.equal(a, b)
    other = B.alloc_cubes()
    B.launch(other)
    for a, b in zip(first, other):
        assert torch.equal(a, b)
    B.close()


def test_batch_exact_capacity_grows(gpu):
    """A reception sphere of 3 m makes far more rays return than the leg
    tables' first capacity (1 in 16 rays) holds: the launch grows the tables
    and re-runs, and the cube equals the single-scene product engine."""
    import paper_2307_15412_amd as rr
    w = sg.workload_tiny(6)
    w.array = sg.array_sparse_grid(8, 8, 11)
    w.array.rx_radius = 3.0
    w.trace.n_rays = 40_000
    w.chirp = sg.Chirp(n_samples=64, n_chirps=4)
    B = rr.Batch(gpu, 1)
    B.set_workload(0, w)
    B.set_engine(0, rr.GEMM_EXACT)
    cubes = B.alloc_cubes()
    counts = B.launch(cubes)
    n, ref = _single(gpu, w, rr.GEMM_EXACT)
    assert counts[0] == n > w.trace.n_rays // 16 + 3
    assert torch.equal(cubes[0], ref)
    B.close()


def test_batch_autotune(gpu):
    import paper_2307_15412_amd as rr
    ws = _workloads()
    B = rr.Batch(gpu, len(ws))
    for i, w in enumerate(ws):
        B.set_workload(i, w)
    cubes = B.alloc_cubes()
    tiles = B.tune(cubes)
    for t, w in zip(tiles, ws):
        K = w.chirp.n_samples
        assert t in (4, 8, 16, 32) and K % t == 0 and K // t <= 256
    eng, pt = B.plan()
    for e, t, tl, w in zip(eng, pt, tiles, ws):
        if e == rr.GEMM_EXACT:
            # a per-element launch takes the product engine only as the
            # sample split (tiles would multiply every path into all Tx rows)
            assert t in ((1, 16, 32, 48, 64, 96) if w.array.mode == sg.MODE_SHARED else (1,))
        else:
            assert e == rr.DIRECT_FP32 and t == tl
    counts = B.launch(cubes)
    for i, w in enumerate(ws):
        n, ref = _single(gpu, w)
        assert counts[i] == n
        assert rel_err(cubes[i].cpu().numpy(), ref.cpu().numpy()) < 2e-5
    B.close()


def test_batch_autotune_picks_product_engine(gpu):
    """Two shared 48 x 64 street scenes (3072 channels) beside a small
    per-element one: the tuner runs the large ones on the product engine (64
    or 48 tiles: 48 rows pad to 64 either way), the small one on whichever
    engine its timing favours; every cube agrees with the single-scene
    launch."""
    import paper_2307_15412_amd as rr
    street = sg.scene_street(3, scale=0.1, n_cars=8, n_poles=10)
    big = [sg.Workload(f"big{i}", street, sg.array_sparse_grid(48, 64, 30 + i),
                       sg.Chirp(n_samples=256, n_chirps=8),
                       sg.TraceParams(n_rays=200_000, max_bounces=3, seed=30 + i)) for i in range(2)]
    small = sg.workload_tiny(7)
    ws = [big[0], small, big[1]]
    B = rr.Batch(gpu, len(ws))
    for i, w in enumerate(ws):
        B.set_workload(i, w)
    cubes = B.alloc_cubes()
    B.tune(cubes)
    eng, tiles = B.plan()
    assert eng[0] == eng[2] == rr.GEMM_EXACT and tiles[1] in (1, 4, 8, 16, 32), (eng, tiles)
    counts = B.launch(cubes)
    for i, w in enumerate(ws):
        n, ref = _single(gpu, w)
        assert counts[i] == n
        assert rel_err(cubes[i].cpu().numpy(), ref.cpu().numpy()) < 2e-5, i
    B.close()


def test_batch_against_oracle(gpu, orc):
    import paper_2307_15412_amd as rr
    ws = _workloads()[:2] + _workloads()[-2:]
    B = rr.Batch(gpu, len(ws))
    for i, w in enumerate(ws):
        B.set_workload(i, w)
    cubes = B.alloc_cubes()
    B.launch(cubes)
    for i, w in enumerate(ws):
        _, op = orc.trace(w.scene, w.array, w.trace, want_hits=False)
        flat = cubes[i].reshape(-1)
        idx = np.random.default_rng(i).choice(flat.numel(), 512, replace=False)
        got = flat[torch.from_numpy(idx).to(flat.device)].cpu().numpy()
        ref = orc.synth(op, w.scene, w.array, w.chirp, model=0, idx=idx)
        assert rel_err(got, ref) < 1e-4, i
    B.close()


def test_batch_full_size_slot(gpu, orc):
    """Slots at the batched configuration's largest size: a street of 5.1e5
    triangles seen by 3072 channels (48 Tx x 64 Rx shared launch), 512 samples
    x 64 chirps, 1e6 rays, 3 bounces, twice among two uneven scenes: once left
    to AUTO (the product engine, 64 x 64 tiles) and once pinned to the direct
    engine.  Each equals the single-scene launch on its engine bit for bit,
    and 1024 seeded entries of each are within 1e-4 of the FP64 oracle (exact
    model)."""
    import paper_2307_15412_amd as rr
    big = sg.Workload("street_3072", sg.scene_street(7), sg.array_sparse_grid(48, 64, 24,
                      mode=sg.MODE_SHARED), sg.Chirp(n_samples=512, n_chirps=64),
                      sg.TraceParams(n_rays=1_000_000, max_bounces=3, seed=7))
    assert big.scene.n_tris >= 500_000 and big.array.n_ch == 3072
    ws = [sg.workload_batch(n_scenes=1, seed0=2010, rays=200_000, tri_hi=1e5, ch_hi=64)[0], big,
          sg.workload_box_family(4, 50_000), big]
    B = rr.Batch(gpu, len(ws))
    for i, w in enumerate(ws):
        B.set_workload(i, w)
    B.set_engine(3, rr.DIRECT_FP32)
    eng, tiles = B.plan()
    assert eng[1] == rr.GEMM_EXACT and tiles[1] == 64 and eng[3] == rr.DIRECT_FP32
    cubes = B.alloc_cubes()
    counts = B.launch(cubes)
    idx = np.random.default_rng(17).choice(cubes[1].numel(), 1024, replace=False)
    ti = torch.from_numpy(idx).to(cubes[1].device)
    got = {s: cubes[s].reshape(-1)[ti].cpu().numpy() for s in (1, 3)}
    for s, e in ((1, rr.GEMM_EXACT), (3, rr.DIRECT_FP32)):
        n, ref_cube = _single(gpu, big, e)
        assert counts[s] == n > 10_000
        assert torch.equal(cubes[s], ref_cube), s
        del ref_cube
    B.close()
    _, op = orc.trace(big.scene, big.array, big.trace, want_hits=False)
    assert len(op) == n
    ref = orc.synth(op, big.scene, big.array, big.chirp, model=0, idx=idx)
    for s in (1, 3):
        err = rel_err(got[s], ref)
        print(f"3072-channel slot {s}: {n} paths, relative error {err:.2e}, max ratio "
              f"{np.abs(got[s] - ref).max() / np.abs(ref).max():.2e}")
        assert err < 1e-4
