"""Back-projection imaging on the GPU against the FP64 oracle, for both
engines (Horner on the vector units, split-bf16 products on the matrix
cores): the same oracle cube imaged by both sides (small grid, every voxel),
the whole pipeline trace -> synthesis -> back-projection on both sides, the
full-size grid of the paper's set-up (94 x 94 square array, 128 frequency
steps, 3.3e6 voxels) on sampled voxels with the focus of a point reflector,
ragged voxel counts and array sizes at the engine's limits; and the maximum
projection in dB."""
import numpy as np
import pytest
import torch

import scenegen as sg
from helpers import rel_err

pytestmark = pytest.mark.gpu

TOL = 1e-4


ENGINES = [1, 3]          # DIRECT_FP32, GEMM_EXACT


def _voxels(grid):
    (x0, y0, z0), st, (nx, ny, nz) = grid
    i, j, k = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    return np.stack([x0 + i * st, y0 + j * st, z0 + k * st], -1).reshape(-1, 3)


def _setup(gpu, scene, array, chirp):
    w = sg.Workload("img", scene, array, chirp, sg.TraceParams(n_rays=0, max_bounces=1))
    gpu.setup(w)
    return w


def _upload(cube):
    return torch.from_numpy(np.ascontiguousarray(cube).astype(np.complex64)).cuda()


@pytest.mark.parametrize("engine", ENGINES)
def test_same_cube_every_voxel(gpu, orc, engine):
    array = sg.array_square(n_side=6, pitch=3e-3)
    chirp = sg.chirp_sfcw(72e9, 82e9, 48)
    scene = sg.scene_hand_proxy(1, step=6e-3)
    tp = sg.TraceParams(n_rays=40_000, max_bounces=2, seed=2, az_min=-0.4, az_max=0.4,
                        el_min=-0.4, el_max=0.4)
    _, op = orc.trace(scene, array, tp, want_hits=False)
    assert len(op) > 50
    cube = orc.synth(op, scene, array, chirp, model=0)
    _setup(gpu, scene, array, chirp)
    grid = ((0.28, -0.03, -0.04), 4e-3, (7, 9, 11))
    img = gpu.backproject(_upload(cube), grid, engine=engine).cpu().numpy().reshape(-1)
    ref = orc.backproject(array, chirp.f0, chirp.bandwidth / chirp.n_samples, cube, _voxels(grid))
    assert rel_err(img, ref) < TOL


@pytest.mark.parametrize("engine", ENGINES)
def test_pipeline_end_to_end(gpu, orc, engine):
    """Trace, synthesis and imaging on both sides from the same scene inputs."""
    array = sg.array_square(n_side=4, pitch=3e-3)
    chirp = sg.chirp_sfcw(72e9, 82e9, 64)
    scene = sg.scene_hand_proxy(2, step=6e-3)
    tp = sg.TraceParams(n_rays=30_000, max_bounces=2, seed=4, az_min=-0.4, az_max=0.4,
                        el_min=-0.4, el_max=0.4)
    w = sg.Workload("img", scene, array, chirp, tp)
    gpu.setup(w)
    gpu.trace_workload(w, record_hits=False)
    cube = gpu.synthesize(model=0, engine=1)
    grid = ((0.29, -0.02, -0.02), 5e-3, (5, 9, 9))
    img = gpu.backproject(cube, grid, engine=engine).cpu().numpy().reshape(-1)
    _, op = orc.trace(scene, array, tp, want_hits=False)
    ocube = orc.synth(op, scene, array, chirp, model=0)
    ref = orc.backproject(array, chirp.f0, chirp.bandwidth / chirp.n_samples, ocube,
                          _voxels(grid))
    assert rel_err(img, ref) < TOL


@pytest.mark.parametrize("engine", ENGINES)
def test_full_size_grid_sampled_and_focus(gpu, orc, engine):
    array = sg.array_square()                      # 94 Tx x 94 Rx
    chirp = sg.chirp_sfcw()                        # 72-82 GHz, 128 steps
    pts = np.array([[0.300, 0.012, -0.021], [0.285, -0.040, 0.050], [0.321, 0.070, 0.003]])
    scene = sg.point_only(pts, aperture=[0.01, 0.006, 0.004])
    _, op = orc.trace(scene, array, sg.TraceParams(n_rays=0, max_bounces=1))
    assert len(op) == 3
    cube = orc.synth(op, scene, array, chirp, model=0)
    _setup(gpu, scene, array, chirp)
    grid = sg.imaging_grid()                       # 81 x 201 x 201 voxels, 1 mm
    img = gpu.backproject(_upload(cube), grid, engine=engine)
    (x0, y0, z0), st, (nx, ny, nz) = grid
    assert img.shape == (nx, ny, nz)
    vox = _voxels(grid)
    rng = np.random.default_rng(3)
    near = [int(round((p[0] - x0) / st)) * ny * nz + int(round((p[1] - y0) / st)) * nz
            + int(round((p[2] - z0) / st)) for p in pts]
    sel = np.concatenate([near, rng.choice(vox.shape[0], 21, replace=False)])
    got = img.reshape(-1)[torch.from_numpy(sel).cuda()].cpu().numpy()
    ref = orc.backproject(array, chirp.f0, chirp.bandwidth / chirp.n_samples, cube, vox[sel])
    assert np.abs(got - ref).max() <= TOL * np.abs(ref).max()
    # the brightest voxel is the voxel of the strongest reflector
    peak = int(torch.argmax(img.abs().reshape(-1)).item())
    assert peak == near[0]


@pytest.mark.parametrize("n_tx,n_rx,K", [(96, 96, 5), (1, 1, 130), (37, 70, 17)])
def test_mfma_limits_and_ragged(gpu, orc, n_tx, n_rx, K):
    """Array sizes at and below the 96 x 96 limit, one channel, odd step
    counts, a voxel count that leaves a partial workgroup; both engines
    against the oracle; beyond the limits the product engine is refused and
    AUTO falls back to Horner."""
    import paper_2307_15412_amd as rr
    rng = np.random.default_rng(n_tx * 1000 + n_rx)
    tx = np.stack([np.zeros(n_tx), rng.uniform(-0.07, 0.07, n_tx), rng.uniform(-0.07, 0.07, n_tx)], 1)
    rx = np.stack([np.zeros(n_rx), rng.uniform(-0.07, 0.07, n_rx), rng.uniform(-0.07, 0.07, n_rx)], 1)
    array = sg.Array(tx, rx, 0.07, sg.MODE_SHARED)
    chirp = sg.chirp_sfcw(72e9, 82e9, K)
    scene = sg.point_only([[0.30, 0.01, -0.02], [0.32, -0.03, 0.04]], aperture=[0.01, 0.005])
    _, op = orc.trace(scene, array, sg.TraceParams(n_rays=0, max_bounces=1))
    cube = orc.synth(op, scene, array, chirp, model=0)
    _setup(gpu, scene, array, chirp)
    grid = ((0.29, -0.03, -0.04), 3e-3, (5, 7, 9))          # 315 voxels
    ref = orc.backproject(array, chirp.f0, chirp.bandwidth / chirp.n_samples, cube, _voxels(grid))
    for engine in ENGINES:
        img = gpu.backproject(_upload(cube), grid, engine=engine).cpu().numpy().reshape(-1)
        assert np.abs(img - ref).max() <= TOL * np.abs(ref).max(), engine
    if n_tx == 96:
        big = sg.Array(np.concatenate([tx, tx[:1] + [0.0, 0.0, 0.001]]), rx, 0.07, sg.MODE_SHARED)
        _setup(gpu, scene, big, chirp)
        c2 = torch.zeros((97 * n_rx, 1, K), dtype=torch.complex64, device="cuda")
        with pytest.raises(rr.RadrayError) as e:
            gpu.backproject(c2, grid, engine=rr.GEMM_EXACT)
        assert e.value.code == rr.binding.RR_EUNSUPPORTED
        gpu.backproject(c2, grid)                            # AUTO: Horner


def test_max_projection_db(gpu, orc):
    array = sg.array_square(n_side=5, pitch=3e-3)
    chirp = sg.chirp_sfcw(72e9, 82e9, 32)
    scene = sg.point_only([[0.30, 0.0, 0.01], [0.31, -0.02, -0.015]], aperture=[0.01, 0.003])
    _, op = orc.trace(scene, array, sg.TraceParams(n_rays=0, max_bounces=1))
    cube = orc.synth(op, scene, array, chirp, model=0)
    grid = ((0.28, -0.04, -0.04), 4e-3, (11, 21, 21))
    ref = orc.backproject(array, chirp.f0, chirp.bandwidth / chirp.n_samples, cube,
                          _voxels(grid)).reshape(11, 21, 21)
    _setup(gpu, scene, array, chirp)
    proj = gpu.max_projection(_upload(ref), grid, floor_db=-15.0).cpu().numpy()
    m = np.abs(ref).max(axis=0)
    want = np.maximum(20 * np.log10(m / m.max()), -15.0)
    assert np.abs(proj - want).max() < 1e-3
    assert proj.max() == 0.0 and proj.min() >= -15.0


def test_far_volume_falls_back(gpu, orc):
    """A volume whose phases exceed the matrix engine's FP32 range (metres
    away at 80 GHz): AUTO uses the Horner engine and matches the oracle, the
    matrix engine is refused."""
    import paper_2307_15412_amd as rr
    array = sg.array_square(n_side=4, pitch=3e-3)
    chirp = sg.chirp_sfcw(72e9, 82e9, 16)
    scene = sg.point_only([[2.0, 0.01, 0.0]], aperture=[0.05])
    _, op = orc.trace(scene, array, sg.TraceParams(n_rays=0, max_bounces=1))
    cube = orc.synth(op, scene, array, chirp, model=0)
    _setup(gpu, scene, array, chirp)
    grid = ((1.99, -0.01, -0.01), 5e-3, (3, 5, 5))
    with pytest.raises(rr.RadrayError) as e:
        gpu.backproject(_upload(cube), grid, engine=rr.GEMM_EXACT)
    assert e.value.code == rr.binding.RR_EUNSUPPORTED
    img = gpu.backproject(_upload(cube), grid).cpu().numpy().reshape(-1)
    ref = orc.backproject(array, chirp.f0, chirp.bandwidth / chirp.n_samples, cube, _voxels(grid))
    assert np.abs(img - ref).max() <= TOL * np.abs(ref).max()
