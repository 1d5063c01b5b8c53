"""GPU synthesis parity with the FP64 oracle (Eq. 4 with the FMCW
instantaneous frequency): direct FP32 engine within 1e-4 relative (Frobenius)
of the oracle cube, FP64 sampled-entry kernel within 1e-6."""
import numpy as np
import pytest
import torch

import scenegen as sg
from helpers import oracle_to_soa, rel_err

pytestmark = pytest.mark.gpu

TOL_DIRECT = 1e-4
TOL_SAMPLED = 1e-6


def _upload_oracle_paths(gpu, op):
    soa = oracle_to_soa(op)
    gpu.set_paths({k: torch.from_numpy(np.ascontiguousarray(v)) for k, v in soa.items()})


@pytest.mark.parametrize("model", [0, 1])
def test_tiny_full_cube(gpu, orc, model):
    w = sg.workload_tiny()
    gpu.setup(w)
    gpu.trace_workload(w)
    cube = gpu.synthesize(model=model, engine=1).cpu().numpy()
    _, op = orc.trace(w.scene, w.array, w.trace)
    ref = orc.synth(op, w.scene, w.array, w.chirp, model=model)
    assert cube.shape == ref.shape
    assert rel_err(cube, ref) < TOL_DIRECT
    idx = np.random.default_rng(1).choice(ref.size, 512, replace=False)
    s = gpu.synthesize(model=model, engine=1, sample_idx=idx).cpu().numpy()
    assert rel_err(s, ref.reshape(-1)[idx]) < TOL_SAMPLED


def test_ragged_sample_counts(gpu, orc):
    """Sample counts that are not multiples of the per-lane run (ragged
    rows), single-sample and single-chirp cubes, empty path list."""
    w = sg.workload_tiny()
    w.trace.n_rays = 20_000
    _, op = orc.trace(w.scene, w.array, w.trace)
    gpu.setup(w)
    for K, M in ((50, 3), (1, 1), (7, 5), (96, 2)):
        ch = sg.Chirp(n_samples=K, n_chirps=M)
        gpu.set_chirp(ch.f0, ch.bandwidth, ch.t_chirp, ch.t_rep, K, M)
        _upload_oracle_paths(gpu, op)
        cube = gpu.synthesize(model=0, engine=1).cpu().numpy()
        ref = orc.synth(op, w.scene, w.array, ch)
        assert rel_err(cube, ref) < TOL_DIRECT, (K, M)
    _upload_oracle_paths(gpu, op[:0])
    cube = gpu.synthesize(model=0, engine=1)
    assert torch.count_nonzero(cube).item() == 0


def test_point_reflector_closed_form(gpu):
    """Monostatic point at R moving at v: the cube is a exp(-j 2 pi f_k 2 (R +
    v m T) / c) (closed form, no oracle)."""
    ch = sg.Chirp(n_samples=256, n_chirps=64)
    R, v = 23.4, -7.1
    sc = sg.point_only([[R, 0, 0.5]], vel=[[v, 0, 0]], aperture=0.01)
    w = sg.Workload("pt", sc, sg.Array(np.array([[0, 0, 0.5]]), np.array([[0, 0, 0.5]])), ch,
                    sg.TraceParams(n_rays=10))
    gpu.setup(w)
    assert gpu.trace_workload(w) == 1
    amp = gpu.paths()["amp"].cpu().numpy()[0]
    cube = gpu.synthesize(model=0, engine=1).cpu().numpy()[0]
    m = np.arange(64)[:, None]
    k = np.arange(256)[None, :]
    fk = ch.f0 + ch.bandwidth * k / 256
    ref = amp * np.exp(-2j * np.pi * fk * 2 * (R + v * m * ch.t_rep) / sg.C0)
    assert rel_err(cube, ref) < TOL_DIRECT


def test_street_cube_sampled(gpu, orc):
    """Street (192 channels, 128 x 256) from 1.2e5 rays: full GPU cube against
    4096 seeded oracle entries computed from the oracle's own paths."""
    w = sg.workload_street(0, n_rays=120_000)
    gpu.setup(w)
    gpu.trace_workload(w, record_hits=False)
    cube = gpu.synthesize(model=0, engine=1).cpu().numpy().reshape(-1)
    _, op = orc.trace(w.scene, w.array, w.trace, want_hits=False)
    idx = np.random.default_rng(7).choice(cube.size, 4096, replace=False)
    ref = orc.synth(op, w.scene, w.array, w.chirp, model=0, idx=idx)
    assert rel_err(cube[idx], ref) < TOL_DIRECT


@pytest.mark.parametrize("model", [0, 1])
def test_large_mimo_shape_sampled(gpu, orc, model):
    """3072 channels x 256 chirps x 512 samples (the large-MIMO cube, 3.2 GB)
    from oracle paths of a shared launch on the street: sampled entries."""
    w = sg.workload_large_mimo(0)
    w.trace.n_rays = 150_000
    _, op = orc.trace(w.scene, w.array, w.trace, want_hits=False)
    assert len(op) > 50
    gpu.setup(w)
    _upload_oracle_paths(gpu, op)
    cube = gpu.synthesize(model=model, engine=1)
    idx = np.random.default_rng(3).choice(cube.numel(), 1024, replace=False)
    got = cube.reshape(-1)[torch.from_numpy(idx).to(cube.device)].cpu().numpy()
    del cube
    ref = orc.synth(op, w.scene, w.array, w.chirp, model=model, idx=idx)
    assert rel_err(got, ref) < TOL_DIRECT
