"""Exact-model synthesis as split-bf16 complex products on the matrix cores
(per (chirp, sample) over Tx x Rx tiles, or per (channel, chirp) over the
samples split k = k1 S + k2) against the FP64 oracle.  ENGINE_AUTO sends the
exact model here, so the engine is held to the exact model's FP32 bar
(relative error <= 1e-4, the direct engine's), not the split-bf16 GEMM's
1e-3; it measures ~5e-7: full cubes at Tx / Rx counts around the 16- and
32-row blocks and the 16-, 32-, 48-, 64- and 96-wide tiles, the sample split
at 1 to 1024 samples (ragged S), several chirps of a moving scene, the
per-element launch (paths feed only their own Tx; the sample split reads only
each transmitter's path group), path counts around the
path steps and the split boundaries, an empty path list; the hand set-up
and the full-size street (per-element) against the direct FP32 engine and
sampled oracle entries; invalid requests refused."""
import math

import numpy as np
import pytest
import torch

import scenegen as sg
from helpers import oracle_to_soa, rel_err

pytestmark = pytest.mark.gpu

TOL = 1e-4


def _upload(gpu, op):
    soa = oracle_to_soa(op)
    gpu.set_paths({k: torch.from_numpy(np.ascontiguousarray(v)) for k, v in soa.items()})


def _exact(gpu):
    import paper_2307_15412_amd as rr
    return gpu.synthesize(model=rr.EXACT, engine=rr.GEMM_EXACT).cpu().numpy()


@pytest.mark.parametrize("n_tx,n_rx,K,M", [(3, 7, 32, 2), (33, 97, 16, 1), (96, 96, 8, 1),
                                           (97, 5, 12, 3), (1, 1, 40, 1), (5, 9, 13, 2),
                                           (2, 3, 3, 1), (55, 55, 16, 2), (100, 190, 8, 1),
                                           (190, 95, 8, 1), (15, 15, 24, 2), (42, 42, 8, 1),
                                           (17, 50, 9, 1), (47, 40, 5, 2), (6, 7, 512, 1),
                                           (4, 5, 1024, 1), (8, 9, 300, 2), (3, 4, 257, 1)])
def test_tile_edges(gpu, orc, n_tx, n_rx, K, M):
    w = sg.workload_tiny(1)
    w.array = sg.array_sparse_grid(n_tx, n_rx, 3, grid=128, mode=sg.MODE_SHARED)
    w.chirp = sg.Chirp(n_samples=K, n_chirps=M)
    w.trace.n_rays = 20_000
    _, op = orc.trace(w.scene, w.array, w.trace)
    op = op[:300]
    gpu.setup(w)
    _upload(gpu, op)
    got = _exact(gpu)
    ref = orc.synth(op, w.scene, w.array, w.chirp, model=0)
    assert got.shape == ref.shape
    assert rel_err(got, ref) < TOL


def test_moving_scene_chirps_and_per_element(gpu, orc):
    """The tiny scene's box moves at 5 m/s: every chirp has its own lengths;
    then a per-element launch (12 Tx) whose paths feed only their own Tx."""
    w = sg.workload_tiny(2)
    w.array = sg.array_sparse_grid(8, 12, 5, mode=sg.MODE_SHARED)
    w.chirp = sg.Chirp(n_samples=64, n_chirps=16)
    w.trace.n_rays = 30_000
    gpu.setup(w)
    gpu.trace_workload(w, record_hits=False)
    _, op = orc.trace(w.scene, w.array, w.trace)
    assert rel_err(_exact(gpu), orc.synth(op, w.scene, w.array, w.chirp, model=0)) < TOL
    w2 = sg.workload_tiny(3)
    w2.array = sg.array_ula(12, 8, mode=sg.MODE_PER_TX)
    w2.chirp = sg.Chirp(n_samples=32, n_chirps=4)
    w2.trace.n_rays = 36_000
    gpu.setup(w2)
    gpu.trace_workload(w2, record_hits=False)
    _, op2 = orc.trace(w2.scene, w2.array, w2.trace)
    assert rel_err(_exact(gpu), orc.synth(op2, w2.scene, w2.array, w2.chirp, model=0)) < TOL


@pytest.mark.parametrize("n_tx,n_rx,K", [(12, 16, 256), (5, 7, 512), (3, 4, 1000)])
def test_per_element_sample_split(gpu, orc, n_tx, n_rx, K):
    """Per-element launches on the sample split: each channel's wavefronts
    read only their transmitter's path group (widened to whole 32-path steps,
    the neighbours' paths masked by source); the whole cube against the
    direct FP32 engine and sampled entries against the FP64 oracle."""
    import paper_2307_15412_amd as rr
    w = sg.Workload("street_pe", sg.scene_street(4, scale=0.05, n_cars=5, n_poles=6),
                    sg.array_ula(n_tx, n_rx, mode=sg.MODE_PER_TX), sg.Chirp(n_samples=K, n_chirps=4),
                    sg.TraceParams(n_rays=120_000, max_bounces=3, seed=11))
    gpu.setup(w)
    n = gpu.trace_workload(w, record_hits=False)
    assert n > 100
    prod = gpu.synthesize(model=rr.EXACT, engine=rr.GEMM_EXACT).clone()
    direct = gpu.synthesize(model=rr.EXACT, engine=rr.DIRECT_FP32)
    assert rel_err(prod.cpu().numpy(), direct.cpu().numpy()) < TOL
    # AUTO takes the product engine here (the sample split models well above
    # 1.5x the direct engine) and so returns the same cube bit for bit
    auto = gpu.synthesize(model=rr.EXACT, engine=rr.ENGINE_AUTO)
    assert torch.equal(auto, prod)
    _, op = orc.trace(w.scene, w.array, w.trace, want_hits=False)
    idx = np.random.default_rng(K).choice(prod.numel(), 384, replace=False)
    ref = orc.synth(op, w.scene, w.array, w.chirp, model=0, idx=idx)
    got = prod.reshape(-1)[torch.from_numpy(idx).cuda()].cpu().numpy()
    assert rel_err(got, ref) < TOL


def test_street_full_size_per_element(gpu, orc):
    """The street configuration at full size, in the launch the benchmark
    times: 1e7 rays, 12 Tx x 16 Rx per-element launch, 128 chirps x 256
    samples, every path kept.  AUTO takes the product engine (the sample split
    over each transmitter's path group, one X word per path and chirp) and
    returns its cube bit for bit; the whole cube against the direct FP32
    engine, and 4096 seeded entries against the oracle's own trace of the
    same rays."""
    import paper_2307_15412_amd as rr
    w = sg.workload_street(0)
    gpu.setup(w)
    n = gpu.trace_workload(w, record_hits=False)
    prod = gpu.synthesize(model=rr.EXACT, engine=rr.GEMM_EXACT).clone()
    auto = gpu.synthesize(model=rr.EXACT, engine=rr.ENGINE_AUTO)
    assert torch.equal(auto, prod)
    del auto
    direct = gpu.synthesize(model=rr.EXACT, engine=rr.DIRECT_FP32)
    assert rel_err(prod.cpu().numpy(), direct.cpu().numpy()) < TOL
    del direct
    _, op = orc.trace(w.scene, w.array, w.trace, want_hits=False)
    assert len(op) == n
    idx = np.random.default_rng(23).choice(prod.numel(), 4096, replace=False)
    ref = orc.synth(op, w.scene, w.array, w.chirp, model=0, idx=idx)
    got = prod.reshape(-1)[torch.from_numpy(idx).cuda()].cpu().numpy()
    err = rel_err(got, ref)
    print(f"street full size: {n} paths, sampled error vs oracle {err:.2e}")
    assert err < TOL


@pytest.mark.parametrize("n_keep", [1, 15, 16, 17, 4097])
def test_ragged_paths(gpu, orc, n_keep):
    w = sg.workload_tiny(4)
    w.array = sg.array_sparse_grid(5, 9, 2, mode=sg.MODE_SHARED)
    w.chirp = sg.Chirp(n_samples=16, n_chirps=1)
    w.trace.n_rays = 200_000
    _, op = orc.trace(w.scene, w.array, w.trace, want_hits=False)
    assert len(op) >= n_keep
    op = op[:n_keep]
    gpu.setup(w)
    _upload(gpu, op)
    assert rel_err(_exact(gpu), orc.synth(op, w.scene, w.array, w.chirp, model=0)) < TOL


def test_empty_and_refused(gpu, orc):
    import paper_2307_15412_amd as rr
    w = sg.workload_tiny()
    w.array = sg.array_sparse_grid(4, 4, 1, mode=sg.MODE_SHARED)
    w.chirp = sg.Chirp(n_samples=16, n_chirps=2)
    _, op = orc.trace(w.scene, w.array, w.trace)
    gpu.setup(w)
    _upload(gpu, op[:0])
    assert torch.count_nonzero(gpu.synthesize(model=rr.EXACT, engine=rr.GEMM_EXACT)).item() == 0
    _upload(gpu, op)
    for kw in (dict(model=rr.SEPARABLE, engine=rr.GEMM_EXACT),
               dict(model=rr.EXACT, engine=rr.GEMM_EXACT, sample_idx=np.arange(4))):
        with pytest.raises(rr.RadrayError) as e:
            gpu.synthesize(**kw)
        assert e.value.code == rr.binding.RR_EUNSUPPORTED


def test_hand_against_direct_and_oracle(gpu, orc):
    """The paper's set-up: 94 x 94 array, 128 steps, 2e5 rays; the product
    engine against the direct FP32 engine on the whole cube and against the
    oracle on sampled entries; AUTO picks the product engine here."""
    import paper_2307_15412_amd as rr
    w = sg.workload_hand(0, n_rays=200_000)
    gpu.setup(w)
    n = gpu.trace_workload(w, record_hits=False)
    assert n > 1000
    prod = gpu.synthesize(model=rr.EXACT, engine=rr.GEMM_EXACT).clone()
    direct = gpu.synthesize(model=rr.EXACT, engine=rr.DIRECT_FP32)
    assert rel_err(prod.cpu().numpy(), direct.cpu().numpy()) < TOL
    auto = gpu.synthesize(model=rr.EXACT, engine=rr.ENGINE_AUTO)
    assert torch.equal(auto, prod)
    _, op = orc.trace(w.scene, w.array, w.trace, want_hits=False)
    idx = np.random.default_rng(2).choice(prod.numel(), 512, replace=False)
    ref = orc.synth(op, w.scene, w.array, w.chirp, model=0, idx=idx)
    got = prod.reshape(-1)[torch.from_numpy(idx).cuda()].cpu().numpy()
    assert rel_err(got, ref) < TOL
