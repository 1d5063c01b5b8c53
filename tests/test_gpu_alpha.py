"""Material mix per face and alpha sweeps (Eq. 3; the paper sweeps alpha from
0 to 1 by 0.1 and suggests per-face variation for data diversity): hit lists
and path records bitwise equal to the FP64 oracle for per-face alpha on the
tiny scene and on the hand proxy, for every value of the sweep set without
re-uploading the scene, and for per-slot sweeps in the batched launch (each
slot = the single-scene launch of the scene at that alpha); invalid calls are
rejected."""
import math

import numpy as np
import pytest
import torch

import scenegen as sg
from helpers import assert_paths_equal, gpu_soa_np, oracle_to_soa, traced_rows

pytestmark = pytest.mark.gpu


def _compare(gpu, orc, w, upload=True):
    if upload:
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
    return n


def _hand(n_rays=20_000, step=4e-3):
    deg = math.pi / 180
    return sg.Workload("hand_small", sg.scene_hand_proxy(3, step=step),
                       sg.array_square(n_side=6, pitch=3e-3, rx_radius=0.07), sg.chirp_sfcw(),
                       sg.TraceParams(n_rays=n_rays, max_bounces=2, seed=9, az_min=-25 * deg,
                                      az_max=25 * deg, el_min=-25 * deg, el_max=25 * deg))


def test_per_face_alpha_bitwise(gpu, orc):
    w = sg.workload_tiny(2)
    w.trace.n_rays = 40_000
    w.scene = sg.vary_alpha(w.scene, seed=1, spread=0.5)
    assert _compare(gpu, orc, w) > 100
    h = _hand()
    h.scene = sg.vary_alpha(h.scene, seed=2, spread=0.3)
    assert _compare(gpu, orc, h) > 20


def test_sweep_without_reupload(gpu, orc):
    """The paper's sweep alpha = 0, 0.1, ..., 1 on one uploaded hand mesh,
    then a per-face override, then back to per-object values."""
    import paper_2307_15412_amd as rr
    w = _hand()
    gpu.setup(w)
    counts = []
    for a in sg.alpha_sweep():
        gpu.set_alpha([a])
        ws = sg.Workload(w.name, sg.with_alpha(w.scene, a), w.array, w.chirp, w.trace)
        counts.append(_compare(gpu, orc, ws, upload=False))
    assert len(set(counts)) > 1
    var = sg.vary_alpha(sg.with_alpha(w.scene, 0.5), seed=7, spread=0.5)
    gpu.set_alpha(var.tri_alpha, per=rr.ALPHA_PER_TRIANGLE)
    _compare(gpu, orc, sg.Workload(w.name, var, w.array, w.chirp, w.trace), upload=False)
    gpu.set_alpha([0.25])
    _compare(gpu, orc, sg.Workload(w.name, sg.with_alpha(w.scene, 0.25), w.array, w.chirp,
                                   w.trace), upload=False)


def test_batch_sweep_slots(gpu):
    """Eleven slots of one street, each set to one alpha of the sweep after
    upload; every slot = the single-scene launch at that alpha, bitwise."""
    import paper_2307_15412_amd as rr
    base = sg.Workload("street_small", sg.scene_street(2, scale=0.05, n_cars=5, n_poles=6),
                       sg.array_ula(2, 4), sg.Chirp(n_samples=64, n_chirps=16),
                       sg.TraceParams(n_rays=60_000, max_bounces=3, seed=4))
    vals = sg.alpha_sweep()
    B = rr.Batch(gpu, len(vals))
    for i, a in enumerate(vals):
        B.set_workload(i, base)
        B.set_alpha(i, [a] * base.scene.n_obj)
    cubes = B.alloc_cubes()
    counts = B.launch(cubes)
    for i, a in enumerate(vals):
        w = sg.Workload(base.name, sg.with_alpha(base.scene, a), base.array, base.chirp, base.trace)
        gpu.setup(w)
        n = gpu.trace_workload(w, record_hits=False)
        ref = gpu.synthesize(model=rr.EXACT, engine=rr.DIRECT_FP32)
        assert counts[i] == n, (a, counts[i], n)
        assert torch.equal(cubes[i], ref), a
    assert len(set(counts.tolist())) > 1
    # a changed alpha is seen by the next replay of the captured launch
    B.set_alpha(0, [1.0] * base.scene.n_obj)
    counts2 = B.launch(cubes)
    assert counts2[0] == counts[-1]
    B.close()


def test_alpha_errors(gpu):
    import paper_2307_15412_amd as rr
    w = sg.workload_tiny()
    gpu.setup(w)
    for args in (([0.5] * (w.scene.n_obj + 1), rr.ALPHA_PER_OBJECT),
                 ([0.5] * (w.scene.n_tris - 1), rr.ALPHA_PER_TRIANGLE),
                 ([1.5] * w.scene.n_obj, rr.ALPHA_PER_OBJECT),
                 ([float("nan")] * w.scene.n_obj, rr.ALPHA_PER_OBJECT),
                 ([0.5] * w.scene.n_obj, 7)):
        with pytest.raises(rr.RadrayError) as e:
            gpu.set_alpha(*args)
        assert e.value.code == rr.binding.RR_EINVAL
