"""rr_trace_rays (caller-supplied rays) against the oracle: hit lists and
path records bitwise on random rays (tiny scene in both launch modes, the
street with its BVH), the launch's own rays reproducing rr_trace, a cube
synthesised from such paths, and malformed inputs refused before tracing."""
import math

import numpy as np
import pytest

import scenegen as sg
from helpers import assert_paths_equal, gpu_soa_np, oracle_to_soa, rel_err, traced_rows

pytestmark = pytest.mark.gpu


def _random_rays(array, n, seed):
    """Rays from near the elements into the forward half space, with
    unnormalised directions and random amplitudes; sources ascending."""
    rng = np.random.default_rng(seed)
    if array.mode == sg.MODE_SHARED:
        src = np.full(n, -1, dtype=np.int32)
        base = np.repeat(array.tx.mean(axis=0)[None, :], n, axis=0)
    else:
        src = np.sort(rng.integers(0, array.n_tx, n)).astype(np.int32)
        base = array.tx[src]
    orig = base + rng.normal(0.0, 0.05, (n, 3))
    d = rng.normal(0.0, 1.0, (n, 3))
    d[:, 0] = np.abs(d[:, 0]) + 0.2
    d *= rng.uniform(0.1, 10.0, (n, 1))
    amp = rng.uniform(0.5, 2.0, n) / n
    return orig, d, amp, src


@pytest.mark.parametrize("mode", [sg.MODE_PER_TX, sg.MODE_SHARED])
def test_random_rays_bit_exact(gpu, orc, mode):
    w = sg.workload_tiny(4)
    w.array = sg.array_ula(3, 4, mode=mode)
    o, d, a, s = _random_rays(w.array, 40_000, 7)
    gpu.setup(w)
    n = gpu.trace_rays(o, d, a, s, max_bounces=3, seed=21)
    hits = gpu.hits().cpu().numpy()
    oh, op = orc.trace_rays(w.scene, w.array, o, d, a, s, 3, 21)
    assert n == len(op) > 100
    assert np.array_equal(hits, oh)
    assert_paths_equal(gpu_soa_np(gpu), oracle_to_soa(op))


def test_street_random_rays_bit_exact(gpu, orc):
    w = sg.workload_street(3, n_rays=1)
    o, d, a, s = _random_rays(w.array, 20_000, 11)
    gpu.setup(w)
    gpu.trace_rays(o, d, a, s, max_bounces=3, seed=5)
    oh, op = orc.trace_rays(w.scene, w.array, o, d, a, s, 3, 5)
    assert np.array_equal(gpu.hits().cpu().numpy(), oh)
    assert_paths_equal(gpu_soa_np(gpu), oracle_to_soa(op))


@pytest.mark.parametrize("mode", [sg.MODE_PER_TX, sg.MODE_SHARED])
def test_launch_rays_reproduce_trace(gpu, orc, mode):
    """The launch's own rays (origins, directions, w / N_t, sources) given
    to rr_trace_rays give rr_trace's hit list and paths bit for bit."""
    w = sg.workload_tiny(5)
    w.array = sg.array_ula(2, 4, mode=mode)
    w.trace.n_rays = 6000
    w.trace.max_bounces = 3
    gpu.setup(w)
    gpu.trace_workload(w, record_hits=True)
    rows = traced_rows(orc, w.scene, w.array, w.trace)
    ref_hits = gpu.hits().cpu().numpy()
    ref = gpu_soa_np(gpu)
    per = orc.n_per_src(w.scene, w.array, w.trace)
    o, d, a, s = [], [], [], []
    for t in range(orc.n_src(w.array)):
        for i in range(per):
            v = orc.launch_dir(w.scene, w.array, w.trace, i, t)
            src = w.array.tx.mean(axis=0) if mode == sg.MODE_SHARED else w.array.tx[t]
            if mode == sg.MODE_SHARED:
                # the phase centre summed in element order, as the library does
                acc = [0.0, 0.0, 0.0]
                for e in w.array.tx:
                    for k in range(3):
                        acc[k] += float(e[k])
                src = np.array(acc) / w.array.n_tx
            o.append(src)
            d.append(v[:3])
            a.append(v[3] / per)
            s.append(-1 if mode == sg.MODE_SHARED else t)
    gpu.trace_rays(np.array(o), np.array(d), np.array(a), np.array(s, np.int32),
                   max_bounces=3, seed=w.trace.seed)
    assert np.array_equal(gpu.hits().cpu().numpy(), ref_hits)
    got = gpu_soa_np(gpu)
    # rr_trace numbers virtual rays per source including point reflectors
    pts = ref["K"].shape[0] - got["K"].shape[0]
    keep = np.isin(ref["ray"], np.asarray(rows)) if pts else np.ones(len(ref["ray"]), bool)
    ref = {k: (v[..., keep] if v.ndim == 2 else v[keep]) for k, v in ref.items()}
    vps = per + w.scene.n_pts
    ref["ray"] = (ref["ray"] // vps) * per + ref["ray"] % vps
    assert_paths_equal(got, ref)


def test_cube_from_caller_rays(gpu, orc):
    w = sg.workload_tiny(6)
    o, d, a, s = _random_rays(w.array, 30_000, 3)
    gpu.setup(w)
    gpu.trace_rays(o, d, a, s, max_bounces=2, seed=8, record_hits=False)
    cube = gpu.synthesize(model=0, engine=1).cpu().numpy()
    _, op = orc.trace_rays(w.scene, w.array, o, d, a, s, 2, 8, want_hits=False)
    assert rel_err(cube, orc.synth(op, w.scene, w.array, w.chirp, model=0)) < 1e-4


def test_malformed_rays_refused(gpu):
    import paper_2307_15412_amd as rr
    w = sg.workload_tiny()
    w.array = sg.array_ula(2, 2)
    gpu.setup(w)
    o = np.zeros((3, 3))
    d = np.array([[1.0, 0, 0]] * 3)
    a = np.ones(3)
    assert gpu.trace_rays(o, d, a, np.array([0, 0, 1], np.int32)) >= 0
    for src, dd, aa in [(np.array([1, 0, 1], np.int32), d, a),
                        (np.array([0, 0, 2], np.int32), d, a),
                        (np.array([0, 0, 1], np.int32), np.array([[1.0, 0, 0], [0, 0, 0], [1, 0, 0]]), a),
                        (np.array([0, 0, 1], np.int32), np.array([[1.0, 0, 0], [math.nan, 0, 0], [1, 0, 0]]), a),
                        (np.array([0, 0, 1], np.int32), d, np.array([1.0, math.inf, 1.0]))]:
        with pytest.raises(rr.RadrayError) as e:
            gpu.trace_rays(o, dd, aa, src)
        assert e.value.code == rr.binding.RR_EINVAL
    assert gpu.trace_rays(np.zeros((0, 3)), np.zeros((0, 3)), np.zeros(0), np.zeros(0, np.int32)) == 0
