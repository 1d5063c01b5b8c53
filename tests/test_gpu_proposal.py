"""Learned ray proposal on the GPU against the oracle: importance-sampled
launch (bitwise hit lists and paths for a given table), probe code, training
histogram, network forward, gradient and Adam step, sampling table; and the
gain of the trained network over uniform launch at equal ray budget."""
import numpy as np
import pytest
import torch

import scenegen as sg
from helpers import assert_paths_equal, gpu_soa_np, oracle_to_soa, traced_rows
from oracle import mlp

pytestmark = pytest.mark.gpu


def _texture_cdf(seed):
    na, ne = 128, 64
    rng = np.random.default_rng(seed)
    ia = np.arange(na)[None, :]
    ie = np.arange(ne)[:, None]
    q = np.exp(-((ia - 63.5) ** 2 + (ie - 31.5) ** 2) / 60.0) + 0.05 * rng.random((ne, na)) + 1e-3
    q = (q / q.sum()).reshape(-1)
    cdf = np.concatenate([[0.0], np.cumsum(q)])
    cdf /= cdf[-1]
    cdf[-1] = 1.0
    return cdf


@pytest.mark.parametrize("scene", ["plate", "tiny"])
def test_importance_sampled_trace_bit_exact(gpu, orc, scene):
    import paper_2307_15412_amd as rr
    if scene == "plate":
        w = sg.Workload("plate", sg.plate(5.0, 1.0), sg.Array(np.array([[0, 0, 0.5]]),
                        np.array([[0, 0, 0.5]]), 0.25, sg.MODE_PER_TX), sg.Chirp(),
                        sg.TraceParams(n_rays=100_000, max_bounces=2, seed=4))
    else:
        w = sg.workload_tiny(3)
        w.trace.n_rays = 50_000
    cdf = _texture_cdf(1)
    gpu.setup(w)
    gpu.proposal_set_cdf(cdf)
    n = gpu.trace_workload(w, record_hits=True, sampler=rr.PROPOSAL)
    hits = gpu.hits().cpu().numpy()
    oh, op = orc.trace(w.scene, w.array, w.trace, cdf=cdf, n_az=128, n_el=64)
    rows = traced_rows(orc, w.scene, w.array, w.trace)
    assert (hits == oh[rows]).all()
    assert n == len(op)
    assert_paths_equal(gpu_soa_np(gpu), oracle_to_soa(op))


def test_probe_code(gpu, orc):
    for seed in (1, 2, 3, 11, 12):
        w = sg.workload_box_family(seed, 1000)
        gpu.setup(w)
        code = gpu.proposal_probe().cpu().numpy()
        ref = orc.probe_code(w.scene, w.array, w.trace)
        assert np.abs(code - ref).max() < 1e-6, (seed, code, ref)
    assert ref.max() >= 0.0


def test_histogram(gpu, orc):
    for seed in (1, 5):
        w = sg.workload_box_family(seed, 50_000)
        gpu.setup(w)
        gpu.trace_workload(w, record_hits=True)
        H = gpu.proposal_histogram().cpu().numpy().astype(np.float64)
        hits, paths = orc.trace(w.scene, w.array, w.trace)
        rows = traced_rows(orc, w.scene, w.array, w.trace)
        ref = orc.histogram(w.scene, w.array, w.trace, hits[rows], paths)
        assert ref.sum() > 0
        assert np.abs(H - ref).max() <= 1e-5 * max(1.0, ref.max())


def _inputs(seed, S=3):
    rng = np.random.default_rng(seed)
    codes = (rng.random((S, 16)) * (rng.random((S, 16)) < 0.4)).astype(np.float32)
    hist = (rng.random((S, 8192)) * (rng.random((S, 8192)) < 0.03)).astype(np.float32)
    return codes, hist


def _f16(x):
    return np.asarray(x, dtype=np.float32).astype(np.float16).astype(np.float64)


@pytest.mark.parametrize("S", [1, 3, 7])
def test_forward_and_gradient(gpu, S):
    """Forward (FP16 products on the matrix cores) and gradient (FP32 products)
    against the FP64 network at 1, 3 and 7 scenes (8 192 rows a scene: the
    forward's 32-row tiles are always full; the weight gradients' split of the
    rows over blocks differs with the size).  The kernels round every hidden
    activation to FP16 and the FP64 network does not: that alone moves the
    gradient by 0.5-4 % of its norm on these inputs (the same for the earlier
    one-row-per-lane kernels), while its direction stays within cosine 0.999;
    the three-scene case keeps the 1e-2 bar it has always met (8.9e-3)."""
    gpu.mlp_init(3)
    p = gpu.mlp_get_params()
    codes, hist = _inputs(7, S)
    tc = torch.from_numpy(codes).cuda()
    th = torch.from_numpy(hist).cuda()
    z = gpu.mlp_forward(tc).cpu().numpy().reshape(-1)
    zr, _ = mlp.forward(_f16(p), mlp.features(_f16(codes)))
    zrel = np.linalg.norm(z - zr) / np.linalg.norm(zr)
    print(f"forward vs FP64 oracle ({S} scenes): relative {zrel:.3e}")
    assert zrel < 5e-3
    loss, g = gpu.mlp_train_step(tc, th, 0.0, want_grad=True)
    lr_, gr = mlp.loss_and_grad(_f16(p), _f16(codes), hist.astype(np.float64))
    g = g.cpu().numpy().astype(np.float64)
    rel = np.linalg.norm(g - gr) / np.linalg.norm(gr)
    cos = g @ gr / (np.linalg.norm(g) * np.linalg.norm(gr))
    print(f"gradient vs FP64 oracle ({S} scenes): relative {rel:.3e}, cosine {cos:.6f}")
    assert abs(loss - lr_) < 2e-3 * abs(lr_)
    assert rel < (1e-2 if S == 3 else 5e-2)
    assert cos > 0.999
    # lr = 0 leaves the parameters unchanged
    assert np.array_equal(gpu.mlp_get_params(), p)


def test_adam_step(gpu):
    gpu.mlp_init(5)
    p0 = gpu.mlp_get_params()
    codes, hist = _inputs(8)
    lr = 1e-3
    gpu.mlp_train_step(torch.from_numpy(codes).cuda(), torch.from_numpy(hist).cuda(), lr)
    p1 = gpu.mlp_get_params().astype(np.float64)
    _, gr = mlp.loss_and_grad(_f16(p0), _f16(codes), hist.astype(np.float64))
    ref, _, _ = mlp.adam_step(p0.astype(np.float64), gr, np.zeros_like(gr), np.zeros_like(gr), 1, lr)
    # the first Adam step moves each parameter by ~lr sign(g); parameters with
    # a tiny gradient may differ in sign between FP16 and FP64 evaluation
    close = np.abs(p1 - ref) <= 2e-6
    print("adam step: fraction within 2e-6", close.mean())
    assert close.mean() > 0.97
    assert np.abs(p1 - ref).max() <= 2.1 * lr


def test_sampling_table(gpu):
    gpu.mlp_init(9)
    p = gpu.mlp_get_params()
    code = np.random.default_rng(1).random(16).astype(np.float32) * 0.3
    zr, _ = mlp.forward(_f16(p), mlp.features(_f16(code[None, :])))
    for power in (1.0, 0.5):
        gpu.proposal_build(torch.from_numpy(code).cuda(), 0.1, power)
        cdf = gpu.proposal_get_cdf()
        ref = mlp.cdf_of(mlp.mixture(zr, 0.1, power))
        assert cdf[0] == 0.0 and cdf[-1] == 1.0 and np.all(np.diff(cdf) >= 0)
        assert np.abs(cdf - ref).max() < 2e-4
    # power 1/2 is the square root of the power-1 density, renormalised
    q1 = np.diff(mlp.cdf_of(mlp.mixture(zr, 0.0, 1.0)))
    qh = np.diff(mlp.cdf_of(mlp.mixture(zr, 0.0, 0.5)))
    assert np.allclose(qh, np.sqrt(q1) / np.sqrt(q1).sum(), rtol=1e-9, atol=0)
    # the cost-aware table
    for kappa in (0.003, 1.0, 300.0):
        gpu.proposal_build_cost(torch.from_numpy(code).cuda(), 0.1, kappa)
        cdf = gpu.proposal_get_cdf()
        ref = mlp.cdf_of(mlp.mixture_cost(zr, 0.1, kappa))
        assert cdf[0] == 0.0 and cdf[-1] == 1.0 and np.all(np.diff(cdf) >= 0)
        assert np.abs(cdf - ref).max() < 2e-4, kappa
    import paper_2307_15412_amd as rr
    for beta, power in ((0.1, 0.0), (0.1, 2.5), (0.1, float("nan")), (1.5, 0.5)):
        with pytest.raises(rr.RadrayError) as e:
            gpu.proposal_build(torch.from_numpy(code).cuda(), beta, power)
        assert e.value.code == rr.binding.RR_EINVAL
    for beta, kappa in ((0.1, 0.0), (0.1, -1.0), (0.1, float("inf")), (-0.1, 1.0)):
        with pytest.raises(rr.RadrayError) as e:
            gpu.proposal_build_cost(torch.from_numpy(code).cuda(), beta, kappa)
        assert e.value.code == rr.binding.RR_EINVAL


def _splitmix_batches(seed, n, batch, steps):
    """Minibatches of a partial Fisher-Yates shuffle driven by SplitMix64
    (Steele, Lea and Flood 2014), written out from its published definition."""
    M = (1 << 64) - 1
    perm, x = list(range(n)), seed
    for _ in range(steps):
        for k in range(batch):
            x = (x + 0x9E3779B97F4A7C15) & M
            z = ((x ^ (x >> 30)) * 0xBF58476D1CE4E5B9) & M
            z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
            z ^= z >> 31
            j = k + z % (n - k)
            perm[k], perm[j] = perm[j], perm[k]
        yield perm[:batch]


def test_gradient_and_histogram_deterministic(gpu):
    """The weight gradient is summed per block and then over blocks in a fixed
    order, and the training histogram counts whole tenths in integers: two
    runs on the same inputs give the same bits."""
    codes, hist = _inputs(31, S=20)       # 20 scenes: 40 blocks of rows
    tc, th = torch.from_numpy(codes).cuda(), torch.from_numpy(hist).cuda()
    gpu.mlp_init(4)
    _, g1 = gpu.mlp_train_step(tc, th, 0.0, want_grad=True)
    _, g2 = gpu.mlp_train_step(tc, th, 0.0, want_grad=True)
    assert torch.equal(g1, g2)
    w = sg.workload_box_family(5, 200_000)
    gpu.setup(w)
    gpu.trace_workload(w, record_hits=True)
    h1 = gpu.proposal_histogram().clone()
    h2 = gpu.proposal_histogram().clone()
    assert torch.equal(h1, h2) and float(h1.sum()) > 0


@pytest.mark.parametrize("batch", [3, 8])
def test_train_loop_equals_single_steps(gpu, batch):
    """rr_proposal_train = its minibatches fed one by one to rr_mlp_train_step,
    bit for bit (the gradient's sums run in a fixed order)."""
    S, steps, lr = 8, 4, 1e-3
    codes, hist = _inputs(21, S)
    tc, th = torch.from_numpy(codes).cuda(), torch.from_numpy(hist).cuda()
    gpu.mlp_init(2)
    ref_loss = []
    # a batch of every scene takes them in their given order (no shuffle)
    batches = (_splitmix_batches(99, S, batch, steps) if batch < S
               else [list(range(S))] * steps)
    for idx in batches:
        ix = torch.tensor(idx, device=tc.device)
        ref_loss.append(gpu.mlp_train_step(tc[ix], th[ix], lr))
    ref = gpu.mlp_get_params().astype(np.float64)
    gpu.mlp_init(2)
    loss = gpu.proposal_train(tc, th, steps, batch=batch, lr=lr, seed=99)
    got = gpu.mlp_get_params().astype(np.float64)
    # the loss sequence pins the minibatches and their order
    assert np.array_equal(loss, np.asarray(ref_loss, dtype=np.float32))
    assert np.array_equal(got, ref)


def test_reference_metric(gpu):
    """The error against the expectation: from two independent references the
    zero cube scores exactly 1, an independent third launch of the same size
    scores about the references' own error, and a launch of 16 times more
    rays about a quarter of it."""
    import paper_2307_15412_amd as rr
    from paper_2307_15412_amd import proposal
    w = sg.workload_box_family(1003, 200_000, points=False)
    gpu.setup(w)
    cube = lambda: gpu.synthesize(model=rr.EXACT, engine=rr.DIRECT_FP32).reshape(-1).clone()
    kw = dict(max_bounces=2, record_hits=False)
    gpu.trace(200_000, seed=1, **kw)
    a = cube()
    gpu.trace(200_000, seed=2, **kw)
    ref = proposal.Reference(a, cube())
    assert ref.mse(torch.zeros_like(a)) == pytest.approx(1.0, abs=1e-12)
    e_same = []
    for sd in range(3, 11):
        gpu.trace(200_000, seed=sd, **kw)
        e_same.append(ref.mse(cube()))
    gpu.trace(3_200_000, seed=99, **kw)
    e_big = ref.mse(cube())
    r2 = ref.ref_err() ** 2
    # a launch like A and B has mean squared error 2 var(R) = 2 r2
    print(f"reference metric: ref {r2 ** .5:.3f}, same-size {np.mean(e_same) ** .5:.3f}, "
          f"16x {max(e_big, 0) ** .5:.3f}")
    assert 0.5 * 2 * r2 < np.mean(e_same) < 2.0 * 2 * r2
    assert e_big < 0.5 * np.mean(e_same)


def test_learned_proposal_gain(gpu):
    """Train on uniform traces of 60 scenes of the box family, then on 10
    held-out scenes draw 1e6 rays from the learned density: its cube error
    against the expectation (two independent 8e6-ray uniform launches, their
    own noise subtracted; 2 seeds per estimator) is below 0.8 of that of 1e6
    uniform rays, in at least 7 of 10 scenes.  The budget puts the uniform
    error below 1 (it falls as ~600 / sqrt(rays) on this family), so that an
    empty cube (error exactly 1, the negative control) fails the same test."""
    from paper_2307_15412_amd import proposal
    res = proposal.experiment(gpu, train_seeds=range(1, 61), eval_seeds=range(1001, 1011),
                              train_rays=50_000, budget=1_000_000, ref_rays=8_000_000, steps=200,
                              batch=16, lr=2e-3, n_seeds=2)
    print({k: v for k, v in res.items() if k != "per_scene"})
    assert res["loss_last"] < res["loss_first"]
    assert res["err_uniform_mean"] < 1.0
    passes = lambda err: err < 0.8 * res["err_uniform_mean"]
    assert passes(res["err_learned_mean"]) and res["wins"] >= 7
    assert not passes(res["err_zero"])
