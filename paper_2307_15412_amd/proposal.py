"""Training and evaluation of the learned ray proposal on top of the C ABI.

Orchestration only: probing, tracing, histograms, the network's forward,
backward and Adam steps and the sampling table all run in the library's HIP
kernels (include/radray.h, "Learned ray proposal").

Training data: for every training scene, the 16-value probe code and the
per-bin returned-power histogram of a uniform trace.  Evaluation: for held-out
scenes, the cube from a reduced ray budget drawn from the learned density
(mixed with the uniform density) against the cube from the same budget drawn
uniformly, both measured against a large uniform reference cube.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import binding as B


def collect(ctx, workloads):
    """Probe codes [S][16] and histograms [S][8192] (device tensors)."""
    torch = ctx.torch
    codes, hists = [], []
    for w in workloads:
        ctx.setup(w)
        tp = w.trace
        codes.append(ctx.proposal_probe(tp.az_min, tp.az_max))
        ctx.trace_workload(w, record_hits=True, sampler=B.UNIFORM)
        hists.append(ctx.proposal_histogram())
    return torch.stack(codes), torch.stack(hists)


def train(ctx, codes, hists, steps=300, batch=16, lr=1e-3, seed=0, log=None):
    """Adam on random minibatches of scenes; returns the loss history."""
    ctx.mlp_init(seed)
    rng = np.random.default_rng(seed)
    S = codes.shape[0]
    losses = []
    for it in range(steps):
        idx = rng.choice(S, size=min(batch, S), replace=False)
        ix = ctx.torch.as_tensor(idx, device=codes.device)
        loss = ctx.mlp_train_step(codes[ix], hists[ix], lr)
        losses.append(loss)
        if log and (it % 50 == 0 or it == steps - 1):
            log(f"step {it} loss {loss:.4f}")
    return losses


def _cube(ctx):
    return ctx.synthesize(model=B.EXACT, engine=B.DIRECT_FP32).reshape(-1)


def evaluate(ctx, workloads, budget, ref_rays, beta=0.1):
    """Per held-out scene: relative cube error of uniform and learned launches
    of `budget` rays against a `ref_rays` uniform cube, and their trace times."""
    out = []
    for w in workloads:
        ctx.setup(w)
        tp = w.trace
        kw = dict(max_bounces=tp.max_bounces, az_min=tp.az_min, az_max=tp.az_max,
                  el_min=tp.el_min, el_max=tp.el_max, record_hits=False)
        ctx.trace(ref_rays, seed=tp.seed + 7919, sampler=B.UNIFORM, **kw)
        ref = _cube(ctx).clone()
        nref = float(ref.abs().pow(2).sum().sqrt())
        ctx.trace(budget, seed=tp.seed, sampler=B.UNIFORM, **kw)
        t_u = ctx.kernel_ms(0)
        eu = float((_cube(ctx) - ref).abs().pow(2).sum().sqrt()) / max(nref, 1e-30)
        code = ctx.proposal_probe(tp.az_min, tp.az_max)
        ctx.proposal_build(code, beta)
        ctx.trace(budget, seed=tp.seed, sampler=B.PROPOSAL, **kw)
        t_l = ctx.kernel_ms(0)
        el = float((_cube(ctx) - ref).abs().pow(2).sum().sqrt()) / max(nref, 1e-30)
        out.append(dict(seed=tp.seed, err_uniform=eu, err_learned=el, ms_uniform=t_u, ms_learned=t_l))
    return out


def experiment(ctx, train_seeds, eval_seeds, train_rays=50_000, budget=12_500, ref_rays=100_000,
               steps=300, batch=16, lr=1e-3, beta=0.1, log=None):
    import scenegen as sg
    t0 = time.time()
    tw = [sg.workload_box_family(s, train_rays, points=False) for s in train_seeds]
    codes, hists = collect(ctx, tw)
    t1 = time.time()
    if log:
        log(f"collected {len(tw)} training scenes in {t1 - t0:.1f} s")
    losses = train(ctx, codes, hists, steps=steps, batch=batch, lr=lr, log=log)
    t2 = time.time()
    ew = [sg.workload_box_family(s, budget, points=False) for s in eval_seeds]
    res = evaluate(ctx, ew, budget, ref_rays, beta)
    if log:
        log(f"evaluated {len(res)} held-out scenes in {time.time() - t2:.1f} s")
    eu = np.array([r["err_uniform"] for r in res])
    el = np.array([r["err_learned"] for r in res])
    return dict(collect_s=t1 - t0, train_s=t2 - t1, loss_first=losses[0], loss_last=losses[-1],
                err_uniform_mean=float(eu.mean()), err_learned_mean=float(el.mean()),
                err_ratio_mean=float(np.mean(el / eu)), wins=int((el < eu).sum()),
                n_eval=len(res), per_scene=res)
