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
    """Adam on random minibatches of scenes (drawn and run in the library);
    returns the loss history."""
    ctx.mlp_init(seed)
    losses = ctx.proposal_train(codes, hists, steps, batch=batch, lr=lr, seed=seed).tolist()
    if log and losses:
        log(f"{steps} steps: loss {losses[0]:.4f} -> {losses[-1]:.4f}")
    return losses


def _cube(ctx):
    return ctx.synthesize(model=B.EXACT, engine=B.DIRECT_FP32).reshape(-1)


def evaluate(ctx, workloads, budget, ref_rays, beta=0.1, power=0.5, alt_power=None):
    """Per held-out scene: relative cube error of uniform and learned launches
    of `budget` rays against a `ref_rays` uniform cube, and their trace times;
    the learned table with softmax power `power` (and, for comparison, with
    `alt_power`)."""
    out = []
    for w in workloads:
        ctx.setup(w)
        tp = w.trace
        kw = dict(max_bounces=tp.max_bounces, az_min=tp.az_min, az_max=tp.az_max,
                  el_min=tp.el_min, el_max=tp.el_max, record_hits=False)
        ctx.trace(ref_rays, seed=tp.seed + 7919, sampler=B.UNIFORM, **kw)
        ref = _cube(ctx).clone()
        nref = float(ref.abs().pow(2).sum().sqrt())
        p_u = ctx.trace(budget, seed=tp.seed, sampler=B.UNIFORM, **kw)
        t_u = ctx.kernel_ms(0)
        eu = float((_cube(ctx) - ref).abs().pow(2).sum().sqrt()) / max(nref, 1e-30)
        code = ctx.proposal_probe(tp.az_min, tp.az_max)
        alt = {}
        if alt_power is not None:
            ctx.proposal_build(code, beta, alt_power)
            p_a = ctx.trace(budget, seed=tp.seed, sampler=B.PROPOSAL, **kw)
            alt = dict(err_learned_alt=float((_cube(ctx) - ref).abs().pow(2).sum().sqrt())
                       / max(nref, 1e-30), paths_learned_alt=p_a)
        ctx.proposal_build(code, beta, power)
        p_l = ctx.trace(budget, seed=tp.seed, sampler=B.PROPOSAL, **kw)
        t_l = ctx.kernel_ms(0)
        el = float((_cube(ctx) - ref).abs().pow(2).sum().sqrt()) / max(nref, 1e-30)
        # per-triangle casting (the triangles in view) with at most the same
        # number of rays
        fov = (tp.az_min, tp.az_max, tp.el_min, tp.el_max)
        ctx.set_casting(0.0, 8)
        n_in = ctx.casting_pieces(*fov)
        g = int(math.isqrt(budget // max(n_in, 1)))
        rec = dict(seed=tp.seed, err_uniform=eu, err_learned=el, ms_uniform=t_u, ms_learned=t_l,
                   paths_uniform=p_u, paths_learned=p_l, **alt)
        if g >= 1:
            p_t = ctx.trace(g * g, seed=tp.seed, sampler=B.PER_TRIANGLE, **kw)
            # an empty cube scores exactly 1: read it with paths_tri
            rec.update(err_tri=float((_cube(ctx) - ref).abs().pow(2).sum().sqrt()) / max(nref, 1e-30),
                       ms_tri=ctx.kernel_ms(0), rays_tri=g * g * n_in, paths_tri=p_t)
        # the same with the triangles cut into pieces by solid angle (up to 16
        # levels: a piece of the 2e4 m^2 ground half a metre below the radar
        # needs about 13 to come down to the threshold), 4 rays per piece, the
        # threshold raised until the pieces fit the budget
        om_fov = (tp.az_max - tp.az_min) * (math.sin(tp.el_max) - math.sin(tp.el_min))
        om = om_fov * 4.0 / budget
        ctx.set_casting(om, 16)
        while ctx.casting_pieces(*fov) * 4 > budget:
            om *= 1.25
            ctx.set_casting(om, 16)
        n_pc = ctx.casting_pieces(*fov)
        p_c = ctx.trace(4, seed=tp.seed, sampler=B.PER_TRIANGLE, **kw)
        rec.update(err_cut=float((_cube(ctx) - ref).abs().pow(2).sum().sqrt()) / max(nref, 1e-30),
                   ms_cut=ctx.kernel_ms(0), rays_cut=4 * n_pc, paths_cut=p_c, omega_cut=om)
        ctx.set_casting(0.0, 8)
        out.append(rec)
    return out


def _rel(ctx, a, b, nb):
    return float((a - b).abs().pow(2).sum().sqrt()) / max(nb, 1e-30)


def _loglog(xs, ys, y):
    """x where the piecewise log-log line through (xs, ys) reaches y (ys
    decreasing); extrapolated from the end segments."""
    lx, ly, t = np.log(xs), np.log(ys), math.log(y)
    i = int(np.clip(np.searchsorted(-ly, -t) - 1, 0, len(xs) - 2))
    f = (t - ly[i]) / (ly[i + 1] - ly[i])
    return float(math.exp(lx[i] + f * (lx[i + 1] - lx[i])))


def equal_error(ctx, eval_seeds, budget=12_500, uniform_budgets=(12_500, 25_000, 50_000, 100_000,
                                                                   200_000),
                ref_rays=1_000_000, beta=0.1, power=0.5, log=None):
    """Wall time at equal cube error on the large-MIMO array (3072 channels,
    512 samples x 256 chirps) over box-family scenes, with the network as
    trained in `ctx`.

    Learned pipeline: probe code, sampling table, `budget` rays from the
    learned density, GEMM synthesis.  Plain pipeline: uniform rays and direct
    summation, at each of `uniform_budgets` (and, timed alongside, the same
    uniform rays with GEMM synthesis, which separates the proposal's share).  Both against a `ref_rays`
    uniform reference (GEMM); all cubes in the separable model.  The uniform
    budget of equal mean error is interpolated in log-log, and so is the
    plain pipeline's time there."""
    torch = ctx.torch
    import scenegen as sg
    per = []
    ref = work = None
    for s in eval_seeds:
        w = sg.workload_box_mimo(s, budget)
        ctx.setup(w)
        tp = w.trace
        C, M, K = w.array.n_ch, w.chirp.n_chirps, w.chirp.n_samples
        if ref is None:
            ref = torch.empty((C, M, K), dtype=torch.complex64, device=ctx.device)
            work = torch.empty_like(ref)
        kw = dict(max_bounces=tp.max_bounces, az_min=tp.az_min, az_max=tp.az_max,
                  el_min=tp.el_min, el_max=tp.el_max, record_hits=False)
        ctx.trace(ref_rays, seed=tp.seed + 7919, sampler=B.UNIFORM, **kw)
        ctx.synthesize(model=B.SEPARABLE, engine=B.GEMM_BF16X3, out=ref)
        nref = float(ref.abs().pow(2).sum().sqrt())
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        code = ctx.proposal_probe(tp.az_min, tp.az_max)
        ctx.proposal_build(code, beta, power)
        n_l = ctx.trace(budget, seed=tp.seed, sampler=B.PROPOSAL, **kw)
        ctx.synthesize(model=B.SEPARABLE, engine=B.GEMM_BF16X3, out=work)
        torch.cuda.synchronize()
        t_l = time.perf_counter() - t0
        row = dict(seed=s, err_learned=_rel(ctx, work, ref, nref), s_learned=t_l, paths_learned=n_l)
        for n in uniform_budgets:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            n_u = ctx.trace(n, seed=tp.seed, sampler=B.UNIFORM, **kw)
            ctx.synthesize(model=B.SEPARABLE, engine=B.DIRECT_FP32, out=work)
            torch.cuda.synchronize()
            row[f"s_uniform_{n}"] = time.perf_counter() - t0
            row[f"err_uniform_{n}"] = _rel(ctx, work, ref, nref)
            row[f"paths_uniform_{n}"] = n_u
            # the same uniform paths through the GEMM engine (time only)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.trace(n, seed=tp.seed, sampler=B.UNIFORM, **kw)
            ctx.synthesize(model=B.SEPARABLE, engine=B.GEMM_BF16X3, out=work)
            torch.cuda.synchronize()
            row[f"s_uniform_gemm_{n}"] = time.perf_counter() - t0
        per.append(row)
        if log:
            log(f"equal-error scene {s}: learned err {row['err_learned']:.3f} in "
                f"{row['s_learned'] * 1e3:.1f} ms")
    el = float(np.mean([r["err_learned"] for r in per]))
    tl = float(np.mean([r["s_learned"] for r in per[1:] or per]))
    eu = np.array([np.mean([r[f"err_uniform_{n}"] for r in per]) for n in uniform_budgets])
    tu = np.array([np.mean([r[f"s_uniform_{n}"] for r in per[1:] or per]) for n in uniform_budgets])
    tg = np.array([np.mean([r[f"s_uniform_gemm_{n}"] for r in per[1:] or per])
                   for n in uniform_budgets])
    pl = float(np.mean([r["paths_learned"] for r in per]))
    pu = np.array([np.mean([r[f"paths_uniform_{n}"] for r in per]) for n in uniform_budgets])
    xs = np.array(uniform_budgets, dtype=np.float64)
    n_eq = _loglog(xs, eu, el)
    t_eq = _loglog_time(xs, tu, n_eq)
    tg_eq = _loglog_time(xs, tg, n_eq)
    return dict(budget=budget, err_learned_mean=el, s_learned_mean=tl, paths_learned_mean=pl,
                uniform_budgets=list(uniform_budgets), err_uniform_mean=eu.tolist(),
                s_uniform_mean=tu.tolist(), s_uniform_gemm_mean=tg.tolist(),
                paths_uniform_mean=pu.tolist(), uniform_rays_at_equal_error=n_eq,
                s_uniform_at_equal_error=t_eq, speedup_at_equal_error=t_eq / tl,
                s_uniform_gemm_at_equal_error=tg_eq,
                speedup_vs_uniform_gemm_at_equal_error=tg_eq / tl, per_scene=per)


def _loglog_time(xs, ts, x):
    """Time at x on the piecewise log-log line through (xs, ts) (increasing)."""
    lx, lt, t = np.log(xs), np.log(ts), math.log(x)
    i = int(np.clip(np.searchsorted(lx, t) - 1, 0, len(xs) - 2))
    f = (t - lx[i]) / (lx[i + 1] - lx[i])
    return float(math.exp(lt[i] + f * (lt[i + 1] - lt[i])))


def experiment(ctx, train_seeds, eval_seeds, train_rays=50_000, budget=12_500, ref_rays=100_000,
               steps=300, batch=16, lr=1e-3, beta=0.1, power=0.5, alt_power=None, log=None):
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
    res = evaluate(ctx, ew, budget, ref_rays, beta, power, alt_power)
    if log:
        log(f"evaluated {len(res)} held-out scenes in {time.time() - t2:.1f} s")
    eu = np.array([r["err_uniform"] for r in res])
    el = np.array([r["err_learned"] for r in res])
    out = dict(collect_s=t1 - t0, train_s=t2 - t1, loss_first=losses[0], loss_last=losses[-1],
               err_uniform_mean=float(eu.mean()), err_learned_mean=float(el.mean()),
               err_ratio_mean=float(np.mean(el / eu)), wins=int((el < eu).sum()),
               n_eval=len(res), per_scene=res)
    if all("err_tri" in r for r in res):
        et = np.array([r["err_tri"] for r in res])
        out.update(err_tri_mean=float(et.mean()), err_ratio_tri_mean=float(np.mean(et / eu)),
                   wins_tri=int((et < eu).sum()),
                   rays_tri_mean=float(np.mean([r["rays_tri"] for r in res])),
                   paths_tri_mean=float(np.mean([r["paths_tri"] for r in res])),
                   empty_tri=int(sum(r["paths_tri"] == 0 for r in res)))
    if all("err_cut" in r for r in res):
        ec = np.array([r["err_cut"] for r in res])
        out.update(err_cut_mean=float(ec.mean()), err_ratio_cut_mean=float(np.mean(ec / eu)),
                   wins_cut=int((ec < eu).sum()),
                   rays_cut_mean=float(np.mean([r["rays_cut"] for r in res])),
                   paths_cut_mean=float(np.mean([r["paths_cut"] for r in res])))
    if alt_power is not None:
        ea = np.array([r["err_learned_alt"] for r in res])
        out.update(alt_power=alt_power, err_learned_alt_mean=float(ea.mean()),
                   err_ratio_alt_mean=float(np.mean(ea / eu)), wins_alt=int((ea < eu).sum()),
                   paths_learned_alt_mean=float(np.mean([r["paths_learned_alt"] for r in res])))
    out.update(paths_uniform_mean=float(np.mean([r["paths_uniform"] for r in res])),
               paths_learned_mean=float(np.mean([r["paths_learned"] for r in res])))
    return out
