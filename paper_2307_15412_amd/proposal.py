"""Training and evaluation of the learned ray proposal on top of the C ABI.

Orchestration only: probing, tracing, histograms, the network's forward,
backward and Adam steps and the sampling table all run in the library's HIP
kernels (include/radray.h, "Learned ray proposal").

Training data: for every training scene, the 16-value probe code and the
per-bin returned-power histogram of a uniform trace.  Evaluation: for held-out
scenes, the cube from a ray budget drawn from the learned density (mixed with
the uniform density) against the cube from the same budget drawn uniformly,
each scored by its error against the expectation of the cube (estimated from
two independent uniform launches, whose own noise is subtracted).
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


class Reference:
    """The expectation of a scene's cube, estimated by two independent
    uniform launches A and B of the same size: R = (A + B) / 2.  For an
    unbiased estimate s independent of both, E |s - R|^2 = MSE(s) + var(R)
    and E |A - B|^2 = 4 var(R), so |s - R|^2 - |A - B|^2 / 4 estimates the
    squared error of s against the expectation itself, and |R|^2 - |A - B|^2
    / 4 the squared norm of the expectation: the relative error below is
    free of the reference's own noise (a zero cube scores exactly 1)."""

    def __init__(self, a, b):
        self.R = (a + b) * 0.5
        self.noise2 = float((a - b).abs().pow(2).sum()) / 4.0
        self.norm2 = float(self.R.abs().pow(2).sum()) - self.noise2

    def mse(self, s):
        """Relative mean squared error of s against the expectation."""
        return (float((s - self.R).abs().pow(2).sum()) - self.noise2) / max(self.norm2, 1e-300)

    def ref_err(self):
        """Relative error of R itself."""
        return math.sqrt(max(self.noise2, 0.0) / max(self.norm2, 1e-300))


def _err(mses):
    return math.sqrt(max(float(np.mean(mses)), 0.0))


def evaluate(ctx, workloads, budget, ref_rays, beta=0.1, power=0.5, alt_power=None, n_seeds=4,
             kappa=None):
    """Per held-out scene: relative cube error against the expectation (see
    Reference: two independent uniform launches of `ref_rays`) of uniform
    and learned launches of `budget` rays, each averaged over `n_seeds`
    independent seeds; the learned table with softmax power `power` (and,
    for comparison, `alt_power`, or the cost-aware table with `kappa`), and
    per-triangle casting with at most the same number of rays.  The zero
    cube scores 1."""
    out = []
    for w in workloads:
        ctx.setup(w)
        tp = w.trace
        kw = dict(max_bounces=tp.max_bounces, az_min=tp.az_min, az_max=tp.az_max,
                  el_min=tp.el_min, el_max=tp.el_max, record_hits=False)
        ctx.trace(ref_rays, seed=tp.seed + 7919, sampler=B.UNIFORM, **kw)
        a = _cube(ctx).clone()
        ctx.trace(ref_rays, seed=tp.seed + 15887, sampler=B.UNIFORM, **kw)
        ref = Reference(a, _cube(ctx).clone())
        del a
        seeds = [tp.seed + 104729 * i for i in range(n_seeds)]

        def run(n, sampler, **extra):
            mses, paths, ms = [], [], []
            for sd in seeds:
                paths.append(ctx.trace(n, seed=sd, sampler=sampler, **kw, **extra))
                ms.append(ctx.kernel_ms(0))
                mses.append(ref.mse(_cube(ctx)))
            return _err(mses), float(np.mean(paths)), float(np.mean(ms))

        eu, p_u, t_u = run(budget, B.UNIFORM)
        code = ctx.proposal_probe(tp.az_min, tp.az_max)
        rec = dict(seed=tp.seed, err_uniform=eu, paths_uniform=p_u, ms_uniform=t_u,
                   err_ref=ref.ref_err())
        if alt_power is not None:
            ctx.proposal_build(code, beta, alt_power)
            e, p_, _ = run(budget, B.PROPOSAL)
            rec.update(err_learned_alt=e, paths_learned_alt=p_)
        if kappa is not None:
            ctx.proposal_build_cost(code, beta, kappa)
            e, p_, _ = run(budget, B.PROPOSAL)
            rec.update(err_learned_cost=e, paths_learned_cost=p_)
        ctx.proposal_build(code, beta, power)
        el, p_l, t_l = run(budget, B.PROPOSAL)
        rec.update(err_learned=el, paths_learned=p_l, ms_learned=t_l)
        # per-triangle casting (the triangles in view) with at most the same
        # number of rays
        fov = (tp.az_min, tp.az_max, tp.el_min, tp.el_max)
        ctx.set_casting(0.0, 8)
        n_in = ctx.casting_pieces(*fov)
        g = int(math.isqrt(budget // max(n_in, 1)))
        if g >= 1:
            e, p_, t_ = run(g * g, B.PER_TRIANGLE)
            rec.update(err_tri=e, ms_tri=t_, rays_tri=g * g * n_in, paths_tri=p_)
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
        e, p_, t_ = run(4, B.PER_TRIANGLE)
        rec.update(err_cut=e, ms_cut=t_, rays_cut=4 * n_pc, paths_cut=p_, omega_cut=om)
        ctx.set_casting(0.0, 8)
        out.append(rec)
    return out


def _loglog(xs, ys, y):
    """x where the piecewise log-log line through (xs, ys) reaches y (ys
    decreasing); extrapolated from the end segments."""
    lx, ly, t = np.log(xs), np.log(ys), math.log(y)
    i = int(np.clip(np.searchsorted(-ly, -t) - 1, 0, len(xs) - 2))
    f = (t - ly[i]) / (ly[i + 1] - ly[i])
    return float(math.exp(lx[i] + f * (lx[i + 1] - lx[i])))


def equal_error(ctx, eval_seeds, budget=250_000, uniform_budgets=(250_000, 500_000, 1_000_000,
                                                                    2_000_000, 4_000_000),
                ref_rays=4_000_000, beta=0.1, power=0.5, direct_max=1_000_000, log=None):
    """Wall time at equal cube error on the large-MIMO array (3072 channels,
    512 samples x 256 chirps) over box-family scenes, with the network as
    trained in `ctx`; errors against the expectation (Reference: two
    independent `ref_rays` uniform launches), all cubes in the separable
    model.

    Learned pipelines (probe code, sampling table, `budget` rays, GEMM
    synthesis): the square-root table (softmax power `power`) and the
    cost-aware table, whose kappa = c_ray / (c_path rho_mean) is the trace
    time over the synthesis time of a uniform launch (measured on the first
    scene).  Uniform pipelines at each of `uniform_budgets`: with the GEMM
    engine, and the plain tracer (direct summation; timed up to `direct_max`
    rays, beyond that scaled from its measured time per path, which is
    exact for a sum over paths).  The uniform budget of equal mean error, and
    the time there, are interpolated in log-log."""
    torch = ctx.torch
    import scenegen as sg
    per = []
    buf = {}
    kappa = None
    for s in eval_seeds:
        w = sg.workload_box_mimo(s, budget)
        ctx.setup(w)
        tp = w.trace
        C, M, K = w.array.n_ch, w.chirp.n_chirps, w.chirp.n_samples
        if not buf:
            for k in ("a", "b", "work"):
                buf[k] = torch.empty((C, M, K), dtype=torch.complex64, device=ctx.device)
        kw = dict(max_bounces=tp.max_bounces, az_min=tp.az_min, az_max=tp.az_max,
                  el_min=tp.el_min, el_max=tp.el_max, record_hits=False)
        gemm = lambda out: ctx.synthesize(model=B.SEPARABLE, engine=B.GEMM_BF16X3, out=out)
        ctx.trace(ref_rays, seed=tp.seed + 7919, sampler=B.UNIFORM, **kw)
        t_tr = ctx.kernel_ms(0)
        gemm(buf["a"])
        t_sy = ctx.kernel_ms(1)
        if kappa is None:
            kappa = t_tr / t_sy
            if log:
                log(f"kappa = trace {t_tr:.3f} ms / synthesis {t_sy:.2f} ms = {kappa:.3g}")
        ctx.trace(ref_rays, seed=tp.seed + 15887, sampler=B.UNIFORM, **kw)
        gemm(buf["b"])
        ref = Reference(buf["a"], buf["b"])
        work = buf["work"]
        row = dict(seed=s, err_ref=ref.ref_err())

        def timed(fn):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            n = fn()
            torch.cuda.synchronize()
            return n, time.perf_counter() - t0

        for name, build in (("learned", lambda c: ctx.proposal_build(c, beta, power)),
                            ("learned_cost", lambda c: ctx.proposal_build_cost(c, beta, kappa))):
            def pipe():
                code = ctx.proposal_probe(tp.az_min, tp.az_max)
                build(code)
                n = ctx.trace(budget, seed=tp.seed, sampler=B.PROPOSAL, **kw)
                gemm(work)
                return n
            n_l, t_l = timed(pipe)
            row[f"err_{name}"] = math.sqrt(max(ref.mse(work), 0.0))
            row[f"s_{name}"] = t_l
            row[f"paths_{name}"] = n_l
        for n in uniform_budgets:
            def pipe_gemm():
                m_ = ctx.trace(n, seed=tp.seed, sampler=B.UNIFORM, **kw)
                gemm(work)
                return m_
            n_u, t_g = timed(pipe_gemm)
            row[f"err_uniform_{n}"] = math.sqrt(max(ref.mse(work), 0.0))
            row[f"paths_uniform_{n}"] = n_u
            row[f"s_uniform_gemm_{n}"] = t_g
            if n <= direct_max:
                def pipe_direct():
                    ctx.trace(n, seed=tp.seed, sampler=B.UNIFORM, **kw)
                    ctx.synthesize(model=B.SEPARABLE, engine=B.DIRECT_FP32, out=work)
                _, t_d = timed(pipe_direct)
                row[f"s_uniform_{n}"] = t_d
        # the plain tracer beyond direct_max: its measured time per path
        meas = [n for n in uniform_budgets if n <= direct_max]
        per_path = max(row[f"s_uniform_{n}"] / max(row[f"paths_uniform_{n}"], 1) for n in meas[-1:])
        for n in uniform_budgets:
            if n > direct_max:
                row[f"s_uniform_{n}"] = per_path * row[f"paths_uniform_{n}"]
        per.append(row)
        if log:
            log(f"equal-error scene {s}: err learned {row['err_learned']:.3f} cost-aware "
                f"{row['err_learned_cost']:.3f} uniform@{uniform_budgets[0]} "
                f"{row[f'err_uniform_{uniform_budgets[0]}']:.3f} ref {row['err_ref']:.3f}")
    xs = np.array(uniform_budgets, dtype=np.float64)
    mean = lambda key: float(np.mean([r[key] for r in per]))
    # times: the first scene is a warm-up for the timing of every pipeline
    tmean = lambda key: float(np.mean([r[key] for r in (per[1:] or per)]))
    eu = np.array([mean(f"err_uniform_{n}") for n in uniform_budgets])
    tu = np.array([tmean(f"s_uniform_{n}") for n in uniform_budgets])
    tg = np.array([tmean(f"s_uniform_gemm_{n}") for n in uniform_budgets])
    pu = np.array([mean(f"paths_uniform_{n}") for n in uniform_budgets])
    out = dict(budget=budget, kappa=kappa, uniform_budgets=list(uniform_budgets),
               err_uniform_mean=eu.tolist(), s_uniform_mean=tu.tolist(),
               s_uniform_gemm_mean=tg.tolist(), paths_uniform_mean=pu.tolist(),
               err_ref_mean=mean("err_ref"), direct_timed_up_to=direct_max)
    for name in ("learned", "learned_cost"):
        el, tl, pl = mean(f"err_{name}"), tmean(f"s_{name}"), mean(f"paths_{name}")
        n_eq = _loglog(xs, eu, el)
        t_eq = _loglog_time(xs, tu, n_eq)
        tg_eq = _loglog_time(xs, tg, n_eq)
        out[name] = dict(err_mean=el, s_mean=tl, paths_mean=pl, uniform_rays_at_equal_error=n_eq,
                         uniform_paths_at_equal_error=_loglog_time(xs, pu, n_eq),
                         s_plain_at_equal_error=t_eq, speedup_vs_plain=t_eq / tl,
                         s_uniform_gemm_at_equal_error=tg_eq, speedup_vs_uniform_gemm=tg_eq / tl)
    out["per_scene"] = per
    return out


def _loglog_time(xs, ts, x):
    """Time at x on the piecewise log-log line through (xs, ts) (increasing)."""
    lx, lt, t = np.log(xs), np.log(ts), math.log(x)
    i = int(np.clip(np.searchsorted(lx, t) - 1, 0, len(xs) - 2))
    f = (t - lx[i]) / (lx[i + 1] - lx[i])
    return float(math.exp(lt[i] + f * (lt[i + 1] - lt[i])))


def experiment(ctx, train_seeds, eval_seeds, train_rays=50_000, budget=125_000, ref_rays=4_000_000,
               steps=300, batch=16, lr=1e-3, beta=0.1, power=0.5, alt_power=None, kappa=None,
               n_seeds=4, log=None):
    """Train on uniform traces of `train_seeds`, then evaluate the held-out
    `eval_seeds` at `budget` rays (see evaluate); errors against the
    expectation, so that the zero cube's error, 1, is the negative control."""
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
    res = evaluate(ctx, ew, budget, ref_rays, beta, power, alt_power, n_seeds=n_seeds, kappa=kappa)
    if log:
        log(f"evaluated {len(res)} held-out scenes in {time.time() - t2:.1f} s")
    eu = np.array([r["err_uniform"] for r in res])
    el = np.array([r["err_learned"] for r in res])
    out = dict(collect_s=t1 - t0, train_s=t2 - t1, loss_first=losses[0], loss_last=losses[-1],
               budget=budget, ref_rays=ref_rays, n_seeds=n_seeds,
               err_zero=1.0, err_ref_mean=float(np.mean([r["err_ref"] for r in res])),
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
    if kappa is not None:
        ek = np.array([r["err_learned_cost"] for r in res])
        out.update(kappa=kappa, err_learned_cost_mean=float(ek.mean()),
                   err_ratio_cost_mean=float(np.mean(ek / eu)), wins_cost=int((ek < eu).sum()),
                   paths_learned_cost_mean=float(np.mean([r["paths_learned_cost"] for r in res])))
    out.update(paths_uniform_mean=float(np.mean([r["paths_uniform"] for r in res])),
               paths_learned_mean=float(np.mean([r["paths_learned"] for r in res])))
    return out
