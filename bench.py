"""Benchmark of the radar ray-tracing hot path on one MI355X.

A step is one pass of the whole path over the large-MIMO workload: trace the
procedural street (5.1e5 triangles, 4e6 rays launched from the Tx phase
centre, up to 3 bounces, reception, path bookkeeping), keep the first 1e5
returned paths, and synthesise the 3072-channel x 256-chirp x 512-sample FMCW
cube from them.  Inputs are resident in HBM before the timed region (the
scene, array and chirp are uploaded once; BVH build excluded).

Prints one JSON line: value = path-samples synthesised per second over the
whole step (P x C x M x K / step time), plus the tracer's Mrays/s, the cube's
relative error against the FP64 oracle on sampled entries, the roofline of
the dominant kernel and the oracle's own throughput on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0
FP32_PEAK_TFLOPS = 157.3
FLOPS_PER_PATH_SAMPLE = 8.0      # one complex multiply-accumulate


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--engine", choices=["auto", "gemm", "direct"], default="auto")
    ap.add_argument("--rays", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true", help="skip the oracle rel-err check")
    ap.add_argument("--no-street", action="store_true", help="skip the street trace leg")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (hardware-counter calibration)")
    ap.add_argument("--mfma-calibration", action="store_true",
                    help="only time vendor-library bf16 and fp32 GEMMs (reachable matrix peak)")
    ap.add_argument("--batch-scenes", type=int, default=64)
    ap.add_argument("--workload", choices=["large_mimo", "batch", "proposal", "hand", "alpha_sweep",
                                           "tri_cast", "hand_motion", "street_trace", "mlp"],
                    default="large_mimo",
                    help="large_mimo (default): the benchmarked step; batch: 64 uneven scenes in "
                         "one captured launch; proposal: learned-proposal training and gain; "
                         "hand: SFCW hand imaging (trace, synthesis, back-projection, projection); "
                         "alpha_sweep: the hand imaged at alpha = 0, 0.1, ..., 1; tri_cast: "
                         "per-triangle casting vs the uniform launch at equal rays; hand_motion: "
                         "32 frames of a moving hand (refit, trace, synthesis per frame); mlp: "
                         "the proposal network's forward rate and training-step time")
    return ap.parse_args()


def run_batch(args):
    """64 procedural scenes (1e4-1e6 triangles, 4-3072 channels, 128-512
    samples, 64-256 chirps, 1e6 rays each, 3 bounces) traced and synthesised
    (exact model, FP32 cubes) by one captured launch after autotuning (per
    scene the direct engine or the exact product engine, and its tile)."""
    import torch
    import scenegen as sg
    import paper_2307_15412_amd as rr
    log = lambda m: print(f"[batch] {m}", file=sys.stderr, flush=True)
    t0 = time.time()
    ws = sg.workload_batch(n_scenes=args.batch_scenes, seed0=2000, rays=1_000_000)
    gen_s = time.time() - t0
    log(f"generated {len(ws)} scenes in {gen_s:.1f} s")
    ctx = rr.Context(0)
    B = rr.Batch(ctx, len(ws))
    t0 = time.time()
    for i, w in enumerate(ws):
        B.set_workload(i, w)
        if i % 8 == 7:
            log(f"uploaded {i + 1} scenes")
    upload_s = time.time() - t0
    cubes = B.alloc_cubes()
    t0 = time.time()
    tiles = B.tune(cubes)
    tune_s = time.time() - t0
    eng, ptile = B.plan()
    # per scene: "x<tile>" on the exact product engine, "d<samples per lane>"
    # on the direct engine
    plan = [("x" if e == rr.GEMM_EXACT else "d") + str(int(t)) for e, t in zip(eng, ptile)]
    n_prod = int(np.sum(eng == rr.GEMM_EXACT))
    log(f"autotune {tune_s:.1f} s: {n_prod} scenes on the product engine, plan {plan}")
    for _ in range(args.warmup):
        B.launch(cubes, want_counts=False)
        log("warmup launch done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        counts = B.launch(cubes)
        log("timed launch done")
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    ps = sum(float(n) * np.prod(s) for n, s in zip(counts, B.shapes))
    rays = sum(w.trace.n_rays for w in ws)
    # sampled entries of the timed launch's cubes against the FP64 oracle
    # (exact model): the slot with the most channels, the one with the most
    # triangles and four seeded others, 256 entries each
    check = None
    if not args.no_check:
        import oracle
        slots = [int(np.argmax([w.array.n_ch for w in ws])), int(np.argmax([w.scene.n_tris for w in ws]))]
        for s in np.random.default_rng(5).permutation(len(ws)):
            if len(slots) >= 6:
                break
            if int(s) not in slots:
                slots.append(int(s))
        errs, ratios, t0 = [], [], time.perf_counter()
        for s in slots:
            w = ws[s]
            _, op = oracle.trace(w.scene, w.array, w.trace, want_hits=False)
            if len(op) != counts[s]:
                raise SystemExit(f"slot {s}: {counts[s]} paths, oracle {len(op)}")
            flat = cubes[s].reshape(-1)
            idx = np.random.default_rng(100 + s).choice(flat.numel(), 256, replace=False)
            got = flat[torch.from_numpy(idx).to(flat.device)].cpu().numpy()
            ref = oracle.synth(op, w.scene, w.array, w.chirp, model=0, idx=idx)
            errs.append(float(np.linalg.norm(got - ref) / np.linalg.norm(ref)))
            ratios.append(float(np.abs(got - ref).max() / np.abs(ref).max()))
            log(f"slot {s}: {w.array.n_ch} ch, {w.scene.n_tris} tris, rel err {errs[-1]:.2e}")
        check = {"slots": slots, "rel_err": errs, "max_err_ratio": ratios,
                 "rel_err_max": max(errs), "oracle_s": time.perf_counter() - t0,
                 "entries_per_slot": 256}
    print(json.dumps({
        "metric": "batched Gpath-samples/s (64 uneven scenes, one captured launch)",
        "value": ps / dt / 1e9, "unit": "Gpath-samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True,
        "dtype": "f64-phase/f32", "data": "synthetic (procedural streets, seeded)",
        "config": {"workload": f"batch: {len(ws)} streets, 1e4-1e6 tris, 4-3072 ch, 128-512 samples, "
                               "64-256 chirps, 1e6 rays each, <=3 bounces, exact model"},
        "scenes": len(ws), "rays": rays, "paths": int(np.sum(counts)),
        "cube_gb": sum(np.prod(s) for s in B.shapes) * 8 / 1e9,
        "mrays_per_s_incl_synth": rays / dt / 1e6, "plan": plan, "product_engine_scenes": n_prod,
        "autotune_s": tune_s,
        "scene_gen_s": gen_s, "bvh_upload_s": upload_s, "graph_ms": B.stats()["ms_total"],
        "oracle_check": check}))


def run_proposal(args):
    """Learned proposal: train on 200 scenes x 5e4 uniform rays, evaluate 50
    held-out scenes at 1.25e5 and 1e6 rays (learned, cost-aware learned,
    uniform, per-triangle casting; 4 seeds each), every cube scored by its
    error against the expectation (two independent 8e6-ray uniform launches,
    their own noise subtracted: the zero cube scores 1); then, on 20 held-out
    scenes seen by the 3072-channel array (512 samples x 256 chirps), the wall
    time of learned launch + GEMM synthesis against uniform launch with GEMM
    synthesis and with direct summation (the plain tracer) at equal error."""
    import torch
    import scenegen as sg
    import paper_2307_15412_amd as rr
    from paper_2307_15412_amd import proposal
    ctx = rr.Context(0)
    out = {}
    log = lambda m: print(f"[proposal] {m}", file=sys.stderr, flush=True)
    # kappa of the small array: trace time / synthesis time of a uniform launch
    w = sg.workload_box_family(1, 100_000, points=False)
    ctx.setup(w)
    for _ in range(2):
        ctx.trace_workload(w, record_hits=False)
        t_tr = ctx.kernel_ms(0)
        ctx.synthesize(model=rr.EXACT, engine=rr.DIRECT_FP32)
        t_sy = ctx.kernel_ms(1)
    kappa = t_tr / t_sy
    log(f"small-array kappa = {t_tr:.3f} / {t_sy:.3f} ms = {kappa:.3g}")
    for budget in (125_000, 1_000_000):
        res = proposal.experiment(ctx, train_seeds=range(1, 201), eval_seeds=range(1001, 1051),
                                  train_rays=50_000, budget=budget, ref_rays=8_000_000, steps=600,
                                  batch=16, lr=2e-3, power=0.5, alt_power=1.0, kappa=kappa,
                                  n_seeds=4, log=log)
        log(f"budget {budget}: uniform {res['err_uniform_mean']:.3f}, learned "
            f"{res['err_learned_mean']:.3f}, cost-aware {res['err_learned_cost_mean']:.3f}")
        out[f"budget_{budget}"] = {k: v for k, v in res.items() if k != "per_scene"}
    # equal cube error on the 3072-channel array
    eq = proposal.equal_error(ctx, eval_seeds=range(1001, 1021), log=log)
    for name in ("learned", "learned_cost"):
        e = eq[name]
        log(f"equal error, {name}: uniform needs {e['uniform_rays_at_equal_error']:.0f} rays; "
            f"x{e['speedup_vs_plain']:.2f} vs plain, x{e['speedup_vs_uniform_gemm']:.2f} vs "
            f"uniform + GEMM")
    r = out["budget_1000000"]
    ratio = r["err_learned_mean"] / r["err_uniform_mean"]
    print(json.dumps({
        "metric": "learned-proposal cube error / uniform cube error at 1e6 rays, errors against "
                  "the expectation (lower is better)",
        "value": ratio, "unit": "ratio", "higher_is_better": False, "n_gpus": 1,
        "equal_error_ray_saving": 1.0 / (ratio * ratio),
        "config": {"workload": "box family: 200 training scenes x 5e4 rays, 50 held-out scenes, "
                               "1.25e5 and 1e6 rays, 4 seeds, references 2 x 8e6 uniform rays, "
                               "beta 0.1"},
        "results": out,
        "equal_error": {k: v for k, v in eq.items() if k != "per_scene"}}))


def run_mlp(args):
    """The proposal network alone: logits for every bin of 128 scenes (1.05e6
    evaluations) and one training step (forward, softmax gradient, backward,
    weight gradients, Adam) at 16 scenes (the training batch) and at 128;
    seeded synthetic scene codes and histograms, wall time around synchronised
    repetitions."""
    import torch
    import paper_2307_15412_amd as rr
    ctx = rr.Context(0)
    g = torch.Generator().manual_seed(5)
    nbins = 128 * 64
    macs = 18 * 64 + 64 * 64 + 64 * 64 + 64          # per evaluation (forward)
    out = {}
    ctx.mlp_init(3)
    for ns in (16, 128):
        codes = torch.rand((ns, 16), generator=g).to("cuda:0")
        hists = torch.rand((ns, nbins), generator=g).to("cuda:0")
        for _ in range(args.warmup + 1):
            ctx.mlp_forward(codes)
            ctx.mlp_train_step(codes, hists, 1e-3)
        torch.cuda.synchronize()
        reps = max(args.steps, 1) * 10
        t0 = time.perf_counter()
        for _ in range(reps):
            ctx.mlp_forward(codes)
        torch.cuda.synchronize()
        t_fwd = (time.perf_counter() - t0) / reps
        t0 = time.perf_counter()
        for _ in range(reps):
            ctx.mlp_train_step(codes, hists, 1e-3)
        torch.cuda.synchronize()
        t_step = (time.perf_counter() - t0) / reps
        out[f"scenes_{ns}"] = {"rows": ns * nbins, "forward_ms": t_fwd * 1e3,
                               "train_step_ms": t_step * 1e3,
                               "evaluations_per_s": ns * nbins / t_fwd}
    big = out["scenes_128"]
    achieved = 2.0 * macs * big["evaluations_per_s"] / 1e12
    print(json.dumps({
        "metric": "proposal-network evaluations/s (forward, all bins of 128 scenes)",
        "value": big["evaluations_per_s"], "unit": "evaluations/s", "higher_is_better": True,
        "n_gpus": 1, "dtype": "fp16 forward / fp32 backward, fp32 accumulation",
        "data": "synthetic (seeded codes and histograms)",
        "config": {"workload": "MLP 18-64-64-64-1, 128 x 64 bins a scene; training step at 16 "
                               "and 128 scenes"},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": 2500.0, "unit": "TFLOP/s",
                     "frac": achieved / 2500.0, "kernel": "k_mlp_fwd",
                     "note": "wall time of the forward call (launch included), "
                             "2 x 9 408 flops per evaluation"},
        "results": out}))


def run_hand(args, sweep=False):
    """The paper's imaging set-up on a synthetic hand: trace 1e7 rays (+-25
    degrees, 2 bounces) from the 94 x 94 square array, synthesise the
    8836-channel x 128-step SFCW cube with the exact model (one split-bf16
    complex product per frequency on the matrix cores), back-project it
    onto the 81 x 201 x 201 grid of 1 mm voxels (per frequency a split-bf16
    product on the matrix cores) and take the maximum
    projection over range in dB.  A step is that whole chain; the dominant
    kernel is the back-projection (one complex multiply-add per voxel,
    channel and frequency step).  With sweep, a step images the hand at every
    alpha of the paper's sweep (0 to 1 by 0.1), set on the uploaded mesh."""
    import torch
    import scenegen as sg
    import paper_2307_15412_amd as rr
    log = lambda m: print(f"[hand] {m}", file=sys.stderr, flush=True)
    w = sg.workload_hand(0)
    if args.rays:
        w.trace.n_rays = args.rays
    grid = sg.imaging_grid()
    (x0, y0, z0), st, (nx, ny, nz) = grid
    C, K = w.array.n_ch, w.chirp.n_samples
    n_vox = nx * ny * nz
    terms = float(n_vox) * C * K
    ctx = rr.Context(0)
    ctx.setup(w)
    cube = torch.empty((C, 1, K), dtype=torch.complex64, device="cuda:0")
    img = torch.empty((nx, ny, nz), dtype=torch.complex64, device="cuda:0")
    proj = torch.empty((ny, nz), dtype=torch.float32, device="cuda:0")

    alphas = sg.alpha_sweep() if sweep else [float(w.scene.obj_alpha[0])]
    tr, sy, bp, per_alpha = [], [], [], []
    projs = [torch.empty((ny, nz), dtype=torch.float32, device="cuda:0") for _ in alphas]

    def step(record):
        ns = []
        for a, pr in zip(alphas, projs):
            if sweep:
                ctx.set_alpha([a] * w.scene.n_obj)
            ns.append(ctx.trace_workload(w, record_hits=False))
            ctx.synthesize(model=rr.EXACT, engine=rr.GEMM_EXACT, out=cube)
            ctx.backproject(cube, grid, out=img)
            ctx.max_projection(img, grid, out=pr)
            if record:
                tr.append(ctx.kernel_ms(0))
                sy.append(ctx.kernel_ms(1))
                bp.append(ctx.kernel_ms(2))
        return ns

    for _ in range(args.warmup):
        step(False)
        log("warmup step done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ns = step(True)
        log("timed step done")
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    log(f"timed {args.steps} steps, {dt * 1e3:.1f} ms each")
    P = int(round(float(np.mean(ns))))   # paths per image (mean over the sweep)
    if sweep:
        # how the image changes with alpha: pixels above the -15 dB floor and
        # the correlation of each dB image with the specular (alpha = 0) one
        ref = projs[0].reshape(-1)
        for a, n, pr in zip(alphas, ns, projs):
            v = pr.reshape(-1)
            corr = torch.corrcoef(torch.stack([ref, v]))[0, 1].item()
            per_alpha.append({"alpha": a, "paths": n,
                              "frac_above_floor": (v > -15.0).float().mean().item(),
                              "corr_with_alpha0": corr})
        ctx.set_alpha(list(w.scene.obj_alpha))
    bp_ms = float(np.mean(bp))
    flops = terms * FLOPS_PER_PATH_SAMPLE
    # the back-projection runs on the matrix cores (split bf16: three products
    # per real multiply-add are issued; the roofline counts the algorithmic 8)
    roof = {"bound": "mfma", "achieved": flops / (bp_ms * 1e-3) / 1e12, "peak": BF16_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "traffic": profiled_traffic("paper_2307_15412_amd/csrc/k_bpmfma.hip",
                                        "profiles/k_bp_mfma_hand.md"),
            "kernel": "bp_mfma", "flops_per_launch": flops, "issued_flops_per_launch": 3 * flops}
    roof["frac"] = roof["achieved"] / roof["peak"]

    cube_rel = img_rel = cpu = None
    if not args.no_check or not args.no_cpu_baseline:
        import oracle
        rng = np.random.default_rng(13)
        sub = sg.workload_hand(0)
        sub.trace.n_rays = 2_000_000
        t1 = time.perf_counter()
        _, op = oracle.trace(sub.scene, sub.array, sub.trace, want_hits=False)
        t_trace = time.perf_counter() - t1
        idx = rng.choice(C * K, 2048, replace=False)
        t1 = time.perf_counter()
        ref = oracle.synth(op, sub.scene, sub.array, sub.chirp, model=0, idx=idx)
        t_syn = time.perf_counter() - t1
        log(f"oracle trace {t_trace:.1f} s ({len(op)} paths), synthesis {t_syn:.1f} s")
        # image check: the oracle's full cube of its first 32 paths, imaged by
        # both sides, compared on seeded voxels
        few = op[:32]
        ocube = oracle.synth(few, sub.scene, sub.array, sub.chirp, model=0)
        i, j, k = (rng.integers(0, n, 480) for n in (nx, ny, nz))
        vox = np.stack([x0 + i * st, y0 + j * st, z0 + k * st], -1)
        t1 = time.perf_counter()
        oimg = oracle.backproject(sub.array, sub.chirp.f0, sub.chirp.bandwidth / K, ocube, vox)
        t_bp = time.perf_counter() - t1
        log(f"oracle back-projection of {len(vox)} voxels {t_bp:.1f} s")
        if not args.no_check:
            soa = oracle.to_soa(op)
            ctx.set_paths({kk: torch.from_numpy(np.ascontiguousarray(v)) for kk, v in soa.items()})
            full = ctx.synthesize(model=rr.EXACT, engine=rr.GEMM_EXACT, out=cube)
            got = full.reshape(-1)[torch.from_numpy(idx).to(full.device)].cpu().numpy()
            cube_rel = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
            cin = torch.from_numpy(ocube.reshape(C, 1, K).astype(np.complex64)).cuda()
            gimg = ctx.backproject(cin, grid, out=img)
            flat = torch.from_numpy((i * ny + j) * nz + k).cuda()
            gv = gimg.reshape(-1)[flat].cpu().numpy()
            img_rel = float(np.abs(gv - oimg).max() / np.abs(oimg).max())
        if not args.no_cpu_baseline:
            t_full = t_trace * (w.trace.n_rays / sub.trace.n_rays) + \
                t_syn * (float(P) * C * K) / (len(op) * len(idx)) + t_bp * (n_vox / len(vox))
            cpu = {"value": 1.0 / t_full, "unit": "images/s", "cores": 1, "kind": "oracle",
                   "sample": f"single-threaded FP64 oracle: trace of {sub.trace.n_rays} of "
                             f"{w.trace.n_rays} rays ({t_trace:.2f} s), {len(idx)} exact-model "
                             f"cube entries over its {len(op)} paths ({t_syn:.2f} s) and "
                             f"{len(vox)} back-projected voxels ({t_bp:.2f} s), each scaled "
                             f"to the full step ({P} paths, {C} x {K} cube, {n_vox} voxels); "
                             f"host {cpu_model()}, nproc {os.cpu_count()}"}
    if sweep and cpu is not None:
        cpu["sample"] += "; the sweep's images each cost the same"
    out = {
        "metric": ("hand images/s over the alpha sweep 0..1 by 0.1 (trace + SFCW synthesis + "
                   "back-projection + max projection per alpha)") if sweep else
                  "hand images/s (trace + SFCW synthesis + back-projection + max projection)",
        "value": len(alphas) / dt, "unit": "images/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64-phase/f32",
        "data": "synthetic (procedural hand proxy, seeded)",
        "config": {"workload": f"hand: 94 Tx x 94 Rx square array, {w.trace.n_rays} rays within "
                               "+-25 deg, <=2 bounces, 72-82 GHz SFCW 128 steps, exact model, "
                               f"{nx} x {ny} x {nz} voxels at 1 mm",
                   "paths": P},
        "trace_ms": float(np.mean(tr)), "synth_ms": float(np.mean(sy)), "synth_engine": "gemm_exact",
        "backproject_ms": bp_ms, "backproject_engine": "mfma_split_bf16",
        "backproject_tterms_per_s": terms / (bp_ms * 1e-3) / 1e12,
        "cube_rel_err": cube_rel, "image_rel_err": img_rel,
        "roofline": roof, "cpu_baseline": cpu}
    if sweep:
        out["config"]["workload"] = "alpha sweep: " + out["config"]["workload"] + \
            f", alpha in {alphas[0]}..{alphas[-1]} ({len(alphas)} images per step)"
        out["per_alpha"] = per_alpha
    print(json.dumps(out))


def run_tri_cast(args):
    """Per-triangle casting against the uniform launch at equal ray counts on
    the hand set-up (94 x 94 array, 128 steps, exact model): relative cube
    error against an independent 1e8-ray uniform reference at about 1e5, 1e6
    and 1e7 rays (g^2 rays per triangle in view, the uniform launch given exactly as
    many rays), and each launch's trace + synthesis time."""
    import torch
    import scenegen as sg
    import paper_2307_15412_amd as rr
    log = lambda m: print(f"[tri_cast] {m}", file=sys.stderr, flush=True)
    w = sg.workload_hand(0)
    tp = w.trace
    ctx = rr.Context(0)
    ctx.setup(w)
    C, K = w.array.n_ch, w.chirp.n_samples
    kw = dict(max_bounces=tp.max_bounces, az_min=tp.az_min, az_max=tp.az_max, el_min=tp.el_min,
              el_max=tp.el_max, record_hits=False)
    ref_rays = 100_000_000
    ctx.trace(ref_rays, seed=tp.seed + 7919, sampler=rr.UNIFORM, **kw)
    ref = ctx.synthesize(model=rr.EXACT, engine=rr.GEMM_EXACT)
    nref = float(ref.abs().pow(2).sum().sqrt())
    log(f"reference: {ctx.n_paths} paths from {ref_rays} rays")
    cube = torch.empty_like(ref)
    nt = w.scene.n_tris
    ctx.set_casting(0.0, 8)
    n_in = ctx.casting_pieces(tp.az_min, tp.az_max, tp.el_min, tp.el_max)   # triangles in view
    rows = []
    for target in (1e5, 1e6, 1e7):
        g = max(1, int(round(math.sqrt(target / n_in))))
        rays = g * g * n_in
        row = {"rays": rays, "g": g}
        for name, n, sampler in (("uniform", rays, rr.UNIFORM), ("per_triangle", g * g, rr.PER_TRIANGLE)):
            ctx.trace(n, seed=tp.seed, sampler=sampler, **kw)      # warm
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            P = ctx.trace(n, seed=tp.seed, sampler=sampler, **kw)
            ctx.synthesize(model=rr.EXACT, engine=rr.GEMM_EXACT, out=cube)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            err = float((cube - ref).abs().pow(2).sum().sqrt()) / nref
            row[name] = {"paths": P, "err": err, "ms": dt * 1e3, "trace_ms": ctx.kernel_ms(0)}
        row["err_ratio"] = row["per_triangle"]["err"] / row["uniform"]["err"]
        rows.append(row)
        log(f"{rays} rays: uniform err {row['uniform']['err']:.4f}, per-triangle "
            f"{row['per_triangle']['err']:.4f} (ratio {row['err_ratio']:.3f})")
    mid = rows[1]
    print(json.dumps({
        "metric": "per-triangle / uniform cube error at equal rays (hand, ~1e6 rays; lower is better)",
        "value": mid["err_ratio"], "unit": "ratio", "higher_is_better": False, "n_gpus": 1,
        "equal_error_ray_saving": 1.0 / mid["err_ratio"] ** 2,
        "data": "synthetic (procedural hand proxy, seeded)",
        "config": {"workload": f"hand: {nt} triangles ({n_in} in view), 94 Tx x 94 Rx, 72-82 GHz SFCW 128 steps, "
                               f"+-25 deg, <=2 bounces, exact model; reference {ref_rays} uniform rays"},
        "rows": rows}))


def run_hand_motion(args):
    """Radar responses of a moving hand: 32 frames of the hand proxy (fingers
    curling, thumb swinging, the hand drifting); per frame the vertices are
    moved and the BVH refit on the GPU, 1e7 rays traced from the 94 x 94
    array and the 8836 x 128 SFCW cube synthesised (exact model).  A step is
    the whole sequence.  Also timed: the refit alone against a host rebuild
    and upload of the same frame."""
    import torch
    import scenegen as sg
    import paper_2307_15412_amd as rr
    log = lambda m: print(f"[motion] {m}", file=sys.stderr, flush=True)
    n_frames = 32
    sc, frames = sg.hand_motion(0, n_frames=n_frames)
    w = sg.workload_hand(0)
    if args.rays:
        w.trace.n_rays = args.rays
    w.scene = sc
    C, K = w.array.n_ch, w.chirp.n_samples
    ctx = rr.Context(0)
    ctx.setup(w)
    cubes = torch.empty((n_frames, C, 1, K), dtype=torch.complex64, device="cuda:0")

    def step():
        ns = []
        for f in range(n_frames):
            ctx.update_vertices(frames[f])
            ns.append(ctx.trace_workload(w, record_hits=False))
            ctx.synthesize(model=rr.EXACT, engine=rr.GEMM_EXACT, out=cubes[f])
        return ns

    for _ in range(args.warmup):
        step()
        log("warmup step done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ns = step()
        log("timed step done")
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    # refit alone vs host rebuild + upload, per frame
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for f in range(n_frames):
        ctx.update_vertices(frames[f])
    torch.cuda.synchronize()
    refit_ms = (time.perf_counter() - t1) / n_frames * 1e3
    t1 = time.perf_counter()
    for f in range(4):
        ctx.upload(sg.with_verts(sc, frames[f]))
    torch.cuda.synchronize()
    rebuild_ms = (time.perf_counter() - t1) / 4 * 1e3
    # frame-to-frame change of the response
    d = [float((cubes[f] - cubes[0]).abs().pow(2).sum().sqrt() / cubes[0].abs().pow(2).sum().sqrt())
         for f in (1, n_frames // 4, n_frames // 2)]
    log(f"{dt * 1e3:.1f} ms per sequence, refit {refit_ms:.3f} ms, rebuild {rebuild_ms:.1f} ms")
    print(json.dumps({
        "metric": "moving-hand radar frames/s (vertex update + BVH refit + trace + SFCW synthesis)",
        "value": n_frames / dt, "unit": "frames/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64-phase/f32",
        "data": "synthetic (procedural hand proxy in motion, seeded)",
        "config": {"workload": f"hand motion: {n_frames} frames, {sc.n_tris} triangles, 94 Tx x 94 Rx, "
                               f"{w.trace.n_rays} rays within +-25 deg, <=2 bounces, 72-82 GHz SFCW "
                               "128 steps, exact model"},
        "paths_per_frame": [int(x) for x in ns], "refit_ms_per_frame": refit_ms,
        "host_rebuild_ms_per_frame": rebuild_ms,
        "cube_change_vs_frame0": {"frame1": d[0], f"frame{n_frames // 4}": d[1],
                                  f"frame{n_frames // 2}": d[2]}}))


def mfma_calibration():
    """The matrix peak reachable on this GPU, measured with the vendor BLAS:
    square bf16 GEMMs (FP32 accumulation) of 8192 and 16384 and a device copy
    of 1 GiB, timed with events after a warm-up; the published dense peaks
    (2.5 PFLOP/s bf16, 8 TB/s) are what the bench's roofline divides by."""
    import torch
    out = {}
    for n in (8192, 16384):
        a = torch.randn(n, n, dtype=torch.bfloat16, device="cuda:0")
        b = torch.randn(n, n, dtype=torch.bfloat16, device="cuda:0")
        c = torch.empty(n, n, dtype=torch.bfloat16, device="cuda:0")
        for _ in range(3):
            torch.matmul(a, b, out=c)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 20 if n == 8192 else 5
        e0.record()
        for _ in range(reps):
            torch.matmul(a, b, out=c)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[f"bf16_gemm_{n}"] = {"ms": ms, "tflops": 2.0 * n ** 3 / (ms * 1e-3) / 1e12}
        del a, b, c
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / 10
    out["copy_1gib"] = {"ms": ms, "gb_per_s": 2.0 * (1 << 30) / (ms * 1e-3) / 1e9}
    print(json.dumps(out))


def copy_calibration():
    """A plain device-to-device copy of exactly 1 GiB, five times: the
    FETCH_SIZE / WRITE_SIZE counters of this kernel calibrate the byte counts
    read for the library's kernels."""
    import torch
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": src.numel() * 4, "repeats": 5}))


TRACE_RECORD_BYTES = 164        # one appended path record (temporary SoA, 4 bounce slots)


def street_trace(ctx, scene, args, reps=None):
    """The street configuration's tracer throughput: 5.1e5 triangles, 12 Tx x
    16 Rx per-element launch, 1e7 rays, up to 3 bounces (the scene is the one
    already uploaded).  Mrays/s and segments/s over the whole trace stage
    (tracing kernel, scan, scatter), and the tracing kernel's memory roofline
    from the work the counting variant of the kernel reports: BVH nodes
    (64 B) + leaf triangle records (48 B) fetched + one count byte per ray +
    one appended path record per path.  Then the configuration's exact-model
    cube from those paths, with AUTO's engine and with the direct engine."""
    import torch
    import scenegen as sg
    wc = sg.workload_street(0) if scene is None else sg.Workload(
        "street", scene, sg.array_ula(12, 16), sg.Chirp(n_samples=256, n_chirps=128),
        sg.TraceParams(n_rays=10_000_000, max_bounces=3, seed=0))
    if scene is None:
        ctx.upload(wc.scene)
    a, ch, tp = wc.array, wc.chirp, wc.trace
    ctx.set_array(a.tx, a.rx, a.rx_radius, a.mode)
    ctx.set_chirp(ch.f0, ch.bandwidth, ch.t_chirp, ch.t_rep, ch.n_samples, ch.n_chirps)
    reps = reps or max(3, args.steps // 2)
    for _ in range(2):
        n = ctx.trace_workload(wc, record_hits=False)
    torch.cuda.synchronize()
    stage, kern = [], []
    t0 = time.perf_counter()
    for _ in range(reps):
        n = ctx.trace_workload(wc, record_hits=False)
        stage.append(ctx.kernel_ms(0))
        kern.append(ctx.kernel_ms(3))
    wall = (time.perf_counter() - t0) / reps
    n2, work = ctx.trace_work(tp.n_rays, tp.max_bounces, tp.seed, tp.az_min, tp.az_max,
                              tp.el_min, tp.el_max)
    if n2 != n:
        raise SystemExit(f"counting trace returned {n2} paths, the timed trace {n}")
    st, kt = float(np.median(stage)), float(np.median(kern))
    alg = work["nodes"] * 64 + work["tris"] * 48 + work["rays"] + n * TRACE_RECORD_BYTES
    ach = alg / (kt * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS, "kernel": "k_trace",
            "traffic": profiled_traffic("paper_2307_15412_amd/csrc/k_trace.hip",
                                        "profiles/k_trace_street.md"),
            "algorithmic_bytes": alg,
            "note": "algorithmic bytes count every lane's node and triangle fetch; the rays of a "
                    "wavefront are traced in a coherent order and share those fetches, and the "
                    "30 MB BVH stays in L2/MALL, so they can exceed what HBM delivers (the kernel "
                    "is bound by the latency of dependent node fetches, not by HBM)"}
    # the configuration's cube (exact model, FP32 bar): AUTO's engine (the
    # product engine's per-element sample split) and the direct engine; a
    # path of the per-element launch feeds its own transmitter's 16 channels
    import paper_2307_15412_amd as rr
    n = ctx.trace_workload(wc, record_hits=False)
    cube = torch.empty((a.n_ch, ch.n_chirps, ch.n_samples), dtype=torch.complex64, device="cuda:0")
    syn = {}
    for name, eng in (("auto", rr.ENGINE_AUTO), ("direct", rr.DIRECT_FP32)):
        ts = []
        for _ in range(3):
            ctx.synthesize(model=rr.EXACT, engine=eng, out=cube)
            ts.append(ctx.kernel_ms(1))
        syn[name] = float(np.median(ts))
    ps = float(n) * a.rx.shape[0] * ch.n_chirps * ch.n_samples
    return {"workload": "street: 5.1e5 tris, 12 Tx x 16 Rx per-element launch, 1e7 rays, "
                        "<=3 bounces, no path cap",
            "rays": tp.n_rays, "paths": n, "trace_stage_ms": st, "trace_kernel_ms": kt,
            "wall_ms": wall * 1e3, "mrays_per_s": tp.n_rays / (st * 1e-3) / 1e6,
            "segments_per_s": work["queries"] / (st * 1e-3), "work": work, "roofline": roof,
            "synth": {"cube": "192 ch x 128 chirps x 256 samples, exact model",
                      "path_samples": ps, "auto_ms": syn["auto"], "direct_ms": syn["direct"],
                      "gpath_samples_per_s_auto": ps / (syn["auto"] * 1e-3) / 1e9,
                      "gpath_samples_per_s_direct": ps / (syn["direct"] * 1e-3) / 1e9}}


def run_street_trace(args):
    """Only the street trace leg (for profiling the tracer)."""
    import paper_2307_15412_amd as rr
    ctx = rr.Context(0)
    print(json.dumps(street_trace(ctx, None, args, reps=args.steps)))


def profiled_traffic(kernel_src: str, summary: str):
    """HBM bytes per launch recorded in a committed rocprofv3 summary, if that
    summary was taken on the current source of the kernel (else None)."""
    import hashlib
    try:
        src = open(os.path.join(ROOT, kernel_src), "rb").read()
        txt = open(os.path.join(ROOT, summary)).read()
    except OSError:
        return None
    sha = hashlib.sha256(src).hexdigest()[:16]
    vals = {}
    for line in txt.splitlines():
        line = line.strip()
        if ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != sha or "traffic_bytes_per_launch" not in vals:
        return None
    return float(vals["traffic_bytes_per_launch"])


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def main():
    args = parse()
    if args.mfma_calibration:
        mfma_calibration()
        return
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch":
        run_batch(args)
        return
    if args.workload == "proposal":
        run_proposal(args)
        return
    if args.workload == "tri_cast":
        run_tri_cast(args)
        return
    if args.workload == "hand_motion":
        run_hand_motion(args)
        return
    if args.workload == "street_trace":
        run_street_trace(args)
        return
    if args.workload == "mlp":
        run_mlp(args)
        return
    if args.workload in ("hand", "alpha_sweep"):
        run_hand(args, sweep=args.workload == "alpha_sweep")
        return
    import torch
    import scenegen as sg
    import paper_2307_15412_amd as rr

    w = sg.workload_large_mimo(0)
    if args.rays:
        w.trace.n_rays = args.rays
    C, M, K = w.array.n_ch, w.chirp.n_chirps, w.chirp.n_samples
    ctx = rr.Context(0)
    t0 = time.time()
    ctx.setup(w)
    bvh_s = time.time() - t0
    engine = {"auto": rr.ENGINE_AUTO, "gemm": rr.GEMM_BF16X3, "direct": rr.DIRECT_FP32}[args.engine]
    model = rr.SEPARABLE
    cube = torch.empty((C, M, K), dtype=torch.complex64, device="cuda:0")

    def step():
        n = ctx.trace_workload(w, record_hits=False)
        ctx.synthesize(model=model, engine=engine, out=cube)
        return n

    if engine == rr.ENGINE_AUTO:
        # the library's own choice for the separable model: the GEMM engine
        # when its 64-sample tiling pads a chirp by at most a quarter
        engine = rr.GEMM_BF16X3 if 4 * (-(-K // 64) * 64) <= 5 * K else rr.DIRECT_FP32
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    trace_ms, synth_ms = [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        P = step()
        trace_ms.append(ctx.kernel_ms(0))
        synth_ms.append(ctx.kernel_ms(1))
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    n_rays = w.trace.n_rays
    path_samples = float(P) * C * M * K
    value = path_samples / dt / 1e9
    tr = float(np.mean(trace_ms))
    sy = float(np.mean(synth_ms))
    eng_name = "gemm_bf16x3" if engine == rr.GEMM_BF16X3 else "direct_fp32"
    if sy >= tr:
        kern_flops = path_samples * FLOPS_PER_PATH_SAMPLE
        ach = kern_flops / (sy * 1e-3) / 1e12
        if engine == rr.GEMM_BF16X3:
            roof = {"bound": "mfma", "achieved": ach, "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "traffic": profiled_traffic("paper_2307_15412_amd/csrc/k_gemm.hip",
                                                "profiles/k_gemm_large_mimo.md")}
        else:
            roof = {"bound": "alu", "achieved": ach, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "traffic": profiled_traffic("paper_2307_15412_amd/csrc/k_synth.hip",
                                                "profiles/k_synth_direct_large_mimo.md")}
        roof["kernel"] = "synth_" + eng_name
        roof["flops_per_launch"] = kern_flops
    else:
        # tracer bytes per segment are counted by the profile; report the rate only
        roof = {"bound": "hbm", "achieved": None, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "kernel": "trace", "traffic": None}
    if roof["achieved"] is not None:
        roof["frac"] = roof["achieved"] / roof["peak"]
    else:
        roof["frac"] = None

    # the timed cube (GPU trace, then synthesis) against the FP64 oracle on
    # 4096 seeded entries: the oracle traces the same rays and keeps the same
    # first paths in (ray, bounce) order; its own time on that work is the
    # CPU baseline
    rel = max_ratio = None
    cpu = None
    if not args.no_check or not args.no_cpu_baseline:
        import oracle
        idx = np.random.default_rng(11).choice(C * M * K, 4096, replace=False)
        got = cube.reshape(-1)[torch.from_numpy(idx).to(cube.device)].cpu().numpy()
        t0 = time.perf_counter()
        _, op = oracle.trace(w.scene, w.array, w.trace, want_hits=False)
        t_trace = time.perf_counter() - t0
        op = op[: w.path_cap]
        t0 = time.perf_counter()
        ref = oracle.synth(op, w.scene, w.array, w.chirp, model=1, idx=idx)
        t_syn = time.perf_counter() - t0
        if not args.no_check:
            if len(op) != int(P):
                raise SystemExit(f"path count differs from the oracle: {P} vs {len(op)}")
            d = got - ref
            rel = float(np.linalg.norm(d) / np.linalg.norm(ref))
            max_ratio = float(np.abs(d).max() / np.abs(ref).max())
        if not args.no_cpu_baseline:
            t_full = t_trace + t_syn * (path_samples / (len(op) * len(idx)))
            cpu = {"value": path_samples / t_full / 1e9, "unit": "Gpath-samples/s", "cores": 1,
                   "kind": "oracle",
                   "sample": f"single-threaded FP64 oracle: trace of all {n_rays} rays "
                             f"({t_trace:.2f} s, BVH build included) and {len(idx)} sampled cube "
                             f"entries over the first {len(op)} paths ({t_syn:.2f} s), the "
                             f"synthesis scaled to {P} x {C} x {M} x {K} path-samples; host "
                             f"{cpu_model()}, nproc {os.cpu_count()}"}
    c2 = None if args.no_street else street_trace(ctx, w.scene, args)
    out = {
        "metric": "Mrays/s + Gpath-samples/s synthesized at 3072 ch; cube rel err vs FP64",
        "value": value, "unit": "Gpath-samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64-phase/" + ("bf16x3" if engine == rr.GEMM_BF16X3 else "f32"),
        "data": "synthetic (procedural street, seeded)",
        "config": {"workload": "large_mimo: street 5.1e5 tris, 48Tx x 64Rx shared launch, "
                               f"{n_rays} rays, <=3 bounces, first {w.path_cap} paths, "
                               f"{C} ch x {M} chirps x {K} samples, separable model",
                   "engine": eng_name, "paths": P, "rays": n_rays},
        "mrays_per_s": n_rays / (tr * 1e-3) / 1e6, "trace_ms": tr, "synth_ms": sy,
        "bvh_build_s": bvh_s, "cube_rel_err": rel, "cube_max_err_ratio": max_ratio,
        "cube_check": "4096 seeded entries of the timed cube vs the FP64 oracle's separable model "
                      "over its own paths for the same rays",
        "mrays_per_s_c2": c2["mrays_per_s"] if c2 else None,
        "segments_per_s_c2": c2["segments_per_s"] if c2 else None,
        "roofline": roof, "roofline_trace": c2["roofline"] if c2 else None,
        "trace_c2": c2, "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
