#!/usr/bin/env python
"""Throughput of one render-and-compare refinement iteration on one MI355X.

Workload (synthetic stand-in for an InterHand2.6M-like multiframe): one
procedural skinned hand seen by 8 calibrated cameras of 334x512 pixels on a
0.6-0.9 m shell, 16 camera samples per pixel, a 512x512 RGB colour map, target
images rendered from the true parameters at 64 samples per pixel, L1 loss over
hand masks, Adam on the 64 hand parameters and the colour map.

A step is one full iteration: skin -> render (vertex normals, BVH refit, screen
bounds, ray tracing) -> L1 loss -> backward (interior adjoint, silhouette edge
sampling, normals + skinning backward) -> Adam.  Inputs are resident in HBM
before the timed region.  Iterations 0..49 optimise the colour map only (the
warm-up phase of the paper's schedule) and always run untimed, whatever
--warmup asks for (more if it asks for more), so the timed steps are
iterations of the all-variables phase.

Prints one JSON line: the metric, per-kernel times, the roofline of the render launch and the CPU baseline.
"""
import argparse
import dataclasses
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2107_05509_amd import binding, refine, scene  # noqa: E402

METRIC = "fwd+bwd diff-render Mrays/s + refine iters/s (8 views 334x512, 16 spp)"
CAL_FLOATS = 1 << 27   # calibration copy: 512 MiB in, 512 MiB out
# Published MI355X FP32 vector peak.  It counts packed FP32: 256 CUs x 64 lanes
# (4 SIMDs of 16 lanes, a wave64 instruction every 4 cycles) x 2 FMAs per lane
# and cycle (v_pk_fma_f32) x 2 FLOP x 2.4 GHz.  This library is compiled without
# packed FP32, so its own ceiling is half of it (78.6 TFLOP/s of FMAs, or 39.3 T
# lane operations/s of any other VALU instruction); the fraction is reported
# against the published figure.
PEAK_FP32_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0

# Algorithmic FLOP per unit of ray-tracing work, the per-unit figures of the
# hot-path measurement plan: per ray (Philox share and ray set-up), per node
# visit of the ray's own traversal (two child slab tests), per ray/triangle
# test of the ray's own traversal (watertight test), per hit (shading; the
# interior adjoint adds 100 for the hit-point derivative and the chain rule)
OPS_PER_RAY = 20
OPS_PER_NODE = 24
OPS_PER_TRI = 40
OPS_PER_HIT = {"k_render": 70, "k_adjoint_interior": 170, "k_edge_sample": 70}


def kernel_source_hash():
    from paper_2107_05509_amd.build import source_hash
    return source_hash()


def make_refiner(w, dev="cuda:0", seed=0, tune=True, cover_spp=64):
    """Scene, synthetic targets (true parameters, 64 samples per pixel, an
    independent sample key), coverage masks (samples of a cover_spp render of
    the true pose) and the loop buffers; hierarchy built at the initial pose;
    launch grids tuned.  Set-up, never timed."""
    th, tw = w.albedo_true.shape[1:3]
    g = binding.Scene(w.model, w.cams, w.n_hands, w.spp, th, tw, seed=1000 + seed)
    t = lambda a, dt=torch.float32: torch.as_tensor(np.ascontiguousarray(a)).to(dev, dt)
    bg = t(w.packed_background().astype(np.float32))
    gt = binding.Scene(w.model, w.cams, w.n_hands, 64, th, tw, seed=7000 + seed)
    vt = torch.empty(w.n_hands, w.model.n_verts, 3, device=dev)
    gt.skin(t(w.params_true.astype(np.float32)), vt)
    gt.build_hierarchy(vt)
    target = torch.empty(g.P, 3, device=dev)
    alb_true = t(w.albedo_true.astype(np.float32))
    if cover_spp >= 64:
        hits = torch.empty(g.P, 64, device=dev, dtype=torch.int32)
        gt.render(vt, alb_true, bg, 0, target, hits)
    else:
        gt.render(vt, alb_true, bg, 0, target)
        gc = binding.Scene(w.model, w.cams, w.n_hands, cover_spp, th, tw, seed=7500 + seed)
        gc.skin(t(w.params_true.astype(np.float32)), vt)
        gc.build_hierarchy(vt)
        hits = torch.empty(g.P, cover_spp, device=dev, dtype=torch.int32)
        gc.render(vt, alb_true, bg, 0, torch.empty_like(target), hits)
        del gc
    mask = refine.coverage_mask(hits, w.cams, w.pixel_offsets(), 9)
    del hits, gt, alb_true
    r = refine.Refiner(g, t(w.params_init.astype(np.float32)), t(w.albedo_init.astype(np.float32)), bg, target,
                       mask, warm=50, graph_chunk=50)
    r.build_hierarchy()
    if tune:
        r.tune(reps=10)
    return r


def cpu_baseline(w, views=1):
    """The oracle (float64, brute force, OpenMP) on the first `views` views of the
    same workload: forward render + loss + interior adjoint + edge term, and
    the per-iteration time that extrapolates to all views (and to the 200
    iterations of a refinement), labelled as an extrapolation."""
    import oracle
    oracle.build(force=False)
    cams = w.cams[:views]
    tab = scene.camera_arrays(cams)
    osc = oracle.Scene(w.model.faces, w.model.uv, tab, scene.SHADING, w.model.edges, w.model.edge_faces)
    om = oracle.Model(w.model)
    P = int(tab["pix_off"][-1])
    p = torch.as_tensor(w.params_init.astype(np.float32).astype(np.float64))
    # host inputs only (nothing the GPU computed): the views' backgrounds,
    # a seeded target of the same shape, every pixel in the mask
    bg = np.asarray(w.packed_background(), np.float64)[:P]
    alb = w.albedo_init.astype(np.float64)
    target = np.clip(bg + np.random.default_rng(7).normal(0.0, 0.1, bg.shape), 0.0, 1.0)
    mask = np.ones(P, np.uint8)
    t0 = time.perf_counter()
    v, _ = oracle.skin(om, p)
    n = oracle.vertex_normals(v, om.faces)
    v, n = v.numpy(), n.numpy()
    img = oracle.render(osc, v, n, alb, bg, w.spp, 1000, 60)
    _, dimg = oracle.l1_loss(img, target, mask, tab["pix_off"], tab["hand"], 1)
    oracle.backward_interior(osc, v, n, alb, dimg, w.spp, 1000, 60)
    oracle.backward_edges(osc, v, n, alb, bg, dimg, 1000, 60)
    dt = time.perf_counter() - t0
    samples = P * w.spp
    s_iter = dt * len(w.cams) / views
    return {"value": samples / dt / 1e6, "unit": "Mrays/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{views} of {len(w.cams)} views ({cams[0].W}x{cams[0].H}), {w.spp} spp: forward render, "
                      f"loss, interior adjoint and edge term, float64 brute force; {dt:.1f} s",
            "seconds": dt,
            "extrapolated_s_per_iteration": round(s_iter, 2),
            "extrapolated_min_per_200_iterations": round(s_iter * 200 / 60, 1),
            "extrapolation": f"linear in views: {views} measured -> {len(w.cams)}"}


def timed(fn):
    """Milliseconds of the work fn enqueues, bracketed by synchronisations."""
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    fn()
    stop.record()
    torch.cuda.synchronize()
    return start.elapsed_time(stop)


def bench_batched(args):
    """Many hands per launch: per-iteration latency percentiles of graph-replayed
    iterations (one graph launch per iteration, events between launches)."""
    w = scene.workload_batched(args.seed)
    print(f"[bench] workload: {w.name}, {len(w.cams)} views, {w.n_pixels} pixels", file=sys.stderr, flush=True)
    ref = make_refiner(w, seed=args.seed, tune=not args.no_tune, cover_spp=4)
    ref.chunk = 1
    g = ref.scene
    warm, steps = min(args.warmup, 5), min(args.steps, 30)
    ref.warm = 0                      # all variables from the first iteration
    ref.run(warm)
    ref.prepare_graphs(steps)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record()
    for i in range(steps):
        ref.run(1)
        ev[i + 1].record()
    torch.cuda.synchronize()
    lat = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(steps)])
    ms = float(lat.mean())
    cam_samples = w.n_pixels * w.spp
    g.set_counting(True)
    ref.step()
    counts = g.read_counts()
    g.set_counting(False)
    traced = sum(int(counts[k][0]) for k in counts)
    out = {
        "metric": "batched refine: camera samples/s and per-iteration latency (64 hands, 8 spp)",
        "value": round(cam_samples / (ms * 1e-3) / 1e6, 2), "unit": "Mrays/s", "n_gpus": 1,
        "steps": steps, "warmup": warm, "ms_per_step": round(ms, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": w.name + ": views U{4..40} per hand, 128x128/256x256/334x512, 256x256 albedo",
                   "hands": w.n_hands, "views": len(w.cams), "pixels": int(w.n_pixels), "spp": w.spp,
                   "camera_samples_per_step": int(cam_samples)},
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3), "p99": round(float(np.percentile(lat, 99)), 3),
                       "max": round(float(lat.max()), 3)},
        "refine_iters_per_s": round(1e3 / ms, 3),
        "hand_iters_per_s": round(w.n_hands * 1e3 / ms, 1),
        "traced_mrays_per_s": round(traced / (ms * 1e-3) / 1e6, 2),
        "launch_grids": list(g.grids()),
        "loss_mean": round(float(ref.loss.mean().item()), 5),
    }
    print(json.dumps(out), flush=True)


def bench_proposal(args):
    """Learned edge proposal against length-proportional sampling on the
    realistic workload: (1) refinement with the proposal trained online
    (iterations/s), for the learned proposal also at half the edge-sample
    budget (one sample per two pixels of silhouette); (2) at the learned run's
    final pose, the spread of the boundary term's 64-parameter gradient over
    256 sample keys (trace of the covariance over the 61 free parameters; the
    means must agree within their standard errors: unbiasedness), for length
    sampling at the full budget and the learned proposal at the full and at
    half the budget; (3) loss trajectories.  Refine/s at equal variance:
    the learned proposal at the budget whose covariance matches length
    sampling's at the full budget."""
    w = scene.workload_realistic(args.seed)
    n_iter = 200
    out = {"metric": "learned edge proposal: gradient variance ratio and refine iters/s", "unit": "ratio",
           "config": {"workload": w.name, "iterations": n_iter, "seeds": 256}}
    runs = (("length", 256), ("learned", 256), ("learned", 512))
    traj, refs = {}, {}
    for kind, div in runs:
        name = kind if div == 256 else f"{kind}_half_budget"
        ref = make_refiner(w, seed=args.seed, tune=False)
        ref.scene.set_edge_budget(div)
        if kind == "learned":
            ref.scene.proposal_set(binding.HR_PROPOSAL_LEARNED, scene.mlp_init(args.seed), lr=3e-3, ema=0.9)
        ref.run(5)
        torch.cuda.synchronize()
        losses = []
        t0 = time.perf_counter()
        for _ in range(n_iter // 10):
            ref.run(10)
            losses.append(float(ref.loss.item()))
        dt = time.perf_counter() - t0
        traj[name] = losses
        out[f"{name}_iters_per_s"] = round(n_iter / dt, 2)
        refs[name] = ref
        print(f"[bench] {name}: {n_iter / dt:.1f} it/s, loss {losses[-1]:.5f}", file=sys.stderr, flush=True)
    # gradient spread at the learned run's final state
    ref = refs["learned"]
    g_learned = ref.scene
    th, tw = w.albedo_true.shape[1:3]
    g_length = binding.Scene(w.model, w.cams, w.n_hands, w.spp, th, tw, seed=1000 + args.seed)
    q = ref.state
    g_learned.skin(q.params, q.verts)
    g_learned.render(q.verts, q.albedo, q.background, 0, q.image)
    g_learned.loss(q.image, q.target, q.mask, q.loss, q.dimage)
    d = q.dimage.clone()
    gp = torch.empty_like(q.params)
    ga = torch.empty_like(q.albedo)
    res = {}
    for name, g, div in (("length", g_length, 256), ("learned", g_learned, 256), ("learned_half_budget", g_learned, 512)):
        g.set_edge_budget(div)
        rows = []
        for s in range(256):
            g.backward(q.params, q.verts, q.albedo, q.background, d, 5000 + s, gp, ga, flags=binding.HR_GRAD_EDGES)
            rows.append(gp[0].double().cpu().numpy())
        res[name] = np.array(rows)
    g_learned.set_edge_budget(256)
    free = np.r_[3:64]
    mu = {k: v.mean(0) for k, v in res.items()}
    se = {k: v.std(0, ddof=1) / np.sqrt(len(v)) for k, v in res.items()}
    tr = {k: float(np.trace(np.cov(v[:, free].T))) for k, v in res.items()}
    zs = {k: float((np.abs(mu[k] - mu["length"]) / np.sqrt(se[k] ** 2 + se["length"] ** 2 + 1e-300))[free].max())
          for k in ("learned", "learned_half_budget")}
    out["value"] = round(tr["length"] / tr["learned"], 3)
    out["trace_cov"] = tr
    out["variance_ratio_length_over_learned"] = out["value"]
    out["variance_ratio_length_over_learned_half_budget"] = round(tr["length"] / tr["learned_half_budget"], 3)
    out["unbiasedness_max_abs_z"] = {k: round(v, 2) for k, v in zs.items()}
    out["equal_variance_iters_per_s"] = {"length_full_budget": out["length_iters_per_s"],
                                         "learned_half_budget": out["learned_half_budget_iters_per_s"]}
    out["loss"] = traj
    print(json.dumps(out), flush=True)


def bench_raster(args):
    """Ray tracing against hard rasterisation in refinement (Section 4.2.2,
    "Ray tracing vs rasterization"): the same problem (8 views 334x512,
    targets ray traced from the true pose at 64 samples per pixel, coverage
    masks, colour map from 0.5, 50 colour-only iterations then 150 on every
    variable) started ever further from the true pose (finger angles + N(0,
    sigma^2), translation 5 mm x sigma / 0.1), with only the renderer
    changed: the Monte Carlo ray tracer (16 spp, edge samples) or hard
    rasterisation (one sample at each pixel centre, no visibility
    gradient).  Error = mean distance between the refined and the true
    vertices."""
    sigmas = (0.05, 0.1, 0.2, 0.3)
    seeds = tuple(range(args.seed, args.seed + 3))
    n_iter = 200
    dev = "cuda:0"
    t = lambda a, dt=torch.float32: torch.as_tensor(np.ascontiguousarray(a)).to(dev, dt)
    rows = []
    for seed in seeds:
        w = scene.workload_realistic(seed)
        base = make_refiner(w, seed=seed, tune=False)   # targets and masks
        target, mask, bg = base.state.target, base.state.mask, base.state.background
        gref = base.scene
        vtrue = torch.empty(1, gref.V, 3, device=dev)
        gref.skin(t(w.params_true.astype(np.float32)), vtrue)
        th, tw = w.albedo_true.shape[1:3]
        for sigma in sigmas:
            p0 = scene.perturb_params(w.params_true[0], np.random.default_rng([seed, int(sigma * 1000), 31]),
                                      sigma, 5.0 * sigma / 0.1)[None].astype(np.float32)
            v0 = torch.empty_like(vtrue)
            gref.skin(t(p0), v0)
            e0 = float((v0 - vtrue).norm(dim=-1).mean()) * 1e3
            row = {"seed": seed, "sigma": sigma, "initial_error_mm": round(e0, 3)}
            for kind in ("ray", "raster"):
                spp = w.spp if kind == "ray" else 1
                g = binding.Scene(w.model, w.cams, 1, spp, th, tw, seed=1000 + seed)
                if kind == "raster":
                    g.set_renderer(binding.HR_RENDERER_RASTER)
                r = refine.Refiner(g, t(p0), t(w.albedo_init.astype(np.float32)), bg, target, mask, warm=50,
                                   graph_chunk=50)
                r.build_hierarchy()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                r.run(n_iter)
                torch.cuda.synchronize()
                dt = (time.perf_counter() - t0) / n_iter
                v = torch.empty_like(vtrue)
                g.skin(r.params, v)
                err = float((v - vtrue).norm(dim=-1).mean()) * 1e3
                row[kind] = {"error_mm": round(err, 3), "loss": round(float(r.loss.item()), 5),
                             "ms_per_iteration": round(dt * 1e3, 4)}
                del r, g
            rows.append(row)
            print(f"[bench] seed {seed} sigma {sigma}: initial {e0:.2f} mm, ray {row['ray']['error_mm']:.2f} mm, "
                  f"raster {row['raster']['error_mm']:.2f} mm", file=sys.stderr, flush=True)
        del base
    summary = {}
    for sigma in sigmas:
        rs = [r for r in rows if r["sigma"] == sigma]
        summary[str(sigma)] = {k: round(float(np.mean([r[k]["error_mm"] for r in rs])), 3) for k in ("ray", "raster")}
        summary[str(sigma)]["initial"] = round(float(np.mean([r["initial_error_mm"] for r in rs])), 3)
    out = {"metric": "ray tracing vs hard rasterisation: mean vertex error after 200 refinement iterations",
           "unit": "mm", "higher_is_better": False, "n_gpus": 1,
           "config": {"workload": "realistic 8x334x512; ray: 16 spp + edge samples; raster: 1 sample at each pixel "
                                  "centre", "iterations": n_iter, "seeds": list(seeds), "sigmas": list(sigmas)},
           "mean_error_mm": summary, "runs": rows}
    print(json.dumps(out), flush=True)


def bench_coverage(args):
    """Camera-coverage ordering (Eq. 6) on 40 views 334x512 at 16 spp: faces seen
    per view from the render's hit ids, then each hand's greedy view order."""
    w = scene.workload_realistic(args.seed, n_views=40)
    print(f"[bench] workload: coverage, {len(w.cams)} views, {w.n_pixels} pixels", file=sys.stderr, flush=True)
    dev = "cuda:0"
    th, tw = w.albedo_true.shape[1:3]
    g = binding.Scene(w.model, w.cams, w.n_hands, w.spp, th, tw, seed=args.seed)
    t = lambda a, dt=torch.float32: torch.as_tensor(np.ascontiguousarray(a)).to(dev, dt)
    verts = torch.empty(w.n_hands, w.model.n_verts, 3, device=dev)
    g.skin(t(w.params_init), verts)
    img = torch.empty(g.P, 3, device=dev)
    hits = torch.empty(g.P, w.spp, dtype=torch.int32, device=dev)
    g.render(verts, t(w.albedo_true), t(w.packed_background()), 0, img, hits)
    vis = torch.empty(len(w.cams), g.F, dtype=torch.int32, device=dev)
    order = torch.empty(len(w.cams), dtype=torch.int32, device=dev)
    covered = torch.empty_like(order)

    def once():
        g.face_visibility(hits, vis)
        g.camera_order(vis, order, covered)

    for _ in range(3):
        once()
    reps = max(1, min(args.steps, 50))
    g.timing_enable(True)
    g.timing_read()
    ms = timed(lambda: [once() for _ in range(reps)]) / reps
    k = g.timing_read()
    g.timing_enable(False)
    per = {n: round(v / max(c, 1) * 1e3, 2) for n, (v, c) in k.items()}
    samples = g.P * w.spp
    vis_us = per.get("k_face_visibility", float("nan"))
    achieved = samples * 4 / (vis_us * 1e-6) / 1e9
    cov = covered.cpu().numpy()
    out = {
        "metric": "camera-coverage ordering time (40 views 334x512, 16 spp)",
        "value": round(ms, 4), "unit": "ms", "n_gpus": 1, "steps": reps, "warmup": 3, "ms_per_step": round(ms, 4),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "i32", "data": "synthetic",
        "config": {"workload": "coverage: 1 hand, 40 views 334x512, 16 spp hit ids (109.4 M samples)",
                   "views": len(w.cams), "samples": int(samples)},
        "kernels": per, "kernels_unit": "us per launch",
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": 8000.0, "unit": "GB/s",
                     "frac": round(achieved / 8000.0, 4), "traffic": None, "kernel": "k_face_visibility",
                     "bytes_per_launch": int(samples * 4)},
        "order": order.cpu().numpy().tolist(), "covered": cov.tolist(),
        "faces_seen_by_7": int(cov[6]), "faces_seen_by_all": int(cov[-1]),
    }
    print(json.dumps(out), flush=True)


def oracle_phases(w, iters=10):
    """The oracle's refinement of the small case, `iters` iterations from the
    initial parameters, each timed per phase (skinning with vertex normals,
    render, loss, backward: interior and edge terms and the chain through the
    normals and the skinning, Adam step); host-made inputs only (target: the
    oracle's own render of the true parameters at 16 samples per pixel)."""
    import oracle
    oracle.build(force=False)
    tab = scene.camera_arrays(w.cams)
    osc = oracle.Scene(w.model.faces, w.model.uv, tab, scene.SHADING, w.model.edges, w.model.edge_faces)
    om = oracle.Model(w.model)
    P = int(tab["pix_off"][-1])
    bg = np.asarray(w.packed_background(), np.float64)
    vt, _ = oracle.skin(om, torch.as_tensor(w.params_true.astype(np.float64)))
    vt = vt.numpy()
    target = oracle.render(osc, vt, oracle.vertex_normals(torch.as_tensor(vt), om.faces).numpy(),
                           w.albedo_true.astype(np.float64), bg, 16, 7000, 0)
    mask = np.ones(P, np.uint8)
    params = w.params_init.astype(np.float32).astype(np.float64)
    alb = w.albedo_init.astype(np.float64)
    mp, vp, ma, va = np.zeros_like(params), np.zeros_like(params), np.zeros_like(alb), np.zeros_like(alb)
    lr = np.zeros(64)
    lr[0:3], lr[3:48], lr[48:58], lr[58:61], lr[61:64] = refine.LR_ALL[:5]
    ph = {k: 0.0 for k in ("skin", "render", "loss", "backward", "step")}
    for it in range(iters):
        t0 = time.perf_counter()
        p = torch.as_tensor(params).requires_grad_(True)
        verts, _ = oracle.skin(om, p)
        normals = oracle.vertex_normals(verts, om.faces)
        v_np, n_np = verts.detach().numpy(), normals.detach().numpy()
        t1 = time.perf_counter()
        img = oracle.render(osc, v_np, n_np, alb, bg, w.spp, 1000, it)
        t2 = time.perf_counter()
        _, dimg = oracle.l1_loss(img, target, mask, tab["pix_off"], tab["hand"], w.n_hands)
        t3 = time.perf_counter()
        ga, gv, gn = oracle.backward_interior(osc, v_np, n_np, alb, dimg, w.spp, 1000, it)
        gv = gv + oracle.backward_edges(osc, v_np, n_np, alb, bg, dimg, 1000, it)
        torch.autograd.backward([verts, normals], [torch.as_tensor(gv), torch.as_tensor(gn)])
        gp = p.grad.numpy()
        t4 = time.perf_counter()
        params, mp, vp = oracle.adam_step(params, gp, mp, vp, it + 1, lr)
        alb, ma, va = oracle.adam_step(alb, ga, ma, va, it + 1, refine.LR_ALL[5], lo=0.0, hi=1.0)
        t5 = time.perf_counter()
        for k, a, b in (("skin", t0, t1), ("render", t1, t2), ("loss", t2, t3), ("backward", t3, t4),
                        ("step", t4, t5)):
            ph[k] += b - a
    total = sum(ph.values())
    return {"value": round(iters / total, 3), "unit": "iters/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"all {iters} iterations of the small case, float64 brute force; {total:.2f} s",
            "seconds": round(total, 3), "seconds_per_phase": {k: round(v, 4) for k, v in ph.items()}}


def bench_tiny(args):
    """The small case (1 hand, 4 views 64x64, 4 spp, 64x64 colour map; a
    refinement of 10 iterations): the GPU's time for the 10 iterations (one
    graph launch, every variable from the first iteration, repeated from the
    initial state) beside the oracle's 10 iterations timed per phase on the
    host cores."""
    w = scene.workload_tiny(args.seed)
    print(f"[bench] workload: {w.name}, {w.n_pixels} pixels", file=sys.stderr, flush=True)
    ref = make_refiner(w, seed=args.seed, tune=False, cover_spp=64)
    ref.warm = 0
    ref.chunk = 10
    q = ref.state
    start = {k: getattr(q, k).clone() for k in ("params", "albedo")}

    def restart():
        # every timed refinement starts from the initial state
        for k, v in start.items():
            getattr(q, k).copy_(v)
        for t in (q.m_params, q.v_params, q.m_albedo, q.v_albedo, q.iter):
            t.zero_()
        ref.it = 0

    ref.run(10)                         # captures the graph
    reps = max(1, min(args.steps, 100))
    ms = []
    for _ in range(reps + 2):
        restart()
        ms.append(timed(lambda: ref.run(10)))
    ms10 = float(np.mean(ms[2:]))
    samples = w.n_pixels * w.spp
    out = {
        "metric": "small case: refine iterations/s (4 views 64x64, 4 spp, 10 iterations)",
        "value": round(10 / (ms10 * 1e-3), 1), "unit": "iters/s", "n_gpus": 1, "steps": 10 * reps, "warmup": 30,
        "ms_per_step": round(ms10 / 10, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "tiny: 1 hand, 4 views 64x64, 4 spp, 64x64 albedo", "views": len(w.cams),
                   "camera_samples_per_step": int(samples)},
        "ms_per_10_iterations": round(ms10, 4), "repetitions": reps,
        "camera_msamples_per_s": round(samples / (ms10 / 10 * 1e-3) / 1e6, 1),
    }
    if not args.no_cpu_baseline:
        print("[bench] oracle: 10 iterations, per phase ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = oracle_phases(w, 10)
    print(json.dumps(out), flush=True)


def bench_adam(args):
    """The colour-map Adam step as a streaming pass (hr_step, k_adam): 4 hands
    x 2048 x 2048 x 3 entries, each step reading the map, its gradient and
    both moments and writing the map and the moments (28 B per entry)."""
    w = scene.workload_tiny(args.seed)
    H, T = 4, 2048
    cams = []
    for h in range(H):
        c = dataclasses.replace(w.cams[0], hand=h)
        cams.append(c)
    g = binding.Scene(w.model, cams, H, 1, T, T, seed=0)
    gen = torch.Generator(device="cuda").manual_seed(args.seed)
    p = torch.zeros(H, 64, device="cuda")
    gp = torch.rand(H, 64, device="cuda", generator=gen)
    mp, vp = torch.zeros_like(p), torch.zeros_like(p)
    a = torch.rand(H, T, T, 3, device="cuda", generator=gen)
    ga = torch.rand(H, T, T, 3, device="cuda", generator=gen) - 0.5
    ma, va = torch.zeros_like(a), torch.zeros_like(a)
    lrs = (1e-2,) * 6
    for i in range(5):
        g.step(p, a, gp, ga, mp, vp, ma, va, i + 1, lrs)
    reps = max(1, min(args.steps, 100))
    ms = timed(lambda: [g.step(p, a, gp, ga, mp, vp, ma, va, i + 6, lrs) for i in range(reps)]) / reps
    nbytes = a.numel() * 28 + 64 * H * 28
    out = {
        "metric": "colour-map Adam streaming pass (4 hands x 2048x2048x3)",
        "value": round(nbytes / (ms * 1e-3) / 1e9, 1), "unit": "GB/s", "n_gpus": 1, "steps": reps, "warmup": 5,
        "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "adam: 4 hands, 2048x2048x3 colour map each (50.3 M entries)", "entries": a.numel()},
        "roofline": {"bound": "hbm", "achieved": round(nbytes / (ms * 1e-3) / 1e9, 1), "peak": 8000.0, "unit": "GB/s",
                     "frac": round(nbytes / (ms * 1e-3) / 1e9 / 8000.0, 4), "traffic": None, "kernel": "k_adam",
                     "bytes_per_launch": int(nbytes)},
    }
    print(json.dumps(out), flush=True)


def bench_full(args):
    """The paper's full data term on the realistic workload: colour transforms,
    two-level colour map, blurred-Canny edge term beside the colour term
    (refine.FullRefiner, eager enqueue); iterations of the all-variables
    phase timed after the 50-iteration warm-up on {T, V_low}."""
    w = scene.workload_realistic(args.seed)
    print(f"[bench] workload: full data term, {w.name}", file=sys.stderr, flush=True)
    base = make_refiner(w, seed=args.seed, tune=not args.no_tune)
    g = base.scene
    st = base.state
    r = refine.FullRefiner(g, st.params, st.background, st.target, st.mask, warm=50)
    n_warm = max(args.warmup, r.warm)
    r.run(n_warm)
    torch.cuda.synchronize()
    steps = min(args.steps, 50)
    g.timing_enable(True)
    g.timing_read()
    ms = timed(lambda: r.run(steps)) / steps
    kern = g.timing_read()
    g.timing_enable(False)
    per = {k: round(v[0] / v[1] * 1e3, 2) for k, v in kern.items()}
    cam = sum(c.W * c.H for c in w.cams) * w.spp
    out = {"metric": "full data term refine iteration (8 views 334x512, 16 spp, colour transforms, "
                     "8x8 + 512x512 colour map, blurred-Canny edge term)",
           "value": round(1e3 / ms, 2), "unit": "iters/s", "n_gpus": 1, "steps": steps, "warmup": n_warm,
           "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32 render, f64 data term", "data": "synthetic",
           "config": {"workload": "realistic with the full data term", "camera_samples_per_step": cam},
           "kernels_us": per, "loss": [round(float(x), 5) for x in r.loss.cpu()],
           "data_term_us": round(sum(v for k, v in per.items() if k.startswith("k_dt_")), 1)}
    print(json.dumps(out), flush=True)


def dense_iteration(args):
    """fwd+bwd time of one iteration of the dense workload (one hand, 40 views
    334x512, 4 spp, 1024x1024 colour map): graph-replayed iterations of the
    all-variables phase, fixed launch grids (untuned, the benchmark's own)."""
    w = scene.workload_dense(args.seed)
    ref = make_refiner(w, seed=args.seed, tune=False, cover_spp=4)
    g = ref.scene
    g.set_grid(4096, 4096)
    ref.run(ref.warm)
    steps = 20
    ref.prepare_graphs(steps)
    ms = timed(lambda: ref.run(steps)) / steps
    samples = sum(c.W * c.H for c in w.cams) * w.spp
    out = {"workload": "dense: 1 hand, 40 views 334x512, 4 spp, 1024x1024 albedo", "steps": steps,
           "ms_per_iteration": round(ms, 4), "refine_iters_per_s": round(1e3 / ms, 2),
           "camera_samples_per_step": int(samples), "camera_msamples_per_s": round(samples / (ms * 1e-3) / 1e6, 1),
           "launch_grids": list(g.grids())}
    del ref, g
    torch.cuda.synchronize()
    return out


def bench_dense(args):
    """The dense workload alone (1 hand, 40 views 334x512, 4 spp, 1024x1024
    colour map): one JSON line with its iteration time."""
    print("[bench] workload: dense, 40 views 334x512, 4 spp", file=sys.stderr, flush=True)
    d = dense_iteration(args)
    ms = d["ms_per_iteration"]
    out = {"metric": "dense: fwd+bwd refine iterations/s (40 views 334x512, 4 spp, 1024x1024 albedo)",
           "value": d["refine_iters_per_s"], "unit": "iters/s", "n_gpus": 1, "steps": d["steps"], "warmup": 50,
           "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic", "config": {"workload": d["workload"], "views": 40, "spp": 4,
                                           "camera_samples_per_step": d["camera_samples_per_step"]},
           "camera_msamples_per_s": d["camera_msamples_per_s"], "launch_grids": d["launch_grids"]}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=150)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--mode", choices=("graph", "eager"), default="graph",
                    help="graph: replay captured iterations (hr_graph); eager: one hr_iterate per iteration")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--grids", default=None,
                    help="R,A: persistent render/adjoint grid sizes to use instead of tuning")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--joint-prior", action="store_true",
                    help="add the joint prior (lambda 1, gamma 5 mm) against the true joints plus 5 mm noise")
    ap.add_argument("--cpu-views", type=int, default=2)
    ap.add_argument("--no-dense", action="store_true",
                    help="skip the dense-workload iteration time (40 views, 4 spp, 1024x1024 albedo)")
    ap.add_argument("--workload",
                    choices=("realistic", "batched", "proposal", "coverage", "full", "raster", "adam", "tiny", "dense"),
                    default="realistic",
                    help="batched: 64 hands, 4-40 views each at 128x128/256x256/334x512, 8 spp "
                         "(per-iteration latency percentiles; not the headline metric)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the workload would shard by hand or by view, one all-reduce of the gradients per iteration)", file=sys.stderr)
        sys.exit(2)
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.workload == "batched":
        return bench_batched(args)
    if args.workload == "proposal":
        return bench_proposal(args)
    if args.workload == "coverage":
        return bench_coverage(args)
    if args.workload == "full":
        return bench_full(args)
    if args.workload == "raster":
        return bench_raster(args)
    if args.workload == "adam":
        return bench_adam(args)
    if args.workload == "tiny":
        return bench_tiny(args)
    if args.workload == "dense":
        return bench_dense(args)
    w = scene.workload_realistic(args.seed)
    print(f"[bench] workload: {w.name}, {w.n_pixels} pixels", file=sys.stderr, flush=True)
    ref = make_refiner(w, seed=args.seed, tune=not (args.no_tune or args.grids))
    g = ref.scene
    if args.joint_prior:
        # target joints: the true pose's joints with seeded 5 mm noise (an initial joint estimate)
        jt = torch.empty(w.n_hands, g.J, 3, device="cuda:0")
        g.skin(torch.as_tensor(w.params_true, dtype=torch.float32).to("cuda:0").contiguous(),
               torch.empty(w.n_hands, g.V, 3, device="cuda:0"), jt)
        gen = torch.Generator().manual_seed(args.seed + 17)
        jt += (0.005 * torch.randn(jt.shape, generator=gen)).to(jt.device)
        g.set_joint_prior(jt.contiguous(), 1.0, 0.005)
    if args.grids:
        g.set_grid(*[int(x) for x in args.grids.split(",")])
    print(f"[bench] launch grids (render, adjoint): {g.grids()}, tiles (w, h, bin) log2: {g.tiles()}",
          file=sys.stderr, flush=True)
    graph = args.mode == "graph"
    # the colour-only phase (iterations 0..warm-1) always runs untimed
    n_warm = max(args.warmup, ref.warm)
    ref.run(n_warm, graph=graph)
    torch.cuda.synchronize()
    print(f"[bench] warmup done ({n_warm} iterations; timed: iterations {n_warm}..{n_warm + args.steps - 1}, "
          f"all variables)", file=sys.stderr, flush=True)
    # a plain device copy of known size (CAL_FLOATS float32 in and out, far
    # beyond the L2 and last-level caches): profiler runs of this command
    # scale their HBM byte counters by what they read for it
    cal_src = torch.rand(CAL_FLOATS, device="cuda")
    cal_dst = torch.empty_like(cal_src)
    for _ in range(3):
        cal_dst.copy_(cal_src)
    del cal_src, cal_dst
    if graph:
        ref.prepare_graphs(args.steps)   # capture before the timed region
    if not graph:
        g.timing_enable(True)
        g.timing_read()
    total_ms = timed(lambda: ref.run(args.steps, graph=graph))
    ms = total_ms / args.steps
    print(f"[bench] timed {args.steps} steps ({args.mode}): {ms:.4f} ms/step, loss {ref.loss.item():.5f}",
          file=sys.stderr, flush=True)
    eager_ms = None
    if graph:
        # per-kernel durations: HIP events around every launch of the same
        # number of iterations, enqueued one by one right after the timed region
        g.timing_enable(True)
        g.timing_read()
        eager_ms = timed(lambda: ref.run(args.steps, graph=False)) / args.steps
    kern = g.timing_read()
    g.timing_enable(False)
    # work counts of one more iteration (untimed)
    g.set_counting(True)
    ref.step()
    counts = g.read_counts()
    g.set_counting(False)
    tot, bud = g.edge_stats()
    torch.cuda.synchronize()

    cam_samples = sum(c.W * c.H for c in w.cams) * w.spp
    # rays that enter a hierarchy: camera rays of the render, both side rays of
    # every edge sample, rays the adjoint traces again (none: it reads the
    # render's stored hits)
    traced = sum(int(counts[k][0]) for k in counts)
    n_it = args.steps
    per_kernel = {k: {"ms_per_launch": v[0] / v[1], "launches": v[1], "ms_per_step": v[0] / n_it}
                  for k, v in kern.items()}
    for k, v in sorted(per_kernel.items(), key=lambda kv: -kv[1]["ms_per_step"]):
        print(f"[bench]   {k:22s} {v['ms_per_launch'] * 1e3:9.1f} us/launch", file=sys.stderr)
    # roofline of the dominant ray-tracing kernel (the backward launch carries
    # both the interior adjoint and the edge samples)
    dom = max(("k_render", "k_backward_trace"), key=lambda k: per_kernel[k]["ms_per_step"])
    # the render launch also traces the edge samples' side points; the
    # backward launch weighs them (tracing only samples beyond the stored ones)
    parts = ["k_render", "k_edge_sample"] if dom == "k_render" else ["k_adjoint_interior"]
    rays = sum(counts[p][0] for p in parts)
    nodes = sum(counts[p][1] for p in parts)
    tris = sum(counts[p][2] for p in parts)
    hits = sum(counts[p][3] for p in parts)
    nodes_w = sum(counts[p][4] for p in parts)
    tris_w = sum(counts[p][5] for p in parts)
    # the adjoint's samples are counted by their hits (it traces no ray)
    ops = sum(counts[p][0] * OPS_PER_RAY + counts[p][1] * OPS_PER_NODE + counts[p][2] * OPS_PER_TRI
              + counts[p][3] * OPS_PER_HIT[p] for p in parts)
    ach = ops / (per_kernel[dom]["ms_per_launch"] * 1e-3) / 1e12
    traffic = None
    tfile = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tfile):
        tj = json.load(open(tfile))
        if tj.get("source_hash") == kernel_source_hash() and dom in tj.get("kernels", {}):
            traffic = tj["kernels"][dom]
    roof = {"bound": "alu", "achieved": round(ach, 3), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
            "frac": round(ach / PEAK_FP32_TFLOPS, 4), "traffic": traffic, "kernel": dom,
            "kernel_us": round(per_kernel[dom]["ms_per_launch"] * 1e3, 2),
            "ops_per_launch": int(ops), "rays": int(rays), "node_visits": int(nodes), "tri_tests": int(tris),
            "hits": int(hits),
            "flop_per_unit": {"ray": OPS_PER_RAY, "node": OPS_PER_NODE, "tri": OPS_PER_TRI,
                              "hit": {p: OPS_PER_HIT[p] for p in parts}},
            # lane utilisation of the wave-packet traversal: the rays' own
            # node visits / triangle tests over those executed per active lane
            "packet_node_visits": int(nodes_w), "packet_tri_tests": int(tris_w),
            "lane_util_nodes": round(nodes / max(nodes_w, 1), 4),
            "lane_util_tris": round(tris / max(tris_w, 1), 4)}
    out = {
        "metric": METRIC,
        "value": round(cam_samples / (ms * 1e-3) / 1e6, 2),
        "unit": "Mrays/s",
        "n_gpus": 1, "steps": args.steps, "warmup": n_warm, "warmup_requested": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "realistic: 1 hand (778 verts, 1538 tris), 8 views 334x512, 16 spp, "
                               "512x512 albedo, L1 over hand masks, Adam on 64 params + albedo"
                               + (", joint prior (lambda 1, gamma 5 mm)" if args.joint_prior else ""),
                   "views": len(w.cams), "W": 334, "H": 512, "spp": w.spp, "tex": 512,
                   "camera_samples_per_step": cam_samples},
        "mode": args.mode,
        "launch_grids": list(g.grids()),
        "launch_tiles": dict(zip(("tile_w_log2", "tile_h_log2", "bin_log2"), g.tiles())),
        "refine_iters_per_s": round(1e3 / ms, 2),
        "traced_mrays_per_s": round(traced / (ms * 1e-3) / 1e6, 2),
        "edge_samples_per_step": int(bud.sum()),
        "eager_ms_per_step": None if eager_ms is None else round(eager_ms, 4),
        "kernels": {k: round(v["ms_per_launch"] * 1e3, 2) for k, v in per_kernel.items()},
        "work_counts": {k: {"rays": int(v[0]), "node_visits": int(v[1]), "tri_tests": int(v[2]), "hits": int(v[3]),
                            "packet_node_visits": int(v[4]), "packet_tri_tests": int(v[5])}
                        for k, v in counts.items()},
        "kernels_unit": "us per launch",
        "roofline": roof,
    }
    if not args.no_dense:
        print("[bench] dense workload (40 views, 4 spp) ...", file=sys.stderr, flush=True)
        del ref, g
        out["dense"] = dense_iteration(args)
        print(f"[bench] dense: {out['dense']['ms_per_iteration']:.4f} ms/iteration", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_views)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
