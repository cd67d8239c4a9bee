#!/usr/bin/env python
"""Training-step benchmark of the MI355X surfel rasterizer.

Workload: 1 M surfels on a synthetic 1 km^2 aerial city (fBm terrain + 200 box buildings, 5 %
elongated surfels, SH degree 3), 16 aerial cameras at 1600x1066.  One step = one view's
project -> bin/sort -> render_fwd -> L1+SSIM loss -> render_bwd (+ chain to parameters) ->
densify_stats, all through the C ABI on one GPU; steps cycle through the 16 cameras.  The
target of each view is the render of a perturbed copy of the scene (made before timing).

Prints one JSON line: iterations/s (value), Mpix/s, the per-call split, the roofline of the
dominant kernel (algorithmic flops from the counted pixel-entry pairs) and the FP64 CPU oracle
timed on one full view on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3       # MI355X vector FP32 (packed); 78.6 without packed math
PEAK_FP32_NONPACKED = 78.6
PEAK_HBM_GBS = 8000.0
# Algorithmic flops per (pixel, list entry) pair, counted on the oracle's operation list (each add,
# subtract, multiply, divide and exp is one flop; compares and selects none):
#   evaluation (every pair the forward evaluates, every pair the reverse walks): the ray-splat
#     intersection a x b (12 + 9), u, v and rho_3d (5), rho_2d (6), exp(-rho / 2) (2), o G (1) = 35;
#   forward blend per contributing pair: T (1 - alpha) (2), w (1), colour (6), normal (6), intersection
#     depth (4) and its sum (2) = 21;
#   reverse per contributing pair with a colour upstream and the SSIM-only view-space gradient (the
#     timed step's variant): T step (2), w (1), dL/dalpha (18), colour gradient (6), after-sums (6),
#     opacity (2), dL/drho (3), dL/dp (16), dL/da, dL/db (18), rows of M (18), and for the SSIM part
#     dL/dalpha (18), dL/drho (3), dL/dp (16), dL/da, dL/db (18), rows 1-2 of M (6) = 151;
#   contribution pass per contributing pair: T (1 - alpha) (2), alpha^g T^(1-g) (3), sum and count (2) = 7.
F_FWD_EVAL, F_FWD_CON = 35, 21
F_BWD_WALK, F_BWD_CON = 35, 151
F_CON_EVAL, F_CON_CON = 35, 7


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_hash():
    h = hashlib.sha256()
    for f in sorted(os.listdir(os.path.join(ROOT, "paper_2411_00771_amd", "csrc"))):
        with open(os.path.join(ROOT, "paper_2411_00771_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def cpu_baseline(scene, cams, targets, min_seconds=10.0, one_thread=True):
    """The FP64 oracle, as it stands, on whole views of the same workload: on all the host cores (steps
    over the cameras until min_seconds have passed, at most one pass over them), then on one thread
    (one view)."""
    import oracle

    def run(views):
        t0 = time.perf_counter()
        k = 0
        while k < views and (k == 0 or time.perf_counter() - t0 < min_seconds):
            cam, target = cams[k], targets[k]
            proj, off, ids, img = oracle.forward_view(scene, cam)
            lo = oracle.ssim_loss(img["rgb"], target)
            bw = oracle.backward_view(scene, cam, proj, off, ids, dict(d_rgb=lo["d_total"], d_rgb_ssim=lo["d_ssim"]))
            st = oracle.new_densify_state(scene.n)
            oracle.densify_stats(bw["g_total"], bw["g_ssim"], (proj["flags"] & 1) > 0, proj["radius"],
                                 scene.log_scale, st)
            k += 1
        return k, time.perf_counter() - t0

    cores = len(os.sched_getaffinity(0))
    threads = oracle.set_threads(int(os.environ.get("OMP_NUM_THREADS", 0)) or cores)
    k, dt = run(len(cams))
    out = dict(value=k / dt, unit="iters/s", cores=threads, kind="oracle",
               sample=f"{k} full 1600x1066 training steps (views) of the 1M-surfel scene (fwd+loss+bwd, both "
                      f"view-space gradients, densify) on {threads} threads, {dt:.1f} s")
    if one_thread:
        oracle.set_threads(1)
        k1, dt1 = run(1)
        oracle.set_threads(threads)
        out["one_thread"] = dict(value=k1 / dt1, unit="iters/s", cores=1, seconds=round(dt1, 1),
                                 sample="1 full 1600x1066 training step (view 0) on one thread")
    return out


def bench_contribution(eng, params, cams, counts, gamma=0.5, ratio=0.025, reps=3):
    """Trimming pass of Sec. 3.3 over every view of the block: per-view contribution (Eq. 3) into a
    running sum, the average of Eq. 4, and the percentile mask.  Only the contribution calls and the
    trim are timed (the per-view project + bin_sort that provide the bins are not); each view's time is
    its median over the repetitions (a call's events also see any host stall before its launch)."""
    import torch
    from paper_2411_00771_amd import raster
    n = eng.n
    c_sum = torch.zeros(n, device="cuda:0")
    times, flops = [], 0.0
    for rep in range(reps):
        c_sum.zero_()
        for k, c in enumerate(cams):
            eng.project(params, c)
            eng.bin_sort(c)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            eng.contribution(c, gamma, c_sum=c_sum)
            e1.record()
            times.append((rep, k, e0, e1))
            if rep == reps - 1:
                flops += F_CON_EVAL * counts[k][0] + F_CON_CON * counts[k][1]
    c_avg = c_sum / len(cams)
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    bound, mask, removed = raster.trim_mask(c_avg, ratio)
    t1.record()
    torch.cuda.synchronize()
    ms = [float(np.median([a.elapsed_time(b) for r, kk, a, b in times if kk == k])) for k in range(len(cams))]
    per_view = float(np.mean(ms))
    return {"views": len(cams), "gamma": gamma, "ratio": ratio, "ms_per_view": round(per_view, 4),
            "views_per_s": round(1e3 / per_view, 2),
            "tflops": round(flops / (sum(ms) * 1e-3) / 1e12, 3),
            "trim_ms": round(t0.elapsed_time(t1), 4), "removed": int(removed.item()),
            "bound": float(bound.item())}, mask


def camera_extent(cams):
    """Scene extent as the 3DGS family sets it: 1.1 x the largest camera-centre distance from their mean."""
    C = np.array([-np.asarray(c.R, np.float64).reshape(3, 3).T @ np.asarray(c.t, np.float64) for c in cams])
    return 1.1 * float(np.linalg.norm(C - C.mean(0), axis=1).max())


def bench_densify_action(params, cand_mask, trim_mask, dense_scale, reps=5):
    """Densification action on the training step's candidate mask and the trimming mask: the plan, then
    (after the output size is read back) the apply.  Each is event-timed; bytes are the algorithmic ones:
    plan 23 B per surfel (mask, removal, log-scales, logit in; action and two slots out), apply
    9 B per surfel (action, slots) + one read of every surviving surfel + one write of every output
    surfel with its slot-map entry."""
    import torch
    from paper_2411_00771_amd import raster, scenes
    n = params.n
    _, _, z = scenes.densify_inputs(4242, n)
    zt = torch.from_numpy(z).cuda()
    K = (params.sh_degree + 1) ** 2
    surfel_bytes = 4 * (3 + 2 + 4 + 1 + 3 * K)
    t_plan, t_apply = [], []
    plan = raster.densify_plan(params, cand_mask, trim_mask, dense_scale=dense_scale)
    n_out = plan.n_out()
    # outputs allocated once, outside the timed calls (the call itself allocates nothing)
    out, src = raster.densify_apply(params, plan, zt, n_out=n_out)
    for _ in range(reps):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        e[0].record()
        plan = raster.densify_plan(params, cand_mask, trim_mask, dense_scale=dense_scale)
        e[1].record()
        n_out = plan.n_out()
        e[2].record()
        raster.densify_apply(params, plan, zt, n_out=n_out, out=out, src=src)
        e[3].record()
        torch.cuda.synchronize()
        t_plan.append(e[0].elapsed_time(e[1]))
        t_apply.append(e[2].elapsed_time(e[3]))
    del out, src
    cnt = plan.counts.cpu().numpy()
    tp, ta = float(np.median(t_plan)), float(np.median(t_apply))
    b_plan = 23.0 * n
    b_apply = 9.0 * n + surfel_bytes * (n - cnt[3]) + (surfel_bytes + 4) * n_out
    return {"surfels": n, "dense_scale": round(dense_scale, 4), "keep": int(cnt[0]), "clone": int(cnt[1]),
            "split": int(cnt[2]), "removed": int(cnt[3]), "n_out": int(n_out),
            "plan_ms": round(tp, 4), "apply_ms": round(ta, 4),
            "plan_gbs": round(b_plan / (tp * 1e-3) / 1e9, 1), "apply_gbs": round(float(b_apply) / (ta * 1e-3) / 1e9, 1),
            "apply_hbm_frac": round(float(b_apply) / (ta * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)}


def bench_crop(reps=3, rho=0.8, filter_px=2.1213, tau=3):
    """Visibility-frequency crop volume (Sec. 4) on its quoted scale: 31.4 M points, 958 views at
    1920x1080 over 1.47 km^2.  Times the visibility count (median of reps; points in Morton order, as
    stored; one pass in a random order for comparison) and the crop statistics."""
    import torch
    from paper_2411_00771_amd import _lib, crop, scenes
    t0 = time.time()
    w = scenes.crop_workload()
    P, cams = w["points"], w["cameras"]
    gen_s = time.time() - t0
    m, V = P.shape[1], len(cams)
    pt = torch.from_numpy(P).cuda()
    arr = _lib.camera_array(cams)
    cnt = torch.zeros(m, dtype=torch.int32, device="cuda")
    crop.visibility_count(pt, arr, rho, filter_px, count=cnt)  # warm-up
    ms = []
    for _ in range(reps):
        cnt.zero_()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        crop.visibility_count(pt, arr, rho, filter_px, count=cnt)
        e1.record()
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    perm = torch.randperm(m, device="cuda")
    pr = pt[:, perm].contiguous()
    cr = torch.zeros(m, dtype=torch.int32, device="cuda")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    crop.visibility_count(pr, arr, rho, filter_px, count=cr)
    e1.record()
    torch.cuda.synchronize()
    ms_rand = e0.elapsed_time(e1)
    same = bool(torch.equal(cr, cnt[perm]))
    del pr, cr, perm
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    keep, ground, (h0, h1) = crop.crop_volume(pt, cnt, tau, np.hstack([np.eye(3), np.zeros((3, 1))]))
    e1.record()
    torch.cuda.synchronize()
    t = float(np.median(ms))
    c = cnt.float()
    return {"points": m, "views": V, "resolution": [cams[0].width, cams[0].height], "radius": rho,
            "filter_px": filter_px, "generate_s": round(gen_s, 1), "count_ms": round(t, 3),
            "decisions_per_s": round(m * V / (t * 1e-3), 1), "count_ms_random_order": round(ms_rand, 3),
            "random_order_same_counts": same, "crop_ms_incl_readback": round(e0.elapsed_time(e1), 3),
            "mean_views_per_point": round(float(c.mean()), 2), "kept": int(ground.shape[1]), "tau": tau,
            "height_range": [round(h0, 3), round(h1, 3)]}


def bench_batched(steps, warmup, n=None):
    """Differentiation form: 8 views per launch through the autograd Functions at 4 M surfels, against the
    plain single-view path over the same 8 views on the same scene."""
    import torch
    from paper_2411_00771_amd import raster, scenes
    w = scenes.workload(2, n_override=n)
    sc, cams_all = w["scene"], w["cameras"]
    V = len(cams_all)
    dev = torch.device("cuda:0")
    params = raster.Params.from_scene(sc, dev)
    W, H = cams_all[0].width, cams_all[0].height
    eng = raster.Engine(sc.n, W, H, V)
    cs = eng.cams(cams_all)
    need = eng.fit_capacity(params, cs)
    eng.set_capacity(int(need * 1.25) + 4096)
    tp = raster.Params.from_scene(scenes.perturbed(sc, 77), dev)
    eng.forward(tp, cs)
    target = eng.rgb.clone()
    del tp
    leaves = [t.clone().requires_grad_(True) for t in (params.mean, params.log_scale, params.quat,
                                                       params.opacity_logit, params.sh)]
    state = raster.DensifyState(sc.n, V)

    def step():
        for t in leaves:
            t.grad = None
        out = raster.rasterize(leaves, eng, cs, sc.sh_degree)
        loss = raster.L1SSIMLoss.apply(out[0], target, eng, 0.2)
        loss.backward()
        eng.densify(params, eng.grads, state)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    ms_b = e0.elapsed_time(e1) / steps
    assert eng.status.item() == 0
    # plain single-view path over the same views
    e1v = raster.Engine(sc.n, W, H, 1)
    c1 = [e1v.cams([c]) for c in cams_all]
    need1 = max(e1v.fit_capacity(params, c) for c in c1)
    e1v.set_capacity(int(need1 * 1.25) + 4096)
    g1 = raster.Grads(params, 1)
    st1 = raster.DensifyState(sc.n)

    def step1():
        for v, c in enumerate(c1):
            e1v.forward(params, c)
            e1v.loss(target[v:v + 1].contiguous())
            e1v.backward(params, c, g1, d_rgb=e1v.d_img, d_rgb_ssim=e1v.d_img_ssim)
            e1v.densify(params, g1, st1)

    for _ in range(max(1, warmup // 2)):
        step1()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        step1()
    e1.record()
    torch.cuda.synchronize()
    ms_p = e0.elapsed_time(e1) / steps
    assert e1v.status.item() == 0
    return {"workload": w["name"], "surfels": sc.n, "views_per_launch": V,
            "batched_views_per_s": round(V * 1e3 / ms_b, 2), "plain_views_per_s": round(V * 1e3 / ms_p, 2),
            "batched_ms_per_step": round(ms_b, 3), "plain_ms_per_8_views": round(ms_p, 3),
            "speedup": round(ms_p / ms_b, 3), "steps": steps}


def _trace_stats(done, warmup_s):
    """p50 / p99 latency and served Mpix/s of the requests that arrived after the warm-up window."""
    t_first = min(r.arrival for r in done)
    win = [r for r in done if r.arrival - t_first >= warmup_s and r.error is None]
    lat = np.array([r.latency for r in win])
    px = sum(r.cam.width * r.cam.height for r in win)
    span = max(r.done_t for r in win) - min(r.arrival for r in win)
    arr = max(r.arrival for r in win) - min(r.arrival for r in win)
    return {"requests": len(done), "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
            "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3), "mpix_per_s": round(px / span / 1e6, 2),
            "offered_mpix_per_s_window": round(px / max(arr, 1e-9) / 1e6, 2),
            "readmitted": sum(r.tries for r in done), "errors": sum(r.error is not None for r in done)}


def _serve_trace(srv, city, rate, seconds, seed):
    from paper_2411_00771_amd import scenes, server
    reqs = scenes.poisson_requests(seed, rate, seconds, scenes.SERVE_RESOLUTIONS)
    rng = np.random.default_rng(seed + 1)
    cams = [scenes.orbit_camera(rng, city, *scenes.SERVE_RESOLUTIONS[k]) for _, k in reqs]
    offered = sum(c.width * c.height for c in cams) / seconds / 1e6
    done, _ = server.run_trace(srv, cams, [t for t, _ in reqs])
    return done, offered


def bench_serving(seconds, warmup_s, slots, n=None, slo_ms=50.0, knee_seconds=6.0, max_batch=4,
                  rates=(200, 300, 400, 500, 600, 800, 1000, 1300)):
    """Serving form: Poisson requests (200/s) of mixed resolutions against 5 M resident surfels, through
    the continuous-batching server (slots, real-byte admission) and through a plain one-slot queue; then
    the capacity: the Poisson rate raised step by step until p99 exceeds slo_ms or the served rate falls
    below 95 % of the offered one (the knee is the last rate that met both)."""
    import torch
    from paper_2411_00771_amd import raster, scenes, server
    w = scenes.workload(3, n_override=n)
    sc, city = w["scene"], w["city"]
    params = raster.Params.from_scene(sc, torch.device("cuda:0"))
    reqs = [r for r in w["requests"] if r[0] < seconds]
    rng = np.random.default_rng(3004)
    cams = [scenes.orbit_camera(rng, city, *scenes.SERVE_RESOLUTIONS[k]) for _, k in reqs]
    arrivals = [t for t, _ in reqs]
    out = {}
    for name, ns, mb in (("continuous", slots, 1), ("continuous_batched", slots, max_batch), ("plain_queue", 1, 1)):
        srv = server.Server(params, max_slots=ns, arena_bytes=32 << 30, intersections_per_pixel=3.0,
                            keep_results=False, max_batch=mb)
        # warm the kernels
        for c in cams[:8]:
            srv.render_alone(c)
        srv.finished.clear()
        dur = seconds if name == "continuous" else min(seconds, 10.0)
        k = sum(1 for t in arrivals if t < dur)
        done, wall = server.run_trace(srv, cams[:k], arrivals[:k])
        out[name] = dict(_trace_stats(done, warmup_s), slots=ns, max_batch=mb, seconds=dur,
                         launches=srv.launches, budget_gb=round(srv.arena_bytes / 2 ** 30, 1),
                         fixed_gb=round(srv.fixed_bytes / 2 ** 30, 2))
        log(f"[bench] serving {name}: {out[name]}")
        del srv
        torch.cuda.empty_cache()
    offered = sum(scenes.SERVE_RESOLUTIONS[k][0] * scenes.SERVE_RESOLUTIONS[k][1] for _, k in reqs) / seconds
    out.update(workload=w["name"], surfels=sc.n, rate_per_s=200, offered_mpix_per_s=round(offered / 1e6, 1),
               warmup_s=warmup_s)
    # capacity: the knee of the batched server
    srv = server.Server(params, max_slots=slots, arena_bytes=32 << 30, intersections_per_pixel=3.0,
                        keep_results=False, max_batch=max_batch)
    for c in cams[:8]:
        srv.render_alone(c)
    sweep, knee = [], None
    for rate in rates:
        srv.finished.clear()
        done, offered_r = _serve_trace(srv, city, rate, knee_seconds, 3100 + rate)
        st = dict(_trace_stats(done, 1.0), rate_per_s=rate, offered_mpix_per_s=round(offered_r, 1))
        sweep.append(st)
        log(f"[bench] serving capacity: {st}")
        if st["p99_ms"] > slo_ms or st["mpix_per_s"] < 0.95 * st["offered_mpix_per_s_window"]:
            break
        knee = st
    out["capacity"] = {"slo_p99_ms": slo_ms, "slots": slots, "max_batch": max_batch, "seconds_per_rate": knee_seconds,
                       "knee_rate_per_s": knee["rate_per_s"] if knee else None,
                       "knee_mpix_per_s": knee["mpix_per_s"] if knee else None, "sweep": sweep}
    del srv
    return out


def bench_largest(train_steps=5, slots=4):
    """The largest workload: 10 M surfels (log-normal scales, 10 % degenerate elongated); one 8-view
    1600x1066 training step (forward, loss, backward, densification statistics) timed alone, the 64
    served 3840x2160 depth/normal renders of the nadir grid through the server alone, then both at once
    (the training step on its own stream while the server admits the renders)."""
    import torch
    from paper_2411_00771_amd import raster, scenes, server
    t0 = time.time()
    w = scenes.workload(4)
    sc, cams, serve_cams = w["scene"], w["cameras"], w["serve_cameras"]
    gen_s = time.time() - t0
    dev = torch.device("cuda:0")
    params = raster.Params.from_scene(sc, dev)
    V = len(cams)
    W, H = cams[0].width, cams[0].height
    eng = raster.Engine(sc.n, W, H, V, capacity=1 << 20)
    cs = eng.cams(cams)
    need = eng.fit_capacity(params, cs)
    eng.set_capacity(int(need * 1.25) + 4096)
    tp = raster.Params.from_scene(scenes.perturbed(sc, 78), dev)
    eng.forward(tp, cs)
    targets = eng.rgb.clone()
    del tp
    grads = raster.Grads(params, V)
    state = raster.DensifyState(sc.n, V)

    def train_step():
        grads.zero_()
        eng.forward(params, cs)
        eng.loss(targets)
        eng.backward(params, cs, grads, d_rgb=eng.d_img, d_rgb_ssim=eng.d_img_ssim)
        eng.densify(params, grads, state)

    train_step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(train_steps):
        train_step()
    e1.record()
    torch.cuda.synchronize()
    assert eng.status.item() == 0
    ms_train = e0.elapsed_time(e1) / train_steps
    srv = server.Server(params, max_slots=slots, arena_bytes=48 << 30, intersections_per_pixel=3.0,
                        keep_results=False)
    srv.render_alone(serve_cams[0])
    srv.finished.clear()
    t = time.perf_counter()
    for c in serve_cams:
        srv.submit(c, arrival=t)
    srv.drain()
    alone_wall = time.perf_counter() - t
    alone = list(srv.finished)
    srv.finished.clear()
    px = sum(c.width * c.height for c in serve_cams)
    # both: the 64 renders queued at once, the training step on its own stream while the server admits them
    ts = torch.cuda.Stream()
    t = time.perf_counter()
    for c in serve_cams:
        srv.submit(c, arrival=t)
    srv.poll()
    with torch.cuda.stream(ts):
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(ts)
        train_step()
        ev1.record(ts)
    srv.drain()
    torch.cuda.synchronize()
    mix_wall = time.perf_counter() - t
    mixed = list(srv.finished)
    lat = lambda rs, q: round(float(np.percentile([r.latency for r in rs], q)) * 1e3, 2)
    return {"workload": w["name"], "surfels": sc.n, "generate_s": round(gen_s, 1), "train_views": V,
            "train_step_ms": round(ms_train, 3), "train_views_per_s": round(V * 1e3 / ms_train, 1),
            "train_mpix_per_s": round(V * W * H / (ms_train * 1e-3) / 1e6, 1), "intersections": int(need),
            "serve_alone": {"renders": len(alone), "wall_ms": round(alone_wall * 1e3, 1),
                            "p50_ms": lat(alone, 50), "p99_ms": lat(alone, 99),
                            "mpix_per_s": round(px / alone_wall / 1e6, 1)},
            "mixed": {"wall_ms": round(mix_wall * 1e3, 1), "train_step_ms": round(ev0.elapsed_time(ev1), 3),
                      "serve_p50_ms": lat(mixed, 50), "serve_p99_ms": lat(mixed, 99),
                      "mpix_per_s_total": round((px + V * W * H) / mix_wall / 1e6, 1)}}


def bench_storage(seconds=10.0, warmup_s=2.0, slots=4, n=None, ratio=0.4, codebook_size=8192, iters=10):
    """Serving storage (Sec. 3.3 SH degree 2; the appendix's vector-tree quantization): the serving scene
    with SH of degree 2, its Eq. 3/4 contributions over 16 orbit views, the compression (partition,
    k-means on the matrix cores, float16 packing), then the Poisson trace against the compact set and
    against its float32 source."""
    import torch
    from paper_2411_00771_amd import raster, scenes, server, storage
    w = scenes.workload(3, n_override=n)
    city = w["city"]
    sc = scenes.city_scene(3, w["scene"].n, L=1600.0, sh_degree=2, city=city)
    params = raster.Params.from_scene(sc, torch.device("cuda:0"))
    rng = np.random.default_rng(3005)
    views = [scenes.orbit_camera(rng, city, 1280, 720) for _ in range(16)]
    eng = raster.Engine(sc.n, 1280, 720, 1)
    need = max(eng.fit_capacity(params, eng.cams([c])) for c in views)
    eng.set_capacity(int(need * 1.25) + 4096)
    c_sum = torch.zeros(sc.n, device="cuda:0")
    for c in views:
        cc = eng.cams([c])
        eng.project(params, cc)
        eng.bin_sort(cc)
        eng.contribution(cc, 0.5, c_sum=c_sum)
    c_avg = c_sum / len(views)
    del eng
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cp, info = storage.compress(params, c_avg, ratio=ratio, codebook_size=codebook_size, iters=iters)
    torch.cuda.synchronize()
    t_comp = time.perf_counter() - t0
    # one assignment pass, event-timed: m x K x D multiply-adds on the matrix cores
    D = 27
    rows = cp.order[cp.n_full:]
    x = params.sh.reshape(sc.n, D)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    storage.vq_assign(x, D, rows, info["codebook"])
    e1.record()
    torch.cuda.synchronize()
    t_assign = e0.elapsed_time(e1)
    m, K = rows.numel(), info["codebook_size"]
    flops = 2.0 * m * K * 28  # padded to 7 MFMA steps of 4
    full_bytes = sum(t.numel() * 4 for t in (params.mean, params.log_scale, params.quat, params.opacity_logit,
                                             params.sh))
    out = {"surfels": sc.n, "sh_degree": 2, "quantized": m, "codebook_size": K, "iters": iters,
           "compress_s": round(t_comp, 3), "assign_ms": round(t_assign, 3),
           "assign_tflops": round(flops / (t_assign * 1e-3) / 1e12, 2),
           "bytes_full": full_bytes, "bytes_compact": cp.nbytes(), "ratio": round(cp.nbytes() / full_bytes, 3)}
    reqs = [r for r in w["requests"] if r[0] < seconds]
    rng = np.random.default_rng(3004)
    cams = [scenes.orbit_camera(rng, city, *scenes.SERVE_RESOLUTIONS[k]) for _, k in reqs]
    arrivals = [t for t, _ in reqs]
    for name, ps in (("compact", cp), ("float32", params)):
        srv = server.Server(ps, max_slots=slots, arena_bytes=32 << 30, intersections_per_pixel=3.0,
                            keep_results=False)
        for c in cams[:8]:
            srv.render_alone(c)
        srv.finished.clear()
        done, wall = server.run_trace(srv, cams, arrivals)
        t_first = min(r.arrival for r in done)
        win = [r for r in done if r.arrival - t_first >= warmup_s and r.error is None]
        lat = np.array([r.latency for r in win])
        px = sum(r.cam.width * r.cam.height for r in win)
        span = max(r.done_t for r in win) - min(r.arrival for r in win)
        out[name] = {"requests": len(done), "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
                     "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
                     "mpix_per_s": round(px / span / 1e6, 2)}
        log(f"[bench] storage serving {name}: {out[name]}")
        del srv
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=320)
    ap.add_argument("--warmup", type=int, default=32)
    ap.add_argument("--n", type=int, default=None, help="surfel count override (default 1,000,000)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--breakdown-steps", type=int, default=32)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-steps", type=int, default=10)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-contribution", action="store_true")
    ap.add_argument("--no-densify-action", action="store_true")
    ap.add_argument("--no-crop", action="store_true")
    ap.add_argument("--no-storage", action="store_true")
    ap.add_argument("--no-largest", action="store_true")
    ap.add_argument("--no-capacity", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=30.0)
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one 256 MiB read + 256 MiB write elementwise kernel (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this rasterizer build has no multi-GPU path "
              "(the sharding design is described in DESIGN.md); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2411_00771_amd import raster, scenes

    if args.calibrate_copy:
        # one elementwise kernel that reads 256 MiB and writes 256 MiB
        src = torch.ones(64 << 20, device="cuda:0")
        dst = torch.empty_like(src)
        torch.mul(src, 2.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    t0 = time.time()
    w = scenes.workload(1, n_override=args.n)
    sc, cams_all = w["scene"], w["cameras"]
    log(f"[bench] workload {w['name']}: n={sc.n}, {len(cams_all)} cameras, generated in {time.time() - t0:.1f}s")
    dev = torch.device("cuda:0")
    params = raster.Params.from_scene(sc, dev)
    W, H = cams_all[0].width, cams_all[0].height
    eng = raster.Engine(sc.n, W, H, 1)
    cams = [eng.cams([c]) for c in cams_all]

    # capacity from the largest view, then targets (renders of a perturbed copy), outside timing
    need = max(eng.fit_capacity(params, c) for c in cams)
    eng.set_capacity(int(need * 1.25) + 4096)
    eng.status.zero_()
    tp = raster.Params.from_scene(scenes.perturbed(sc, 77), dev)
    targets = []
    for c in cams:
        eng.forward(tp, c)
        targets.append(eng.rgb.clone())
    del tp
    counts = []
    for c in cams:
        eng.forward(params, c)
        counts.append(eng.count(c))
    torch.cuda.synchronize()
    log(f"[bench] max intersections {need}, capacity {eng.capacity}; setup {time.time() - t0:.1f}s")

    grads = raster.Grads(params, 1)
    state = raster.DensifyState(sc.n)

    names = ["zero_grads", "project", "bin_sort", "render_fwd", "loss", "render_bwd", "project_bwd", "densify"]

    # The parameter gradients accumulate (+=) over the views of a call, so a step starts from zeroed
    # gradients.  In the timed loop the zeroing runs on a second stream (default priority), after the
    # previous step's chain to the parameters and overlapped with this step's forward; the chain waits
    # for it.  The per-call split zeroes in line.
    zstream = torch.cuda.Stream()
    grads_free = torch.cuda.Event()   # the previous step's parameter gradients are done
    grads_zeroed = torch.cuda.Event()
    grads_free.record()

    def step(k, ev=None, overlap=False):
        """One training step on view k; ev maps a call index i to the event recorded before call i
        (index len(names) = after the last call)."""
        c = cams[k % len(cams)]

        def mark(i):
            if ev is not None and i in ev:
                ev[i].record()

        mark(0)
        if overlap:
            zstream.wait_event(grads_free)
            with torch.cuda.stream(zstream):
                grads.zero_()
                grads_zeroed.record(zstream)
        else:
            grads.zero_()
        mark(1)
        eng.project(params, c)
        mark(2)
        eng.bin_sort(c)
        mark(3)
        eng.render(c)
        mark(4)
        eng.loss(targets[k % len(cams)])
        mark(5)
        eng.backward_records(c, d_rgb=eng.d_img, d_rgb_ssim=eng.d_img_ssim)
        mark(6)
        if overlap:
            torch.cuda.current_stream().wait_event(grads_zeroed)
        eng.project_backward(params, c, grads)
        if overlap:
            grads_free.record()
        mark(7)
        eng.densify(params, grads, state)
        mark(8)

    def events(idx):
        return {i: torch.cuda.Event(enable_timing=True) for i in idx}

    for k in range(args.warmup):
        step(k, overlap=True)
    torch.cuda.synchronize()
    log(f"[bench] warmup {args.warmup} steps done")
    # events around the dominant kernel (the reverse render) are recorded inside the timed region (same
    # stream); the forward render is timed in the per-call pass below.  Each recorded event costs the
    # stream a few microseconds, so the timed region holds only the two the roofline needs.
    live = [events((5, 6)) for _ in range(args.steps)]
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for k in range(args.steps):
        step(k, live[k], overlap=True)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop)
    if eng.status.item() != 0:
        raise RuntimeError("intersection capacity overflowed during the timed region; result invalid")
    log(f"[bench] timed {args.steps} steps: {ms:.2f} ms")
    per_bwd = [(k % len(cams), ev[5].elapsed_time(ev[6])) for k, ev in enumerate(live)]

    # per-call split with events between all calls (separate pass); it also times the forward render
    tot = np.zeros(len(names))
    per_step = []
    per_fwd = []
    for k in range(args.breakdown_steps):
        ev = events(range(len(names) + 1))
        step(k, ev)
        torch.cuda.synchronize()
        tot += [ev[i].elapsed_time(ev[i + 1]) for i in range(len(names))]
        per_step.append(ev[0].elapsed_time(ev[len(names)]))
        per_fwd.append((k % len(cams), ev[3].elapsed_time(ev[4])))
    split = {nm: tot[i] / max(args.breakdown_steps, 1) for i, nm in enumerate(names)}
    log("[bench] split (ms/step): " + ", ".join(f"{k} {v:.3f}" for k, v in split.items()))

    # roofline of the dominant kernel: flops from the counted pairs of each timed view over the
    # kernel's event-timed durations (the reverse render's in the timed region)
    if not per_fwd:
        raise SystemExit("--breakdown-steps must be at least 1 (the forward render is timed there)")
    f_fwd = sum(F_FWD_EVAL * counts[v][0] + F_FWD_CON * counts[v][1] for v, _ in per_fwd)
    t_fwd = sum(t for _, t in per_fwd) * 1e-3
    f_bwd = sum(F_BWD_WALK * counts[v][2] + F_BWD_CON * counts[v][1] for v, _ in per_bwd)
    t_bwd = sum(t for _, t in per_bwd) * 1e-3
    dom = "render_bwd" if t_bwd / len(per_bwd) >= t_fwd / len(per_fwd) else "render_fwd"
    ach = (f_bwd / t_bwd if dom == "render_bwd" else f_fwd / t_fwd) / 1e12
    traffic = None
    tf = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tf):
        tj = json.load(open(tf))
        if tj.get("kernel_hash") == kernel_hash() and dom in tj.get("bytes_per_launch", {}):
            traffic = tj["bytes_per_launch"][dom]
    roof = dict(bound="alu", kernel=dom, achieved=round(ach, 3), peak=PEAK_FP32_TFLOPS, unit="TFLOP/s",
                frac=round(ach / PEAK_FP32_TFLOPS, 4), frac_nonpacked=round(ach / PEAK_FP32_NONPACKED, 4),
                traffic=traffic,
                kernel_ms=round(1e3 * (t_bwd / len(per_bwd) if dom == "render_bwd" else t_fwd / len(per_fwd)), 4),
                render_fwd_tflops=round(f_fwd / t_fwd / 1e12, 3), render_bwd_tflops=round(f_bwd / t_bwd / 1e12, 3))

    ips = args.steps / (ms * 1e-3)
    mean_counts = np.mean(np.array(counts, np.float64), 0)
    out = {
        "metric": "fwd+bwd iters/s (1M surfels, 1600x1066)",
        "value": round(ips, 2),
        "unit": "iters/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms / args.steps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": w["name"], "surfels": sc.n, "width": W, "height": H, "views": len(cams),
                   "sh_degree": sc.sh_degree, "step": "zero_grads+project+bin_sort+render_fwd+loss+render_bwd+project_bwd+densify"},
        "mpix_per_s": round(ips * W * H / 1e6, 2),
        "split_ms": {k: round(v, 4) for k, v in split.items()},
        # one step per view of the 16, each synchronized on its own (the breakdown pass)
        "step_ms_percentiles": ({f"p{q}": round(float(np.percentile(per_step, q)), 4) for q in (10, 50, 90)}
                                if per_step else None),
        "pairs_per_view": {"evaluated": int(mean_counts[0]), "contributing": int(mean_counts[1]),
                           "reverse_walked": int(mean_counts[2])},
        "intersections_max": int(need),
        "roofline": roof,
    }
    trim = None
    if not args.no_contribution:
        out["contribution"], trim = bench_contribution(eng, params, cams, counts)
        log(f"[bench] contribution/trim: {out['contribution']}")
    if not args.no_densify_action:
        out["densify_action"] = bench_densify_action(params, state.mask, trim, 0.01 * camera_extent(cams_all))
        log(f"[bench] densify action: {out['densify_action']}")
    targets_host = [t[0].cpu().numpy().astype(np.float64) for t in targets[:8]]
    if not args.no_crop:
        log("[bench] crop-volume visibility pass (31.4M points, 958 views)")
        out["crop"] = bench_crop()
        log(f"[bench] crop: {out['crop']}")
        torch.cuda.empty_cache()
    del eng, grads, state, params, targets
    torch.cuda.empty_cache()
    if not args.no_batched:
        log("[bench] batched differentiation form (8 views per launch, 4M surfels)")
        out["batched"] = bench_batched(args.batched_steps, 2)
        log(f"[bench] batched: {out['batched']}")
        torch.cuda.empty_cache()
    if not args.no_serve:
        log("[bench] serving form (5M surfels, Poisson 200/s, mixed resolutions)")
        out["serving"] = bench_serving(args.serve_seconds, 2.0, args.serve_slots,
                                       rates=(() if args.no_capacity else (200, 300, 400, 500, 600, 800, 1000, 1300)))
        torch.cuda.empty_cache()
    if not args.no_storage:
        log("[bench] serving storage (SH degree 2, float16 + vector quantization)")
        out["storage"] = bench_storage()
        log(f"[bench] storage: {out['storage']}")
        torch.cuda.empty_cache()
    if not args.no_largest:
        log("[bench] largest: 10M surfels, 8-view training step and 64 served 4K renders")
        out["largest"] = bench_largest()
        log(f"[bench] largest: {out['largest']}")
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log("[bench] timing the FP64 oracle on one view (CPU)")
        out["cpu_baseline"] = cpu_baseline(sc, cams_all[:8], targets_host)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
