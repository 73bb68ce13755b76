#!/usr/bin/env python3
"""Throughput of the 4D Gaussian render hot path on one MI355X.

One step = render a batch of (camera, time) views of a 300k-primitive scene
(1352x1014, SH degree 3 x Fourier order 2), L1 loss against seeded targets,
and the full backward to every primitive parameter. The batched step renders
all views in one library call; the per-view step issues one call per view
(gradients accumulated in place). Inputs are resident in HBM before timing.

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

# Algorithmic work per evaluated fragment (one pixel x one list entry up to the
# pixel's last contributor), counted in FP32 lane operations (an FMA is one):
#   forward:  offset 2, quadratic form 5, floor test 1, exp 1, clamp 1,
#             transmittance 1, weight 1, colour+depth accumulation 4      = 16
#   backward: offset 2, quadratic form 5, floor test 1, exp 1, clamp 1,
#             transmittance recovery 3 (1 - a, reciprocal, product),
#             colour dot 3, behind term 2, dL/da 1, dL/dpower 1, weight 1,
#             per-primitive tile sums 6 (g, g m, g m^2, w dL/dC x 3)      = 27
OPS_FWD = 16
OPS_BWD = 27
UNITS_NAME = ("list positions up to each pixel's last contributor (sum over pixels of pix_last; the "
              "quadrant cull skips some of them, which still count as work the method defines)")
# counter summaries under profiles/ (taken with the same kernel sources)
TRAFFIC_SUMMARY = "traffic_bench_300k_8x1352x1014.md"
SQ_SUMMARY = "sq_counters_raster_bench_300k_8x1352x1014.md"
# FP32 vector peak without packed math: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
ALU_PEAK_OPS = 256 * 4 * 16 * 2.4e9
HBM_PEAK = 8.0e12


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_oracle_baseline(wl, seconds: float):
    """Times the FP64 oracle (forward + autograd backward) on one view of the
    workload for growing tile samples; a linear fit over the sample size
    extrapolates to the full view (fixed cost: preprocessing all primitives)."""
    import numpy as np
    import torch
    from oracle import render4d as O

    cam, t = wl.cameras[0], float(wl.times[0])
    ocam = O.to_ocamera(cam)
    n_tiles = ocam.tiles_x * ocam.tiles_y
    rng = np.random.default_rng(5)
    order = rng.permutation(n_tiles)

    def run(k):
        t0 = time.perf_counter()
        params = O.params_from_scene(wl.scene, requires_grad=True)
        pre = O.preprocess(params, ocam, t, wl.scene.sh_degree, wl.scene.t_order, wl.scene.t_period)
        loss = torch.zeros((), dtype=torch.float64)
        for tid in order[:k]:
            part = O.composite_tile(pre, ocam, int(tid), (0.0, 0.0, 0.0), with_flags=False)
            loss = loss + part["rgb"].sum()
        loss.backward()
        return time.perf_counter() - t0

    def fit(budget):
        # samples of 4, 8, 16, ... tiles until the next one would overrun the
        # budget; the last two fix the per-tile slope and the fixed cost
        ks, ts = [], []
        k = 4
        while True:
            ks.append(k)
            ts.append(run(k))
            if k >= n_tiles or (len(ks) >= 2 and sum(ts) + 2.2 * ts[-1] > budget):
                break
            k = min(2 * k, n_tiles)
        if len(ks) == 1:  # the sample was the whole view
            b, a = ts[0] / ks[0], 0.0
        else:
            b = max((ts[-1] - ts[-2]) / (ks[-1] - ks[-2]), 1e-9)
            a = max(ts[-1] - b * ks[-1], 0.0)
        return ks, ts, a, b

    px = cam.width * cam.height
    threads = int(torch.get_num_threads())
    ks, ts, a, b = fit(seconds)
    full = a + b * n_tiles
    # the same oracle on one thread, over a smaller sample
    torch.set_num_threads(1)
    try:
        ks1, ts1, a1, b1 = fit(seconds / 2)
    finally:
        torch.set_num_threads(threads)
    full1 = a1 + b1 * n_tiles
    return dict(value=px / full / 1e6, unit="Mpix/s (fwd+bwd, one view, extrapolated)",
                cores=threads, kind="oracle",
                sample=(f"1 of {len(wl.cameras)} views at {cam.width}x{cam.height}, {wl.scene.n} primitives: "
                        f"FP64 preprocess of all primitives + fwd/bwd of random 16x16 tiles, samples of "
                        f"{ks} tiles took {[round(x, 2) for x in ts]} s; full view = {a:.2f}s + {b:.4f}s x "
                        f"{n_tiles} tiles"),
                seconds=round(sum(ts), 2),
                value_1_thread=px / full1 / 1e6,
                sample_1_thread=(f"samples of {ks1} tiles took {[round(x, 2) for x in ts1]} s on one thread; "
                                 f"full view = {a1:.2f}s + {b1:.4f}s x {n_tiles} tiles"),
                seconds_1_thread=round(sum(ts1), 2))


def other_workloads(log_fn, steps: int, cfgs=(2, 3, 4)):
    """The other seeded workloads in their own right (not the headline):
    batched forward of 1M primitives over 16 mixed views, batched fwd+bwd of
    500k over 8 views with an L2 loss, and one call rendering 3M primitives
    over 60 frames x 4 cameras at 1920x1080 (several rounds)."""
    import numpy as np
    import torch
    import scenegen
    from paper_2310_10642_amd import g4d

    dev = torch.device("cuda", 0)
    res = {}
    for cfg in cfgs:
        t0 = time.perf_counter()
        wl = scenegen.make_workload(cfg)
        sc = wl.scene
        r = g4d.Renderer(sc.sh_degree, sc.t_order, sc.t_period)
        params = [torch.from_numpy(a).to(dev) for a in (sc.means4, sc.log_scales4, sc.q_left, sc.q_right,
                                                           sc.opacity_logit, sc.coeffs)]
        r.set_primitives(*params)
        cams, times = wl.cameras, [float(x) for x in wl.times]
        P = sum(c.width * c.height for c in cams)
        rgb = torch.empty(3 * P, device=dev)
        if wl.loss is None:
            def step():
                r.render(cams, times, depth=False, alpha=False, out=(rgb, None, None))
            kind = "forward"
        else:
            target = torch.from_numpy(np.concatenate([t.reshape(-1) for t in wl.targets])).to(dev)
            loss = torch.zeros(1, device=dev)
            dl = torch.empty_like(rgb)
            grads = r.grad_buffers(dev)
            scale = 1.0 / (3 * cams[0].width * cams[0].height)

            def step():
                r.render(cams, times, depth=False, alpha=False, out=(rgb, None, None))
                r.image_loss(g4d.G4D_LOSS_L2 if wl.loss == "l2" else g4d.G4D_LOSS_L1, rgb, target, scale, loss, dl)
                r.backward(dl, out=grads)
            kind = "fwd+bwd"
        n = steps if cfg != 4 else max(2, steps // 5)
        step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(n):
            step()
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t1) / n
        st = r.stats()
        # the batch also as a sync-free call captured into a HIP graph
        graph_sec = None
        try:
            r.set_tuning(g4d.G4D_TUNE_SYNC_FREE, 1)
            step()
            torch.cuda.synchronize()
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph):
                step()
            graph.replay()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(n):
                graph.replay()
            torch.cuda.synchronize()
            graph_sec = (time.perf_counter() - t1) / n
            r.stats()  # raises if a replay overflowed the instance arena
            del graph
        except Exception as e:
            log_fn(f"[bench] {wl.name}: graph replay unavailable: {e}")
            graph_sec = None
        finally:
            r.set_tuning(g4d.G4D_TUNE_SYNC_FREE, 0)
        res[wl.name] = dict(kind=kind, ms_per_call=sec * 1e3, mpix_per_s=P / sec / 1e6, views=len(cams),
                            primitives=sc.n, rounds=st["rounds"], instances=st["instances"],
                            active_mean=float(np.mean(st["active_per_view"])), calls_timed=n,
                            graph_ms_per_call=graph_sec * 1e3 if graph_sec else None,
                            graph_mpix_per_s=P / graph_sec / 1e6 if graph_sec else None)
        log_fn(f"[bench] {wl.name}: {kind} {sec * 1e3:.2f} ms per call, {P / sec / 1e6:.0f} Mpix/s, "
               f"{st['rounds']} round(s)" + (f", graph replay {graph_sec * 1e3:.2f} ms" if graph_sec else "") +
               f" ({time.perf_counter() - t0:.1f} s with setup)")
        del r, params, rgb
        torch.cuda.empty_cache()
    return res


CSRC = os.path.join(HERE, "paper_2310_10642_amd", "csrc")
PROFILES = os.path.join(HERE, "profiles")


def kernel_sources_sha256() -> str:
    """SHA-256 over the library's kernel sources (every file of csrc/, by name):
    a counter summary taken before any of them changed carries the same value."""
    import hashlib
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".h")):
            h.update(name.encode())
            h.update(open(os.path.join(CSRC, name), "rb").read())
    return h.hexdigest()


def profile_fields(summary: str):
    """The `key: value` lines of a counter summary under profiles/, or None
    when the file is missing or the kernels changed since it was taken."""
    try:
        text = open(os.path.join(PROFILES, summary)).read()
    except OSError:
        return None
    fields = {}
    for line in text.splitlines():
        if ": " in line and not line.startswith(("|", " ", "`", "#")):
            k, v = line.split(": ", 1)
            fields[k.strip()] = v.strip()
    if fields.get("source_sha256") != kernel_sources_sha256():
        return None
    out = {}
    for k, v in fields.items():
        try:
            out[k] = float(v)
        except ValueError:
            pass
    return out


def sq_figures(f, prefix: str, seconds: float, units: float):
    """Issue figures of one kernel from its SQ counters (per launch): VALU and
    LDS instructions per unit of work (lane instructions: wave instructions
    x 64), the VALU issue time as a share of the launch if every wave64 VALU
    instruction took 4 cycles of its 16-lane SIMD (1024 SIMDs at 2.4 GHz; an
    estimate: values above 1 show that some issue faster), and LDS
    bank-conflict cycles over LDS active cycles."""
    if not f or f.get(prefix + ".SQ_INSTS_VALU") is None:
        return None
    valu, lds = f[prefix + ".SQ_INSTS_VALU"], f.get(prefix + ".SQ_INSTS_LDS", float("nan"))
    out = dict(valu_lane_instr_per_unit=valu * 64 / units, lds_instr_per_unit=lds * 64 / units,
               valu_issue_frac_at_4_cycles=valu * 4 / (1024 * 2.4e9 * seconds))
    conf, act = f.get(prefix + ".SQ_LDS_BANK_CONFLICT"), f.get(prefix + ".SQ_ACTIVE_INST_LDS")
    if conf is not None and act:
        out["lds_bank_conflict_frac"] = conf / act
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--views", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-per-view", action="store_true")
    ap.add_argument("--no-fused-loss", action="store_true",
                    help="skip timing the step with the loss folded into the backward (its backward launches "
                         "would share the two-call step's kernel name in a profile)")
    ap.add_argument("--no-other-workloads", action="store_true",
                    help="skip the 1M x 16-view, 500k x 8-view and 3M x 240-view figures")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="first run a plain device copy of this many MiB three times (counter calibration)")
    ap.add_argument("--only-other", type=int, choices=(2, 3, 4), default=None,
                    help="profiling aid: time only that other workload (2: 1M x 16 views, 3: 500k x 8 views, "
                         "4: 3M x 240 views) and print its figures as the JSON line")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (the path would shard by "
              f"view with one process per GPU; only the one-GPU path exists)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import scenegen
    from paper_2310_10642_amd import g4d

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.copy_probe_mb > 0:
        nfl = args.copy_probe_mb * (1 << 20) // 4
        src = torch.ones(nfl, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log(f"[bench] copy probe: 3 x {args.copy_probe_mb} MiB device copies")
    if args.only_other is not None:
        print(json.dumps(other_workloads(log, args.steps, (args.only_other,))), flush=True)
        return
    log(f"[bench] building workload ({args.views} views)")
    wl = scenegen.bench_workload(args.views)
    sc = wl.scene
    r = g4d.Renderer(sc.sh_degree, sc.t_order, sc.t_period)
    params = [torch.from_numpy(a).to(dev) for a in (sc.means4, sc.log_scales4, sc.q_left, sc.q_right,
                                                       sc.opacity_logit, sc.coeffs)]
    r.set_primitives(*params)
    cams, times = wl.cameras, [float(x) for x in wl.times]
    V = len(cams)
    hw = [(c.height, c.width) for c in cams]
    P_total = sum(h * w for h, w in hw)
    target = torch.from_numpy(np.concatenate([t.reshape(-1) for t in wl.targets])).to(dev)
    tgt_v = []
    o = 0
    for h, w in hw:
        tgt_v.append(target[o:o + 3 * h * w])
        o += 3 * h * w
    scale = 1.0 / (3 * hw[0][0] * hw[0][1])   # per-view mean L1, summed over views
    grads = r.grad_buffers(dev)
    loss = torch.zeros(1, device=dev)
    dl = torch.empty(3 * P_total, device=dev)
    dl_v = [torch.empty(3 * h * w, device=dev) for h, w in hw]

    rgb_b = torch.empty(3 * P_total, device=dev)

    def step_batched():
        r.render(cams, times, depth=False, alpha=False, out=(rgb_b, None, None))
        loss.zero_()
        r.image_loss(g4d.G4D_LOSS_L1, rgb_b, target, scale, loss, dl)
        r.backward(dl, out=grads)

    # the same training step with the loss folded into the backward
    # (g4d_render_backward_loss: the values of image_loss + render_backward
    # without the gradient image), reported beside the headline step
    def step_fused():
        r.render(cams, times, depth=False, alpha=False, out=(rgb_b, None, None))
        loss.zero_()
        r.backward_loss(g4d.G4D_LOSS_L1, rgb_b, target, scale, loss, out=grads)

    def step_per_view():
        for v in range(V):
            rgb, _, _ = r.render([cams[v]], [times[v]], depth=False, alpha=False)
            r.image_loss(g4d.G4D_LOSS_L1, rgb, tgt_v[v], scale, loss, dl_v[v])
            r.backward(dl_v[v], out=grads, accumulate=v > 0)

    def forward_batched():
        r.render(cams, times, depth=False, alpha=False)

    def forward_per_view():
        for v in range(V):
            r.render([cams[v]], [times[v]], depth=False, alpha=False)

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    log("[bench] warmup + timed batched fwd+bwd")
    for _ in range(args.warmup):
        step_batched()
    torch.cuda.synchronize()
    r.stage_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step_batched()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / args.steps
    stages = r.stage_times()
    r.stage_timing(False)
    stats = r.stats()
    log(f"[bench] batched step {sec * 1e3:.3f} ms; stages {stages}; stats {stats}")

    # the same step, sync-free, captured once into a HIP graph and replayed
    graph_sec = None
    try:
        r.set_tuning(g4d.G4D_TUNE_SYNC_FREE, 1)
        step_batched()
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            step_batched()
        graph_sec = timed(graph.replay, args.steps, args.warmup)
        r.stats()  # raises if a replay overflowed the instance arena
        log(f"[bench] graph replay step {graph_sec * 1e3:.3f} ms")
    except Exception as e:  # capture unsupported: the eager figure stands
        log(f"[bench] graph replay unavailable: {e}")
        graph_sec = None
    finally:
        r.set_tuning(g4d.G4D_TUNE_SYNC_FREE, 0)
    best = min(sec, graph_sec) if graph_sec else sec

    fused_sec = fused_graph_sec = None
    if not args.no_fused_loss:
        fused_sec = timed(step_fused, args.steps, args.warmup)
        try:
            r.set_tuning(g4d.G4D_TUNE_SYNC_FREE, 1)
            step_fused()
            torch.cuda.synchronize()
            graph_f = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph_f):
                step_fused()
            fused_graph_sec = timed(graph_f.replay, args.steps, args.warmup)
            r.stats()  # raises if a replay overflowed the instance arena
        except Exception as e:  # capture unsupported: the eager figure stands
            log(f"[bench] fused-loss graph replay unavailable: {e}")
            fused_graph_sec = None
        finally:
            r.set_tuning(g4d.G4D_TUNE_SYNC_FREE, 0)
        log(f"[bench] fused-loss step {fused_sec * 1e3:.3f} ms, graph "
            f"{fused_graph_sec * 1e3 if fused_graph_sec else float('nan'):.3f} ms")

    # the fused Adam step over every parameter group (outside the headline step)
    m_buf = torch.zeros(sc.n * (17 + 3 * sc.coeffs.shape[1]), device=dev)
    v_buf = torch.zeros_like(m_buf)
    adam_state = {"step": 0}
    lr = [1.6e-4, 5e-3, 1e-3, 1e-3, 5e-2, 2.5e-3]

    def adam():
        adam_state["step"] += 1
        r.adam_step(params, grads, m_buf, v_buf, adam_state["step"], lr)
    adam_sec = timed(adam, max(3, args.steps // 2), 2)
    adam_bytes = 28 * m_buf.numel()           # read p, g, m, v; write p, m, v (4 B each)
    log(f"[bench] adam step {adam_sec * 1e3:.3f} ms, {adam_bytes / adam_sec / 1e9:.0f} GB/s")

    fwd_b = timed(forward_batched, max(3, args.steps // 2), 2)
    extra = {}
    if not args.no_per_view:
        log("[bench] per-view comparison")
        fwd_pv = timed(forward_per_view, max(3, args.steps // 2), 2)
        step_pv = timed(step_per_view, max(3, args.steps // 2), 2)
        extra = dict(per_view_fwd_bwd_mpix_per_s=P_total / step_pv / 1e6,
                     per_view_fwd_bwd_steps_per_s=1.0 / step_pv,
                     per_view_forward_mpix_per_s=P_total / fwd_pv / 1e6,
                     batched_over_per_view_fwd_bwd=step_pv / best)

    # per-stage rooflines; the line's own roofline is the dominant stage's
    sec_step = {k: ms * 1e-3 / args.steps for k, (ms, n) in stages.items()}
    frag = stats["fragments"]
    A, I, N = stats["active_total"], stats["instances"], sc.n
    F = sc.coeffs.shape[1] * 3                   # 4DSH coefficient floats per primitive
    traffic_f = profile_fields(TRAFFIC_SUMMARY)
    sq_f = profile_fields(SQ_SUMMARY)
    stage_roof = {}

    def hbm(name, byts, sec, note, counter_key=None):
        d = dict(bound="hbm", bytes=byts, ms=sec * 1e3, achieved_gb_s=byts / sec / 1e9,
                 frac=byts / sec / HBM_PEAK, bytes_rule=note)
        if counter_key and traffic_f and traffic_f.get(counter_key):
            cb = traffic_f[counter_key]
            d.update(counter_bytes=cb, counter_frac=cb / sec / HBM_PEAK)
        stage_roof[name] = d
    # preprocess + its colour pass: read every primitive's 17 geometry/opacity
    # floats and F coefficients once, write one 48-byte record per active pair
    hbm("preprocess", (17 + F) * 4 * N + 48 * A, sec_step["preprocess"] + sec_step["colour"],
        "(17+F)*4*N + 48*sum(A), time = k_preprocess + k_colour", "preprocess_bytes_per_render")
    # binning: 28 bytes per (tile, record) instance, what the two-pass instance
    # sort moves with 16-bit tile keys (emission writes 6 B, the first pass
    # reads and writes 6 B, the last reads 6 B and writes the 4-byte record)
    hbm("binning", 28 * I, sec_step["binning"], "28*I", "binning_bytes_per_render")
    # backward of the preprocess: parameters in and gradients out once, one
    # 128-byte FP64 gradient line per active record
    hbm("preprocess_bwd", (17 + F) * 4 * N * 2 + 128 * A, sec_step["preprocess_bwd"],
        "(17+F)*4*N*2 + 128*sum(A)", "preprocess_bwd_bytes_per_step")
    hbm("loss", 12 * 3 * P_total, sec_step["loss"], "12*3*pixels (image and target in, gradient out)")
    for name, ops in (("raster_fwd", OPS_FWD), ("raster_bwd", OPS_BWD)):
        t_r = sec_step[name]
        d = dict(bound="alu", ops_per_unit=ops, units=frag, ms=t_r * 1e3,
                 achieved_tops=ops * frag / t_r / 1e12, frac=ops * frag / t_r / ALU_PEAK_OPS)
        sq = sq_figures(sq_f, name, t_r, frag)
        if sq:
            d.update(sq)
        stage_roof[name] = d
    dom = max(("preprocess", "binning", "raster_fwd", "raster_bwd", "preprocess_bwd", "loss"),
              key=lambda k: sec_step[k])
    if dom in ("raster_bwd", "raster_fwd"):
        ops = frag * (OPS_BWD if dom == "raster_bwd" else OPS_FWD)
        achieved = ops / sec_step[dom]
        traffic = traffic_f.get(dom + "_bytes_per_launch") if traffic_f else None
        roof = dict(kernel=dom, bound="alu", achieved=achieved / 1e12, peak=ALU_PEAK_OPS / 1e12,
                    unit="Tops/s (FP32 lane ops)", frac=achieved / ALU_PEAK_OPS, traffic=traffic,
                    ms_per_launch=sec_step[dom] * 1e3, units=frag, units_name=UNITS_NAME)
    else:
        d = stage_roof[dom]
        roof = dict(kernel=dom, bound="hbm", achieved=d["achieved_gb_s"], peak=HBM_PEAK / 1e9, unit="GB/s",
                    frac=d["frac"], traffic=d.get("counter_bytes"), ms_per_launch=d["ms"])
    others = None
    if not args.no_other_workloads:
        log("[bench] other workloads")
        others = other_workloads(log, max(3, args.steps // 2))
    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline")
        torch.set_num_threads(os.cpu_count() or 1)
        cpu = cpu_oracle_baseline(wl, args.cpu_seconds)
        log(f"[bench] cpu {cpu}")

    out = {
        "metric": "Mpix/s render and fwd+bwd steps/s, 300k 4D Gaussians, batched vs per-view",
        "value": P_total / best / 1e6,
        "unit": "Mpix/s (fwd+bwd training step, batched)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": best * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": wl.name, "primitives": sc.n, "views": V, "resolution": f"{hw[0][1]}x{hw[0][0]}",
                   "sh_degree": sc.sh_degree, "t_order": sc.t_order, "loss": "l1", "batched": True},
        "fwd_bwd_steps_per_s": 1.0 / best,
        "batched_step_mode": "graph replay" if best != sec else "eager",
        "eager_ms_per_step": sec * 1e3,
        "graph_ms_per_step": graph_sec * 1e3 if graph_sec else None,
        "fused_loss_step": None if fused_sec is None else {
            "eager_ms": fused_sec * 1e3, "graph_ms": fused_graph_sec * 1e3 if fused_graph_sec else None,
            "entry": "g4d_render_backward_loss"},
        "forward_mpix_per_s": P_total / fwd_b / 1e6,
        **extra,
        "stage_ms_per_step": {k: ms / args.steps for k, (ms, n) in stages.items()},
        "adam_step_ms": adam_sec * 1e3, "adam_step_gb_per_s": adam_bytes / adam_sec / 1e9,
        "active_per_view": stats["active_per_view"], "instances": stats["instances"],
        "fragments": frag, "max_tile_list": stats["max_tile_list"],
        "roofline": roof,
        "stage_roofline": stage_roof,
        "other_workloads": others,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
