#!/usr/bin/env python
"""Throughput of the differentiable edge-sampling path tracer on one MI355X.

One step = drRender + drRenderBackward of the whole image: forward path
tracing with checkpoints, primary edge samples, and the path backward pass
(secondary edge samples at every vertex, interior adjoint, gradient scatter),
including the per-view edge table and edge hierarchy builds.

Workload (the benchmark metric's configuration): 512x512 pixels, 64 samples
per pixel, path depth 3, a level-6 icosphere (81,920 triangles) displaced by
seeded value noise inside a 12-triangle box lit by two quad lights (81,936
triangles), gradients w.r.t. vertices, per-triangle albedo and camera.
Inputs are seeded and synthetic and resident in HBM before timing starts.

Prints one JSON line (see the field list at the bottom).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0           # MI355X HBM3E, public figure
BVH_NODE_B = 64                 # bytes per BVH node fetch (two child boxes + links)
TRI_B = 48                      # bytes per triangle fetch (v0, e1, e2 as 3 x float4)
TREE_NODE_B = 168               # bytes per edge-tree node fetch (two children's bounds + links)
ATOMIC_B = 8                    # read + write of one FP32 gradient entry
BWD_UNIT_B = 2 * (4 + 12) + 1 + 4 + 4   # checkpoint reads (2 vertices), NEE bits, d_image, unit mask/ids


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1904_12228_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_traffic(workload: str):
    """HBM bytes per backward launch from the committed rocprofv3 --pmc summary
    (FETCH_SIZE + WRITE_SIZE), if it was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", f"k_backward_{workload}_traffic.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_hash") != kernel_source_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(cfg, threads):
    """The FP64 oracle (as it stands) on a bounded sample of the same workload:
    a 512x128-pixel band at the full 64 spp and depth 3, forward + backward."""
    import numpy as np

    import oracle
    cam = cfg.camera.with_window(0, 192, 512, 320)
    x0, y0, x1, y1 = cam.win()
    dimg = np.random.default_rng(1).normal(size=(y1 - y0, x1 - x0)) + 0.5
    units = (x1 - x0) * (y1 - y0) * cfg.spp
    t0 = time.perf_counter()
    oracle.render(cfg.scene, cam, cfg.spp, cfg.max_depth, 0, d_image=dimg, threads=threads)
    dt = time.perf_counter() - t0
    return {"value": units / dt, "unit": "samples/s", "cores": threads, "kind": "oracle",
            "sample": f"{x1 - x0}x{y1 - y0} pixel window of the 512x512 image at {cfg.spp} spp, depth "
                      f"{cfg.max_depth}: {units} fwd+bwd pixel samples in {dt:.1f} s (FP64, {threads} threads)"}


def proposal_leg(threads_note=None):
    """Learned edge proposal on the 1,000-triangle scene (direct lighting):
    harvest per-edge boundary magnitudes over 332 seeded training views
    (128x128, 16 spp: ~1.0 M (edge, view) rows), train the 32-64-64-1 network
    (600 full-batch Adam steps on the GPU), then compare the plain sampler and
    the 0.8/0.2 mixture on 16 held-out views at the configuration's 256x256
    and 16 spp, 64 seeds per view and sampler: gradient variance x backward
    time per term and for the whole gradient (d_image = 1), the learned time
    including its per-view proposal, with bootstrap 95% intervals and a
    per-entry Welch test of equal means."""
    from paper_1904_12228_amd import api, proposal, scenegen

    cfg = scenegen.config2()
    S = api.Scene(cfg.scene)
    train = [c for c, _ in scenegen.orbit_views(1, 332)]
    t0 = proposal.seconds()
    ds = proposal.harvest(S, train, 16, 1)
    t1 = proposal.seconds()
    prop = proposal.EdgeProposal(scenegen.mlp_params(0))
    loss0 = prop.loss(ds)
    prop.train(ds, 600)
    t2 = proposal.seconds()
    loss1 = prop.loss(ds)
    held = scenegen.orbit_views(99, 16, sizes=((256, 256),), spp=(16,))
    print("proposal: trained, evaluating", file=sys.stderr, flush=True)
    res = proposal.evaluate_protocol(S, prop, held, 1, list(range(1, 65)))
    S.close()
    return {"workload": "1,000-triangle soup + ground + quad light, depth 1; 16 held-out views 256x256 at 16 spp, "
                        "64 seeds per view and sampler; mixture 0.8 learned / 0.2 plain",
            "metric": "gradient variance x time gain (plain / learned), higher is better; 95% bootstrap interval",
            "train_views": len(train), "train_rows": int(ds.x.shape[0]), "harvest_s": t1 - t0, "train_s": t2 - t1,
            "train_loss": [loss0, loss1], "per_term": res, "gain_total": res["total"]["gain"],
            "gain_total_ci95": res["total"]["gain_ci95"]}


def _sampler_comparison(variants):
    """Gradient variance x backward time of the secondary term and of the whole
    gradient (d_image = 1), 64 seeds per sampler, on 4 views of the
    1,000-triangle scene (256x256, 16 spp, depth 1) and on a 128x128 window of
    the 81,936-triangle depth-3 scene (8 spp): the default sampler against each
    variant (keyword arguments of render_backward), with bootstrap intervals."""
    from paper_1904_12228_amd import api, proposal, scenegen

    out = {}
    for name, cfg, depth in (("config2", scenegen.config2(), 1), ("config3_window", scenegen.config3(), 3)):
        S = api.Scene(cfg.scene)
        if depth == 1:
            views = [(cfg.camera, 16)] + scenegen.orbit_views(77, 3, sizes=((256, 256),), spp=(16,))
        else:
            views = [(cfg.camera.with_window(192, 192, 320, 320), 8)]
        res = {}
        for term, terms in (("secondary", 4), ("total", 0)):
            base = []
            for i, (cam, spp) in enumerate(views):
                seeds = [s + 1000 * i for s in range(64)]
                G, ta = proposal.gradient_samples(S, cam, spp, depth, seeds, terms=terms)
                base.append((G, sorted(ta)[len(ta) // 2]))
            for vname, kw in variants:
                other = []
                for i, (cam, spp) in enumerate(views):
                    seeds = [s + 1000 * i + 500 for s in range(64)]
                    H, tb = proposal.gradient_samples(S, cam, spp, depth, seeds, terms=terms, **kw)
                    other.append((H, sorted(tb)[len(tb) // 2]))
                res.setdefault(vname, {})[term] = proposal.variance_time_stats(base, other)
            del base
        out[name] = res
        S.close()
        print(f"sampler comparison: {name} done", file=sys.stderr, flush=True)
    return out


def edge_points_leg():
    """Points on secondary edges drawn by the clamped cosine against uniform
    points (see _sampler_comparison)."""
    res = _sampler_comparison([("cosine", {"edge_t": 1})])
    return {"metric": "gradient variance x time gain (uniform points / clamped-cosine points), 95% bootstrap "
                      "interval", **{k: v["cosine"] for k, v in res.items()}}


def selection_leg():
    """Secondary edges chosen by M samples down the hierarchy and weighted
    reservoir selection (M = 4, 16) against one descent (see
    _sampler_comparison)."""
    res = _sampler_comparison([(f"M{m}", {"edge_candidates": m}) for m in (4, 16)])
    return {"metric": "gradient variance x time gain (one descent / M-sample selection), 95% bootstrap interval",
            **res}


def edge_nee_leg(alpha=0.25):
    """Next event estimation for edges (the strip strategy mixed in with
    probability alpha) against the hierarchy alone, secondary term (the only
    term it changes), 64 seeds per sampler and view, on 4 views of the
    1,000-triangle scene (256x256, 16 spp, depth 1), the same scene under a
    0.1 x 0.1 light of the same power, and a 128x128 window of the
    81,936-triangle depth-3 scene (8 spp). Two measures: the per-seed
    variance x backward time (as for the other samplers), and the squared
    error of the 64-seed mean against an independent 128-seed reference of
    the strip mixture, which also counts what a heavy-tailed sampler's seeds
    missed."""
    from paper_1904_12228_amd import api, proposal, scenegen

    scenes = (("config2", scenegen.config2(), 1),
              ("config2_small_light", scenegen.soup(0, 1000, 256, 256, 16, light_emission=250.0, light_size=0.1), 1),
              ("config3_window", scenegen.config3(), 3))
    out = {"metric": f"secondary-term gain (hierarchy / hierarchy mixed with edge strips crossed by segments to "
                     f"light points, probability {alpha}): variance x time and reference error x time, "
                     f"95% bootstrap intervals"}
    for name, cfg, depth in scenes:
        S = api.Scene(cfg.scene)
        if depth == 1:
            views = [(cfg.camera, 16)] + scenegen.orbit_views(77, 3, sizes=((256, 256),), spp=(16,))
        else:
            views = [(cfg.camera.with_window(192, 192, 320, 320), 8)]
        plain, other, refs, covered = [], [], [], [0, 0]
        for i, (cam, spp) in enumerate(views):
            G, ta = proposal.gradient_samples(S, cam, spp, depth, [s + 1000 * i for s in range(64)], terms=4)
            H, tb = proposal.gradient_samples(S, cam, spp, depth, [s + 1000 * i + 500 for s in range(64)], terms=4,
                                              edge_nee=alpha)
            R, _ = proposal.gradient_samples(S, cam, spp, depth, [s + 1000 * i + 100000 for s in range(128)],
                                             terms=4, edge_nee=alpha)
            plain.append((G, sorted(ta)[len(ta) // 2]))
            other.append((H, sorted(tb)[len(tb) // 2]))
            refs.append(R)
            covered[0] += int(((G != 0).double().mean(0) >= 0.9).sum())
            covered[1] += int(((H != 0).double().mean(0) >= 0.9).sum())
        out[name] = {"variance": proposal.variance_time_stats(plain, other),
                     "reference_error": proposal.reference_error_stats(plain, other, refs),
                     "entries_nonzero_in_90pct_of_seeds": covered}
        del plain, other, refs
        S.close()
        print(f"edge nee: {name} done", file=sys.stderr, flush=True)
    return out


def gbuffer_leg(S, cam, spp, d_image, reps=3):
    """Geometry buffers at the benchmark workload: position (3 channels),
    normal (3) and albedo, each rendered and differentiated (first hit,
    interior + primary edge term) with the same loss gradient image."""
    import torch

    H, W = d_image.shape
    dev = d_image.device
    bufs = torch.empty((7, H, W), dtype=torch.float32, device=dev)
    dv = torch.empty((S.num_vertices, 3), dtype=torch.float32, device=dev)
    da = torch.empty((S.num_triangles,), dtype=torch.float32, device=dev)
    dc = torch.empty((9,), dtype=torch.float32, device=dev)

    d7 = d_image.expand(7, H, W).contiguous()

    def all_step(i):
        S.render(cam, spp, 0, seed=i, out=bufs, aov=8)
        S.render_backward(cam, spp, 0, d7, seed=i, outs=(dv, da, dc), aov=8)

    def per_channel_step(i):
        for ch in range(1, 8):
            S.render(cam, spp, 0, seed=i, out=bufs[ch - 1], aov=ch)
            S.render_backward(cam, spp, 0, d_image, seed=i, outs=(dv, da, dc), aov=ch)

    res = {}
    for name, fn in (("all_channels_one_pass", all_step), ("one_pass_per_channel", per_channel_step)):
        fn(100)
        S.set_profiling(events=True, counters=False)
        S.profile(reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(reps):
            fn(i)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / reps
        prof = S.profile(reset=True)
        assert torch.isfinite(bufs).all() and torch.isfinite(dv).all(), "non-finite G-buffer output"
        res[name] = {"ms_per_gbuffer_step": ms, "pixel_samples_per_s": W * H * spp / (ms * 1e-3),
                     "kernel_ms_per_step": {k: prof[f"{k}_ms"] / reps for k in ("forward", "primary", "backward")}}
    return {"workload": f"{W}x{H}, {spp} spp, 7 channels (position xyz, normal xyz, albedo), forward + backward",
            **res}


# Adam learning rate by step for the inverse-rendering leg (piecewise constant)
INVERSE_SCHEDULE = [(0, 1e-3), (100, 5e-4), (150, 2.5e-4)]


def inverse_leg(steps=200):
    """Batched inverse rendering on the 1,000-triangle scene: 32 seeded views
    (128^2 to 512^2, 8 to 64 spp, depth 1) in one batch, target images of the
    true scene at 256 spp, the soup's vertices perturbed by N(0, 0.02^2) per
    coordinate, then `steps` Adam steps (learning rate INVERSE_SCHEDULE), each
    render -> loss gradient -> backward -> Adam -> refit captured as a HIP
    graph and replayed; launch shape from the autotuner."""
    import torch

    from paper_1904_12228_amd import api, batch, scenegen

    cfg = scenegen.config2()
    S = api.Scene(cfg.scene)
    views = scenegen.orbit_views(4, 32, sizes=((128, 128), (192, 192), (256, 256), (384, 384), (512, 512)),
                                 spp=(8, 16, 32, 64))
    B = batch.Batch(S, views, 1, seed=3)
    for d in B.d_images:
        d.fill_(1.0)
    tune = batch.autotune(B, reps=1, use_cache=False)
    true_v = S.vertices.clone()
    T = batch.Batch(S, [(c, 256) for c, _ in views], 1, seed=999)
    T.set_launch(*B.launch)
    T.forward()
    targets = [t.clone() for t in T.images]
    T.close()
    # vertices some view observes: nonzero gradient of a random weighting of
    # the images (hidden vertices cannot be recovered from images)
    g = torch.Generator(device="cuda").manual_seed(0)
    for d in B.d_images:
        d.copy_(torch.randn(d.shape, device="cuda", generator=g))
    infl = torch.empty((S.num_vertices, 3), dtype=torch.float32, device="cuda")
    B.forward()
    B.backward(infl)
    n_infl = infl.norm(dim=1)
    soup = torch.zeros(S.num_vertices, dtype=torch.bool, device="cuda")
    soup[:3 * 1000] = True
    thr = 1e-2 * float(n_infl[soup].max())
    mask = (soup & (n_infl > thr)).float()
    v0 = (true_v + 0.02 * torch.randn(true_v.shape, device="cuda", generator=g) * mask[:, None]).contiguous()
    inv = batch.InverseRendering(B, v0, targets, mask, schedule=INVERSE_SCHEDULE)
    err = lambda: float(((inv.v - true_v) ** 2 * mask[:, None]).sum().sqrt())
    curve = {0: err()}
    t0 = time.perf_counter()
    inv.step()
    loss0 = inv.loss()
    torch.cuda.synchronize()
    eager_ms = (time.perf_counter() - t0) * 1e3
    inv.capture()
    torch.cuda.synchronize()
    graph_ms = 0.0
    for i in range(inv.steps_done, steps):
        t1 = time.perf_counter()
        inv.step()
        torch.cuda.synchronize()
        graph_ms += (time.perf_counter() - t1) * 1e3
        if inv.steps_done in (50, 100, 150, 200):
            curve[inv.steps_done] = err()
            print(f"inverse rendering: step {inv.steps_done}", file=sys.stderr, flush=True)
    graph_ms /= max(steps - 2, 1)
    e1 = err()
    loss = inv.loss()
    B.close()
    S.close()
    return {"workload": "1,000-triangle soup + ground + light, 32 views 128^2..512^2 at 8..64 spp, depth 1; "
                        "Adam on the observed soup vertices from a N(0, 0.02^2) perturbation",
            "observed_vertices": int(mask.sum()), "samples_per_step": B.samples, "steps": steps, "ms_per_step_graph": graph_ms,
            "ms_per_step_eager_first": eager_ms, "samples_per_s": B.samples / (graph_ms * 1e-3),
            "autotune": tune, "lr_schedule": INVERSE_SCHEDULE, "vertex_error": [curve[0], e1],
            "vertex_error_by_step": curve, "error_ratio": e1 / curve[0], "hierarchy_rebuilds": inv.rebuilds,
            "image_loss": [loss0, loss]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="config3", choices=["config1", "config2", "config3"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-proposal", action="store_true", help="skip the learned-proposal variance x time leg")
    ap.add_argument("--no-inverse", action="store_true", help="skip the batched inverse-rendering leg")
    ap.add_argument("--no-gbuffer", action="store_true", help="skip the geometry-buffer leg")
    ap.add_argument("--no-selection", action="store_true",
                    help="skip the multi-sample edge selection vs one descent variance x time leg")
    ap.add_argument("--no-nee", action="store_true",
                    help="skip the next-event-estimation-for-edges vs hierarchy variance x time leg")
    ap.add_argument("--no-edge-points", action="store_true",
                    help="skip the clamped-cosine vs uniform edge-point variance x time leg")
    ap.add_argument("--cpu-threads", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--pmc-calibration", action="store_true",
                    help="first run one plain device copy of 256 MiB (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the renderer runs on one GPU; --gpus {args.gpus} is not supported "
              "(the gradient all-reduce across GPUs is not implemented)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1904_12228_amd import api, scenegen

    if args.pmc_calibration:
        src = torch.empty(64 << 20, dtype=torch.float32, device="cuda:0").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)              # reads and writes exactly 256 MiB
        torch.cuda.synchronize()
        del src, dst

    cfg = scenegen.CONFIGS[args.workload]()
    cam = cfg.camera
    W, H, spp, depth = cam.width, cam.height, cfg.spp, cfg.max_depth
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    S = api.Scene(cfg.scene, device=dev)
    d_image = torch.as_tensor(np.random.default_rng(0).normal(size=(H, W)) + 0.5, dtype=torch.float32, device=dev)
    img = torch.empty((H, W), dtype=torch.float32, device=dev)
    dv = torch.empty((S.num_vertices, 3), dtype=torch.float32, device=dev)
    da = torch.empty((S.num_triangles,), dtype=torch.float32, device=dev)
    dc = torch.empty((9,), dtype=torch.float32, device=dev)

    def step(i):
        S.render(cam, spp, depth, seed=i, out=img)
        S.render_backward(cam, spp, depth, d_image, seed=i, outs=(dv, da, dc))

    for i in range(args.warmup):
        step(1000 + i)
    torch.cuda.synchronize()
    print(f"warmup done ({args.warmup} steps)", file=sys.stderr, flush=True)

    # work counts per kernel launch (outside the timed region)
    S.set_profiling(events=False, counters=True)
    step(999)
    counts = S.profile(reset=True)["counts"]
    print("counting pass done", file=sys.stderr, flush=True)

    # timed region: per-kernel HIP events on the library's stream
    S.set_profiling(events=True, counters=False)
    S.profile(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(i)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = S.profile(reset=True)
    assert not S.device_error(), "device-side error flag set"
    assert torch.isfinite(img).all() and torch.isfinite(dv).all(), "non-finite output"
    print("timed steps done", file=sys.stderr, flush=True)

    ms = (t1 - t0) * 1e3 / args.steps
    samples = W * H * spp
    value = samples / (ms * 1e-3)
    units = W * H * spp
    bw = counts["backward"]
    bwd_bytes = (bw["bvh_nodes"] * BVH_NODE_B + bw["bvh_tris"] * TRI_B + bw["tree_nodes"] * TREE_NODE_B
                 + bw["atomics"] * ATOMIC_B + units * BWD_UNIT_B)
    bwd_ms = prof["backward_ms"] / max(prof["backward_launches"], 1)
    achieved = bwd_bytes / (bwd_ms * 1e-3) / 1e9
    kernels = {
        "forward_ms": prof["forward_ms"] / max(prof["forward_launches"], 1),
        "primary_ms": prof["primary_ms"] / max(prof["primary_launches"], 1),
        "backward_ms": bwd_ms,
        "other_ms": ms - (prof["forward_ms"] + prof["primary_ms"] + prof["backward_ms"]) / args.steps,
        "counts_per_step": counts,
        "tree_depths": {"bvh": prof["bvh_depth"], "edge_tree": prof["edge_tree_depth"]},
    }
    out = {
        "metric": "fwd+bwd samples/s at 512^2 64spp; grad variance x time, learned vs plain edge pdf",
        "value": value,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded scene generator)",
        "config": {"workload": f"{args.workload}: {W}x{H}, {spp} spp, depth {depth}, "
                               f"{S.num_triangles} triangles, {S.num_edges} edges",
                   "width": W, "height": H, "spp": spp, "max_depth": depth,
                   "triangles": S.num_triangles, "edges": S.num_edges},
        "roofline": {"bound": "hbm",
                     "kernel": "path backward (k_bwd_sample_v + k_side + k_bwd_adjoint: secondary edges, "
                               "interior adjoint, scatter)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": read_traffic(args.workload),
                     "algorithmic_bytes_per_launch": bwd_bytes,
                     # the numerator counts measured fetches: a worse tree would raise it, so the
                     # fetches per ray and per descent are reported beside it
                     "bvh_nodes_per_ray": bw["bvh_nodes"] / max(bw["rays"], 1),
                     "edge_tree_nodes_per_unit_vertex": bw["tree_nodes"] / max(units * depth, 1)},
        "kernels": kernels,
    }
    if not args.no_gbuffer:
        print("running the geometry-buffer leg", file=sys.stderr, flush=True)
        out["gbuffer"] = gbuffer_leg(S, cam, spp, d_image)
    if not args.no_proposal:
        print("running the learned-proposal leg", file=sys.stderr, flush=True)
        out["proposal"] = proposal_leg()
    if not args.no_edge_points:
        print("running the edge-point sampling leg", file=sys.stderr, flush=True)
        out["edge_points"] = edge_points_leg()
    if not args.no_selection:
        print("running the edge-selection leg", file=sys.stderr, flush=True)
        out["edge_selection"] = selection_leg()
    if not args.no_nee:
        print("running the next-event-estimation-for-edges leg", file=sys.stderr, flush=True)
        out["edge_nee"] = edge_nee_leg()
    if not args.no_inverse:
        print("running the batched inverse-rendering leg", file=sys.stderr, flush=True)
        out["inverse_rendering"] = inverse_leg()
    if not args.no_cpu_baseline:
        print("running the CPU oracle baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_threads)
    S.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
