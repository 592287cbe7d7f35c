"""Learned edge proposal: bindings of drEdgeFeatures / drMlpForward /
drMlpSoftmaxXent / drMlpBackward, and the harvest -> train -> propose loop.

The thesis samples edges by importance with a hand-built pdf (Ch. 5,
Importance Sampling the Edges). Here a 32-64-64-1 network, evaluated and
trained by the library's BF16 matrix-core kernels, proposes a per-view
distribution over edges; drRenderBackward mixes it with the plain pdf
(weight `mix`), so the gradient estimate stays unbiased. The training target
is the renderer's own harvest statistic: per edge, sum of P |c|^2 over its
boundary samples, whose expectation E|G_e|^2 does not depend on the sampler.
The variance-optimal probability of an edge is proportional to sqrt(E|G_e|^2)
(minimise sum_e E|G_e|^2 / P_e subject to sum_e P_e = 1), so the target
distribution of a view is sqrt(harvest) normalised.

Tensors only carry device memory; every step runs in libdiffrt.so.
"""
from __future__ import annotations

import ctypes as C
import time
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib, api


def _s():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _p(t):
    return C.c_void_p(0 if t is None else t.data_ptr())


def _f32(t, dev):
    return torch.as_tensor(t, dtype=torch.float32, device=dev).contiguous()


def mlp_forward(theta: torch.Tensor, x: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
    n = int(x.shape[0])
    assert theta.numel() == _lib.MLP_PARAMS and x.shape[1] == _lib.EDGE_FEATURES and x.is_contiguous()
    z = out if out is not None else torch.empty(n, dtype=torch.float32, device=x.device)
    _lib.check(_lib.load().drMlpForward(_p(theta), _p(x), n, _p(z), _s()), "drMlpForward")
    return z


def softmax_xent(z: torch.Tensor, target: torch.Tensor | None, offsets: torch.Tensor, want_prob=True):
    """Per-view softmax (and cross-entropy with the normalised target):
    returns prob, d_logits, per-view loss (the latter two None without target)."""
    nv = int(offsets.numel()) - 1
    assert offsets.dtype == torch.int32 and offsets.is_contiguous()
    prob = torch.empty_like(z) if want_prob else None
    dz = torch.empty_like(z) if target is not None else None
    vl = torch.empty(max(nv, 1), dtype=torch.float32, device=z.device) if target is not None else None
    scratch = torch.empty(max(nv, 1), dtype=torch.float32, device=z.device)
    _lib.check(_lib.load().drMlpSoftmaxXent(_p(z), _p(target), _p(offsets), nv, _p(prob), _p(dz), _p(vl),
                                            _p(scratch), _s()), "drMlpSoftmaxXent")
    return prob, dz, vl


def mlp_backward(theta: torch.Tensor, x: torch.Tensor, dz: torch.Tensor, out: torch.Tensor | None = None):
    g = out if out is not None else torch.empty(_lib.MLP_PARAMS, dtype=torch.float32, device=x.device)
    _lib.check(_lib.load().drMlpBackward(_p(theta), _p(x), int(x.shape[0]), _p(dz), _p(g), _s()), "drMlpBackward")
    return g


def adam_step(x, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    _lib.check(_lib.load().drAdamStep(_p(x), _p(g), _p(m), _p(v), x.numel(), float(lr), float(b1), float(b2),
                                      float(eps), int(step), _s()), "drAdamStep")


# ---------------------------------------------------------------------------
# harvest -> train -> propose
# ---------------------------------------------------------------------------
@dataclass
class Dataset:
    x: torch.Tensor          # [views * E, 32]
    target: torch.Tensor     # [views * E] sqrt(harvest), per view
    offsets: torch.Tensor    # [views + 1] int32


def harvest(scene: api.Scene, cams, spp, depth, seed0=0, d_image=1.0, terms=0) -> Dataset:
    """Features and targets of every (edge, view): one backward pass per view
    with the plain sampler and the harvest statistic on."""
    dev = scene.device
    E = scene.num_edges
    xs, ts = [], []
    stats = torch.empty(E, dtype=torch.float32, device=dev)
    for i, cam in enumerate(cams):
        x0, y0, x1, y1 = cam.win()
        dimg = torch.full((y1 - y0, x1 - x0), float(d_image), dtype=torch.float32, device=dev)
        scene.render_backward(cam, spp, depth, dimg, seed=seed0 + i, terms=terms, want=(), edge_stats=stats)
        ts.append(torch.sqrt(torch.clamp(stats, min=0.0)))
        xs.append(scene.edge_features(cam))
    off = torch.arange(0, (len(cams) + 1) * E, E, dtype=torch.int32, device=dev)
    return Dataset(torch.cat(xs).contiguous(), torch.cat(ts).contiguous(), off)


class EdgeProposal:
    """The network's FP32 master parameters and Adam state on the device."""

    def __init__(self, theta0: np.ndarray, device="cuda"):
        self.theta = _f32(theta0, device)
        self.m = torch.zeros_like(self.theta)
        self.v = torch.zeros_like(self.theta)
        self.grad = torch.zeros_like(self.theta)
        self.step = 0

    def train(self, data: Dataset, steps: int, lr=3e-3, log_every=0):
        """Full-batch Adam on the mean per-view cross-entropy; returns the losses."""
        z = torch.empty(data.x.shape[0], dtype=torch.float32, device=data.x.device)
        losses = []
        for it in range(steps):
            mlp_forward(self.theta, data.x, out=z)
            _, dz, vl = softmax_xent(z, data.target, data.offsets, want_prob=False)
            mlp_backward(self.theta, data.x, dz, out=self.grad)
            self.step += 1
            adam_step(self.theta, self.grad, self.m, self.v, self.step, lr)
            if log_every and (it % log_every == 0 or it == steps - 1):
                used = (vl != 0).sum().clamp(min=1)
                losses.append(float(vl.sum() / used))
        return losses

    def loss(self, data: Dataset) -> float:
        z = mlp_forward(self.theta, data.x)
        _, _, vl = softmax_xent(z, data.target, data.offsets, want_prob=False)
        return float(vl.sum() / (vl != 0).sum().clamp(min=1))

    def propose(self, scene: api.Scene, cam) -> torch.Tensor:
        """The proposal distribution over the scene's edges for this view."""
        x = scene.edge_features(cam)
        z = mlp_forward(self.theta, x)
        off = torch.tensor([0, scene.num_edges], dtype=torch.int32, device=x.device)
        p, _, _ = softmax_xent(z, None, off)
        return p


def gradient_variance_time(scene: api.Scene, cam, spp, depth, seeds, edge_pdf=None, mix=0.0, mix_terms=0,
                           d_image=1.0, terms=0, edge_t=0, edge_candidates=0, edge_nee=0.0):
    """Sum over vertex-gradient entries of the variance of the estimate across
    seeds, the mean gradient, and the mean time of one drRenderBackward (HIP
    events around the call, forward checkpoints excluded)."""
    dev = scene.device
    x0, y0, x1, y1 = cam.win()
    dimg = torch.full((y1 - y0, x1 - x0), float(d_image), dtype=torch.float32, device=dev)
    dv = torch.empty((scene.num_vertices, 3), dtype=torch.float32, device=dev)
    acc = torch.zeros((scene.num_vertices, 3), dtype=torch.float64, device=dev)
    acc2 = torch.zeros_like(acc)
    ms = 0.0
    st = torch.cuda.current_stream()
    for sd in seeds:
        scene.render(cam, spp, depth, seed=sd)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        scene.render_backward(cam, spp, depth, dimg, seed=sd, terms=terms, want=("vertices",), outs=(dv, None, None),
                              edge_pdf=edge_pdf, edge_mix=mix, edge_mix_terms=mix_terms, edge_t=edge_t,
                              edge_candidates=edge_candidates, edge_nee=edge_nee)
        e1.record(st)
        e1.synchronize()
        ms += e0.elapsed_time(e1)
        g = dv.double()
        acc += g
        acc2 += g * g
    n = len(seeds)
    mean = acc / n
    var = (acc2 / n - mean * mean) * n / (n - 1)
    return float(var.clamp(min=0).sum()), mean, ms / n


def gradient_samples(scene: api.Scene, cam, spp, depth, seeds, edge_pdf=None, mix=0.0, mix_terms=0, d_image=1.0,
                     terms=0, edge_t=0, edge_candidates=0, edge_nee=0.0):
    """Per-seed vertex gradients [len(seeds), 3V] (float64, device) and the
    drRenderBackward duration of each seed in ms (HIP events around the call,
    forward checkpoints excluded)."""
    dev = scene.device
    x0, y0, x1, y1 = cam.win()
    dimg = torch.full((y1 - y0, x1 - x0), float(d_image), dtype=torch.float32, device=dev)
    dv = torch.empty((scene.num_vertices, 3), dtype=torch.float32, device=dev)
    out = torch.empty((len(seeds), 3 * scene.num_vertices), dtype=torch.float64, device=dev)
    ms = []
    st = torch.cuda.current_stream()
    for i, sd in enumerate(seeds):
        scene.render(cam, spp, depth, seed=sd)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        scene.render_backward(cam, spp, depth, dimg, seed=sd, terms=terms, want=("vertices",), outs=(dv, None, None),
                              edge_pdf=edge_pdf, edge_mix=mix, edge_mix_terms=mix_terms, edge_t=edge_t,
                              edge_candidates=edge_candidates, edge_nee=edge_nee)
        e1.record(st)
        e1.synchronize()
        ms.append(e0.elapsed_time(e1))
        out[i] = dv.reshape(-1).double()
    return out, ms


def variance_time_stats(plain, other, n_boot=500, seed=0):
    """Gradient variance x time of two samplers over the same views.
    plain / other: lists (one per view) of (samples [K, N], time_ms). The
    variance is the per-entry sample variance across seeds summed over entries
    and views; the time the mean over views of each view's time. Returns the
    gain (plain / other) with a bootstrap 95% interval (seeds resampled with
    replacement per view and sampler, times held fixed), and a per-entry Welch
    test of equal means (fraction of (view, entry) pairs beyond 4 standard
    errors)."""
    def var_sum(G, idx=None):
        X = G if idx is None else G[idx]
        return float(X.var(0, unbiased=True).sum())

    vp = sum(var_sum(G) for G, _ in plain)
    vo = sum(var_sum(G) for G, _ in other)
    tp = sum(t for _, t in plain) / len(plain)
    to = sum(t for _, t in other) / len(other)
    gain = (vp * tp) / (vo * to) if vo * to > 0 else float("nan")
    gen = torch.Generator(device=plain[0][0].device).manual_seed(seed)
    boots = []
    for _ in range(n_boot):
        bp = bo = 0.0
        for (G, _), (H, _) in zip(plain, other):
            K, L = G.shape[0], H.shape[0]
            bp += var_sum(G, torch.randint(0, K, (K,), device=G.device, generator=gen))
            bo += var_sum(H, torch.randint(0, L, (L,), device=H.device, generator=gen))
        boots.append((bp * tp) / (bo * to) if bo > 0 else float("nan"))
    boots = sorted(boots)
    lo, hi = boots[int(0.025 * n_boot)], boots[int(0.975 * n_boot) - 1]
    beyond = total = 0
    for (G, _), (H, _) in zip(plain, other):
        se = torch.sqrt(G.var(0) / G.shape[0] + H.var(0) / H.shape[0])
        ok = se > 0
        z = (G.mean(0) - H.mean(0)).abs()[ok] / se[ok]
        beyond += int((z > 4).sum())
        total += int(ok.sum())
    return {"var_plain": vp, "var_other": vo, "ms_plain": tp, "ms_other": to, "gain": gain,
            "gain_ci95": [lo, hi], "welch_beyond_4se": beyond, "welch_entries": total}


def reference_error_stats(plain, other, refs, n_boot=500, seed=0):
    """Squared error of each sampler's seed-averaged gradient against an
    independent reference of the same expectation. plain / other: lists (one
    per view) of (samples [K, N], time_ms); refs: per view, reference samples
    [R, N] from seeds neither sampler used. Per sampler, err = K x (sum over
    views and entries of (mean over its K seeds - reference mean)^2 minus the
    reference mean's own variance): an estimate of the per-seed variance that
    also charges a heavy-tailed sampler for the contributions its seeds
    missed (the sample variance around the sample's own mean does not).
    Returns both errors, the gain err_plain t_plain / (err_other t_other)
    and a bootstrap 95% interval (the samplers' seeds resampled, the
    reference held fixed)."""
    def err(pairs, idx_fn=None):
        tot = 0.0
        for (G, _), R in zip(pairs, refs):
            X = G if idx_fn is None else G[idx_fn(G.shape[0])]
            rm = R.mean(0)
            tot += X.shape[0] * (float(((X.mean(0) - rm) ** 2).sum()) - float(R.var(0).sum()) / R.shape[0])
        return tot

    ep, eo = err(plain), err(other)
    tp = sum(t for _, t in plain) / len(plain)
    to = sum(t for _, t in other) / len(other)
    gain = (ep * tp) / (eo * to) if eo * to > 0 else float("nan")
    gen = torch.Generator(device=plain[0][0].device).manual_seed(seed)
    pick = lambda K: torch.randint(0, K, (K,), device=plain[0][0].device, generator=gen)
    boots = sorted((err(plain, pick) * tp) / (err(other, pick) * to) for _ in range(n_boot))
    lo, hi = boots[int(0.025 * n_boot)], boots[int(0.975 * n_boot) - 1]
    return {"err_plain": ep, "err_other": eo, "ms_plain": tp, "ms_other": to, "gain": gain, "gain_ci95": [lo, hi]}


def seconds() -> float:
    torch.cuda.synchronize()
    return time.perf_counter()


def propose_ms(scene: api.Scene, prop: "EdgeProposal", cam, reps=5) -> float:
    """Median time of one proposal (edge features, network, softmax) in ms."""
    st = torch.cuda.current_stream()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        prop.propose(scene, cam)
        e1.record(st)
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    return sorted(ts)[len(ts) // 2]


def evaluate_protocol(scene: api.Scene, prop: "EdgeProposal", views, depth, seeds, mix=0.8, d_image=1.0,
                      n_boot=500) -> dict:
    """The learned mixture against the plain sampler on held-out views: per
    term (primary edges, secondary edges, whole gradient) the variance x time
    gain with a bootstrap 95% interval and a Welch test of equal means. The
    learned sampler's time includes its proposal (features, network,
    softmax); times are medians over seeds."""
    out = {}
    qs = [prop.propose(scene, cam) for cam, _ in views]
    pms = [propose_ms(scene, prop, cam) for cam, _ in views]
    for name, terms, mterms in (("primary", 2, 2), ("secondary", 4, 4), ("total", 0, 6)):
        plain, learned = [], []
        for i, (cam, spp) in enumerate(views):
            G, ta = gradient_samples(scene, cam, spp, depth, [s + 10007 * i for s in seeds], terms=terms,
                                     d_image=d_image)
            H, tb = gradient_samples(scene, cam, spp, depth, [s + 10007 * i + 5003 for s in seeds], edge_pdf=qs[i],
                                     mix=mix, mix_terms=mterms, terms=terms, d_image=d_image)
            plain.append((G, sorted(ta)[len(ta) // 2]))
            learned.append((H, sorted(tb)[len(tb) // 2] + pms[i]))
        out[name] = variance_time_stats(plain, learned, n_boot=n_boot)
    out["propose_ms"] = sum(pms) / len(pms)
    return out


def evaluate(scene: api.Scene, prop: EdgeProposal, views, depth, seeds, mix=0.8, d_image=1.0) -> dict:
    """Gradient variance x time of the plain sampler and of the learned
    mixture on the given views [(Camera, spp)], per term of the estimator
    (primary edges, secondary edges) and for the whole gradient. Variances
    are summed over views; times are the mean drRenderBackward durations."""
    out = {}
    for name, terms, mterms in (("primary", 2, 2), ("secondary", 4, 4), ("total", 0, 6)):
        vp = vm = tp = tm = 0.0
        for i, (cam, spp) in enumerate(views):
            q = prop.propose(scene, cam)
            a, _, ta = gradient_variance_time(scene, cam, spp, depth, [s + 10007 * i for s in seeds], terms=terms,
                                              d_image=d_image)
            b, _, tb = gradient_variance_time(scene, cam, spp, depth, [s + 10007 * i + 5003 for s in seeds],
                                              edge_pdf=q, mix=mix, mix_terms=mterms, terms=terms, d_image=d_image)
            vp += a
            vm += b
            tp += ta / len(views)
            tm += tb / len(views)
        out[name] = {"var_plain": vp, "var_learned": vm, "ms_plain": tp, "ms_learned": tm,
                     "gain": (vp * tp) / (vm * tm) if vm * tm > 0 else float("nan")}
    return out
