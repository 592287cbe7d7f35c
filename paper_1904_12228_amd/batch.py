"""Batched multi-view rendering, a torch.autograd.Function over a batch, an
inverse-rendering loop captured in one HIP graph, and a launch autotuner.

The thesis optimises scene parameters from images with Adam, rendering and
differentiating each iteration (Ch. 5, Results). Here all views of a step
(each with its own image size and sample count) go through one kernel launch
per pass (drBatchForward / drBatchBackward), and one optimisation step --
vertex refit, per-view table refit, forward, loss gradient, backward, Adam --
is captured once as a HIP graph and replayed. Tensors only carry device
memory and streams; every step of the path runs in libdiffrt.so.
"""
from __future__ import annotations

import ctypes as C
import hashlib
import json
import os
import time

import torch

from . import _lib, api


def _s():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _p(t):
    return C.c_void_p(0 if t is None else t.data_ptr())


def scene_refit(scene: api.Scene, vertices: torch.Tensor):
    """Capturable vertex update (BVH refit over the existing topology)."""
    assert vertices.dtype == torch.float32 and vertices.is_contiguous() and vertices.numel() == 3 * scene.num_vertices
    _lib.check(_lib.load().drSceneRefit(scene._h, _p(vertices), _s()), "drSceneRefit")


class Batch:
    """Views [(Camera, spp)] of one scene, all with path depth `depth`.
    images[v] / d_images[v] are [H, W] device tensors owned here."""

    def __init__(self, scene: api.Scene, views, depth: int, seed: int = 0, unit_masks=None):
        self.scene = scene
        self.views = list(views)
        n = len(self.views)
        dev = scene.device
        self.images, self.d_images = [], []
        cams = (_lib.Camera * n)()
        opts = (_lib.RenderOptions * n)()
        for i, (cam, spp) in enumerate(self.views):
            x0, y0, x1, y1 = cam.win()
            self.images.append(torch.zeros((y1 - y0, x1 - x0), dtype=torch.float32, device=dev))
            self.d_images.append(torch.zeros((y1 - y0, x1 - x0), dtype=torch.float32, device=dev))
            cams[i] = api.camera_struct(cam)
            opts[i] = api.options_struct(spp, depth, seed, i)
            if unit_masks is not None and unit_masks[i] is not None:
                opts[i].unit_mask = unit_masks[i].data_ptr()
        self.unit_masks = unit_masks      # read by every pass: kept alive with the batch
        ip = (C.c_void_p * n)(*[t.data_ptr() for t in self.images])
        dp = (C.c_void_p * n)(*[t.data_ptr() for t in self.d_images])
        h = C.c_void_p()
        _lib.check(_lib.load().drBatchCreate(C.byref(h), scene._h, n, cams, opts, ip, dp, _s()), "drBatchCreate")
        self._h = h
        self.depth = depth
        self.samples = sum((c.win()[2] - c.win()[0]) * (c.win()[3] - c.win()[1]) * spp for c, spp in self.views)
        self.launch = (0, 1)

    def set_launch(self, ctas: int, chunk: int):
        _lib.check(_lib.load().drBatchSetLaunch(self._h, int(ctas), int(chunk)), "drBatchSetLaunch")
        self.launch = (int(ctas), int(chunk))

    def refit(self):
        _lib.check(_lib.load().drBatchRefit(self._h, _s()), "drBatchRefit")

    def check_hierarchy(self) -> bool:
        """Rebuilds the views' edge hierarchies if the last refit moved an
        edge into a discontinuity class its kept hierarchy cannot represent
        (synchronises); returns whether it rebuilt."""
        flag = C.c_int32(0)
        _lib.check(_lib.load().drBatchCheckHierarchy(self._h, C.byref(flag), _s()), "drBatchCheckHierarchy")
        return bool(flag.value)

    def advance_seed(self):
        _lib.check(_lib.load().drBatchAdvanceSeed(self._h, _s()), "drBatchAdvanceSeed")

    def forward(self):
        _lib.check(_lib.load().drBatchForward(self._h, _s()), "drBatchForward")

    def backward(self, d_vertices=None, d_albedo=None, d_cameras=None):
        _lib.check(_lib.load().drBatchBackward(self._h, _p(d_vertices), _p(d_albedo), _p(d_cameras), _s()),
                   "drBatchBackward")

    def config_hash(self) -> str:
        h = hashlib.sha256()
        h.update(f"{self.scene.num_triangles}/{self.scene.num_edges}/{self.depth}".encode())
        for cam, spp in self.views:
            h.update(f"{cam.win()}/{spp}".encode())
        return h.hexdigest()[:16]

    def close(self):
        if getattr(self, "_h", None):
            _lib.load().drBatchDestroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchRenderFn(torch.autograd.Function):
    """images = render(vertices) for every view of a batch; backward gives
    d loss / d vertices through drBatchBackward."""

    @staticmethod
    def forward(ctx, vertices, batch: Batch):
        scene_refit(batch.scene, vertices.detach().contiguous())
        batch.refit()
        batch.check_hierarchy()
        batch.advance_seed()
        batch.forward()
        ctx.batch = batch
        return tuple(img.clone() for img in batch.images)

    @staticmethod
    def backward(ctx, *grads):
        b = ctx.batch
        for dst, g in zip(b.d_images, grads):
            if g is None:
                dst.zero_()
            else:
                dst.copy_(g)
        dv = torch.empty((b.scene.num_vertices, 3), dtype=torch.float32, device=b.scene.device)
        b.backward(dv)
        return dv, None


def render_views(vertices: torch.Tensor, batch: Batch):
    return BatchRenderFn.apply(vertices, batch)


class InverseRendering:
    """Adam on vertex positions to match target images of every view:
    loss = sum over views of mean over pixels (I_v - T_v)^2. `mask` [V] (1 =
    optimised). One step is new seed -> forward -> loss gradient -> backward
    -> Adam -> refit of the scene and the views to the new vertices, all on
    one stream; `capture()` records it once as a HIP graph for replay. After
    every step the host reads the refit's hierarchy flag and, when an edge
    changed discontinuity class, rebuilds the hierarchies (and captures the
    graph again) before the next step renders."""

    def __init__(self, batch: Batch, vertices0: torch.Tensor, targets, mask: torch.Tensor, lr=2e-3, schedule=None):
        dev = batch.scene.device
        self.b = batch
        self.v = vertices0.detach().clone().contiguous()
        self.targets = [t.detach().to(dev, torch.float32).contiguous() for t in targets]
        self.mask = mask.to(dev, torch.float32).reshape(-1, 1).expand(-1, 3).contiguous()
        self.grad = torch.zeros_like(self.v)
        self.m = torch.zeros_like(self.v)
        self.s = torch.zeros_like(self.v)
        self.step_count = torch.zeros(1, dtype=torch.int64, device=dev)
        # learning-rate schedule: [(first step, lr), ...], piecewise constant;
        # a change re-captures the graph (its Adam launch carries the rate)
        self.schedule = sorted((int(k), float(v)) for k, v in (schedule or [(0, lr)]))
        self.lr = self.schedule[0][1]
        self.steps_done = 0
        self.scale = [2.0 / t.numel() for t in self.targets]
        self.graph = None
        self.rebuilds = 0
        scene_refit(batch.scene, self.v)
        batch.refit()
        self._check()

    def _check(self):
        if self.b.check_hierarchy():
            self.rebuilds += 1
            if self.graph is not None:
                self.graph = None
                self._capture_only()

    def _step(self):
        b = self.b
        b.advance_seed()
        b.forward()
        for img, tgt, dimg, sc in zip(b.images, self.targets, b.d_images, self.scale):
            torch.sub(img, tgt, out=dimg)
            dimg.mul_(sc)
        b.backward(self.grad)
        self.grad.mul_(self.mask)
        _lib.check(_lib.load().drAdamStepCounted(_p(self.v), _p(self.grad), _p(self.m), _p(self.s), self.v.numel(),
                                                 self.lr, 0.9, 0.999, 1e-8, _p(self.step_count), _s()),
                   "drAdamStepCounted")
        scene_refit(b.scene, self.v)
        b.refit()

    def _lr_at(self, k):
        lr = self.schedule[0][1]
        for first, v in self.schedule:
            if k >= first:
                lr = v
        return lr

    def step(self):
        lr = self._lr_at(self.steps_done)
        if lr != self.lr:
            self.lr = lr
            if self.graph is not None:
                self._capture_only()
        if self.graph is not None:
            self.graph.replay()
        else:
            self._step()
        self.steps_done += 1
        self._check()

    def _capture_only(self):
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self._step()
        self.graph = g

    def capture(self):
        """Record one step as a HIP graph (after one eager warm-up step on the
        capture stream, which also advances the optimisation by one step)."""
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        self.lr = self._lr_at(self.steps_done)
        with torch.cuda.stream(side):
            self._step()
        torch.cuda.current_stream().wait_stream(side)
        self.steps_done += 1
        self._check()
        self.lr = self._lr_at(self.steps_done)
        self._capture_only()
        return self.graph

    def loss(self) -> float:
        return float(sum(((img - t) ** 2).mean() for img, t in zip(self.b.images, self.targets)))


# ---------------------------------------------------------------------------
# launch autotuner
# ---------------------------------------------------------------------------
CANDIDATES = [(0, 1), (0, 2), (0, 4), (1024, 1), (2048, 1), (2048, 2), (4096, 1), (4096, 4), (8192, 2)]


def _cache_path():
    base = os.environ.get("XDG_CACHE_HOME") or os.path.join(os.path.expanduser("~"), ".cache")
    return os.path.join(base, "paper_1904_12228_amd", "autotune.json")


def autotune(batch: Batch, reps: int = 2, use_cache: bool = True, candidates=CANDIDATES) -> dict:
    """Times forward + backward of the batch for each launch shape (workgroups
    per launch, blocks per work item), keeps the fastest, and caches the
    choice per (GPU name, batch configuration)."""
    key = f"{torch.cuda.get_device_name()}|{batch.config_hash()}"
    path = _cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            cache = json.load(open(path))
        except (OSError, ValueError):
            cache = {}
    if use_cache and key in cache:
        ctas, chunk = cache[key]["launch"]
        batch.set_launch(ctas, chunk)
        return dict(cache[key], cached=True)
    dv = torch.empty((batch.scene.num_vertices, 3), dtype=torch.float32, device=batch.scene.device)
    times = {}
    for ctas, chunk in candidates:
        batch.set_launch(ctas, chunk)
        batch.forward()
        batch.backward(dv)             # warm-up of this shape
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            batch.forward()
            batch.backward(dv)
        torch.cuda.synchronize()
        times[f"{ctas}/{chunk}"] = (time.perf_counter() - t0) * 1e3 / reps
    best = min(times, key=times.get)
    ctas, chunk = (int(x) for x in best.split("/"))
    batch.set_launch(ctas, chunk)
    res = {"launch": [ctas, chunk], "ms": times[best], "all_ms": times}
    if use_cache:
        cache[key] = res
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            json.dump(cache, open(path, "w"), indent=1)
        except OSError:
            pass
    return dict(res, cached=False)
