"""PyTorch integration: a torch.autograd.Function around drRender /
drRenderBackward, and Adam on device (drAdamStep).

The thesis's renderer takes scenes as PyTorch tensors and back-propagates a
scalar loss of the output image to the scene parameters, optimising them with
Adam (Ch. 5, Results). Here the tensors only carry device memory: rendering,
differentiation and the optimiser step all run in libdiffrt.so.
"""
from __future__ import annotations

import ctypes as C

import torch

from . import _lib, api
from .scenegen import Camera


class _RenderFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, vertices, camera9, albedo, scene: api.Scene, cam: Camera, spp: int, depth: int, seed: int,
                view_id: int, unit_mask):
        # the BVH topology is kept (refit): no host build inside an optimisation loop
        scene.refit_vertices(vertices.detach())
        if albedo is not None:
            scene.update_albedo(albedo.detach())
        c = Camera.from_params9(camera9.detach().cpu().numpy(), cam)
        img = scene.render(c, spp, depth, seed=seed, view_id=view_id, unit_mask=unit_mask)
        ctx.args = (scene, c, spp, depth, seed, view_id, unit_mask)
        ctx.cam_device = camera9.device
        ctx.has_albedo = albedo is not None
        return img

    @staticmethod
    def backward(ctx, d_img):
        scene, c, spp, depth, seed, view_id, unit_mask = ctx.args
        want = ("vertices", "camera", "albedo") if ctx.has_albedo else ("vertices", "camera")
        dv, da, dc = scene.render_backward(c, spp, depth, d_img.contiguous(), seed=seed, view_id=view_id,
                                           unit_mask=unit_mask, want=want)
        return dv, dc.to(ctx.cam_device), da, None, None, None, None, None, None, None


def render(scene: api.Scene, vertices: torch.Tensor, camera9: torch.Tensor, cam: Camera, spp: int, depth: int,
           seed: int = 0, view_id: int = 0, albedo: torch.Tensor | None = None, unit_mask=None) -> torch.Tensor:
    """Differentiable render: image of `scene` with the given vertex positions
    ([V,3] on the scene's device), camera (9 numbers: position, look_at, up;
    fov and image size from `cam`) and, optionally, per-triangle albedo ([T];
    then its gradient is returned too). unit_mask as in Scene.render."""
    return _RenderFn.apply(vertices, camera9, albedo, scene, cam, spp, depth, seed, view_id, unit_mask)


ALL_CHANNELS = (1, 2, 3, 4, 5, 6, 7)


class _GBufferFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, vertices, camera9, albedo, scene: api.Scene, cam: Camera, spp: int, seed: int, channels, unit_mask):
        scene.update_vertices(vertices)
        if albedo is not None:
            scene.update_albedo(albedo)
        c = Camera.from_params9(camera9.detach().cpu().numpy(), cam)
        x0, y0, x1, y1 = c.win()
        out = torch.empty((len(channels), y1 - y0, x1 - x0), dtype=torch.float32, device=vertices.device)
        if tuple(channels) == ALL_CHANNELS:
            scene.render(c, spp, 0, seed=seed, unit_mask=unit_mask, out=out, aov=8)
        else:
            for i, ch in enumerate(channels):
                scene.render(c, spp, 0, seed=seed, unit_mask=unit_mask, out=out[i], aov=ch)
        ctx.args = (scene, c, spp, seed, tuple(channels), unit_mask)
        ctx.cam_device = camera9.device
        ctx.has_albedo = albedo is not None
        return out

    @staticmethod
    def backward(ctx, d_out):
        scene, c, spp, seed, channels, unit_mask = ctx.args
        if channels == ALL_CHANNELS:
            dv, da, dc = scene.render_backward(c, spp, 0, d_out.contiguous(), seed=seed, unit_mask=unit_mask, aov=8)
            return dv, dc.to(ctx.cam_device), da if ctx.has_albedo else None, None, None, None, None, None, None
        dv = dc = da = None
        for i, ch in enumerate(channels):
            g = d_out[i].contiguous()
            v, a, k = scene.render_backward(c, spp, 0, g, seed=seed, unit_mask=unit_mask, aov=ch)
            dv = v if dv is None else dv + v
            da = a if da is None else da + a
            dc = k if dc is None else dc + k
        return dv, dc.to(ctx.cam_device), da if ctx.has_albedo else None, None, None, None, None, None, None


def gbuffer(scene: api.Scene, vertices: torch.Tensor, camera9: torch.Tensor, cam: Camera, spp: int, seed: int = 0,
            channels=ALL_CHANNELS, albedo: torch.Tensor | None = None, unit_mask=None) -> torch.Tensor:
    """Differentiable geometry buffers [len(channels), H, W] (channel numbers
    as in api.AOV: 1-3 position, 4-6 normal facing the camera, 7 albedo), each
    the box-filtered mean of its value at the first hit of `spp` camera rays
    per pixel (0 where a ray escapes). Gradients reach vertices, camera and,
    when given, albedo ([T]); a deferred-shading function of the buffers
    written in torch differentiates through them (Ch. 5, Results: G-buffers
    and deferred shading). The seven channels in order take one forward and
    one backward call (aov = 8), other selections one call per channel."""
    return _GBufferFn.apply(vertices, camera9, albedo, scene, cam, spp, seed, tuple(channels), unit_mask)


class DeviceAdam:
    """Adam with bias correction, one drAdamStep launch per parameter tensor."""

    def __init__(self, params, lr=1e-3, betas=(0.9, 0.999), eps=1e-8):
        self.params = [p for p in params]
        for p in self.params:
            if p.dtype != torch.float32 or not p.is_cuda or not p.is_contiguous():
                raise ValueError("DeviceAdam needs contiguous float32 CUDA tensors")
        self.lr, self.betas, self.eps = float(lr), betas, float(eps)
        self.m = [torch.zeros_like(p) for p in self.params]
        self.v = [torch.zeros_like(p) for p in self.params]
        self.t = 0

    def zero_grad(self):
        for p in self.params:
            p.grad = None

    @torch.no_grad()
    def step(self):
        self.t += 1
        lib = _lib.load()
        st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
        for p, m, v in zip(self.params, self.m, self.v):
            if p.grad is None:
                continue
            g = p.grad.contiguous()
            _lib.check(lib.drAdamStep(C.c_void_p(p.data_ptr()), C.c_void_p(g.data_ptr()), C.c_void_p(m.data_ptr()),
                                      C.c_void_p(v.data_ptr()), p.numel(), self.lr, float(self.betas[0]),
                                      float(self.betas[1]), self.eps, self.t, st), "drAdamStep")
