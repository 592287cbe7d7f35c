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
    def forward(ctx, vertices, camera9, scene: api.Scene, cam: Camera, spp: int, depth: int, seed: int, view_id: int):
        scene.update_vertices(vertices)
        c = Camera.from_params9(camera9.detach().cpu().numpy(), cam)
        img = scene.render(c, spp, depth, seed=seed, view_id=view_id)
        ctx.args = (scene, c, spp, depth, seed, view_id)
        ctx.cam_device = camera9.device
        return img

    @staticmethod
    def backward(ctx, d_img):
        scene, c, spp, depth, seed, view_id = ctx.args
        dv, _, dc = scene.render_backward(c, spp, depth, d_img.contiguous(), seed=seed, view_id=view_id,
                                          want=("vertices", "camera"))
        return dv, dc.to(ctx.cam_device), None, None, None, None, None, None


def render(scene: api.Scene, vertices: torch.Tensor, camera9: torch.Tensor, cam: Camera, spp: int, depth: int,
           seed: int = 0, view_id: int = 0) -> torch.Tensor:
    """Differentiable render: image of `scene` with the given vertex positions
    ([V,3] on the scene's device) and camera (9 numbers: position, look_at,
    up; fov and image size from `cam`)."""
    return _RenderFn.apply(vertices, camera9, scene, cam, spp, depth, seed, view_id)


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
