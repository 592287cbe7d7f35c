"""Python binding of the C ABI: argument marshalling only.

PyTorch provides device memory and the stream; every step of rendering and
differentiation runs in the HIP kernels of libdiffrt.so.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(0 if t is None else t.data_ptr())


def _dev(a, dtype, device):
    if isinstance(a, torch.Tensor):
        return a.detach().to(device=device, dtype=dtype).contiguous()
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=device).contiguous()


def camera_struct(cam) -> _lib.Camera:
    c = _lib.Camera()
    c.position[:] = [float(v) for v in cam.position]
    c.look_at[:] = [float(v) for v in cam.look_at]
    c.up[:] = [float(v) for v in cam.up]
    c.fov_y_deg = float(cam.fov_y_deg)
    c.near_clip = float(cam.near_clip)
    c.width, c.height = int(cam.width), int(cam.height)
    c.window[:] = list(cam.win())
    return c


def options_struct(spp, max_depth, seed=0, view_id=0, terms=0, unit_mask=None, edge_pdf=None, edge_mix=0.0,
                   edge_mix_terms=0, edge_stats=None, aov=0, edge_t=0, edge_candidates=0, edge_nee=0.0,
                   edge_nee_width=0.0) -> _lib.RenderOptions:
    return _lib.RenderOptions(int(spp), int(max_depth), int(seed), int(view_id), int(terms), _ptr(unit_mask),
                              _ptr(edge_pdf), float(edge_mix), int(edge_mix_terms), _ptr(edge_stats), int(aov),
                              int(edge_t), int(edge_candidates), float(edge_nee), float(edge_nee_width))


# geometry-buffer channels of drRenderOptions.aov
AOV = {"radiance": 0, "position_x": 1, "position_y": 2, "position_z": 3, "normal_x": 4, "normal_y": 5,
       "normal_z": 6, "albedo": 7, "all": 8}


class Scene:
    """A scene uploaded to the GPU (owns the library's scene handle)."""

    def __init__(self, scene, device="cuda"):
        lib = _lib.load()
        self.device = torch.device(device)
        self.vertices = _dev(scene.vertices, torch.float32, self.device)
        self.indices = _dev(scene.indices, torch.int32, self.device)
        self.albedo = _dev(scene.albedo, torch.float32, self.device)
        self.emission = _dev(scene.emission, torch.float32, self.device)
        self.normals = None if scene.normals is None else _dev(scene.normals, torch.float32, self.device)
        self.num_vertices = int(self.vertices.shape[0])
        self.num_triangles = int(self.indices.shape[0])
        desc = _lib.SceneDesc(self.num_vertices, self.num_triangles, _ptr(self.vertices), _ptr(self.indices),
                              _ptr(self.normals), _ptr(self.albedo), _ptr(self.emission),
                              int(bool(scene.emission_two_sided)), float(scene.background))
        h = C.c_void_p()
        _lib.check(lib.drSceneCreate(C.byref(h), C.byref(desc), _stream()), "drSceneCreate")
        self._h = h
        ne = C.c_int32()
        lib.drSceneGetInfo(self._h, None, None, C.byref(ne))
        self.num_edges = int(ne.value)

    def update_vertices(self, vertices):
        v = _dev(vertices, torch.float32, self.device)
        assert v.shape == (self.num_vertices, 3)
        self.vertices = v
        _lib.check(_lib.load().drSceneUpdateVertices(self._h, _ptr(v), _stream()), "drSceneUpdateVertices")

    def refit_vertices(self, vertices):
        """Vertex update over the existing BVH topology (drSceneRefit): kernel
        launches only, no host synchronisation and no host BVH build."""
        v = _dev(vertices, torch.float32, self.device).contiguous()
        assert v.shape == (self.num_vertices, 3)
        self.vertices = v
        _lib.check(_lib.load().drSceneRefit(self._h, _ptr(v), _stream()), "drSceneRefit")

    def update_albedo(self, albedo):
        a = _dev(albedo, torch.float32, self.device)
        assert a.shape == (self.num_triangles,)
        self.albedo = a
        _lib.check(_lib.load().drSceneUpdateAlbedo(self._h, _ptr(a), _stream()), "drSceneUpdateAlbedo")

    def render(self, cam, spp, max_depth, seed=0, view_id=0, unit_mask=None, out=None, aov=0):
        """Window image [H, W]: radiance, or with aov in 1..7 one geometry-buffer
        channel (AOV names them); aov = 8: all seven channels, [7, H, W]."""
        x0, y0, x1, y1 = cam.win()
        shape = (7, y1 - y0, x1 - x0) if aov == 8 else (y1 - y0, x1 - x0)
        img = out if out is not None else torch.empty(shape, dtype=torch.float32, device=self.device)
        assert img.numel() == 7 ** (aov == 8) * (y1 - y0) * (x1 - x0) and img.is_contiguous() and img.dtype == torch.float32
        c = camera_struct(cam)
        o = options_struct(spp, max_depth, seed, view_id, 0, unit_mask, aov=aov)
        _lib.check(_lib.load().drRender(self._h, C.byref(c), C.byref(o), _ptr(img), _stream()), "drRender")
        return img

    def render_backward(self, cam, spp, max_depth, d_image, seed=0, view_id=0, terms=0, unit_mask=None,
                        want=("vertices", "albedo", "camera"), outs=None, edge_pdf=None, edge_mix=0.0,
                        edge_mix_terms=0, edge_stats=None, aov=0, edge_t=0, edge_candidates=0, edge_nee=0.0,
                        edge_nee_width=0.0):
        """Gradients w.r.t. vertices [V,3], albedo [T] and camera [9]. With
        edge_pdf ([E] device distribution) and edge_mix > 0 the edge samples
        are drawn from the proposal mixture; edge_stats ([E] float32 device
        tensor) receives the harvest statistic. aov selects the image being
        differentiated, as in render. edge_t = 1 draws the point on each
        secondary edge by the clamped cosine instead of uniformly.
        edge_candidates = M > 1 selects each secondary edge by M samples down
        the hierarchy and reservoir selection. edge_nee = alpha in (0, 1)
        draws each secondary edge sample with probability alpha from the
        edge strips crossed by a segment to a light point (next event
        estimation for edges), edge_nee_width their width (0: the scene's
        default)."""
        d_image = _dev(d_image, torch.float32, self.device)
        x0, y0, x1, y1 = cam.win()
        assert d_image.numel() == (7 if aov == 8 else 1) * (y1 - y0) * (x1 - x0), "d_image size"
        if outs is None:
            dv = torch.empty((self.num_vertices, 3), dtype=torch.float32, device=self.device) if "vertices" in want else None
            da = torch.empty((self.num_triangles,), dtype=torch.float32, device=self.device) if "albedo" in want else None
            dc = torch.empty((9,), dtype=torch.float32, device=self.device) if "camera" in want else None
        else:
            dv, da, dc = outs
        c = camera_struct(cam)
        if edge_pdf is not None:
            assert edge_pdf.dtype == torch.float32 and edge_pdf.is_contiguous() and edge_pdf.numel() == self.num_edges
        if edge_stats is not None:
            assert edge_stats.dtype == torch.float32 and edge_stats.is_contiguous() and edge_stats.numel() == self.num_edges
        o = options_struct(spp, max_depth, seed, view_id, terms, unit_mask, edge_pdf, edge_mix, edge_mix_terms,
                           edge_stats, aov, edge_t, edge_candidates, edge_nee, edge_nee_width)
        _lib.check(_lib.load().drRenderBackward(self._h, C.byref(c), C.byref(o), _ptr(d_image), _ptr(dv), _ptr(da),
                                                _ptr(dc), _stream()), "drRenderBackward")
        return dv, da, dc

    def edge_features(self, cam, out=None):
        """[E, 32] float32 features of every edge seen from `cam`."""
        f = out if out is not None else torch.empty((self.num_edges, _lib.EDGE_FEATURES), dtype=torch.float32,
                                                     device=self.device)
        c = camera_struct(cam)
        _lib.check(_lib.load().drEdgeFeatures(self._h, C.byref(c), _ptr(f), _stream()), "drEdgeFeatures")
        return f

    def set_profiling(self, events=True, counters=False):
        _lib.check(_lib.load().drSetProfiling(self._h, int(events), int(counters)), "drSetProfiling")

    def profile(self, reset=True) -> dict:
        p = _lib.Profile()
        _lib.check(_lib.load().drGetProfile(self._h, C.byref(p), int(reset)), "drGetProfile")
        out = {name: getattr(p, name) for name, _ in _lib.Profile._fields_ if name != "counts"}
        out["counts"] = {k: {n: int(p.counts[i][j]) for j, n in enumerate(_lib.COUNT_NAMES)}
                         for i, k in enumerate(_lib.KERNELS)}
        return out

    def device_error(self) -> bool:
        return _lib.load().drGetLastDeviceError(self._h) != _lib.DR_SUCCESS

    def close(self):
        if getattr(self, "_h", None):
            _lib.load().drSceneDestroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
