"""ctypes binding of the FP64 CPU oracle (oracle/oracle.cpp).

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the
benchmark's CPU-baseline leg. The product package never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC = os.path.join(_HERE, "oracle.cpp")


def build(verbose: bool = False) -> str:
    """Compile liboracle.so with g++ (plain C++17, no FP contraction)."""
    cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off", "-fopenmp",
           "-o", LIB_PATH, SRC]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    return LIB_PATH


class _Scene(C.Structure):
    _fields_ = [("num_vertices", C.c_int32), ("num_triangles", C.c_int32),
                ("vertices", C.c_void_p), ("indices", C.c_void_p), ("albedo", C.c_void_p),
                ("emission", C.c_void_p), ("normals", C.c_void_p),
                ("emission_two_sided", C.c_int32), ("background", C.c_float),
                ("vertices64", C.c_void_p), ("albedo64", C.c_void_p)]


class _Camera(C.Structure):
    _fields_ = [("position", C.c_float * 3), ("look_at", C.c_float * 3), ("up", C.c_float * 3),
                ("fov_y_deg", C.c_float), ("near_clip", C.c_float),
                ("width", C.c_int32), ("height", C.c_int32),
                ("win_x0", C.c_int32), ("win_y0", C.c_int32), ("win_x1", C.c_int32), ("win_y1", C.c_int32),
                ("params64", C.c_void_p)]


class _Options(C.Structure):
    _fields_ = [("spp", C.c_int32), ("max_depth", C.c_int32), ("seed", C.c_uint64),
                ("view_id", C.c_uint32), ("interior", C.c_int32), ("primary_edges", C.c_int32),
                ("secondary_edges", C.c_int32), ("use_bvh", C.c_int32), ("exclude_flagged", C.c_int32),
                ("num_threads", C.c_int32), ("unit_mask", C.c_void_p),
                ("dir_mode", C.c_int32), ("dir_log", C.c_void_p),
                ("edge_pdf", C.c_void_p), ("mix", C.c_double), ("mix_terms", C.c_int32), ("aov", C.c_int32),
                ("edge_t_mode", C.c_int32), ("edge_candidates", C.c_int32),
                ("enee", C.c_double), ("enee_width", C.c_double)]


class _Outputs(C.Structure):
    _fields_ = [("image", C.c_void_p), ("d_image", C.c_void_p), ("d_vertices", C.c_void_p),
                ("d_albedo", C.c_void_p), ("d_camera", C.c_void_p), ("mass_vertices", C.c_void_p),
                ("mass_albedo", C.c_void_p), ("mass_camera", C.c_void_p), ("unit_flags", C.c_void_p),
                ("stats", C.c_void_p), ("edge_stats", C.c_void_p), ("edge_stats_mass", C.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC):
            build()
        _lib = C.CDLL(LIB_PATH)
        _lib.orc_render.restype = C.c_int
        _lib.orc_edges.restype = C.c_int
        _lib.orc_closest_hit.restype = C.c_int
        _lib.orc_edge_tree_pdf.restype = C.c_int
        _lib.orc_edge_tree_sample.restype = C.c_int
        _lib.orc_edge_tree_select.restype = C.c_int
        _lib.orc_edge_t_cosine.restype = C.c_int
        _lib.orc_edge_t_cosine_pdf.restype = C.c_double
        _lib.orc_edge_nee_width.restype = C.c_double
        _lib.orc_edge_nee_sample.restype = C.c_int
        _lib.orc_edge_nee_pdf.restype = C.c_int
        _lib.orc_edge_nee_mix_sample.restype = C.c_int
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def _vp(a):
    """Pointer argument for a foreign call (ctypes would truncate a bare int)."""
    return C.c_void_p(None if a is None else a.ctypes.data)


def _scene_struct(scene, keep, vertices64=None, albedo64=None):
    v = np.ascontiguousarray(scene.vertices, np.float32)
    v64 = None if vertices64 is None else np.ascontiguousarray(vertices64, np.float64)
    a64 = None if albedo64 is None else np.ascontiguousarray(albedo64, np.float64)
    keep += [v64, a64]
    i = np.ascontiguousarray(scene.indices, np.int32)
    a = np.ascontiguousarray(scene.albedo, np.float32)
    e = np.ascontiguousarray(scene.emission, np.float32)
    n = None if scene.normals is None else np.ascontiguousarray(scene.normals, np.float32)
    keep += [v, i, a, e, n]
    return _Scene(v.shape[0], i.shape[0], _ptr(v), _ptr(i), _ptr(a), _ptr(e), _ptr(n),
                  int(bool(scene.emission_two_sided)), float(scene.background), _ptr(v64), _ptr(a64))


def _camera_struct(cam, keep=None, params64=None):
    x0, y0, x1, y1 = cam.win()
    c = _Camera()
    if params64 is not None:
        p64 = np.ascontiguousarray(params64, np.float64)
        keep.append(p64)
        c.params64 = p64.ctypes.data
    c.position[:] = [float(t) for t in cam.position]
    c.look_at[:] = [float(t) for t in cam.look_at]
    c.up[:] = [float(t) for t in cam.up]
    c.fov_y_deg = cam.fov_y_deg
    c.near_clip = cam.near_clip
    c.width, c.height = cam.width, cam.height
    c.win_x0, c.win_y0, c.win_x1, c.win_y1 = x0, y0, x1, y1
    return c


def render(scene, cam, spp, max_depth, seed=0, d_image=None, *, interior=True, primary=True,
           secondary=True, use_bvh=True, exclude_flagged=False, threads=1, unit_mask=None,
           view_id=0, want_flags=False, vertices64=None, albedo64=None, camera64=None,
           dir_mode=0, dir_log=None, edge_pdf=None, mix=0.0, mix_terms=3, edge_stats=False, aov=0, edge_t=0,
           edge_candidates=0, enee=0.0, enee_width=0.0):
    """Returns a dict with image, (if d_image) d_vertices, d_albedo, d_camera,
    the matching mass arrays, unit flags and stats; with edge_stats=True also
    the per-edge harvest statistic. edge_pdf (a distribution over all edges)
    and mix in [0, 1) select the proposal mixture (mix_terms: bit 0 primary,
    bit 1 secondary). aov selects a geometry buffer instead of radiance
    (1-3 position, 4-6 shading normal, 7 albedo). edge_t = 1 draws the point
    on each secondary edge by the clamped cosine instead of uniformly.
    edge_candidates = M > 1 selects each secondary edge by M samples
    distributed down the hierarchy and weighted reservoir selection.
    enee = alpha in (0, 1) mixes the billboard strategy (next event
    estimation for edges) into the secondary edge sample with probability
    alpha; enee_width is the billboard width (0: the scene's default)."""
    keep = []
    s = _scene_struct(scene, keep, vertices64, albedo64)
    c = _camera_struct(cam, keep, camera64)
    x0, y0, x1, y1 = cam.win()
    Ww, Hw = x1 - x0, y1 - y0
    M = Ww * Hw * spp
    mask = None if unit_mask is None else np.ascontiguousarray(unit_mask, np.uint8)
    if dir_mode:
        assert dir_log is not None and dir_log.dtype == np.float64 and dir_log.size == M * 64
    q = None if edge_pdf is None else np.ascontiguousarray(edge_pdf, np.float64)
    o = _Options(spp, max_depth, seed, view_id, int(interior), int(primary), int(secondary),
                 int(use_bvh), int(exclude_flagged), threads, _ptr(mask), int(dir_mode), _ptr(dir_log),
                 _ptr(q), float(mix), int(mix_terms), int(aov), int(edge_t), int(edge_candidates),
                 float(enee), float(enee_width))
    res = {"image": np.zeros((Hw, Ww), np.float64), "stats": np.zeros(8, np.int64)}
    if d_image is not None:
        dimg = np.ascontiguousarray(np.broadcast_to(np.asarray(d_image, np.float64), (Hw, Ww)))
        keep.append(dimg)
        V, T = scene.num_vertices, scene.num_triangles
        for k, shape in (("d_vertices", (V, 3)), ("d_albedo", (T,)), ("d_camera", (9,)),
                         ("mass_vertices", (V, 3)), ("mass_albedo", (T,)), ("mass_camera", (9,))):
            res[k] = np.zeros(shape, np.float64)
    else:
        dimg = None
    if want_flags:
        res["unit_flags"] = np.zeros(M, np.uint8)
    if edge_stats and d_image is not None:
        res["edge_stats"] = np.zeros(num_edges(scene), np.float64)
        res["edge_stats_mass"] = np.zeros(num_edges(scene), np.float64)
    out = _Outputs(_ptr(res["image"]), _ptr(dimg), _ptr(res.get("d_vertices")), _ptr(res.get("d_albedo")),
                   _ptr(res.get("d_camera")), _ptr(res.get("mass_vertices")), _ptr(res.get("mass_albedo")),
                   _ptr(res.get("mass_camera")), _ptr(res.get("unit_flags")), _ptr(res["stats"]),
                   _ptr(res.get("edge_stats")), _ptr(res.get("edge_stats_mass")))
    rc = lib().orc_render(C.byref(s), C.byref(c), C.byref(o), C.byref(out))
    if rc != 0:
        raise RuntimeError(f"orc_render failed with code {rc}")
    return res


TIE_REASONS = ["near_miss_in_front", "equal_t_hits", "hit_near_edge", "hit_near_tmin", "grazing_hit",
               "shadow_near_edge", "shadow_near_ends", "cdf_tie", "inside_box_tie", "horizon_tie",
               "vsphere_tie", "branch_tie", "ill_conditioned_edge", "pixel_boundary", "silhouette_sign",
               "mixture_component", "grazing_departure", "split_tie", "reservoir_tie", "billboard_crossing",
               "billboard_race", "billboard_light_hit", "billboard_strategy"]


def tie_reasons(reset=True):
    out = np.zeros(24, np.int64)
    lib().orc_tie_reasons(_vp(out), int(reset))
    return {k: int(v) for k, v in zip(TIE_REASONS, out) if v}


def philox4x32_10(ctr, key):
    c = (C.c_uint32 * 4)(*ctr)
    k = (C.c_uint32 * 2)(*key)
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [int(x) for x in o]


def num_edges(scene):
    keep = []
    s = _scene_struct(scene, keep)
    n = C.c_int32()
    rc = lib().orc_edges(C.byref(s), C.byref(n), None)
    if rc:
        raise RuntimeError(f"orc_edges failed {rc}")
    return int(n.value)


def edges(scene):
    keep = []
    s = _scene_struct(scene, keep)
    n = C.c_int32()
    rc = lib().orc_edges(C.byref(s), C.byref(n), None)
    if rc:
        raise RuntimeError(f"orc_edges failed {rc}")
    rows = np.zeros((n.value, 4), np.int32)
    lib().orc_edges(C.byref(s), C.byref(n), _vp(rows))
    return rows


def closest_hit(scene, o, d, tmin, tmax, use_bvh=True):
    keep = []
    s = _scene_struct(scene, keep)
    o = np.ascontiguousarray(o, np.float64)
    d = np.ascontiguousarray(d, np.float64)
    n = o.shape[0]
    tri = np.zeros(n, np.int32)
    t = np.zeros(n, np.float64)
    rc = lib().orc_closest_hit(C.byref(s), n, _vp(o), _vp(d), C.c_double(tmin), C.c_double(tmax),
                               int(use_bvh), _vp(tri), _vp(t))
    if rc:
        raise RuntimeError(f"orc_closest_hit failed {rc}")
    return tri, t


def edge_tree_pdf(scene, cam, p, n):
    keep = []
    s = _scene_struct(scene, keep)
    c = _camera_struct(cam)
    E = edges(scene).shape[0]
    pdf = np.zeros(E, np.float64)
    fail = C.c_double()
    p = np.ascontiguousarray(p, np.float64)
    n = np.ascontiguousarray(n, np.float64)
    rc = lib().orc_edge_tree_pdf(C.byref(s), C.byref(c), _vp(p), _vp(n), _vp(pdf), C.byref(fail))
    if rc:
        raise RuntimeError(f"orc_edge_tree_pdf failed {rc}")
    return pdf, fail.value


def edge_tree_pdf_of(scene, cam, p, n, edge_ids):
    """Descent probability of each given edge, by its root-to-leaf path."""
    keep = []
    s = _scene_struct(scene, keep)
    c = _camera_struct(cam)
    ids = np.ascontiguousarray(edge_ids, np.int32)
    pdf = np.zeros(ids.size, np.float64)
    p = np.ascontiguousarray(p, np.float64)
    n = np.ascontiguousarray(n, np.float64)
    rc = lib().orc_edge_tree_pdf_of(C.byref(s), C.byref(c), _vp(p), _vp(n), ids.size, _vp(ids), _vp(pdf))
    if rc:
        raise RuntimeError(f"orc_edge_tree_pdf_of failed {rc}")
    return pdf


def edge_tree_sample(scene, cam, p, n, u):
    keep = []
    s = _scene_struct(scene, keep)
    c = _camera_struct(cam)
    u = np.ascontiguousarray(u, np.float64)
    assert u.shape[1] == 65
    cnt = u.shape[0]
    edge = np.zeros(cnt, np.int32)
    pdf = np.zeros(cnt, np.float64)
    p = np.ascontiguousarray(p, np.float64)
    n = np.ascontiguousarray(n, np.float64)
    rc = lib().orc_edge_tree_sample(C.byref(s), C.byref(c), _vp(p), _vp(n), cnt, _vp(u), _vp(edge), _vp(pdf))
    if rc:
        raise RuntimeError(f"orc_edge_tree_sample failed {rc}")
    return edge, pdf


def edge_tree_select(scene, cam, p, n, M, u):
    """Stratified M-sample descent with reservoir selection from shading point
    p with normal n: one draw per row of u (the row's uniforms used in order).
    Returns (edge [count], weight [count]) with weight = W / (M imp) of the
    kept edge."""
    keep = []
    s = _scene_struct(scene, keep)
    c = _camera_struct(cam)
    u = np.ascontiguousarray(u, np.float64)
    cnt, stride = u.shape
    edge = np.zeros(cnt, np.int32)
    w = np.zeros(cnt, np.float64)
    p = np.ascontiguousarray(p, np.float64)
    n = np.ascontiguousarray(n, np.float64)
    rc = lib().orc_edge_tree_select(C.byref(s), C.byref(c), _vp(p), _vp(n), int(M), cnt, _vp(u), stride, _vp(edge),
                                    _vp(w))
    if rc:
        raise RuntimeError(f"orc_edge_tree_select failed {rc}")
    return edge, w


def secondary_forms(p, v0, v1, t, m0, nm):
    arr = [np.ascontiguousarray(x, np.float64) for x in (p, v0, v1, m0, nm)]
    af = np.zeros(9)
    df = np.zeros(9)
    lib().orc_secondary_forms(_vp(arr[0]), _vp(arr[1]), _vp(arr[2]), C.c_double(t), _vp(arr[3]),
                              _vp(arr[4]), _vp(af), _vp(df))
    return af.reshape(3, 3), df.reshape(3, 3)


def edge_t_cosine(p, n, v0, v1, u):
    """Clamped-cosine edge-point sampler: (t, pdf_t) per uniform in u (t = -1
    where there is no sample)."""
    u = np.ascontiguousarray(u, np.float64)
    t = np.zeros(u.size)
    pt = np.zeros(u.size)
    args = [np.ascontiguousarray(x, np.float64) for x in (p, n, v0, v1)]
    lib().orc_edge_t_cosine(*[_vp(a) for a in args], int(u.size), _vp(u), _vp(t), _vp(pt))
    return t, pt


def edge_t_cosine_pdf(p, n, v0, v1, t):
    args = [np.ascontiguousarray(x, np.float64) for x in (p, n, v0, v1)]
    return float(lib().orc_edge_t_cosine_pdf(*[_vp(a) for a in args], C.c_double(t)))


def edge_nee_width(scene):
    """Default billboard width of next event estimation for edges: the L2 norm
    over the coordinates of 2% of the vertex positions' mean absolute deviation."""
    keep = []
    s = _scene_struct(scene, keep)
    w = lib().orc_edge_nee_width(C.byref(s))
    if not w >= 0:
        raise RuntimeError("orc_edge_nee_width failed")
    return float(w)


def _nee_point(p, n):
    return (np.ascontiguousarray(p, np.float64), np.ascontiguousarray(n, np.float64))


def edge_nee_sample(scene, p, n, tri, width, count, seed=0):
    """count draws of the billboard strategy at (p, n) on triangle tri (-1:
    none): (edge or -1, t, s, near-tie flags)."""
    keep = []
    s = _scene_struct(scene, keep)
    p, n = _nee_point(p, n)
    e = np.zeros(count, np.int32)
    t = np.zeros(count)
    sv = np.zeros(count)
    fl = np.zeros(count, np.uint8)
    rc = lib().orc_edge_nee_sample(C.byref(s), _vp(p), _vp(n), int(tri), C.c_double(width), int(count),
                                   C.c_uint64(seed), _vp(e), _vp(t), _vp(sv), _vp(fl))
    if rc:
        raise RuntimeError(f"orc_edge_nee_sample failed with code {rc}")
    return e, t, sv, fl.astype(bool)


def edge_nee_pdf(scene, p, n, tri, width, edges, t, sv):
    """Density of the billboard strategy in dt ds at the given (edge, t, s)."""
    keep = []
    s = _scene_struct(scene, keep)
    p, n = _nee_point(p, n)
    e = np.ascontiguousarray(edges, np.int32)
    t = np.ascontiguousarray(t, np.float64)
    sv = np.ascontiguousarray(sv, np.float64)
    out = np.zeros(len(e))
    rc = lib().orc_edge_nee_pdf(C.byref(s), _vp(p), _vp(n), int(tri), C.c_double(width), len(e), _vp(e), _vp(t),
                                _vp(sv), _vp(out))
    if rc:
        raise RuntimeError(f"orc_edge_nee_pdf failed with code {rc}")
    return out


def edge_nee_mix_sample(scene, cam, p, n, tri, width, alpha, count, seed=0):
    """count draws of the mixture of the billboard strategy (probability
    alpha) and the edge hierarchy of camera cam: (edge or -1, t, mixture
    density in (e, t))."""
    keep = []
    s = _scene_struct(scene, keep)
    c = _camera_struct(cam, keep)
    p, n = _nee_point(p, n)
    e = np.zeros(count, np.int32)
    t = np.zeros(count)
    pdf = np.zeros(count)
    rc = lib().orc_edge_nee_mix_sample(C.byref(s), C.byref(c), _vp(p), _vp(n), int(tri), C.c_double(width),
                                       C.c_double(alpha), int(count), C.c_uint64(seed), _vp(e), _vp(t), _vp(pdf))
    if rc:
        raise RuntimeError(f"orc_edge_nee_mix_sample failed with code {rc}")
    return e, t, pdf
