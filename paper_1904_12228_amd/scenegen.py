"""Seeded synthetic scene generators shared by the HIP path and the FP64 oracle.

This module only builds input data (triangle meshes, materials, cameras). It
holds none of the renderer's arithmetic: no intersection, shading, edge
sampling or derivatives. Random numbers come from numpy's own Philox
bit generator (seeded), which is unrelated to the Philox4x32-10 streams the
renderer consumes.

The workloads follow the thesis's scene assumptions (Ch. 5, Method): triangle
meshes, no interpenetration, area lights only. Sizes and distributions are
the ones the benchmark configurations name:

* ``config1``: two emissive triangles, one partly occluding the other, over a
  constant background, 64x64, primary visibility only.
* ``config2``: 1,000-triangle random soup on a ground quad with one quad area
  light, 256x256, direct lighting.
* ``config3``: icosphere (level 6, 81,920 triangles) displaced by value noise,
  inside a 12-triangle box with two quad lights, 512x512, depth 3.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class Scene:
    vertices: np.ndarray            # [V,3] float32, world space
    indices: np.ndarray             # [T,3] int32
    albedo: np.ndarray              # [T] float32
    emission: np.ndarray            # [T] float32, 0 = not an emitter
    normals: np.ndarray | None = None   # [V,3] float32 shading normals, None = flat
    emission_two_sided: bool = False
    background: float = 0.0         # radiance of camera rays that escape

    @property
    def num_vertices(self) -> int:
        return int(self.vertices.shape[0])

    @property
    def num_triangles(self) -> int:
        return int(self.indices.shape[0])

    def copy(self) -> "Scene":
        return Scene(self.vertices.copy(), self.indices.copy(), self.albedo.copy(),
                     self.emission.copy(),
                     None if self.normals is None else self.normals.copy(),
                     self.emission_two_sided, self.background)


@dataclasses.dataclass
class Camera:
    position: tuple
    look_at: tuple
    up: tuple
    fov_y_deg: float
    width: int
    height: int
    near_clip: float = 1e-2
    window: tuple | None = None     # (x0, y0, x1, y1) pixel window, None = full

    def win(self):
        if self.window is None:
            return (0, 0, self.width, self.height)
        return tuple(int(v) for v in self.window)

    def with_window(self, x0, y0, x1, y1) -> "Camera":
        return dataclasses.replace(self, window=(x0, y0, x1, y1))

    def params9(self) -> np.ndarray:
        return np.array(list(self.position) + list(self.look_at) + list(self.up), np.float32)

    @staticmethod
    def from_params9(p, like: "Camera") -> "Camera":
        p = [float(v) for v in np.asarray(p, np.float32)]
        return dataclasses.replace(like, position=tuple(p[0:3]), look_at=tuple(p[3:6]),
                                   up=tuple(p[6:9]))


@dataclasses.dataclass
class Config:
    name: str
    scene: Scene
    camera: Camera
    spp: int
    max_depth: int


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(key=int(seed)))


# --------------------------------------------------------------------------
# small geometric helpers used only for rejection tests and mesh building
# --------------------------------------------------------------------------

def _seg_tri_hits(p0, p1, a, b, c):
    """Vectorised test: does segment p0->p1 cross triangle (a,b,c)?  a,b,c: [N,3]."""
    d = p1 - p0
    e1 = b - a
    e2 = c - a
    pv = np.cross(np.broadcast_to(d, e2.shape), e2)
    det = np.einsum("ij,ij->i", e1, pv)
    ok = np.abs(det) > 1e-14
    inv = np.where(ok, 1.0 / np.where(ok, det, 1.0), 0.0)
    tv = p0 - a
    u = np.einsum("ij,ij->i", tv, pv) * inv
    qv = np.cross(tv, e1)
    v = np.einsum("j,ij->i", d, qv) * inv
    t = np.einsum("ij,ij->i", e2, qv) * inv
    return ok & (u >= 0) & (v >= 0) & (u + v <= 1) & (t >= 0) & (t <= 1)


def _tris_intersect(tri, others):
    """tri: [3,3]; others: [N,3,3] -> bool [N] (edge-crossing test, both ways)."""
    if others.shape[0] == 0:
        return np.zeros(0, bool)
    hit = np.zeros(others.shape[0], bool)
    a, b, c = others[:, 0], others[:, 1], others[:, 2]
    for i in range(3):
        hit |= _seg_tri_hits(tri[i], tri[(i + 1) % 3], a, b, c)
    ta = np.broadcast_to(tri[0], a.shape)
    tb = np.broadcast_to(tri[1], a.shape)
    tc = np.broadcast_to(tri[2], a.shape)
    for p, q in ((a, b), (b, c), (c, a)):
        d = q - p
        e1 = tb - ta
        e2 = tc - ta
        pv = np.cross(d, e2)
        det = np.einsum("ij,ij->i", e1, pv)
        ok = np.abs(det) > 1e-14
        inv = np.where(ok, 1.0 / np.where(ok, det, 1.0), 0.0)
        tv = p - ta
        u = np.einsum("ij,ij->i", tv, pv) * inv
        qv = np.cross(tv, e1)
        v = np.einsum("ij,ij->i", d, qv) * inv
        t = np.einsum("ij,ij->i", e2, qv) * inv
        hit |= ok & (u >= 0) & (v >= 0) & (u + v <= 1) & (t >= 0) & (t <= 1)
    return hit


def _quad(p0, p1, p2, p3):
    """Two triangles (p0,p1,p2), (p0,p2,p3); normal = (p1-p0)x(p2-p0)."""
    v = np.array([p0, p1, p2, p3], np.float64)
    return v, np.array([[0, 1, 2], [0, 2, 3]], np.int64)


def _random_rotation(u):
    """Uniform random rotation from three uniforms (Shoemake's quaternion)."""
    u1, u2, u3 = u
    q = np.array([math.sqrt(1 - u1) * math.sin(2 * math.pi * u2),
                  math.sqrt(1 - u1) * math.cos(2 * math.pi * u2),
                  math.sqrt(u1) * math.sin(2 * math.pi * u3),
                  math.sqrt(u1) * math.cos(2 * math.pi * u3)])
    x, y, z, w = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def _assemble(parts, normals=None):
    verts, idx, alb, emi = [], [], [], []
    base = 0
    for v, f, a, e in parts:
        verts.append(np.asarray(v, np.float64))
        idx.append(np.asarray(f, np.int64) + base)
        alb.append(np.broadcast_to(np.asarray(a, np.float64), (len(f),)))
        emi.append(np.broadcast_to(np.asarray(e, np.float64), (len(f),)))
        base += len(v)
    scene = Scene(np.concatenate(verts).astype(np.float32),
                  np.concatenate(idx).astype(np.int32),
                  np.concatenate(alb).astype(np.float32),
                  np.concatenate(emi).astype(np.float32))
    if normals is not None:
        scene.normals = np.concatenate(normals).astype(np.float32)
    return scene


# --------------------------------------------------------------------------
# configuration 1: two triangles, primary visibility
# --------------------------------------------------------------------------

def _proj_cfg1(p, w, h, fov_deg):
    t = math.tan(math.radians(fov_deg) / 2)
    sx = w / 2 * (1 + (-p[..., 0]) / (p[..., 2] * t * (w / h)))
    sy = h / 2 * (1 - p[..., 1] / (p[..., 2] * t))
    return np.stack([sx, sy], -1)


def _inside(pts, tri2):
    a, b, c = tri2
    def s(p, q, r):
        return (q[0] - p[0]) * (r[..., 1] - p[1]) - (q[1] - p[1]) * (r[..., 0] - p[0])
    d1, d2, d3 = s(a, b, pts), s(b, c, pts), s(c, a, pts)
    neg = (d1 < 0) | (d2 < 0) | (d3 < 0)
    pos = (d1 > 0) | (d2 > 0) | (d3 > 0)
    return ~(neg & pos)


def two_triangles(seed=0, width=64, height=64, spp=4):
    """Two emissive triangles, vertices x,y ~ U[-1,1], z ~ U[2,4]; one partly
    occludes the other. Rejection keeps them non-intersecting, with a
    projected overlap of 5-95% of the smaller one, edges longer than 2 px and
    every pair of projected edges more than 1 degree apart."""
    rng = _rng(seed)
    fov = 60.0
    grid = (np.stack(np.meshgrid(np.arange(256) + 0.5, np.arange(256) + 0.5), -1)
            * (width / 256.0))
    for _ in range(100000):
        xy = rng.uniform(-1, 1, size=(2, 3, 2))
        z = rng.uniform(2, 4, size=(2, 3, 1))
        tris = np.concatenate([xy, z], -1)
        if _tris_intersect(tris[0], tris[1:2])[0]:
            continue
        s = [_proj_cfg1(t, width, height, fov) for t in tris]
        edges = [s[i][(j + 1) % 3] - s[i][j] for i in range(2) for j in range(3)]
        if min(np.linalg.norm(e) for e in edges) < 2.0:
            continue
        ang_ok = True
        for i in range(6):
            for j in range(i + 1, 6):
                c = abs(np.dot(edges[i], edges[j])) / (np.linalg.norm(edges[i]) * np.linalg.norm(edges[j]))
                if c > math.cos(math.radians(1.0)):
                    ang_ok = False
        if not ang_ok:
            continue
        in0 = _inside(grid, s[0])
        in1 = _inside(grid, s[1])
        small = min(in0.sum(), in1.sum())
        if small == 0:
            continue
        frac = (in0 & in1).sum() / small
        if not (0.05 <= frac <= 0.95):
            continue
        emi = rng.uniform(0.2, 1.0, size=2)
        scene = Scene(tris.reshape(6, 3).astype(np.float32),
                      np.array([[0, 1, 2], [3, 4, 5]], np.int32),
                      np.zeros(2, np.float32), emi.astype(np.float32),
                      None, True, 0.1)
        cam = Camera((0.0, 0.0, 0.0), (0.0, 0.0, 1.0), (0.0, 1.0, 0.0), fov, width, height)
        return Config("two_triangles", scene, cam, spp, 0)
    raise RuntimeError("rejection sampling failed")


def config1(seed=0):
    return two_triangles(seed, 64, 64, 4)


# --------------------------------------------------------------------------
# configuration 2: random soup, ground, one quad light, direct lighting
# --------------------------------------------------------------------------

def soup(seed=0, n_tris=1000, width=256, height=256, spp=16, light_emission=10.0, light_size=0.5):
    """Random non-intersecting triangle soup in the unit cube on a ground quad
    under one light_size x light_size quad light (Lambertian, albedo
    U[0.2,0.8])."""
    rng = _rng(seed)
    ground_y = -0.05
    gv, gf = _quad((-1.5, ground_y, -1.5), (-1.5, ground_y, 2.5),
                   (2.5, ground_y, 2.5), (2.5, ground_y, -1.5))
    # light at y=1.8 above the cube centre, facing -y
    h = 0.5 * light_size
    lv, lf = _quad((0.5 - h, 1.8, 0.5 - h), (0.5 + h, 1.8, 0.5 - h),
                   (0.5 + h, 1.8, 0.5 + h), (0.5 - h, 1.8, 0.5 + h))
    tris = []
    centers = []
    radii = []
    ground_tris = gv[gf]
    while len(tris) < n_tris:
        c = rng.uniform(0, 1, size=3)
        L = rng.uniform(0.02, 0.2, size=3)
        a, b, cc = np.sort(L)
        if a + b <= cc * 1.05:
            continue
        # triangle with side lengths (L0, L1, L2) in its plane
        l0, l1, l2 = L
        x = (l0 * l0 + l2 * l2 - l1 * l1) / (2 * l0)
        y2 = l2 * l2 - x * x
        if y2 <= 1e-8:
            continue
        p = np.array([[0, 0, 0], [l0, 0, 0], [x, math.sqrt(y2), 0]], np.float64)
        p -= p.mean(0)
        R = _random_rotation(rng.uniform(0, 1, size=3))
        p = p @ R.T + c
        if p[:, 1].min() <= ground_y + 1e-3:
            continue
        r = np.linalg.norm(p - c, axis=1).max()
        if tris:
            C = np.array(centers)
            Rr = np.array(radii)
            near = np.nonzero(np.linalg.norm(C - c, axis=1) <= Rr + r + 1e-3)[0]
            if near.size and _tris_intersect(p, np.array(tris)[near]).any():
                continue
        tris.append(p)
        centers.append(c)
        radii.append(r)
    tv = np.array(tris).reshape(-1, 3)
    tf = np.arange(3 * n_tris).reshape(n_tris, 3)
    alb = rng.uniform(0.2, 0.8, size=n_tris)
    scene = _assemble([(tv, tf, alb, 0.0), (gv, gf, 0.5, 0.0), (lv, lf, 0.0, light_emission)])
    scene.background = 0.0
    cam = Camera((0.5, 1.2, -1.8), (0.5, 0.4, 0.5), (0.0, 1.0, 0.0), 45.0, width, height)
    return Config("soup", scene, cam, spp, 1)


def config2(seed=0):
    return soup(seed, 1000, 256, 256, 16)


# --------------------------------------------------------------------------
# configuration 3: displaced icosphere in a box with two lights, depth 3
# --------------------------------------------------------------------------

def icosphere(level):
    t = (1 + 5 ** 0.5) / 2
    v = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t),
         (0, -1, -t), (0, 1, -t), (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    f = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4),
         (11, 10, 2), (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8),
         (3, 8, 9), (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    verts = [np.array(p, np.float64) / np.linalg.norm(p) for p in v]
    faces = np.array(f, np.int64)
    for _ in range(level):
        cache = {}
        new_faces = []
        def mid(a, b):
            key = (a, b) if a < b else (b, a)
            if key not in cache:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            new_faces += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = np.array(new_faces, np.int64)
    return np.array(verts), faces


def _value_noise(rng, freq=4):
    lattice = rng.uniform(-1, 1, size=(freq + 2, freq + 2, freq + 2))

    def f(p):
        q = (p + 1.0) * 0.5 * freq   # map [-1,1] -> [0,freq]
        i = np.clip(np.floor(q).astype(np.int64), 0, freq)
        r = q - i
        s = r * r * (3 - 2 * r)
        out = 0.0
        for dx in (0, 1):
            for dy in (0, 1):
                for dz in (0, 1):
                    w = ((s[:, 0] if dx else 1 - s[:, 0]) * (s[:, 1] if dy else 1 - s[:, 1])
                         * (s[:, 2] if dz else 1 - s[:, 2]))
                    out = out + w * lattice[i[:, 0] + dx, i[:, 1] + dy, i[:, 2] + dz]
        return out
    return f


def _vertex_normals(v, f):
    n = np.zeros_like(v)
    fn = np.cross(v[f[:, 1]] - v[f[:, 0]], v[f[:, 2]] - v[f[:, 0]])   # area weighted
    for k in range(3):
        np.add.at(n, f[:, k], fn)
    return n / np.linalg.norm(n, axis=1, keepdims=True)


def sphere_box(seed=0, level=6, width=512, height=512, spp=64, max_depth=3):
    """Icosphere of radius 0.5 displaced along its normals by seeded value noise
    (amplitude 0.1), smooth shading normals, inside a [-1,1]^3 box of 12
    inward-facing flat triangles, lit by two 0.3x0.3 quad lights under the
    ceiling. Sphere albedo 0.5 on every triangle (kept per triangle)."""
    rng = _rng(seed)
    sv, sf = icosphere(level)
    noise = _value_noise(rng)
    sv = sv * 0.5
    nrm = sv / np.linalg.norm(sv, axis=1, keepdims=True)
    sv = sv + nrm * (0.1 * noise(sv / 0.6))[:, None]
    sn = _vertex_normals(sv, sf)
    parts, normals = [], []
    parts.append((sv, sf, 0.5, 0.0))
    normals.append(sn)
    walls = [  # inward-facing quads: (corners), inward normal
        (((-1, -1, -1), (1, -1, -1), (1, -1, 1), (-1, -1, 1)), (0, 1, 0)),    # floor
        (((-1, 1, -1), (-1, 1, 1), (1, 1, 1), (1, 1, -1)), (0, -1, 0)),       # ceiling
        (((-1, -1, 1), (1, -1, 1), (1, 1, 1), (-1, 1, 1)), (0, 0, -1)),       # back (+z)
        (((-1, -1, -1), (-1, 1, -1), (1, 1, -1), (1, -1, -1)), (0, 0, 1)),    # front (-z)
        (((-1, -1, -1), (-1, -1, 1), (-1, 1, 1), (-1, 1, -1)), (1, 0, 0)),    # left (-x)
        (((1, -1, -1), (1, 1, -1), (1, 1, 1), (1, -1, 1)), (-1, 0, 0)),       # right (+x)
    ]
    wall_alb = rng.uniform(0.2, 0.8, size=6)
    for (corners, n), a in zip(walls, wall_alb):
        v, f = _quad(*corners)
        if np.dot(np.cross(v[1] - v[0], v[2] - v[0]), n) < 0:
            v, f = _quad(*corners[::-1])
        assert np.dot(np.cross(v[1] - v[0], v[2] - v[0]), n) > 0
        parts.append((v, f, a, 0.0))
        normals.append(np.tile(np.array(n, np.float64), (4, 1)))
    h = 0.15
    for cx in (-0.5, 0.5):
        y = 0.99
        v, f = _quad((cx - h, y, -h), (cx + h, y, -h), (cx + h, y, h), (cx - h, y, h))
        fn = np.cross(v[1] - v[0], v[2] - v[0])
        assert fn[1] < 0
        parts.append((v, f, 0.0, 15.0))
        normals.append(np.tile(np.array((0.0, -1.0, 0.0)), (4, 1)))
    scene = _assemble(parts, normals)
    scene.background = 0.0
    cam = Camera((0.0, 0.1, -0.9), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 70.0, width, height)
    return Config("sphere_box", scene, cam, spp, max_depth)


def config3(seed=0):
    return sphere_box(seed, 6, 512, 512, 64, 3)


CONFIGS = {"config1": config1, "config2": config2, "config3": config3}


# ---------------------------------------------------------------------------
# learned edge proposal: seeded network parameters and synthetic inputs
# ---------------------------------------------------------------------------
MLP_PARAMS = 32 * 64 + 64 + 64 * 64 + 64 + 64 + 1    # W1 | b1 | W2 | b2 | W3 | b3


def mlp_params(seed: int, bias_scale: float = 0.0) -> np.ndarray:
    """He-style random initial parameters (float32, W1 [32][64] | b1 [64] |
    W2 [64][64] | b2 [64] | W3 [64] | b3 [1]); biases N(0, bias_scale)."""
    rng = np.random.Generator(np.random.Philox(seed))
    th = np.zeros(MLP_PARAMS, np.float32)
    o = 0
    for rows, cols, fan in ((32, 64, 29), (64, 64, 64), (64, 1, 64)):
        th[o:o + rows * cols] = rng.normal(0.0, np.sqrt(2.0 / fan), rows * cols)
        o += rows * cols
        th[o:o + cols] = rng.normal(0.0, bias_scale, cols) if bias_scale > 0 else 0.0
        o += cols
    assert o == MLP_PARAMS
    return th


def mlp_inputs(seed: int, n: int) -> np.ndarray:
    """Synthetic [n][32] float32 inputs with the value ranges of edge features
    (29 used columns, zero padding)."""
    rng = np.random.Generator(np.random.Philox(seed))
    x = np.zeros((n, 32), np.float32)
    x[:, :29] = rng.normal(0.0, 1.0, (n, 29))
    return x


# ---------------------------------------------------------------------------
# many views of one scene (training views of the edge proposal, batched
# inverse rendering)
# ---------------------------------------------------------------------------
def orbit_views(seed: int, n: int, center=(0.5, 0.4, 0.5), radius=(2.0, 2.8), elevation_deg=(10.0, 45.0),
                fov_deg=(40.0, 50.0), sizes=((128, 128),), spp=(8,)) -> list:
    """n seeded cameras on a spherical shell around `center` (azimuth uniform,
    elevation and distance uniform in the given ranges), each looking at the
    centre jittered by up to 0.1, with a size and a sample count drawn from the
    given lists. Returns [(Camera, spp)]."""
    rng = np.random.Generator(np.random.Philox(seed))
    c = np.asarray(center, np.float64)
    out = []
    for _ in range(n):
        az = rng.uniform(0.0, 2.0 * np.pi)
        el = np.radians(rng.uniform(*elevation_deg))
        r = rng.uniform(*radius)
        pos = c + r * np.array([np.cos(el) * np.sin(az), np.sin(el), -np.cos(el) * np.cos(az)])
        look = c + rng.uniform(-0.1, 0.1, 3)
        w, h = sizes[int(rng.integers(len(sizes)))]
        s = int(spp[int(rng.integers(len(spp)))])
        cam = Camera(tuple(float(v) for v in pos), tuple(float(v) for v in look), (0.0, 1.0, 0.0),
                     float(rng.uniform(*fov_deg)), int(w), int(h))
        out.append((cam, s))
    return out
