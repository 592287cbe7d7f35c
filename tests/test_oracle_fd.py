"""End-to-end pins of the FP64 oracle's gradient against finite differences
(Ch. 5, Results, "Verification of the method": the gradient of the image is
compared with central finite differences of high-sample renders).

* Near-clipped edges (exact): two emissive triangles at depth 0, one of them
  reaching behind the camera so that two of its edges cross the near plane.
  The exact box-filtered image (3D near-plane clipping, projection, polygon
  clipping) is a closed form; its central differences w.r.t. all 18 vertex
  coordinates and the 9 camera numbers must match the oracle's mean gradient.
  This pins the near-clipped edge construction of the primary boundary term
  and the primary term's camera gradient.
* Depth 1 (renders): a floor lit by a quad light through a two-triangle
  occluder; the occluder's silhouette, its shadow and the light's outline are
  all on screen. Directions: the 9 camera numbers, single vertex coordinates
  of the occluder and the light, random directions over all vertex
  coordinates, and albedo entries.
* Depth 3 (renders): a floor, a roof-shaped occluder (two faces meeting in a
  visible crease), a tilted floating quad and a quad light, three path
  vertices with continuation paths, so the secondary term's side paths carry
  continuation radiance.

For the renders the loss is L = sum_p w_p I_p with fixed weights w. Central
differences use common random numbers (the same seeds on both sides) and
FP64 vertex / camera / albedo inputs; the gradient is the mean over seeds of
the oracle's backward pass. Each direction must agree within 4.5 standard
errors of the two Monte Carlo estimates, and the sum of squared z-scores must
pass a chi-square test. The thesis's own acceptance figure, the L1 error
relative to the L1 norm of the gradient, is printed with the Monte Carlo
noise floor; DIFFRT_FD_SCALE=k runs k times the samples.
"""
import math
import os

import numpy as np
import pytest

import oracle
from paper_1904_12228_amd import scenegen as sg

from . import analytic

SCALE = int(os.environ.get("DIFFRT_FD_SCALE", "1"))
THREADS = min(16, os.cpu_count() or 1)
# chi-square 0.999 quantiles by degrees of freedom
CHI2_999 = {12: 32.9, 14: 36.1, 16: 39.3, 18: 42.3, 20: 45.3}


# ---------------------------------------------------------------------------
# scenes
# ---------------------------------------------------------------------------

def near_clip_scene():
    v = np.array([[-0.9, -0.6, -0.4], [0.35, -0.35, 3.0], [-0.5, 0.55, 2.4],     # first vertex behind the camera
                  [0.45, 0.35, 2.2], [-0.25, 0.15, 3.6], [0.3, -0.45, 3.2]], np.float32)
    scene = sg.Scene(v, np.array([[0, 1, 2], [3, 4, 5]], np.int32), np.zeros(2, np.float32),
                     np.array([0.8, 0.4], np.float32), None, True, 0.1)
    cam = sg.Camera((0.0, 0.0, 0.0), (0.0, 0.0, 1.0), (0.0, 1.0, 0.0), 60.0, 32, 32, near_clip=0.05)
    return scene, cam


def shadow_scene():
    floor = ([-3, 0, -3], [-3, 0, 3], [3, 0, 3], [3, 0, -3])
    light = ([-0.25, 1.2, -0.25], [0.25, 1.2, -0.25], [0.25, 1.2, 0.25], [-0.25, 1.2, 0.25])
    occ = ([-0.3, 0.5, -0.2], [0.25, 0.45, -0.3], [0.05, 0.55, 0.3], [0.45, 0.6, 0.25])
    v = np.array(list(floor) + list(light) + list(occ), np.float32)
    f = np.array([[0, 1, 2], [0, 2, 3], [4, 5, 6], [4, 6, 7], [8, 9, 10], [9, 11, 10]], np.int32)
    scene = sg.Scene(v, f, np.array([0.6, 0.6, 0, 0, 0.5, 0.7], np.float32),
                     np.array([0, 0, 6.0, 6.0, 0, 0], np.float32), None, False, 0.0)
    cam = sg.Camera((0.2, 2.2, -2.0), (0.0, 0.3, 0.1), (0.0, 1.0, 0.0), 55.0, 32, 32)
    return scene, cam


def crease_scene():
    floor = ([-3, 0, -3], [-3, 0, 3], [3, 0, 3], [3, 0, -3])
    light = ([-0.3, 1.6, -0.1], [0.3, 1.6, -0.1], [0.3, 1.6, 0.5], [-0.3, 1.6, 0.5])
    roof = ([-0.5, 0.55, -0.3], [0.1, 0.75, -0.35], [0.05, 0.7, 0.35], [-0.45, 0.5, 0.3], [0.55, 0.5, -0.25],
            [0.5, 0.48, 0.3])
    tilt = ([0.3, 0.25, 0.45], [0.9, 0.35, 0.55], [0.8, 0.6, 1.0], [0.25, 0.45, 0.95])
    v = np.array(list(floor) + list(light) + list(roof) + list(tilt), np.float32)
    f = np.array([[0, 1, 2], [0, 2, 3], [4, 5, 6], [4, 6, 7], [8, 9, 10], [8, 10, 11], [9, 12, 13], [9, 13, 10],
                  [14, 15, 16], [14, 16, 17]], np.int32)
    alb = np.array([0.6, 0.6, 0, 0, 0.5, 0.5, 0.7, 0.7, 0.4, 0.4], np.float32)
    emi = np.array([0, 0, 6.0, 6.0, 0, 0, 0, 0, 0, 0], np.float32)
    scene = sg.Scene(v, f, alb, emi, None, False, 0.0)
    cam = sg.Camera((0.4, 2.0, -2.2), (0.2, 0.4, 0.3), (0.0, 1.0, 0.0), 50.0, 32, 32)
    return scene, cam


def test_scenes_are_what_the_docstring_says():
    """Light faces down, the roof's crease is convex and not coplanar, the
    near-clipped triangle's cut along the near plane projects outside the
    image (it is not a mesh edge, so it must not be on screen)."""
    for sc in (shadow_scene, crease_scene):
        scene, _ = sc()
        v = scene.vertices.astype(np.float64)
        assert np.cross(v[5] - v[4], v[6] - v[4])[1] < 0
    scene, _ = crease_scene()
    v = scene.vertices.astype(np.float64)
    n0 = np.cross(v[9] - v[8], v[10] - v[8])
    n1 = np.cross(v[12] - v[9], v[13] - v[9])
    assert np.linalg.norm(np.cross(n0, n1)) > 0.05 * np.linalg.norm(n0) * np.linalg.norm(n1)
    scene, cam = near_clip_scene()
    cam9 = cam.params9().astype(np.float64)
    poly = analytic.near_clip(scene.vertices[:3].astype(np.float64), cam9, cam.near_clip)
    cut = [p for p in poly if abs((p - cam9[:3]) @ np.array([0, 0, 1.0]) - cam.near_clip) < 1e-12]
    assert len(cut) == 2
    for t in np.linspace(0, 1, 101):
        q = analytic.project(cut[0] + t * (cut[1] - cut[0]), cam9, cam.fov_y_deg, cam.width, cam.height)
        assert q[0] > cam.width + 100 or q[0] < -100 or q[1] > cam.height + 100 or q[1] < -100


# ---------------------------------------------------------------------------
# near-clipped edges against the exact image
# ---------------------------------------------------------------------------

@pytest.mark.slow
def test_near_clipped_edges_match_exact_coverage():
    scene, cam = near_clip_scene()
    W, H, fov, near = cam.width, cam.height, cam.fov_y_deg, cam.near_clip
    rng = np.random.default_rng(21)
    dimg = rng.normal(size=(H, W)) + 1.0
    cam9 = cam.params9().astype(np.float64)
    v0 = scene.vertices.astype(np.float64)
    emi = scene.emission.astype(np.float64)
    bg = float(np.float32(scene.background))

    def J(v, c):
        return float((dimg * analytic.near_clipped_two_triangle_image(v, emi, bg, c, fov, W, H, near)).sum())

    exact_img = analytic.near_clipped_two_triangle_image(v0, emi, bg, cam9, fov, W, H, near)
    exact = np.zeros(27)
    h = 1e-6
    for k in range(27):
        vp, vm, cp, cm = v0.copy(), v0.copy(), cam9.copy(), cam9.copy()
        if k < 18:
            vp.ravel()[k] += h
            vm.ravel()[k] -= h
        else:
            cp[k - 18] += h
            cm[k - 18] -= h
        exact[k] = (J(vp, cp) - J(vm, cm)) / (2 * h)
    K = 48 * SCALE
    gs, ims = [], []
    for seed in range(K):
        r = oracle.render(scene, cam, 8, 0, seed, d_image=dimg, threads=THREADS)
        gs.append(np.concatenate([r["d_vertices"].ravel(), r["d_camera"]]))
        ims.append(r["image"])
    gs, ims = np.array(gs), np.array(ims)
    g, se = gs.mean(0), gs.std(0, ddof=1) / math.sqrt(K)
    print("exact", np.round(exact, 3))
    print("oracle", np.round(g, 3))
    print("se", np.round(se, 3))
    assert (np.abs(g - exact) <= 5 * se + 1e-9).all(), np.nonzero(np.abs(g - exact) > 5 * se + 1e-9)
    # the edges that cross the near plane carry a large part of the gradient
    assert np.abs(exact[:3]).max() > 0.1 * np.abs(exact).max()
    assert np.abs(g - exact).max() < 0.05 * np.abs(exact).max()
    mse = ims.std(0, ddof=1) / math.sqrt(K)
    n = K * 8
    assert (np.abs(ims.mean(0) - exact_img) <= 5 * mse + 3 * 0.7 / n + 1e-7).all()


# ---------------------------------------------------------------------------
# gradient vs central differences of renders
# ---------------------------------------------------------------------------

def _fd_check(scene, cam, depth, directions, n_grad, spp_grad, n_fd, spp_fd, h_geom):
    """Returns rows (name, g, se_g, fd, se_fd) for each direction (name, u)
    over the flattened parameters [vertices (3V) | albedo (T) | camera (9)]."""
    x0, y0, x1, y1 = cam.win()
    w = np.random.default_rng(0).uniform(0.5, 1.5, size=(y1 - y0, x1 - x0))
    V, T = scene.num_vertices, scene.num_triangles
    gs = []
    for s in range(n_grad):
        r = oracle.render(scene, cam, spp_grad, depth, 1000 + s, d_image=w, threads=THREADS)
        gs.append(np.concatenate([r["d_vertices"].ravel(), r["d_albedo"], r["d_camera"]]))
    gs = np.array(gs)
    v64 = scene.vertices.astype(np.float64)
    a64 = scene.albedo.astype(np.float64)
    c64 = cam.params9().astype(np.float64)

    def L(d, seed):
        r = oracle.render(scene, cam, spp_fd, depth, seed, threads=THREADS, vertices64=v64 + d[:3 * V].reshape(V, 3),
                          albedo64=a64 + d[3 * V:3 * V + T], camera64=c64 + d[3 * V + T:])
        return float((w * r["image"]).sum())

    rows = []
    for name, u in directions:
        h = 1e-2 if name.startswith("albedo") else h_geom
        proj = gs @ u
        vals = np.array([(L(u * h, s) - L(-u * h, s)) / (2 * h) for s in range(n_fd)])
        rows.append((name, proj.mean(), proj.std(ddof=1) / math.sqrt(n_grad), vals.mean(),
                     vals.std(ddof=1) / math.sqrt(n_fd)))
    return rows


def _directions(scene, vertex_coords, albedos, rng, n_random=4):
    V, T = scene.num_vertices, scene.num_triangles
    n = 3 * V + T + 9
    out = []
    for k, nm in enumerate(["pos.x", "pos.y", "pos.z", "look.x", "look.y", "look.z", "up.x"]):
        u = np.zeros(n)
        u[3 * V + T + k] = 1.0
        out.append((f"camera {nm}", u))
    for vi, c in vertex_coords:
        u = np.zeros(n)
        u[3 * vi + c] = 1.0
        out.append((f"vertex {vi}.{'xyz'[c]}", u))
    for k in range(n_random):
        u = np.zeros(n)
        u[:3 * V] = rng.normal(size=3 * V)
        u[:3 * V] /= np.linalg.norm(u[:3 * V])
        out.append((f"random vertex direction {k}", u))
    for t in albedos:
        u = np.zeros(n)
        u[3 * V + t] = 1.0
        out.append((f"albedo {t}", u))
    return out


def _assert_agreement(rows):
    z2 = 0.0
    l1_err = l1 = noise = 0.0
    for name, g, se, fd, fse in rows:
        s = math.hypot(se, fse)
        z = (g - fd) / s if s > 0 else 0.0
        print(f"{name:28s} gradient {g: .5e} +- {se:.1e}   central difference {fd: .5e} +- {fse:.1e}   z {z: .2f}")
        assert abs(z) <= 4.5, name
        z2 += z * z
        l1_err += abs(g - fd)
        l1 += abs(fd)
        noise += se + fse
    print(f"L1 error / L1 norm = {l1_err / l1:.4f} (Monte Carlo noise floor {noise / l1:.4f}); sum z^2 = {z2:.1f}"
          f" over {len(rows)} directions")
    assert z2 <= CHI2_999[len(rows)]
    return l1_err / l1, noise / l1


@pytest.mark.slow
def test_depth1_gradient_matches_central_differences():
    scene, cam = shadow_scene()
    # occluder vertices (8..11), a light vertex (5), the floor and occluder albedos
    dirs = _directions(scene, [(8, 0), (9, 1), (11, 2), (10, 0), (5, 0)], [0, 4, 5], np.random.default_rng(5), 3)
    assert len(dirs) == 18
    D = float(np.linalg.norm(scene.vertices.max(0) - scene.vertices.min(0)))
    rows = _fd_check(scene, cam, 1, dirs, 16 * SCALE, 256, 4 * SCALE, 1024, 3e-3 * D)
    err, noise = _assert_agreement(rows)
    assert noise < 0.05


@pytest.mark.slow
def test_depth3_gradient_matches_central_differences():
    scene, cam = crease_scene()
    # the roof's crease vertices (9, 10), a roof corner (12), the tilted quad (15), a light vertex (6)
    dirs = _directions(scene, [(9, 1), (10, 0), (12, 2), (15, 1), (6, 2)], [4, 6, 8], np.random.default_rng(6), 3)
    assert len(dirs) == 18
    D = float(np.linalg.norm(scene.vertices.max(0) - scene.vertices.min(0)))
    rows = _fd_check(scene, cam, 3, dirs, 32 * SCALE, 128, 4 * SCALE, 512, 3e-3 * D)
    err, noise = _assert_agreement(rows)
    assert noise < 0.08
