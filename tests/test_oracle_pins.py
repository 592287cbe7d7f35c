"""Pins of the FP64 oracle against what the thesis and mathematics fix.

Each test checks the oracle against something other than itself: published
known-answer vectors, closed forms, finite differences of exact or
fixed-random-number functions, invariants, or brute force.
"""
import math
import os

import numpy as np
import pytest

import oracle
from paper_1904_12228_amd import scenegen as sg

from . import analytic

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def small_soup(n=12, w=24, h=20, spp=2, seed=3):
    cfg = sg.soup(seed=seed, n_tris=n, width=64, height=64, spp=spp)
    cam = cfg.camera.with_window(20, 22, 20 + w, 22 + h)
    return cfg.scene, cam, cfg


def small_sphere(level=2, w=20, h=16, spp=2, x0=14, y0=16):
    cfg = sg.sphere_box(seed=1, level=level, width=48, height=48, spp=spp, max_depth=3)
    cam = cfg.camera.with_window(x0, y0, x0 + w, y0 + h)
    return cfg.scene, cam, cfg


# ---------------------------------------------------------------------------
# Philox4x32-10: published known-answer vectors
# ---------------------------------------------------------------------------

def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        assert oracle.philox4x32_10(v[0:4], v[4:6]) == v[6:10]


# ---------------------------------------------------------------------------
# topology and ray casting
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("level", [0, 1, 2, 3])
def test_icosphere_edges_euler(level):
    v, f = sg.icosphere(level)
    scene = sg.Scene(v.astype(np.float32), f.astype(np.int32), np.full(len(f), 0.5, np.float32),
                     np.zeros(len(f), np.float32))
    e = oracle.edges(scene)
    assert e.shape[0] == 30 * 4 ** level                 # closed mesh: E = 3F/2
    assert len(v) - e.shape[0] + len(f) == 2             # Euler characteristic of a sphere
    assert (e[:, 3] >= 0).all() and (e[:, 0] < e[:, 1]).all()


def test_bvh_matches_brute_force():
    scene, cam, cfg = small_soup(n=60)
    rng = np.random.default_rng(0)
    o = rng.uniform(-0.5, 1.5, size=(3000, 3))
    d = rng.normal(size=(3000, 3))
    t1, tt1 = oracle.closest_hit(scene, o, d, 1e-4, 1e30, use_bvh=True)
    t2, tt2 = oracle.closest_hit(scene, o, d, 1e-4, 1e30, use_bvh=False)
    assert (t1 == t2).all()
    assert np.array_equal(tt1, tt2)
    assert (t1 >= 0).sum() > 300


# ---------------------------------------------------------------------------
# secondary edge term: the thesis's area-measure form vs the direction form
# ---------------------------------------------------------------------------

def test_secondary_area_form_equals_direction_form():
    rng = np.random.default_rng(1)
    for _ in range(200):
        p = rng.normal(size=3)
        v0 = p + rng.normal(size=3) + np.array([0, 0, 3.0])
        v1 = p + rng.normal(size=3) + np.array([0, 0, 3.0])
        t = rng.uniform()
        w = v0 + (v1 - v0) * t - p
        m0 = p + w * rng.uniform(1.5, 3.0) + rng.normal(size=3) * 0.1
        nm = rng.normal(size=3)
        if abs(nm @ w) < 0.2 * np.linalg.norm(nm) * np.linalg.norm(w):
            continue
        af, df = oracle.secondary_forms(p, v0, v1, t, m0, nm)
        # The area form multiplies the area-measure integrand h, the direction
        # form the solid-angle integrand F = h |m'|^2 / |cos theta_m|.
        nmu = nm / np.linalg.norm(nm)
        tau = ((m0 - p) @ nmu) / (w @ nmu)
        mp = tau * w
        conv = abs(nmu @ mp) / np.linalg.norm(mp) / (mp @ mp)
        # endpoint terms agree exactly: tau, cos theta_m and |n_m x n_h| cancel
        # against the Jacobian J_m of the appendix derivation
        np.testing.assert_allclose(af[0] * conv, df[0], rtol=1e-9, atol=1e-12)
        np.testing.assert_allclose(af[1] * conv, df[1], rtol=1e-9, atol=1e-12)
        # shading-point terms differ by exactly the -(v0' x v1') term of m-fixed
        v0p, v1p = v0 - p, v1 - p
        c = np.cross(v0p, v1p)
        sc = np.linalg.norm(af[0]) / np.linalg.norm(np.cross(v1p, mp))
        np.testing.assert_allclose((af[2] - (-c) * sc) * conv, df[2], rtol=1e-8, atol=1e-10)


def test_edge_equation_partials_match_thesis_closed_form():
    """eq. redner_dirac_jacobian: partials of the 2D edge equation, checked by
    finite differences of eq. edge_equation, plus translation invariance."""
    rng = np.random.default_rng(2)
    for _ in range(50):
        ax, ay, bx, by, x, y = rng.normal(size=6)
        alpha = lambda ax, ay, bx, by, x, y: (ay - by) * x + (bx - ax) * y + (ax * by - bx * ay)
        closed = [by - y, x - bx, y - ay, ax - x, ay - by, bx - ax]
        args = [ax, ay, bx, by, x, y]
        for k in range(6):
            h = 1e-6
            ap = list(args); ap[k] += h
            am = list(args); am[k] -= h
            fd = (alpha(*ap) - alpha(*am)) / (2 * h)
            assert abs(fd - closed[k]) < 1e-7
        assert abs(closed[0] + closed[2] + closed[4]) < 1e-12
        assert abs(closed[1] + closed[3] + closed[5]) < 1e-12


# ---------------------------------------------------------------------------
# edge hierarchy: the explicit pdf is a distribution and matches sampling
# ---------------------------------------------------------------------------

def _shading_points(scene, n, rng):
    pts = []
    I = scene.indices
    V = scene.vertices.astype(np.float64)
    for f in rng.integers(0, len(I), size=n):
        a, b, c = V[I[f]]
        u, v = rng.uniform(size=2)
        if u + v > 1:
            u, v = 1 - u, 1 - v
        p = a + (b - a) * u + (c - a) * v
        nn = np.cross(b - a, c - a)
        nn /= np.linalg.norm(nn)
        pts.append((p + nn * 1e-3, nn))
    return pts


@pytest.mark.parametrize("which", ["soup", "sphere"])
def test_edge_tree_pdf_is_normalised(which):
    scene, cam, cfg = small_soup(n=40) if which == "soup" else small_sphere(level=2)
    rng = np.random.default_rng(4)
    for p, n in _shading_points(scene, 12, rng):
        pdf, fail = oracle.edge_tree_pdf(scene, cam, p, n)
        assert (pdf >= 0).all()
        assert abs(pdf.sum() + fail - 1.0) < 1e-12


def test_edge_tree_sampling_matches_pdf():
    scene, cam, cfg = small_sphere(level=1)
    rng = np.random.default_rng(5)
    (p, n), = _shading_points(scene, 1, rng)
    pdf, fail = oracle.edge_tree_pdf(scene, cam, p, n)
    N = 200000
    u = rng.uniform(size=(N, 65))
    e, pd = oracle.edge_tree_sample(scene, cam, p, n, u)
    ok = e >= 0
    # the pdf reported by a descent equals the enumerated pdf of that edge
    np.testing.assert_allclose(pd[ok], pdf[e[ok]], rtol=1e-12)
    assert abs((~ok).mean() - fail) < 5 * math.sqrt(max(fail, 1e-6) / N) + 1e-4
    counts = np.bincount(e[ok], minlength=len(pdf))
    big = pdf * N > 50
    chi2 = (((counts[big] - pdf[big] * N) ** 2) / (pdf[big] * N)).sum()
    dof = big.sum() - 1
    assert chi2 < dof + 6 * math.sqrt(2 * dof)


# ---------------------------------------------------------------------------
# interior term: reverse mode equals finite differences of the per-sample
# estimator with its integration variables held fixed (screen point, sampled
# world directions and their solid-angle pdfs) and no decision changes
# ---------------------------------------------------------------------------

def _interior_fd(scene, cam, spp, depth, seed, n_params, rng):
    win = cam.win()
    dimg = rng.normal(size=(win[3] - win[1], win[2] - win[0]))
    M = (win[3] - win[1]) * (win[2] - win[0]) * spp
    dlog = np.zeros(M * 64)
    base = oracle.render(scene, cam, spp, depth, seed, d_image=dimg, primary=False, secondary=False,
                         want_flags=True, dir_mode=1, dir_log=dlog)
    mask = 1 - base["unit_flags"]
    g = oracle.render(scene, cam, spp, depth, seed, d_image=dimg, primary=False, secondary=False, unit_mask=mask)
    v64 = scene.vertices.astype(np.float64)
    a64 = scene.albedo.astype(np.float64)
    c64 = cam.params9().astype(np.float64)
    touched = np.nonzero(np.abs(g["d_vertices"]).ravel() > 0)[0]
    assert touched.size > 10
    picks = [("v", int(i)) for i in rng.choice(touched, size=min(n_params, touched.size), replace=False)]
    picks += [("c", k) for k in range(9)]
    at = np.nonzero(g["d_albedo"])[0]
    picks += [("a", int(i)) for i in rng.choice(at, size=min(4, at.size), replace=False)]
    h = 1e-7
    for kind, i in picks:
        def img(delta):
            v, a, c = v64.copy(), a64.copy(), c64.copy()
            if kind == "v":
                v.ravel()[i] += delta
            elif kind == "a":
                a[i] += delta
            else:
                c[i] += delta
            return oracle.render(scene, cam, spp, depth, seed, unit_mask=mask, vertices64=v, albedo64=a,
                                 camera64=c, dir_mode=2, dir_log=dlog)["image"]
        fd = float((dimg * (img(h) - img(-h))).sum() / (2 * h))
        an = {"v": lambda: g["d_vertices"].ravel()[i], "a": lambda: g["d_albedo"][i], "c": lambda: g["d_camera"][i]}[kind]()
        scale = max(abs(an), abs(fd), 1e-3 * np.abs(g["d_vertices"]).max())
        assert abs(fd - an) <= 2e-5 * scale, (kind, i, fd, an)


def test_interior_reverse_mode_matches_fd_direct_lighting():
    scene, cam, cfg = small_soup(n=12)
    _interior_fd(scene, cam, 2, 1, 7, 25, np.random.default_rng(6))


def test_interior_reverse_mode_matches_fd_path_tracing_smooth_normals():
    scene, cam, cfg = small_sphere(level=2)
    _interior_fd(scene, cam, 2, 3, 8, 25, np.random.default_rng(7))


# ---------------------------------------------------------------------------
# invariants of the full estimator (interior + primary + secondary)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("which", ["soup", "sphere"])
def test_translation_invariance_pins_camera_gradient(which):
    """Translating the camera and every vertex together leaves every sample
    unchanged, so sum_v dV + d_position + d_look_at = 0 for every sample."""
    scene, cam, cfg = small_soup(n=12) if which == "soup" else small_sphere(level=2, w=30, h=22, x0=2, y0=4)
    depth = cfg.max_depth
    win = cam.win()
    rng = np.random.default_rng(9)
    dimg = rng.normal(size=(win[3] - win[1], win[2] - win[0]))
    r = oracle.render(scene, cam, 2, depth, 11, d_image=dimg)
    tot = r["d_vertices"].sum(0) + r["d_camera"][0:3] + r["d_camera"][3:6]
    mass = r["mass_vertices"].sum(0) + r["mass_camera"][0:3] + r["mass_camera"][3:6]
    assert (mass > 0).all()
    assert (np.abs(tot) <= 1e-9 * mass).all(), (tot, mass)
    assert r["stats"][2] > 0                      # primary edge samples were used
    assert r["stats"][3] > 0                      # secondary edge samples were used


def test_albedo_gradient_is_exact_polynomial_derivative():
    """With random numbers fixed the image is a polynomial in each albedo
    (degree <= depth); its Lagrange-interpolated derivative is exact."""
    scene, cam, cfg = small_sphere(level=2)
    win = cam.win()
    rng = np.random.default_rng(10)
    dimg = rng.normal(size=(win[3] - win[1], win[2] - win[0]))
    r = oracle.render(scene, cam, 2, 3, 12, d_image=dimg, primary=False, secondary=False)
    a64 = scene.albedo.astype(np.float64)
    for i in np.argsort(-np.abs(r["d_albedo"]))[:5]:
        xs = a64[i] + np.array([-0.2, -0.1, 0.1, 0.2])
        ys = []
        for x in xs:
            a = a64.copy()
            a[i] = x
            ys.append(float((dimg * oracle.render(scene, cam, 2, 3, 12, albedo64=a)["image"]).sum()))
        coef = np.polyfit(xs - a64[i], ys, 3)
        assert abs(coef[2] - r["d_albedo"][i]) <= 1e-8 * max(1.0, abs(r["d_albedo"][i]))


def test_hidden_triangle_has_exactly_zero_gradient():
    """Occlusion (thesis: an occluded edge sample lands on the continuous part):
    a triangle fully behind another gets exactly zero gradient per sample."""
    verts = np.array([[-1, -1, 2], [1, -1, 2], [0, 1.2, 2],          # big front triangle
                      [-0.2, -0.2, 3], [0.2, -0.2, 3], [0, 0.2, 3]],  # small one behind it
                     np.float32)
    scene = sg.Scene(verts, np.array([[0, 1, 2], [3, 4, 5]], np.int32), np.zeros(2, np.float32),
                     np.array([0.7, 0.3], np.float32), None, True, 0.1)
    cam = sg.Camera((0, 0, 0), (0, 0, 1), (0, 1, 0), 60.0, 32, 32)
    r = oracle.render(scene, cam, 4, 0, 0, d_image=np.random.default_rng(0).normal(size=(32, 32)))
    assert np.all(r["d_vertices"][3:] == 0)
    assert np.abs(r["d_vertices"][:3]).max() > 0


# ---------------------------------------------------------------------------
# statistical pins of the boundary terms against exact closed forms
# ---------------------------------------------------------------------------

@pytest.mark.slow
def test_primary_edges_match_exact_pixel_coverage():
    """Configuration-1 scene: mean of the oracle over seeds equals the exact
    box-filtered image and the exact derivative of sum_p d_p I_p (FD of the
    closed-form coverage), within the Monte Carlo error."""
    cfg = sg.config1()
    scene, cam = cfg.scene, cfg.camera
    W, H, fov = cam.width, cam.height, cam.fov_y_deg
    rng = np.random.default_rng(12)
    dimg = rng.normal(size=(H, W)) + 1.0
    cam9 = cam.params9().astype(np.float64)
    v0 = scene.vertices.astype(np.float64)
    emi = scene.emission.astype(np.float64)
    bg = float(np.float32(scene.background))           # the renderer's input is FP32
    exact_img = analytic.two_triangle_image(v0, emi, bg, cam9, fov, W, H)
    J = lambda v: float((dimg * analytic.two_triangle_image(v, emi, bg, cam9, fov, W, H)).sum())
    exact_g = np.zeros(18)
    for k in range(18):
        h = 1e-6
        vp = v0.copy(); vp.ravel()[k] += h
        vm = v0.copy(); vm.ravel()[k] -= h
        exact_g[k] = (J(vp) - J(vm)) / (2 * h)
    K = 48
    gs, ims = [], []
    for seed in range(K):
        r = oracle.render(scene, cam, cfg.spp, 0, seed, d_image=dimg, threads=8)
        gs.append(r["d_vertices"].ravel())
        ims.append(r["image"])
    gs = np.array(gs)
    ims = np.array(ims)
    se = gs.std(0, ddof=1) / math.sqrt(K)
    assert (np.abs(gs.mean(0) - exact_g) <= 5 * se + 1e-9).all(), (gs.mean(0), exact_g, se)
    # and the estimate is informative: error well below the gradient scale
    assert np.abs(gs.mean(0) - exact_g).max() < 0.05 * np.abs(exact_g).max()
    mse = ims.std(0, ddof=1) / math.sqrt(K)
    err = np.abs(ims.mean(0) - exact_img)
    # a pixel region of area < ~3/n may never be sampled by n samples (zero
    # sample variance); allow that much of the value range
    n = K * cfg.spp
    vrange = max(emi.max(), bg) - min(emi.min(), bg)
    assert (err <= 5 * mse + 3 * vrange / n + 1e-12).all()
    assert np.abs(ims.mean(0).sum() - exact_img.sum()) < 5 * math.sqrt((mse ** 2).sum()) + 1e-9


def _lambert_scene():
    """Large floor (y=0) seen at a grazing angle, a quad light above, a
    triangle occluder in between, neither visible to the camera."""
    floor = ([-10, 0, -10], [-10, 0, 10], [10, 0, 10], [10, 0, -10])
    light = ([-0.15, 1.0, 0.15], [0.15, 1.0, 0.15], [0.15, 1.0, 0.45], [-0.15, 1.0, 0.45])
    occ = [[-0.05, 0.55, 0.2], [0.12, 0.5, 0.25], [0.0, 0.52, 0.42]]
    v = np.array(list(floor) + list(light) + occ, np.float64)
    f = np.array([[0, 1, 2], [0, 2, 3], [4, 5, 6], [4, 6, 7], [8, 9, 10]], np.int32)
    ln = np.cross(v[5] - v[4], v[6] - v[4])
    assert ln[1] < 0                                   # light faces down
    scene = sg.Scene(v.astype(np.float32), f, np.array([0.6, 0.6, 0, 0, 0.4], np.float32),
                     np.array([0, 0, 8.0, 8.0, 0], np.float32), None, False, 0.0)
    cam = sg.Camera((0.0, 0.3, -1.6), (0.0, 0.0, 0.3), (0.0, 1.0, 0.0), 12.0, 6, 6)
    return scene, cam


@pytest.mark.slow
def test_secondary_edges_match_lambert_polygon_irradiance():
    scene, cam = _lambert_scene()
    W, H, fov = cam.width, cam.height, cam.fov_y_deg
    v0 = scene.vertices.astype(np.float64)
    cam9 = cam.params9().astype(np.float64)
    rho = 0.6
    Le = 8.0
    G = 10                                    # quadrature points per pixel side
    s = (np.arange(W * G) + 0.5) / G
    sx, sy = np.meshgrid(s, (np.arange(H * G) + 0.5) / G)
    o, d = analytic.screen_ray(sx.ravel(), sy.ravel(), cam9, fov, W, H)
    t = -o[1] / d[:, 1]
    X = o[None] + d * t[:, None]
    n = np.array([0.0, 1.0, 0.0])
    rng = np.random.default_rng(13)
    dimg = rng.uniform(0.5, 1.5, size=(H, W))
    wq = dimg[(sy.ravel() // 1).astype(int), (sx.ravel() // 1).astype(int)] / G ** 2

    def J(v):
        light = v[[4, 5, 6, 7]]
        occ = v[[8, 9, 10]]
        return sum(w * rho / math.pi * analytic.shadowed_irradiance(x, n, light, occ, Le) for x, w in zip(X, wq))

    params = [(8, 0), (8, 1), (8, 2), (9, 0), (9, 1), (10, 2), (5, 0), (6, 2)]
    exact = {}
    for vi, k in params:
        h = 1e-5
        vp = v0.copy(); vp[vi, k] += h
        vm = v0.copy(); vm[vi, k] -= h
        exact[(vi, k)] = (J(vp) - J(vm)) / (2 * h)
    K = 40
    gs = []
    for seed in range(K):
        r = oracle.render(scene, cam, 256, 1, seed, d_image=dimg, threads=8)
        assert r["stats"][1] < 0.01 * 36 * 256        # near-tie units are rare
        gs.append([r["d_vertices"][vi, k] for vi, k in params])
    gs = np.array(gs)
    se = gs.std(0, ddof=1) / math.sqrt(K)
    ex = np.array([exact[p] for p in params])
    assert (np.abs(gs.mean(0) - ex) <= 5 * se + 1e-9).all(), (gs.mean(0), ex, se)
    assert np.abs(gs.mean(0) - ex).max() < 0.1 * np.abs(ex).max()
