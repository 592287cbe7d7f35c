"""Pins of the oracle's geometry buffers (position, shading normal, albedo at
the first camera hit; thesis Ch. 5, Results: G-buffer / AOV outputs), CPU.

* albedo buffer of the two-triangle scene: the mean over seeds equals the exact
  box-filtered albedo image (polygon clipping), and its vertex and albedo
  gradients equal finite differences of that closed form;
* position and normal buffers: the interior gradient equals central finite
  differences of the per-sample estimator (screen samples fixed, no decision
  changes), on a flat triangle soup and on a smooth-normal sphere;
* translating camera and scene together inside a closed box (every camera ray
  hits): the position buffer moves rigidly, so sum_v dV + d_position +
  d_look_at = sum_p d_p per coordinate; normals and albedos do not move, so the
  same sum is 0 for them.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1904_12228_amd import scenegen as sg

from . import analytic
from .test_oracle_pins import small_soup, small_sphere


def test_albedo_buffer_and_gradient_match_exact_coverage():
    cfg = sg.config1()
    s = cfg.scene
    alb = np.array([0.3, 0.8], np.float32)
    scene = sg.Scene(s.vertices, s.indices, alb, np.zeros(2, np.float32), None, False, 0.0)
    cam = cfg.camera
    W, H, fov = cam.width, cam.height, cam.fov_y_deg
    dimg = np.random.default_rng(12).normal(size=(H, W)) + 1.0
    cam9 = cam.params9().astype(np.float64)
    v0 = scene.vertices.astype(np.float64)
    a64 = alb.astype(np.float64)
    exact_img = analytic.two_triangle_image(v0, a64, 0.0, cam9, fov, W, H)
    J = lambda v, a: float((dimg * analytic.two_triangle_image(v, a, 0.0, cam9, fov, W, H)).sum())
    exact_g = np.zeros(18)
    for k in range(18):
        h = 1e-6
        vp = v0.copy(); vp.ravel()[k] += h
        vm = v0.copy(); vm.ravel()[k] -= h
        exact_g[k] = (J(vp, a64) - J(vm, a64)) / (2 * h)
    exact_ga = np.array([(J(v0, a64 + 1e-3 * np.eye(2)[i]) - J(v0, a64 - 1e-3 * np.eye(2)[i])) / 2e-3 for i in range(2)])
    K = 48
    gs, gas, ims = [], [], []
    for seed in range(K):
        r = oracle.render(scene, cam, cfg.spp, 0, seed, d_image=dimg, threads=8, aov=7)
        gs.append(r["d_vertices"].ravel())
        gas.append(r["d_albedo"])
        ims.append(r["image"])
    for est, exact in ((np.array(gs), exact_g), (np.array(gas), exact_ga)):
        se = est.std(0, ddof=1) / math.sqrt(K)
        assert (np.abs(est.mean(0) - exact) <= 5 * se + 1e-9).all(), (est.mean(0), exact, se)
        assert np.abs(est.mean(0) - exact).max() < 0.05 * np.abs(exact).max()
    ims = np.array(ims)
    mse = ims.std(0, ddof=1) / math.sqrt(K)
    # a pixel region of area < ~3/n may never be sampled by n samples (zero
    # sample variance); allow that much of the value range (0 .. 0.8)
    n = K * cfg.spp
    assert (np.abs(ims.mean(0) - exact_img) <= 5 * mse + 3 * 0.8 / n + 1e-12).all()


def _interior_fd(scene, cam, aov, seed, rng, n_params=12):
    win = cam.win()
    dimg = rng.normal(size=(win[3] - win[1], win[2] - win[0]))
    base = oracle.render(scene, cam, 2, 0, seed, d_image=dimg, primary=False, want_flags=True, aov=aov)
    mask = 1 - base["unit_flags"]
    g = oracle.render(scene, cam, 2, 0, seed, d_image=dimg, primary=False, unit_mask=mask, aov=aov)
    v64 = scene.vertices.astype(np.float64)
    c64 = cam.params9().astype(np.float64)
    touched = np.nonzero(np.abs(g["d_vertices"]).ravel() > 0)[0]
    assert touched.size > 6
    picks = [("v", int(i)) for i in rng.choice(touched, size=min(n_params, touched.size), replace=False)]
    picks += [("c", k) for k in range(9)]
    h = 1e-7
    for kind, i in picks:
        def img(delta):
            v, c = v64.copy(), c64.copy()
            if kind == "v":
                v.ravel()[i] += delta
            else:
                c[i] += delta
            return oracle.render(scene, cam, 2, 0, seed, unit_mask=mask, vertices64=v, camera64=c, aov=aov)["image"]
        fd = float((dimg * (img(h) - img(-h))).sum() / (2 * h))
        an = g["d_vertices"].ravel()[i] if kind == "v" else g["d_camera"][i]
        scale = max(abs(an), abs(fd), 1e-3 * np.abs(g["d_vertices"]).max())
        assert abs(fd - an) <= 2e-5 * scale, (aov, kind, i, fd, an)


@pytest.mark.parametrize("aov", [1, 2, 3, 4, 5, 6])
def test_position_and_normal_buffer_interior_gradients_match_fd(aov):
    rng = np.random.default_rng(aov)
    scene, cam, _ = small_soup(n=12)
    _interior_fd(scene, cam, aov, 3, rng)
    if aov >= 4:
        scene, cam, _ = small_sphere(level=2)
        _interior_fd(scene, cam, aov, 4, rng)


def test_translation_of_camera_and_scene_moves_only_the_position_buffer():
    # the camera sits inside the closed box: every camera ray hits a surface
    scene, cam, cfg = small_sphere(level=2, w=30, h=22, x0=2, y0=4)
    win = cam.win()
    dimg = np.random.default_rng(7).normal(size=(win[3] - win[1], win[2] - win[0]))
    for aov in range(1, 8):
        r = oracle.render(scene, cam, 2, 0, 5, d_image=dimg, aov=aov)
        tot = r["d_vertices"].sum(0) + r["d_camera"][0:3] + r["d_camera"][3:6]
        mass = r["mass_vertices"].sum(0) + r["mass_camera"][0:3] + r["mass_camera"][3:6] + np.abs(dimg).sum()
        expect = np.zeros(3)
        if aov <= 3:
            expect[aov - 1] = dimg.sum()
        assert (np.abs(tot - expect) <= 1e-9 * mass).all(), (aov, tot, expect)


def test_one_sample_buffers_are_hit_points_on_the_reported_triangle():
    # one sample per pixel: the position buffer is one ray's first hit, which
    # must project into its own pixel and lie on the triangle whose albedo the
    # albedo buffer reports; the normal buffer is that triangle's unit normal,
    # turned towards the camera
    cfg = sg.config1()
    s = cfg.scene
    alb = np.array([0.3, 0.8], np.float32)
    scene = sg.Scene(s.vertices, s.indices, alb, np.zeros(2, np.float32), None, False, 0.0)
    cam = cfg.camera
    W, H = cam.width, cam.height
    cam9 = cam.params9().astype(np.float64)
    buf = {a: oracle.render(scene, cam, 1, 0, 21, aov=a)["image"] for a in range(1, 8)}
    hit = buf[7] > 0
    assert 200 < hit.sum() < W * H
    P = np.stack([buf[1], buf[2], buf[3]], -1)[hit]
    N = np.stack([buf[4], buf[5], buf[6]], -1)[hit]
    ys, xs = np.nonzero(hit)
    sxy = analytic.project(P, cam9, cam.fov_y_deg, W, H)
    assert (sxy[:, 0] >= xs - 1e-9).all() and (sxy[:, 0] <= xs + 1 + 1e-9).all()
    assert (sxy[:, 1] >= ys - 1e-9).all() and (sxy[:, 1] <= ys + 1 + 1e-9).all()
    v = scene.vertices.astype(np.float64).reshape(2, 3, 3)
    tri = np.where(np.isclose(buf[7][hit], 0.8), 1, 0)
    assert np.isclose(buf[7][hit], alb[tri]).all()
    for t in (0, 1):
        a, b, c = v[t]
        n = np.cross(b - a, c - a)
        n /= np.linalg.norm(n)
        sel = tri == t
        assert sel.sum() > 20
        np.testing.assert_allclose((P[sel] - a) @ n, 0.0, atol=1e-9)
        np.testing.assert_allclose(np.abs(N[sel] @ n), 1.0, atol=1e-12)
        np.testing.assert_allclose(np.linalg.norm(N[sel], axis=1), 1.0, atol=1e-12)
        assert ((N[sel] * (P[sel] - cam9[0:3])).sum(1) < 0).all()
    assert (np.abs(np.stack([buf[k] for k in range(1, 7)])[:, ~hit]) == 0).all()
