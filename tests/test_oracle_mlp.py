"""Pins of the proposal network's FP64 oracle (oracle/mlp.py), on the CPU.

* bfloat16 rounding against torch's float32 -> bfloat16 conversion (round to
  nearest even), ties included;
* the forward pass and the hand-written backward against torch autograd in
  float64, both without rounding and with the kernels' BF16 inputs and
  weights (straight-through rounding);
* the smooth (unrounded) loss gradient against central finite differences;
* softmax cross-entropy against torch's cross entropy with soft targets;
* edge features against closed-form camera facts and invariances.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import mlp
from paper_1904_12228_amd import scenegen as sg

torch = pytest.importorskip("torch")


def test_bf16_matches_torch_round_to_nearest_even():
    rng = np.random.default_rng(0)
    x = (rng.normal(size=20000) * np.exp(rng.uniform(-20, 20, 20000))).astype(np.float32)
    bits = x.view(np.uint32)
    ties = ((bits & np.uint32(0xFFFF0000)) | np.uint32(0x8000)).view(np.float32)   # exact midpoints
    x = np.concatenate([x, ties, np.float32([0.0, -0.0, 1.0, -3.0])])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(mlp.bf16(x.astype(np.float64)), ref)


def _torch_net(theta, X, rounding):
    W1, b1, W2, b2, W3, b3 = [torch.tensor(np.atleast_1d(a), dtype=torch.float64) for a in mlp.unpack(theta)]
    for t in (W1, b1, W2, b2, W3, b3):
        t.requires_grad_(True)
    r = (lambda v: v.to(torch.bfloat16).to(torch.float64)) if rounding else (lambda v: v)
    st = lambda v: v + (r(v) - v).detach()
    Xb = r(torch.tensor(X, dtype=torch.float64))
    h1 = torch.relu(Xb @ st(W1) + b1)
    h2 = torch.relu(h1 @ st(W2) + b2)
    z = h2 @ st(W3) + b3
    return z, (W1, b1, W2, b2, W3, b3)


@pytest.mark.parametrize("rounding", [False, True])
def test_forward_and_backward_match_torch_autograd(rounding):
    theta = sg.mlp_params(3, bias_scale=0.1)
    X = sg.mlp_inputs(4, 300)
    dz = np.random.default_rng(5).normal(size=300)
    z, mz, flag, cache = mlp.forward(theta, X, rounding=rounding)
    g, mass = mlp.backward(theta, cache, dz)
    zt, params = _torch_net(theta, X, rounding)
    np.testing.assert_allclose(z, zt.detach().numpy(), rtol=1e-12, atol=1e-12)
    (zt * torch.tensor(dz)).sum().backward()
    gt = np.concatenate([p.grad.numpy().ravel() for p in params])
    np.testing.assert_allclose(g, gt, rtol=1e-10, atol=1e-12 * np.abs(gt).max())
    assert (mass >= np.abs(g) * (1 - 1e-12)).all()
    assert flag.mean() < 0.02


def test_smooth_loss_gradient_matches_finite_differences():
    theta = sg.mlp_params(6, bias_scale=0.1).astype(np.float64)
    X = sg.mlp_inputs(7, 120)
    offsets = [0, 50, 50, 120]
    target = np.abs(np.random.default_rng(8).normal(size=120))

    def loss(th):
        z, _, _, _ = mlp.forward(th, X, rounding=False)
        return mlp.softmax_xent(z, target, offsets)[1]

    z, _, _, cache = mlp.forward(theta, X, rounding=False)
    _, _, dz = mlp.softmax_xent(z, target, offsets)
    g, _ = mlp.backward(theta, cache, dz)
    rng = np.random.default_rng(9)
    h = 1e-6
    for i in list(rng.choice(mlp.N_PARAMS, 30, replace=False)) + [mlp.OFF_B3, mlp.OFF_W3, mlp.OFF_B1]:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (loss(tp) - loss(tm)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(g).max()), (i, fd, g[i])


def test_softmax_cross_entropy_matches_torch():
    rng = np.random.default_rng(10)
    z = rng.normal(size=70) * 3
    target = np.abs(rng.normal(size=70))
    target[40:55] = 0.0                       # a view with zero target is skipped
    offsets = [0, 40, 55, 70]
    p, loss, dz = mlp.softmax_xent(z, target, offsets)
    zt = torch.tensor(z, requires_grad=True)
    ls = []
    for lo, hi in ((0, 40), (55, 70)):
        t = torch.tensor(target[lo:hi] / target[lo:hi].sum())
        ls.append(torch.nn.functional.cross_entropy(zt[lo:hi][None], t[None]))
    lt = sum(ls) / len(ls)
    lt.backward()
    assert abs(loss - lt.item()) < 1e-12
    np.testing.assert_allclose(dz, zt.grad.numpy(), atol=1e-14)
    for lo, hi in ((0, 40), (40, 55), (55, 70)):
        assert abs(p[lo:hi].sum() - 1) < 1e-12


def _features(scene, cam):
    return mlp.edge_features(scene, cam, oracle.edges(scene))


def test_features_at_closed_form_camera_points():
    # camera at the origin looking down +z with +y up: the view axis maps to
    # screen (0, 0); a point on the upper frustum plane to y = 1; a point on
    # the right frustum plane to x = 1.
    fov, W, H = 60.0, 64, 48
    th = math.tan(math.radians(fov) / 2)
    asp = W / H
    z = 2.0
    right = np.cross([0.0, 0.0, 1.0], [0.0, 1.0, 0.0])        # image right in world space
    v = np.array([[0, 0, z], [0, z * th, z], right * z * th * asp + [0, 0, z]], np.float32)
    scene = sg.Scene(v, np.array([[0, 1, 2]], np.int32), np.float32([0.3]), np.float32([0.0]), None, False, 0.0)
    cam = sg.Camera((0, 0, 0), (0, 0, 1), (0, 1, 0), fov, W, H)
    X = _features(scene, cam)
    e = oracle.edges(scene)
    for row, (va, vb, f0, f1) in zip(X, e):
        for j, vi in ((24, va), (26, vb)):
            expect = {0: (0.0, 0.0), 1: (0.0, 1.0), 2: (1.0, 0.0)}[int(vi)]
            np.testing.assert_allclose(row[j:j + 2], expect, atol=1e-12)
        assert row[22] == 1.0 and row[23] == 0.0 and row[18] == np.float32(0.3)
        np.testing.assert_allclose(row[28], np.linalg.norm(v[vb].astype(np.float64) - v[va]), rtol=1e-12)
        # the triangle faces the camera: its normal is -forward or +forward, unit length
        np.testing.assert_allclose(abs(row[8]), 1.0, rtol=1e-12)
        assert (row[29:] == 0).all()


def test_features_are_invariant_to_a_rigid_motion_of_scene_and_camera():
    cfg = sg.soup(seed=1, n_tris=20, width=40, height=30, spp=1)
    scene, cam = cfg.scene, cfg.camera
    X0 = _features(scene, cam)
    ang = 0.7
    Rm = np.array([[math.cos(ang), 0, math.sin(ang)], [0, 1, 0], [-math.sin(ang), 0, math.cos(ang)]])
    Rm = Rm @ np.array([[1, 0, 0], [0, math.cos(0.3), -math.sin(0.3)], [0, math.sin(0.3), math.cos(0.3)]])
    t = np.array([0.25, -0.5, 0.125])
    move = lambda p: (Rm @ np.asarray(p, np.float64)) + t
    # float64 positions through the same motion; float32 rounding of the moved
    # scene bounds the comparison
    v1 = np.array([move(p) for p in scene.vertices.astype(np.float64)], np.float32)
    s1 = sg.Scene(v1, scene.indices, scene.albedo, scene.emission, scene.normals, scene.emission_two_sided,
                  scene.background)
    c1 = sg.Camera(tuple(move(cam.position)), tuple(move(cam.look_at)), tuple(Rm @ np.asarray(cam.up, np.float64)),
                   cam.fov_y_deg, cam.width, cam.height, near_clip=cam.near_clip)
    X1 = _features(s1, c1)
    keep = [j for j in range(32) if not 12 <= j < 18]
    np.testing.assert_allclose(X1[:, keep], X0[:, keep], atol=2e-5)
    np.testing.assert_allclose(X1[:, 12:18], np.concatenate([v1[oracle.edges(scene)[:, 0]],
                                                             v1[oracle.edges(scene)[:, 1]]], 1), atol=0)
