"""Geometry buffers (position, shading normal, albedo at the first camera hit;
thesis Ch. 5, Results: G-buffers) on the HIP path against the FP64 oracle,
element by element, with the harness and tolerance of test_gpu_parity:
every channel on a triangle soup, the normal channels on a smooth-normal
sphere, the two-triangle scene, a window across the 81,936-triangle sphere's
silhouette, and the argument checks."""
import numpy as np
import pytest

from paper_1904_12228_amd import scenegen as sg

from .test_gpu_parity import _run

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("aov", [1, 2, 3, 4, 5, 6, 7])
def test_soup_every_channel(aov):
    cfg = sg.soup(seed=3, n_tris=40, width=96, height=80, spp=2)
    cam = cfg.camera.with_window(20, 15, 67, 52)
    res, orc = _run(cfg.scene, cam, 2, 1, 5, aov=aov)
    assert np.abs(orc["d_vertices"]).max() > 0


@pytest.mark.parametrize("aov", [4, 5, 6])
def test_smooth_sphere_normals(aov):
    cfg = sg.sphere_box(seed=1, level=3, width=64, height=64, spp=2, max_depth=3)
    cam = cfg.camera.with_window(6, 10, 49, 41)
    _run(cfg.scene, cam, 3, 3, 2, aov=aov)


@pytest.mark.parametrize("aov,spp", [(7, 4), (3, 1)])
def test_two_triangles(aov, spp):
    cfg = sg.config1()
    s = cfg.scene
    # albedos of their own (the scene's triangles are black emitters)
    scene = sg.Scene(s.vertices, s.indices, np.float32([0.3, 0.8]), s.emission, None, False, s.background)
    res, orc = _run(scene, cfg.camera.with_window(5, 9, 58, 46), spp, 0, 7, aov=aov)
    assert np.abs(orc["d_vertices"]).max() > 0


@pytest.mark.parametrize("aov", [1, 6])
def test_config3_silhouette_window(aov):
    cfg = sg.config3()
    _run(cfg.scene, cfg.camera.with_window(440, 230, 471, 255), 2, 3, 0, aov=aov)


def test_max_depth_does_not_change_a_geometry_buffer():
    from paper_1904_12228_amd import api
    cfg = sg.sphere_box(seed=1, level=2, width=48, height=48, spp=2, max_depth=3)
    S = api.Scene(cfg.scene)
    d = torch.as_tensor(np.random.default_rng(1).normal(size=(48, 48)), dtype=torch.float32, device="cuda")
    out = []
    for depth in (0, 3):
        img = S.render(cfg.camera, 2, depth, seed=4, aov=5)
        g = S.render_backward(cfg.camera, 2, depth, d, seed=4, aov=5)
        out.append([img.cpu().numpy()] + [t.cpu().numpy() for t in g])
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out[0][0], out[1][0])
    for a, b in zip(out[0][1:], out[1][1:]):
        np.testing.assert_allclose(a, b, rtol=1e-4, atol=1e-5 * np.abs(b).max())
    S.close()


@pytest.mark.parametrize("spp", [2, 3])
def test_all_channels_in_one_pass_equal_the_single_channel_passes(spp):
    # spp = 3 does not divide the wave: the image is accumulated with atomics
    from paper_1904_12228_amd import api
    cfg = sg.sphere_box(seed=1, level=3, width=64, height=64, spp=2, max_depth=3)
    cam = cfg.camera.with_window(3, 5, 61, 50)
    H, W = 45, 58
    S = api.Scene(cfg.scene)
    d = torch.as_tensor(np.random.default_rng(4).normal(size=(7, H, W)), dtype=torch.float32, device="cuda")
    allc = S.render(cam, spp, 0, seed=8, aov=8).cpu().numpy()
    g_all = [t.cpu().numpy() for t in S.render_backward(cam, spp, 0, d, seed=8, aov=8)]
    one = []
    g_sum = None
    for ch in range(1, 8):
        one.append(S.render(cam, spp, 0, seed=8, aov=ch).cpu().numpy())
        g = [t.double() for t in S.render_backward(cam, spp, 0, d[ch - 1].contiguous(), seed=8, aov=ch)]
        g_sum = g if g_sum is None else [a + b for a, b in zip(g_sum, g)]
    torch.cuda.synchronize()
    assert not S.device_error()
    if spp == 2:
        np.testing.assert_array_equal(allc, np.stack(one))
    else:
        np.testing.assert_allclose(allc, np.stack(one), rtol=1e-6, atol=1e-6)
    for name, a, b in zip(("d_vertices", "d_albedo", "d_camera"), g_all, g_sum):
        b = b.cpu().numpy()
        np.testing.assert_allclose(a, b, rtol=1e-4, atol=1e-5 * np.abs(b).max(), err_msg=name)
    S.close()


def test_all_channel_backward_recomputes_its_own_forward_pass():
    # no matching forward pass before the backward: the library re-renders all
    # seven channels into a buffer of its own
    from paper_1904_12228_amd import api
    cfg = sg.soup(seed=3, n_tris=40, width=96, height=80, spp=2)
    cam = cfg.camera.with_window(20, 15, 67, 52)
    d = torch.as_tensor(np.random.default_rng(6).normal(size=(7, 37, 47)), dtype=torch.float32, device="cuda")
    S = api.Scene(cfg.scene)
    cold = [t.cpu().numpy() for t in S.render_backward(cam, 2, 0, d, seed=5, aov=8)]
    S.render(cam, 2, 0, seed=5, aov=8)
    warm = [t.cpu().numpy() for t in S.render_backward(cam, 2, 0, d, seed=5, aov=8)]
    torch.cuda.synchronize()
    assert not S.device_error()
    for a, b in zip(cold, warm):
        np.testing.assert_allclose(a, b, rtol=1e-4, atol=1e-5 * np.abs(b).max())
    S.close()


def test_deferred_shading_of_a_channel_subset():
    from paper_1904_12228_amd import api
    from paper_1904_12228_amd.autograd import gbuffer
    cfg = sg.soup(seed=3, n_tris=40, width=96, height=80, spp=2)
    cam = cfg.camera.with_window(20, 15, 67, 52)
    S = api.Scene(cfg.scene)
    v = S.vertices.clone().requires_grad_(True)
    c9 = torch.as_tensor(cam.params9(), device="cuda").requires_grad_(True)
    w = torch.as_tensor(np.random.default_rng(2).normal(size=(3, 37, 47)), dtype=torch.float32, device="cuda")
    out = gbuffer(S, v, c9, cam, 2, 3, channels=(7, 4, 1))
    (out * w).sum().backward()
    full = torch.zeros((7, 37, 47), device="cuda")
    full[6], full[3], full[0] = w[0], w[1], w[2]
    dv, _, dc = S.render_backward(cam, 2, 0, full, seed=3, aov=8)
    ref = S.render(cam, 2, 0, seed=3, aov=8)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.detach().cpu().numpy(), ref[[6, 3, 0]].cpu().numpy())
    np.testing.assert_allclose(v.grad.cpu().numpy(), dv.cpu().numpy(), rtol=1e-4, atol=1e-5 * float(dv.abs().max()))
    np.testing.assert_allclose(c9.grad.cpu().numpy(), dc.cpu().numpy(), rtol=1e-4, atol=1e-5 * float(dc.abs().max()))
    S.close()


def test_invalid_geometry_buffer_arguments_are_rejected():
    from paper_1904_12228_amd import _lib, api
    cfg = sg.config1()
    S = api.Scene(cfg.scene)
    cam = cfg.camera
    d = torch.zeros((cam.height, cam.width), device="cuda")
    for bad in (-1, 9):
        with pytest.raises(_lib.DiffrtError):
            S.render(cam, 4, 0, out=torch.empty((cam.height, cam.width), device="cuda"), aov=bad)
    with pytest.raises(_lib.DiffrtError):
        S.render_backward(cam, 4, 0, d, aov=1, edge_pdf=torch.full((S.num_edges,), 1.0 / S.num_edges, device="cuda"),
                          edge_mix=0.5)
    with pytest.raises(_lib.DiffrtError):
        S.render_backward(cam, 4, 0, d, aov=7, edge_stats=torch.zeros(S.num_edges, device="cuda"))
    S.close()


def _shade(G, w):
    # a smooth deferred-shading function of the buffers: half-Lambert lighting
    # from a point light with distance falloff, times albedo
    p, n, a = G[0:3], G[3:6], G[6]
    light = torch.tensor([0.3, 0.9, -0.4], dtype=G.dtype, device=G.device)[:, None, None]
    d = light - p
    r2 = (d * d).sum(0)
    cos = (n * d).sum(0) / torch.sqrt(r2 + 1e-6)
    return (w * a * (0.6 + 0.4 * cos) / (1.0 + 0.2 * r2)).sum()


@pytest.mark.parametrize("which", ["soup", "sphere"])
def test_deferred_shading_through_the_buffers_matches_the_oracle(which):
    import oracle
    from paper_1904_12228_amd import api
    from paper_1904_12228_amd.autograd import gbuffer
    from .gpu_common import compare
    if which == "soup":
        cfg = sg.soup(seed=3, n_tris=40, width=96, height=80, spp=2)
        cam = cfg.camera.with_window(20, 15, 67, 52)
    else:
        cfg = sg.sphere_box(seed=1, level=3, width=64, height=64, spp=2, max_depth=3)
        cam = cfg.camera.with_window(6, 10, 49, 41)
    s = cfg.scene
    alb = np.random.default_rng(5).uniform(0.2, 0.9, s.num_triangles).astype(np.float32)
    scene = sg.Scene(s.vertices, s.indices, alb, s.emission, s.normals, s.emission_two_sided, s.background)
    spp, seed = 2, 6
    x0, y0, x1, y1 = cam.win()
    print(f"deferred shading: {which} win={cam.win()}", flush=True)
    # units near a tie for any channel are left out on both sides
    mask = np.ones((y1 - y0) * (x1 - x0) * spp, np.uint8)
    zero = np.zeros((y1 - y0, x1 - x0))
    for ch in range(1, 8):
        r = oracle.render(scene, cam, spp, 0, seed, d_image=zero, want_flags=True, exclude_flagged=True, aov=ch)
        mask &= (1 - r["unit_flags"]).astype(np.uint8)
    assert mask.sum() > 0.9 * mask.size
    G = np.stack([oracle.render(scene, cam, spp, 0, seed, unit_mask=mask, aov=ch)["image"] for ch in range(1, 8)])
    w = np.random.default_rng(8).normal(size=zero.shape) + 0.5
    Gt = torch.tensor(G, dtype=torch.float64, requires_grad=True)
    _shade(Gt, torch.tensor(w)).backward()
    dG = Gt.grad.numpy()
    ref = {"d_vertices": 0, "d_camera": 0, "d_albedo": 0, "mass_vertices": 0, "mass_camera": 0, "mass_albedo": 0}
    for ch in range(1, 8):
        r = oracle.render(scene, cam, spp, 0, seed, d_image=dG[ch - 1], unit_mask=mask, aov=ch)
        for k in ref:
            ref[k] = ref[k] + r[k]
    S = api.Scene(scene)
    v = S.vertices.clone().requires_grad_(True)
    c9 = torch.as_tensor(cam.params9(), device="cuda").requires_grad_(True)
    a = torch.as_tensor(alb, device="cuda").requires_grad_(True)
    out = gbuffer(S, v, c9, cam, spp, seed, albedo=a, unit_mask=torch.as_tensor(mask, device="cuda"))
    _shade(out, torch.as_tensor(w, dtype=torch.float32, device="cuda")).backward()
    torch.cuda.synchronize()
    assert not S.device_error()
    for ch in range(7):
        compare(f"buffer {ch + 1}", out[ch].detach().cpu().numpy(), G[ch])
    compare("d_vertices", v.grad.cpu().numpy(), ref["d_vertices"], ref["mass_vertices"])
    compare("d_camera", c9.grad.cpu().numpy(), ref["d_camera"], ref["mass_camera"])
    compare("d_albedo", a.grad.cpu().numpy(), ref["d_albedo"], ref["mass_albedo"])
    assert np.abs(ref["d_vertices"]).max() > 0 and np.abs(ref["d_albedo"]).max() > 0
    S.close()


def test_albedo_update_equals_a_scene_created_with_those_albedos():
    from paper_1904_12228_amd import api
    cfg = sg.sphere_box(seed=1, level=2, width=48, height=48, spp=2, max_depth=3)
    s = cfg.scene
    alb = np.random.default_rng(2).uniform(0.1, 0.9, s.num_triangles).astype(np.float32)
    alb[s.emission > 0] = 0.0
    other = sg.Scene(s.vertices, s.indices, alb, s.emission, s.normals, s.emission_two_sided, s.background)
    d = torch.as_tensor(np.random.default_rng(3).normal(size=(48, 48)), dtype=torch.float32, device="cuda")
    A, B = api.Scene(s), api.Scene(other)
    A.update_albedo(alb)
    res = []
    for S in (A, B):
        img = S.render(cfg.camera, 2, 3, seed=9)
        g = S.render_backward(cfg.camera, 2, 3, d, seed=9)
        res.append([img.cpu().numpy()] + [t.cpu().numpy() for t in g])
    torch.cuda.synchronize()
    np.testing.assert_array_equal(res[0][0], res[1][0])
    for x, y in zip(res[0][1:], res[1][1:]):
        np.testing.assert_allclose(x, y, rtol=1e-4, atol=1e-5 * np.abs(y).max())
    A.close()
    B.close()
