"""Edge cases of the HIP path against the FP64 oracle (same harness as
test_gpu_parity): the depth-6 kernel instantiation (depths 4..6) and depth 2,
a one-triangle scene, a scene without emitters, one-pixel windows, sample
counts that do not divide the wave, an all-zero loss gradient, and the C
ABI's argument checks."""
import numpy as np
import pytest

from paper_1904_12228_amd import scenegen as sg

from .test_gpu_parity import _run

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("depth", [2, 4, 5])
def test_sphere_box_other_depths(depth):
    cfg = sg.sphere_box(seed=1, level=2, width=48, height=48, spp=2, max_depth=depth)
    cam = cfg.camera.with_window(8, 10, 39, 35)
    _run(cfg.scene, cam, 2, depth, 3)


def test_single_emissive_triangle():
    v = np.array([[-0.6, -0.4, 2.5], [0.7, -0.5, 3.0], [0.1, 0.6, 2.2]], np.float32)
    scene = sg.Scene(v, np.array([[0, 1, 2]], np.int32), np.float32([0.0]), np.float32([0.8]), None, True, 0.2)
    cam = sg.Camera((0, 0, 0), (0, 0, 1), (0, 1, 0), 60.0, 40, 32)
    res, orc = _run(scene, cam, 4, 0, 1)
    assert np.abs(orc["d_vertices"]).max() > 0


def test_scene_without_emitters_lit_only_by_background():
    cfg = sg.soup(seed=3, n_tris=20, width=48, height=48, spp=2)
    s = cfg.scene
    scene = sg.Scene(s.vertices, s.indices, s.albedo, np.zeros_like(s.emission), None, False, 0.3)
    cam = cfg.camera.with_window(6, 6, 40, 38)
    res, orc = _run(scene, cam, 2, 2, 4)
    # light comes only from escaping camera rays: each pixel is the background
    # times the fraction of its 2 samples that escape
    img = orc["image"]
    np.testing.assert_allclose(np.round(img / 0.15) * 0.15, img, atol=1e-9)


@pytest.mark.parametrize("win,spp", [((31, 17, 32, 18), 1), ((20, 30, 21, 33), 5), ((0, 0, 64, 1), 7)])
def test_tiny_and_ragged_windows(win, spp):
    cfg = sg.config1()
    _run(cfg.scene, cfg.camera.with_window(*win), spp, 0, 9)


def test_zero_loss_gradient_gives_exactly_zero():
    from paper_1904_12228_amd import api
    cfg = sg.sphere_box(seed=1, level=2, width=32, height=32, spp=2, max_depth=3)
    S = api.Scene(cfg.scene)
    S.render(cfg.camera, 2, 3, seed=1)
    dv, da, dc = S.render_backward(cfg.camera, 2, 3, torch.zeros((32, 32), device="cuda"), seed=1)
    torch.cuda.synchronize()
    assert float(dv.abs().max()) == 0.0 and float(da.abs().max()) == 0.0 and float(dc.abs().max()) == 0.0
    S.close()


def test_invalid_arguments_are_rejected():
    from paper_1904_12228_amd import _lib, api
    cfg = sg.config1()
    S = api.Scene(cfg.scene)
    cam = cfg.camera
    for bad in (cam.with_window(0, 0, cam.width + 1, 4), cam.with_window(5, 5, 5, 9)):
        with pytest.raises(_lib.DiffrtError):
            S.render(bad, 4, 0)
    with pytest.raises(_lib.DiffrtError):
        S.render(cam, 0, 0)
    with pytest.raises(_lib.DiffrtError):
        S.render(cam, 4, 7)
    with pytest.raises(_lib.DiffrtError):
        S.render_backward(cam, 4, 0, torch.zeros((cam.height, cam.width), device="cuda"), edge_mix=1.0,
                          edge_pdf=torch.full((S.num_edges,), 1.0 / S.num_edges, device="cuda"))
    S.close()
    # a non-finite vertex coordinate
    cfg2 = sg.soup(seed=3, n_tris=20, width=32, height=32, spp=2)
    bad = cfg2.scene.copy()
    bad.vertices[5, 1] = np.nan
    with pytest.raises(_lib.DiffrtError):
        api.Scene(bad)
    # a triangle repeating a vertex, and an edge shared by three triangles
    v = np.array([[0, 0, 1], [1, 0, 1], [0, 1, 1], [1, 1, 1], [0.5, 0.5, 2]], np.float32)
    for idx in ([[0, 1, 1]], [[0, 1, 2], [0, 1, 3], [0, 1, 4]]):
        scene = sg.Scene(v, np.array(idx, np.int32), np.full(len(idx), 0.5, np.float32),
                         np.zeros(len(idx), np.float32))
        with pytest.raises(_lib.DiffrtError):
            api.Scene(scene)
    # a triangle of zero area (three collinear vertices)
    v = np.array([[0, 0, 1], [1, 0, 1], [2, 0, 1], [0, 1, 1]], np.float32)
    scene = sg.Scene(v, np.array([[0, 1, 3], [0, 1, 2]], np.int32), np.full(2, 0.5, np.float32), np.zeros(2, np.float32))
    with pytest.raises(_lib.DiffrtError, match="degenerate"):
        api.Scene(scene)


def test_sah_and_morton_bvh_give_the_same_results(monkeypatch):
    # the BVH only decides which triangles are tested; closest hits, images
    # and gradients do not depend on it (up to the order of atomic additions)
    from paper_1904_12228_amd import api
    cfg = sg.sphere_box(seed=1, level=3, width=48, height=48, spp=2, max_depth=3)
    d = torch.as_tensor(np.random.default_rng(9).normal(size=(48, 48)), dtype=torch.float32, device="cuda")
    res = []
    for kind in ("sah", "lbvh"):
        monkeypatch.setenv("DIFFRT_BVH", kind)
        S = api.Scene(cfg.scene)
        img = S.render(cfg.camera, 2, 3, seed=4)
        g = S.render_backward(cfg.camera, 2, 3, d, seed=4)
        res.append([img.cpu().numpy()] + [t.cpu().numpy() for t in g])
        assert not S.device_error()
        S.close()
    torch.cuda.synchronize()
    np.testing.assert_allclose(res[0][0], res[1][0], rtol=1e-6, atol=1e-7)
    for a, b in zip(res[0][1:], res[1][1:]):
        np.testing.assert_allclose(a, b, rtol=1e-4, atol=1e-5 * np.abs(b).max())


@pytest.mark.parametrize("depth,masked", [(2, False), (3, False), (3, True)])
def test_wavefront_forward_matches_the_single_kernel(monkeypatch, depth, masked):
    """The wavefront forward (camera hits, then one compacted queue per
    bounce) against the single-kernel forward: bit-identical images, and the
    checkpoints they leave give the same gradients."""
    from paper_1904_12228_amd import api
    cfg = sg.sphere_box(seed=2, level=3, width=64, height=48, spp=4, max_depth=3)
    cam = cfg.camera.with_window(3, 5, 61, 44)
    x0, y0, x1, y1 = cam.win()
    M = (x1 - x0) * (y1 - y0) * 4
    mask = None
    if masked:
        mask = torch.as_tensor((np.random.default_rng(1).uniform(size=M) < 0.7).astype(np.uint8), device="cuda")
    dimg = torch.as_tensor(np.random.default_rng(3).normal(size=(y1 - y0, x1 - x0)), dtype=torch.float32, device="cuda")
    out = {}
    for wf in ("1", "0"):
        monkeypatch.setenv("DIFFRT_WAVEFRONT_FORWARD", wf)
        print(f"case: wavefront={wf} depth={depth} masked={masked}", flush=True)
        S = api.Scene(cfg.scene)
        img = S.render(cam, 4, depth, seed=7, unit_mask=mask)
        dv, da, dc = S.render_backward(cam, 4, depth, dimg, seed=7, unit_mask=mask)
        torch.cuda.synchronize()
        assert not S.device_error()
        out[wf] = [t.cpu().numpy() for t in (img, dv, da, dc)]
        S.close()
    assert np.array_equal(out["1"][0], out["0"][0])
    for a, b in zip(out["1"][1:], out["0"][1:]):
        np.testing.assert_allclose(a, b, rtol=1e-5, atol=1e-6 * max(np.abs(b).max(), 1e-30))
