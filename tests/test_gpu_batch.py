"""Batched multi-view rendering, refits, HIP-graph replay and the batched
inverse-rendering loop, on the GPU through the C ABI.

The batch runs the same per-unit code as the single-view entry points (whose
parity with the FP64 oracle is tested elsewhere), so its results must equal
the per-view results up to the order of FP32 atomic additions.
"""
import numpy as np
import pytest

from paper_1904_12228_amd import scenegen as sg

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _views(cfg):
    cam = cfg.camera
    return [(cam, 4), (cam.with_window(5, 9, 58, 46), 3),
            (sg.Camera((0.9, 1.0, -1.2), (0.5, 0.35, 0.5), (0.0, 1.0, 0.0), 50.0, 40, 32), 8)]


def _close(name, a, b, rel=1e-4, floor=1e-5):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    tol = rel * np.abs(b) + floor * max(np.abs(b).max(), 1e-30)
    bad = np.abs(a - b) > tol
    assert not bad.any(), (name, np.argwhere(bad)[:5], a[bad][:5], b[bad][:5])


def _single(S, views, depth, seed):
    imgs, dv = [], None
    for i, (cam, spp) in enumerate(views):
        x0, y0, x1, y1 = cam.win()
        img = S.render(cam, spp, depth, seed=seed, view_id=i)
        d = torch.as_tensor(np.random.default_rng(i).normal(size=(y1 - y0, x1 - x0)) + 0.5, dtype=torch.float32,
                            device="cuda")
        g, _, _ = S.render_backward(cam, spp, depth, d, seed=seed, view_id=i, want=("vertices",))
        imgs.append(img.cpu().numpy())
        dv = g.double() if dv is None else dv + g.double()
    return imgs, dv.cpu().numpy()


@pytest.mark.parametrize("which", ["soup", "sphere"])
def test_batch_equals_single_views_for_every_launch_shape(which):
    from paper_1904_12228_amd import api, batch
    if which == "soup":
        cfg, depth = sg.soup(seed=3, n_tris=40, width=64, height=64, spp=4), 1
    else:
        cfg, depth = sg.sphere_box(seed=1, level=3, width=64, height=64, spp=2, max_depth=3), 3
    views = _views(cfg)
    S = api.Scene(cfg.scene)
    ref_imgs, ref_dv = _single(S, views, depth, 7)
    B = batch.Batch(S, views, depth, seed=7)
    for i, (cam, spp) in enumerate(views):
        x0, y0, x1, y1 = cam.win()
        B.d_images[i].copy_(torch.as_tensor(np.random.default_rng(i).normal(size=(y1 - y0, x1 - x0)) + 0.5))
    dv = torch.empty((S.num_vertices, 3), dtype=torch.float32, device="cuda")
    for ctas, chunk in [(0, 1), (0, 4), (512, 2), (4096, 1)]:
        print(f"{which}: launch ctas={ctas} chunk={chunk}", flush=True)
        B.set_launch(ctas, chunk)
        B.forward()
        B.backward(dv)
        torch.cuda.synchronize()
        for i in range(len(views)):
            _close(f"image {i}", B.images[i].cpu().numpy(), ref_imgs[i], rel=1e-5, floor=1e-7)
        _close("d_vertices", dv.cpu().numpy(), ref_dv)
    B.close()
    S.close()


def test_refit_with_unchanged_vertices_changes_nothing():
    from paper_1904_12228_amd import api, batch
    cfg = sg.sphere_box(seed=1, level=3, width=64, height=64, spp=2, max_depth=3)
    views = _views(cfg)
    S = api.Scene(cfg.scene)
    B = batch.Batch(S, views, 3, seed=2)
    for d in B.d_images:
        d.fill_(1.0)
    dv0 = torch.empty((S.num_vertices, 3), dtype=torch.float32, device="cuda")
    dv1 = torch.empty_like(dv0)
    B.forward()
    B.backward(dv0)
    imgs0 = [t.clone() for t in B.images]
    batch.scene_refit(S, S.vertices.contiguous())
    B.refit()
    B.forward()
    B.backward(dv1)
    torch.cuda.synchronize()
    for a, b in zip(B.images, imgs0):
        _close("image", a.cpu().numpy(), b.cpu().numpy(), rel=1e-5, floor=1e-7)
    _close("d_vertices", dv1.cpu().numpy(), dv0.cpu().numpy())
    B.close()
    S.close()


def _inverse_setup(n_views=4, sigma=0.02, seed=0, spp=4, sizes=((64, 64), (48, 40))):
    from paper_1904_12228_amd import api, batch
    cfg = sg.soup(seed=3, n_tris=40, width=64, height=64, spp=4)
    views = [(c, spp) for c, _ in sg.orbit_views(11, n_views, sizes=sizes)]
    S = api.Scene(cfg.scene)
    true_v = S.vertices.clone()
    # targets: the true scene at 64 spp
    T = batch.Batch(S, [(c, 64) for c, _ in views], 1, seed=1000)
    T.forward()
    targets = [t.clone() for t in T.images]
    T.close()
    mask = torch.zeros(S.num_vertices, device="cuda")
    mask[:3 * 40] = 1.0                      # the soup's vertices; ground and light stay
    g = torch.Generator(device="cuda").manual_seed(seed)
    v0 = (true_v + sigma * torch.randn(true_v.shape, device="cuda", generator=g) * mask[:, None]).contiguous()
    B = batch.Batch(S, views, 1, seed=5)
    return S, B, true_v, v0, targets, mask


def test_graph_replays_match_eager_steps():
    from paper_1904_12228_amd import batch
    SA, BA, true_v, v0, targets, mask = _inverse_setup()
    SB, BB, _, _, _, _ = _inverse_setup()
    IA = batch.InverseRendering(BA, v0, targets, mask)
    IB = batch.InverseRendering(BB, v0, targets, mask)
    IA.capture()            # one eager warm-up step, then the recorded step
    IB.step()
    for k in range(4):
        IA.step()           # graph replay
        IB.step()           # eager
        torch.cuda.synchronize()
        _ = (IA.v - IB.v).abs().max().item()        # eager work between replays
        for a, b in zip(BA.images, BB.images):
            _close(f"replay {k} image", a.cpu().numpy(), b.cpu().numpy(), rel=1e-5, floor=1e-6)
        _close(f"replay {k} gradient", IA.grad.cpu().numpy(), IB.grad.cpu().numpy(), rel=1e-3, floor=1e-4)
        np.testing.assert_allclose(IA.v.cpu().numpy(), IB.v.cpu().numpy(), atol=1e-5)
    assert int(IA.step_count.item()) == 5 and int(IB.step_count.item()) == 5
    BA.close(); BB.close(); SA.close(); SB.close()


def test_batched_inverse_rendering_recovers_perturbed_vertices():
    from paper_1904_12228_amd import batch
    S, B, true_v, v0, targets, mask = _inverse_setup(n_views=8, spp=8, sizes=((96, 96),))
    inv = batch.InverseRendering(B, v0, targets, mask, lr=2e-3)
    err = lambda: float(((inv.v - true_v) ** 2 * mask[:, None]).sum().sqrt())
    e0 = err()
    inv.capture()
    for _ in range(200):
        inv.step()
    torch.cuda.synchronize()
    e1 = err()
    print(f"vertex error {e0:.4f} -> {e1:.4f}, image loss {inv.loss():.3e}", flush=True)
    assert e1 < 0.6 * e0
    B.close()
    S.close()


def test_refit_that_folds_coplanar_faces_rebuilds_the_hierarchy():
    """Lowering one corner of the ground quad folds its two coplanar faces
    (their shared diagonal was no discontinuity) into a crease. The refit must
    flag the batch, the check must rebuild the hierarchies, and the batch's
    gradient must then equal that of a batch built from scratch on a scene
    with the moved vertices. A refit that moves only soup triangles (whose
    edges are all boundary edges) flags nothing."""
    import copy

    from paper_1904_12228_amd import api, batch
    cfg = sg.soup(seed=3, n_tris=40, width=64, height=64, spp=4)
    views = _views(cfg)
    S = api.Scene(cfg.scene)
    B = batch.Batch(S, views, 1, seed=7)

    def grads(Bx):
        for i, (cam, spp) in enumerate(views):
            x0, y0, x1, y1 = cam.win()
            Bx.d_images[i].copy_(torch.as_tensor(np.random.default_rng(i).normal(size=(y1 - y0, x1 - x0)) + 0.5))
        dv = torch.empty((S.num_vertices, 3), dtype=torch.float32, device="cuda")
        Bx.forward()
        Bx.backward(dv)
        torch.cuda.synchronize()
        return [t.cpu().numpy() for t in Bx.images], dv.cpu().numpy()

    v = S.vertices.clone()
    v[:3 * 40] += 0.01                       # soup triangles only
    batch.scene_refit(S, v.contiguous())
    B.refit()
    assert not B.check_hierarchy()
    v[3 * 40 + 1, 1] -= 0.3                  # a ground corner off the diagonal down: the diagonal becomes a crease
    batch.scene_refit(S, v.contiguous())
    B.refit()
    assert B.check_hierarchy()
    assert not B.check_hierarchy()           # flag cleared by the rebuild
    imgs, dv = grads(B)
    moved = copy.deepcopy(cfg.scene)
    moved.vertices = v.cpu().numpy().astype(np.float32)
    S2 = api.Scene(moved)
    B2 = batch.Batch(S2, views, 1, seed=7)
    imgs2, dv2 = grads(B2)
    for i in range(len(views)):
        _close(f"image {i}", imgs[i], imgs2[i], rel=1e-5, floor=1e-7)
    _close("d_vertices", dv, dv2)
    B.close(); B2.close(); S.close(); S2.close()
