"""HIP path vs FP64 oracle at the benchmark configurations' own sizes and
sample counts, and through the batched and autograd entry points.

* config 2 in full: 256x256 pixels, 16 spp, depth 1, 1,004 triangles;
* config 3 on a 64x64 crop at its 64 spp, depth 3, 81,936 triangles;
* a batch of three views (uneven windows and sample counts) rendered and
  differentiated in one launch per pass, each view against the oracle;
* the torch.autograd.Function (vertices, albedo, camera) against the oracle.

Units whose discrete decisions lie within rounding of a tie are masked on
both sides (unit masks), as in test_gpu_parity; the rest must agree to the
tolerance of gpu_common.
"""
import numpy as np
import pytest

from paper_1904_12228_amd import scenegen as sg

from .gpu_common import compare, oracle_reference

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

THREADS = 16


def _dimg(cam, seed):
    x0, y0, x1, y1 = cam.win()
    return np.random.default_rng(seed).normal(size=(y1 - y0, x1 - x0)) + 0.5


def _check(case, res, orc):
    compare("image", res["img"], orc["image"], case=case)
    compare("d_vertices", res["dv"], orc["d_vertices"], orc["mass_vertices"], case=case)
    compare("d_albedo", res["da"], orc["d_albedo"], orc["mass_albedo"], case=case)
    compare("d_camera", res["dc"], orc["d_camera"], orc["mass_camera"], case=case)


def _single(scene, cam, spp, depth, seed, name):
    from paper_1904_12228_amd import api
    dimg = _dimg(cam, 1)
    print(f"case {name}: win={cam.win()} spp={spp} depth={depth}", flush=True)
    orc = oracle_reference(scene, cam, spp, depth, seed, dimg, threads=THREADS)
    M = dimg.size * spp
    flagged = int(orc["stats"][1])
    print(f"  oracle done, near-tie units {flagged}/{M}", flush=True)
    assert flagged <= 0.05 * M
    mask = torch.as_tensor(orc["mask"], device="cuda")
    S = api.Scene(scene)
    img = S.render(cam, spp, depth, seed, unit_mask=mask)
    dv, da, dc = S.render_backward(cam, spp, depth, torch.as_tensor(dimg, dtype=torch.float32, device="cuda"),
                                   seed=seed, unit_mask=mask)
    torch.cuda.synchronize()
    assert not S.device_error()
    res = dict(img=img.cpu().numpy(), dv=dv.cpu().numpy(), da=da.cpu().numpy(), dc=dc.cpu().numpy())
    S.close()
    _check(f"{name} flagged={flagged}/{M}", res, orc)


def test_config2_full_image():
    cfg = sg.config2()
    _single(cfg.scene, cfg.camera, cfg.spp, cfg.max_depth, 0, "config2 256x256 16spp")


def test_config3_crop_at_64_spp():
    """A 64x64 crop across the displaced sphere's silhouette and the box
    behind it, at the benchmark's 64 samples per pixel and depth 3."""
    cfg = sg.config3()
    cam = cfg.camera.with_window(300, 200, 364, 264)
    _single(cfg.scene, cam, cfg.spp, cfg.max_depth, 0, "config3 64x64 crop 64spp")


@pytest.mark.parametrize("which", ["soup", "sphere"])
def test_batch_views_match_oracle(which):
    """drBatchForward / drBatchBackward (one launch per pass for all views)
    against the oracle view by view: images and camera gradients per view,
    vertex and albedo gradients summed over the views."""
    from paper_1904_12228_amd import api, batch
    if which == "soup":
        cfg, depth = sg.soup(seed=3, n_tris=40, width=64, height=64, spp=4), 1
    else:
        cfg, depth = sg.sphere_box(seed=1, level=3, width=64, height=64, spp=2, max_depth=3), 3
    cam = cfg.camera
    views = [(cam, 4), (cam.with_window(5, 9, 58, 46), 3),
             (sg.Camera((0.9, 1.0, -1.2), (0.5, 0.35, 0.5), (0.0, 1.0, 0.0), 50.0, 40, 32), 8)]
    if which == "sphere":
        views[2] = (sg.Camera((0.3, 0.2, -0.8), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 60.0, 40, 32), 8)
    seed = 7
    orcs, masks = [], []
    for i, (c, spp) in enumerate(views):
        print(f"case batch {which} view {i}: win={c.win()} spp={spp}", flush=True)
        o = oracle_reference(cfg.scene, c, spp, depth, seed, _dimg(c, 10 + i), threads=THREADS, view_id=i)
        orcs.append(o)
        masks.append(torch.as_tensor(o["mask"], device="cuda"))
    S = api.Scene(cfg.scene)
    B = batch.Batch(S, views, depth, seed=seed, unit_masks=masks)
    for i, (c, _) in enumerate(views):
        B.d_images[i].copy_(torch.as_tensor(_dimg(c, 10 + i)))
    dv = torch.empty((S.num_vertices, 3), dtype=torch.float32, device="cuda")
    da = torch.empty((S.num_triangles,), dtype=torch.float32, device="cuda")
    dcs = torch.empty((len(views), 9), dtype=torch.float32, device="cuda")
    B.forward()
    B.backward(dv, da, dcs)
    torch.cuda.synchronize()
    case = f"batch {which} ({len(views)} views)"
    for i, o in enumerate(orcs):
        compare(f"image {i}", B.images[i].cpu().numpy(), o["image"], case=case)
        compare(f"d_camera {i}", dcs[i].cpu().numpy(), o["d_camera"], o["mass_camera"], case=case)
    compare("d_vertices", dv.cpu().numpy(), sum(o["d_vertices"] for o in orcs),
            sum(o["mass_vertices"] for o in orcs), case=case)
    compare("d_albedo", da.cpu().numpy(), sum(o["d_albedo"] for o in orcs), sum(o["mass_albedo"] for o in orcs),
            case=case)
    B.close()
    S.close()


def test_autograd_function_matches_oracle():
    """autograd.render: image, and the gradients that torch's backward hands
    to the vertex, albedo and camera tensors, against the oracle."""
    from paper_1904_12228_amd import api
    from paper_1904_12228_amd.autograd import render
    cfg = sg.soup(seed=2, n_tris=30, width=48, height=40, spp=2)
    cam, spp, depth, seed = cfg.camera, 3, 1, 3
    dimg = _dimg(cam, 4)
    print("case autograd soup 48x40", flush=True)
    orc = oracle_reference(cfg.scene, cam, spp, depth, seed, dimg, threads=THREADS)
    mask = torch.as_tensor(orc["mask"], device="cuda")
    S = api.Scene(cfg.scene)
    v = S.vertices.clone().requires_grad_(True)
    alb = torch.as_tensor(cfg.scene.albedo, dtype=torch.float32, device="cuda").clone().requires_grad_(True)
    c9 = torch.as_tensor(cam.params9(), dtype=torch.float32, device="cuda").requires_grad_(True)
    img = render(S, v, c9, cam, spp, depth, seed=seed, albedo=alb, unit_mask=mask)
    (img * torch.as_tensor(dimg, dtype=torch.float32, device="cuda")).sum().backward()
    torch.cuda.synchronize()
    res = dict(img=img.detach().cpu().numpy(), dv=v.grad.cpu().numpy(), da=alb.grad.cpu().numpy(),
               dc=c9.grad.cpu().numpy())
    S.close()
    _check("autograd soup", res, orc)
