"""Learned edge proposal on the GPU vs the FP64 oracle, through the C ABI.

* edge features (drEdgeFeatures) vs oracle/mlp.edge_features;
* the network's forward (drMlpForward), per-view softmax cross-entropy
  (drMlpSoftmaxXent) and backward (drMlpBackward) vs oracle/mlp on seeded
  parameters and inputs (ragged row counts, uneven and empty views);
* drRenderBackward with the proposal mixture (a seeded distribution over
  edges, mix 0.8) and the harvest statistic vs the oracle's mixture.

Tolerances: 1e-4 relative plus a floor from FP32 rounding of the kernels'
sums (the oracle's absolute-value mass of each entry times a bound on the
relative error of its longest FP32 chain).
"""
import numpy as np
import pytest

import oracle
from oracle import mlp as omlp
from paper_1904_12228_amd import scenegen as sg

from .gpu_common import compare, oracle_reference

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

U32 = 2.0 ** -24


def _cams(cfg):
    base = cfg.camera
    other = sg.Camera((1.6, 1.1, -0.9), (0.45, 0.2, 0.5), (0.0, 1.0, 0.0), 50.0, 96, 80, near_clip=0.05)
    near = sg.Camera((0.5, 0.3, 0.2), (0.5, 0.3, 1.0), (0.0, 1.0, 0.0), 80.0, 64, 64, near_clip=0.01)
    return [base, other, near]


def test_edge_features_match_oracle():
    from paper_1904_12228_amd import api
    cfg = sg.config2()
    S = api.Scene(cfg.scene)
    edges = oracle.edges(cfg.scene)
    assert S.num_edges == len(edges)
    for cam in _cams(cfg):
        print(f"camera {cam.position} -> {cam.look_at}", flush=True)
        g = S.edge_features(cam).cpu().numpy().astype(np.float64)
        o = omlp.edge_features(cfg.scene, cam, edges)
        # FP32 evaluation of O(1) geometry; screen coordinates divide by depth
        # (clamped to the near plane), amplifying position rounding by up to
        # |x| / z
        depth = np.maximum(np.minimum(o[:, 2:3], o[:, 5:6]), cam.near_clip)
        tol = 1e-5 * (1.0 + np.abs(o))
        tol[:, 24:28] += 4e-6 * (1.0 + np.abs(o[:, 24:28])) * (1.0 + 1.0 / depth)
        bad = np.abs(g - o) > tol
        assert not bad.any(), (np.argwhere(bad)[:5], g[bad][:5], o[bad][:5])
    S.close()


def _net_case(seed, n):
    theta = sg.mlp_params(seed, bias_scale=0.1)
    X = sg.mlp_inputs(seed + 1, n)
    return theta, X


def _z_bound(cache, mz):
    """FP32 error bound of the kernels' logits: layer-1 sums (33 terms),
    layer-2 sums (3 split terms x 64 + bias), the 64-term output sum."""
    W2b, W3b = np.abs(cache["W2b"]), np.abs(cache["W3b"])
    on1, on2 = cache["a1"] > 0, cache["a2"] > 0
    e1 = 34 * U32 * cache["m1"] * on1
    e2 = (200 * U32 * cache["m2"] + e1 @ W2b) * on2
    return e2 @ W3b + 70 * U32 * mz


@pytest.mark.parametrize("n", [16, 1037, 20000])
def test_mlp_forward_matches_oracle(n):
    from paper_1904_12228_amd import proposal
    theta, X = _net_case(2, n)
    z = proposal.mlp_forward(torch.as_tensor(theta, device="cuda"), torch.as_tensor(X, device="cuda"))
    z = z.cpu().numpy().astype(np.float64)
    zo, mz, flag, cache = omlp.forward(theta, X)
    assert flag.mean() < 0.02
    ok = ~flag
    tol = 1e-4 * np.abs(zo) + 4 * _z_bound(cache, mz)
    err = np.abs(z - zo)
    bad = ok & (err > tol)
    assert not bad.any(), (np.nonzero(bad)[0][:5], z[bad][:5], zo[bad][:5], tol[bad][:5])


def test_softmax_cross_entropy_matches_oracle():
    from paper_1904_12228_amd import proposal
    rng = np.random.default_rng(3)
    sizes = [300, 0, 1, 1000, 57, 250]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
    n = int(off[-1])
    z = (rng.normal(size=n) * 3).astype(np.float32)
    t = np.abs(rng.normal(size=n)).astype(np.float32)
    t[off[4]:off[5]] = 0.0            # a view without target
    p, dz, vl = proposal.softmax_xent(torch.as_tensor(z, device="cuda"), torch.as_tensor(t, device="cuda"),
                                      torch.as_tensor(off, device="cuda"))
    po, lo, dzo = omlp.softmax_xent(z.astype(np.float64), t.astype(np.float64), list(off))
    p, dz, vl = (a.cpu().numpy().astype(np.float64) for a in (p, dz, vl))
    # exp of arguments up to ~20 in FP32: relative error ~ 20 u per term
    np.testing.assert_allclose(p, po, rtol=1e-5, atol=1e-12)
    np.testing.assert_allclose(dz, dzo, rtol=1e-4, atol=1e-6 * np.abs(dzo).max())
    used = [v for v in range(len(sizes)) if sizes[v] > 0 and t[off[v]:off[v + 1]].sum() > 0]
    assert abs(vl[used].mean() - lo) <= 1e-5 * abs(lo)
    assert (vl[[v for v in range(len(sizes)) if v not in used]] == 0).all()


@pytest.mark.parametrize("n", [1037, 40000])
def test_mlp_backward_matches_oracle(n):
    from paper_1904_12228_amd import proposal
    theta, X = _net_case(5, n)
    zo, mz, flag, cache = omlp.forward(theta, X)
    dz = np.random.default_rng(6).normal(size=n).astype(np.float32) / n
    dz[flag] = 0.0                    # rows whose ReLU decision FP32 may take the other way
    g = proposal.mlp_backward(torch.as_tensor(theta, device="cuda"), torch.as_tensor(X, device="cuda"),
                              torch.as_tensor(dz, device="cuda")).cpu().numpy().astype(np.float64)
    go, mass = omlp.backward(theta, cache, dz.astype(np.float64))
    # each gradient entry: a sum of n FP32-accurate products (three-term BF16
    # splits), accumulated in FP32 over at most n rows
    tol = 1e-4 * np.abs(go) + 4e-5 * mass
    bad = np.abs(g - go) > tol
    assert not bad.any(), (np.nonzero(bad)[0][:5], g[bad][:5], go[bad][:5], tol[bad][:5])


def _proposal_pdf(E, seed):
    rng = np.random.default_rng(seed)
    q = rng.gamma(0.5, size=E) + 1e-3
    return (q / q.sum()).astype(np.float32)


def _mixture_case(scene, cam, spp, depth, seed, mix_terms):
    from paper_1904_12228_amd import api
    x0, y0, x1, y1 = cam.win()
    dimg = np.random.default_rng(9).normal(size=(y1 - y0, x1 - x0)) + 0.5
    E = oracle.num_edges(scene)
    q = _proposal_pdf(E, seed)
    mix = np.float32(0.8)
    print(f"mixture case: T={scene.num_triangles} win={cam.win()} spp={spp} depth={depth} terms={mix_terms}", flush=True)
    orc = oracle_reference(scene, cam, spp, depth, seed, dimg, edge_pdf=q.astype(np.float64), mix=float(mix),
                           mix_terms=mix_terms, edge_stats=True)
    M = (x1 - x0) * (y1 - y0) * spp
    assert orc["stats"][1] <= 0.05 * M
    S = api.Scene(scene)
    mask = torch.as_tensor(orc["mask"], device="cuda")
    S.render(cam, spp, depth, seed, unit_mask=mask)
    stats = torch.empty(S.num_edges, dtype=torch.float32, device="cuda")
    dv, da, dc = S.render_backward(cam, spp, depth, torch.as_tensor(dimg, dtype=torch.float32, device="cuda"),
                                   seed=seed, unit_mask=mask, edge_pdf=torch.as_tensor(q, device="cuda"),
                                   edge_mix=float(mix), edge_mix_terms=(2 if mix_terms & 1 else 0) | (4 if mix_terms & 2 else 0),
                                   edge_stats=stats)
    torch.cuda.synchronize()
    assert not S.device_error()
    compare("d_vertices", dv.cpu().numpy(), orc["d_vertices"], orc["mass_vertices"])
    compare("d_albedo", da.cpu().numpy(), orc["d_albedo"], orc["mass_albedo"])
    compare("d_camera", dc.cpu().numpy(), orc["d_camera"], orc["mass_camera"])
    st = stats.cpu().numpy().astype(np.float64)
    so = orc["edge_stats"]
    # sums of P |c|^2: relative error twice that of the contributions
    compare("edge_stats", st, so, mass=2 * orc["edge_stats_mass"])
    assert (so > 0).sum() > 10
    S.close()
    return orc


@pytest.mark.parametrize("mix_terms", [1, 2, 3])
def test_mixture_soup_direct_lighting(mix_terms):
    cfg = sg.soup(seed=3, n_tris=40, width=64, height=64, spp=4)
    _mixture_case(cfg.scene, cfg.camera.with_window(16, 12, 52, 44), 4, 1, 21, mix_terms)


def test_mixture_config2_window():
    cfg = sg.config2()
    _mixture_case(cfg.scene, cfg.camera.with_window(100, 120, 141, 153), 4, 1, 5, 3)


def test_mixture_smooth_sphere_depth3():
    cfg = sg.sphere_box(seed=1, level=3, width=64, height=64, spp=2, max_depth=3)
    _mixture_case(cfg.scene, cfg.camera.with_window(14, 20, 44, 46), 2, 3, 8, 3)


def test_harvest_with_plain_sampler_matches_oracle():
    from paper_1904_12228_amd import api
    cfg = sg.soup(seed=3, n_tris=40, width=64, height=64, spp=4)
    cam = cfg.camera.with_window(10, 10, 50, 46)
    dimg = np.ones((36, 40))
    orc = oracle_reference(cfg.scene, cam, 4, 1, 2, dimg, edge_stats=True)
    S = api.Scene(cfg.scene)
    mask = torch.as_tensor(orc["mask"], device="cuda")
    S.render(cam, 4, 1, 2, unit_mask=mask)
    stats = torch.empty(S.num_edges, dtype=torch.float32, device="cuda")
    S.render_backward(cam, 4, 1, torch.ones((36, 40), device="cuda"), seed=2, unit_mask=mask, edge_stats=stats)
    compare("edge_stats", stats.cpu().numpy(), orc["edge_stats"], mass=2 * orc["edge_stats_mass"])
    S.close()
