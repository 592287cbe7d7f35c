"""Pins of the clamped-cosine edge-point sampler (Ch. 5, Importance sampling
on an edge: for a Lambertian surface the lobe integrated along the edge is the
clamped cosine) and of the estimator that uses it.

* The density in the edge parameter t is proportional to max(n . w^, 0) times
  the arc-length Jacobian |e x w^| / |w| (computed here independently), and
  integrates to 1 (quadrature): this pins the closed-form normaliser.
* Samples follow the density: chi-square of 10^5 draws against bin
  probabilities integrated by quadrature, for edges wholly above the tangent
  plane, crossing it, seen at grazing angles and nearly end-on.
* The secondary-edge estimator with cosine-sampled points has the same
  expectation as with uniform points (gradients and the harvest statistic),
  on a direct-lighting soup and a depth-3 sphere in a box.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1904_12228_amd import scenegen as sg


def _geom_weight(p, n, v0, v1, t):
    e = v1 - v0
    w = v0 + e * t - p
    wl = np.linalg.norm(w)
    wh = w / wl
    return max(float(n @ wh), 0.0) * np.linalg.norm(np.cross(e, wh)) / wl


CASES = [
    # p, n, v0, v1
    (np.zeros(3), np.array([0, 1.0, 0]), np.array([-1, 0.5, 0.3]), np.array([1.2, 0.2, 0.4])),     # above
    (np.zeros(3), np.array([0, 1.0, 0]), np.array([-1, -0.4, 0.3]), np.array([1.0, 0.6, 0.2])),    # crosses the plane
    (np.array([0.1, 0, 0]), np.array([0, 0, 1.0]), np.array([0.3, -2, 0.05]), np.array([0.2, 2, 0.02])),  # grazing
    (np.zeros(3), np.array([0.3, 0.9, 0.1]) / np.linalg.norm([0.3, 0.9, 0.1]),
     np.array([0.02, 0.01, 0.03]), np.array([-0.5, 1.4, 0.2])),                                       # near one end
    (np.zeros(3), np.array([0, 1.0, 0]), np.array([0.5, 1.0, 1.0]), np.array([0.5005, 1.001, 1.0005])),  # nearly end-on
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_density_is_the_normalised_clamped_cosine_in_arc_length(case):
    p, n, v0, v1 = CASES[case]
    ts = np.linspace(0, 1, 20001)
    pdf = np.array([oracle.edge_t_cosine_pdf(p, n, v0, v1, t) for t in ts])
    g = np.array([_geom_weight(p, n, v0, v1, t) for t in ts])
    assert abs(np.trapezoid(pdf, ts) - 1.0) < 2e-4
    ratio = pdf[g > 1e-3 * g.max()] / g[g > 1e-3 * g.max()]
    assert ratio.std() <= 1e-10 * ratio.mean()
    assert (pdf[g == 0] == 0).all()


@pytest.mark.parametrize("case", range(len(CASES)))
def test_samples_follow_the_density(case):
    p, n, v0, v1 = CASES[case]
    u = np.random.default_rng(100 + case).uniform(size=100000)
    t, pt = oracle.edge_t_cosine(p, n, v0, v1, u)
    assert (t >= 0).all() and (t <= 1).all()
    np.testing.assert_allclose(pt, [oracle.edge_t_cosine_pdf(p, n, v0, v1, x) for x in t[:200]] + list(pt[200:]))
    bins = 40
    edges = np.linspace(0, 1, bins + 1)
    probs = []
    for a, b in zip(edges[:-1], edges[1:]):
        ts = np.linspace(a, b, 401)
        probs.append(np.trapezoid([oracle.edge_t_cosine_pdf(p, n, v0, v1, x) for x in ts], ts))
    probs = np.array(probs)
    h, _ = np.histogram(t, bins=edges)
    exp = probs * t.size
    keep = exp > 5
    chi2 = float((((h - exp) ** 2)[keep] / exp[keep]).sum())
    dof = int(keep.sum()) - 1
    # 0.999 quantile of chi-square with dof <= 39 degrees of freedom is below 73
    assert chi2 < 73, (chi2, dof)
    assert h[~keep].sum() <= 5 * max(exp[~keep].sum(), 1.0)


def _agree(scene, cam, spp, depth, K, seed0=0):
    x0, y0, x1, y1 = cam.win()
    dimg = np.random.default_rng(2).normal(size=(y1 - y0, x1 - x0)) + 0.5
    res = {}
    for mode in (0, 1):
        gs, hs = [], []
        for k in range(K):
            r = oracle.render(scene, cam, spp, depth, seed0 + k, d_image=dimg, interior=False, primary=False,
                              threads=8, edge_t=mode, edge_stats=True)
            gs.append(r["d_vertices"].ravel())
            hs.append(r["edge_stats"])
        res[mode] = (np.array(gs), np.array(hs))
    for which in (0, 1):
        a, b = res[0][which], res[1][which]
        ma, mb = a.mean(0), b.mean(0)
        se = np.sqrt(a.var(0, ddof=1) / K + b.var(0, ddof=1) / K)
        big = np.abs(ma) > 0.05 * np.abs(ma).max()
        z = np.abs(ma - mb)[big] / np.maximum(se[big], 1e-300)
        assert (z <= 5).all(), (which, np.sort(z)[-5:])
        assert big.sum() >= 5
    return res


@pytest.mark.slow
def test_cosine_points_leave_the_expectation_unchanged_direct_lighting():
    cfg = sg.soup(seed=3, n_tris=12, width=64, height=64, spp=2)
    cam = cfg.camera.with_window(20, 22, 44, 42)
    _agree(cfg.scene, cam, 16, 1, 40)


@pytest.mark.slow
def test_cosine_points_leave_the_expectation_unchanged_path_tracing():
    cfg = sg.sphere_box(seed=1, level=2, width=48, height=48, spp=2, max_depth=3)
    cam = cfg.camera.with_window(14, 16, 34, 32)
    _agree(cfg.scene, cam, 8, 3, 40)
