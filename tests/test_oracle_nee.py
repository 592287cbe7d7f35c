"""Pins of next event estimation for edges (Ch. 5, Next event estimation for
edges) in the oracle.

The billboard strategy draws a light point y, widens every edge into a strip
of width w facing the shading point x, and picks one of the strips that the
segment x -> y crosses in proportion to the edge's importance. What fixes the
expected values, independently of the oracle's density code:

* the strategy's density p_N over strip coordinates (t, s) integrates, over
  the part of a strip where it is positive, to the probability of drawing
  that edge; so E[1{edge = e} / p_N] is the area of that part. For a strip
  whose every point is seen from x in front of the light (checked here with
  numpy geometry), that area is the whole strip, 1 x w in (t, s). A wrong
  Jacobian, light-area normaliser, edge length or selection probability in
  p_N moves the mean away from w;
* the one-sample mixture with the hierarchy is unbiased: for any weights g_e,
  E[g_e / pdf] is the sum of g over the edges the hierarchy can reach (the
  integrand g_e is constant in t, whose range has length 1);
* the default width is 2% of the mean absolute deviation of the vertex
  positions per coordinate, combined in L2 (a hand-computed example);
* the estimator's expectation does not change when the strategy is mixed in
  (gradients of a small-light shadow scene, with and without it).
"""
import math

import numpy as np
import pytest

import oracle
from paper_1904_12228_amd import scenegen as sg

LIGHT_Y, LIGHT_HALF = 2.0, 0.6
WIDTH = 0.03
X = np.array([0.01, 0.0, 0.02])
N_UP = np.array([0.0, 1.0, 0.0])


def shadow_scene(seed=0, n_occ=8):
    """Ground (y = 0, facing up), a square light at y = 2 facing down, and
    small one-sided triangles between them near the vertical through x."""
    rng = np.random.default_rng(seed)
    v = [(-3, 0, -3), (3, 0, -3), (3, 0, 3), (-3, 0, 3)]
    f = [(0, 2, 1), (0, 3, 2)]
    alb = [0.5, 0.5]
    emi = [0.0, 0.0]
    h = LIGHT_HALF
    base = len(v)
    v += [(-h, LIGHT_Y, -h), (h, LIGHT_Y, -h), (h, LIGHT_Y, h), (-h, LIGHT_Y, h)]
    f += [(base, base + 1, base + 2), (base, base + 2, base + 3)]
    alb += [0.0, 0.0]
    emi += [5.0, 5.0]
    for _ in range(n_occ):
        c = np.array([rng.uniform(-0.15, 0.15), rng.uniform(0.9, 1.3), rng.uniform(-0.15, 0.15)])
        b = len(v)
        for k in range(3):
            ang = 2 * math.pi * k / 3 + rng.uniform(-0.3, 0.3)
            v.append(tuple(c + 0.07 * np.array([math.cos(ang), rng.uniform(-0.3, 0.3), math.sin(ang)])))
        f.append((b, b + 1, b + 2))
        alb.append(0.6)
        emi.append(0.0)
    scene = sg.Scene(np.array(v, np.float32), np.array(f, np.int32), np.array(alb, np.float32),
                     np.array(emi, np.float32))
    cam = sg.Camera((0.0, 1.2, 3.0), (0.0, 0.6, 0.0), (0.0, 1.0, 0.0), 45.0, 32, 32)
    return scene, cam


def _strip(p, a_end, b_end, x):
    a = b_end - a_end
    ah = a / np.linalg.norm(a)
    c = np.cross(ah, a_end - x)
    return a, c / np.linalg.norm(c)


def _fully_covered(scene, e, x, w):
    """Every point of e's strip lies below the light and the ray from x
    through it meets the light square (the strip is convex: its corners
    decide)."""
    P = scene.vertices.astype(np.float64)
    pa, pb = P[e[0]], P[e[1]]
    a, v = _strip(None, pa, pb, x)
    for t in (0.0, 1.0):
        for s in (-w / 2, w / 2):
            b = pa + t * a + s * v
            d = b - x
            if not (0 < b[1] < LIGHT_Y):
                return False
            y = x + d * (LIGHT_Y - x[1]) / d[1]
            if max(abs(y[0]), abs(y[2])) > LIGHT_HALF * 0.98:
                return False
    return True


def test_default_width_is_two_percent_of_the_mean_absolute_deviation():
    # x: mean 1, deviations all 1; y: mean 2, deviations all 2; z: all 0
    v = np.array([(0, 0, 0), (2, 0, 0), (0, 4, 0), (2, 4, 0)], np.float32)
    scene = sg.Scene(v, np.array([(0, 1, 2), (1, 3, 2)], np.int32), np.full(2, 0.5, np.float32),
                     np.zeros(2, np.float32))
    assert oracle.edge_nee_width(scene) == pytest.approx(0.02 * math.sqrt(1 + 4), rel=1e-12)


def test_draws_lie_on_crossed_strips_in_front_of_the_light():
    scene, _ = shadow_scene(1)
    e, t, s, fl = oracle.edge_nee_sample(scene, X, N_UP, -1, WIDTH, 20000, seed=3)
    ok = e >= 0
    assert ok.mean() > 0.05
    rows = oracle.edges(scene)
    P = scene.vertices.astype(np.float64)
    for i in np.flatnonzero(ok)[:2000]:
        va, vb = rows[e[i], 0], rows[e[i], 1]
        a, v = _strip(None, P[va], P[vb], X)
        assert 0 <= t[i] <= 1 and abs(s[i]) <= WIDTH / 2
        b = P[va] + t[i] * a + s[i] * v
        d = b - X
        y = X + d * (LIGHT_Y - X[1]) / d[1]
        assert d[1] > 0 and b[1] < LIGHT_Y and max(abs(y[0]), abs(y[2])) <= LIGHT_HALF * (1 + 1e-9)
    # only the occluders' edges (never the ground's or the light's)
    assert (rows[e[ok], 2] >= 4).all()


@pytest.mark.parametrize("seed", [1, 2])
def test_fully_covered_strips_have_their_area(seed):
    scene, _ = shadow_scene(seed)
    N = 1000000
    e, t, s, fl = oracle.edge_nee_sample(scene, X, N_UP, -1, WIDTH, N, seed=11 + seed)
    ok = e >= 0
    pdf = np.zeros(N)
    pdf[ok] = oracle.edge_nee_pdf(scene, X, N_UP, -1, WIDTH, e[ok], t[ok], s[ok])
    assert (pdf[ok] > 0).all()
    rows = oracle.edges(scene)
    covered = [k for k in range(len(rows)) if rows[k, 2] >= 4 and _fully_covered(scene, rows[k], X, WIDTH)]
    assert len(covered) >= 8
    pooled = np.zeros(N)
    for k in covered:
        x = np.where(e == k, 1.0 / np.where(ok, pdf, 1.0), 0.0)
        mean, se = x.mean(), x.std() / math.sqrt(N)
        assert abs(mean - WIDTH) < 5 * se + 1e-12, (k, mean, WIDTH, se)
        assert se < 0.03 * WIDTH
        pooled += x
    # all covered strips together: a 2% error in the density is some 6 standard errors
    mean, se = pooled.mean() / len(covered), pooled.std() / math.sqrt(N) / len(covered)
    assert se < 0.004 * WIDTH
    assert abs(mean - WIDTH) < 5 * se, (mean / WIDTH, se / WIDTH)


def test_mixture_is_unbiased_for_edge_sums():
    scene, cam = shadow_scene(1)
    pdf_h, _ = oracle.edge_tree_pdf(scene, cam, X, N_UP)
    reach = pdf_h > 0
    N = 400000
    e, t, pdf = oracle.edge_nee_mix_sample(scene, cam, X, N_UP, -1, WIDTH, 0.5, N, seed=5)
    ok = e >= 0
    assert (pdf[ok] > 0).all() and (t[ok] >= 0).all() and (t[ok] <= 1).all()
    # every edge the billboards reach is also one the hierarchy can reach
    assert reach[e[ok]].all()
    E = len(pdf_h)
    gs = [np.ones(E)] + [np.random.default_rng(40 + k).uniform(size=E) for k in range(6)]
    for g in gs:
        x = np.where(ok, g[np.maximum(e, 0)] / np.where(ok, pdf, 1.0), 0.0)
        assert abs(x.mean() - g[reach].sum()) < 5 * x.std() / math.sqrt(N) + 1e-9
    # per edge: E[1{e} / pdf] = 1 for every reachable edge
    for k in np.flatnonzero(reach):
        x = np.where(e == k, 1.0 / np.where(ok, pdf, 1.0), 0.0)
        assert abs(x.mean() - 1.0) < 5 * x.std() / math.sqrt(N) + 1e-9, k
    # the billboards carry real weight: a fair share of the draws come from them
    e0, _, _ = oracle.edge_nee_mix_sample(scene, cam, X, N_UP, -1, WIDTH, 0.0, 20000, seed=5)
    assert (e[:20000] != e0).mean() > 0.2


def test_rejects_bad_arguments():
    scene, cam = shadow_scene(1)
    with pytest.raises(RuntimeError):
        oracle.edge_nee_sample(scene, X, N_UP, -1, 0.0, 1)
    with pytest.raises(RuntimeError):
        oracle.edge_nee_mix_sample(scene, cam, X, N_UP, -1, WIDTH, 1.0, 1)
    for kw in ({"enee": 1.0}, {"enee": -0.5}, {"enee": 0.5, "edge_t": 1}, {"enee": 0.5, "edge_candidates": 4}):
        with pytest.raises(RuntimeError):
            oracle.render(scene, cam, 1, 1, 0, d_image=np.ones((32, 32)), **kw)


@pytest.mark.slow
def test_estimator_expectation_unchanged():
    """Gradients of a soup under a small light, secondary term only, with and
    without the billboard strategy: equal means (z <= 5 per large entry)."""
    cfg = sg.soup(seed=3, n_tris=12, width=64, height=64, spp=2, light_size=0.15, light_emission=60.0)
    cam = cfg.camera.with_window(20, 22, 44, 42)
    x0, y0, x1, y1 = cam.win()
    dimg = np.random.default_rng(2).normal(size=(y1 - y0, x1 - x0)) + 0.5
    K = 40
    res = {}
    for alpha in (0.0, 0.5):
        gs = []
        for k in range(K):
            r = oracle.render(cfg.scene, cam, 16, 1, k, d_image=dimg, interior=False, primary=False, threads=8,
                              enee=alpha)
            gs.append(r["d_vertices"].ravel())
        res[alpha] = np.array(gs)
    a, b = res[0.0], res[0.5]
    ma, mb = a.mean(0), b.mean(0)
    se = np.sqrt(a.var(0, ddof=1) / K + b.var(0, ddof=1) / K)
    big = np.abs(ma) > 0.05 * np.abs(ma).max()
    z = np.abs(ma - mb)[big] / np.maximum(se[big], 1e-300)
    assert big.sum() >= 5
    assert (z <= 5).all(), np.sort(z)[-5:]
