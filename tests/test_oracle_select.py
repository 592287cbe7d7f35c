"""Pins of the oracle's stratified multi-sample edge selection (CPU).

M samples go down the edge hierarchy, divided between the children of every
node in proportion to importance; one of the leaves reached is kept by
weighted reservoir sampling and weighted by W / (M imp) (Ch. 5, Edge
selection). What fixes the expected values, independently of the oracle's
own code:

* a selection scheme with weight w is unbiased for a sum over edges exactly
  when E[1{z = e} w] = 1 for every edge e the integrand may reach, so the
  per-edge means are checked against 1 (the enumerated descent pdf tells
  which edges are reachable: those with pdf > 0);
* with one sample the scheme is a single descent: the kept edge is
  distributed as the descent pdf and its weight is 1 / pdf.

The hierarchy's own pdf is pinned separately (test_oracle_pins.py).
"""
import math

import numpy as np
import pytest

import oracle

from .test_oracle_pins import _shading_points, small_soup, small_sphere

USTRIDE = 256


@pytest.mark.parametrize("which,M", [("soup", 2), ("soup", 16), ("sphere", 4), ("sphere", 16)])
def test_every_reachable_edge_is_selected_with_unit_expected_weight(which, M):
    scene, cam, cfg = small_soup(n=40) if which == "soup" else small_sphere(level=1)
    rng = np.random.default_rng(21 + M)
    (p, n), = _shading_points(scene, 1, rng)
    pdf, fail = oracle.edge_tree_pdf(scene, cam, p, n)
    # 400,000 draws in chunks (a few edges have rare weights far above their
    # usual one, so the means need many draws)
    N = 400000
    parts = [oracle.edge_tree_select(scene, cam, p, n, M, rng.uniform(size=(50000, USTRIDE))) for _ in range(8)]
    e = np.concatenate([a for a, _ in parts])
    w = np.concatenate([b for _, b in parts])
    ok = e >= 0
    # never an edge the descent cannot reach
    assert (pdf[e[ok]] > 0).all()
    E = len(pdf)
    reach = pdf > 0
    # linear functionals of the per-edge means: E[g(z) w] = sum of g over the
    # reachable edges, for g = 1 and for random positive g (a bias on any
    # edge that carries weight shows in them)
    gs = [np.ones(E)] + [np.random.default_rng(100 + k).uniform(size=E) for k in range(8)]
    for g in gs:
        x = np.where(ok, g[np.maximum(e, 0)] * w, 0.0)
        assert abs(x.mean() - g[reach].sum()) < 5 * x.std() / math.sqrt(N) + 1e-9
    # per edge, where the weights of its selections are light-tailed enough
    # for a standard error to mean something (a few edges get rare weights
    # of tens of times their usual one: kept when the others reached in the
    # same draw dominate the reservoir)
    cnt = np.bincount(e[ok], minlength=E)
    sums = np.bincount(e[ok], weights=w[ok], minlength=E)
    sq = np.bincount(e[ok], weights=w[ok] ** 2, minlength=E)
    mean = sums / N
    se = np.sqrt(np.maximum(sq / N - mean ** 2, 0.0) / N)
    light = np.array([cnt[k] >= 30 and w[e == k].max() <= 20 * np.median(w[e == k]) for k in range(E)])
    tested = reach & light
    assert tested.sum() >= 0.6 * reach.sum()
    z = np.abs(mean[tested] - 1.0) / np.maximum(se[tested], 1e-12)
    assert z.max() < 5.5, (z.max(), np.flatnonzero(tested)[np.argmax(z)])


def test_single_sample_is_one_descent():
    scene, cam, cfg = small_sphere(level=1)
    rng = np.random.default_rng(5)
    (p, n), = _shading_points(scene, 1, rng)
    pdf, fail = oracle.edge_tree_pdf(scene, cam, p, n)
    N = 200000
    u = rng.uniform(size=(N, 64))
    e, w = oracle.edge_tree_select(scene, cam, p, n, 1, u)
    ok = e >= 0
    np.testing.assert_allclose(w[ok], 1.0 / pdf[e[ok]], rtol=1e-12)
    assert abs((~ok).mean() - fail) < 5 * math.sqrt(max(fail, 1e-6) / N) + 1e-4
    counts = np.bincount(e[ok], minlength=len(pdf))
    big = pdf * N > 50
    chi2 = (((counts[big] - pdf[big] * N) ** 2) / (pdf[big] * N)).sum()
    dof = big.sum() - 1
    assert chi2 < dof + 6 * math.sqrt(2 * dof)


def test_more_samples_lower_the_weight_spread():
    """The point of several samples: for the same query the kept edge's
    weight varies less (relative to its mean) than a single descent's."""
    scene, cam, cfg = small_soup(n=40)
    rng = np.random.default_rng(8)
    (p, n), = _shading_points(scene, 1, rng)
    N = 40000
    u = rng.uniform(size=(N, USTRIDE))
    cv = []
    for M in (1, 16):
        e, w = oracle.edge_tree_select(scene, cam, p, n, M, u)
        cv.append(w.std() / w.mean())
    assert cv[1] < cv[0]


def test_rejects_bad_arguments():
    scene, cam, cfg = small_soup(n=10)
    p, n = np.zeros(3), np.array([0.0, 1.0, 0.0])
    with pytest.raises(RuntimeError):
        oracle.edge_tree_select(scene, cam, p, n, 0, np.zeros((1, 8)))
    with pytest.raises(RuntimeError):
        oracle.edge_tree_select(scene, cam, p, n, 64, np.full((1, 1), 0.5))
