"""Pins of the oracle's learned-proposal mixture and its harvest statistic (CPU).

The proposal q is any distribution over all edges; the mixture draws an edge
from q with probability `mix` and from the plain sampler otherwise, and weights
every sample by the mixture pdf. Two facts fix what the oracle must compute,
independently of its own code:

* an importance-sampled estimator is unbiased for every sampling pdf that is
  positive wherever the integrand is, so plain and mixture estimates of the
  same gradient agree in expectation;
* the harvest adds P * |c|^2 for a sample drawn with probability P whose
  contribution c carries a factor 1/P, so its expectation, sum over units of
  P * E[|G|^2 / P^2] = E|G|^2 per unit, does not depend on the sampler either.

Each check compares means over independent seeds within 5 standard errors.
"""
import numpy as np
import pytest

import oracle

from .test_oracle_pins import _shading_points, small_soup, small_sphere


def _proposal(E, seed):
    rng = np.random.default_rng(seed)
    q = rng.gamma(0.5, size=E) + 1e-3
    return q / q.sum()


@pytest.mark.parametrize("which", ["soup", "sphere"])
def test_tree_pdf_of_a_given_edge_equals_enumeration(which):
    scene, cam, cfg = small_soup(n=40) if which == "soup" else small_sphere(level=2)
    rng = np.random.default_rng(11)
    ids = np.arange(oracle.num_edges(scene))
    for p, n in _shading_points(scene, 8, rng):
        pdf, fail = oracle.edge_tree_pdf(scene, cam, p, n)
        np.testing.assert_allclose(oracle.edge_tree_pdf_of(scene, cam, p, n, ids), pdf, rtol=1e-13, atol=1e-300)


def _runs(scene, cam, cfg, seeds, terms, q, mix, key):
    out = []
    for sd in seeds:
        r = oracle.render(scene, cam, cfg.spp, cfg.max_depth, sd, d_image=1.0, interior=False,
                          primary=terms == 1, secondary=terms == 2, threads=8, edge_pdf=q, mix=mix,
                          mix_terms=terms, edge_stats=True)
        out.append(r[key].ravel().copy())
    return np.array(out)


def _agree(a, b, min_entries):
    ma, mb = a.mean(0), b.mean(0)
    se = np.sqrt(a.var(0, ddof=1) / len(a) + b.var(0, ddof=1) / len(b))
    sig = se > 0
    assert sig.sum() >= min_entries
    z = np.abs(ma - mb)[sig] / se[sig]
    assert z.max() < 5.0, z.max()
    # the estimates are not trivially equal: the mixture draws other samples
    assert not np.allclose(a[0], b[0])


@pytest.mark.parametrize("terms", [1, 2])
@pytest.mark.parametrize("key", ["d_vertices", "edge_stats"])
def test_mixture_and_plain_estimators_agree_in_expectation(terms, key):
    scene, cam, cfg = small_soup(n=40, w=20, h=20, spp=4)
    q = _proposal(oracle.num_edges(scene), 1)
    seeds = range(40)
    plain = _runs(scene, cam, cfg, seeds, terms, None, 0.0, key)
    mixed = _runs(scene, cam, cfg, [s + 1000 for s in seeds], terms, q, 0.8, key)
    _agree(plain, mixed, 20)


def test_mixture_weight_zero_is_the_plain_sampler():
    scene, cam, cfg = small_soup(n=40, w=12, h=12, spp=2)
    q = _proposal(oracle.num_edges(scene), 2)
    a = oracle.render(scene, cam, cfg.spp, cfg.max_depth, 5, d_image=1.0, threads=1, edge_stats=True)
    b = oracle.render(scene, cam, cfg.spp, cfg.max_depth, 5, d_image=1.0, threads=1, edge_pdf=q, mix=0.0,
                      edge_stats=True)
    for k in ("d_vertices", "d_albedo", "d_camera", "edge_stats"):
        np.testing.assert_array_equal(a[k], b[k])
