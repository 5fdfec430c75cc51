"""Search-difficulty analysis (section V.B): the library's fitness-flow-graph
PageRank against the oracle's dense solve, and the oracle against closed forms."""
import itertools

import numpy as np
import pytest

import paper_2211_07260_amd as gt
from oracle import ffg as offg


@pytest.fixture(scope="module", autouse=True)
def host_only():
    gt.init(0, gt.INIT_HOST_ONLY)
    yield
    gt.shutdown()


def test_oracle_two_nodes_closed_form():
    # a -> b (b better, b a sink): x_a = (1-d)/2 + d x_b / 2 ; x_b = (1-d)/2 + d x_b / 2 + d x_a
    d = 0.85
    pr, is_min = offg.ffg_pagerank([(1, 0, 0, 0, 0, 0), (2, 0, 0, 0, 0, 0)], [2.0, 1.0], d)
    a = np.array([[1.0, -d / 2], [-d, 1 - d / 2]])
    xa, xb = np.linalg.solve(a, [(1 - d) / 2, (1 - d) / 2])
    assert pr[0] == pytest.approx(xa) and pr[1] == pytest.approx(xb)
    assert list(is_min) == [False, True] and pr.sum() == pytest.approx(1.0)


def test_oracle_flat_fitness_is_uniform():
    cfgs = list(itertools.product((16, 32), (1, 2), (1,), (1,), (0,), (0,)))
    pr, is_min = offg.ffg_pagerank(cfgs, [5.0] * len(cfgs))
    assert np.allclose(pr, 1.0 / len(cfgs)) and is_min.all()


def test_oracle_single_minimum_gets_all_minimum_mass():
    cfgs = list(itertools.product((1, 2, 3, 4), (1, 2, 3), (0,), (0,), (0,), (0,)))
    fit = [abs(c[0] - 3) + abs(c[1] - 2) + 1.0 for c in cfgs]   # unimodal, optimum (3, 2)
    assert offg.proportion_of_centrality(cfgs, fit, [1.0]) == [1.0]


SPACE = dict(bx=(16, 32, 64), by=(1, 2, 4, 8), tx=(1, 2, 4, 8), ty=(1, 2, 3), pad=(0, 1), rp=(0, 1))


@pytest.mark.parametrize("seed", range(3))
def test_library_matches_oracle(seed):
    rng = np.random.default_rng(seed)
    cfgs = [c for c in itertools.product(*SPACE.values()) if rng.random() < 0.7]
    fit = rng.lognormal(0.0, 0.3, len(cfgs))
    ps = [1.0, 1.05, 1.1, 1.25, 1.5, 2.0]
    pr, im, prop = gt.ffg_centrality(cfgs, fit, ps)
    opr, omin = offg.ffg_pagerank(cfgs, fit)
    np.testing.assert_allclose(pr, opr, rtol=1e-9, atol=1e-15)
    assert [bool(v) for v in im] == list(omin)
    np.testing.assert_allclose(prop, offg.proportion_of_centrality(cfgs, fit, ps), rtol=1e-9)
