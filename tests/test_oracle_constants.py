"""Pins of the oracle's velocity set and weights (readings R1, R2, R11).

The weights are solved from shell-aggregated equations; here every moment is
re-summed by brute force over the 37 explicit hops and compared with Gaussian
moments from Gauss-Hermite quadrature, an independent route.
"""
import json
import math
import os

import numpy as np
import pytest
from numpy.polynomial.hermite_e import hermegauss

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_counts.json")


def _gold(key):
    with open(GOLD) as fh:
        return json.load(fh)[key]["value"]


def _gauss_moment(p: int) -> float:
    """E[X^p] for a standard normal X, by 20-node Gauss-Hermite quadrature."""
    x, w = hermegauss(20)
    return float((w * x ** p).sum() / math.sqrt(2.0 * math.pi))


def test_population_count_and_reach():
    E, shell, opp = oracle.velocity_set()
    assert E.shape == (_gold("populations"), 2)
    assert len({tuple(v) for v in E.tolist()}) == _gold("populations")
    assert int(np.abs(E).max()) == _gold("max_hop")
    assert (E[0] == 0).all()


def test_boundary_crossing_count():
    """Populations that cross a vertical boundary, counted per distance.

    A hop with e_x = k > 0 needs the k columns beyond the boundary, so the
    populations to move per boundary site are sum_l max(e_x, 0).
    """
    E, _, _ = oracle.velocity_set()
    ex = E[:, 0]
    assert int(np.maximum(ex, 0).sum()) == _gold("populations_per_boundary_site")
    assert int(np.maximum(-ex, 0).sum()) == _gold("populations_per_boundary_site")
    # by distance: 15 populations reach 1 column, 8 reach 2, 3 reach 3
    assert [int((ex >= d).sum()) for d in (1, 2, 3)] == [15, 8, 3]
    assert int(np.abs(ex).max()) == _gold("halo_columns")


def test_opposite_and_order():
    E, shell, opp = oracle.velocity_set()
    assert (E[opp] == -E).all()
    assert (opp[opp] == np.arange(37)).all()
    # canonical order: shells in order, lexicographic within a shell
    assert list(shell) == sorted(shell)
    for s in range(8):
        vs = [tuple(v) for v in E[shell == s].tolist()]
        assert vs == sorted(vs)
    assert [int((shell == s).sum()) for s in range(8)] == [1, 4, 4, 4, 8, 4, 4, 8]


def test_weights_positive_unique_and_normalised():
    k = oracle.constants()
    assert (k.w > 0).all()
    assert abs(k.w.sum() - 1.0) < 1e-15
    assert 1.0 < k.r < 1.5
    # weights depend on |e| only
    n2 = (k.E ** 2).sum(1)
    for v in np.unique(n2):
        assert len(set(k.w[n2 == v].tolist())) == 1


@pytest.mark.parametrize("order", range(0, 11))
def test_isotropy_by_brute_force(order):
    """sum_l w_l cx^p cy^q = E[X^p] E[Y^q] for every p + q <= 8 (exact
    quadrature of degree 9), and the degree-10 moments differ."""
    k = oracle.constants()
    for p in range(order + 1):
        q = order - p
        disc = float((k.w * k.cx ** p * k.cy ** q).sum())
        cont = _gauss_moment(p) * _gauss_moment(q)
        if order <= 9:
            assert abs(disc - cont) <= 2e-13 * max(1.0, abs(cont)), (p, q, disc, cont)
    if order == 10:
        disc = float((k.w * k.cx ** 10).sum())
        assert abs(disc - _gauss_moment(10)) > 1.0  # degree 9 is the limit


def test_extended_precision_solution_satisfies_conditions():
    """The 60-digit solution satisfies every moment condition to 1e-40."""
    import mpmath as mp
    r_str, w_str = oracle.solve_isotropy()
    E, shell, _ = oracle.velocity_set()
    with mp.workdps(60):
        r = mp.mpf(r_str)
        W = [mp.mpf(x) for x in w_str]
        for p in range(0, 9, 2):
            for q in range(0, 9 - p, 2):
                s = mp.mpf(0)
                for l in range(37):
                    s += W[shell[l]] * (r * int(E[l, 0])) ** p * (r * int(E[l, 1])) ** q
                exact = mp.mpf(math.prod(range(p - 1, 0, -2))) * math.prod(range(q - 1, 0, -2))
                assert abs(s - exact) < mp.mpf(10) ** -40, (p, q)


def test_binary64_constants_are_correctly_rounded():
    k = oracle.constants()
    assert k.r == float(k.r_str)
    assert k.w_shell.tolist() == [float(x) for x in k.w_shell_str]
