"""Pins of the oracle's 1D rules and Lagrange bases against exact integrals and polynomial identities."""
import numpy as np
import pytest

from oracle import rules


@pytest.mark.parametrize("nq", range(1, 13))
def test_gauss_exact_to_degree_2nq_minus_1(nq):
    x, w = rules.gauss_legendre(nq)
    for m in range(2 * nq):
        assert abs(np.sum(w * x ** m) - 1.0 / (m + 1)) < 1e-14
    # not exact one degree higher: the squared node polynomial has a positive
    # integral (here with a larger rule) while the rule itself returns 0
    xb, wb = rules.gauss_legendre(nq + 2)
    node_poly2 = np.prod((xb[:, None] - x[None, :]) ** 2, axis=1)
    assert np.sum(wb * node_poly2) > 1e3 * np.sum(w * np.prod((x[:, None] - x[None, :]) ** 2, axis=1)) + 1e-300


@pytest.mark.parametrize("n", range(2, 13))
def test_lobatto_points(n):
    x = rules.gauss_lobatto_points(n)
    assert x[0] == 0.0 and x[-1] == 1.0
    assert np.allclose(x + x[::-1], 1.0, atol=1e-14)           # symmetric
    # the LGL quadrature with these points (weights from the moment equations) is exact to 2n-3
    V = np.vander(x, n, increasing=True).T
    w = np.linalg.solve(V, 1.0 / np.arange(1, n + 1))
    for m in range(2 * n - 2):
        assert abs(np.sum(w * x ** m) - 1.0 / (m + 1)) < 1e-12
    assert np.all(w > 0)


def test_lobatto_known_values():
    # closed forms on [-1,1]: n=3 -> 0; n=4 -> +-1/sqrt(5); n=5 -> 0, +-sqrt(3/7)
    assert np.allclose(rules.gauss_lobatto_points(3), [0, 0.5, 1])
    assert np.allclose(rules.gauss_lobatto_points(4), 0.5 * (1 + np.array([-1, -1 / np.sqrt(5), 1 / np.sqrt(5), 1])))
    assert np.allclose(rules.gauss_lobatto_points(5), 0.5 * (1 + np.array([-1, -np.sqrt(3 / 7), 0, np.sqrt(3 / 7), 1])))


@pytest.mark.parametrize("basis", ["LGL", "GL"])
@pytest.mark.parametrize("k", [1, 2, 3, 5, 7])
def test_lagrange_interpolates_and_differentiates_polynomials(basis, k):
    nodes = rules.support_points(k, basis)
    xs = np.linspace(-0.1, 1.1, 17)
    V = rules.lagrange_values(nodes, xs)
    D = rules.lagrange_derivatives(nodes, xs)
    assert np.allclose(rules.lagrange_values(nodes, nodes), np.eye(k + 1), atol=1e-14)
    for m in range(k + 1):
        assert np.allclose(V @ nodes ** m, xs ** m, atol=1e-12)
        dm = m * xs ** (m - 1) if m > 0 else np.zeros_like(xs)
        assert np.allclose(D @ nodes ** m, dm, atol=1e-10)


def test_three_halves_rule():
    # n_q = ceil((3k+1)/2): the values the paper's Table 1 implies for k = 2, 3, 5, 7, 11, 15
    assert [rules.nq_three_halves(k) for k in (2, 3, 4, 5, 7, 11, 15)] == [4, 5, 7, 8, 11, 17, 23]
