"""One-dimensional rules and Lagrange bases on the reference interval [0, 1].

Oracle (test infrastructure only).

Paper: Sec. 2.2.1 (reference element [0,1]^d, tensor-product Lagrange basis on
Legendre-Gauss-Lobatto support points) and Sec. 2.2.3 (Gauss-Legendre
quadrature with n_q points, exact to polynomial degree 2 n_q - 1).
"""

import numpy as np
from numpy.polynomial import legendre as npleg


def gauss_legendre(nq):
    """Gauss-Legendre points and weights on [0, 1] (Sec. 2.2.3).

    numpy's rule on [-1, 1] is mapped affinely; the weights then sum to 1.
    """
    x, w = npleg.leggauss(nq)
    return 0.5 * (x + 1.0), 0.5 * w


def gauss_lobatto_points(n):
    """The n Legendre-Gauss-Lobatto points on [0, 1] (Sec. 2.2.1).

    They are the two interval ends plus the roots of P'_{n-1}.
    """
    if n < 2:
        raise ValueError("an LGL rule needs at least 2 points")
    coef = np.zeros(n)
    coef[-1] = 1.0                       # P_{n-1} as a Legendre series
    inner = npleg.legroots(npleg.legder(coef)) if n > 2 else np.zeros(0)
    x = np.concatenate(([-1.0], np.sort(np.real(inner)), [1.0]))
    return 0.5 * (x + 1.0)


def support_points(k, basis):
    """Nodes of the degree-k nodal basis: 'LGL' (the paper's) or 'GL'."""
    if basis == "LGL":
        return gauss_lobatto_points(k + 1)
    if basis == "GL":
        return gauss_legendre(k + 1)[0]
    raise ValueError(basis)


def lagrange_values(nodes, x):
    """V[p, i] = l_i(x_p), the Lagrange polynomial of node i, by its product formula."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    V = np.ones((len(x), n))
    for i in range(n):
        for j in range(n):
            if j != i:
                V[:, i] *= (x - nodes[j]) / (nodes[i] - nodes[j])
    return V


def lagrange_derivatives(nodes, x):
    """D[p, i] = l_i'(x_p), by the product rule applied to the product formula."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    D = np.zeros((len(x), n))
    for i in range(n):
        for m in range(n):
            if m == i:
                continue
            term = np.full(len(x), 1.0 / (nodes[i] - nodes[m]))
            for j in range(n):
                if j != i and j != m:
                    term *= (x - nodes[j]) / (nodes[i] - nodes[j])
            D[:, i] += term
    return D


def nq_three_halves(k):
    """The paper's over-integration rule n_q = ceil((3k+1)/2) (Sec. 2.2.3)."""
    return (3 * k + 2) // 2
