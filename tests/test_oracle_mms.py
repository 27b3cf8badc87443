"""Consistency pin of the whole oracle operator: a manufactured solution converges.

The source of the manufactured solution is derived symbolically from the PDE of
the paper's Sec. 2.1 in primitive variables (tests/mms.py), the oracle integrates
dU/dt = L(U) + M^{-1}(phi, S) with its Runge-Kutta scheme, and the L2 error at
the final time must fall at least at rate k + 0.7 under h-refinement.  A dropped
or sign-flipped consistent term (a flux component, the face flux, the viscous
stress or heat flux) leaves an O(1) error and fails this test.
"""
import math

import pytest
import torch

from oracle import initial, mesh, operator, physics, timeint
from tests import mms


def _error(k, ne, t_final=0.05):
    fl = physics.Fluid(gamma=mms.GAMMA, R=mms.RGAS, mu=mms.MU, lam=mms.LAM)
    m = mesh.BoxMesh((ne,) * 3, (0, 0, 0), (1, 1, 1), k)
    op = operator.DGOperator(m, fl, k + 2)
    proj = lambda tt: initial.l2_project(op, lambda X: torch.as_tensor(mms.exact(X, tt)))
    U = proj(0.0)
    dt = timeint.time_step(0.2, 0.01, 1.5, 3, k, 1.0 / ne, 0.4, 0.4 / 1.06, 0.1)
    nst = int(math.ceil(t_final / dt))
    dt = t_final / nst
    t = 0.0
    for _ in range(nst):
        U = timeint.lsrk_step(lambda V, tt: op.apply(V, source=mms.source, t=tt), U, t, dt)
        t += dt
    d = U - proj(t_final)
    M = op.mass_matrices()
    return math.sqrt(float(torch.einsum("cei,eij,cej->", d, M, d)))


@pytest.mark.parametrize("k,meshes", [(1, (4, 8)), (2, (2, 4))])
def test_manufactured_solution_convergence(k, meshes):
    e0, e1 = (_error(k, ne) for ne in meshes)
    rate = math.log2(e0 / e1)
    assert rate > k + 0.7, (e0, e1, rate)
