"""Small seeded states and operators shared by the oracle pin tests (CPU only)."""
import math

import numpy as np
import torch

from oracle import mesh, operator, physics


def random_state(E, N, seed, rho=1.0, u=(0.3, -0.2, 0.1), p=2.0, amp=0.05, gamma=1.4):
    """A smooth-enough, strictly admissible state: mean (rho, u, p) plus seeded noise."""
    rng = np.random.default_rng(seed)
    r = rho * (1 + amp * rng.uniform(-1, 1, (E, N)))
    v = np.asarray(u)[None, None, :] + amp * rng.uniform(-1, 1, (E, N, 3))
    P = p * (1 + amp * rng.uniform(-1, 1, (E, N)))
    U = np.zeros((5, E, N))
    U[0] = r
    U[1:4] = np.moveaxis(r[..., None] * v, -1, 0)
    U[4] = P / (gamma - 1) + 0.5 * r * (v * v).sum(-1)
    return torch.as_tensor(U)


def make(n=(2, 2, 2), k=2, nq=3, basis="LGL", kind=mesh.AFFINE, periodic=(True, True, True),
         lo=(0.0, 0.0, 0.0), hi=(1.0, 1.3, 0.8), mu=0.02, lam=0.03, amp=0.0, wall_T=None, force=None):
    m = mesh.BoxMesh(n, lo, hi, k, periodic=periodic, kind=kind, deform_amp=amp)
    fl = physics.Fluid(gamma=1.4, R=287.0, mu=mu, lam=lam, rho_ref=1.0)
    return operator.DGOperator(m, fl, nq, basis=basis, body_force=force, wall_T=wall_T)
