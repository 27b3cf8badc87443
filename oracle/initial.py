"""Initial states: Taylor-Green vortex, channel flow, uniform flow; L2 projection.

Oracle (test infrastructure only).

Taylor-Green (Sec. 5.2.1): on [-pi L, pi L]^3,
    u1 =  U0 sin(x1/L) cos(x2/L) cos(x3/L),  u2 = -U0 cos(x1/L) sin(x2/L) cos(x3/L),  u3 = 0,
    p  = p0 + rho0 U0^2/16 (cos(2 x1/L) + cos(2 x2/L)) (cos(2 x3/L) + 2),
    T = T0 = c0^2 / (gamma R),  c0 = U0 / M,  p0 = rho0 R T0,  rho = p / (R T0).
Channel (Sec. 5.3.1): rho = 1, T = T0 = c^2/(gamma R) with c = u_max / M,
    u1 = u_max (1 - x2^2)  (laminar parabola; the paper's (1 - x2^6) is an option)
    plus a seeded perturbation of the velocity at the nodes (channel_perturbed).
The paper does not say how the initial state enters the discrete space; here it
is the L2 projection M^{-1} int phi U0(x), the right-hand side integrated with
the operator's n_q-point rule.
"""

import numpy as np
import torch

from . import physics as ph


def taylor_green(x, fl, U0=1.0, L=1.0, mach=0.1, rho0=1.0):
    c0 = U0 / mach
    T0 = c0 ** 2 / (fl.gamma * fl.R)
    p0 = rho0 * fl.R * T0
    x1, x2, x3 = x[..., 0] / L, x[..., 1] / L, x[..., 2] / L
    u = np.stack([U0 * np.sin(x1) * np.cos(x2) * np.cos(x3),
                  -U0 * np.cos(x1) * np.sin(x2) * np.cos(x3),
                  np.zeros_like(x1)], axis=-1)
    p = p0 + rho0 * U0 ** 2 / 16.0 * (np.cos(2 * x1) + np.cos(2 * x2)) * (np.cos(2 * x3) + 2.0)
    rho = p / (fl.R * T0)
    return ph.conserved_from_primitive(torch.as_tensor(rho), torch.as_tensor(u), torch.as_tensor(p), fl)


def channel_laminar(x, fl, umax=18.3, mach=0.1, power=2):
    c = umax / mach
    T0 = c ** 2 / (fl.gamma * fl.R)
    rho = np.ones(x.shape[:-1])
    u = np.zeros(x.shape)
    u[..., 0] = umax * (1.0 - x[..., 1] ** power)
    p = rho * fl.R * T0
    return ph.conserved_from_primitive(torch.as_tensor(rho), torch.as_tensor(u), torch.as_tensor(p), fl)


def channel_perturbed(op, U, r, umax=18.3, power=2, amp=0.1):
    """The perturbed channel initial state (Sec. 5.3.1): at every node of the nodal basis
    the velocity gets u_a += amp * u1(x2) * r_a with u1(x2) = umax (1 - |x2|^power) the
    laminar profile, so that the perturbation vanishes at the walls x2 = -1, 1, while the
    density and the temperature of the node are kept (rho E is recomputed from them).

    U: the state (5, E, N) (for a Lagrange basis its coefficients are its nodal values),
    r: the random numbers (3, E, N) in [-1, 1], drawn by the caller.  Returns a new array.
    The paper perturbs the laminar profile with random noise without fixing the recipe;
    this one scales the noise by the local laminar velocity."""
    fl = op.fl
    k = op.k
    pts = np.array([[op.nodes[a0], op.nodes[a1], op.nodes[a2]]
                    for a2 in range(k + 1) for a1 in range(k + 1) for a0 in range(k + 1)])
    x, _ = op.mesh.map_at(pts)                               # (E, N, 3)
    U = torch.as_tensor(U, dtype=torch.float64)
    Un = U.permute(1, 2, 0)                                  # (E, N, 5)
    rho = Un[..., 0]
    T = ph.temperature(Un, fl)
    u = ph.velocity(Un)
    lam = torch.as_tensor(umax * (1.0 - np.abs(x[..., 1]) ** power))
    u = u + amp * lam[..., None] * torch.as_tensor(np.asarray(r, dtype=np.float64)).permute(1, 2, 0)
    out = torch.zeros_like(Un)
    out[..., 0] = rho
    out[..., 1:4] = rho[..., None] * u
    out[..., 4] = rho * (fl.c_v * T + 0.5 * (u * u).sum(-1))
    return out.permute(2, 0, 1).contiguous()


def uniform(x, fl, rho=1.0, u=(0.3, -0.2, 0.1), p=None):
    p = 1.0 / fl.gamma if p is None else p
    shape = x.shape[:-1]
    return ph.conserved_from_primitive(torch.full(shape, rho, dtype=torch.float64),
                                       torch.as_tensor(np.broadcast_to(np.asarray(u), shape + (3,)).copy()),
                                       torch.full(shape, p, dtype=torch.float64), fl)


def l2_project(op, func, cells=None):
    """U_h = M^{-1} (phi_i, U0) with the right-hand side on the n_q-point rule.

    With `cells`, only those cells are projected (shape (5, len(cells), N))."""
    cells = np.arange(op.mesh.n_cells) if cells is None else np.asarray(cells, dtype=np.int64)
    x, _, detJ = op._geometry(cells, op.cell_pts)
    vals = func(x.numpy())                                   # (E, P, 5)
    rhs = torch.einsum("pi,epc->cei", op.Phi, vals * (detJ * torch.as_tensor(op.cell_w))[..., None])
    return op.apply_inverse_mass(rhs, cells)
