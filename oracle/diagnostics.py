"""Kinetic energy, dissipation rate and conserved totals.

Oracle (test infrastructure only).

Paper Sec. 5.2.3: computed as for the incompressible case,
    e_k = 1/V int 1/2 u.u,   eps = nu/V int grad u : grad u,
    eps_num = -d e_k/dt - eps,
with u = (rho u)/rho and the element-wise (broken) gradient of u.  The exact
rate -d e_k/dt = -1/V int u . du/dt with du/dt = (L_m - u L_rho)/rho follows
from dU/dt = L(U).  Integrals of e_k, eps and the rate use the n_q-point rule of
the operator; the conserved totals int U_h use the (k+1)-point rule, i.e. they
equal 1^T M U.
"""

import numpy as np
import torch

from . import physics as ph


def diagnostics(op, U, L=None):
    """Returns dict e_k, eps, rate (=-de_k/dt or nan), mass, mom (3,), energy, volume."""
    fl = op.fl
    cells = np.arange(op.mesh.n_cells)
    out = dict(e_k=0.0, eps=0.0, rate=0.0, mass=0.0, mom=np.zeros(3), energy=0.0, volume=0.0)
    for c0 in range(0, len(cells), 1024):
        cc = cells[c0:c0 + 1024]
        _, Jinv, detJ = op._geometry(cc, op.cell_pts)
        JxW = detJ * torch.as_tensor(op.cell_w)
        Uq, Gx = op._values(U[:, cc, :], op.Phi, op.dPhi, Jinv)
        u = ph.velocity(Uq)
        gu = ph.velocity_gradient(Uq, Gx)
        out["volume"] += float(JxW.sum())
        out["e_k"] += float((0.5 * (u * u).sum(-1) * JxW).sum())
        out["eps"] += float(((gu * gu).sum((-1, -2)) * JxW).sum())
        if L is not None:
            Lq = torch.einsum("pi,cei->epc", op.Phi, L[:, cc, :])
            dudt = ph.velocity_rate(Uq, Lq)
            out["rate"] += float(-((u * dudt).sum(-1) * JxW).sum())
        _, _, detJm = op._geometry(cc, op.mass_pts)
        JxWm = detJm * torch.as_tensor(op.mass_w)
        Um = torch.einsum("pi,cei->epc", op.Phi_m, U[:, cc, :])
        tot = (Um * JxWm[..., None]).sum((0, 1)).numpy()
        out["mass"] += tot[0]
        out["mom"] = out["mom"] + tot[1:4]
        out["energy"] += tot[4]
    V = out["volume"]
    out["e_k"] /= V
    out["eps"] *= fl.nu / V
    out["rate"] = out["rate"] / V if L is not None else float("nan")
    return out


def channel_statistics(op, U):
    """Plane averages for the statistics of the channel flow (Sec. 5.3), where x and z
    are homogeneous: for each wall-normal Gauss point (cell row j in direction 1, point
    p of the n_q rule) the |det J| w weighted averages over all cells of the row and all
    (x, z) Gauss points of y, rho, u, v, w, uu, vv, ww, uv with u = (rho u)/rho.

    Returns an (n[1] * n_q, 9) array, rows ordered by j, then p.  Meant for meshes on
    which y depends on the second reference coordinate alone (box and channel)."""
    m = op.mesh
    nx, ny, nz = m.n
    q = op.n_q
    py = (np.arange(q ** 3) // q) % q       # point p = px + q (py + q pz)
    out = np.zeros((ny * q, 9))
    for j in range(ny):
        cells = np.array([i + nx * (j + ny * k) for k in range(nz) for i in range(nx)], dtype=np.int64)
        x, _, detJ = op._geometry(cells, op.cell_pts)
        w = (detJ * torch.as_tensor(op.cell_w)).numpy()                 # [E, P]
        Uq = torch.einsum("pi,cei->epc", op.Phi, U[:, cells, :]).numpy()  # [E, P, 5]
        rho = Uq[..., 0]
        u = Uq[..., 1:4] / rho[..., None]
        x = np.asarray(x)
        fields = [x[..., 1], rho, u[..., 0], u[..., 1], u[..., 2],
                  u[..., 0] * u[..., 0], u[..., 1] * u[..., 1], u[..., 2] * u[..., 2], u[..., 0] * u[..., 1]]
        for p in range(q):
            sel = py == p
            ws = w[:, sel]
            out[j * q + p] = [float((f[:, sel] * ws).sum() / ws.sum()) for f in fields]
    return out
