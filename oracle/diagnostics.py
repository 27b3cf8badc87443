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


def channel_wall_shear(op, U):
    """Mean wall shear stress over both walls in x2 (Sec. 5.3, u_tau = sqrt(tau_w / rho)):
    at the face points of every wall face, mu du_1/dn with n the wall normal into the fluid
    (+x2 at the lower wall, -x2 at the upper), averaged with the face weights dA.
    Returns (tau_w, rho_w, wall area), rho_w the same average of the density."""
    m, fl = op.mesh, op.fl
    tot = np.zeros(3)
    for s, sign in ((0, 1.0), (1, -1.0)):
        cells = np.nonzero(m.nb[:, 1, s] < 0)[0]
        pts, wf, P, dP = op.face[1, s]
        _, Jinv, detJ = op._geometry(cells, pts)
        _, dA = op._face_measure(Jinv, detJ, wf, 1, s)
        Uq, Gx = op._values(U[:, cells, :], P, dP, Jinv)
        gu = ph.velocity_gradient(Uq, Gx)                    # [e, p, a, j] = du_a / dx_j
        tau = fl.mu * gu[..., 0, 1] * sign
        tot += [float((tau * dA).sum()), float((Uq[..., 0] * dA).sum()), float(dA.sum())]
    return tot[0] / tot[2], tot[1] / tot[2], tot[2]


def channel_plus_statistics(profiles, walls, nu, y_lo):
    """Time averages over the samples (Sec. 5.3) in wall units.  profiles: list of the
    (rows, 9) plane averages [y, rho, u, v, w, uu, vv, ww, uv] of channel_statistics, walls:
    list of (tau_w, rho_w, area) of channel_wall_shear, one per sample.  u_tau =
    sqrt(<tau_w> / <rho_w>); rows [y, y+ = (y - y_lo) u_tau / nu, <u>/u_tau, rms u_i / u_tau
    (rms u = sqrt(<uu> - <u>^2)), (<uv> - <u><v>) / u_tau^2, <rho>].  Returns (rows, u_tau)."""
    A = np.mean(np.stack(profiles), axis=0)
    tau = np.mean([w[0] for w in walls])
    rho_w = np.mean([w[1] for w in walls])
    u_tau = np.sqrt(tau / rho_w)
    y, rho, u, v, w, uu, vv, ww, uv = A.T
    out = np.stack([y, (y - y_lo) * u_tau / nu, u / u_tau,
                    np.sqrt(np.maximum(uu - u * u, 0.0)) / u_tau,
                    np.sqrt(np.maximum(vv - v * v, 0.0)) / u_tau,
                    np.sqrt(np.maximum(ww - w * w, 0.0)) / u_tau,
                    (uv - u * v) / u_tau ** 2, rho], axis=1)
    return out, u_tau

