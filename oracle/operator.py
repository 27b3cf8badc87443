"""The DG spatial operator L(U) = M^{-1} (-F_c(U) - F_v(U) + F_rhs(U)), evaluated directly.

Oracle (test infrastructure only).

Paper: Sec. 2.2.2 eq. (WeakFormulationConservedVariables) with the local
Lax-Friedrichs flux and the symmetric interior penalty flux; Sec. 2.2.3 eqs.
(IntegralsReferenceSpace, IntegralsNumericalQuadrature) for the transformation
to the reference cell and Gauss quadrature; Sec. 2.4 eq.
(SpatiallyDiscretizedProblem) for L.

With V_h the test function phi_i of the cell e (its own basis), the weak form
moved to the right-hand side reads, per conserved component c,

  R_i =  sum_cell-points  w |det J| grad phi_i . (F_c - F_v)(U, grad U)
       + sum_face-points  dA [ phi_i ( - F*_c.n  +  Q*.n )
                                + 1/2 grad phi_i . F_v(U^-, [[U]]) ]
       + sum_mass-points  w |det J| phi_i F_rhs

  F*_c.n = {{F_c}}.n + Lambda/2 (U^- - U^+),   Lambda = max(|u^-|+c^-, |u^+|+c^+)
  Q*.n   = {{F_v}}.n - tau_IP (U^- - U^+),      [[U]] = (U^- - U^+) (x) n^-

where n is the outward normal of e and dA = |det J| |J^{-T} n_xi| w (eq.
IntegralsReferenceSpace).  The symmetry term comes from the auxiliary-variable
equation integrated by parts with U* = {{U}}: (U* - U^-) (x) n = -[[U]]/2 enters
the primal form with a plus sign, i.e. -1/2 on the left, +1/2 here.  Mass matrix
and body force use k+1 points per direction, the fluxes n_q points (Sec. 2.2.3).
dU/dt = L = M^{-1} R.

Readings where the paper is silent (listed with the design notes):
 * Lambda is evaluated pointwise at each face quadrature point.
 * the symmetry term uses each side's own state in G(U^-).
 * tau_IP,e (eq. TauIP_Element) uses areas and volume from the n_q-point rules;
   periodic faces count as interior faces; interior faces take the max over the
   two cells, wall faces the cell's own value.
 * walls (channel): mirror exterior state rho+ = rho-, u+ = -u-,
   T+ = 2 T_wall - T-, grad U+ = grad U-.
"""

import numpy as np
import torch

from . import rules
from . import mesh as meshmod
from . import physics as ph

CONVECTIVE = "c"
VISCOUS = "v"
FORCE = "f"

# Factor of the SIPG symmetry term 1/2 <grad V, F_v(U, [[U]])> (eq.
# WeakFormulationConservedVariables).  Module-level only so that a test can plant a
# wrong value and show that the symmetry pin detects it.
SYMMETRY_FACTOR = 0.5


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64)


class DGOperator:
    """Direct quadrature-point evaluation of the weak form on a BoxMesh.

    U is a float64 torch tensor of shape (5, n_cells, (k+1)^3):
    component, cell, node with the first coordinate fastest.
    """

    def __init__(self, mesh, fluid, n_q, basis="LGL", body_force=None, wall_T=None):
        self.mesh = mesh
        self.fl = fluid
        self.k = mesh.k
        self.n = self.k + 1
        self.N = self.n ** 3
        self.n_q = int(n_q)
        self.basis = basis
        self.body_force = None if body_force is None else np.asarray(body_force, dtype=np.float64)
        self.wall_T = wall_T
        self.nodes = rules.support_points(self.k, basis)
        self._geo_cache = {}

        xq, wq = rules.gauss_legendre(self.n_q)
        self.cell_pts, self.cell_w = meshmod.cell_points(xq, wq)
        Phi, dPhi = meshmod.tensor_basis(self.nodes, self.cell_pts)
        self.Phi, self.dPhi = _t(Phi), _t(dPhi)

        self.face = {}
        for d in range(3):
            for s in range(2):
                pts, w = meshmod.face_points(xq, wq, d, s)
                P, dP = meshmod.tensor_basis(self.nodes, pts)
                self.face[d, s] = (pts, _t(w), _t(P), _t(dP))

        xm, wm = rules.gauss_legendre(self.k + 1)
        self.mass_pts, self.mass_w = meshmod.cell_points(xm, wm)
        Pm, _ = meshmod.tensor_basis(self.nodes, self.mass_pts)
        self.Phi_m = _t(Pm)
        self._tau = np.full(mesh.n_cells, np.nan)
        if mesh.n_cells <= 64:
            # tiny meshes: all penalties up front, so that a residual evaluated
            # under a function transform (torch.func.jvp) never computes them
            self._penalty(np.arange(mesh.n_cells))

    # -- geometry ----------------------------------------------------------
    def _geometry(self, cells, pts):
        """x, J^{-1}, |det J| of the given cells at reference points pts (cached on small meshes)."""
        cells = np.asarray(cells, dtype=np.int64)
        key = None
        if self.mesh.n_cells <= 4096:
            key = (cells.tobytes(), np.asarray(pts).tobytes())
            hit = self._geo_cache.get(key)
            if hit is not None:
                return hit
        out = self._geometry_uncached(cells, pts)
        if key is not None:
            self._geo_cache[key] = out
        return out

    def _geometry_uncached(self, cells, pts):
        x, J = self.mesh.map_at(pts, cells)
        det = np.linalg.det(J)
        if not np.all(det > 0):
            raise ValueError("the cell mapping is folded (det J <= 0 at a quadrature point)")
        return _t(x), _t(np.linalg.inv(J)), _t(det)

    def _face_measure(self, Jinv, detJ, w, d, s):
        """Outward unit normal n and dA = |det J| |J^{-T} n_xi| w at face points."""
        sign = 1.0 if s == 1 else -1.0
        nn = sign * Jinv[..., d, :]                # (J^{-T} n_xi)_j = sum_a Jinv[a, j] n_xi[a]
        norm = torch.linalg.norm(nn, dim=-1)
        return nn / norm[..., None], detJ * norm * w

    @property
    def tau_cell(self):
        return self.tau_of(np.arange(self.mesh.n_cells))

    def tau_of(self, cells):
        """Penalty of the given cells, computed on first use."""
        cells = np.asarray(cells, dtype=np.int64)
        missing = np.unique(cells[np.isnan(self._tau[cells])])
        if len(missing):
            self._penalty(missing)
        return self._tau[cells]

    def _penalty(self, todo):
        """tau_IP,e = nu (k+1)^2 (A(interior)/2 + A(boundary)) / V(e)  (eq. TauIP_Element)."""
        tau = self._tau
        w = _t(self.cell_w)
        for c0 in range(0, len(todo), 2048):
            cells = todo[c0:c0 + 2048]
            _, _, detJ = self._geometry(cells, self.cell_pts)
            V = (detJ * w).sum(-1)
            A = torch.zeros(len(cells), dtype=torch.float64)
            for d in range(3):
                for s in range(2):
                    pts, wf, _, _ = self.face[d, s]
                    _, Jinv, dJ = self._geometry(cells, pts)
                    _, dA = self._face_measure(Jinv, dJ, wf, d, s)
                    boundary = torch.as_tensor(self.mesh.nb[cells, d, s] < 0)
                    A = A + torch.where(boundary, 1.0, 0.5) * dA.sum(-1)
            tau[cells] = (self.fl.nu * (self.k + 1) ** 2 * A / V).numpy()

    # -- evaluation at points ---------------------------------------------
    def _values(self, Ue, P, dP, Jinv):
        """U and physical grad U at points: Uq[e, p, c], Gx[e, p, c, j]."""
        Uq = torch.einsum("pi,cei->epc", P.to(Ue.dtype), Ue)
        Gr = torch.einsum("pid,cei->epcd", dP.to(Ue.dtype), Ue)
        Gx = torch.einsum("epdj,epcd->epcj", Jinv.to(Ue.dtype), Gr)
        return Uq, Gx

    def _mirror(self, Um, Gm):
        """Wall exterior state: rho+ = rho-, u+ = -u-, T+ = 2 T_wall - T-, grad U+ = grad U-."""
        fl = self.fl
        rho = Um[..., 0]
        u = ph.velocity(Um)
        T = ph.temperature(Um, fl)
        Tp = 2.0 * self.wall_T - T
        Up = torch.zeros_like(Um)
        Up[..., 0] = rho
        Up[..., 1:4] = -Um[..., 1:4]
        Up[..., 4] = rho * (fl.c_v * Tp + 0.5 * (u * u).sum(-1))
        return Up, Gm

    # -- the residual --------------------------------------------------------
    def residual(self, U, cells=None, terms="cvf", source=None, t=0.0, chunk=512):
        """R = -F_c - F_v + F_rhs tested against every basis function of the given cells.

        terms: any of 'c' (convective cell+face), 'v' (viscous cell+face),
        'f' (body force).  source(x, t) -> (..., 5) adds a volume source
        integrated with the n_q rule (manufactured solutions; tests only).
        Returns a tensor (5, len(cells), N).
        """
        E = self.mesh.n_cells
        cells = np.arange(E) if cells is None else np.asarray(cells, dtype=np.int64)
        out = []
        for c0 in range(0, len(cells), chunk):
            out.append(self._residual_chunk(U, cells[c0:c0 + chunk], terms, source, t))
        return torch.cat(out, dim=1)

    def _residual_chunk(self, U, cells, terms, source, t):
        fl = self.fl
        Ue = U[:, cells, :]
        R = torch.zeros_like(Ue)
        w = _t(self.cell_w)

        # cell integrals: + (grad phi_i, F_c - F_v)
        x, Jinv, detJ = self._geometry(cells, self.cell_pts)
        if CONVECTIVE in terms or VISCOUS in terms:
            Uq, Gx = self._values(Ue, self.Phi, self.dPhi, Jinv)
            F = torch.zeros(Uq.shape + (3,), dtype=Uq.dtype)
            if CONVECTIVE in terms:
                F = F + ph.convective_flux(Uq, fl)
            if VISCOUS in terms:
                F = F - ph.viscous_flux(Uq, Gx, fl)
            Fref = torch.einsum("epdj,epcj->epcd", Jinv.to(F.dtype), F) * (detJ * w)[..., None, None]
            R = R + torch.einsum("pid,epcd->cei", self.dPhi.to(F.dtype), Fref)
        if source is not None:
            S = source(x.numpy(), t)
            S = torch.as_tensor(S, dtype=torch.float64) * (detJ * w)[..., None]
            R = R + torch.einsum("pi,epc->cei", self.Phi, S).to(R.dtype)

        # face integrals (each cell tests its own six faces)
        if CONVECTIVE in terms or VISCOUS in terms:
            for d in range(3):
                for s in range(2):
                    R = R + self._face_term(U, Ue, cells, d, s, terms)

        # body force with the k+1 rule
        if FORCE in terms and self.body_force is not None:
            _, _, detJm = self._geometry(cells, self.mass_pts)
            Um = torch.einsum("pi,cei->epc", self.Phi_m.to(Ue.dtype), Ue)
            Sf = ph.body_force_source(Um, self.body_force) * (detJm * _t(self.mass_w))[..., None]
            R = R + torch.einsum("pi,epc->cei", self.Phi_m.to(Sf.dtype), Sf)
        return R

    def _face_term(self, U, Ue, cells, d, s, terms):
        fl = self.fl
        pts, wf, P, dP = self.face[d, s]
        pts_n, _, Pn, dPn = self.face[d, 1 - s]
        _, Jinv, detJ = self._geometry(cells, pts)
        nrm, dA = self._face_measure(Jinv, detJ, wf, d, s)
        Um, Gm = self._values(Ue, P, dP, Jinv)

        nbr = self.mesh.nb[cells, d, s]
        wall = nbr < 0
        nbr_safe = np.where(wall, cells, nbr)
        _, Jinv_n, _ = self._geometry(nbr_safe, pts_n)
        Up, Gp = self._values(U[:, nbr_safe, :], Pn, dPn, Jinv_n)
        tau = self.tau_of(cells)
        if wall.any():
            if self.wall_T is None:
                raise ValueError("wall faces need wall_T")
            Uw, Gw = self._mirror(Um, Gm)
            wmask = torch.as_tensor(wall)
            Up = torch.where(wmask[:, None, None], Uw, Up)
            Gp = torch.where(wmask[:, None, None, None], Gw, Gp)
        tau = _t(np.where(wall, tau, np.maximum(tau, self.tau_of(nbr_safe))))

        jump = Um - Up
        val = torch.zeros_like(Um)
        grad = torch.zeros(Um.shape + (3,), dtype=Um.dtype)
        n_ = nrm.to(Um.dtype)
        if CONVECTIVE in terms:
            Fm = ph.convective_flux(Um, fl)
            Fp = ph.convective_flux(Up, fl)
            lam_m = torch.linalg.norm(ph.velocity(Um), dim=-1) + ph.speed_of_sound(Um, fl)
            lam_p = torch.linalg.norm(ph.velocity(Up), dim=-1) + ph.speed_of_sound(Up, fl)
            Lam = torch.maximum(lam_m, lam_p)
            Chat = 0.5 * torch.einsum("epcj,epj->epc", Fm + Fp, n_) + 0.5 * Lam[..., None] * jump
            val = val - Chat
        if VISCOUS in terms:
            Vm = ph.viscous_flux(Um, Gm, fl)
            Vp = ph.viscous_flux(Up, Gp, fl)
            Qhat = 0.5 * torch.einsum("epcj,epj->epc", Vm + Vp, n_) - tau[:, None, None].to(Um.dtype) * jump
            val = val + Qhat
            delta = jump[..., :, None] * n_[..., None, :]
            grad = grad + SYMMETRY_FACTOR * ph.viscous_flux(Um, delta, fl)

        dA_ = dA.to(Um.dtype)
        Rf = torch.einsum("pi,epc->cei", P.to(Um.dtype), val * dA_[..., None])
        gref = torch.einsum("epdj,epcj->epcd", Jinv.to(Um.dtype), grad) * dA_[..., None, None]
        Rf = Rf + torch.einsum("pid,epcd->cei", dP.to(Um.dtype), gref)
        return Rf

    # -- mass matrix -----------------------------------------------------------
    def mass_matrices(self, cells=None):
        """M_e[i, j] = sum over the (k+1)^3 Gauss points of w |det J| phi_i phi_j (Sec. 2.2.3)."""
        cells = np.arange(self.mesh.n_cells) if cells is None else np.asarray(cells)
        _, _, detJ = self._geometry(cells, self.mass_pts)
        W = detJ * _t(self.mass_w)
        return torch.einsum("pi,ep,pj->eij", self.Phi_m, W, self.Phi_m)

    def apply_inverse_mass(self, R, cells=None):
        """M^{-1} R cell by cell via a Cholesky solve of the dense block."""
        M = self.mass_matrices(cells)
        Lc = torch.linalg.cholesky(M)
        rhs = R.permute(1, 2, 0)                      # (E, N, 5)
        return torch.cholesky_solve(rhs, Lc).permute(2, 0, 1)

    def apply(self, U, cells=None, terms="cvf", source=None, t=0.0):
        """L(U) = M^{-1} R(U) (Sec. 2.4, eq. SpatiallyDiscretizedProblem)."""
        return self.apply_inverse_mass(self.residual(U, cells, terms, source, t), cells)

    # -- helpers --------------------------------------------------------------
    def physical_cell_points(self):
        x, _, _ = self._geometry(np.arange(self.mesh.n_cells), self.cell_pts)
        return x
