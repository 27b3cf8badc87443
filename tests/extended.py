"""Extended-precision evaluation of the DG residual for a few cells (test infrastructure).

Used to MEASURE the float64 rounding floor of the oracle and of the HIP path: both are
compared with this evaluation, which carries every step in x87 extended precision
(numpy.longdouble: 64-bit significand, unit roundoff 5.4e-20, about 2000 times below
float64's).  The float64 input coefficients and mesh parameters are taken as exact
numbers, so the difference of a float64 evaluation from this one is that evaluation's
own rounding error (to within about 1e-3 of it).

It is written on its own, not derived from the oracle: Gauss and Gauss-Lobatto points
by Newton iteration on the Legendre recurrence in extended precision, Lagrange
matrices by the product formula, the isoparametric map of the paper's meshes, the
weak form of Sec. 2.2.2, eq. (WeakFormulationConservedVariables) tested against the
cell's own basis (element-centric), local Lax-Friedrichs flux with the pointwise wave
speed, SIPG with the penalty of eq. (TauIP_Element) (periodic faces interior, interior
faces the max of both cells), the symmetry term with each side's own state, mirror
states at isothermal walls, body force and mass matrix on k+1 points (Sec. 2.2.3),
and M^{-1} R by Gaussian elimination in extended precision.
"""

import numpy as np
from numpy.polynomial import legendre as npleg

LD = np.longdouble
assert np.finfo(LD).eps < 1e-18, "numpy.longdouble is not an extended type on this platform"

AFFINE, CHANNEL, CURVED = 0, 1, 2


# ---------------------------------------------------------------- 1D rules


def _legendre(n, x):
    """P_n(x), P_n'(x) by the three-term recurrence (x in [-1, 1])."""
    p0, p1 = np.ones_like(x), x.copy()
    if n == 0:
        return p0, np.zeros_like(x)
    for m in range(1, n):
        p0, p1 = p1, ((2 * m + 1) * x * p1 - m * p0) / (m + 1)
    dp = n * (x * p1 - p0) / (x * x - 1)
    return p1, dp


def gauss(n):
    """n Gauss-Legendre points and weights on [0, 1], refined by Newton in extended precision."""
    x = np.asarray(npleg.leggauss(n)[0], dtype=LD)
    for _ in range(6):
        p, dp = _legendre(n, x)
        x = x - p / dp
    _, dp = _legendre(n, x)
    w = 2 / ((1 - x * x) * dp * dp)
    return (x + 1) / 2, w / 2


def lobatto(n):
    """n Gauss-Lobatto points on [0, 1]: the ends and the roots of P'_{n-1} (Newton refined)."""
    m = n - 1
    if n == 2:
        return np.array([LD(0), LD(1)])
    c = np.zeros(n)
    c[-1] = 1.0
    x = np.sort(np.real(npleg.legroots(npleg.legder(c)))).astype(LD)
    for _ in range(6):
        p, dp = _legendre(m, x)
        ddp = (2 * x * dp - m * (m + 1) * p) / (1 - x * x)     # Legendre's equation
        x = x - dp / ddp
    return np.concatenate(([LD(0)], (x + 1) / 2, [LD(1)]))


def lagrange(nodes, pts):
    """V[p, i] = l_i(pts[p]) and D[p, i] = l_i'(pts[p]) of the Lagrange basis on nodes."""
    nodes = np.asarray(nodes, dtype=LD)
    pts = np.asarray(pts, dtype=LD)
    n = len(nodes)
    V = np.ones((len(pts), n), dtype=LD)
    D = np.zeros((len(pts), n), dtype=LD)
    for i in range(n):
        for j in range(n):
            if j != i:
                V[:, i] *= (pts - nodes[j]) / (nodes[i] - nodes[j])
        for m in range(n):
            if m == i:
                continue
            t = np.full(len(pts), 1 / (nodes[i] - nodes[m]), dtype=LD)
            for j in range(n):
                if j != i and j != m:
                    t *= (pts - nodes[j]) / (nodes[i] - nodes[j])
            D[:, i] += t
    return V, D


def tensor(V, D, idx):
    """3D basis values and reference gradients at the tensor points idx[p] = (p0, p1, p2).

    V, D are 1D matrices [point, node]; basis index i = a0 + n (a1 + n a2)."""
    n = V.shape[1]
    P = len(idx)
    Phi = np.zeros((P, n ** 3), dtype=LD)
    dPhi = np.zeros((P, n ** 3, 3), dtype=LD)
    for a2 in range(n):
        for a1 in range(n):
            for a0 in range(n):
                i = a0 + n * (a1 + n * a2)
                v0, v1, v2 = V[idx[:, 0], a0], V[idx[:, 1], a1], V[idx[:, 2], a2]
                d0, d1, d2 = D[idx[:, 0], a0], D[idx[:, 1], a1], D[idx[:, 2], a2]
                Phi[:, i] = v0 * v1 * v2
                dPhi[:, i, 0] = d0 * v1 * v2
                dPhi[:, i, 1] = v0 * d1 * v2
                dPhi[:, i, 2] = v0 * v1 * d2
    return Phi, dPhi


# ---------------------------------------------------------------- the evaluator


class Extended:
    """Residual R_e = -F_c - F_v + F_rhs of chosen cells of a box mesh, in extended precision.

    Mesh and fluid as in the library: n cells per direction on [lo, hi], periodic flags
    (walls otherwise), kind AFFINE / CHANNEL (tanh stretching C in x1) / CURVED (warp of
    amplitude amp), isoparametric degree k with LGL geometry nodes; basis LGL or GL."""

    def __init__(self, n, lo, hi, k, nq, basis="LGL", periodic=(1, 1, 1), kind=AFFINE, stretch_C=1.8,
                 amp=0.0, gamma=1.4, R=287.0, mu=0.0, lam=0.0, rho_ref=1.0, wall_T=None, body_force=None):
        self.n = tuple(int(v) for v in n)
        self.lo = np.array([LD(v) for v in lo])
        self.hi = np.array([LD(v) for v in hi])
        self.k, self.nq, self.N = k, nq, (k + 1) ** 3
        self.periodic = tuple(bool(p) for p in periodic)
        self.kind, self.C, self.amp = kind, LD(stretch_C), LD(amp)
        self.g, self.R, self.mu, self.lam = LD(gamma), LD(R), LD(mu), LD(lam)
        self.nu = LD(mu) / LD(rho_ref)
        self.wall_T = None if wall_T is None else LD(wall_T)
        self.f = None if body_force is None or not any(body_force) else np.array([LD(v) for v in body_force])
        gn = lobatto(k + 1)
        self.gnodes = gn
        self.nodes = gn if basis == "LGL" else gauss(k + 1)[0]
        self.qx, self.qw = gauss(nq)
        self.mx, self.mw = gauss(k + 1)
        q = nq
        cell_idx = np.array([(p0, p1, p2) for p2 in range(q) for p1 in range(q) for p0 in range(q)])
        self.cw = self.qw[cell_idx[:, 0]] * self.qw[cell_idx[:, 1]] * self.qw[cell_idx[:, 2]]
        V, D = lagrange(self.nodes, self.qx)
        self.Phi, self.dPhi = tensor(V, D, cell_idx)
        Vg, Dg = lagrange(gn, self.qx)
        self.gPhi, self.gdPhi = tensor(Vg, Dg, cell_idx)
        # faces: the points of face xi_d = s, tangential axes in increasing order, lower fastest
        ends = np.array([LD(0), LD(1)])
        Ve, De = lagrange(self.nodes, ends)
        Vge, Dge = lagrange(gn, ends)
        self.face = {}
        for d in range(3):
            t0, t1 = [a for a in range(3) if a != d]
            for s in (0, 1):
                idx = np.zeros((q * q, 3), dtype=int)
                w = np.zeros(q * q, dtype=LD)
                for r1 in range(q):
                    for r0 in range(q):
                        p = r0 + q * r1
                        idx[p, t0], idx[p, t1], idx[p, d] = r0, r1, 0
                        w[p] = self.qw[r0] * self.qw[r1]
                # per axis the 1D matrix to use: quadrature points along t0, t1, the end s along d
                self.face[d, s] = (self._face_tensor(V, D, Ve, De, idx, d, s),
                                   self._face_tensor(Vg, Dg, Vge, Dge, idx, d, s), w)
        m_idx = np.array([(p0, p1, p2) for p2 in range(k + 1) for p1 in range(k + 1) for p0 in range(k + 1)])
        self.mwt = self.mw[m_idx[:, 0]] * self.mw[m_idx[:, 1]] * self.mw[m_idx[:, 2]]
        Vm, Dm = lagrange(self.nodes, self.mx)
        self.mPhi, _ = tensor(Vm, Dm, m_idx)
        Vgm, Dgm = lagrange(gn, self.mx)
        self.mgPhi, self.mgdPhi = tensor(Vgm, Dgm, m_idx)
        self._X = {}
        self._tau = {}

    def _face_tensor(self, V, D, Ve, De, idx, d, s):
        n = V.shape[1]
        P = len(idx)
        Phi = np.zeros((P, n ** 3), dtype=LD)
        dPhi = np.zeros((P, n ** 3, 3), dtype=LD)
        mats = []
        for ax in range(3):
            if ax == d:
                mats.append((np.repeat(Ve[s:s + 1], P, 0), np.repeat(De[s:s + 1], P, 0)))
            else:
                mats.append((V[idx[:, ax]], D[idx[:, ax]]))
        for a2 in range(n):
            for a1 in range(n):
                for a0 in range(n):
                    i = a0 + n * (a1 + n * a2)
                    a = (a0, a1, a2)
                    v = [mats[ax][0][:, a[ax]] for ax in range(3)]
                    dv = [mats[ax][1][:, a[ax]] for ax in range(3)]
                    Phi[:, i] = v[0] * v[1] * v[2]
                    dPhi[:, i, 0] = dv[0] * v[1] * v[2]
                    dPhi[:, i, 1] = v[0] * dv[1] * v[2]
                    dPhi[:, i, 2] = v[0] * v[1] * dv[2]
        return Phi, dPhi

    # ---- mesh
    def _box_map(self, s):
        L = self.hi - self.lo
        x = self.lo + L * s
        if self.kind == CHANNEL:
            C = self.C
            x[..., 1] = self.lo[1] + L[1] * (1 + np.tanh(C * (2 * s[..., 1] - 1)) / np.tanh(C)) / 2
        elif self.kind == CURVED:
            pi = np.arccos(LD(-1))
            b = self.amp * np.sin(2 * pi * s[..., 0]) * np.sin(2 * pi * s[..., 1]) * np.sin(2 * pi * s[..., 2])
            x = x + b[..., None]
        return x

    def ijk(self, e):
        return e % self.n[0], (e // self.n[0]) % self.n[1], e // (self.n[0] * self.n[1])

    def X(self, e):
        """Geometry nodes (N, 3) of cell e: the box map at its LGL points."""
        if e not in self._X:
            c = self.ijk(e)
            k1 = self.k + 1
            s = np.zeros((k1 ** 3, 3), dtype=LD)
            for a2 in range(k1):
                for a1 in range(k1):
                    for a0 in range(k1):
                        i = a0 + k1 * (a1 + k1 * a2)
                        for ax, a in enumerate((a0, a1, a2)):
                            s[i, ax] = (LD(c[ax]) + self.gnodes[a]) / LD(self.n[ax])
            self._X[e] = self._box_map(s)
        return self._X[e]

    def neighbor(self, e, d, s):
        c = list(self.ijk(e))
        c[d] += 1 if s == 1 else -1
        if c[d] < 0 or c[d] >= self.n[d]:
            if not self.periodic[d]:
                return None
            c[d] %= self.n[d]
        return c[0] + self.n[0] * (c[1] + self.n[1] * c[2])

    @staticmethod
    def _jac(X, gPhi, gdPhi):
        J = np.einsum("pid,ic->pcd", gdPhi, X)         # J[p, c, d] = dx_c / dxi_d
        det = (J[:, 0, 0] * (J[:, 1, 1] * J[:, 2, 2] - J[:, 1, 2] * J[:, 2, 1])
               - J[:, 0, 1] * (J[:, 1, 0] * J[:, 2, 2] - J[:, 1, 2] * J[:, 2, 0])
               + J[:, 0, 2] * (J[:, 1, 0] * J[:, 2, 1] - J[:, 1, 1] * J[:, 2, 0]))
        # inverse by cofactors: Jinv[p, d, c] = cof(J)[p, c, d] / det
        cof = np.zeros_like(J)
        for a in range(3):
            for b in range(3):
                r = [i for i in range(3) if i != a]
                cc = [j for j in range(3) if j != b]
                m = J[:, r[0], cc[0]] * J[:, r[1], cc[1]] - J[:, r[0], cc[1]] * J[:, r[1], cc[0]]
                cof[:, a, b] = m if (a + b) % 2 == 0 else -m
        Jinv = np.transpose(cof, (0, 2, 1)) / det[:, None, None]
        return Jinv, det

    # ---- physics
    def _prim(self, U):
        rho = U[:, 0]
        u = U[:, 1:4] / rho[:, None]
        p = (self.g - 1) * (U[:, 4] - rho * (u * u).sum(1) / 2)
        return rho, u, p

    def _fc(self, U):
        rho, u, p = self._prim(U)
        F = np.zeros((len(U), 5, 3), dtype=LD)
        F[:, 0] = U[:, 1:4]
        F[:, 1:4] = U[:, 1:4, None] * u[:, None, :]
        for a in range(3):
            F[:, 1 + a, a] += p
        F[:, 4] = (U[:, 4] + p)[:, None] * u
        return F

    def _fv(self, U, G):
        """Viscous flux with the gradient slot G[p, c, j] (linear in G)."""
        rho, u, p = self._prim(U)
        du = (G[:, 1:4, :] - u[:, :, None] * G[:, 0:1, :]) / rho[:, None, None]
        # T = p / (rho R) with p from rho E: dT = ((g-1)(dE - u.dm + |u|^2/2 drho) rho - p drho) / (rho^2 R)
        uu = (u * u).sum(1)
        dp = (self.g - 1) * (G[:, 4, :] - np.einsum("pa,paj->pj", u, G[:, 1:4, :]) + (uu / 2)[:, None] * G[:, 0, :])
        dT = (dp * rho[:, None] - p[:, None] * G[:, 0, :]) / ((rho * rho * self.R)[:, None])
        div = du[:, 0, 0] + du[:, 1, 1] + du[:, 2, 2]
        tau = self.mu * (du + np.transpose(du, (0, 2, 1)))
        for a in range(3):
            tau[:, a, a] -= self.mu * 2 * div / 3
        F = np.zeros((len(U), 5, 3), dtype=LD)
        F[:, 1:4] = tau
        F[:, 4] = np.einsum("pja,pa->pj", tau, u) + self.lam * dT
        return F

    def _mirror(self, U):
        rho, u, p = self._prim(U)
        T = p / (rho * self.R)
        Tp = 2 * self.wall_T - T
        W = np.zeros_like(U)
        W[:, 0] = rho
        W[:, 1:4] = -U[:, 1:4]
        W[:, 4] = rho * (self.R / (self.g - 1) * Tp + (u * u).sum(1) / 2)
        return W

    # ---- penalty
    def tau(self, e):
        if e not in self._tau:
            X = self.X(e)
            _, det = self._jac(X, self.gPhi, self.gdPhi)
            V = (np.abs(det) * self.cw).sum()
            A = LD(0)
            for d in range(3):
                for s in (0, 1):
                    _, (gP, gdP), w = self.face[d, s]
                    Jinv, det_f = self._jac(X, gP, gdP)
                    area = np.abs(det_f) * np.sqrt((Jinv[:, d, :] ** 2).sum(1)) * w
                    A += (LD(1) if self.neighbor(e, d, s) is None else LD(0.5)) * area.sum()
            self._tau[e] = self.nu * (self.k + 1) ** 2 * A / V
        return self._tau[e]

    # ---- residual of one cell
    def residual_cell(self, U, e, terms="cvf"):
        """R_e (5, N) in extended precision; U (5, E, N) float64 coefficients."""
        conv, visc = "c" in terms, "v" in terms
        Ue = np.asarray(U[:, e, :], dtype=LD).T                       # (N, 5)
        X = self.X(e)
        R = np.zeros((self.N, 5), dtype=LD)
        if conv or visc:
            Jinv, det = self._jac(X, self.gPhi, self.gdPhi)
            Uq = self.Phi @ Ue
            Gr = np.einsum("pid,ic->pcd", self.dPhi, Ue)
            G = np.einsum("pcd,pdj->pcj", Gr, Jinv)
            F = np.zeros((len(Uq), 5, 3), dtype=LD)
            if conv:
                F += self._fc(Uq)
            if visc:
                F -= self._fv(Uq, G)
            # grad_x phi_i . F_c = sum_d dphi_i/dxi_d sum_j Jinv[d, j] F[c, j]
            Fr = np.einsum("pdj,pcj->pcd", Jinv, F) * (np.abs(det) * self.cw)[:, None, None]
            R += np.einsum("pid,pcd->ic", self.dPhi, Fr)
            for d in range(3):
                for s in (0, 1):
                    R += self._face(U, e, X, d, s, conv, visc)
        if "f" in terms and self.f is not None:
            _, det = self._jac(X, self.mgPhi, self.mgdPhi)
            Um = self.mPhi @ Ue
            u = Um[:, 1:4] / Um[:, 0:1]
            S = np.zeros((len(Um), 5), dtype=LD)
            S[:, 1:4] = self.f[None, :]
            S[:, 4] = u @ self.f
            R += self.mPhi.T @ (S * (np.abs(det) * self.mwt)[:, None])
        return R.T

    def _face(self, U, e, X, d, s, conv, visc):
        (P, dP), (gP, gdP), w = self.face[d, s]
        Jinv, det = self._jac(X, gP, gdP)
        sign = LD(1) if s == 1 else LD(-1)
        nn = sign * Jinv[:, d, :]                        # J^{-T} n_xi
        nrm = np.sqrt((nn * nn).sum(1))
        n = nn / nrm[:, None]
        dA = np.abs(det) * nrm * w
        Ue = np.asarray(U[:, e, :], dtype=LD).T
        Um = P @ Ue
        Gm = np.einsum("pcd,pdj->pcj", np.einsum("pid,ic->pcd", dP, Ue), Jinv)
        f = self.neighbor(e, d, s)
        if f is None:
            Up, Gp = self._mirror(Um), Gm
            tau = self.tau(e)
        else:
            (Pn, dPn), (gPn, gdPn), _ = self.face[d, 1 - s]
            Jn, _ = self._jac(self.X(f), gPn, gdPn)
            Uf = np.asarray(U[:, f, :], dtype=LD).T
            Up = Pn @ Uf
            Gp = np.einsum("pcd,pdj->pcj", np.einsum("pid,ic->pcd", dPn, Uf), Jn)
            tau = max(self.tau(e), self.tau(f))
        jump = Um - Up
        val = np.zeros_like(Um)
        sym = np.zeros((len(Um), 5, 3), dtype=LD)
        if conv:
            Fm, Fp = self._fc(Um), self._fc(Up)
            _, um, pm = self._prim(Um)
            _, up, pp = self._prim(Up)
            lm = np.sqrt((um * um).sum(1)) + np.sqrt(np.abs(self.g * pm / Um[:, 0]))
            lp = np.sqrt((up * up).sum(1)) + np.sqrt(np.abs(self.g * pp / Up[:, 0]))
            lam = np.maximum(lm, lp)
            val -= np.einsum("pcj,pj->pc", Fm + Fp, n) / 2 + (lam / 2)[:, None] * jump
        if visc:
            Vm, Vp = self._fv(Um, Gm), self._fv(Up, Gp)
            val += np.einsum("pcj,pj->pc", Vm + Vp, n) / 2 - tau * jump
            sym = self._fv(Um, jump[:, :, None] * n[:, None, :]) / 2
        Rf = P.T @ (val * dA[:, None])
        symr = np.einsum("pdj,pcj->pcd", Jinv, sym) * dA[:, None, None]
        Rf += np.einsum("pid,pcd->ic", dP, symr)
        return Rf

    # ---- mass matrix
    def inverse_mass(self, e, R):
        """M_e^{-1} R (5, N) by Gaussian elimination with partial pivoting, extended precision."""
        _, det = self._jac(self.X(e), self.mgPhi, self.mgdPhi)
        M = self.mPhi.T @ (self.mPhi * (np.abs(det) * self.mwt)[:, None])
        A = np.concatenate([M, np.asarray(R, dtype=LD).T], axis=1)
        n = len(M)
        for c in range(n):
            piv = c + int(np.argmax(np.abs(A[c:, c])))
            if piv != c:
                A[[c, piv]] = A[[piv, c]]
            A[c + 1:] -= np.outer(A[c + 1:, c] / A[c, c], A[c])
        x = np.zeros((n, A.shape[1] - n), dtype=LD)
        for c in range(n - 1, -1, -1):
            x[c] = (A[c, n:] - A[c, c + 1:n] @ x[c + 1:]) / A[c, c]
        return x.T

    def residual(self, U, cells, terms="cvf"):
        """R of the given cells, shape (5, len(cells), N), extended precision."""
        return np.stack([self.residual_cell(U, int(e), terms) for e in cells], axis=1)

    def operator(self, U, cells):
        """L = M^{-1} R of the given cells (5, len(cells), N), extended precision."""
        return np.stack([self.inverse_mass(int(e), self.residual_cell(U, int(e))) for e in cells], axis=1)
