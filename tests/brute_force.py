"""Brute-force scalar evaluation of the DG residual, used only to pin the oracle.

Pure Python floats and loops, nothing vectorised and nothing shared with the
oracle except the problem statement:
  * its own 1D rules (Golub-Welsch eigenvalues for Gauss points, numpy roots for
    the LGL points), Lagrange polynomials evaluated one value at a time;
  * its own geometry: nodes placed by its own copy of the box maps, J by loops,
    J^{-1} and the face normal from the cofactor matrix;
  * its own physics: velocity and temperature gradients via grad p
    (p = (gamma-1)(rho E - |m|^2/(2 rho)), T = p/(rho R)), not via grad E;
  * face-centric: each face is visited once and both cells' terms are added.
Intended for meshes of a handful of cells (seconds of run time).
"""

import math

import numpy as np


def gauss_points(n):
    # Golub-Welsch: eigenvalues of the Jacobi matrix of the Legendre recurrence
    if n == 1:
        return [0.5], [1.0]
    beta = [k / math.sqrt(4.0 * k * k - 1.0) for k in range(1, n)]
    T = np.diag(beta, 1) + np.diag(beta, -1)
    lam, vec = np.linalg.eigh(T)
    pts = [0.5 * (1.0 + float(l)) for l in lam]
    wts = [float(vec[0, i]) ** 2 for i in range(n)]      # sums to 1 on [0,1] after the mapping
    return pts, wts


def lobatto_points(n):
    # roots of (1 - x^2) P'_{n-1}(x) via numpy.roots of the power series
    P = [np.poly1d([1.0]), np.poly1d([1.0, 0.0])]
    for m in range(1, n - 1):
        P.append(((2 * m + 1) * np.poly1d([1.0, 0.0]) * P[m] - m * P[m - 1]) / (m + 1))
    inner = sorted(float(r.real) for r in np.roots(P[n - 1].deriv())) if n > 2 else []
    return [0.0] + [0.5 * (1.0 + r) for r in inner] + [1.0]


def lag(nodes, i, x):
    v = 1.0
    for j, xj in enumerate(nodes):
        if j != i:
            v *= (x - xj) / (nodes[i] - xj)
    return v


def dlag(nodes, i, x):
    tot = 0.0
    for m, xm in enumerate(nodes):
        if m == i:
            continue
        v = 1.0 / (nodes[i] - xm)
        for j, xj in enumerate(nodes):
            if j != i and j != m:
                v *= (x - xj) / (nodes[i] - xj)
        tot += v
    return tot


def det3(A):
    return (A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1])
            - A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0])
            + A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]))


def cofactor(A):
    C = [[0.0] * 3 for _ in range(3)]
    for i in range(3):
        for j in range(3):
            r = [a for a in range(3) if a != i]
            c = [b for b in range(3) if b != j]
            m = A[r[0]][c[0]] * A[r[1]][c[1]] - A[r[0]][c[1]] * A[r[1]][c[0]]
            C[i][j] = m if (i + j) % 2 == 0 else -m
    return C


class BruteForce:
    def __init__(self, n, lo, hi, k, nq, basis="LGL", periodic=(True, True, True), kind=0,
                 stretch_C=1.8, amp=0.0, gamma=1.4, R=287.0, mu=0.0, lam=0.0, rho_ref=1.0,
                 wall_T=None, body_force=None):
        self.n, self.lo, self.hi, self.k, self.nq = n, lo, hi, k, nq
        self.periodic, self.kind, self.C, self.amp = periodic, kind, stretch_C, amp
        self.gamma, self.R, self.mu, self.lam, self.nu = gamma, R, mu, lam, mu / rho_ref
        self.wall_T, self.f = wall_T, body_force
        self.nodes = lobatto_points(k + 1) if basis == "LGL" else gauss_points(k + 1)[0]
        self.gnodes = lobatto_points(k + 1)
        self.qx, self.qw = gauss_points(nq)
        self.mx, self.mw = gauss_points(k + 1)
        self.E = n[0] * n[1] * n[2]
        self.nb1 = k + 1

    # ---- mesh ----
    def gmap(self, s):
        x = [self.lo[d] + (self.hi[d] - self.lo[d]) * s[d] for d in range(3)]
        if self.kind == 1:
            x[1] = self.lo[1] + (self.hi[1] - self.lo[1]) * 0.5 * (1 + math.tanh(self.C * (2 * s[1] - 1)) / math.tanh(self.C))
        elif self.kind == 2:
            b = self.amp * math.sin(2 * math.pi * s[0]) * math.sin(2 * math.pi * s[1]) * math.sin(2 * math.pi * s[2])
            x = [v + b for v in x]
        return x

    def ijk(self, e):
        return e % self.n[0], (e // self.n[0]) % self.n[1], e // (self.n[0] * self.n[1])

    def cell_index(self, i, j, k):
        return i + self.n[0] * (j + self.n[1] * k)

    def geo(self, e, xi):
        """x and J at reference point xi of cell e (isoparametric, degree k, LGL nodes)."""
        c = self.ijk(e)
        g, nb = self.gnodes, self.nb1
        x = [0.0] * 3
        J = [[0.0] * 3 for _ in range(3)]
        for a2 in range(nb):
            for a1 in range(nb):
                for a0 in range(nb):
                    X = self.gmap([(c[0] + g[a0]) / self.n[0], (c[1] + g[a1]) / self.n[1], (c[2] + g[a2]) / self.n[2]])
                    v = [lag(g, a0, xi[0]), lag(g, a1, xi[1]), lag(g, a2, xi[2])]
                    dv = [dlag(g, a0, xi[0]), dlag(g, a1, xi[1]), dlag(g, a2, xi[2])]
                    phi = v[0] * v[1] * v[2]
                    grad = [dv[0] * v[1] * v[2], v[0] * dv[1] * v[2], v[0] * v[1] * dv[2]]
                    for i in range(3):
                        x[i] += X[i] * phi
                        for j in range(3):
                            J[i][j] += X[i] * grad[j]
        return x, J

    def basis_at(self, xi):
        """[(node, phi, grad_xi phi)] for all basis functions at xi."""
        out = []
        nd, nb = self.nodes, self.nb1
        for a2 in range(nb):
            for a1 in range(nb):
                for a0 in range(nb):
                    v = [lag(nd, a0, xi[0]), lag(nd, a1, xi[1]), lag(nd, a2, xi[2])]
                    dv = [dlag(nd, a0, xi[0]), dlag(nd, a1, xi[1]), dlag(nd, a2, xi[2])]
                    out.append((a0 + nb * (a1 + nb * a2), v[0] * v[1] * v[2],
                                [dv[0] * v[1] * v[2], v[0] * dv[1] * v[2], v[0] * v[1] * dv[2]]))
        return out

    # ---- physics (primitive route) ----
    def fluxes(self, U, G, want_visc=True):
        g, R = self.gamma, self.R
        rho, m, rE = U[0], U[1:4], U[4]
        u = [mi / rho for mi in m]
        ke = 0.5 * sum(mi * mi for mi in m) / rho
        p = (g - 1) * (rE - ke)
        Fc = [[0.0] * 3 for _ in range(5)]
        for j in range(3):
            Fc[0][j] = m[j]
            for a in range(3):
                Fc[1 + a][j] = m[a] * u[j] + (p if a == j else 0.0)
            Fc[4][j] = (rE + p) * u[j]
        Fv = [[0.0] * 3 for _ in range(5)]
        if want_visc:
            # du_a/dx_j = (dm_a/dx_j - u_a drho/dx_j) / rho
            du = [[(G[1 + a][j] - u[a] * G[0][j]) / rho for j in range(3)] for a in range(3)]
            # dp/dx_j = (g-1) (d rhoE/dx_j - sum_a u_a dm_a/dx_j + |u|^2/2 drho/dx_j)
            uu = sum(ui * ui for ui in u)
            dp = [(g - 1) * (G[4][j] - sum(u[a] * G[1 + a][j] for a in range(3)) + 0.5 * uu * G[0][j]) for j in range(3)]
            # T = p/(rho R): dT = (dp rho - p drho) / (rho^2 R)
            dT = [(dp[j] * rho - p * G[0][j]) / (rho * rho * R) for j in range(3)]
            div = du[0][0] + du[1][1] + du[2][2]
            tau = [[self.mu * (du[a][b] + du[b][a] - (2.0 / 3.0) * div * (1.0 if a == b else 0.0)) for b in range(3)] for a in range(3)]
            for j in range(3):
                for a in range(3):
                    Fv[1 + a][j] = tau[a][j]
                Fv[4][j] = sum(tau[j][a] * u[a] for a in range(3)) + self.lam * dT[j]
        return Fc, Fv, p, u

    def trace(self, Ue, e, xi):
        """U and physical grad U of cell e at reference point xi, plus x, J^{-1}, det J."""
        x, J = self.geo(e, xi)
        dJ = det3(J)
        C = cofactor(J)
        Jinv = [[C[j][i] / dJ for j in range(3)] for i in range(3)]     # inverse = adj / det
        U = [0.0] * 5
        Gr = [[0.0] * 3 for _ in range(5)]
        for (idx, phi, gphi) in self.basis_at(xi):
            for c in range(5):
                U[c] += Ue[c][idx] * phi
                for d in range(3):
                    Gr[c][d] += Ue[c][idx] * gphi[d]
        G = [[sum(Jinv[d][j] * Gr[c][d] for d in range(3)) for j in range(3)] for c in range(5)]
        return U, G, x, Jinv, dJ, C

    def mirror(self, U):
        g, R = self.gamma, self.R
        rho = U[0]
        ke = 0.5 * sum(mi * mi for mi in U[1:4]) / rho
        T = (g - 1) * (U[4] - ke) / (rho * R)
        Tp = 2 * self.wall_T - T
        return [rho, -U[1], -U[2], -U[3], rho * R / (g - 1) * Tp + ke]

    # ---- residual ----
    def residual(self, Ug, terms="cvf"):
        """Ug[c][e][i] nested lists or an array; returns R as numpy (5, E, N)."""
        Ug = np.asarray(Ug, dtype=float)
        N = self.nb1 ** 3
        R = np.zeros((5, self.E, N))
        conv, visc = "c" in terms, "v" in terms
        q = self.nq
        # tau per cell: nu (k+1)^2 (A_int/2 + A_bdry)/V with the n_q rules
        tau = []
        for e in range(self.E):
            V = 0.0
            for p2 in range(q):
                for p1 in range(q):
                    for p0 in range(q):
                        _, J = self.geo(e, [self.qx[p0], self.qx[p1], self.qx[p2]])
                        V += abs(det3(J)) * self.qw[p0] * self.qw[p1] * self.qw[p2]
            A = 0.0
            for d in range(3):
                for s in (0, 1):
                    wall = self.neighbor(e, d, s) is None
                    for r1 in range(q):
                        for r0 in range(q):
                            xi = self.face_xi(d, s, r0, r1)
                            _, J = self.geo(e, xi)
                            C = cofactor(J)
                            area = math.sqrt(sum(C[i][d] ** 2 for i in range(3)))
                            A += (1.0 if wall else 0.5) * area * self.qw[r0] * self.qw[r1]
            tau.append(self.nu * (self.k + 1) ** 2 * A / V)

        # cells
        for e in range(self.E):
            Ue = Ug[:, e, :]
            if conv or visc:
                for p2 in range(q):
                    for p1 in range(q):
                        for p0 in range(q):
                            xi = [self.qx[p0], self.qx[p1], self.qx[p2]]
                            w = self.qw[p0] * self.qw[p1] * self.qw[p2]
                            U, G, x, Jinv, dJ, _ = self.trace(Ue, e, xi)
                            Fc, Fv, _, _ = self.fluxes(U, G, visc)
                            F = [[(Fc[c][j] if conv else 0.0) - (Fv[c][j] if visc else 0.0) for j in range(3)] for c in range(5)]
                            for (idx, phi, gphi) in self.basis_at(xi):
                                gx = [sum(Jinv[d][j] * gphi[d] for d in range(3)) for j in range(3)]
                                for c in range(5):
                                    R[c, e, idx] += w * abs(dJ) * sum(gx[j] * F[c][j] for j in range(3))
            if "f" in terms and self.f is not None:
                mq = self.k + 1
                for p2 in range(mq):
                    for p1 in range(mq):
                        for p0 in range(mq):
                            xi = [self.mx[p0], self.mx[p1], self.mx[p2]]
                            w = self.mw[p0] * self.mw[p1] * self.mw[p2]
                            U, _, _, _, dJ, _ = self.trace(Ue, e, xi)
                            u = [U[1 + a] / U[0] for a in range(3)]
                            S = [0.0, self.f[0], self.f[1], self.f[2], sum(self.f[a] * u[a] for a in range(3))]
                            for (idx, phi, _) in self.basis_at(xi):
                                for c in range(5):
                                    R[c, e, idx] += w * abs(dJ) * phi * S[c]

        if not (conv or visc):
            return R
        # faces, each once: the cell below (side s=1) and the one above (s=0)
        for e in range(self.E):
            for d in range(3):
                for s in (0, 1):
                    f = self.neighbor(e, d, s)
                    if f is None:
                        self.face(Ug, R, e, None, d, s, tau[e], conv, visc)
                    elif s == 1:
                        self.face(Ug, R, e, f, d, s, max(tau[e], tau[f]), conv, visc)
        return R

    def neighbor(self, e, d, s):
        c = list(self.ijk(e))
        c[d] += 1 if s == 1 else -1
        if c[d] < 0 or c[d] >= self.n[d]:
            if not self.periodic[d]:
                return None
            c[d] %= self.n[d]
        return self.cell_index(*c)

    def face_xi(self, d, s, r0, r1):
        t = [a for a in range(3) if a != d]
        xi = [0.0, 0.0, 0.0]
        xi[d] = float(s)
        xi[t[0]] = self.qx[r0]
        xi[t[1]] = self.qx[r1]
        return xi

    def face(self, Ug, R, e, f, d, s, tau, conv, visc):
        q = self.nq
        for r1 in range(q):
            for r0 in range(q):
                w = self.qw[r0] * self.qw[r1]
                xa = self.face_xi(d, s, r0, r1)
                Ua, Ga, _, Jia, dJa, Ca = self.trace(Ug[:, e, :], e, xa)
                sign = 1.0 if s == 1 else -1.0
                nn = [sign * Ca[i][d] for i in range(3)]       # cofactor column = det J * J^{-T} e_d
                area = math.sqrt(sum(v * v for v in nn))
                n = [v / area for v in nn]
                dA = area * w
                if f is None:
                    Ub, Gb = self.mirror(Ua), Ga
                    sides = [(e, xa, Ua, Ga, Jia, Ub, Gb, n)]
                else:
                    xb = self.face_xi(d, 1 - s, r0, r1)
                    Ub, Gb, _, Jib, _, _ = self.trace(Ug[:, f, :], f, xb)
                    sides = [(e, xa, Ua, Ga, Jia, Ub, Gb, n), (f, xb, Ub, Gb, Jib, Ua, Ga, [-v for v in n])]
                for (cell, xi, Um, Gm, Jinv, Up, Gp, nm) in sides:
                    Fcm, Fvm, pm, um = self.fluxes(Um, Gm, visc)
                    Fcp, Fvp, pp, up = self.fluxes(Up, Gp, visc)
                    val = [0.0] * 5
                    jump = [Um[c] - Up[c] for c in range(5)]
                    if conv:
                        cm = math.sqrt(abs(self.gamma * pm / Um[0]))
                        cp = math.sqrt(abs(self.gamma * pp / Up[0]))
                        Lam = max(math.sqrt(sum(v * v for v in um)) + cm, math.sqrt(sum(v * v for v in up)) + cp)
                        for c in range(5):
                            val[c] -= 0.5 * sum((Fcm[c][j] + Fcp[c][j]) * nm[j] for j in range(3)) + 0.5 * Lam * jump[c]
                    sym = None
                    if visc:
                        for c in range(5):
                            val[c] += 0.5 * sum((Fvm[c][j] + Fvp[c][j]) * nm[j] for j in range(3)) - tau * jump[c]
                        Delta = [[jump[c] * nm[j] for j in range(3)] for c in range(5)]
                        _, sym, _, _ = self.fluxes(Um, Delta, True)
                    for (idx, phi, gphi) in self.basis_at(xi):
                        gx = [sum(Jinv[dd][j] * gphi[dd] for dd in range(3)) for j in range(3)]
                        for c in range(5):
                            v = phi * val[c]
                            if sym is not None:
                                v += 0.5 * sum(gx[j] * sym[c][j] for j in range(3))
                            R[c, cell, idx] += dA * v
