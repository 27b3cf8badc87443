"""Hexahedral box meshes, the isoparametric mapping and its geometry.

Oracle (test infrastructure only).

Paper: Sec. 2.2.1 (elements are images of the reference cube [0,1]^3 under
x^e(xi); tensor-product nodal basis), Sec. 2.2.3 eq. (IntegralsReferenceSpace)
(Jacobian J = dx/dxi, |det J| for cell integrals, |det J| |J^{-T} n_xi| for face
integrals), Sec. 5.2.1 (uniform Cartesian Taylor-Green mesh) and Sec. 5.3.1
(channel: tanh wall stretching with factor C, isoparametric mapping of degree k).

Numbering used throughout: cell e = i0 + n0*(i1 + n1*i2); node (a0, a1, a2) of a
cell is a0 + n*(a1 + n*a2) with n = k+1, i.e. the first coordinate is fastest.
"""

import itertools

import numpy as np

from . import rules

AFFINE, CHANNEL, CURVED = 0, 1, 2


def tensor_basis(nodes1d, pts):
    """Dense values and reference gradients of the tensor-product Lagrange basis.

    Returns Phi[p, i] = phi_i(xi_p) and dPhi[p, i, d] = d phi_i / d xi_d at the
    points pts[p, :] (each phi_i the product of three 1D Lagrange polynomials).
    """
    n = len(nodes1d)
    pts = np.asarray(pts, dtype=np.float64)
    V = [rules.lagrange_values(nodes1d, pts[:, d]) for d in range(3)]
    D = [rules.lagrange_derivatives(nodes1d, pts[:, d]) for d in range(3)]
    P = len(pts)
    Phi = np.zeros((P, n ** 3))
    dPhi = np.zeros((P, n ** 3, 3))
    for a2, a1, a0 in itertools.product(range(n), repeat=3):
        i = a0 + n * (a1 + n * a2)
        Phi[:, i] = V[0][:, a0] * V[1][:, a1] * V[2][:, a2]
        dPhi[:, i, 0] = D[0][:, a0] * V[1][:, a1] * V[2][:, a2]
        dPhi[:, i, 1] = V[0][:, a0] * D[1][:, a1] * V[2][:, a2]
        dPhi[:, i, 2] = V[0][:, a0] * V[1][:, a1] * D[2][:, a2]
    return Phi, dPhi


def cell_points(x1d, w1d):
    """Tensor-product points (first coordinate fastest) and weights on [0,1]^3."""
    q = len(x1d)
    pts = np.zeros((q ** 3, 3))
    wts = np.zeros(q ** 3)
    for p2, p1, p0 in itertools.product(range(q), repeat=3):
        p = p0 + q * (p1 + q * p2)
        pts[p] = (x1d[p0], x1d[p1], x1d[p2])
        wts[p] = w1d[p0] * w1d[p1] * w1d[p2]
    return pts, wts


def face_points(x1d, w1d, d, s):
    """Points on the face xi_d = s of [0,1]^3 and their 2D weights.

    The two tangential coordinates are the remaining axes in increasing order,
    the lower one fastest; both cells sharing a face use the same ordering.
    """
    q = len(x1d)
    t0, t1 = [a for a in range(3) if a != d]
    pts = np.zeros((q * q, 3))
    wts = np.zeros(q * q)
    for r1, r0 in itertools.product(range(q), repeat=2):
        p = r0 + q * r1
        pts[p, d] = float(s)
        pts[p, t0] = x1d[r0]
        pts[p, t1] = x1d[r1]
        wts[p] = w1d[r0] * w1d[r1]
    return pts, wts


class BoxMesh:
    """Structured n0 x n1 x n2 hexahedral mesh of a box, possibly deformed.

    kind AFFINE  : x = lo + (hi - lo) s                  (s in [0,1]^3 global)
    kind CHANNEL : as AFFINE, but x_1 = lo_1 + L_1 (1 + tanh(C (2 s_1 - 1)) / tanh(C)) / 2
                   (Sec. 5.3.1, wall-normal stretching towards both walls)
    kind CURVED  : x_i = lo_i + L_i s_i + a prod_j sin(2 pi s_j)  (box-periodic warp)

    The mapping of each cell is the degree-k interpolant of the map at the
    cell's LGL points (isoparametric, Sec. 5.3.1); for AFFINE it is exact.
    Faces in a direction that is not periodic are domain boundary (walls).
    """

    def __init__(self, n, lo, hi, k, periodic=(True, True, True), kind=AFFINE,
                 stretch_C=1.8, deform_amp=0.0):
        self.n = tuple(int(v) for v in n)
        self.lo = np.asarray(lo, dtype=np.float64)
        self.hi = np.asarray(hi, dtype=np.float64)
        self.k = int(k)
        self.periodic = tuple(bool(p) for p in periodic)
        self.kind = kind
        self.stretch_C = float(stretch_C)
        self.deform_amp = float(deform_amp)
        self.n_cells = self.n[0] * self.n[1] * self.n[2]
        self.geo_nodes = rules.gauss_lobatto_points(self.k + 1)
        self._build_geometry_nodes()
        self._build_neighbors()

    # -- the map from the global unit cube to the physical box ---------------
    def global_map(self, s):
        s = np.asarray(s, dtype=np.float64)
        L = self.hi - self.lo
        x = self.lo + L * s
        if self.kind == CHANNEL:
            C = self.stretch_C
            x[..., 1] = self.lo[1] + L[1] * 0.5 * (1.0 + np.tanh(C * (2.0 * s[..., 1] - 1.0)) / np.tanh(C))
        elif self.kind == CURVED:
            bump = self.deform_amp * np.prod(np.sin(2.0 * np.pi * s), axis=-1)
            x = x + bump[..., None]
        return x

    def cell_ijk(self, e):
        n0, n1, _ = self.n
        return e % n0, (e // n0) % n1, e // (n0 * n1)

    def _build_geometry_nodes(self):
        """X[e, :, i] = the exact map at LGL node i of cell e (isoparametric nodes)."""
        n = self.k + 1
        g = self.geo_nodes
        e = np.arange(self.n_cells)
        ijk = np.stack(self.cell_ijk(e), axis=1).astype(np.float64)        # (E, 3)
        a = np.array([[a0, a1, a2] for a2 in range(n) for a1 in range(n) for a0 in range(n)])
        s = (ijk[:, None, :] + g[a][None, :, :]) / np.asarray(self.n, dtype=np.float64)
        self.X = np.ascontiguousarray(np.transpose(self.global_map(s), (0, 2, 1)))

    def _build_neighbors(self):
        """nb[e, d, s] = the cell across face xi_d = s of cell e, or -1 (wall)."""
        e = np.arange(self.n_cells)
        ijk = np.stack(self.cell_ijk(e), axis=1)
        self.nb = np.full((self.n_cells, 3, 2), -1, dtype=np.int64)
        for d in range(3):
            for s in range(2):
                j = ijk.copy()
                j[:, d] += 1 if s == 1 else -1
                outside = (j[:, d] < 0) | (j[:, d] >= self.n[d])
                j[:, d] %= self.n[d]
                idx = j[:, 0] + self.n[0] * (j[:, 1] + self.n[1] * j[:, 2])
                if not self.periodic[d]:
                    idx = np.where(outside, -1, idx)
                self.nb[:, d, s] = idx

    # -- geometry at reference points ------------------------------------------
    def map_at(self, pts, cells=None):
        """Physical points x[e, p, :] and Jacobians J[e, p, i, j] = dx_i/dxi_j."""
        Phi, dPhi = tensor_basis(self.geo_nodes, pts)
        X = self.X if cells is None else self.X[np.asarray(cells, dtype=np.int64)]
        x = np.einsum("pi,eci->epc", Phi, X)
        J = np.einsum("pij,eci->epcj", dPhi, X)
        return x, J

    def vertices(self):
        """The 8 vertices of every cell, V[e, v, :] (v = c0 + 2 c1 + 4 c2)."""
        e = np.arange(self.n_cells)
        ijk = np.stack(self.cell_ijk(e), axis=1).astype(np.float64)
        c = np.array([[c0, c1, c2] for c2 in (0, 1) for c1 in (0, 1) for c0 in (0, 1)], dtype=np.float64)
        s = (ijk[:, None, :] + c[None, :, :]) / np.asarray(self.n, dtype=np.float64)
        return self.global_map(s)

    def h_min(self):
        """Minimum distance between two vertices of one cell over the mesh (Sec. 2.4)."""
        V = self.vertices()
        best = np.inf
        for a in range(8):
            for b in range(a + 1, 8):
                best = min(best, float(np.min(np.linalg.norm(V[:, a] - V[:, b], axis=1))))
        return best

    def volume(self):
        """Domain volume; det J has degree < 3k per direction, so this rule is exact."""
        x1, w1 = rules.gauss_legendre((3 * self.k) // 2 + 2)
        pts, wts = cell_points(x1, w1)
        _, J = self.map_at(pts)
        return float(np.sum(np.abs(np.linalg.det(J)) * wts))
