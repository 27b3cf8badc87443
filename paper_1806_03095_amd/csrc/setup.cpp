// Host-side setup: 1D Gauss and Gauss-Lobatto rules (Newton iterations in long
// double), Lagrange bases, the box meshes and their isoparametric mapping, the
// metric terms of the paper's Sec. 2.2.3 eq. (IntegralsReferenceSpace) at every
// quadrature point, and the interior-penalty parameter of eq. (TauIP_Element).

#include "setup.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <thread>

namespace dgns {

namespace {

// ---------------------------------------------------------------- 1D rules
typedef long double ld;

// Legendre polynomial P_n and its derivative at x in [-1, 1] (three-term recurrence).
void legendre(int n, ld x, ld& p, ld& dp) {
    ld p0 = 1, p1 = x;
    if (n == 0) {
        p = 1;
        dp = 0;
        return;
    }
    for (int k = 2; k <= n; ++k) {
        const ld p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
    }
    p = p1;
    dp = n * (x * p1 - p0) / (x * x - 1);
}

// Gauss-Legendre rule on [0,1] by Newton's method on P_n.
void gauss_rule(int n, double* x, double* w) {
    const ld pi = 3.141592653589793238462643383279502884L;
    for (int i = 0; i < n; ++i) {
        ld z = cosl(pi * (i + 0.75L) / (n + 0.5L));
        for (int it = 0; it < 100; ++it) {
            ld p, dp;
            legendre(n, z, p, dp);
            const ld dz = p / dp;
            z -= dz;
            if (fabsl(dz) < 1e-19L) break;
        }
        ld p, dp;
        legendre(n, z, p, dp);
        // ascending order on [0,1]
        x[n - 1 - i] = (double)(0.5L * (1 + z));
        w[n - 1 - i] = (double)(1.0L / ((1 - z * z) * dp * dp));
    }
}

// Legendre-Gauss-Lobatto points on [0,1]: the ends and the roots of P'_{n-1}.
void lobatto_points(int n, double* x) {
    const ld pi = 3.141592653589793238462643383279502884L;
    const int m = n - 1;
    x[0] = 0.0;
    x[n - 1] = 1.0;
    for (int i = 1; i < m; ++i) {
        ld z = -cosl(pi * i / m);   // Chebyshev-Gauss-Lobatto guess
        for (int it = 0; it < 100; ++it) {
            // f = P'_m, f' = P''_m from the Legendre ODE: (1-z^2) P'' = 2 z P' - m(m+1) P
            ld p, dp;
            legendre(m, z, p, dp);
            const ld ddp = (2 * z * dp - m * (m + 1) * p) / (1 - z * z);
            const ld dz = dp / ddp;
            z -= dz;
            if (fabsl(dz) < 1e-19L) break;
        }
        x[i] = (double)(0.5L * (1 + z));
    }
}

// Lagrange basis on nodes[0..n) at x: values and derivatives (barycentric form).
void lagrange_at(int n, const double* nodes, double x, double* v, double* dv) {
    for (int i = 0; i < n; ++i) {
        ld val = 1, der = 0;
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            const ld f = ((ld)x - nodes[j]) / ((ld)nodes[i] - nodes[j]);
            der = der * f + val / ((ld)nodes[i] - nodes[j]);
            val *= f;
        }
        v[i] = (double)val;
        if (dv) dv[i] = (double)der;
    }
}

bool invert(int n, const double* A, double* Ai) {
    std::vector<ld> M(n * 2 * n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < 2 * n; ++j) M[i * 2 * n + j] = j < n ? A[i * n + j] : (j - n == i ? 1 : 0);
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (fabsl(M[r * 2 * n + c]) > fabsl(M[piv * 2 * n + c])) piv = r;
        if (fabsl(M[piv * 2 * n + c]) < 1e-300L) return false;
        for (int j = 0; j < 2 * n; ++j) std::swap(M[c * 2 * n + j], M[piv * 2 * n + j]);
        const ld d = M[c * 2 * n + c];
        for (int j = 0; j < 2 * n; ++j) M[c * 2 * n + j] /= d;
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            const ld f = M[r * 2 * n + c];
            for (int j = 0; j < 2 * n; ++j) M[r * 2 * n + j] -= f * M[c * 2 * n + j];
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Ai[i * n + j] = (double)M[i * 2 * n + n + j];
    return true;
}

}  // namespace

void build_tables(int k, int q, int basis, Tables1D& t) {
    std::memset(&t, 0, sizeof t);
    const int n = k + 1;
    t.n = n;
    t.q = q;
    double nodes[kMaxN], gnodes[kMaxN], xq[kMaxQ], wq[kMaxQ], xm[kMaxN], wm[kMaxN];
    lobatto_points(n, gnodes);
    if (basis == DGNS_BASIS_LGL) std::memcpy(nodes, gnodes, sizeof(double) * n);
    else {
        double wtmp[kMaxN];
        gauss_rule(n, nodes, wtmp);
    }
    gauss_rule(q, xq, wq);
    gauss_rule(n, xm, wm);
    for (int p = 0; p < q; ++p) {
        lagrange_at(n, nodes, xq[p], t.S[p], t.D[p]);
        lagrange_at(n, gnodes, xq[p], t.Sg[p], nullptr);
        t.w[p] = wq[p];
    }
    for (int s = 0; s < 2; ++s) lagrange_at(n, nodes, (double)s, t.fv[s], t.fd[s]);
    double Sm[kMaxN * kMaxN], Smi[kMaxN * kMaxN];
    for (int p = 0; p < n; ++p) {
        lagrange_at(n, nodes, xm[p], &Sm[p * n], nullptr);
        t.wm[p] = wm[p];
    }
    invert(n, Sm, Smi);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            t.Sm[i][j] = Sm[i * n + j];
            t.Smi[i][j] = Smi[i * n + j];
        }
}

namespace {

template <typename F>
void parallel_for(int64_t n, F f) {
    unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    if (n < 64) nt = 1;
    std::vector<std::thread> th;
    for (unsigned r = 0; r < nt; ++r)
        th.emplace_back([=, &f] {
            for (int64_t i = r; i < n; i += nt) f(i);
        });
    for (auto& x : th) x.join();
}



// the exact box map s in [0,1]^3 -> x
void box_map(const dgns_box_mesh& m, const double s[3], double x[3]) {
    for (int d = 0; d < 3; ++d) x[d] = m.lo[d] + (m.hi[d] - m.lo[d]) * s[d];
    if (m.kind == DGNS_MESH_CHANNEL) {
        const double C = m.stretch_C;
        x[1] = m.lo[1] + (m.hi[1] - m.lo[1]) * 0.5 * (1.0 + std::tanh(C * (2.0 * s[1] - 1.0)) / std::tanh(C));
    } else if (m.kind == DGNS_MESH_CURVED) {
        const double tp = 6.283185307179586476925286766559;
        const double b = m.deform_amp * std::sin(tp * s[0]) * std::sin(tp * s[1]) * std::sin(tp * s[2]);
        for (int d = 0; d < 3; ++d) x[d] += b;
    }
}

struct Mapper {
    const HostSetup* c;
    int n;
    double gn[kMaxN];
    // x and J = dx/dxi of cell e at reference point xi
    void eval(int64_t e, const double xi[3], double x[3], double J[9]) const {
        double v[3][kMaxN], dv[3][kMaxN];
        for (int d = 0; d < 3; ++d) lagrange_at(n, gn, xi[d], v[d], dv[d]);
        for (int i = 0; i < 3; ++i) x[i] = 0;
        for (int i = 0; i < 9; ++i) J[i] = 0;
        const double* X = &c->geo[e * 3 * c->n3];
        for (int a2 = 0; a2 < n; ++a2)
            for (int a1 = 0; a1 < n; ++a1)
                for (int a0 = 0; a0 < n; ++a0) {
                    const int i = a0 + n * (a1 + n * a2);
                    const double phi = v[0][a0] * v[1][a1] * v[2][a2];
                    const double g[3] = {dv[0][a0] * v[1][a1] * v[2][a2], v[0][a0] * dv[1][a1] * v[2][a2],
                                         v[0][a0] * v[1][a1] * dv[2][a2]};
                    for (int r = 0; r < 3; ++r) {
                        const double xr = X[r * c->n3 + i];
                        x[r] += xr * phi;
                        for (int j = 0; j < 3; ++j) J[r * 3 + j] += xr * g[j];
                    }
                }
    }
};

double inv3(const double J[9], double Ji[9]) {
    const double det = J[0] * (J[4] * J[8] - J[5] * J[7]) - J[1] * (J[3] * J[8] - J[5] * J[6]) +
                       J[2] * (J[3] * J[7] - J[4] * J[6]);
    Ji[0] = (J[4] * J[8] - J[5] * J[7]) / det;
    Ji[1] = (J[2] * J[7] - J[1] * J[8]) / det;
    Ji[2] = (J[1] * J[5] - J[2] * J[4]) / det;
    Ji[3] = (J[5] * J[6] - J[3] * J[8]) / det;
    Ji[4] = (J[0] * J[8] - J[2] * J[6]) / det;
    Ji[5] = (J[2] * J[3] - J[0] * J[5]) / det;
    Ji[6] = (J[3] * J[7] - J[4] * J[6]) / det;
    Ji[7] = (J[1] * J[6] - J[0] * J[7]) / det;
    Ji[8] = (J[0] * J[4] - J[1] * J[3]) / det;
    return det;
}

inline int64_t cell_id(const dgns_box_mesh& m, int i0, int i1, int i2) {
    return i0 + (int64_t)m.n[0] * (i1 + (int64_t)m.n[1] * i2);
}

int build_geometry(const dgns_params& prm, const dgns_box_mesh& m, HostSetup* c, std::string& err) {
    const int k = prm.degree, n = k + 1, q = prm.n_q;
    const int64_t E = c->ncell, N3 = c->n3, Q3 = (int64_t)q * q * q, Q2 = (int64_t)q * q;
    double gnodes[kMaxN], xq[kMaxQ], wq[kMaxQ], xm[kMaxN], wm[kMaxN];
    lobatto_points(n, gnodes);
    gauss_rule(q, xq, wq);
    gauss_rule(n, xm, wm);
    double bnodes[kMaxN];
    if (prm.basis == DGNS_BASIS_LGL) std::memcpy(bnodes, gnodes, sizeof bnodes);
    else {
        double wt[kMaxN];
        gauss_rule(n, bnodes, wt);
    }

    c->geo.assign(E * 3 * N3, 0.0);
    c->node_x.assign(3 * E * N3, 0.0);
    parallel_for(E, [&](int64_t e) {
        const int i0 = (int)(e % m.n[0]), i1 = (int)((e / m.n[0]) % m.n[1]), i2 = (int)(e / ((int64_t)m.n[0] * m.n[1]));
        for (int a2 = 0; a2 < n; ++a2)
            for (int a1 = 0; a1 < n; ++a1)
                for (int a0 = 0; a0 < n; ++a0) {
                    const double s[3] = {(i0 + gnodes[a0]) / m.n[0], (i1 + gnodes[a1]) / m.n[1], (i2 + gnodes[a2]) / m.n[2]};
                    double x[3];
                    box_map(m, s, x);
                    for (int r = 0; r < 3; ++r) c->geo[(e * 3 + r) * N3 + a0 + n * (a1 + n * a2)] = x[r];
                }
    });
    Mapper mp{c, n, {}};
    std::memcpy(mp.gn, gnodes, sizeof gnodes);
    parallel_for(E, [&](int64_t e) {
        for (int a2 = 0; a2 < n; ++a2)
            for (int a1 = 0; a1 < n; ++a1)
                for (int a0 = 0; a0 < n; ++a0) {
                    const double xi[3] = {bnodes[a0], bnodes[a1], bnodes[a2]};
                    double x[3], J[9];
                    mp.eval(e, xi, x, J);
                    for (int r = 0; r < 3; ++r) c->node_x[(r * E + e) * N3 + a0 + n * (a1 + n * a2)] = x[r];
                }
    });

    // cell metric, volume and face areas per cell (n_q rules)
    std::vector<double> vol(E), area(E * 6);
    std::vector<int> bad(E, 0);
    std::vector<double>& metric = c->metric;
    std::vector<double>& mass_jxw = c->mass_jxw;
    metric.assign(c->gen ? E * 10 * Q3 : E * 10, 0.0);
    mass_jxw.assign(c->gen ? E * N3 : 0, 0.0);
    parallel_for(E, [&](int64_t e) {
        double V = 0;
        for (int p2 = 0; p2 < q; ++p2)
            for (int p1 = 0; p1 < q; ++p1)
                for (int p0 = 0; p0 < q; ++p0) {
                    const double xi[3] = {xq[p0], xq[p1], xq[p2]};
                    double x[3], J[9], Ji[9];
                    mp.eval(e, xi, x, J);
                    const double det = inv3(J, Ji);
                    if (!(det > 0)) bad[e] = 1;
                    const double jxw = std::fabs(det) * wq[p0] * wq[p1] * wq[p2];
                    V += jxw;
                    const int64_t p = p0 + q * (p1 + q * p2);
                    if (c->gen) {
                        for (int r = 0; r < 9; ++r) metric[(e * 10 + r) * Q3 + p] = Ji[r];
                        metric[(e * 10 + 9) * Q3 + p] = jxw;
                    }
                }
        vol[e] = V;
        if (!c->gen) {
            const double xi[3] = {0.5, 0.5, 0.5};
            double x[3], J[9], Ji[9];
            mp.eval(e, xi, x, J);
            const double det = inv3(J, Ji);
            for (int r = 0; r < 9; ++r) metric[e * 10 + r] = Ji[r];
            metric[e * 10 + 9] = det;
        } else {
            for (int p2 = 0; p2 < n; ++p2)
                for (int p1 = 0; p1 < n; ++p1)
                    for (int p0 = 0; p0 < n; ++p0) {
                        const double xi[3] = {xm[p0], xm[p1], xm[p2]};
                        double x[3], J[9], Ji[9];
                        mp.eval(e, xi, x, J);
                        const double det = inv3(J, Ji);
                        if (!(det > 0)) bad[e] = 1;
                        mass_jxw[e * N3 + p0 + n * (p1 + n * p2)] = std::fabs(det) * wm[p0] * wm[p1] * wm[p2];
                    }
        }
        for (int d = 0; d < 3; ++d) {
            const int t0 = d == 0 ? 1 : 0, t1 = d == 2 ? 1 : 2;
            for (int s = 0; s < 2; ++s) {
                double A = 0;
                for (int r1 = 0; r1 < q; ++r1)
                    for (int r0 = 0; r0 < q; ++r0) {
                        double xi[3];
                        xi[d] = s;
                        xi[t0] = xq[r0];
                        xi[t1] = xq[r1];
                        double x[3], J[9], Ji[9];
                        mp.eval(e, xi, x, J);
                        const double det = inv3(J, Ji);
                        const double l = std::sqrt(Ji[d * 3] * Ji[d * 3] + Ji[d * 3 + 1] * Ji[d * 3 + 1] + Ji[d * 3 + 2] * Ji[d * 3 + 2]);
                        A += std::fabs(det) * l * wq[r0] * wq[r1];
                    }
                area[e * 6 + d * 2 + s] = A;
            }
        }
    });
    for (int64_t e = 0; e < E; ++e)
        if (bad[e]) {
            err = "cell " + std::to_string((long long)e) + ": the mapping folds (det J <= 0)";
            return DGNS_EINVAL;
        }

    // penalty per cell, then per face
    const double nu = prm.mu / prm.rho_ref;
    std::vector<double> tau_cell(E);
    for (int64_t e = 0; e < E; ++e) {
        const int ijk[3] = {(int)(e % m.n[0]), (int)((e / m.n[0]) % m.n[1]), (int)(e / ((int64_t)m.n[0] * m.n[1]))};
        double A = 0;
        for (int d = 0; d < 3; ++d)
            for (int s = 0; s < 2; ++s) {
                const bool boundary = !m.periodic[d] && ((s == 0 && ijk[d] == 0) || (s == 1 && ijk[d] == m.n[d] - 1));
                A += (boundary ? 1.0 : 0.5) * area[e * 6 + d * 2 + s];
            }
        tau_cell[e] = nu * (k + 1) * (k + 1) * A / vol[e];
    }
    for (int d = 0; d < 3; ++d) {
        const int t0 = d == 0 ? 1 : 0, t1 = d == 2 ? 1 : 2;
        const int nd = m.n[d], n0 = m.n[t0], n1 = m.n[t1];
        const int64_t nf = (int64_t)(nd + 1) * n0 * n1;
        std::vector<double>& tau = c->tau[d];
        std::vector<double>& fd = c->face[d];
        tau.assign(nf, 0.0);
        fd.assign(c->gen ? nf * 22 * Q2 : 0, 0.0);
        parallel_for(nf, [&](int64_t f) {
            const int pos = (int)(f % (nd + 1));
            const int j0 = (int)((f / (nd + 1)) % n0), j1 = (int)(f / ((int64_t)(nd + 1) * n0));
            auto cell_at = [&](int id) -> int64_t {
                if (id < 0 || id >= nd) {
                    if (!m.periodic[d]) return -1;
                    id = (id + nd) % nd;
                }
                int ijk[3];
                ijk[d] = id;
                ijk[t0] = j0;
                ijk[t1] = j1;
                return cell_id(m, ijk[0], ijk[1], ijk[2]);
            };
            const int64_t em = cell_at(pos - 1), ep = cell_at(pos);
            if (em >= 0 && ep >= 0) tau[f] = std::max(tau_cell[em], tau_cell[ep]);
            else tau[f] = tau_cell[em >= 0 ? em : ep];
            if (!c->gen) return;
            for (int r1 = 0; r1 < q; ++r1)
                for (int r0 = 0; r0 < q; ++r0) {
                    const int64_t r = r0 + (int64_t)q * r1;
                    double Jim[9] = {0}, Jip[9] = {0}, nn[3], dAw;
                    double xi[3];
                    xi[t0] = xq[r0];
                    xi[t1] = xq[r1];
                    double detm = 0, detp = 0;
                    if (em >= 0) {
                        double x[3], J[9];
                        xi[d] = 1.0;
                        mp.eval(em, xi, x, J);
                        detm = inv3(J, Jim);
                    }
                    if (ep >= 0) {
                        double x[3], J[9];
                        xi[d] = 0.0;
                        mp.eval(ep, xi, x, J);
                        detp = inv3(J, Jip);
                    }
                    const double* Jn = em >= 0 ? Jim : Jip;
                    const double det = em >= 0 ? detm : detp;
                    const double l = std::sqrt(Jn[d * 3] * Jn[d * 3] + Jn[d * 3 + 1] * Jn[d * 3 + 1] + Jn[d * 3 + 2] * Jn[d * 3 + 2]);
                    for (int j = 0; j < 3; ++j) nn[j] = Jn[d * 3 + j] / l;
                    dAw = std::fabs(det) * l * wq[r0] * wq[r1];
                    double* o = &fd[f * 22 * Q2 + r];
                    for (int j = 0; j < 3; ++j) o[j * Q2] = nn[j];
                    o[3 * Q2] = dAw;
                    for (int j = 0; j < 9; ++j) {
                        o[(4 + j) * Q2] = Jim[j];
                        o[(13 + j) * Q2] = Jip[j];
                    }
                }
        });
    }

    // h_min: minimum distance between two vertices of a cell
    double hmin = INFINITY;
    for (int64_t e = 0; e < E; ++e) {
        const int ijk[3] = {(int)(e % m.n[0]), (int)((e / m.n[0]) % m.n[1]), (int)(e / ((int64_t)m.n[0] * m.n[1]))};
        double v[8][3];
        for (int cnr = 0; cnr < 8; ++cnr) {
            const double s[3] = {(double)(ijk[0] + (cnr & 1)) / m.n[0], (double)(ijk[1] + ((cnr >> 1) & 1)) / m.n[1],
                                 (double)(ijk[2] + ((cnr >> 2) & 1)) / m.n[2]};
            box_map(m, s, v[cnr]);
        }
        for (int a = 0; a < 8; ++a)
            for (int b = a + 1; b < 8; ++b) {
                const double dx = v[a][0] - v[b][0], dy = v[a][1] - v[b][1], dz = v[a][2] - v[b][2];
                hmin = std::min(hmin, std::sqrt(dx * dx + dy * dy + dz * dz));
            }
    }
    c->h_min = hmin;
    return 0;
}

}  // namespace

int build_setup(const dgns_params& prm, const dgns_box_mesh& msh, HostSetup& out, std::string& err) {
    out.gen = msh.kind != DGNS_MESH_AFFINE;
    out.ncell = (int64_t)msh.n[0] * msh.n[1] * msh.n[2];
    out.n3 = (int64_t)(prm.degree + 1) * (prm.degree + 1) * (prm.degree + 1);
    build_tables(prm.degree, prm.n_q, prm.basis, out.tab);
    return build_geometry(prm, msh, &out, err);
}

}  // namespace dgns
