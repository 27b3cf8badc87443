// Hand-written adjoint (vector-Jacobian product) of the DG residual:
//
//   Ubar = (dR/dU)^T Rbar,    R = -F_c(U) - F_v(U) + F_rhs(U)  (eq. WeakFormulationConservedVariables)
//
// in gather form: one workgroup per cell e computes Ubar_e, so every output is
// written once (no atomics).  Ubar_e collects
//  * the cell integral of e:  at each quadrature point the cotangent of the flux
//    F = F_c - F_v is w|J| J^{-T} grad_xi Rbar_e (the reference gradient of the
//    function with coefficients Rbar_e), reversed through the pointwise physics
//    to cotangents of U and grad U, then tested with phi_i and grad phi_i;
//  * every face of e: the numerical flux is single-valued (the neighbour's value
//    term is minus e's), so its cotangent is dA (Rbar_e - Rbar_nb) at the face
//    point; the symmetry terms of e and of the neighbour contribute through their
//    cotangents dA/2 J^{-T} grad Rbar of each side.  Only the derivatives with
//    respect to e's own trace are kept (the neighbour's are computed by the
//    neighbour's workgroup).  At walls the exterior state is the mirror of e's;
//  * the body force (k+1 rule).
// The sum-factorised sweeps are those of the forward kernel, applied to the ten
// fields (U_e, Rbar_e); the face test integration is the forward's.

#pragma once

#include "dg_adjoint.h"
#include "op_impl.h"

namespace dgns {

template <int N, int Q>
struct AdjFaceSizes {
    static constexpr int N2 = N * N, Q2 = Q * Q;
    static constexpr int TR = 3 * 8 * 5 * N2;         // traces [f][src*2+side][v/n][c][N^2]
    static constexpr int SW = 3 * 4 * 3 * 5 * N * Q;  // t0 sweep [f][src*2+side][3][c][N][Q]
    static constexpr int OUT = 3 * 4 * 5 * Q2;
    static constexpr int T1 = 3 * 3 * 5 * N * Q;
    static constexpr int W = 3 * 2 * 5 * N2;
    static constexpr int R1 = CMax<SW, T1>::v;
    static constexpr int R2 = CMax<CMax<TR, OUT>::v, W>::v;
    static constexpr int TOTAL = R1 + R2;
};

template <int N, int Q, int P>
struct AdjCellSizes {
    static constexpr int N2 = N * N, Q2 = Q * Q;
    static constexpr int Z = 20 * Q * N2;         // [kind][10 fields][pz][a1][a0]
    static constexpr int Y = 30 * P * Q * N;      // [3][10][pl][py][a0], later [3][5][pl][py][a0]
    static constexpr int F = 20 * P * Q2;         // [4][5][pl][py][px], later [2][5][pl][a1][a0]
    static constexpr int TOTAL = Z + Y + F;
};

template <int N, int Q>
struct AdjSizes {
    static constexpr int fit(int p) {
        return p <= 1 ? 1 : (AdjCellSizes<N, Q, 1>::TOTAL + (p - 1) * (30 * Q * N + 20 * Q * Q) <= AdjFaceSizes<N, Q>::TOTAL ? p : fit(p - 1));
    }
    static constexpr int P = fit(Q);
    static constexpr int WORK = CMax<CMax<AdjCellSizes<N, Q, P>::TOTAL, AdjFaceSizes<N, Q>::TOTAL>::v, 15 * N * N * N>::v;
};

// Adjoint of the three faces xi_d = s.  sX = [U_e; Rbar_e] (10 fields), Rb = Rbar (global).
template <int N, int Q, bool GEN>
__device__ __forceinline__ void adj_face_group(const OpArgs& a, const double* Rb, const KTab<N, Q, double>& lt,
                                               const Phys<double>& ph, bool conv, bool visc, int s, const FaceInfo& fi,
                                               const double* sTau, const double* sFn, const double (&Ji)[9], double detJ,
                                               const double* sX, double* sUb, double* sW) {
    using Real = double;
    using FS = AdjFaceSizes<N, Q>;
    constexpr int N2 = N * N, N3 = N2 * N, Q2 = Q * Q;
    Real* r1 = sW;
    Real* r2 = sW + FS::R1;
    const int tid = threadIdx.x, nth = blockDim.x;
    const int64_t cstride = a.ncell * N3;

    // traces of U and Rbar, own (from LDS) and neighbour (from memory)
    for (int it = tid; it < 3 * 2 * 5 * N2; it += nth) {
        const int ab = it % N2, c = (it / N2) % 5, src = (it / (5 * N2)) % 2, d = it / (10 * N2);
        const int ia = ab % N, ib = ab / N;
        const int t0 = d == 0 ? 1 : 0, t1 = d == 2 ? 1 : 2;
        const int base = ia * axis_stride(t0, N) + ib * axis_stride(t1, N), sd = axis_stride(d, N);
        Real tv = 0, tn = 0, uv = 0, un = 0;
#pragma unroll
        for (int m = 0; m < N; ++m) {
            const Real x = sX[(src * 5 + c) * N3 + base + m * sd];
            tv += lt.fv[s][m] * x;
            tn += lt.fd[s][m] * x;
        }
        if (!fi.wall[d + 3 * s]) {
            const double* g = (src == 0 ? a.U : Rb) + c * cstride + fi.enb[d + 3 * s] * N3 + base;
#pragma unroll
            for (int m = 0; m < N; ++m) {
                const Real x = g[m * sd];
                uv += lt.fv[1 - s][m] * x;
                un += lt.fd[1 - s][m] * x;
            }
        }
        Real* tr = r2 + (d * 8 + src * 4) * 5 * N2 + c * N2 + ab;
        tr[(0 * 2 + 0) * 5 * N2] = tv;
        tr[(0 * 2 + 1) * 5 * N2] = tn;
        tr[(1 * 2 + 0) * 5 * N2] = uv;
        tr[(1 * 2 + 1) * 5 * N2] = un;
    }
    __syncthreads();

    // sweep along t0 of the four trace pairs   r1 [f][src*2+side][3][c][b][q0]
    for (int it = tid; it < 3 * 4 * 5 * N; it += nth) {
        const int ib = it % N, c = (it / N) % 5, ss = (it / (5 * N)) % 4, d = it / (20 * N);
        if ((ss & 1) && fi.wall[d + 3 * s]) continue;
        const Real* tr = r2 + (d * 8 + ss * 2) * 5 * N2 + c * N2 + ib * N;
        Real tv[N], tn[N];
#pragma unroll
        for (int ia = 0; ia < N; ++ia) {
            tv[ia] = tr[ia];
            tn[ia] = tr[5 * N2 + ia];
        }
        Real* o = r1 + ((d * 4 + ss) * 3 * 5 + c) * N * Q + ib * Q;
#pragma unroll
        for (int q0 = 0; q0 < Q; ++q0) {
            Real a0 = 0, a1 = 0, an = 0;
#pragma unroll
            for (int ia = 0; ia < N; ++ia) {
                a0 += lt.S[q0][ia] * tv[ia];
                a1 += lt.D[q0][ia] * tv[ia];
                an += lt.S[q0][ia] * tn[ia];
            }
            o[q0] = a0;
            o[5 * N * Q + q0] = a1;
            o[2 * 5 * N * Q + q0] = an;
        }
    }
    __syncthreads();

    // pointwise adjoint   r2 [f][Ubar, Gbar_t0, Gbar_t1, Gbar_n][c][q1][q0]
    for (int it = tid; it < 3 * Q2; it += nth) {
        const int d = it / Q2, pt = it % Q2, q0 = pt % Q, q1 = pt / Q;
        const int fslot = d + 3 * s;
        const bool wall = fi.wall[fslot] != 0;
        Real Jm[9], Jp[9], nrm[3], dAw;
        if constexpr (GEN) {
            const double* fdp = a.face_data[d] + fi.fid[fslot] * 22 * Q2 + pt;
            const Real sgn = s ? Real(1) : Real(-1);
#pragma unroll
            for (int j = 0; j < 3; ++j) nrm[j] = sgn * fdp[j * Q2];
            dAw = fdp[3 * Q2];
            const int own = s ? 4 : 13, oth = s ? 13 : 4;
#pragma unroll
            for (int m = 0; m < 9; ++m) {
                Jm[m] = fdp[(own + m) * Q2];
                Jp[m] = fdp[(oth + m) * Q2];
            }
        } else {
#pragma unroll
            for (int m = 0; m < 9; ++m) Jm[m] = Ji[m];
            const double* cm = a.cell_metric + fi.enb[fslot] * 10;
#pragma unroll
            for (int m = 0; m < 9; ++m) Jp[m] = cm[m];
            const Real sgn = s ? Real(1) : Real(-1);
            const Real* fn = sFn + 4 * d;
            nrm[0] = sgn * fn[0];
            nrm[1] = sgn * fn[1];
            nrm[2] = sgn * fn[2];
            dAw = detJ * fn[3] * lt.w[q0] * lt.w[q1];
        }
        const Real* A = r1 + d * 4 * 3 * 5 * N * Q;
        constexpr int SS = 3 * 5 * N * Q;
        Real Um[5], Gm[5][3], Up[5], Gp[5][3], rbm[5], gbm[5][3], rbp[5], gbp[5][3];
        load_face_point<N, Q, Real>(lt, A + 0 * SS, d, q0, q1, Jm, Um, Gm);
        load_face_point<N, Q, Real>(lt, A + 2 * SS, d, q0, q1, Jm, rbm, gbm);
        const Prim<Real> sm = primitives(Um, ph);
        if (wall) {
            wall_mirror(Um, sm, ph, Up);
#pragma unroll
            for (int c = 0; c < 5; ++c) {
                rbp[c] = 0;
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    Gp[c][j] = Gm[c][j];
                    gbp[c][j] = 0;
                }
            }
        } else {
            load_face_point<N, Q, Real>(lt, A + 1 * SS, d, q0, q1, Jp, Up, Gp);
            load_face_point<N, Q, Real>(lt, A + 3 * SS, d, q0, q1, Jp, rbp, gbp);
        }
        const Prim<Real> sp = primitives(Up, ph);
        Real jump[5], vb[5];
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            jump[c] = Um[c] - Up[c];
            vb[c] = dAw * (rbm[c] - rbp[c]);
        }
        PrimBar<Real> pbm, pbp;
        zero(pbm);
        zero(pbp);
        Real Ubm[5] = {0, 0, 0, 0, 0}, Ubp[5] = {0, 0, 0, 0, 0}, jb[5] = {0, 0, 0, 0, 0};
        Real Gbm[5][3], Gbp[5][3];
#pragma unroll
        for (int c = 0; c < 5; ++c)
#pragma unroll
            for (int j = 0; j < 3; ++j) Gbm[c][j] = Gbp[c][j] = 0;
        if (conv) {
            Real Fn[5], Fnb[5];
            const Real lm = convective_normal(Um, sm, nrm, ph, Fn);
            const Real lp = convective_normal(Up, sp, nrm, ph, Fn);
            const Real lam = lm > lp ? lm : lp;
            Real lamb = 0;
#pragma unroll
            for (int c = 0; c < 5; ++c) {
                Fnb[c] = Real(-0.5) * vb[c];
                lamb -= Real(0.5) * vb[c] * jump[c];
                jb[c] -= Real(0.5) * lam * vb[c];
            }
            convective_normal_vjp(Um, sm, nrm, ph, Fnb, lm > lp ? lamb : Real(0), pbm, Ubm);
            convective_normal_vjp(Up, sp, nrm, ph, Fnb, lm > lp ? Real(0) : lamb, pbp, Ubp);
        }
        if (visc) {
            Real Fnb[5], Sb[5][3];
#pragma unroll
            for (int c = 0; c < 5; ++c) {
                Fnb[c] = Real(0.5) * vb[c];
                jb[c] -= sTau[fslot] * vb[c];
            }
            viscous_flux_normal_vjp(sm, Gm, nrm, ph, Fnb, pbm, Gbm);
            viscous_flux_normal_vjp(sp, Gp, nrm, ph, Fnb, pbp, Gbp);
            // symmetry term of e: dA/2 grad phi^e . F_v(U_e, jump (x) n)
#pragma unroll
            for (int c = 0; c < 5; ++c)
#pragma unroll
                for (int j = 0; j < 3; ++j) Sb[c][j] = Real(0.5) * dAw * gbm[c][j];
            viscous_flux_rank1_vjp(sm, jump, nrm, ph, Sb, pbm, jb);
            if (!wall) {
                // symmetry term of the neighbour: same jump (x) n, its own state
#pragma unroll
                for (int c = 0; c < 5; ++c)
#pragma unroll
                    for (int j = 0; j < 3; ++j) Sb[c][j] = Real(0.5) * dAw * gbp[c][j];
                viscous_flux_rank1_vjp(sp, jump, nrm, ph, Sb, pbp, jb);
            }
        }
#pragma unroll
        for (int c = 0; c < 5; ++c) Ubm[c] += jb[c];
        if (wall) {
            // U^+ = mirror(U^-), grad U^+ = grad U^-
#pragma unroll
            for (int c = 0; c < 5; ++c) Ubp[c] -= jb[c];
            primitives_vjp(Up, sp, ph, pbp, Ubp);
            wall_mirror_vjp(Um, sm, ph, Ubp, pbm, Ubm);
#pragma unroll
            for (int c = 0; c < 5; ++c)
#pragma unroll
                for (int j = 0; j < 3; ++j) Gbm[c][j] += Gbp[c][j];
        }
        primitives_vjp(Um, sm, ph, pbm, Ubm);
        Real* o = r2 + d * 4 * 5 * Q2 + pt;
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            Real gref[3];
#pragma unroll
            for (int dd = 0; dd < 3; ++dd)
                gref[dd] = Jm[dd * 3] * Gbm[c][0] + Jm[dd * 3 + 1] * Gbm[c][1] + Jm[dd * 3 + 2] * Gbm[c][2];
            o[(0 * 5 + c) * Q2] = Ubm[c];
            o[(1 * 5 + c) * Q2] = d == 0 ? gref[1] : gref[0];
            o[(2 * 5 + c) * Q2] = d == 2 ? gref[1] : gref[2];
            o[(3 * 5 + c) * Q2] = d == 0 ? gref[0] : (d == 1 ? gref[1] : gref[2]);
        }
    }
    __syncthreads();
    face_test_accumulate<N, Q, Real>(lt, s, 0, r1, r2, sUb);
}

template <int N, int Q, bool GEN>
__global__ void __launch_bounds__(kBlock)
dg_adjoint_kernel(OpArgs a, const double* Rb, KTab<N, Q, double> tb, MTab<N, double> mt) {
    using Real = double;
    using Sz = AdjSizes<N, Q>;
    constexpr int P = Sz::P;
    constexpr int N2 = N * N, N3 = N2 * N, Q2 = Q * Q, Q3 = Q2 * Q;
    constexpr int ZS = AdjCellSizes<N, Q, P>::Z, YS = AdjCellSizes<N, Q, P>::Y;
    __shared__ Real sX[10 * N3];
    __shared__ Real sUb[5 * N3];
    __shared__ Real sW[Sz::WORK];
    __shared__ FaceInfo fi;
    __shared__ Real sTau[6];
    __shared__ Real sFn[12];

    const int64_t e = blockIdx.x;
    const int tid = threadIdx.x, nth = blockDim.x;
    const Phys<Real> ph = make_phys<Real>(a);
    const bool conv = (a.terms & 1u) != 0;
    const bool visc = (a.terms & 2u) != 0;
    const int64_t cstride = a.ncell * N3;

    for (int i = tid; i < 5 * N3; i += nth) {
        const int c = i / N3, j = i % N3;
        sX[i] = a.U[c * cstride + e * N3 + j];
        sX[5 * N3 + i] = Rb[c * cstride + e * N3 + j];
        sUb[i] = 0;
    }
    // LDS copies of the 1D tables (every lookup reads LDS; see the forward kernel)
    __shared__ KTab<N, Q, double> lt;
    __shared__ MTab<N, double> lm;
    copy_table<KTab<N, Q, double>, double>(tb, lt);
    copy_table<MTab<N, double>, double>(mt, lm);
    for (int f = tid; f < 6; f += nth) {
        const int i0 = (int)(e % a.n[0]), i1 = (int)((e / a.n[0]) % a.n[1]), i2 = (int)(e / ((int64_t)a.n[0] * a.n[1]));
        const int d = f % 3, s = f / 3;
        const int nd = d == 0 ? a.n[0] : (d == 1 ? a.n[1] : a.n[2]);
        const int per = d == 0 ? a.periodic[0] : (d == 1 ? a.periodic[1] : a.periodic[2]);
        const int id = d == 0 ? i0 : (d == 1 ? i1 : i2);
        const int it0 = d == 0 ? i1 : i0, it1 = d == 2 ? i1 : i2;
        const int nt0 = d == 0 ? a.n[1] : a.n[0];
        int jd = id + (s ? 1 : -1);
        int wall = 0;
        if (jd < 0 || jd >= nd) {
            if (per) jd = (jd + nd) % nd;
            else wall = 1;
        }
        const int j0 = d == 0 ? jd : i0, j1 = d == 1 ? jd : i1, j2 = d == 2 ? jd : i2;
        fi.enb[f] = wall ? e : j0 + (int64_t)a.n[0] * (j1 + (int64_t)a.n[1] * j2);
        fi.fid[f] = (id + s) + (int64_t)(nd + 1) * (it0 + (int64_t)nt0 * it1);
        fi.wall[f] = wall;
        const double* tf = d == 0 ? a.tau_face[0] : (d == 1 ? a.tau_face[1] : a.tau_face[2]);
        sTau[f] = tf[fi.fid[f]];
        if (!GEN && s == 0) {
            const double* row = a.cell_metric + e * 10 + 3 * d;
            const double l = sqrt(row[0] * row[0] + row[1] * row[1] + row[2] * row[2]);
            sFn[4 * d + 0] = row[0] / l;
            sFn[4 * d + 1] = row[1] / l;
            sFn[4 * d + 2] = row[2] / l;
            sFn[4 * d + 3] = l;
        }
    }
    Real Ji[9], detJ = Real(1);
    if constexpr (!GEN) {
#pragma unroll
        for (int m = 0; m < 9; ++m) Ji[m] = a.cell_metric[e * 10 + m];
        detJ = a.cell_metric[e * 10 + 9];
    }
    __syncthreads();

    if (conv || visc) {
        Real* sZ = sW;
        Real* sY = sW + ZS;
        Real* sF = sY + YS;
        // z-sweep of ten fields: value and derivative   [kind][f10][pz][a1][a0]
        for (int it = tid; it < 10 * N2; it += nth) {
            const int c = it / N2, r = it % N2;
            Real v[N];
#pragma unroll
            for (int i = 0; i < N; ++i) v[i] = sX[c * N3 + i * N2 + r];
#pragma unroll
            for (int pz = 0; pz < Q; ++pz) {
                Real z0 = 0, z1 = 0;
#pragma unroll
                for (int i = 0; i < N; ++i) {
                    z0 += lt.S[pz][i] * v[i];
                    z1 += lt.D[pz][i] * v[i];
                }
                sZ[(0 * 10 + c) * Q * N2 + pz * N2 + r] = z0;
                sZ[(1 * 10 + c) * Q * N2 + pz * N2 + r] = z1;
            }
        }
        __syncthreads();
        for (int pz0 = 0; pz0 < Q; pz0 += P) {
            for (int it = tid; it < 10 * P * N; it += nth) {
                const int a0 = it % N, pl = (it / N) % P, c = it / (N * P);
                const int pz = pz0 + pl;
                if (pz >= Q) continue;
                Real z0[N], z1[N];
#pragma unroll
                for (int i = 0; i < N; ++i) {
                    z0[i] = sZ[(0 * 10 + c) * Q * N2 + pz * N2 + i * N + a0];
                    z1[i] = sZ[(1 * 10 + c) * Q * N2 + pz * N2 + i * N + a0];
                }
#pragma unroll
                for (int py = 0; py < Q; ++py) {
                    Real y00 = 0, y10 = 0, y01 = 0;
#pragma unroll
                    for (int i = 0; i < N; ++i) {
                        y00 += lt.S[py][i] * z0[i];
                        y10 += lt.D[py][i] * z0[i];
                        y01 += lt.S[py][i] * z1[i];
                    }
                    sY[((0 * 10 + c) * P + pl) * Q * N + py * N + a0] = y00;
                    sY[((1 * 10 + c) * P + pl) * Q * N + py * N + a0] = y10;
                    sY[((2 * 10 + c) * P + pl) * Q * N + py * N + a0] = y01;
                }
            }
            __syncthreads();

            // pointwise adjoint of F = F_c - F_v
            for (int it = tid; it < P * Q2; it += nth) {
                const int px = it % Q, py = (it / Q) % Q, pl = it / Q2;
                const int pz = pz0 + pl;
                if (pz >= Q) continue;
                Real X[10], Gr[10][3];
#pragma unroll
                for (int c = 0; c < 10; ++c) {
                    Real v = 0, dx = 0, dy = 0, dz = 0;
#pragma unroll
                    for (int i = 0; i < N; ++i) {
                        const Real y00 = sY[((0 * 10 + c) * P + pl) * Q * N + py * N + i];
                        const Real y10 = sY[((1 * 10 + c) * P + pl) * Q * N + py * N + i];
                        const Real y01 = sY[((2 * 10 + c) * P + pl) * Q * N + py * N + i];
                        v += lt.S[px][i] * y00;
                        dx += lt.D[px][i] * y00;
                        dy += lt.S[px][i] * y10;
                        dz += lt.S[px][i] * y01;
                    }
                    X[c] = v;
                    Gr[c][0] = dx;
                    Gr[c][1] = dy;
                    Gr[c][2] = dz;
                }
                Real J[9], jxw;
                const int p = px + Q * (py + Q * pz);
                if constexpr (GEN) {
                    const double* gm = a.cell_metric + e * 10 * Q3 + p;
#pragma unroll
                    for (int m = 0; m < 9; ++m) J[m] = gm[m * Q3];
                    jxw = gm[9 * Q3];
                } else {
#pragma unroll
                    for (int m = 0; m < 9; ++m) J[m] = Ji[m];
                    jxw = detJ * lt.w[px] * lt.w[py] * lt.w[pz];
                }
                Real U[5], G[5][3], Fb[5][3];
#pragma unroll
                for (int c = 0; c < 5; ++c) {
                    U[c] = X[c];
#pragma unroll
                    for (int j = 0; j < 3; ++j) {
                        G[c][j] = J[j] * Gr[c][0] + J[3 + j] * Gr[c][1] + J[6 + j] * Gr[c][2];
                        // cotangent of F[c][j]: w|J| sum_d Jinv[d][j] d_d Rbar
                        Fb[c][j] = jxw * (J[j] * Gr[5 + c][0] + J[3 + j] * Gr[5 + c][1] + J[6 + j] * Gr[5 + c][2]);
                    }
                }
                const Prim<Real> sq = primitives(U, ph);
                PrimBar<Real> pb;
                zero(pb);
                Real Ub[5] = {0, 0, 0, 0, 0}, Gb[5][3];
#pragma unroll
                for (int c = 0; c < 5; ++c)
#pragma unroll
                    for (int j = 0; j < 3; ++j) Gb[c][j] = 0;
                if (conv) convective_flux_vjp(U, sq, Fb, pb, Ub);
                if (visc) {
                    Real Fvb[5][3];
#pragma unroll
                    for (int c = 0; c < 5; ++c)
#pragma unroll
                        for (int j = 0; j < 3; ++j) Fvb[c][j] = -Fb[c][j];
                    viscous_flux_vjp(sq, G, ph, Fvb, pb, Gb);
                }
                primitives_vjp(U, sq, ph, pb, Ub);
#pragma unroll
                for (int c = 0; c < 5; ++c) {
                    sF[((0 * 5 + c) * P + pl) * Q2 + py * Q + px] = Ub[c];
#pragma unroll
                    for (int d = 0; d < 3; ++d)
                        sF[(((1 + d) * 5 + c) * P + pl) * Q2 + py * Q + px] =
                            J[d * 3] * Gb[c][0] + J[d * 3 + 1] * Gb[c][1] + J[d * 3 + 2] * Gb[c][2];
                }
            }
            __syncthreads();

            // x-transposed: B1 = S^T Ub + D^T G0, B2 = S^T G1, B3 = S^T G2   [kind][c][pl][py][a0]
            Real* sB = sY;
            for (int it = tid; it < 5 * P * Q * N; it += nth) {
                const int a0 = it % N, py = (it / N) % Q, pl = (it / (N * Q)) % P, c = it / (N * Q * P);
                if (pz0 + pl >= Q) continue;
                Real b1 = 0, b2 = 0, b3 = 0;
#pragma unroll
                for (int px = 0; px < Q; ++px) {
                    b1 += lt.S[px][a0] * sF[((0 * 5 + c) * P + pl) * Q2 + py * Q + px] +
                          lt.D[px][a0] * sF[((1 * 5 + c) * P + pl) * Q2 + py * Q + px];
                    b2 += lt.S[px][a0] * sF[((2 * 5 + c) * P + pl) * Q2 + py * Q + px];
                    b3 += lt.S[px][a0] * sF[((3 * 5 + c) * P + pl) * Q2 + py * Q + px];
                }
                sB[((0 * 5 + c) * P + pl) * Q * N + py * N + a0] = b1;
                sB[((1 * 5 + c) * P + pl) * Q * N + py * N + a0] = b2;
                sB[((2 * 5 + c) * P + pl) * Q * N + py * N + a0] = b3;
            }
            __syncthreads();
            Real* sE = sF;
            for (int it = tid; it < 5 * P * N2; it += nth) {
                const int a0 = it % N, a1 = (it / N) % N, pl = (it / N2) % P, c = it / (N2 * P);
                if (pz0 + pl >= Q) continue;
                Real e1 = 0, e2 = 0;
#pragma unroll
                for (int py = 0; py < Q; ++py) {
                    e1 += lt.S[py][a1] * sB[((0 * 5 + c) * P + pl) * Q * N + py * N + a0] +
                          lt.D[py][a1] * sB[((1 * 5 + c) * P + pl) * Q * N + py * N + a0];
                    e2 += lt.S[py][a1] * sB[((2 * 5 + c) * P + pl) * Q * N + py * N + a0];
                }
                sE[((0 * 5 + c) * P + pl) * N2 + a1 * N + a0] = e1;
                sE[((1 * 5 + c) * P + pl) * N2 + a1 * N + a0] = e2;
            }
            __syncthreads();
            for (int it = tid; it < 5 * N3; it += nth) {
                const int c = it / N3, r = it % N3, a2 = r / N2, r2 = r % N2;
                Real acc = 0;
#pragma unroll
                for (int pl = 0; pl < P; ++pl) {
                    const int pz = pz0 + pl;
                    if (pz < Q)
                        acc += lt.S[pz][a2] * sE[((0 * 5 + c) * P + pl) * N2 + r2] +
                               lt.D[pz][a2] * sE[((1 * 5 + c) * P + pl) * N2 + r2];
                }
                sUb[it] += acc;
            }
            __syncthreads();
        }

        adj_face_group<N, Q, GEN>(a, Rb, lt, ph, conv, visc, 0, fi, sTau, sFn, Ji, detJ, sX, sUb, sW);
        adj_face_group<N, Q, GEN>(a, Rb, lt, ph, conv, visc, 1, fi, sTau, sFn, Ji, detJ, sX, sUb, sW);
    }

    // body force: R_i += sum_m w|J| phi_i (0, f, f.u); only f.u depends on U
    const bool force = (a.terms & 4u) != 0 && (a.force[0] != 0.0 || a.force[1] != 0.0 || a.force[2] != 0.0);
    if (force) {
        Real* t0b = sW;
        Real* t1b = sW + 5 * N3;
        // U and Rbar at the mass points (fields 0..4 of sX: U, fields 5..9: Rbar)
        sweep_nn<N, Real, false>(lm.Sm, sX, t0b, 0);
        __syncthreads();
        sweep_nn<N, Real, false>(lm.Sm, t0b, t1b, 1);
        __syncthreads();
        sweep_nn<N, Real, false>(lm.Sm, t1b, t0b, 2);
        __syncthreads();
        Real* rb = t1b;   // Rbar_4 at the mass points (only the energy row of F_rhs depends on U)
        sweep_nn<N, Real, false>(lm.Sm, sX + 5 * N3, t1b + 5 * N3, 0);
        __syncthreads();
        sweep_nn<N, Real, false>(lm.Sm, t1b + 5 * N3, rb, 1);
        __syncthreads();
        sweep_nn<N, Real, false>(lm.Sm, rb, t1b + 5 * N3, 2);
        __syncthreads();
        const double* jxw_m = GEN ? a.mass_jxw + e * N3 : nullptr;
        for (int p = tid; p < N3; p += nth) {
            const Real jxw = GEN ? jxw_m[p] : detJ * lm.wm[p % N] * lm.wm[(p / N) % N] * lm.wm[p / N2];
            const Real rho = t0b[p];
            const Real fu = (a.force[0] * t0b[N3 + p] + a.force[1] * t0b[2 * N3 + p] + a.force[2] * t0b[3 * N3 + p]) / rho;
            const Real g = jxw * t1b[5 * N3 + 4 * N3 + p];    // cotangent of f.u
            t0b[p] = -g * fu / rho;
            t0b[N3 + p] = g * a.force[0] / rho;
            t0b[2 * N3 + p] = g * a.force[1] / rho;
            t0b[3 * N3 + p] = g * a.force[2] / rho;
            t0b[4 * N3 + p] = 0;
        }
        __syncthreads();
        sweep_nn<N, Real, true>(lm.Sm, t0b, t1b, 0);
        __syncthreads();
        sweep_nn<N, Real, true>(lm.Sm, t1b, t0b, 1);
        __syncthreads();
        sweep_nn<N, Real, true>(lm.Sm, t0b, t1b, 2);
        __syncthreads();
        for (int i = tid; i < 5 * N3; i += nth) sUb[i] += t1b[i];
        __syncthreads();
    }

    for (int i = tid; i < 5 * N3; i += nth) {
        const int c = i / N3, j = i % N3;
        a.out[c * cstride + e * N3 + j] = sUb[i];
    }
}

template <int N, int Q, bool GEN>
inline int launch_adjoint_t(const OpArgs& a, const double* Rb, const Tables1D& t, hipStream_t st) {
    KTab<N, Q, double> kt;
    MTab<N, double> mt;
    fill_tables<N, Q, double>(t, kt, mt);
    static_assert((AdjSizes<N, Q>::WORK + 15 * N * N * N) * sizeof(double) <= 160 * 1024, "LDS budget");
    hipLaunchKernelGGL((dg_adjoint_kernel<N, Q, GEN>), dim3((unsigned)a.ncell), dim3(kBlock), 0, st, a, Rb, kt, mt);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace dgns
