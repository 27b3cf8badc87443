// Fused cell + face kernel of the DG compressible Navier-Stokes operator.
//
// One workgroup evaluates, for one cell e, the right-hand side of eq.
// (WeakFormulationConservedVariables) of the paper (Sec. 2.2.2) tested against
// all of e's own basis functions, and optionally applies the inverse mass matrix
// so that it writes L = M^{-1} R (eq. SpatiallyDiscretizedProblem, Sec. 2.4):
//
//   cell:  R_i += sum_q w|J| grad_xi phi_i . J^{-1} (F_c - F_v)(U, J^{-T} grad_xi U)
//   faces: R_i += sum_f dA [ phi_i (-F*_c.n + Q*.n) + 1/2 grad phi_i . F_v(U^-, [[U]]) ]
//   force: R_i += sum_m w|J| phi_i (0, f, f.u)   (k+1 rule)
//
// Every contraction with the tensor-product basis is sum-factorised (Sec. 2.3,
// eq. SumFactorization): 1D sweeps of the n x n_q matrices S (values) and D
// (derivatives) along one axis at a time.  Gradients use D along the axis
// directly (n-point contractions) rather than a collocation derivative at the
// n_q points, which is cheaper whenever n_q > n.  The face terms are computed
// element-centrically: each cell evaluates both traces on its six faces and keeps
// only its own test-function contributions, so that every cell's output is written
// exactly once (no atomics, bit-reproducible).
//
// LDS layout per workgroup (Real units): sU[5][N^3] own coefficients, sR[5][N^3]
// accumulated residual, sW = the work area of the current phase (see sizes below).
// The quadrature points are processed in chunks of P planes along xi_2 to bound
// the work area for large n_q.

#pragma once

#include "dg_common.h"

namespace dgns {

template <int A, int B>
struct CMax { static constexpr int v = A > B ? A : B; };

template <int N, int Q, int P>
struct OpSizes {
    static constexpr int N2 = N * N, N3 = N2 * N, Q2 = Q * Q, Q3 = Q2 * Q;
    static constexpr int Z = 10 * Q * N2;                 // z-sweeps: value, derivative
    static constexpr int Y = 15 * P * Q * N;              // y-sweeps (3 kinds), later x-transposed
    static constexpr int F = 15 * P * Q2;                 // reference fluxes, later y-transposed
    static constexpr int CELL = Z + Y + F;
    static constexpr int R1 = CMax<CMax<5 * N3, 30 * Q * N>::v, CMax<20 * Q2, 10 * N2>::v>::v;
    static constexpr int R2 = CMax<CMax<20 * N2, 40 * Q2>::v, 15 * Q * N>::v;
    static constexpr int FACE = R1 + R2;
    static constexpr int MASS = 10 * N3;
    static constexpr int WORK = CMax<CMax<CELL, FACE>::v, MASS>::v;
};

// Applies an N x N matrix M (row-major in M[r][c]) along axis `ax` of the five
// arrays src[5][N^3] -> dst[5][N^3]; transposed uses M^T.  Cooperative over the
// workgroup; the caller synchronises.
template <int N, typename Real, bool TRANS>
__device__ __forceinline__ void sweep_nn(const Real (&M)[N][N], const Real* src, Real* dst, int ax) {
    constexpr int N2 = N * N, N3 = N2 * N;
    const int stride = ax == 0 ? 1 : (ax == 1 ? N : N2);
    for (int it = threadIdx.x; it < 5 * N2; it += blockDim.x) {
        const int c = it / N2, rest = it % N2;
        // rest enumerates the two other coordinates
        int base;
        if (ax == 0) base = rest * N;                                  // (a1, a2)
        else if (ax == 1) base = (rest % N) + (rest / N) * N2;         // (a0, a2)
        else base = rest;                                              // (a0, a1)
        const Real* s = src + c * N3 + base;
        Real* d = dst + c * N3 + base;
        Real v[N];
#pragma unroll
        for (int i = 0; i < N; ++i) v[i] = s[i * stride];
#pragma unroll
        for (int o = 0; o < N; ++o) {
            Real acc = 0;
#pragma unroll
            for (int i = 0; i < N; ++i) acc += (TRANS ? M[i][o] : M[o][i]) * v[i];
            d[o * stride] = acc;
        }
    }
}

// In-LDS inverse mass: sR <- (Smi)^{x3} diag(1/(|J| w)) (Smi^T)^{x3} sR, work >= 5 N^3.
template <int N, typename Real, bool GEN>
__device__ __forceinline__ void inverse_mass_lds(const MTab<N, Real>& mt, Real* sR, Real* work, Real detJ,
                                                 const double* jxw_m) {
    constexpr int N2 = N * N, N3 = N2 * N;
    sweep_nn<N, Real, true>(mt.Smi, sR, work, 0);
    __syncthreads();
    sweep_nn<N, Real, true>(mt.Smi, work, sR, 1);
    __syncthreads();
    sweep_nn<N, Real, true>(mt.Smi, sR, work, 2);
    __syncthreads();
    for (int it = threadIdx.x; it < 5 * N3; it += blockDim.x) {
        const int p = it % N3;
        Real jxw;
        if constexpr (GEN) {
            jxw = (Real)jxw_m[p];
        } else {
            const int p0 = p % N, p1 = (p / N) % N, p2 = p / N2;
            jxw = detJ * mt.wm[p0] * mt.wm[p1] * mt.wm[p2];
        }
        work[it] = work[it] / jxw;
    }
    __syncthreads();
    sweep_nn<N, Real, false>(mt.Smi, work, sR, 0);
    __syncthreads();
    sweep_nn<N, Real, false>(mt.Smi, sR, work, 1);
    __syncthreads();
    sweep_nn<N, Real, false>(mt.Smi, work, sR, 2);
    __syncthreads();
}

// Face terms of one direction d, both sides s = 0, 1, of the cell e (element-centric).
template <int d, int N, int Q, typename Real, bool GEN, typename Sz>
__device__ __forceinline__ void face_terms(const OpArgs& a, const KTab<N, Q, Real>& tb, const Phys<Real>& ph,
                                           bool conv, bool visc, int64_t e, int i0, int i1, int i2,
                                           const Real (&Ji)[9], Real detJ, const Real* sU, Real* sR, Real* sW) {
    constexpr int N2 = N * N, N3 = N2 * N, Q2 = Q * Q;
    Real* r1 = sW;
    Real* r2 = sW + Sz::R1;
    constexpr int t0 = d == 0 ? 1 : 0;
    constexpr int t1 = d == 2 ? 1 : 2;
    constexpr int sd = d == 0 ? 1 : (d == 1 ? N : N2);
    constexpr int s0 = t0 == 0 ? 1 : (t0 == 1 ? N : N2);
    constexpr int s1 = t1 == 0 ? 1 : (t1 == 1 ? N : N2);
    const int tid = threadIdx.x;
    const int64_t cstride = a.ncell * N3;
    const int id = d == 0 ? i0 : (d == 1 ? i1 : i2);
    const int it0 = t0 == 0 ? i0 : (t0 == 1 ? i1 : i2);
    const int it1 = t1 == 0 ? i0 : (t1 == 1 ? i1 : i2);
    const int nd = a.n[d];
    for (int s = 0; s < 2; ++s) {
                // neighbour across face xi_d = s
                int jd = id + (s ? 1 : -1);
                bool wall = false;
                if (jd < 0 || jd >= nd) {
                    if (a.periodic[d]) jd = (jd + nd) % nd;
                    else wall = true;
                }
                const int j0 = d == 0 ? jd : i0, j1 = d == 1 ? jd : i1, j2 = d == 2 ? jd : i2;
                const int64_t enb = wall ? e : j0 + (int64_t)a.n[0] * (j1 + (int64_t)a.n[1] * j2);
                const int64_t fid = (id + s) + (int64_t)(nd + 1) * (it0 + (int64_t)a.n[t0] * it1);
                const Real tau = (Real)a.tau_face[d][fid];

                // neighbour coefficients -> r1
                if (!wall) {
                    for (int i = tid; i < 5 * N3; i += blockDim.x) {
                        const int c = i / N3, j = i % N3;
                        r1[i] = (Real)a.U[c * cstride + enb * N3 + j];
                    }
                }
                __syncthreads();

                // traces: value and normal derivative of both sides at the face nodes
                // r2 layout [side][kind v/n][c][b][a]
                for (int it = tid; it < 5 * N2; it += blockDim.x) {
                    const int c = it / N2, ab = it % N2, ia = ab % N, ib = ab / N;
                    const int base = ia * s0 + ib * s1;
                    Real tv = 0, tn = 0, uv = 0, un = 0;
#pragma unroll
                    for (int m = 0; m < N; ++m) {
                        const Real x = sU[c * N3 + base + m * sd];
                        tv += tb.fv[s][m] * x;
                        tn += tb.fd[s][m] * x;
                    }
                    if (!wall) {
#pragma unroll
                        for (int m = 0; m < N; ++m) {
                            const Real x = r1[c * N3 + base + m * sd];
                            uv += tb.fv[1 - s][m] * x;
                            un += tb.fd[1 - s][m] * x;
                        }
                    }
                    r2[((0 * 2 + 0) * 5 + c) * N2 + ab] = tv;
                    r2[((0 * 2 + 1) * 5 + c) * N2 + ab] = tn;
                    r2[((1 * 2 + 0) * 5 + c) * N2 + ab] = uv;
                    r2[((1 * 2 + 1) * 5 + c) * N2 + ab] = un;
                }
                __syncthreads();

                // sweep along t0: A0 = S tv, A1 = D tv, An = S tn   r1 layout [side][kind3][c][b][r0]
                for (int it = tid; it < 2 * 5 * N; it += blockDim.x) {
                    const int ib = it % N, c = (it / N) % 5, side = it / (5 * N);
                    if (side == 1 && wall) continue;
                    Real tv[N], tn[N];
#pragma unroll
                    for (int ia = 0; ia < N; ++ia) {
                        tv[ia] = r2[((side * 2 + 0) * 5 + c) * N2 + ib * N + ia];
                        tn[ia] = r2[((side * 2 + 1) * 5 + c) * N2 + ib * N + ia];
                    }
#pragma unroll
                    for (int q0 = 0; q0 < Q; ++q0) {
                        Real a0 = 0, a1 = 0, an = 0;
#pragma unroll
                        for (int ia = 0; ia < N; ++ia) {
                            a0 += tb.S[q0][ia] * tv[ia];
                            a1 += tb.D[q0][ia] * tv[ia];
                            an += tb.S[q0][ia] * tn[ia];
                        }
                        r1[((side * 3 + 0) * 5 + c) * N * Q + ib * Q + q0] = a0;
                        r1[((side * 3 + 1) * 5 + c) * N * Q + ib * Q + q0] = a1;
                        r1[((side * 3 + 2) * 5 + c) * N * Q + ib * Q + q0] = an;
                    }
                }
                __syncthreads();

                // sweep along t1: V, D_t0, D_t1, D_n at the face points   r2 layout [side][kind4][c][q1][q0]
                for (int it = tid; it < 2 * 5 * Q; it += blockDim.x) {
                    const int q0 = it % Q, c = (it / Q) % 5, side = it / (5 * Q);
                    if (side == 1 && wall) continue;
                    Real a0[N], a1[N], an[N];
#pragma unroll
                    for (int ib = 0; ib < N; ++ib) {
                        a0[ib] = r1[((side * 3 + 0) * 5 + c) * N * Q + ib * Q + q0];
                        a1[ib] = r1[((side * 3 + 1) * 5 + c) * N * Q + ib * Q + q0];
                        an[ib] = r1[((side * 3 + 2) * 5 + c) * N * Q + ib * Q + q0];
                    }
#pragma unroll
                    for (int q1 = 0; q1 < Q; ++q1) {
                        Real v = 0, g0 = 0, g1 = 0, gn = 0;
#pragma unroll
                        for (int ib = 0; ib < N; ++ib) {
                            v += tb.S[q1][ib] * a0[ib];
                            g0 += tb.S[q1][ib] * a1[ib];
                            g1 += tb.D[q1][ib] * a0[ib];
                            gn += tb.S[q1][ib] * an[ib];
                        }
                        r2[((side * 4 + 0) * 5 + c) * Q2 + q1 * Q + q0] = v;
                        r2[((side * 4 + 1) * 5 + c) * Q2 + q1 * Q + q0] = g0;
                        r2[((side * 4 + 2) * 5 + c) * Q2 + q1 * Q + q0] = g1;
                        r2[((side * 4 + 3) * 5 + c) * Q2 + q1 * Q + q0] = gn;
                    }
                }
                __syncthreads();

                // pointwise numerical fluxes   r1 layout [kind4: val, g_t0, g_t1, g_n][c][q1][q0]
                for (int it = tid; it < Q2; it += blockDim.x) {
                    const int q0 = it % Q, q1 = it / Q;
                    Real Jm[9], Jp[9], nrm[3], dAw;
                    if constexpr (GEN) {
                        const double* fd = a.face_data[d] + fid * 22 * Q2 + it;
                        const Real sgn = s ? Real(1) : Real(-1);
#pragma unroll
                        for (int j = 0; j < 3; ++j) nrm[j] = sgn * (Real)fd[j * Q2];
                        dAw = (Real)fd[3 * Q2];
                        const int own = s ? 4 : 13, oth = s ? 13 : 4;
#pragma unroll
                        for (int m = 0; m < 9; ++m) {
                            Jm[m] = (Real)fd[(own + m) * Q2];
                            Jp[m] = (Real)fd[(oth + m) * Q2];
                        }
                    } else {
#pragma unroll
                        for (int m = 0; m < 9; ++m) Jm[m] = Ji[m];
                        const double* cm = a.cell_metric + enb * 10;
#pragma unroll
                        for (int m = 0; m < 9; ++m) Jp[m] = (Real)cm[m];
                        const Real sgn = s ? Real(1) : Real(-1);
                        const Real l = sqrt(Ji[d * 3] * Ji[d * 3] + Ji[d * 3 + 1] * Ji[d * 3 + 1] + Ji[d * 3 + 2] * Ji[d * 3 + 2]);
#pragma unroll
                        for (int j = 0; j < 3; ++j) nrm[j] = sgn * Ji[d * 3 + j] / l;
                        dAw = detJ * l * tb.w[q0] * tb.w[q1];
                    }
                    Real Um[5], Up[5], Gm[5][3], Gp[5][3];
#pragma unroll
                    for (int c = 0; c < 5; ++c) {
                        Real gr[3];
                        Um[c] = r2[((0 * 4 + 0) * 5 + c) * Q2 + it];
                        gr[t0] = r2[((0 * 4 + 1) * 5 + c) * Q2 + it];
                        gr[t1] = r2[((0 * 4 + 2) * 5 + c) * Q2 + it];
                        gr[d] = r2[((0 * 4 + 3) * 5 + c) * Q2 + it];
#pragma unroll
                        for (int j = 0; j < 3; ++j) Gm[c][j] = Jm[j] * gr[0] + Jm[3 + j] * gr[1] + Jm[6 + j] * gr[2];
                    }
                    if (wall) {
                        wall_mirror(Um, ph, Up);
#pragma unroll
                        for (int c = 0; c < 5; ++c)
#pragma unroll
                            for (int j = 0; j < 3; ++j) Gp[c][j] = Gm[c][j];
                    } else {
#pragma unroll
                        for (int c = 0; c < 5; ++c) {
                            Real gr[3];
                            Up[c] = r2[((1 * 4 + 0) * 5 + c) * Q2 + it];
                            gr[t0] = r2[((1 * 4 + 1) * 5 + c) * Q2 + it];
                            gr[t1] = r2[((1 * 4 + 2) * 5 + c) * Q2 + it];
                            gr[d] = r2[((1 * 4 + 3) * 5 + c) * Q2 + it];
#pragma unroll
                            for (int j = 0; j < 3; ++j) Gp[c][j] = Jp[j] * gr[0] + Jp[3 + j] * gr[1] + Jp[6 + j] * gr[2];
                        }
                    }
                    Real val[5], jump[5];
                    Real gphys[5][3];
#pragma unroll
                    for (int c = 0; c < 5; ++c) {
                        val[c] = 0;
                        jump[c] = Um[c] - Up[c];
#pragma unroll
                        for (int j = 0; j < 3; ++j) gphys[c][j] = 0;
                    }
                    if (conv) {
                        Real Fm[5], Fp[5];
                        const Real lm = convective_normal(Um, nrm, ph, Fm);
                        const Real lp = convective_normal(Up, nrm, ph, Fp);
                        const Real lam = lm > lp ? lm : lp;
#pragma unroll
                        for (int c = 0; c < 5; ++c) val[c] -= Real(0.5) * (Fm[c] + Fp[c]) + Real(0.5) * lam * jump[c];
                    }
                    if (visc) {
                        Real Vm[5][3], Vp[5][3], Dl[5][3], Sy[5][3];
                        viscous_flux(Um, Gm, ph, Vm);
                        viscous_flux(Up, Gp, ph, Vp);
#pragma unroll
                        for (int c = 0; c < 5; ++c) {
                            val[c] += Real(0.5) * ((Vm[c][0] + Vp[c][0]) * nrm[0] + (Vm[c][1] + Vp[c][1]) * nrm[1] +
                                                   (Vm[c][2] + Vp[c][2]) * nrm[2]) -
                                      tau * jump[c];
#pragma unroll
                            for (int j = 0; j < 3; ++j) Dl[c][j] = jump[c] * nrm[j];
                        }
                        viscous_flux(Um, Dl, ph, Sy);
#pragma unroll
                        for (int c = 0; c < 5; ++c)
#pragma unroll
                            for (int j = 0; j < 3; ++j) gphys[c][j] = Real(0.5) * Sy[c][j];
                    }
#pragma unroll
                    for (int c = 0; c < 5; ++c) {
                        Real gref[3];
#pragma unroll
                        for (int dd = 0; dd < 3; ++dd)
                            gref[dd] = (Jm[dd * 3] * gphys[c][0] + Jm[dd * 3 + 1] * gphys[c][1] + Jm[dd * 3 + 2] * gphys[c][2]) * dAw;
                        r1[(0 * 5 + c) * Q2 + it] = val[c] * dAw;
                        r1[(1 * 5 + c) * Q2 + it] = gref[t0];
                        r1[(2 * 5 + c) * Q2 + it] = gref[t1];
                        r1[(3 * 5 + c) * Q2 + it] = gref[d];
                    }
                }
                __syncthreads();

                // transposed along t1: P0 = S^T val + D^T g_t1, P1 = S^T g_t0, Pn = S^T g_n   r2 [kind3][c][b][q0]
                for (int it = tid; it < 5 * Q * N; it += blockDim.x) {
                    const int q0 = it % Q, ib = (it / Q) % N, c = it / (Q * N);
                    Real p0 = 0, p1 = 0, pn = 0;
#pragma unroll
                    for (int q1 = 0; q1 < Q; ++q1) {
                        const int pt = q1 * Q + q0;
                        p0 += tb.S[q1][ib] * r1[(0 * 5 + c) * Q2 + pt] + tb.D[q1][ib] * r1[(2 * 5 + c) * Q2 + pt];
                        p1 += tb.S[q1][ib] * r1[(1 * 5 + c) * Q2 + pt];
                        pn += tb.S[q1][ib] * r1[(3 * 5 + c) * Q2 + pt];
                    }
                    r2[(0 * 5 + c) * N * Q + ib * Q + q0] = p0;
                    r2[(1 * 5 + c) * N * Q + ib * Q + q0] = p1;
                    r2[(2 * 5 + c) * N * Q + ib * Q + q0] = pn;
                }
                __syncthreads();

                // transposed along t0: W0 = S^T P0 + D^T P1, W1 = S^T Pn   r1 [kind2][c][b][a]
                for (int it = tid; it < 5 * N2; it += blockDim.x) {
                    const int ia = it % N, ib = (it / N) % N, c = it / N2;
                    Real w0 = 0, w1 = 0;
#pragma unroll
                    for (int q0 = 0; q0 < Q; ++q0) {
                        w0 += tb.S[q0][ia] * r2[(0 * 5 + c) * N * Q + ib * Q + q0] +
                              tb.D[q0][ia] * r2[(1 * 5 + c) * N * Q + ib * Q + q0];
                        w1 += tb.S[q0][ia] * r2[(2 * 5 + c) * N * Q + ib * Q + q0];
                    }
                    r1[(0 * 5 + c) * N2 + ib * N + ia] = w0;
                    r1[(1 * 5 + c) * N2 + ib * N + ia] = w1;
                }
                __syncthreads();

                // R[c](a, b, m) += W0(a, b) l_m(s) + W1(a, b) l'_m(s)
                for (int it = tid; it < 5 * N3; it += blockDim.x) {
                    const int c = it / N3, r = it % N3;
                    const int x0 = r % N, x1 = (r / N) % N, x2 = r / N2;
                    const int ia = t0 == 0 ? x0 : x1;
                    const int ib = t1 == 1 ? x1 : x2;
                    const int m = d == 0 ? x0 : (d == 1 ? x1 : x2);
                    sR[it] += r1[(0 * 5 + c) * N2 + ib * N + ia] * tb.fv[s][m] +
                              r1[(1 * 5 + c) * N2 + ib * N + ia] * tb.fd[s][m];
                }
                __syncthreads();
    }
}

template <int N, int Q, typename Real, bool GEN, int P>
__global__ void __launch_bounds__(kBlock)
dg_operator_kernel(OpArgs a, KTab<N, Q, Real> tb, MTab<N, Real> mt) {
    using Sz = OpSizes<N, Q, P>;
    constexpr int N2 = Sz::N2, N3 = Sz::N3, Q2 = Sz::Q2, Q3 = Sz::Q3;
    __shared__ Real sU[5 * N3];
    __shared__ Real sR[5 * N3];
    __shared__ Real sW[Sz::WORK];

    const int64_t e = blockIdx.x;
    const int tid = threadIdx.x;
    const Phys<Real> ph = make_phys<Real>(a);
    const bool conv = (a.terms & 1u) != 0;
    const bool visc = (a.terms & 2u) != 0;
    const int64_t cstride = a.ncell * N3;

    for (int i = tid; i < 5 * N3; i += blockDim.x) {
        const int c = i / N3, j = i % N3;
        sU[i] = (Real)a.U[c * cstride + e * N3 + j];
        sR[i] = Real(0);
    }

    // cell-constant metric (affine)
    Real Ji[9], detJ = Real(1);
    if constexpr (!GEN) {
#pragma unroll
        for (int m = 0; m < 9; ++m) Ji[m] = (Real)a.cell_metric[e * 10 + m];
        detJ = (Real)a.cell_metric[e * 10 + 9];
    }
    const int i0 = (int)(e % a.n[0]), i1 = (int)((e / a.n[0]) % a.n[1]), i2 = (int)(e / ((int64_t)a.n[0] * a.n[1]));
    __syncthreads();

    if (conv || visc) {
        // ------------------------------------------------------------ cell term
        Real* sZ = sW;
        Real* sY = sW + Sz::Z;       // later sB
        Real* sF = sY + Sz::Y;       // later sE
        // z-sweep: Z0 = S_z U, Z1 = D_z U     layout [kind][c][pz][a1][a0]
        for (int it = tid; it < 5 * N2; it += blockDim.x) {
            const int c = it / N2, r = it % N2;
            Real v[N];
#pragma unroll
            for (int i = 0; i < N; ++i) v[i] = sU[c * N3 + i * N2 + r];
#pragma unroll
            for (int pz = 0; pz < Q; ++pz) {
                Real z0 = 0, z1 = 0;
#pragma unroll
                for (int i = 0; i < N; ++i) {
                    z0 += tb.S[pz][i] * v[i];
                    z1 += tb.D[pz][i] * v[i];
                }
                sZ[(0 * 5 + c) * Q * N2 + pz * N2 + r] = z0;
                sZ[(1 * 5 + c) * Q * N2 + pz * N2 + r] = z1;
            }
        }
        __syncthreads();

        for (int pz0 = 0; pz0 < Q; pz0 += P) {
            // y-sweep for planes pz0..pz0+P-1: Y00 = S_y Z0, Y10 = D_y Z0, Y01 = S_y Z1
            // layout sY[kind][c][pl][py][a0]
            for (int it = tid; it < 5 * P * N; it += blockDim.x) {
                const int a0 = it % N, pl = (it / N) % P, c = it / (N * P);
                const int pz = pz0 + pl;
                if (pz >= Q) continue;
                Real z0[N], z1[N];
#pragma unroll
                for (int i = 0; i < N; ++i) {
                    z0[i] = sZ[(0 * 5 + c) * Q * N2 + pz * N2 + i * N + a0];
                    z1[i] = sZ[(1 * 5 + c) * Q * N2 + pz * N2 + i * N + a0];
                }
#pragma unroll
                for (int py = 0; py < Q; ++py) {
                    Real y00 = 0, y10 = 0, y01 = 0;
#pragma unroll
                    for (int i = 0; i < N; ++i) {
                        y00 += tb.S[py][i] * z0[i];
                        y10 += tb.D[py][i] * z0[i];
                        y01 += tb.S[py][i] * z1[i];
                    }
                    sY[((0 * 5 + c) * P + pl) * Q * N + py * N + a0] = y00;
                    sY[((1 * 5 + c) * P + pl) * Q * N + py * N + a0] = y10;
                    sY[((2 * 5 + c) * P + pl) * Q * N + py * N + a0] = y01;
                }
            }
            __syncthreads();

            // x-sweep + pointwise physics, one thread per quadrature point
            for (int it = tid; it < P * Q2; it += blockDim.x) {
                const int px = it % Q, py = (it / Q) % Q, pl = it / Q2;
                const int pz = pz0 + pl;
                if (pz >= Q) continue;
                Real Uq[5], Gr[5][3];
#pragma unroll
                for (int c = 0; c < 5; ++c) {
                    Real v = 0, dx = 0, dy = 0, dz = 0;
#pragma unroll
                    for (int i = 0; i < N; ++i) {
                        const Real y00 = sY[((0 * 5 + c) * P + pl) * Q * N + py * N + i];
                        const Real y10 = sY[((1 * 5 + c) * P + pl) * Q * N + py * N + i];
                        const Real y01 = sY[((2 * 5 + c) * P + pl) * Q * N + py * N + i];
                        v += tb.S[px][i] * y00;
                        dx += tb.D[px][i] * y00;
                        dy += tb.S[px][i] * y10;
                        dz += tb.S[px][i] * y01;
                    }
                    Uq[c] = v;
                    Gr[c][0] = dx;
                    Gr[c][1] = dy;
                    Gr[c][2] = dz;
                }
                Real J[9], jxw;
                const int p = px + Q * (py + Q * pz);
                if constexpr (GEN) {
                    const double* gm = a.cell_metric + e * 10 * Q3 + p;
#pragma unroll
                    for (int m = 0; m < 9; ++m) J[m] = (Real)gm[m * Q3];
                    jxw = (Real)gm[9 * Q3];
                } else {
#pragma unroll
                    for (int m = 0; m < 9; ++m) J[m] = Ji[m];
                    jxw = detJ * tb.w[px] * tb.w[py] * tb.w[pz];
                }
                // physical gradient G[c][j] = sum_d Jinv[d][j] Gr[c][d]
                Real G[5][3];
#pragma unroll
                for (int c = 0; c < 5; ++c)
#pragma unroll
                    for (int j = 0; j < 3; ++j)
                        G[c][j] = J[0 * 3 + j] * Gr[c][0] + J[1 * 3 + j] * Gr[c][1] + J[2 * 3 + j] * Gr[c][2];
                Real F[5][3];
#pragma unroll
                for (int c = 0; c < 5; ++c)
#pragma unroll
                    for (int j = 0; j < 3; ++j) F[c][j] = 0;
                if (conv) {
                    Real Fc[5][3];
                    convective_flux(Uq, ph, Fc);
#pragma unroll
                    for (int c = 0; c < 5; ++c)
#pragma unroll
                        for (int j = 0; j < 3; ++j) F[c][j] += Fc[c][j];
                }
                if (visc) {
                    Real Fv[5][3];
                    viscous_flux(Uq, G, ph, Fv);
#pragma unroll
                    for (int c = 0; c < 5; ++c)
#pragma unroll
                        for (int j = 0; j < 3; ++j) F[c][j] -= Fv[c][j];
                }
                // reference flux: w|J| J^{-1} F
#pragma unroll
                for (int c = 0; c < 5; ++c)
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        const Real fr = J[d * 3 + 0] * F[c][0] + J[d * 3 + 1] * F[c][1] + J[d * 3 + 2] * F[c][2];
                        sF[((c * 3 + d) * P + pl) * Q2 + py * Q + px] = jxw * fr;
                    }
            }
            __syncthreads();

            // x-transposed: B1 = D_x^T F_0, B2 = S_x^T F_1, B3 = S_x^T F_2   layout [kind][c][pl][py][a0]
            Real* sB = sY;
            for (int it = tid; it < 5 * P * Q * N; it += blockDim.x) {
                const int a0 = it % N, py = (it / N) % Q, pl = (it / (N * Q)) % P, c = it / (N * Q * P);
                if (pz0 + pl >= Q) continue;
                Real b1 = 0, b2 = 0, b3 = 0;
#pragma unroll
                for (int px = 0; px < Q; ++px) {
                    b1 += tb.D[px][a0] * sF[((c * 3 + 0) * P + pl) * Q2 + py * Q + px];
                    b2 += tb.S[px][a0] * sF[((c * 3 + 1) * P + pl) * Q2 + py * Q + px];
                    b3 += tb.S[px][a0] * sF[((c * 3 + 2) * P + pl) * Q2 + py * Q + px];
                }
                sB[((0 * 5 + c) * P + pl) * Q * N + py * N + a0] = b1;
                sB[((1 * 5 + c) * P + pl) * Q * N + py * N + a0] = b2;
                sB[((2 * 5 + c) * P + pl) * Q * N + py * N + a0] = b3;
            }
            __syncthreads();

            // y-transposed: E1 = S_y^T B1 + D_y^T B2, E2 = S_y^T B3   layout [kind][c][pl][a1][a0]
            Real* sE = sF;
            for (int it = tid; it < 5 * P * N2; it += blockDim.x) {
                const int a0 = it % N, a1 = (it / N) % N, pl = (it / N2) % P, c = it / (N2 * P);
                if (pz0 + pl >= Q) continue;
                Real e1 = 0, e2 = 0;
#pragma unroll
                for (int py = 0; py < Q; ++py) {
                    e1 += tb.S[py][a1] * sB[((0 * 5 + c) * P + pl) * Q * N + py * N + a0] +
                          tb.D[py][a1] * sB[((1 * 5 + c) * P + pl) * Q * N + py * N + a0];
                    e2 += tb.S[py][a1] * sB[((2 * 5 + c) * P + pl) * Q * N + py * N + a0];
                }
                sE[((0 * 5 + c) * P + pl) * N2 + a1 * N + a0] = e1;
                sE[((1 * 5 + c) * P + pl) * N2 + a1 * N + a0] = e2;
            }
            __syncthreads();

            // z-transposed, accumulated over the chunk's planes: R += S_z^T E1 + D_z^T E2
            for (int it = tid; it < 5 * N3; it += blockDim.x) {
                const int c = it / N3, r = it % N3, a2 = r / N2, r2 = r % N2;
                Real acc = 0;
#pragma unroll
                for (int pl = 0; pl < P; ++pl) {
                    const int pz = pz0 + pl;
                    if (pz < Q)
                        acc += tb.S[pz][a2] * sE[((0 * 5 + c) * P + pl) * N2 + r2] +
                               tb.D[pz][a2] * sE[((1 * 5 + c) * P + pl) * N2 + r2];
                }
                sR[it] += acc;
            }
            __syncthreads();
        }

        // ------------------------------------------------------------ face terms
        face_terms<0, N, Q, Real, GEN, Sz>(a, tb, ph, conv, visc, e, i0, i1, i2, Ji, detJ, sU, sR, sW);
        face_terms<1, N, Q, Real, GEN, Sz>(a, tb, ph, conv, visc, e, i0, i1, i2, Ji, detJ, sU, sR, sW);
        face_terms<2, N, Q, Real, GEN, Sz>(a, tb, ph, conv, visc, e, i0, i1, i2, Ji, detJ, sU, sR, sW);
    }

    // ------------------------------------------------------------ body force (k+1 rule)
    const bool force = (a.terms & 4u) != 0 && (a.force[0] != 0.0 || a.force[1] != 0.0 || a.force[2] != 0.0);
    const double* jxw_m = GEN ? a.mass_jxw + e * N3 : nullptr;
    if (force) {
        Real* t0b = sW;
        Real* t1b = sW + 5 * N3;
        // values at the mass points: (Sm)^{x3} U
        sweep_nn<N, Real, false>(mt.Sm, sU, t0b, 0);
        __syncthreads();
        sweep_nn<N, Real, false>(mt.Sm, t0b, t1b, 1);
        __syncthreads();
        sweep_nn<N, Real, false>(mt.Sm, t1b, t0b, 2);
        __syncthreads();
        for (int p = tid; p < N3; p += blockDim.x) {
            Real jxw;
            if constexpr (GEN) jxw = (Real)jxw_m[p];
            else jxw = detJ * mt.wm[p % N] * mt.wm[(p / N) % N] * mt.wm[p / N2];
            const Real rho = t0b[p];
            const Real f0 = (Real)a.force[0], f1 = (Real)a.force[1], f2 = (Real)a.force[2];
            const Real fu = (f0 * t0b[N3 + p] + f1 * t0b[2 * N3 + p] + f2 * t0b[3 * N3 + p]) / rho;
            t0b[p] = 0;
            t0b[N3 + p] = f0 * jxw;
            t0b[2 * N3 + p] = f1 * jxw;
            t0b[3 * N3 + p] = f2 * jxw;
            t0b[4 * N3 + p] = fu * jxw;
        }
        __syncthreads();
        sweep_nn<N, Real, true>(mt.Sm, t0b, t1b, 0);
        __syncthreads();
        sweep_nn<N, Real, true>(mt.Sm, t1b, t0b, 1);
        __syncthreads();
        sweep_nn<N, Real, true>(mt.Sm, t0b, t1b, 2);
        __syncthreads();
        for (int i = tid; i < 5 * N3; i += blockDim.x) sR[i] += t1b[i];
        __syncthreads();
    }

    if (a.fuse_minv) inverse_mass_lds<N, Real, GEN>(mt, sR, sW, detJ, jxw_m);

    for (int i = tid; i < 5 * N3; i += blockDim.x) {
        const int c = i / N3, j = i % N3;
        a.out[c * cstride + e * N3 + j] = (double)sR[i];
    }
}

// Standalone inverse mass: L = M^{-1} R (in place allowed: each cell reads its
// block into LDS before writing it back).
template <int N, typename Real, bool GEN>
__global__ void __launch_bounds__(kBlock)
inverse_mass_kernel(const double* R, double* L, int64_t ncell, const double* cell_metric, const double* mass_jxw,
                    MTab<N, Real> mt) {
    constexpr int N3 = N * N * N;
    __shared__ Real sR[5 * N3];
    __shared__ Real sW[5 * N3];
    const int64_t e = blockIdx.x;
    const int64_t cs = ncell * N3;
    for (int i = threadIdx.x; i < 5 * N3; i += blockDim.x) sR[i] = (Real)R[(i / N3) * cs + e * N3 + i % N3];
    Real detJ = 1;
    if constexpr (!GEN) detJ = (Real)cell_metric[e * 10 + 9];
    __syncthreads();
    inverse_mass_lds<N, Real, GEN>(mt, sR, sW, detJ, GEN ? mass_jxw + e * N3 : nullptr);
    for (int i = threadIdx.x; i < 5 * N3; i += blockDim.x) L[(i / N3) * cs + e * N3 + i % N3] = (double)sR[i];
}

// ------------------------------------------------------------------ dispatch
template <int N, int Q, typename Real, bool GEN>
inline int launch_op_t(const OpArgs& a, const Tables1D& t, hipStream_t st) {
    KTab<N, Q, Real> kt;
    MTab<N, Real> mt;
    for (int p = 0; p < Q; ++p) {
        for (int i = 0; i < N; ++i) {
            kt.S[p][i] = (Real)t.S[p][i];
            kt.D[p][i] = (Real)t.D[p][i];
        }
        kt.w[p] = (Real)t.w[p];
    }
    for (int s = 0; s < 2; ++s)
        for (int i = 0; i < N; ++i) {
            kt.fv[s][i] = (Real)t.fv[s][i];
            kt.fd[s][i] = (Real)t.fd[s][i];
        }
    for (int i = 0; i < N; ++i) {
        for (int j = 0; j < N; ++j) {
            mt.Sm[i][j] = (Real)t.Sm[i][j];
            mt.Smi[i][j] = (Real)t.Smi[i][j];
        }
        mt.wm[i] = (Real)t.wm[i];
    }
    // all n_q planes at once while the workgroup stays within 64 KB of LDS, else one plane at a time
    constexpr int P = (OpSizes<N, Q, Q>::WORK + 10 * N * N * N) * (int)sizeof(Real) <= 64 * 1024 ? Q : 1;
    static_assert((OpSizes<N, Q, P>::WORK + 10 * N * N * N) * sizeof(Real) <= 160 * 1024, "LDS budget");
    hipLaunchKernelGGL((dg_operator_kernel<N, Q, Real, GEN, P>), dim3((unsigned)a.ncell), dim3(kBlock), 0, st, a, kt, mt);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int N, typename Real, bool GEN>
inline int launch_minv_t(const double* R, double* L, int64_t ncell, const double* cm, const double* mj,
                         const Tables1D& t, hipStream_t st) {
    MTab<N, Real> mt;
    for (int i = 0; i < N; ++i) {
        for (int j = 0; j < N; ++j) {
            mt.Sm[i][j] = (Real)t.Sm[i][j];
            mt.Smi[i][j] = (Real)t.Smi[i][j];
        }
        mt.wm[i] = (Real)t.wm[i];
    }
    hipLaunchKernelGGL((inverse_mass_kernel<N, Real, GEN>), dim3((unsigned)ncell), dim3(kBlock), 0, st, R, L, ncell, cm,
                       mj, mt);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace dgns
