// High-degree operator kernels (k >= 8): the same weak form, sum factorisation and face
// terms as op_impl.h, for cells too large to hold in LDS.
//
// At k >= 8 one cell's coefficients and residual alone take 10 (k+1)^3 values (58 KB at
// k = 8, 328 KB at k = 15 in float64), so the resident design of op_impl.h (sU and sR in
// LDS beside the work area) no longer fits a compute unit's 160 KB.  Here a workgroup
// still evaluates one cell, but streams it through the quadrature planes along xi_2:
//  - per chunk of PL planes, the z-interpolation reads the coefficient lines of U from
//    global memory (they stay in the L2 / last-level cache across the chunks; sweeping
//    every plane once into scratch up front fetched a third as much at k = 15 but was up
//    to 10% slower, the up-front phase overlapping nothing);
//  - the chunk's intermediates live in LDS in two regions that alternate between the
//    phases (z-swept values, then point fluxes, then y-transposed sums in region A;
//    y-swept values, then x-transposed sums in region B);
//  - each chunk's y-transposed sums (the two planes E1, E2 per quadrature plane) go to
//    the cell's own area of a scratch buffer behind the face buffer; after the last
//    chunk one pass forms the z-transposed test sweep over all planes, adds the face
//    terms and writes the cell's rows of the output vector once (accumulating into the
//    output chunk by chunk instead read and wrote the whole residual block per chunk:
//    1.4 GB written per evaluation at k = 15, 0.25 GB this way); M^{-1} is the
//    stand-alone kernel applied afterwards.
// The face terms are evaluated once per face by dg_face_hd_kernel (one face of the cell
// at a time, own traces read from global memory) into the face buffer, as for the
// lower degrees.  The 1D tables come from the context's device copy of Tables1D (as
// kernel arguments they would exceed the argument space) into LDS.  Body forces are not
// supported at these degrees (the API rejects them).
#pragma once

#include <type_traits>

#include "dg_kernels.h"
#include "minv_impl.h"

namespace dgns {

constexpr int kHdBlock = 256;

// Cooperative copy of the 1D tables of (N, Q) from the float64 master into LDS.
template <int N, int Q, typename Real>
__device__ __forceinline__ void load_ktab(const Tables1D* t, KTab<N, Q, Real>& lt) {
    for (int i = threadIdx.x; i < Q * N; i += blockDim.x) {
        const int p = i / N, j = i % N;
        lt.S[p][j] = (Real)t->S[p][j];
        lt.D[p][j] = (Real)t->D[p][j];
    }
    for (int i = threadIdx.x; i < Q; i += blockDim.x) lt.w[i] = (Real)t->w[i];
    for (int i = threadIdx.x; i < 2 * N; i += blockDim.x) {
        lt.fv[i / N][i % N] = (Real)t->fv[i / N][i % N];
        lt.fd[i / N][i % N] = (Real)t->fd[i / N][i % N];
    }
}

// Cooperative fill of an even-odd table (see EOMat) from m(p, i), p < NO, i < NI.
template <int NO, int NI, typename Real, typename Get>
__device__ __forceinline__ void fill_eo_dev(EOMat<NO, NI, Real>& M, Get m) {
    constexpr int HO = (NO + 1) / 2, HI = NI / 2 > 0 ? NI / 2 : 1;
    for (int it = threadIdx.x; it < HO * HI; it += blockDim.x) {
        const int p = it / HI, i = it % HI;
        if (i < NI / 2) {
            M.E[p][i] = (Real)(0.5 * (m(p, i) + m(p, NI - 1 - i)));
            M.O[p][i] = (Real)(0.5 * (m(p, i) - m(p, NI - 1 - i)));
        }
    }
    for (int p = threadIdx.x; p < HO; p += blockDim.x) M.C[p] = (NI % 2) ? (Real)m(p, NI / 2) : Real(0);
}

// LDS plan of the streamed cell kernel: PL planes per chunk, as many as keep the two
// regions within about 60 KB (two workgroups, eight waves, per compute unit; 40 or 30 KB
// for the pairs listed below).  Rows of
// the flux arrays (pitch FP, over px) and of the y-swept / x-transposed arrays (pitch BP,
// over a0) that are a multiple of 128 bytes long are padded by one value: the sweeps
// read and write eight or more rows at once per wave, and with a pitch of 128 bytes
// every other row starts on the same bank (n_q = 16 in float64: the eight flux rows that
// a wave of the transposed x sweep reads fall on two bank positions).  Rows of 64 bytes
// (every fourth row aliased) stay unpadded: at k = 7, n_q = 11 in float64 and k = 10,
// n_q = 16 in float32 the padding would cost a workgroup per compute unit.
template <int N, int Q, typename Real>
struct HdPlan {
    static constexpr int RS = (int)sizeof(Real);
    static constexpr int FP = Q * RS % 128 == 0 ? Q + 1 : Q;
    static constexpr int BP = N * RS % 128 == 0 ? N + 1 : N;
    static constexpr int per_plane(int p) { return 15 * p * Q * (FP + BP); }
    // smaller chunks, for more workgroups per compute unit, where they measured faster at about
    // 10M DoFs (us per evaluation, 60 KB against the budget taken): float64 k=6 n_q=10 1449 ->
    // 1298 and k=8 n_q=9 809 -> 770 at 40 KB; float32 k=8 n_q=9 467 -> 436 and k=11 n_q=12 455
    // -> 423 at 30 KB, k=8 n_q=13 853 -> 813, k=9 n_q=10 523 -> 479, n_q=14 945 -> 805 and k=10
    // n_q=11 593 -> 569 at 40 KB.  Elsewhere 40 or 30 KB measured as fast or slower (to -12%).
    static constexpr int BUDGET_KB =
        RS == 8 ? (((N == 7 && Q == 10) || (N == 9 && Q == 9)) ? 40 : 60)
                : (((N == 9 && Q == 9) || (N == 12 && Q == 12))
                       ? 30
                       : (((N == 9 && Q == 13) || (N == 10 && (Q == 10 || Q == 14)) || (N == 11 && Q == 11)) ? 40 : 60));
    static constexpr int fit(int p) { return p <= 1 ? 1 : (per_plane(p) * RS <= BUDGET_KB * 1024 ? p : fit(p - 1)); }
    static constexpr int PL = fit(Q);
    static constexpr int RA = 15 * PL * Q * FP;  // z-swept [2][5][PL][N^2], fluxes [5][3][PL][Q][FP], E [2][5][PL][N^2]
    static constexpr int RB = 15 * PL * Q * BP;  // y-swept [3][5][PL][Q][BP], x-transposed [3][5][PL][Q][BP]
    static_assert(Q * FP >= N * N, "z-swept and E planes inside the flux planes");
    static_assert(Q >= N, "n_q >= k + 1");
    // even-odd sweeps where their tables do not cost a workgroup per compute unit (k = 13
    // in float64: 54,272 against 51,200 bytes, two against three workgroups; 1583 us per
    // evaluation with them, 1280 us without)
    static constexpr int LDS_NOEO = (RA + RB) * RS + (int)sizeof(KTab<N, Q, Real>) + 256;
    static constexpr int LDS_EO = LDS_NOEO + (int)sizeof(EOTab<N, Q, Real>);
    static constexpr bool EO = lds_wg_per_cu(LDS_EO) >= lds_wg_per_cu(LDS_NOEO);
};

// Cell term of the residual, streamed over the quadrature planes along xi_2 (see the
// file comment); then the six lifted face blocks of the face buffer.  Writes R to a.out.
template <int N, int Q, typename Real, bool GEN>
__global__ void __launch_bounds__(kHdBlock) __attribute__((amdgpu_waves_per_eu(2)))
dg_cell_hd_kernel(OpArgs a) {
    using HP = HdPlan<N, Q, Real>;
    constexpr int PL = HP::PL;
    constexpr int FP = HP::FP, BP = HP::BP, FPL = Q * FP, BPL = Q * BP;   // row pitches and plane sizes
    constexpr int N2 = N * N, N3 = N2 * N, Q2 = Q * Q, Q3 = Q2 * Q, FWB = 2 * 5 * N2;
    __shared__ Real rA[HP::RA];
    __shared__ Real rB[HP::RB];
    __shared__ KTab<N, Q, Real> lt;
    // even-odd forms of S and D for the y sweep and the transposed x and y sweeps
    constexpr bool EO = HP::EO;
    __shared__ std::conditional_t<EO, EOTab<N, Q, Real>, char> leo;
    constexpr int HN = N / 2, HQ = Q / 2, HON = (N + 1) / 2, HOQ = (Q + 1) / 2;
    const int64_t e = blockIdx.x;
    const int tid = threadIdx.x, nth = blockDim.x;
    const Phys<Real> ph = make_phys<Real>(a);
    const bool conv = (a.terms & 1u) != 0;
    const bool visc = (a.terms & 2u) != 0;
    const int64_t cstride = a.ncell * N3;
    const double* Ue = a.U + e * N3;
    double* Re = a.out + e * N3;
    // the cell's scratch area behind the face buffer: [n_q][2][5][N^2] values
    Real* ew = static_cast<Real*>(a.fw) + a.ncell * 6 * FWB + e * 10 * Q * N2;
    load_ktab<N, Q, Real>(a.tab_dev, lt);
    if constexpr (EO) {
        const Tables1D* t = a.tab_dev;
        fill_eo_dev(leo.S, [&](int p, int i) { return t->S[p][i]; });
        fill_eo_dev(leo.D, [&](int p, int i) { return t->D[p][i]; });
        fill_eo_dev(leo.St, [&](int i, int p) { return t->S[p][i]; });
        fill_eo_dev(leo.Dt, [&](int i, int p) { return t->D[p][i]; });
    }
    Real Ji[9], detJ = Real(1);
    if constexpr (!GEN) {
#pragma unroll
        for (int m = 0; m < 9; ++m) Ji[m] = (Real)a.cell_metric[e * 10 + m];
        detJ = (Real)a.cell_metric[e * 10 + 9];
    }
    __syncthreads();

    const bool cell = conv || visc;
    for (int pz0 = 0; cell && pz0 < Q; pz0 += PL) {
        const int np = Q - pz0 < PL ? Q - pz0 : PL;
        // z-sweep: Z0 = S_z U, Z1 = D_z U for the chunk's planes   rA [kind][c][pl][a1][a0]
        for (int it = tid; it < 5 * N2; it += nth) {
            const int c = it / N2, r = it % N2;
            Real v[N];
#pragma unroll
            for (int i = 0; i < N; ++i) v[i] = (Real)Ue[c * cstride + i * N2 + r];
            for (int pl = 0; pl < np; ++pl) {
                Real z0 = 0, z1 = 0;
#pragma unroll
                for (int i = 0; i < N; ++i) {
                    z0 += lt.S[pz0 + pl][i] * v[i];
                    z1 += lt.D[pz0 + pl][i] * v[i];
                }
                rA[((0 * 5 + c) * PL + pl) * N2 + r] = z0;
                rA[((1 * 5 + c) * PL + pl) * N2 + r] = z1;
            }
        }
        __syncthreads();
        if constexpr (EO) {
        // y-sweep: Y00 = S_y Z0, Y10 = D_y Z0, Y01 = S_y Z1   rB [kind][c][pl][py][a0], one
        // item per output pair (py, Q-1-py) in even-odd form
        for (int it = tid; it < 5 * np * HOQ * N; it += nth) {
            const int a0 = it % N, ph2 = (it / N) % HOQ, pl = (it / (N * HOQ)) % np, c = it / (N * HOQ * np);
            const Real* z0p = rA + ((0 * 5 + c) * PL + pl) * N2 + a0;
            const Real* z1p = rA + ((1 * 5 + c) * PL + pl) * N2 + a0;
            Real z0[N], z1[N];
#pragma unroll
            for (int i = 0; i < N; ++i) {
                z0[i] = z0p[i * N];
                z1[i] = z1p[i * N];
            }
            Real e0[HN], o0[HN], e1[HN], o1[HN];
            eo_split<N>(z0, e0, o0);
            eo_split<N>(z1, e1, o1);
            const int pm = Q - 1 - ph2;
            Real* y00p = rB + ((0 * 5 + c) * PL + pl) * BPL + a0;
            Real* y10p = rB + ((1 * 5 + c) * PL + pl) * BPL + a0;
            Real* y01p = rB + ((2 * 5 + c) * PL + pl) * BPL + a0;
            Real ev, ov;
            eo_row<Q, N>(leo.S, e0, o0, z0[N / 2], ph2, ev, ov);
            y00p[ph2 * BP] = ev + ov;
            if (ph2 != pm) y00p[pm * BP] = ev - ov;
            eo_row<Q, N>(leo.D, e0, o0, z0[N / 2], ph2, ev, ov);
            y10p[ph2 * BP] = ev + ov;
            if (ph2 != pm) y10p[pm * BP] = ov - ev;
            eo_row<Q, N>(leo.S, e1, o1, z1[N / 2], ph2, ev, ov);
            y01p[ph2 * BP] = ev + ov;
            if (ph2 != pm) y01p[pm * BP] = ev - ov;
        }
        } else {
        // y-sweep: Y00 = S_y Z0, Y10 = D_y Z0, Y01 = S_y Z1   rB [kind][c][pl][py][a0]
        for (int it = tid; it < 5 * np * Q * N; it += nth) {
            const int a0 = it % N, py = (it / N) % Q, pl = (it / (N * Q)) % np, c = it / (N * Q * np);
            const Real* z0p = rA + ((0 * 5 + c) * PL + pl) * N2 + a0;
            const Real* z1p = rA + ((1 * 5 + c) * PL + pl) * N2 + a0;
            Real y00 = 0, y10 = 0, y01 = 0;
#pragma unroll
            for (int i = 0; i < N; ++i) {
                const Real z0 = z0p[i * N], z1 = z1p[i * N];
                y00 += lt.S[py][i] * z0;
                y10 += lt.D[py][i] * z0;
                y01 += lt.S[py][i] * z1;
            }
            rB[((0 * 5 + c) * PL + pl) * BPL + py * BP + a0] = y00;
            rB[((1 * 5 + c) * PL + pl) * BPL + py * BP + a0] = y10;
            rB[((2 * 5 + c) * PL + pl) * BPL + py * BP + a0] = y01;
        }
        }
        __syncthreads();
        // x-sweep and pointwise physics, one point per item   rA [c][dim][pl][py][px]
        for (int it = tid; it < np * Q2; it += nth) {
            const int px = it % Q, py = (it / Q) % Q, pl = it / Q2, pz = pz0 + pl;
            Real Uq[5], Gr[5][3];
#pragma unroll
            for (int c = 0; c < 5; ++c) {
                const Real* y00p = rB + ((0 * 5 + c) * PL + pl) * BPL + py * BP;
                const Real* y10p = rB + ((1 * 5 + c) * PL + pl) * BPL + py * BP;
                const Real* y01p = rB + ((2 * 5 + c) * PL + pl) * BPL + py * BP;
                Real v = 0, dx = 0, dy = 0, dz = 0;
#pragma unroll 4
                for (int i = 0; i < N; ++i) {
                    v += lt.S[px][i] * y00p[i];
                    dx += lt.D[px][i] * y00p[i];
                    dy += lt.S[px][i] * y10p[i];
                    dz += lt.S[px][i] * y01p[i];
                }
                Uq[c] = v;
                Gr[c][0] = dx;
                Gr[c][1] = dy;
                Gr[c][2] = dz;
            }
            Real J[9], jxw;
            if constexpr (GEN) {
                const double* gm = a.cell_metric + e * 10 * Q3 + px + Q * (py + Q * pz);
#pragma unroll
                for (int m = 0; m < 9; ++m) J[m] = (Real)gm[m * Q3];
                jxw = (Real)gm[9 * Q3];
            } else {
#pragma unroll
                for (int m = 0; m < 9; ++m) J[m] = Ji[m];
                jxw = detJ * lt.w[px] * lt.w[py] * lt.w[pz];
            }
            const Prim<Real> sq = primitives(Uq, ph);
            Real F[5][3];
            if (conv) {
                convective_flux(Uq, sq, F);
            } else {
#pragma unroll
                for (int c = 0; c < 5; ++c)
#pragma unroll
                    for (int j = 0; j < 3; ++j) F[c][j] = 0;
            }
            if (visc) {
#pragma unroll
                for (int c = 0; c < 5; ++c) {
                    const Real g0 = Gr[c][0], g1 = Gr[c][1], g2 = Gr[c][2];
#pragma unroll
                    for (int j = 0; j < 3; ++j) Gr[c][j] = J[0 * 3 + j] * g0 + J[1 * 3 + j] * g1 + J[2 * 3 + j] * g2;
                }
                subtract_viscous_flux(sq, Gr, ph, F);
            }
#pragma unroll
            for (int c = 0; c < 5; ++c)
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const Real fr = J[d * 3 + 0] * F[c][0] + J[d * 3 + 1] * F[c][1] + J[d * 3 + 2] * F[c][2];
                    rA[((c * 3 + d) * PL + pl) * FPL + py * FP + px] = jxw * fr;
                }
        }
        __syncthreads();
        if constexpr (EO) {
        // x-transposed: B1 = D_x^T F_0, B2 = S_x^T F_1, B3 = S_x^T F_2   rB [kind][c][pl][py][a0],
        // one item per output pair (a0, N-1-a0) in even-odd form
        for (int it = tid; it < 5 * np * Q * HON; it += nth) {
            const int ah = it % HON, py = (it / HON) % Q, pl = (it / (HON * Q)) % np, c = it / (HON * Q * np);
            const int am = N - 1 - ah;
            Real* bp = rB + (c * PL + pl) * BPL + py * BP;
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                const Real* fr = rA + ((c * 3 + m) * PL + pl) * FPL + py * FP;
                Real f[Q];
#pragma unroll
                for (int px = 0; px < Q; ++px) f[px] = fr[px];
                Real ve[HQ], vo[HQ], ev, ov;
                eo_split<Q>(f, ve, vo);
                Real* b = bp + m * 5 * PL * BPL;
                if (m == 0) {
                    eo_row<N, Q>(leo.Dt, ve, vo, f[Q / 2], ah, ev, ov);
                    b[ah] = ev + ov;
                    if (ah != am) b[am] = ov - ev;
                } else {
                    eo_row<N, Q>(leo.St, ve, vo, f[Q / 2], ah, ev, ov);
                    b[ah] = ev + ov;
                    if (ah != am) b[am] = ev - ov;
                }
            }
        }
        } else {
        // x-transposed: B1 = D_x^T F_0, B2 = S_x^T F_1, B3 = S_x^T F_2   rB [kind][c][pl][py][a0]
        for (int it = tid; it < 5 * np * Q * N; it += nth) {
            const int a0 = it % N, py = (it / N) % Q, pl = (it / (N * Q)) % np, c = it / (N * Q * np);
            const Real* f0 = rA + ((c * 3 + 0) * PL + pl) * FPL + py * FP;
            const Real* f1 = rA + ((c * 3 + 1) * PL + pl) * FPL + py * FP;
            const Real* f2 = rA + ((c * 3 + 2) * PL + pl) * FPL + py * FP;
            Real b1 = 0, b2 = 0, b3 = 0;
#pragma unroll
            for (int px = 0; px < Q; ++px) {
                b1 += lt.D[px][a0] * f0[px];
                b2 += lt.S[px][a0] * f1[px];
                b3 += lt.S[px][a0] * f2[px];
            }
            rB[((0 * 5 + c) * PL + pl) * BPL + py * BP + a0] = b1;
            rB[((1 * 5 + c) * PL + pl) * BPL + py * BP + a0] = b2;
            rB[((2 * 5 + c) * PL + pl) * BPL + py * BP + a0] = b3;
        }
        }
        __syncthreads();
        if constexpr (EO) {
        // y-transposed: E1 = S_y^T B1 + D_y^T B2, E2 = S_y^T B3   rA [kind][c][pl][a1][a0], one
        // item per output pair (a1, N-1-a1) in even-odd form
        for (int it = tid; it < 5 * np * N * HON; it += nth) {
            const int a0 = it % N, ah = (it / N) % HON, pl = (it / (N * HON)) % np, c = it / (N * HON * np);
            const int am = N - 1 - ah;
            Real ve[HQ], vo[HQ], es, os, ed, od;
            Real bv[Q];
            const Real* b1 = rB + ((0 * 5 + c) * PL + pl) * BPL + a0;
            const Real* b2 = rB + ((1 * 5 + c) * PL + pl) * BPL + a0;
            const Real* b3 = rB + ((2 * 5 + c) * PL + pl) * BPL + a0;
#pragma unroll
            for (int py = 0; py < Q; ++py) bv[py] = b1[py * BP];
            eo_split<Q>(bv, ve, vo);
            eo_row<N, Q>(leo.St, ve, vo, bv[Q / 2], ah, es, os);
#pragma unroll
            for (int py = 0; py < Q; ++py) bv[py] = b2[py * BP];
            eo_split<Q>(bv, ve, vo);
            eo_row<N, Q>(leo.Dt, ve, vo, bv[Q / 2], ah, ed, od);
            Real* e1p = rA + ((0 * 5 + c) * PL + pl) * N2 + a0;
            Real* e2p = rA + ((1 * 5 + c) * PL + pl) * N2 + a0;
            e1p[ah * N] = (es + os) + (ed + od);
            if (ah != am) e1p[am * N] = (es - os) + (od - ed);
#pragma unroll
            for (int py = 0; py < Q; ++py) bv[py] = b3[py * BP];
            eo_split<Q>(bv, ve, vo);
            eo_row<N, Q>(leo.St, ve, vo, bv[Q / 2], ah, es, os);
            e2p[ah * N] = es + os;
            if (ah != am) e2p[am * N] = es - os;
        }
        } else {
        // y-transposed: E1 = S_y^T B1 + D_y^T B2, E2 = S_y^T B3   rA [kind][c][pl][a1][a0]
        for (int it = tid; it < 5 * np * N2; it += nth) {
            const int a0 = it % N, a1 = (it / N) % N, pl = (it / N2) % np, c = it / (N2 * np);
            const Real* b1 = rB + ((0 * 5 + c) * PL + pl) * BPL + a0;
            const Real* b2 = rB + ((1 * 5 + c) * PL + pl) * BPL + a0;
            const Real* b3 = rB + ((2 * 5 + c) * PL + pl) * BPL + a0;
            Real e1 = 0, e2 = 0;
#pragma unroll
            for (int py = 0; py < Q; ++py) {
                e1 += lt.S[py][a1] * b1[py * BP] + lt.D[py][a1] * b2[py * BP];
                e2 += lt.S[py][a1] * b3[py * BP];
            }
            rA[((0 * 5 + c) * PL + pl) * N2 + a1 * N + a0] = e1;
            rA[((1 * 5 + c) * PL + pl) * N2 + a1 * N + a0] = e2;
        }
        }
        __syncthreads();
        // the chunk's planes E1, E2 to the cell's scratch area   ew [pz][kind][c][a1][a0]
        for (int it = tid; it < 10 * np * N2; it += nth) {
            const int r2 = it % N2, c = (it / N2) % 5, kind = (it / (5 * N2)) % 2, pl = it / (10 * N2);
            ew[((pz0 + pl) * 2 + kind) * 5 * N2 + c * N2 + r2] = rA[((kind * 5 + c) * PL + pl) * N2 + r2];
        }
        // the next chunk's z-sweep overwrites rA; after the last chunk the barrier also
        // orders the scratch writes before the pass below reads them
        __syncthreads();
    }

    // R = S_z^T E1 + D_z^T E2 over all quadrature planes, plus the six lifted face blocks:
    // R(a, b, m) += W0 l_m(s) + W1 l_m'(s) along each face's normal
    const Real* fw = static_cast<const Real*>(a.fw) + e * 6 * FWB;
    for (int it = tid; it < 5 * N3; it += nth) {
        const int c = it / N3, r = it % N3;
        const int x0 = r % N, x1 = (r / N) % N, x2 = r / N2;
        double zt = 0.0;
        if (cell) {
            const Real* e1 = ew + c * N2 + (r % N2);
            for (int pz = 0; pz < Q; ++pz)
                zt += (double)(lt.S[pz][x2] * e1[pz * 10 * N2] + lt.D[pz][x2] * e1[pz * 10 * N2 + 5 * N2]);
        }
        Real acc = 0;
        if (cell) {
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const Real* w = fw + 3 * s * FWB + c * N2;
                acc += w[0 * FWB + x2 * N + x1] * lt.fv[s][x0] + w[0 * FWB + 5 * N2 + x2 * N + x1] * lt.fd[s][x0];
                acc += w[1 * FWB + x2 * N + x0] * lt.fv[s][x1] + w[1 * FWB + 5 * N2 + x2 * N + x0] * lt.fd[s][x1];
                acc += w[2 * FWB + x1 * N + x0] * lt.fv[s][x2] + w[2 * FWB + 5 * N2 + x1 * N + x0] * lt.fd[s][x2];
            }
        }
        Re[c * cstride + r] = cell ? zt + (double)acc : 0.0;
    }
}

// Workgroup of the streamed face kernel: one face point per thread, 128 threads where the
// n_q^2 points of a face fit at k >= 8 (k = 8..10 at n_q = k+1), else 256 (at k = 6, 7,
// n_q = 10, 11 the two-wave register budget of 128 threads spills 500-700 dwords).
// Float64 at 128 threads and at k >= 13 keeps the traces inside the t0-sweep area (see
// FaceSizes), which frees LDS for more workgroups per compute unit: k = 9 three -> four
// (709 -> 691 us per evaluation at about 10M DoFs), k = 13..15 one -> two, there with the
// registers held to two waves per SIMD (k = 13 1013 -> 931 us, k = 14 889 -> 806 with 6
// dwords spilled, k = 15 1067 -> 1003 with 32).
template <int N, int Q, typename Real>
struct HdFaceBlock {
    static constexpr bool F64 = sizeof(Real) == 8;
    static constexpr int B = N >= 9 && Q * Q <= 128 ? 128 : kHdBlock;
    // waves per SIMD the registers are held to (256 registers at two)
    static constexpr int W = (B == 128 || (F64 && N >= 14)) ? 2 : 1;
    static constexpr bool TRIN = F64 && (B == 128 || N >= 14);
};

// Face terms once per face (see dg_face_kernel in op_impl.h), one face of the cell at a
// time so that the traces of both sides fit in LDS; the cell's own traces come from
// global memory.  One face point per thread: n_q^2 <= 256.
template <int N, int Q, typename Real, bool GEN>
__global__ void __launch_bounds__((HdFaceBlock<N, Q, Real>::B)) __attribute__((amdgpu_waves_per_eu(HdFaceBlock<N, Q, Real>::W)))
dg_face_hd_kernel(OpArgs a) {
    using HB = HdFaceBlock<N, Q, Real>;
    using FS = FaceSizes<N, Q, HB::B, 1, false, HB::TRIN>;
    constexpr int N2 = N * N, Q2 = Q * Q, FWB = 2 * 5 * N2;
    static_assert(FS::ALIAS, "one face point per thread");
    __shared__ Real sW[FS::TOTAL];
    __shared__ FaceInfo fi;
    __shared__ Real sTau[6];
    __shared__ Real sFn[12];
    __shared__ Real sJr[GEN ? 1 : 27];
    __shared__ KTab<N, Q, Real> lt;

    const int64_t e = blockIdx.x;
    const int tid = threadIdx.x;
    const Phys<Real> ph = make_phys<Real>(a);
    const bool conv = (a.terms & 1u) != 0;
    const bool visc = (a.terms & 2u) != 0;
    Real* fw = static_cast<Real*>(a.fw);
    load_ktab<N, Q, Real>(a.tab_dev, lt);
    face_info_setup<Real, GEN>(a, e, fi, sTau, sFn, sJr);
    Real detJ = Real(1);
    if constexpr (!GEN) detJ = (Real)a.cell_metric[e * 10 + 9];
    __syncthreads();

    Real* out = sW + FS::OUT_OFF;
    Real* t1 = sW + FS::T1_OFF;
    Real* o = out + tid;
    const bool act = tid < Q2;
    Real res[20], res1[15];
    // the faces xi_d = 1, both sides
#pragma unroll 1
    for (int d = 0; d < 3; ++d) {
        face_traces_sweep<N, Q, Real, 1, FS, true>(a, lt, 1, d, fi, nullptr, sW);
        if (act) face_point<N, Q, Real, GEN, true>(a, lt, ph, conv, visc, 1, d, fi, sTau, sFn, sJr, detJ, sW, tid, res, res1);
        __syncthreads();
        if (act) {
#pragma unroll
            for (int m = 0; m < 20; ++m) o[m * Q2] = res[m];
        }
        __syncthreads();
        face_lift<N, Q, Real, 1>(lt, out, t1, [&](int) { return fw + (e * 6 + 3 + d) * FWB; });
        // the other side's coefficients replace the own side's (its lift has read them)
        if (act) {
#pragma unroll
            for (int c = 0; c < 5; ++c) o[c * Q2] = -res[c];
#pragma unroll
            for (int m = 0; m < 15; ++m) o[(5 + m) * Q2] = res1[m];
        }
        __syncthreads();
        face_lift<N, Q, Real, 1>(lt, out, t1, [&](int) { return fi.wall[3 + d] ? nullptr : fw + (fi.enb[3 + d] * 6 + d) * FWB; });
        __syncthreads();
    }
    // wall faces xi_d = 0: the own side only
#pragma unroll 1
    for (int d = 0; d < 3; ++d) {
        if (!fi.wall[d]) continue;   // uniform over the workgroup
        face_traces_sweep<N, Q, Real, 1, FS, true>(a, lt, 0, d, fi, nullptr, sW);
        if (act) face_point<N, Q, Real, GEN>(a, lt, ph, conv, visc, 0, d, fi, sTau, sFn, sJr, detJ, sW, tid, res, res1);
        __syncthreads();
        if (act) {
#pragma unroll
            for (int m = 0; m < 20; ++m) o[m * Q2] = res[m];
        }
        __syncthreads();
        face_lift<N, Q, Real, 1>(lt, out, t1, [&](int) { return fw + (e * 6 + d) * FWB; });
        __syncthreads();
    }
}

// Stand-alone inverse mass of the high degrees: RPB = 256 / N^2 (component, cell) blocks per
// workgroup (3 at N = 9, 2 at N = 10, 11, else 1), one line of N values per thread and axis,
// tables from the device copy.  In LDS a block is stored with x-lines XP values apart and
// xi_2-planes YP apart; an x-line of 64 or 128 bytes (N = 16) is padded by one value, since
// consecutive threads own consecutive lines and would otherwise fall on 4 or 2 bank positions.
template <int N, typename Real>
struct MinvHdPlan {
    static constexpr int RPB = kHdBlock / (N * N) > 0 ? kHdBlock / (N * N) : 1;
    // the whole inverse in registers while it fits (float32, N <= 11: 3-5% faster there),
    // else one output at a time from LDS
    static constexpr bool REG = sizeof(Real) == 4 && N <= 11;
    // even-odd rows (minv_line_eo) where they measured faster than whole rows from LDS, odd
    // N >= 11 (at about 10M DoFs, us per launch: N = 13 106 -> 89 in float64, 78 -> 71 in
    // float32; N = 15 92 -> 79 and 68 -> 62; N = 11 float64 72 -> 70); at even N they measured
    // 1-33% slower
    static constexpr bool EO = !REG && N % 2 == 1 && N >= 11;
    static constexpr int XP = N * (int)sizeof(Real) % 64 == 0 ? N + 1 : N;
    static constexpr int YP = N * XP;
    static constexpr int BS = N * YP;
};

// One line of the inverse mass: out(o, sum_m M[o][m] v[m]) for o < N, from the row o of M,
// which the caller passes transposed for M^T; the line's input stays in registers, so the
// outputs may overwrite it in place.  REG: completely unrolled (all of M in registers);
// otherwise one output at a time (unrolled by two), since holding M in registers exceeds
// the register file for N >= 11 in float64.
template <int N, bool REG, typename Real, typename Put>
__device__ __forceinline__ void minv_line_hd(const Real (&M)[N][N], const Real (&v)[N], Put put) {
    if constexpr (REG) {
        Real t[N];
#pragma unroll
        for (int o = 0; o < N; ++o) {
            Real acc = 0;
#pragma unroll
            for (int m = 0; m < N; ++m) acc += M[o][m] * v[m];
            t[o] = acc;
        }
#pragma unroll
        for (int o = 0; o < N; ++o) put(o, t[o]);
    } else {
#pragma unroll 2
        for (int o = 0; o < N; ++o) {
            Real acc = 0;
#pragma unroll
            for (int m = 0; m < N; ++m) acc += M[o][m] * v[m];
            put(o, acc);
        }
    }
}

// One line of the inverse mass in even-odd form (see EOMat): S^{-1} and its transpose are
// centrosymmetric, since the mass points and the nodes are symmetric about the cell centre,
// so the outputs o and N-1-o come from one row pair of E and O, half the multiply-adds of
// minv_line_hd.  The line's input stays in registers, so the outputs may overwrite it.
template <int N, typename Real, typename Put>
__device__ __forceinline__ void minv_line_eo(const EOMat<N, N, Real>& M, const Real (&v)[N], Put put) {
    constexpr int HI = N / 2 > 0 ? N / 2 : 1, HO = (N + 1) / 2;
    Real ve[HI], vo[HI];
    eo_split<N>(v, ve, vo);
#pragma unroll 2
    for (int p = 0; p < HO; ++p) {
        Real e, o;
        eo_row<N, N>(M, ve, vo, v[N / 2], p, e, o);
        put(p, e + o);
        if (p != N - 1 - p) put(N - 1 - p, e - o);
    }
}

template <int N, typename Real, bool GEN>
__global__ void __launch_bounds__(kHdBlock)
inverse_mass_hd_kernel(const double* R, double* L, int64_t ncell, const double* cell_metric, const double* mass_jxw,
                       const Tables1D* t) {
    using MP = MinvHdPlan<N, Real>;
    constexpr int N2 = N * N, N3 = N2 * N, RPB = MP::RPB, XP = MP::XP, YP = MP::YP;
    static_assert(N2 <= kHdBlock, "one line per thread");
    __shared__ Real buf[RPB * MP::BS];
    // S^{-1} and its transpose: whole rows, or in even-odd form
    using MT = std::conditional_t<MP::EO, EOMat<N, N, Real>, Real[N][N]>;
    __shared__ MT Smi;
    __shared__ MT SmiT;
    __shared__ Real lwm[N];
    const int tid = threadIdx.x;
    if constexpr (MP::EO) {
        fill_eo_dev(Smi, [&](int p, int i) { return t->Smi[p][i]; });
        fill_eo_dev(SmiT, [&](int p, int i) { return t->Smi[i][p]; });
    } else {
        for (int i = tid; i < N2; i += blockDim.x) {
            Smi[i / N][i % N] = (Real)t->Smi[i / N][i % N];
            SmiT[i % N][i / N] = (Real)t->Smi[i / N][i % N];
        }
    }
    const auto line = [&](const MT& M, const Real (&v)[N], auto put) {
        if constexpr (MP::EO) minv_line_eo<N>(M, v, put);
        else minv_line_hd<N, MP::REG>(M, v, put);
    };
    if (tid < N) lwm[tid] = (Real)t->wm[tid];
    const int lb = tid / N2, ln = tid % N2, l0 = ln % N, l1 = ln / N;
    const int64_t row = (int64_t)blockIdx.x * RPB + lb;   // c * ncell + e
    const bool act = lb < RPB && row < 5 * ncell;
    Real* blk = buf + lb * MP::BS;
    // the thread's line along x (a1 = l0, a2 = l1), along y (a0 = l0, a2 = l1) and along
    // z (a0 = l0, a1 = l1) in the LDS block
    Real* xl = blk + l0 * XP + l1 * YP;
    Real* yl = blk + l0 + l1 * YP;
    Real* zl = blk + l0 + l1 * XP;
    Real v[N];
    if (act) {
        const double* src = R + row * N3 + ln * N;
#pragma unroll
        for (int m = 0; m < N; ++m) v[m] = (Real)src[m];
    }
    __syncthreads();
    if (act) line(SmiT, v, [&](int o, Real r) { xl[o] = r; });
    __syncthreads();
    if (act) {
#pragma unroll
        for (int m = 0; m < N; ++m) v[m] = yl[m * XP];
        line(SmiT, v, [&](int o, Real r) { yl[o * XP] = r; });
    }
    __syncthreads();
    if (act) {
        // z: S^{-T}, the diagonal 1 / (|J| w) at the mass points, then S^{-1}, on the
        // thread's own line (its writes are visible to its own later reads)
#pragma unroll
        for (int m = 0; m < N; ++m) v[m] = zl[m * YP];
        line(SmiT, v, [&](int o, Real r) { zl[o * YP] = r; });
        const int64_t e = row % ncell;
        if constexpr (GEN) {
            const double* jw = mass_jxw + e * N3 + ln;
#pragma unroll
            for (int m = 0; m < N; ++m) v[m] = zl[m * YP] / (Real)jw[m * N2];
        } else {
            const Real f = Real(1) / ((Real)cell_metric[e * 10 + 9] * lwm[l0] * lwm[l1]);
#pragma unroll
            for (int m = 0; m < N; ++m) v[m] = zl[m * YP] * (f / lwm[m]);
        }
        line(Smi, v, [&](int o, Real r) { zl[o * YP] = r; });
    }
    __syncthreads();
    if (act) {
#pragma unroll
        for (int m = 0; m < N; ++m) v[m] = yl[m * XP];
        line(Smi, v, [&](int o, Real r) { yl[o * XP] = r; });
    }
    __syncthreads();
    if (act) {
#pragma unroll
        for (int m = 0; m < N; ++m) v[m] = xl[m];
        double* dst = L + row * N3 + ln * N;
        line(Smi, v, [&](int o, Real r) { dst[o] = (double)r; });
    }
}

template <int N, typename Real, bool GEN>
inline int launch_minv_hd_t(const double* R, double* L, int64_t ncell, const double* cm, const double* mj,
                            const Tables1D* t_dev, hipStream_t st) {
    constexpr int RPB = MinvHdPlan<N, Real>::RPB;
    const int64_t grid = (5 * ncell + RPB - 1) / RPB;
    hipLaunchKernelGGL((inverse_mass_hd_kernel<N, Real, GEN>), dim3((unsigned)grid), dim3(kHdBlock), 0, st, R, L,
                       ncell, cm, mj, t_dev);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// One evaluation at the high degrees: face kernel, streamed cell kernel (R into the output,
// or into the stage's next-state buffer), then M^{-1} in place and, for a fused Runge-Kutta
// stage, the stage update from that buffer.
template <int N, int Q, typename Real, bool GEN>
inline int launch_op_hd_t(const OpArgs& a0, hipStream_t st) {
    OpArgs a = a0;
    const bool stage = a.rk.dU != nullptr;
    if (stage) a.out = a.rk.U_out;
    const dim3 grid((unsigned)a.ncell);
    constexpr int FB = HdFaceBlock<N, Q, Real>::B;
    if (a.terms & 3u) hipLaunchKernelGGL((dg_face_hd_kernel<N, Q, Real, GEN>), grid, dim3(FB), 0, st, a);
    hipLaunchKernelGGL((dg_cell_hd_kernel<N, Q, Real, GEN>), grid, dim3(kHdBlock), 0, st, a);
    if (hipGetLastError() != hipSuccess) return -1;
    if (a.fuse_minv || stage) {
        if (launch_minv_hd_t<N, Real, GEN>(a.out, a.out, a.ncell, a.cell_metric, a.mass_jxw, a.tab_dev, st) != 0)
            return -1;
    }
    if (stage)
        return launch_rk_update_to(a.U, a.rk.U_out, a.rk.dU, a.rk.U_out, 5 * a.ncell * N * N * N, a.rk.A, a.rk.B,
                                   a.rk.dt, st);
    return 0;
}

}  // namespace dgns
