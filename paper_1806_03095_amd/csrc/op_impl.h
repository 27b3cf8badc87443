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
// Work organisation: a workgroup of B threads; every phase is a cooperative loop
// over independent items (lines of a sweep, quadrature points) separated by
// barriers.  The cell's quadrature points are processed in chunks of P planes
// along xi_2; the faces in groups (the three faces xi_d = 0, then the three faces
// xi_d = 1, each phase covering all three faces of a group; or one face per group
// where the LDS plan asks for it, see OpSizes).  The sweep along the second
// tangential direction of a face is fused into the pointwise flux phase (each face
// point contracts its own line), so no n_q^2 intermediate is stored.  LDS holds
// sU[5][N^3] (own coefficients), sR[5][N^3] (residual), copies of the 1D tables
// and a work area sized for the largest phase.  With a Runge-Kutta stage attached
// (OpArgs::rk), the epilogue applies the stage update instead of writing L.

#pragma once

#include "dg_common.h"

namespace dgns {

template <int A, int B>
struct CMax { static constexpr int v = A > B ? A : B; };

template <int N, int Q, int B, int NF = 3, bool FUSED = (N <= 4), bool TRIN = false>
struct FaceSizes {
    static constexpr int N2 = N * N, Q2 = Q * Q;
    // FUSED: the traces are computed inside the sweep along t0 and never stored.
    static constexpr bool FUSED_TRACE = FUSED;
    // group of NF faces xi_d = s (NF = 3: all three directions; NF = 1: one face)
    static constexpr int TR = FUSED_TRACE ? 0 : NF * 2 * 2 * 5 * N2;   // traces [f][side][v/n][c][N^2]
    static constexpr int SW = NF * 2 * 3 * 5 * N * Q;   // t0 sweep [f][side][3][c][N][Q]
    static constexpr int OUT = NF * 4 * 5 * Q2;         // point outputs [f][4][c][Q^2]
    static constexpr int T1 = NF * 3 * 5 * N * Q;       // t1-transposed [f][3][c][N][Q]
    static constexpr int W = NF * 2 * 5 * N2;           // lifted [f][2][c][N^2]
    // Two regions that alternate between phases: R1 = {SW, T1}, R2 = {TR, OUT, W}.
    static constexpr int R1 = CMax<SW, T1>::v;
    static constexpr int R2 = CMax<CMax<TR, OUT>::v, W>::v;
    static constexpr int SPLIT_TOTAL = R1 + R2;
    // With one face point per thread, OUT can overwrite SW (the point results wait
    // in registers across a barrier): SW | TR, then OUT | T1, then W | T1.
    static constexpr bool ALIAS = NF * Q2 <= B;
    // TRIN: the traces also lie at the start of SW.  With one t0-sweep item per thread, each
    // item loads its two trace lines into registers before a barrier and then writes its
    // sweep over them, so TR takes no room of its own.
    static constexpr bool TR_IN_SW = TRIN && ALIAS && !FUSED && NF * 2 * 5 * N <= B;
    static_assert(!TRIN || TR_IN_SW, "traces inside SW: one face point and one sweep item per thread");
    static_assert(TR <= SW, "traces fit in SW");
    static constexpr int TR_OFF = TR_IN_SW ? 0 : (ALIAS ? SW : R1);
    static constexpr int OUT_OFF = ALIAS ? 0 : R1;
    static constexpr int T1_OFF = ALIAS ? OUT : 0;
    static constexpr int TOTAL = TR_IN_SW ? CMax<CMax<SW, OUT + T1>::v, W>::v
                                          : (ALIAS ? CMax<CMax<SW + TR, OUT + T1>::v, W>::v : SPLIT_TOTAL);
};

template <int N, int Q, int P>
struct CellSizes {
    static constexpr int N2 = N * N, Q2 = Q * Q;
    static constexpr int Z = 10 * Q * N2;   // z-sweeps: value, derivative
    static constexpr int Y = 15 * P * Q * N;  // y-sweeps (3 kinds), later x-transposed
    static constexpr int F = 15 * P * Q2;     // reference fluxes, later y-transposed
    static constexpr int TOTAL = Z + Y + F;
};

// Planes per chunk: as many as fit in the split face-phase layout (at least one).
template <int N, int Q>
struct ChooseP {
    static constexpr int fit(int p) {
        return p <= 1 ? 1 : (CellSizes<N, Q, 1>::TOTAL + (p - 1) * (15 * Q * N + 15 * Q * Q) <= FaceSizes<N, Q, 1>::SPLIT_TOTAL ? p : fit(p - 1));
    }
    static constexpr int v = fit(Q);
};

// LDS plan of the operator kernel for block size B and RS-byte reals: the number NF
// of faces per face group, the number P of planes per cell chunk, the work area
// (largest of the cell chunk, the face group and the mass-matrix sweeps) and whether
// the 1D table copies fit beside it.  The preferred plan is three faces per group
// and ChooseP's plane count.  When LDS keeps that plan below two waves per SIMD
// (eight per compute unit):
//  - fewer planes, if that reaches two waves;
//  - else, for 256-thread workgroups, one face per group if that reaches two waves
//    and the face-point phase still gains: 3 ceil(n_q^2 / B) passes at w1 waves per
//    SIMD against ceil(3 n_q^2 / B) passes at w3 waves;
//  - else one face per group only when three faces leave no room for the tables.
template <int N, int Q, int B, int RS, bool FUSED = (N <= 4), bool SPLIT = false>
struct OpSizes {
    static constexpr int N3 = N * N * N, Q2 = Q * Q;
    // KTab + MTab entries, and the even-odd tables of the cell sweeps (EOTab)
    static constexpr int TABLES = 2 * Q * N + Q + 4 * N + 2 * N * N + N +
                                  2 * ((Q + 1) / 2) * (2 * (N / 2 > 0 ? N / 2 : 1) + 1) +
                                  2 * ((N + 1) / 2) * (2 * (Q / 2 > 0 ? Q / 2 : 1) + 1);
    static constexpr int LDS_MAX = 160 * 1024;
    // LDS per workgroup at eight waves per CU; for the float32 kernels whose registers allow
    // more, fewer planes per chunk for 12 or 16 waves where that measured faster (k=3, n_q=6
    // and 7: 467 -> 443 and 795 -> 646 us; k=4, n_q=6 and 7: 431 -> 401 and 606 -> 582 us;
    // elsewhere the extra chunks cost more than the occupancy gains, up to 19%)
    static constexpr int WAVES_CU = RS != 4 ? 8 : ((N == 4 && (Q == 6 || Q == 7)) ? 16 : ((N == 5 && (Q == 6 || Q == 7)) ? 12 : 8));
    static constexpr int TARGET = kLdsGranules / (WAVES_CU * 64 / B) * kLdsGranule;
    static constexpr int cell(int p) { return 10 * Q * N * N + 15 * p * Q * (N + Q); }
    // the face phases, or with the face terms in a kernel of their own (SPLIT) the staging
    // of the cell's six lifted face blocks
    static constexpr int face(int nf) {
        return SPLIT ? 6 * 2 * 5 * N * N
                     : (nf == 3 ? FaceSizes<N, Q, B, 3, FUSED>::TOTAL : FaceSizes<N, Q, B, 1, FUSED>::TOTAL);
    }
    static constexpr int work(int nf, int p) {
        return cell(p) > face(nf) ? (cell(p) > 10 * N3 ? cell(p) : 10 * N3) : (face(nf) > 10 * N3 ? face(nf) : 10 * N3);
    }
    static constexpr int lds(int nf, int p) { return (work(nf, p) + 10 * N3 + TABLES) * RS + 1024; }
    static constexpr int fewer(int nf, int p) { return p <= 1 || lds(nf, p) <= TARGET ? p : fewer(nf, p - 1); }
    // waves per SIMD that the LDS footprint allows, at most two (the register budget)
    static constexpr int waves(int bytes) {
        return lds_wg_per_cu(bytes) * (B / 64) / 4 < 2 ? lds_wg_per_cu(bytes) * (B / 64) / 4 : 2;
    }
    static constexpr int P0 = SPLIT ? Q : ChooseP<N, Q>::v;
    static constexpr bool REACH3 = lds(3, fewer(3, P0)) <= TARGET;
    static constexpr bool REACH1 = B == 256 && lds(1, fewer(1, P0)) <= TARGET &&
                                   3 * ((Q2 + B - 1) / B) * waves(lds(3, P0)) <
                                       ((3 * Q2 + B - 1) / B) * waves(lds(1, fewer(1, P0)));
    static constexpr int NF = REACH3 ? 3 : (REACH1 ? 1 : (lds(3, P0) <= LDS_MAX ? 3 : 1));
    static constexpr int P = SPLIT || lds(NF, fewer(NF, P0)) <= TARGET ? fewer(NF, P0) : P0;
    static constexpr int CELL = cell(P);
    static constexpr int WORK = work(NF, P);
    static constexpr bool LDS_TAB = lds(NF, P) <= LDS_MAX;
    static_assert(CELL == CellSizes<N, Q, P>::TOTAL, "cell work area");
};

// Workgroup size of the operator kernel: 64 threads (one wave) per cell when the
// n_q^3 cell points fit in one wave (n_q <= 4): such small cells would leave most of a
// larger workgroup idle in every phase, and one-wave workgroups put twice as many
// cells on a compute unit.  Otherwise 128 threads (two waves) while four workgroups
// fit in a compute unit's LDS, so that every SIMD holds two waves; 256 threads for
// the larger (N, n_q) whose LDS footprint allows fewer workgroups (unless the 1D
// tables do not fit in LDS: that kernel spills, and more waves of it only add spill
// traffic).
// The face kernel (each face once, both sides lifted): one workgroup per cell for its
// three faces xi_d = 1 (and its wall faces xi_d = 0), one face point per thread --
// 64 threads for n_q <= 4, else 128 or 256 as 3 n_q^2 requires.  The face terms move to
// this kernel (SPLIT) for every (N, n_q, precision) where one pass covers the points
// of the three faces and the plan fits a compute unit.
// LDS layout of the face kernel's copy of the cell's coefficients: component stride CS
// and xi_2-plane stride PS, padded where that spreads the trace phase's reads over the
// banks (a model of the 64 banks: at N = 4 the fused trace reads take 160 bank passes
// unpadded against 44 padded, at N = 6 192 against 146, at N = 8 1040 against 280).
template <int N>
struct FaceSU {
    static constexpr int PS = N == 4 ? 17 : (N == 6 ? 37 : (N == 8 ? 67 : N * N));
    static constexpr int CS = N == 4 ? 75 : (N == 6 ? 228 : (N == 8 ? 536 : N * N * N));
};

template <int N, int Q, typename Real>
struct FaceBlock {
    static constexpr bool fused = N <= 4;
    template <int B>
    static constexpr int lds_for = (FaceSizes<N, Q, B, 3, fused>::TOTAL + 5 * FaceSU<N>::CS + 2 * Q * N + Q + 4 * N) *
                                       (int)sizeof(Real) + 1024;
    // 128 threads only while four workgroups fit in a compute unit's LDS (two waves per SIMD)
    static constexpr int threads = Q <= 4 ? 64 : (3 * Q * Q <= 128 && lds_for<128> <= 40 * 1024 ? 128 : 256);
    using FS = FaceSizes<N, Q, threads, 3, fused>;
    using FS1 = FaceSizes<N, Q, threads, 1, fused>;
    static constexpr bool one_pass = 3 * Q * Q <= threads;
    static constexpr int lds = lds_for<threads>;
    static_assert(FS1::TOTAL <= FS::TOTAL, "single-face layout inside the three-face layout");
};

// Measured on MI355X (about 10M DoFs per mesh, DoF/s of one evaluation with and without the
// face kernel): the split is 2-22% faster for k >= 2 except k=5 n_q=6 float32 (9% slower)
// and k=7 n_q=8 float64 (17% slower), and 5-8% slower for k = 1 except k=1 n_q=3 float32;
// those keep the element-centric faces.
template <int N, int Q, typename Real>
constexpr bool split_measured_slower() {
    constexpr bool fp64 = sizeof(Real) == sizeof(double);
    return (N == 2 && (fp64 || Q == 2)) || (N == 6 && Q == 6 && !fp64) || (N == 8 && Q == 8 && fp64);
}

template <int N, int Q, typename Real>
struct FaceSplit {
    static constexpr bool value = FaceBlock<N, Q, Real>::one_pass && FaceBlock<N, Q, Real>::lds <= 160 * 1024 &&
                                  !split_measured_slower<N, Q, Real>();
};

template <int N, int Q, typename Real>
struct OpBlock {
    static constexpr bool split = FaceSplit<N, Q, Real>::value;
    using S128 = OpSizes<N, Q, 128, (int)sizeof(Real), (N <= 4), split>;
    using S128F = OpSizes<N, Q, 128, (int)sizeof(Real), true, split>;
    static constexpr int lds128 = (S128::WORK + 10 * N * N * N + S128::TABLES) * (int)sizeof(Real) + 1024;
    static constexpr int lds128f = (S128F::WORK + 10 * N * N * N + S128F::TABLES) * (int)sizeof(Real) + 1024;
    // traces fused into the t0 sweep: always for N <= 4; for larger N only where dropping
    // their LDS area is what admits 128-thread workgroups (for N >= 5 the separate trace
    // phase is otherwise faster: more items per phase)
    static constexpr bool fused = N <= 4 || (!split && lds128 > 40 * 1024 && lds128f <= 40 * 1024 && S128F::LDS_TAB);
    static constexpr int threads =
        Q <= 4 ? 64 : (((fused ? lds128f : lds128) <= 40 * 1024 || !S128::LDS_TAB) ? 128 : 256);
    // even-odd form of the cell term's sweeps: measured 5-7% faster for k = 3, 5, 7 (float64
    // and float32), even at k = 3 n_q = 4 and k = 4 n_q = 7, and 2% slower at k = 2
    static constexpr bool even_odd = N >= 4;
};

// Loops that the compiler would otherwise unroll completely and whose operands it then
// loads all ahead, past the register budget (spills): unrolled only partly where that
// measured faster at about 10M DoFs.  face: the line loop of a face point (by four) and
// the output loop of the traces' first tangential sweep (not unrolled); cell: the x
// contraction at a cell point (by three).  Float64: k = 5 (both n_q: 918 -> 764 and
// 1090 -> 988 us) and k = 6, n_q = 7 (1070 -> 911 us), which no longer spill; float32
// (face only): k = 6, n_q = 7 (511 -> 457 us) and k = 7, n_q = 8 (355 -> 337 us); and
// every degree >= 8.  Elsewhere the full unroll measured as fast or faster (k = 4: up to
// 11% slower limited; k = 5 float32: 6-10% slower).
template <int N, int Q, typename Real>
struct UnrollLimit {
    static constexpr bool fp64 = sizeof(Real) == sizeof(double);
    static constexpr bool face = N > 8 || (fp64 && (N == 6 || (N == 7 && Q == 7))) ||
                                 (!fp64 && ((N == 7 && Q == 7) || (N == 8 && Q == 8)));
    static constexpr bool cell = fp64 && (N == 6 || (N == 7 && Q == 7));
};

// Applies an N x N matrix M along axis `ax` of the NC arrays src[NC][N^3] ->
// dst[NC][N^3]; TRANS uses M^T.  Cooperative over the workgroup; the caller syncs.
template <int N, typename Real, bool TRANS, int NC = 5>
__device__ __forceinline__ void sweep_nn(const Real (&M)[N][N], const Real* src, Real* dst, int ax) {
    constexpr int N2 = N * N, N3 = N2 * N;
    const int stride = ax == 0 ? 1 : (ax == 1 ? N : N2);
    for (int it = threadIdx.x; it < NC * N2; it += blockDim.x) {
        const int c = it / N2, rest = it % N2;
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

// Even-odd contraction: the split input v_e, v_o, v_mid of one line, and the pair of
// outputs (p, NO-1-p) of an EOMat (see dg_common.h).  eo_row returns e and o; the caller
// forms e + o and sg (e - o).
template <int NI, typename Real>
__device__ __forceinline__ void eo_split(const Real (&v)[NI], Real (&ve)[NI / 2 > 0 ? NI / 2 : 1],
                                         Real (&vo)[NI / 2 > 0 ? NI / 2 : 1]) {
#pragma unroll
    for (int i = 0; i < NI / 2; ++i) {
        ve[i] = v[i] + v[NI - 1 - i];
        vo[i] = v[i] - v[NI - 1 - i];
    }
}

template <int NO, int NI, typename Real>
__device__ __forceinline__ void eo_row(const EOMat<NO, NI, Real>& M, const Real (&ve)[NI / 2 > 0 ? NI / 2 : 1],
                                       const Real (&vo)[NI / 2 > 0 ? NI / 2 : 1], Real vmid, int p, Real& e, Real& o) {
    e = (NI % 2) ? M.C[p] * vmid : Real(0);
    o = Real(0);
#pragma unroll
    for (int i = 0; i < NI / 2; ++i) {
        e += M.E[p][i] * ve[i];
        o += M.O[p][i] * vo[i];
    }
}

// Fills the even-odd tables from the 1D tables (host).
template <int NO, int NI, typename Real, typename Get>
inline void fill_eo(EOMat<NO, NI, Real>& M, Get m) {
    for (int p = 0; p < (NO + 1) / 2; ++p) {
        for (int i = 0; i < NI / 2; ++i) {
            M.E[p][i] = (Real)(0.5 * (m(p, i) + m(p, NI - 1 - i)));
            M.O[p][i] = (Real)(0.5 * (m(p, i) - m(p, NI - 1 - i)));
        }
        M.C[p] = (NI % 2) ? (Real)m(p, NI / 2) : Real(0);
    }
}

// In-LDS inverse mass: sR <- (Smi)^{x3} diag(1/(|J| w)) (Smi^T)^{x3} sR, work >= 5 N^3.
template <int N, typename Real, bool GEN>
__device__ __forceinline__ void inverse_mass_lds(const MTab<N, Real>& mt, const Real* wm, Real* sR, Real* work,
                                                 Real detJ, const double* jxw_m) {
    // In place on sR, one line of one component per thread and phase; a thread writes back
    // exactly the line it read, and the lines of one axis are disjoint, so one barrier per
    // change of axis suffices: x, y, then z with the scaling and the backward z sweep
    // fused, then y and x.  (work is not needed.)
    (void)work;
    constexpr int N2 = N * N, N3 = N2 * N;
    const int tid = threadIdx.x, nth = blockDim.x;
    const auto line = [&](int ax, int it) {
        const int c = it / N2, rest = it % N2;
        const int base = ax == 0 ? rest * N : (ax == 1 ? (rest % N) + (rest / N) * N2 : rest);
        return c * N3 + base;
    };
    const auto apply = [&](bool trans, Real (&v)[N]) {
        Real t[N];
#pragma unroll
        for (int o = 0; o < N; ++o) {
            Real acc = 0;
#pragma unroll
            for (int i = 0; i < N; ++i) acc += (trans ? mt.Smi[i][o] : mt.Smi[o][i]) * v[i];
            t[o] = acc;
        }
#pragma unroll
        for (int o = 0; o < N; ++o) v[o] = t[o];
    };
    for (int ax = 0; ax < 2; ++ax) {
        const int stride = ax == 0 ? 1 : N;
        for (int it = tid; it < 5 * N2; it += nth) {
            Real* r = sR + line(ax, it);
            Real v[N];
#pragma unroll
            for (int i = 0; i < N; ++i) v[i] = r[i * stride];
            apply(true, v);
#pragma unroll
            for (int i = 0; i < N; ++i) r[i * stride] = v[i];
        }
        __syncthreads();
    }
    for (int it = tid; it < 5 * N2; it += nth) {
        const int rest = it % N2, a0 = rest % N, a1 = rest / N;
        Real* r = sR + line(2, it);
        Real v[N];
#pragma unroll
        for (int i = 0; i < N; ++i) v[i] = r[i * N2];
        apply(true, v);
#pragma unroll
        for (int i = 0; i < N; ++i) {
            Real jxw;
            if constexpr (GEN) jxw = (Real)jxw_m[a0 + N * a1 + N2 * i];
            else jxw = detJ * wm[a0] * wm[a1] * wm[i];
            v[i] = v[i] / jxw;
        }
        apply(false, v);
#pragma unroll
        for (int i = 0; i < N; ++i) r[i * N2] = v[i];
    }
    __syncthreads();
    for (int ax = 1; ax >= 0; --ax) {
        const int stride = ax == 0 ? 1 : N;
        for (int it = tid; it < 5 * N2; it += nth) {
            Real* r = sR + line(ax, it);
            Real v[N];
#pragma unroll
            for (int i = 0; i < N; ++i) v[i] = r[i * stride];
            apply(false, v);
#pragma unroll
            for (int i = 0; i < N; ++i) r[i * stride] = v[i];
        }
        __syncthreads();
    }
}

__device__ __forceinline__ int axis_stride(int ax, int N) { return ax == 0 ? 1 : (ax == 1 ? N : N * N); }

// Workgroup copy of a table struct of Real values (kernel argument -> LDS).
template <typename T, typename Real>
__device__ __forceinline__ void copy_table(const T& src, T& dst) {
    constexpr int n = (int)(sizeof(T) / sizeof(Real));
    const Real* s = reinterpret_cast<const Real*>(&src);
    Real* d = reinterpret_cast<Real*>(&dst);
    for (int i = threadIdx.x; i < n; i += blockDim.x) d[i] = s[i];
}

// Neighbour, face id and penalty of the six faces, computed once per workgroup.
struct FaceInfo {
    int64_t enb[6];   // neighbour cell (own cell for walls), index d + 3 s
    int64_t fid[6];
    int wall[6];
};

// Fills fi, the penalties sTau and, on affine meshes, the per-direction unit normals
// and permuted metric rows (sFn, sJr) of cell e's six faces (threads 0..5; the caller syncs).
template <typename Real, bool GEN>
__device__ __forceinline__ void face_info_setup(const OpArgs& a, int64_t e, FaceInfo& fi, Real* sTau, Real* sFn,
                                                Real* sJr) {
    for (int f = threadIdx.x; f < 6; f += blockDim.x) {
        const int i0 = (int)(e % a.n[0]), i1 = (int)((e / a.n[0]) % a.n[1]), i2 = (int)(e / ((int64_t)a.n[0] * a.n[1]));
        const int d = f % 3, s = f / 3;
        const int nd = d == 0 ? a.n[0] : (d == 1 ? a.n[1] : a.n[2]);
        const int per = d == 0 ? a.periodic[0] : (d == 1 ? a.periodic[1] : a.periodic[2]);
        const int id = d == 0 ? i0 : (d == 1 ? i1 : i2);
        // tangential indices (t0 < t1) and the extent of t0
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
        sTau[f] = (Real)tf[fi.fid[f]];
        if (!GEN && s == 0) {
            const double* row = a.cell_metric + e * 10 + 3 * d;
            const double l = sqrt(row[0] * row[0] + row[1] * row[1] + row[2] * row[2]);
            sFn[4 * d + 0] = (Real)(row[0] / l);
            sFn[4 * d + 1] = (Real)(row[1] / l);
            sFn[4 * d + 2] = (Real)(row[2] / l);
            sFn[4 * d + 3] = (Real)l;
            const int rows[3] = {d == 0 ? 1 : 0, d == 2 ? 1 : 2, d};
            for (int r = 0; r < 3; ++r)
                for (int j = 0; j < 3; ++j) sJr[9 * d + 3 * r + j] = (Real)a.cell_metric[e * 10 + 3 * rows[r] + j];
        }
    }
}

// Value and physical gradient of one side at face point (q0, q1): the sweep along
// t1 of the t0-swept traces A[3][c][N][Q] (value, t0-derivative, normal derivative).
template <int N, int Q, typename Real>
__device__ __forceinline__ void load_face_point(const KTab<N, Q, Real>& tb, const Real* A, int d, int q0, int q1,
                                                const Real (&J)[9], Real U[5], Real G[5][3]) {
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        Real v = 0, g0 = 0, g1 = 0, gn = 0;
#pragma unroll
        for (int ib = 0; ib < N; ++ib) {
            const Real a0 = A[(0 * 5 + c) * N * Q + ib * Q + q0];
            const Real a1 = A[(1 * 5 + c) * N * Q + ib * Q + q0];
            const Real an = A[(2 * 5 + c) * N * Q + ib * Q + q0];
            v += tb.S[q1][ib] * a0;
            g0 += tb.S[q1][ib] * a1;
            g1 += tb.D[q1][ib] * a0;
            gn += tb.S[q1][ib] * an;
        }
        // reference gradient in the cell's axes: (t0, t1, d) -> (0, 1, 2)
        const Real gr0 = d == 0 ? gn : g0;
        const Real gr1 = d == 1 ? gn : (d == 0 ? g0 : g1);
        const Real gr2 = d == 2 ? gn : g1;
#pragma unroll
        for (int j = 0; j < 3; ++j) G[c][j] = J[j] * gr0 + J[3 + j] * gr1 + J[6 + j] * gr2;
        U[c] = v;
    }
}

// As load_face_point, with the metric rows already permuted to the face's axes:
// Jr = rows (t0, t1, d) of J^{-1}, so the physical gradient needs no per-lane
// selection of reference components.
// (The line loop is unrolled by four only where UnrollLimit says so: fully unrolled, the
// compiler loads all 15 N operands ahead and spills.)
template <int N, int Q, typename Real>
__device__ __forceinline__ void load_face_point_rows(const KTab<N, Q, Real>& tb, const Real* A, int q0, int q1,
                                                     const Real (&Jr)[9], Real U[5], Real G[5][3]) {
    constexpr int UF = UnrollLimit<N, Q, Real>::face ? 4 : N;
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        Real v = 0, g0 = 0, g1 = 0, gn = 0;
#pragma unroll UF
        for (int ib = 0; ib < N; ++ib) {
            const Real a0 = A[(0 * 5 + c) * N * Q + ib * Q + q0];
            const Real a1 = A[(1 * 5 + c) * N * Q + ib * Q + q0];
            const Real an = A[(2 * 5 + c) * N * Q + ib * Q + q0];
            v += tb.S[q1][ib] * a0;
            g0 += tb.S[q1][ib] * a1;
            g1 += tb.D[q1][ib] * a0;
            gn += tb.S[q1][ib] * an;
        }
#pragma unroll
        for (int j = 0; j < 3; ++j) G[c][j] = Jr[j] * g0 + Jr[3 + j] * g1 + Jr[6 + j] * gn;
        U[c] = v;
    }
}

// Test integration of the face-point coefficients out [f][val, g_t0, g_t1, g_n][c][q1][q0]
// of NF faces against the face-local tensor basis (a along t0, b along t1): the value
// part and the tangential gradient parts through phi_a(t0) phi_b(t1), the normal part
// separately, giving per face W0 (to be multiplied by l_m(s) of the normal direction)
// and W1 (by l_m'(s)), [2][c][b][a] at wb(f) (wb(f) == nullptr: face skipped).  Two
// cooperative phases through t1 [f][3][c][N][Q]; the caller syncs after the second.
template <int N, int Q, typename Real, int NF, typename WB>
__device__ __forceinline__ void face_lift(const KTab<N, Q, Real>& tb, const Real* out, Real* t1, WB wb) {
    constexpr int N2 = N * N, Q2 = Q * Q;
    const int tid = threadIdx.x, nth = blockDim.x;
    // transposed along t1: P0 = S^T val + D^T g_t1, P1 = S^T g_t0, Pn = S^T g_n    t1 [f][3][c][b][q0]
    for (int it = tid; it < NF * 5 * N * Q; it += nth) {
        const int q0 = it % Q, ib = (it / Q) % N, c = (it / (Q * N)) % 5, d = it / (5 * Q * N);
        const Real* o = out + d * 4 * 5 * Q2 + c * Q2 + q0;
        Real p0 = 0, p1 = 0, pn = 0;
#pragma unroll
        for (int q1 = 0; q1 < Q; ++q1) {
            p0 += tb.S[q1][ib] * o[q1 * Q] + tb.D[q1][ib] * o[2 * 5 * Q2 + q1 * Q];
            p1 += tb.S[q1][ib] * o[1 * 5 * Q2 + q1 * Q];
            pn += tb.S[q1][ib] * o[3 * 5 * Q2 + q1 * Q];
        }
        Real* t = t1 + d * 3 * 5 * N * Q + c * N * Q + ib * Q + q0;
        t[0] = p0;
        t[5 * N * Q] = p1;
        t[2 * 5 * N * Q] = pn;
    }
    __syncthreads();

    // transposed along t0: W0 = S^T P0 + D^T P1, W1 = S^T Pn    [2][c][b][a]
    for (int it = tid; it < NF * 5 * N2; it += nth) {
        const int ia = it % N, ib = (it / N) % N, c = (it / N2) % 5, d = it / (5 * N2);
        Real* w = wb(d);
        if (!w) continue;
        const Real* t = t1 + d * 3 * 5 * N * Q + c * N * Q + ib * Q;
        Real w0 = 0, w1 = 0;
#pragma unroll
        for (int q0 = 0; q0 < Q; ++q0) {
            w0 += tb.S[q0][ia] * t[q0] + tb.D[q0][ia] * t[5 * N * Q + q0];
            w1 += tb.S[q0][ia] * t[2 * 5 * N * Q + q0];
        }
        w[c * N2 + ib * N + ia] = w0;
        w[5 * N2 + c * N2 + ib * N + ia] = w1;
    }
}

// R[c](a, b, m) += sum_f W0_f(a, b) l_m(s) + W1_f(a, b) l'_m(s) over the NF faces xi_d = s,
// d = d0 .. d0 + NF - 1, whose lifted blocks W_f [2][c][b][a] follow each other at w.
template <int N, typename Real, int NF, typename Tab>
__device__ __forceinline__ void face_accumulate(const Tab& tb, int s, int d0, const Real* w, Real* sR) {
    constexpr int N2 = N * N, N3 = N2 * N;
    for (int it = threadIdx.x; it < 5 * N3; it += blockDim.x) {
        const int c = it / N3, r = it % N3;
        const int x0 = r % N, x1 = (r / N) % N, x2 = r / N2;
        const Real* wc = w + c * N2;
        Real acc;
        if constexpr (NF == 3) {
            // face d = 0: (a, b, m) = (x1, x2, x0); d = 1: (x0, x2, x1); d = 2: (x0, x1, x2)
            acc = wc[0 * 2 * 5 * N2 + x2 * N + x1] * tb.fv[s][x0] + wc[(0 * 2 + 1) * 5 * N2 + x2 * N + x1] * tb.fd[s][x0];
            acc += wc[1 * 2 * 5 * N2 + x2 * N + x0] * tb.fv[s][x1] + wc[(1 * 2 + 1) * 5 * N2 + x2 * N + x0] * tb.fd[s][x1];
            acc += wc[2 * 2 * 5 * N2 + x1 * N + x0] * tb.fv[s][x2] + wc[(2 * 2 + 1) * 5 * N2 + x1 * N + x0] * tb.fd[s][x2];
        } else {
            // the single face d0 (uniform over the workgroup)
            const int ab = d0 == 0 ? x2 * N + x1 : (d0 == 1 ? x2 * N + x0 : x1 * N + x0);
            const int m = d0 == 0 ? x0 : (d0 == 1 ? x1 : x2);
            acc = wc[ab] * tb.fv[s][m] + wc[5 * N2 + ab] * tb.fd[s][m];
        }
        sR[it] += acc;
    }
}

// Test integration of one face group into sR: face_lift into the W area (r2), then
// face_accumulate.
template <int N, int Q, typename Real, int NF = 3>
__device__ __forceinline__ void face_test_accumulate(const KTab<N, Q, Real>& tb, int s, int d0, Real* r1, Real* r2,
                                                     Real* sR) {
    constexpr int N2 = N * N;
    face_lift<N, Q, Real, NF>(tb, r2, r1, [r2](int f) { return r2 + f * 2 * 5 * N2; });
    __syncthreads();
    face_accumulate<N, Real, NF>(tb, s, d0, r2, sR);
    __syncthreads();
}

// One face point it = f * n_q^2 + q0 + n_q q1 of the group of faces xi_d = s,
// d = d0 + f: the t1 contraction of both sides' t0-swept traces A (layout
// [f][side][3][c][N][Q]), the numerical fluxes, and the reference-space test
// coefficients res[kind * 5 + c], kind = value, g_t0, g_t1, g_n, of the own side.
// TWO: also those of the other side (not at walls), whose value part is the negative
// of the own side's (the numerical flux is single-valued and the normals opposite):
// res1[(kind - 1) * 5 + c] for the three gradient kinds, with the other side's state
// in the symmetry term and its own metric rows.
template <int N, int Q, typename Real, bool GEN, bool TWO = false>
__device__ __forceinline__ void face_point(const OpArgs& a, const KTab<N, Q, Real>& lt, const Phys<Real>& ph, bool conv,
                                           bool visc, int s, int d0, const FaceInfo& fi, const Real* sTau,
                                           const Real* sFn, const Real* sJr, Real detJ, const Real* r1, int it,
                                           Real (&res)[20], Real (&res1)[15]) {
    constexpr int Q2 = Q * Q;
    const int f = it / Q2, d = d0 + f, pt = it % Q2, q0 = pt % Q, q1 = pt / Q;
    const int fslot = d + 3 * s;
    const bool wall = fi.wall[fslot] != 0;
    // reference axes of the face: tangential t0 < t1, normal d; rows[r] is the
    // row of J^{-1} that multiplies the derivative along the face's axis r
    const int rows[3] = {d == 0 ? 1 : 0, d == 2 ? 1 : 2, d};
    Real Jm[9], Jp[9], nrm[3], dAw;
    const double* fdp = nullptr;
    if constexpr (GEN) {
        fdp = a.face_data[d] + fi.fid[fslot] * 22 * Q2 + pt;
        const Real sgn = s ? Real(1) : Real(-1);
#pragma unroll
        for (int j = 0; j < 3; ++j) nrm[j] = sgn * (Real)fdp[j * Q2];
        dAw = (Real)fdp[3 * Q2];
        const int own = s ? 4 : 13;
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int j = 0; j < 3; ++j) Jm[3 * r + j] = (Real)fdp[(own + 3 * rows[r] + j) * Q2];
    } else {
#pragma unroll
        for (int m = 0; m < 9; ++m) Jm[m] = sJr[9 * d + m];
        const Real sgn = s ? Real(1) : Real(-1);
        const Real* fn = sFn + 4 * d;     // unit normal of face xi_d = 1 and |row d of J^{-1}|
        nrm[0] = sgn * fn[0];
        nrm[1] = sgn * fn[1];
        nrm[2] = sgn * fn[2];
        dAw = detJ * fn[3] * lt.w[q0] * lt.w[q1];
    }
    // one side at a time, to keep a single gradient live: the side's value,
    // physical gradient, F_c.n and F_v.n go straight into the point's coefficient
    //   val = -1/2 (F_c^- + F_c^+).n + 1/2 (F_v^- + F_v^+).n - (Lambda/2 + tau)(U^- - U^+)
    Real Um[5], Up[5], val[5], lam_m = 0, lam_p = 0;
    Prim<Real> sm, sp;
    {
        Real G[5][3], Fn[5];
        load_face_point_rows<N, Q, Real>(lt, r1 + (f * 2 + 0) * 3 * 5 * N * Q, q0, q1, Jm, Um, G);
        sm = primitives(Um, ph);
#pragma unroll
        for (int c = 0; c < 5; ++c) val[c] = 0;
        if (conv) {
            lam_m = convective_normal(Um, sm, nrm, ph, Fn);
#pragma unroll
            for (int c = 0; c < 5; ++c) val[c] -= Real(0.5) * Fn[c];
        }
        if (visc) {
            viscous_flux_normal(sm, G, nrm, ph, Fn);
#pragma unroll
            for (int c = 0; c < 5; ++c) val[c] += Real(0.5) * Fn[c];
        }
        if (wall) {
            wall_mirror(Um, sm, ph, Up);   // the exterior gradient is the interior one: G is kept
        } else {
            if constexpr (GEN) {
                const int oth = s ? 13 : 4;
#pragma unroll
                for (int r = 0; r < 3; ++r)
#pragma unroll
                    for (int j = 0; j < 3; ++j) Jp[3 * r + j] = (Real)fdp[(oth + 3 * rows[r] + j) * Q2];
            } else {
                const double* cm = a.cell_metric + fi.enb[fslot] * 10;
#pragma unroll
                for (int r = 0; r < 3; ++r)
#pragma unroll
                    for (int j = 0; j < 3; ++j) Jp[3 * r + j] = (Real)cm[3 * rows[r] + j];
            }
            load_face_point_rows<N, Q, Real>(lt, r1 + (f * 2 + 1) * 3 * 5 * N * Q, q0, q1, Jp, Up, G);
        }
        sp = primitives(Up, ph);
        if (conv) {
            lam_p = convective_normal(Up, sp, nrm, ph, Fn);
#pragma unroll
            for (int c = 0; c < 5; ++c) val[c] -= Real(0.5) * Fn[c];
        }
        if (visc) {
            viscous_flux_normal(sp, G, nrm, ph, Fn);
#pragma unroll
            for (int c = 0; c < 5; ++c) val[c] += Real(0.5) * Fn[c];
        }
    }
    Real jump[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) jump[c] = Um[c] - Up[c];
    {
        const Real lam = lam_m > lam_p ? lam_m : lam_p;
        const Real pen = (conv ? Real(0.5) * lam : Real(0)) + (visc ? sTau[fslot] : Real(0));
#pragma unroll
        for (int c = 0; c < 5; ++c) val[c] -= pen * jump[c];
    }
    Real gphys[5][3];
    if (visc) {
        viscous_flux_rank1(sm, jump, nrm, ph, gphys);
    } else {
#pragma unroll
        for (int c = 0; c < 5; ++c)
#pragma unroll
            for (int j = 0; j < 3; ++j) gphys[c][j] = 0;
    }
    const Real half_dAw = Real(0.5) * dAw;
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        // reference-space coefficients along the face axes (t0, t1, n): the rows of Jm
        res[c] = val[c] * dAw;
#pragma unroll
        for (int r = 0; r < 3; ++r)
            res[(1 + r) * 5 + c] =
                (Jm[r * 3] * gphys[c][0] + Jm[r * 3 + 1] * gphys[c][1] + Jm[r * 3 + 2] * gphys[c][2]) * half_dAw;
    }
    if constexpr (TWO) {
        // the other side: F_v(U^+, [[U]]) with the same jump tensor (U^- - U^+) (x) n^-,
        // projected on the other cell's metric rows
        if (visc && !wall) {
            viscous_flux_rank1(sp, jump, nrm, ph, gphys);
#pragma unroll
            for (int c = 0; c < 5; ++c)
#pragma unroll
                for (int r = 0; r < 3; ++r)
                    res1[r * 5 + c] =
                        (Jp[r * 3] * gphys[c][0] + Jp[r * 3 + 1] * gphys[c][1] + Jp[r * 3 + 2] * gphys[c][2]) * half_dAw;
        } else {
#pragma unroll
            for (int m = 0; m < 15; ++m) res1[m] = 0;
        }
    }
}

// Traces of U and of its normal derivative on both sides of the NF faces xi_d = s,
// d = d0 .. d0 + NF - 1 (own side from sU, or with OWNG from the cell's coefficients in
// global memory; the neighbour's from global memory; nothing for the exterior side of a
// wall), swept along t0: SW = sW [f][side][3][c][N][Q] (value, t0-derivative, normal
// derivative), using the TR area of the layout FS for unfused traces.  Ends with a barrier.
// The own coefficients in LDS are laid out [c][a2][a1][a0] with component stride CS and
// a2-plane stride PS (N^3 and N^2 unless padded against bank conflicts, see FaceSU).
template <int N, int Q, typename Real, int NF, typename FS, bool OWNG = false, int CS = N * N * N, int PS = N * N>
__device__ __forceinline__ void face_traces_sweep(const OpArgs& a, const KTab<N, Q, Real>& lt, int s, int d0,
                                                  const FaceInfo& fi, const Real* sU, Real* sW) {
    constexpr int N2 = N * N, N3 = N2 * N;
    static_assert(!(OWNG && FS::FUSED_TRACE), "own coefficients from global memory: unfused traces only");
    const auto lstr = [](int ax) { return ax == 0 ? 1 : (ax == 1 ? N : PS); };
    Real* r1 = sW;                 // SW
    const int tid = threadIdx.x, nth = blockDim.x;
    const int64_t cstride = a.ncell * N3;

    if constexpr (FS::FUSED_TRACE) {
        // traces and the sweep along t0 in one phase: item (side, f, c, ib) computes the N
        // traces (value and normal derivative) on its line a0 = 0..N-1 -- from sU on the own
        // side, from the neighbour's coefficients in global memory on the other -- and sweeps
        // them: A0 = S tv, A1 = D tv, An = S tn  ->  r1 [f][side][3][c][b][q0].  The items of
        // one side fill whole waves, so the own / neighbour branch is uniform in each wave.
        constexpr int PER_SIDE = NF * 5 * N, SIDE_SPAN = (PER_SIDE + 63) / 64 * 64;
        for (int it = tid; it < 2 * SIDE_SPAN; it += nth) {
            const int side = it / SIDE_SPAN, k = it % SIDE_SPAN;
            if (k >= PER_SIDE) continue;
            const int ib = k % N, c = (k / N) % 5, f = k / (5 * N), d = d0 + f;
            if (side == 1 && fi.wall[d + 3 * s]) continue;
            const int t0 = d == 0 ? 1 : 0, t1 = d == 2 ? 1 : 2;
            const int sd = axis_stride(d, N), st0 = axis_stride(t0, N), bb = ib * axis_stride(t1, N);
            Real tv[N], tn[N];
            if (side == 0) {
                const Real* own = sU + c * CS + ib * lstr(t1);
                const int lst0 = lstr(t0), lsd = lstr(d);
    #pragma unroll
                for (int ia = 0; ia < N; ++ia) {
                    Real v = 0, n = 0;
    #pragma unroll
                    for (int m = 0; m < N; ++m) {
                        const Real x = own[ia * lst0 + m * lsd];
                        v += lt.fv[s][m] * x;
                        n += lt.fd[s][m] * x;
                    }
                    tv[ia] = v;
                    tn[ia] = n;
                }
            } else {
                const double* un_line = a.U + c * cstride + fi.enb[d + 3 * s] * N3 + bb;
    #pragma unroll
                for (int ia = 0; ia < N; ++ia) {
                    Real v = 0, n = 0;
    #pragma unroll
                    for (int m = 0; m < N; ++m) {
                        const Real x = (Real)un_line[ia * st0 + m * sd];
                        v += lt.fv[1 - s][m] * x;
                        n += lt.fd[1 - s][m] * x;
                    }
                    tv[ia] = v;
                    tn[ia] = n;
                }
            }
            Real* o = r1 + ((f * 2 + side) * 3 * 5 + c) * N * Q + ib * Q;
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
    } else {
        // larger N: the traces as a phase of their own (N^2 lines per face), then the sweep
        // traces: value and normal derivative of both sides at the face nodes
        Real* rtr = sW + FS::TR_OFF;   // TR
        for (int it = tid; it < NF * 5 * N2; it += nth) {
            const int f = it / (5 * N2), d = d0 + f, c = (it / N2) % 5, ab = it % N2, ia = ab % N, ib = ab / N;
            const int t0 = d == 0 ? 1 : 0, t1 = d == 2 ? 1 : 2;
            const int base = ia * axis_stride(t0, N) + ib * axis_stride(t1, N), sd = axis_stride(d, N);
            Real tv = 0, tn = 0, uv = 0, un = 0;
    #pragma unroll
            for (int m = 0; m < N; ++m) {
                const Real x = OWNG ? (Real)a.U[c * cstride + (int64_t)blockIdx.x * N3 + base + m * sd]
                                    : sU[c * CS + ia * lstr(t0) + ib * lstr(t1) + m * lstr(d)];
                tv += lt.fv[s][m] * x;
                tn += lt.fd[s][m] * x;
            }
            if (!fi.wall[d + 3 * s]) {
                const double* un_line = a.U + c * cstride + fi.enb[d + 3 * s] * N3 + base;
    #pragma unroll
                for (int m = 0; m < N; ++m) {
                    const Real x = (Real)un_line[m * sd];
                    uv += lt.fv[1 - s][m] * x;
                    un += lt.fd[1 - s][m] * x;
                }
            }
            Real* tr = rtr + f * (2 * 2 * 5 * N2) + c * N2 + ab;
            tr[(0 * 2 + 0) * 5 * N2] = tv;
            tr[(0 * 2 + 1) * 5 * N2] = tn;
            tr[(1 * 2 + 0) * 5 * N2] = uv;
            tr[(1 * 2 + 1) * 5 * N2] = un;
        }
        __syncthreads();

        // sweep along t0: A0 = S tv, A1 = D tv, An = S tn     r1 [f][side][3][c][b][q0]
        if constexpr (FS::TR_IN_SW) {
            // one item per thread: its two trace lines into registers, a barrier that
            // separates every read of TR from the writes of SW over it, then the sweep
            const int it = tid;
            const int ib = it % N, c = (it / N) % 5, side = (it / (5 * N)) % 2, f = it / (10 * N), d = d0 + f;
            const bool on = it < NF * 2 * 5 * N && !(side == 1 && fi.wall[d + 3 * s]);
            Real tv[N], tn[N];
            if (on) {
                const Real* tr = rtr + f * (2 * 2 * 5 * N2) + side * (2 * 5 * N2) + c * N2 + ib * N;
    #pragma unroll
                for (int ia = 0; ia < N; ++ia) {
                    tv[ia] = tr[ia];
                    tn[ia] = tr[5 * N2 + ia];
                }
            }
            __syncthreads();
            if (on) {
                Real* o = r1 + ((f * 2 + side) * 3 * 5 + c) * N * Q + ib * Q;
                constexpr int UQ = UnrollLimit<N, Q, Real>::face ? 1 : Q;
    #pragma unroll UQ
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
        } else {
        for (int it = tid; it < NF * 2 * 5 * N; it += nth) {
            const int ib = it % N, c = (it / N) % 5, side = (it / (5 * N)) % 2, f = it / (10 * N), d = d0 + f;
            if (side == 1 && fi.wall[d + 3 * s]) continue;
            const Real* tr = rtr + f * (2 * 2 * 5 * N2) + side * (2 * 5 * N2) + c * N2 + ib * N;
            Real tv[N], tn[N];
    #pragma unroll
            for (int ia = 0; ia < N; ++ia) {
                tv[ia] = tr[ia];
                tn[ia] = tr[5 * N2 + ia];
            }
            Real* o = r1 + ((f * 2 + side) * 3 * 5 + c) * N * Q + ib * Q;
            // (UnrollLimit: the output loop is not unrolled, else the compiler loads the
            // whole 2 n_q N table ahead and spills)
            constexpr int UQ = UnrollLimit<N, Q, Real>::face ? 1 : Q;
    #pragma unroll UQ
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
        }
        __syncthreads();
    }

}

// The three faces xi_d = s (d = 0, 1, 2) of the cell: traces, fluxes, test
// integration, accumulated into sR.  NF = 3 processes the faces of all three
// directions together (d0 = 0); NF = 1 the single face xi_{d0} = s.
template <int N, int Q, typename Real, bool GEN, int NF>
__device__ __forceinline__ void face_group(const OpArgs& a, const KTab<N, Q, Real>& lt, const Phys<Real>& ph, bool conv,
                                           bool visc, int s, int d0, const FaceInfo& fi, const Real* sTau,
                                           const Real* sFn, const Real* sJr, Real detJ, const Real* sU, Real* sR,
                                           Real* sW) {
    using FS = FaceSizes<N, Q, OpBlock<N, Q, Real>::threads, NF, OpBlock<N, Q, Real>::fused>;
    constexpr int Q2 = Q * Q;
    // work regions: SW (swept traces, read by the point phase), TR (traces), OUT
    // (point results), T1 (t1-transposed), W (lifted): see FaceSizes
    Real* r1 = sW;                 // SW
    Real* r2 = sW + FS::OUT_OFF;   // OUT, later W
    Real* rt1 = sW + FS::T1_OFF;   // T1
    const int tid = threadIdx.x, nth = blockDim.x;

    face_traces_sweep<N, Q, Real, NF, FS>(a, lt, s, d0, fi, sU, sW);

    // pointwise: numerical fluxes and reference-space test coefficients at every
    // face point, stored as OUT [f][kind: val, g_t0, g_t1, g_n][c][q1][q0].  When one
    // pass of the workgroup covers all face points, the results wait in registers
    // across a barrier and overwrite the swept traces (smaller LDS footprint).
    if constexpr (FS::ALIAS) {
        Real res[20], res1[15];
        const bool act = tid < NF * Q2;
        if (act) face_point<N, Q, Real, GEN>(a, lt, ph, conv, visc, s, d0, fi, sTau, sFn, sJr, detJ, r1, tid, res, res1);
        __syncthreads();
        if (act) {
            Real* o = r2 + (tid / Q2) * 4 * 5 * Q2 + tid % Q2;
#pragma unroll
            for (int m = 0; m < 20; ++m) o[m * Q2] = res[m];
        }
    } else {
        for (int it = tid; it < NF * Q2; it += nth) {
            Real res[20], res1[15];
            face_point<N, Q, Real, GEN>(a, lt, ph, conv, visc, s, d0, fi, sTau, sFn, sJr, detJ, r1, it, res, res1);
            Real* o = r2 + (it / Q2) * 4 * 5 * Q2 + it % Q2;
#pragma unroll
            for (int m = 0; m < 20; ++m) o[m * Q2] = res[m];
        }
    }
    __syncthreads();

    face_test_accumulate<N, Q, Real, NF>(lt, s, d0, rt1, r2, sR);
}

// Registers: at most 256 VGPRs (two waves per SIMD), except for k = 1, whose float64
// kernels fit in 168 without spilling, so that three waves share a SIMD.
template <int N, int Q, typename Real, bool GEN>
__global__ void __launch_bounds__((OpBlock<N, Q, Real>::threads)) __attribute__((amdgpu_waves_per_eu(N <= 2 ? 3 : 2)))
dg_operator_kernel(OpArgs a, KTab<N, Q, Real> tb, MTab<N, Real> mt, EOTab<N, Q, Real> eot) {
    constexpr bool SPLIT = OpBlock<N, Q, Real>::split;
    constexpr bool EO = OpBlock<N, Q, Real>::even_odd;
    constexpr int HN = N / 2 > 0 ? N / 2 : 1, HQ = Q / 2 > 0 ? Q / 2 : 1;
    using Sz = OpSizes<N, Q, OpBlock<N, Q, Real>::threads, (int)sizeof(Real), OpBlock<N, Q, Real>::fused, SPLIT>;
    constexpr int P = Sz::P;
    constexpr int N2 = N * N, N3 = N2 * N, Q2 = Q * Q, Q3 = Q2 * Q;
    constexpr int ZS = CellSizes<N, Q, P>::Z, YS = CellSizes<N, Q, P>::Y;
    __shared__ Real sU[5 * N3];
    __shared__ Real sR[5 * N3];
    __shared__ Real sW[Sz::WORK];
    __shared__ FaceInfo fi;
    __shared__ Real sTau[6];
    __shared__ Real sFn[12];   // affine: per direction the unit normal and |row of J^{-1}|
    __shared__ Real sJr[GEN ? 1 : 27];   // affine: per direction d the rows (t0, t1, d) of J^{-1}
    __shared__ Real lwm[N];

    const int64_t e = blockIdx.x;
    const int tid = threadIdx.x, nth = blockDim.x;
    const Phys<Real> ph = make_phys<Real>(a);
    const bool conv = (a.terms & 1u) != 0;
    const bool visc = (a.terms & 2u) != 0;
    const int64_t cstride = a.ncell * N3;

    for (int i = tid; i < 5 * N3; i += nth) {
        const int c = i / N3, j = i % N3;
        sU[i] = (Real)a.U[c * cstride + e * N3 + j];
        sR[i] = Real(0);
    }
    // face terms lifted by the face kernel: the cell's six blocks [slot][2][5][N^2], loaded
    // into registers now so that their latency overlaps the cell term, and added to the
    // residual after it
    constexpr int FWB = 2 * 5 * N2;
    constexpr int FWV = SPLIT ? (6 * FWB + OpBlock<N, Q, Real>::threads - 1) / OpBlock<N, Q, Real>::threads : 1;
    const bool gather = SPLIT && (conv || visc);
    Real fwr[FWV];
    if (gather) {
        const Real* fw = static_cast<const Real*>(a.fw) + e * 6 * FWB;
#pragma unroll
        for (int v = 0; v < FWV; ++v) {
            const int i = tid + v * OpBlock<N, Q, Real>::threads;
            fwr[v] = i < 6 * FWB ? fw[i] : Real(0);
        }
    }
    // Fused Runge-Kutta stage: in the 128-thread float64 kernels (k <= 3), whose register
    // budget has the room for a thread's share of the cell's dU (at most three values),
    // load it now, so that its latency overlaps the whole evaluation instead of the
    // epilogue's.
    constexpr int B = OpBlock<N, Q, Real>::threads;
    constexpr int RKV = (5 * N3 + B - 1) / B;
    constexpr bool RK_PREFETCH = RKV <= 3 && B == 128 && sizeof(Real) == sizeof(double);
    double dU_old[RK_PREFETCH ? RKV : 1];
    if constexpr (RK_PREFETCH) {
        if (a.rk.dU && a.rk.A != 0.0) {
#pragma unroll
            for (int v = 0; v < RKV; ++v) {
                const int i = tid + v * B;
                dU_old[v] = i < 5 * N3 ? a.rk.dU[(i / N3) * cstride + e * N3 + i % N3] : 0.0;
            }
        }
    }
    // LDS copy of the 1D tables when it fits beside the work arrays (otherwise the
    // kernel argument is read directly).  Reading every table entry from LDS keeps
    // the tables out of the scalar registers: held there for the whole kernel they
    // exceed the scalar register file and spill through vector lanes.
    const KTab<N, Q, Real>* ltp;
    const MTab<N, Real>* lmp;
    if constexpr (Sz::LDS_TAB) {
        __shared__ KTab<N, Q, Real> lt_lds;
        copy_table<KTab<N, Q, Real>, Real>(tb, lt_lds);
        ltp = &lt_lds;
        __shared__ MTab<N, Real> lm_lds;
        copy_table<MTab<N, Real>, Real>(mt, lm_lds);
        lmp = &lm_lds;
    } else {
        ltp = &tb;
        lmp = &mt;
    }
    const MTab<N, Real>& lm = *lmp;
    const KTab<N, Q, Real>& lt = *ltp;
    // even-odd tables of the cell sweeps, in LDS
    __shared__ EOTab<N, Q, Real> leo;
    if constexpr (EO) copy_table<EOTab<N, Q, Real>, Real>(eot, leo);
    for (int i = tid; i < N; i += nth) lwm[i] = mt.wm[i];
    if constexpr (!SPLIT) face_info_setup<Real, GEN>(a, e, fi, sTau, sFn, sJr);

    // cell-constant metric (affine)
    Real Ji[9], detJ = Real(1);
    if constexpr (!GEN) {
#pragma unroll
        for (int m = 0; m < 9; ++m) Ji[m] = (Real)a.cell_metric[e * 10 + m];
        detJ = (Real)a.cell_metric[e * 10 + 9];
    }
    __syncthreads();


    if (conv || visc) {
        // ------------------------------------------------------------ cell term
        Real* sZ = sW;
        Real* sY = sW + ZS;       // later sB
        Real* sF = sY + YS;       // later sE
        // z-sweep: Z0 = S_z U, Z1 = D_z U     layout [kind][c][pz][a1][a0]
        for (int it = tid; it < 5 * N2; it += nth) {
            const int c = it / N2, r = it % N2;
            Real v[N];
#pragma unroll
            for (int i = 0; i < N; ++i) v[i] = sU[c * N3 + i * N2 + r];
            Real* z0p = sZ + (0 * 5 + c) * Q * N2 + r;
            Real* z1p = sZ + (1 * 5 + c) * Q * N2 + r;
            if constexpr (EO) {
                Real ve[HN], vo[HN];
                eo_split<N>(v, ve, vo);
#pragma unroll
                for (int ph = 0; ph < (Q + 1) / 2; ++ph) {
                    Real e, o;
                    eo_row<Q, N>(leo.S, ve, vo, v[N / 2], ph, e, o);
                    z0p[ph * N2] = e + o;
                    if (ph != Q - 1 - ph) z0p[(Q - 1 - ph) * N2] = e - o;
                    eo_row<Q, N>(leo.D, ve, vo, v[N / 2], ph, e, o);
                    z1p[ph * N2] = e + o;
                    if (ph != Q - 1 - ph) z1p[(Q - 1 - ph) * N2] = o - e;
                }
            } else {
#pragma unroll
                for (int pz = 0; pz < Q; ++pz) {
                    Real z0 = 0, z1 = 0;
#pragma unroll
                    for (int i = 0; i < N; ++i) {
                        z0 += lt.S[pz][i] * v[i];
                        z1 += lt.D[pz][i] * v[i];
                    }
                    z0p[pz * N2] = z0;
                    z1p[pz * N2] = z1;
                }
            }
        }
        __syncthreads();

        for (int pz0 = 0; pz0 < Q; pz0 += P) {
            // y-sweep for planes pz0..pz0+P-1: Y00 = S_y Z0, Y10 = D_y Z0, Y01 = S_y Z1
            for (int it = tid; it < 5 * P * N; it += nth) {
                const int a0 = it % N, pl = (it / N) % P, c = it / (N * P);
                const int pz = pz0 + pl;
                if (pz >= Q) continue;
                Real z0[N], z1[N];
#pragma unroll
                for (int i = 0; i < N; ++i) {
                    z0[i] = sZ[(0 * 5 + c) * Q * N2 + pz * N2 + i * N + a0];
                    z1[i] = sZ[(1 * 5 + c) * Q * N2 + pz * N2 + i * N + a0];
                }
                Real* y00p = sY + ((0 * 5 + c) * P + pl) * Q * N + a0;
                Real* y10p = sY + ((1 * 5 + c) * P + pl) * Q * N + a0;
                Real* y01p = sY + ((2 * 5 + c) * P + pl) * Q * N + a0;
                if constexpr (EO) {
                    Real e0[HN], o0[HN], e1v[HN], o1v[HN];
                    eo_split<N>(z0, e0, o0);
                    eo_split<N>(z1, e1v, o1v);
#pragma unroll
                    for (int ph = 0; ph < (Q + 1) / 2; ++ph) {
                        const int pm = Q - 1 - ph;
                        Real e, o;
                        eo_row<Q, N>(leo.S, e0, o0, z0[N / 2], ph, e, o);
                        y00p[ph * N] = e + o;
                        if (ph != pm) y00p[pm * N] = e - o;
                        eo_row<Q, N>(leo.D, e0, o0, z0[N / 2], ph, e, o);
                        y10p[ph * N] = e + o;
                        if (ph != pm) y10p[pm * N] = o - e;
                        eo_row<Q, N>(leo.S, e1v, o1v, z1[N / 2], ph, e, o);
                        y01p[ph * N] = e + o;
                        if (ph != pm) y01p[pm * N] = e - o;
                    }
                } else {
#pragma unroll
                    for (int py = 0; py < Q; ++py) {
                        Real y00 = 0, y10 = 0, y01 = 0;
#pragma unroll
                        for (int i = 0; i < N; ++i) {
                            y00 += lt.S[py][i] * z0[i];
                            y10 += lt.D[py][i] * z0[i];
                            y01 += lt.S[py][i] * z1[i];
                        }
                        y00p[py * N] = y00;
                        y10p[py * N] = y10;
                        y01p[py * N] = y01;
                    }
                }
            }
            __syncthreads();

            // x-sweep + pointwise physics, one thread per quadrature point
            for (int it = tid; it < P * Q2; it += nth) {
                const int px = it % Q, py = (it / Q) % Q, pl = it / Q2;
                const int pz = pz0 + pl;
                if (pz >= Q) continue;
                Real Uq[5], Gr[5][3];
#pragma unroll
                for (int c = 0; c < 5; ++c) {
                    Real v = 0, dx = 0, dy = 0, dz = 0;
#pragma unroll (UnrollLimit<N, Q, Real>::cell ? 3 : N)
                    for (int i = 0; i < N; ++i) {
                        const Real y00 = sY[((0 * 5 + c) * P + pl) * Q * N + py * N + i];
                        const Real y10 = sY[((1 * 5 + c) * P + pl) * Q * N + py * N + i];
                        const Real y01 = sY[((2 * 5 + c) * P + pl) * Q * N + py * N + i];
                        v += lt.S[px][i] * y00;
                        dx += lt.D[px][i] * y00;
                        dy += lt.S[px][i] * y10;
                        dz += lt.S[px][i] * y01;
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
                    // physical gradient in place: Gr <- J^{-T} Gr
#pragma unroll
                    for (int c = 0; c < 5; ++c) {
                        const Real g0 = Gr[c][0], g1 = Gr[c][1], g2 = Gr[c][2];
#pragma unroll
                        for (int j = 0; j < 3; ++j) Gr[c][j] = J[0 * 3 + j] * g0 + J[1 * 3 + j] * g1 + J[2 * 3 + j] * g2;
                    }
                    subtract_viscous_flux(sq, Gr, ph, F);
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
            if constexpr (EO) {
                // one item per output pair (a0, N-1-a0)
                constexpr int HO = (N + 1) / 2;
                for (int it = tid; it < 5 * P * Q * HO; it += nth) {
                    const int ah = it % HO, py = (it / HO) % Q, pl = (it / (HO * Q)) % P, c = it / (HO * Q * P);
                    if (pz0 + pl >= Q) continue;
                    Real f[3][Q];
#pragma unroll
                    for (int m = 0; m < 3; ++m)
#pragma unroll
                        for (int px = 0; px < Q; ++px) f[m][px] = sF[((c * 3 + m) * P + pl) * Q2 + py * Q + px];
                    const int am = N - 1 - ah;
                    Real* bp = sB + (c * P + pl) * Q * N + py * N;
#pragma unroll
                    for (int m = 0; m < 3; ++m) {
                        Real ve[HQ], vo[HQ], e, o;
                        eo_split<Q>(f[m], ve, vo);
                        Real* b = bp + m * 5 * P * Q * N;
                        if (m == 0) {
                            eo_row<N, Q>(leo.Dt, ve, vo, f[m][Q / 2], ah, e, o);
                            b[ah] = e + o;
                            if (ah != am) b[am] = o - e;
                        } else {
                            eo_row<N, Q>(leo.St, ve, vo, f[m][Q / 2], ah, e, o);
                            b[ah] = e + o;
                            if (ah != am) b[am] = e - o;
                        }
                    }
                }
            } else {
                for (int it = tid; it < 5 * P * Q * N; it += nth) {
                    const int a0 = it % N, py = (it / N) % Q, pl = (it / (N * Q)) % P, c = it / (N * Q * P);
                    if (pz0 + pl >= Q) continue;
                    Real b1 = 0, b2 = 0, b3 = 0;
#pragma unroll
                    for (int px = 0; px < Q; ++px) {
                        b1 += lt.D[px][a0] * sF[((c * 3 + 0) * P + pl) * Q2 + py * Q + px];
                        b2 += lt.S[px][a0] * sF[((c * 3 + 1) * P + pl) * Q2 + py * Q + px];
                        b3 += lt.S[px][a0] * sF[((c * 3 + 2) * P + pl) * Q2 + py * Q + px];
                    }
                    sB[((0 * 5 + c) * P + pl) * Q * N + py * N + a0] = b1;
                    sB[((1 * 5 + c) * P + pl) * Q * N + py * N + a0] = b2;
                    sB[((2 * 5 + c) * P + pl) * Q * N + py * N + a0] = b3;
                }
            }
            __syncthreads();

            // y-transposed: E1 = S_y^T B1 + D_y^T B2, E2 = S_y^T B3   layout [kind][c][pl][a1][a0]
            Real* sE = sF;
            if constexpr (EO) {
                // one item per output pair (a1, N-1-a1)
                constexpr int HO = (N + 1) / 2;
                for (int it = tid; it < 5 * P * N * HO; it += nth) {
                    const int a0 = it % N, ah = (it / N) % HO, pl = (it / (N * HO)) % P, c = it / (N * HO * P);
                    if (pz0 + pl >= Q) continue;
                    Real bv[3][Q];
#pragma unroll
                    for (int m = 0; m < 3; ++m)
#pragma unroll
                        for (int py = 0; py < Q; ++py) bv[m][py] = sB[((m * 5 + c) * P + pl) * Q * N + py * N + a0];
                    const int am = N - 1 - ah;
                    Real ve[HQ], vo[HQ], es, os, ed, od;
                    eo_split<Q>(bv[0], ve, vo);
                    eo_row<N, Q>(leo.St, ve, vo, bv[0][Q / 2], ah, es, os);
                    eo_split<Q>(bv[1], ve, vo);
                    eo_row<N, Q>(leo.Dt, ve, vo, bv[1][Q / 2], ah, ed, od);
                    Real* e1p = sE + ((0 * 5 + c) * P + pl) * N2 + a0;
                    Real* e2p = sE + ((1 * 5 + c) * P + pl) * N2 + a0;
                    e1p[ah * N] = (es + os) + (ed + od);
                    if (ah != am) e1p[am * N] = (es - os) + (od - ed);
                    eo_split<Q>(bv[2], ve, vo);
                    eo_row<N, Q>(leo.St, ve, vo, bv[2][Q / 2], ah, es, os);
                    e2p[ah * N] = es + os;
                    if (ah != am) e2p[am * N] = es - os;
                }
            } else {
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
            }
            __syncthreads();

            // z-transposed, accumulated over the chunk's planes: R += S_z^T E1 + D_z^T E2
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
                sR[it] += acc;
            }
            // The next chunk's y sweep writes only sY, which this phase does not read, and
            // each thread updates the same sR entries in every chunk, so the barrier after
            // its y sweep suffices; after the last chunk the face phase reuses sF's space.
            if (pz0 + P >= Q) __syncthreads();
        }

        // ------------------------------------------------------------ face terms
        if constexpr (SPLIT) {
            // the face kernel's lifted blocks, held in registers since the start: staged in
            // the work area, then R += the six faces: slots 0..2 (xi_d = 0), 3..5 (xi_d = 1)
#pragma unroll
            for (int v = 0; v < FWV; ++v) {
                const int i = tid + v * B;
                if (i < 6 * FWB) sW[i] = fwr[v];
            }
            __syncthreads();
            face_accumulate<N, Real, 3>(lt, 0, 0, sW, sR);
            face_accumulate<N, Real, 3>(lt, 1, 0, sW + 3 * FWB, sR);
            __syncthreads();
        } else if constexpr (Sz::NF == 3) {
            face_group<N, Q, Real, GEN, 3>(a, lt, ph, conv, visc, 0, 0, fi, sTau, sFn, sJr, detJ, sU, sR, sW);
            face_group<N, Q, Real, GEN, 3>(a, lt, ph, conv, visc, 1, 0, fi, sTau, sFn, sJr, detJ, sU, sR, sW);
        } else {
            for (int s = 0; s < 2; ++s)
                for (int d0 = 0; d0 < 3; ++d0)
                    face_group<N, Q, Real, GEN, 1>(a, lt, ph, conv, visc, s, d0, fi, sTau, sFn, sJr, detJ, sU, sR, sW);
        }
    }

    // ------------------------------------------------------------ body force (k+1 rule)
    const bool force = (a.terms & 4u) != 0 && (a.force[0] != 0.0 || a.force[1] != 0.0 || a.force[2] != 0.0);
    const double* jxw_m = GEN ? a.mass_jxw + e * N3 : nullptr;
    if (force) {
        Real* t0b = sW;
        Real* t1b = sW + 5 * N3;
        // values at the mass points: (Sm)^{x3} U
        sweep_nn<N, Real, false>(lm.Sm, sU, t0b, 0);
        __syncthreads();
        sweep_nn<N, Real, false>(lm.Sm, t0b, t1b, 1);
        __syncthreads();
        sweep_nn<N, Real, false>(lm.Sm, t1b, t0b, 2);
        __syncthreads();
        for (int p = tid; p < N3; p += nth) {
            Real jxw;
            if constexpr (GEN) jxw = (Real)jxw_m[p];
            else jxw = detJ * lwm[p % N] * lwm[(p / N) % N] * lwm[p / N2];
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
        sweep_nn<N, Real, true>(lm.Sm, t0b, t1b, 0);
        __syncthreads();
        sweep_nn<N, Real, true>(lm.Sm, t1b, t0b, 1);
        __syncthreads();
        sweep_nn<N, Real, true>(lm.Sm, t0b, t1b, 2);
        __syncthreads();
        for (int i = tid; i < 5 * N3; i += nth) sR[i] += t1b[i];
        __syncthreads();
    }

    if (a.fuse_minv) inverse_mass_lds<N, Real, GEN>(lm, lwm, sR, sW, detJ, jxw_m);

    if (a.rk.dU) {
        // fused Runge-Kutta stage on the cell's own DoFs; the old state comes from sU when
        // that holds it exactly (float64), else it is re-read
        const bool first = a.rk.A == 0.0;
        if constexpr (RK_PREFETCH) {
#pragma unroll
            for (int v = 0; v < RKV; ++v) {
                const int i = tid + v * B;
                if (i < 5 * N3) {
                    const int64_t g = (i / N3) * cstride + e * N3 + i % N3;
                    const double u = sizeof(Real) == sizeof(double) ? (double)sU[i] : a.U[g];
                    const double d = rk_increment(first, a.rk.A, first ? 0.0 : dU_old[v], a.rk.dt, (double)sR[i]);
                    a.rk.dU[g] = d;
                    a.rk.U_out[g] = rk_advance(u, a.rk.B, d);
                }
            }
        } else {
            for (int i = tid; i < 5 * N3; i += nth) {
                const int64_t g = (i / N3) * cstride + e * N3 + i % N3;
                const double u = sizeof(Real) == sizeof(double) ? (double)sU[i] : a.U[g];
                const double d = rk_increment(first, a.rk.A, first ? 0.0 : a.rk.dU[g], a.rk.dt, (double)sR[i]);
                a.rk.dU[g] = d;
                a.rk.U_out[g] = rk_advance(u, a.rk.B, d);
            }
        }
    } else {
        for (int i = tid; i < 5 * N3; i += nth) {
            const int c = i / N3, j = i % N3;
            a.out[c * cstride + e * N3 + j] = (double)sR[i];
        }
    }
}

// Face kernel: every face of the mesh once, both sides (face-centric), for the cells
// whose operator kernel gathers its face terms instead of computing them (SPLIT).  One
// workgroup per cell e takes its three faces xi_d = 1, shared with the upper neighbour
// across each (or with the exterior mirror state at a wall), and any wall face xi_d = 0.
// For each face it forms the traces of both sides, the numerical fluxes at the n_q^2
// points (one point per thread; the coefficients wait in registers across barriers),
// and lifts both sides' terms onto the face-local tensor basis; the lifted blocks
// [2][5][N^2] go to the face buffer slot of the cell that owns that side: e's slot
// d + 3 for its own side, the neighbour's slot d for the other.  Each slot is written by
// exactly one workgroup, so the buffer needs no clearing and no atomics.
template <int N, int Q, typename Real, bool GEN>
__global__ void __launch_bounds__((FaceBlock<N, Q, Real>::threads)) __attribute__((amdgpu_waves_per_eu(2)))
dg_face_kernel(OpArgs a, KTab<N, Q, Real> tb) {
    using FB = FaceBlock<N, Q, Real>;
    using FS = typename FB::FS;
    using FS1 = typename FB::FS1;
    constexpr int N2 = N * N, N3 = N2 * N, Q2 = Q * Q, FWB = 2 * 5 * N2;
    static_assert(FB::one_pass && FS::ALIAS && FS1::ALIAS, "one face point per thread");
    constexpr int CS = FaceSU<N>::CS, PS = FaceSU<N>::PS;
    __shared__ Real sU[5 * CS];
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
    const int64_t cstride = a.ncell * N3;
    Real* fw = static_cast<Real*>(a.fw);

    for (int i = tid; i < 5 * N3; i += blockDim.x) {
        const int c = i / N3, j = i % N3;
        sU[c * CS + (j / N2) * PS + j % N2] = (Real)a.U[c * cstride + e * N3 + j];
    }
    copy_table<KTab<N, Q, Real>, Real>(tb, lt);
    face_info_setup<Real, GEN>(a, e, fi, sTau, sFn, sJr);
    Real detJ = Real(1);
    if constexpr (!GEN) detJ = (Real)a.cell_metric[e * 10 + 9];
    __syncthreads();

    // the three faces xi_d = 1, both sides
    face_traces_sweep<N, Q, Real, 3, FS, false, CS, PS>(a, lt, 1, 0, fi, sU, sW);
    Real res[20], res1[15];
    const bool act = tid < 3 * Q2;
    if (act) face_point<N, Q, Real, GEN, true>(a, lt, ph, conv, visc, 1, 0, fi, sTau, sFn, sJr, detJ, sW, tid, res, res1);
    __syncthreads();
    Real* out = sW + FS::OUT_OFF;
    Real* t1 = sW + FS::T1_OFF;
    Real* o = out + (tid / Q2) * 4 * 5 * Q2 + tid % Q2;
    if (act) {
#pragma unroll
        for (int m = 0; m < 20; ++m) o[m * Q2] = res[m];
    }
    __syncthreads();
    face_lift<N, Q, Real, 3>(lt, out, t1, [&](int f) { return fw + (e * 6 + 3 + f) * FWB; });
    // the other side's coefficients replace the own side's (its lift above has read them):
    // value part negated, gradient parts from res1
    if (act) {
#pragma unroll
        for (int c = 0; c < 5; ++c) o[c * Q2] = -res[c];
#pragma unroll
        for (int m = 0; m < 15; ++m) o[(5 + m) * Q2] = res1[m];
    }
    __syncthreads();
    face_lift<N, Q, Real, 3>(lt, out, t1, [&](int f) { return fi.wall[3 + f] ? nullptr : fw + (fi.enb[3 + f] * 6 + f) * FWB; });
    __syncthreads();

    // wall faces xi_d = 0 (the lower end of a direction with walls): the own side only
    for (int d = 0; d < 3; ++d) {
        if (!fi.wall[d]) continue;   // uniform over the workgroup
        face_traces_sweep<N, Q, Real, 1, FS1, false, CS, PS>(a, lt, 0, d, fi, sU, sW);
        const bool act1 = tid < Q2;
        if (act1) face_point<N, Q, Real, GEN>(a, lt, ph, conv, visc, 0, d, fi, sTau, sFn, sJr, detJ, sW, tid, res, res1);
        __syncthreads();
        Real* out1 = sW + FS1::OUT_OFF;
        if (act1) {
#pragma unroll
            for (int m = 0; m < 20; ++m) out1[m * Q2 + tid] = res[m];
        }
        __syncthreads();
        face_lift<N, Q, Real, 1>(lt, out1, sW + FS1::T1_OFF, [&](int) { return fw + (e * 6 + d) * FWB; });
        __syncthreads();
    }
}

// ------------------------------------------------------------------ launchers
template <int N, int Q, typename Real>
inline void fill_tables(const Tables1D& t, KTab<N, Q, Real>& kt, MTab<N, Real>& mt) {
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
}

// One evaluation: with the face terms in their own kernel (SPLIT) the face kernel runs
// first and the operator kernel gathers its output from a.fw (both on stream st).
template <int N, int Q, typename Real, bool GEN>
inline int launch_op_t(const OpArgs& a, const Tables1D& t, hipStream_t st) {
    KTab<N, Q, Real> kt;
    MTab<N, Real> mt;
    fill_tables<N, Q, Real>(t, kt, mt);
    constexpr int B = OpBlock<N, Q, Real>::threads;
    constexpr bool SPLIT = OpBlock<N, Q, Real>::split;
    static_assert((OpSizes<N, Q, B, (int)sizeof(Real), OpBlock<N, Q, Real>::fused, SPLIT>::WORK + 10 * N * N * N) *
                          sizeof(Real) <= 160 * 1024, "LDS budget");
    if constexpr (SPLIT) {
        if ((a.terms & 3u) != 0) {
            if (!a.fw) return -1;
            hipLaunchKernelGGL((dg_face_kernel<N, Q, Real, GEN>), dim3((unsigned)a.ncell),
                               dim3(FaceBlock<N, Q, Real>::threads), 0, st, a, kt);
            if (hipGetLastError() != hipSuccess) return -1;
        }
    }
    EOTab<N, Q, Real> eo;
    fill_eo(eo.S, [&](int p, int i) { return t.S[p][i]; });
    fill_eo(eo.D, [&](int p, int i) { return t.D[p][i]; });
    fill_eo(eo.St, [&](int i, int p) { return t.S[p][i]; });
    fill_eo(eo.Dt, [&](int i, int p) { return t.D[p][i]; });
    hipLaunchKernelGGL((dg_operator_kernel<N, Q, Real, GEN>), dim3((unsigned)a.ncell), dim3(B), 0, st, a, kt, mt, eo);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Bytes of the face buffer a context needs for (N, n_q, precision): six lifted blocks
// [2][5][N^2] per cell when the face terms have a kernel of their own, else none.
template <int N, int Q, typename Real>
constexpr int64_t face_buffer_bytes_per_cell() {
    return OpBlock<N, Q, Real>::split ? (int64_t)6 * 2 * 5 * N * N * (int64_t)sizeof(Real) : 0;
}

}  // namespace dgns
