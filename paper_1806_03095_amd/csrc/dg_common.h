// Shared definitions of the DG operator kernels and the host library.
//
// Pointwise physics of the compressible Navier-Stokes equations (paper Sec. 2.1):
// conserved U = (rho, rho u, rho E); Newtonian stress with zero bulk viscosity,
// Fourier heat flux, ideal gas, E = c_v T + |u|^2/2; fluxes of eq.
// (CompressibleNavierStokesFluxes).  Numerical fluxes of Sec. 2.2.2: local
// Lax-Friedrichs and symmetric interior penalty.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dgns {

constexpr int kMaxN = 16;   // nodes per direction, k <= 15
constexpr int kMaxQ = 16;   // quadrature points per direction
constexpr int kBlock = 128; // threads per workgroup of the cell kernels

// A compute unit's 160 KB of LDS taken as 128 granules of 1280 bytes, a workgroup holding
// whole granules: measured, three workgroups of 54,272 bytes did not share a compute unit
// (waves per busy cycle 11.8) while three of 51,200 bytes did (20.5).
constexpr int kLdsGranule = 1280;
constexpr int kLdsGranules = 128;
__host__ __device__ constexpr int lds_wg_per_cu(int bytes) {
    return kLdsGranules / ((bytes + kLdsGranule - 1) / kLdsGranule);
}

// 1D tables of one (k, n_q, basis) combination, float64 master copy.
struct Tables1D {
    int n, q;
    double S[kMaxQ][kMaxN];   // l_i(x_p) at the n_q Gauss points of the flux rule
    double D[kMaxQ][kMaxN];   // l_i'(x_p)
    double w[kMaxQ];          // Gauss weights on [0,1]
    double fv[2][kMaxN];      // l_i(0), l_i(1)
    double fd[2][kMaxN];      // l_i'(0), l_i'(1)
    double Sm[kMaxN][kMaxN];  // l_i(x^m_p) at the k+1 Gauss points of the mass rule
    double Smi[kMaxN][kMaxN]; // inverse of Sm
    double wm[kMaxN];         // mass-rule weights
    double Sg[kMaxQ][kMaxN];  // geometry (LGL) basis l^g_i(x_p) at the flux points
};

// Exactly sized copy in the operator's working precision, passed by value as a
// kernel argument; the kernels copy it to LDS where it fits (held in scalar
// registers for a whole kernel, the larger tables spill).
template <int N, int Q, typename Real>
struct KTab {
    // rows of 16 values (k = 15) padded by one: a wave's points read the rows of up to 16
    // quadrature points at once, and rows 128 (64) bytes apart put 8 (4) of them on the
    // same banks (measured at k = 15 in float64: cell kernel 1452 -> 1019 us)
    static constexpr int NP = N % 16 == 0 ? N + 1 : N;
    Real S[Q][NP];
    Real D[Q][NP];
    Real w[Q];
    Real fv[2][N];
    Real fd[2][N];
};

// Even-odd form of an NO x NI matrix M on point sets symmetric about 1/2, for which
// M[NO-1-p][NI-1-i] = sg M[p][i] (sg = +1 for the values S, -1 for the derivatives D):
// E[p][i] = (M[p][i] + M[p][NI-1-i]) / 2, O[p][i] = (M[p][i] - M[p][NI-1-i]) / 2 for
// p < (NO+1)/2, i < NI/2, and C[p] = M[p][NI/2] (the middle column, odd NI).  Then with
// v_e = v_i + v_{NI-1-i}, v_o = v_i - v_{NI-1-i}:  e = E v_e + C v_mid, o = O v_o,
// (M v)[p] = e + o and (M v)[NO-1-p] = sg (e - o): half the multiply-adds (Sec. 2.3).
template <int NO, int NI, typename Real>
struct EOMat {
    static constexpr int HO = (NO + 1) / 2, HI = NI / 2 > 0 ? NI / 2 : 1;
    Real E[HO][HI];
    Real O[HO][HI];
    Real C[HO];
};

// The even-odd forms of S and D (NO = n_q rows, NI = k+1 columns) and of their transposes.
template <int N, int Q, typename Real>
struct EOTab {
    EOMat<Q, N, Real> S, D;
    EOMat<N, Q, Real> St, Dt;
};

template <int N, typename Real>
struct MTab {
    Real Sm[N][N];
    Real Smi[N][N];
    Real wm[N];
};

// Metric storage.
//  affine : cell_metric[e*10 + m], m = 0..8 J^{-1} row-major (row = reference
//           direction), m = 9 det J; face normal/area follow from J^{-1}.
//  general: cell_metric[(e*10 + m)*Q^3 + p], m = 0..8 J^{-1}, m = 9 |det J| w_p;
//           face_data[d][(f*22 + m)*Q^2 + r]: m = 0..2 unit normal pointing from
//           the lower cell (minus) to the upper cell (plus) in direction d, m = 3
//           dA * w_r, m = 4..12 J^{-1} of the minus cell, 13..21 of the plus cell;
//           mass_jxw[e*N^3 + p] = |det J| w at the mass-rule points.
// Face numbering in direction d: position pos = i_d (lower face of cell i_d, 0..n_d),
// f = pos + (n_d + 1) * (i_t0 + n_t0 * i_t1), t0 < t1 the two other directions.
// One stage of the 2N-storage Runge-Kutta scheme (Sec. 2.4) fused into the operator
// kernel: with dU set, the kernel writes dU <- A dU + dt L and U_out <- U + B dU in
// place of L.  U_out must not alias U, which the other workgroups read as neighbour
// data.  A == 0 marks the first stage, where the old dU is not read.
struct RkStage {
    double* dU;
    double* U_out;
    double A, B, dt;
};

// The stage arithmetic at one DoF, shared by the fused and the standalone update so
// that both round alike: dU <- A dU + dt L (dt L alone in the first stage), U <- U + B dU.
__host__ __device__ inline double rk_increment(bool first, double A, double dU_old, double dt, double L) {
    return first ? dt * L : fma(A, dU_old, dt * L);
}
__host__ __device__ inline double rk_advance(double U, double B, double dU) { return fma(B, dU, U); }

struct OpArgs {
    const double* U;
    double* out;
    int64_t ncell;
    int n[3];
    int periodic[3];
    const double* cell_metric;
    const double* face_data[3];
    const double* tau_face[3];
    const double* mass_jxw;
    double gamma, R, mu, lam, wall_T;
    double force[3];
    unsigned terms;
    int fuse_minv;
    RkStage rk;   // dU == nullptr: write L (or R) to out
    // face buffer of the kernels that evaluate each face once (a separate face kernel
    // lifts both sides' face terms; the cell kernel gathers its six): per cell and face
    // slot d + 3 s, [2][5][(k+1)^2] values in the operator's working precision
    void* fw;
    // device copy of the context's 1D tables (read by the kernels of degree >= 8, whose
    // tables would not fit in the kernel arguments)
    const Tables1D* tab_dev;
};

template <typename Real>
struct Phys {
    Real gamma, gm1, R, mu, lam, inv_cv, wall_T, cv;
};

template <typename Real>
__host__ __device__ inline Phys<Real> make_phys(const OpArgs& a) {
    Phys<Real> p;
    p.gamma = (Real)a.gamma;
    p.gm1 = (Real)(a.gamma - 1.0);
    p.R = (Real)a.R;
    p.mu = (Real)a.mu;
    p.lam = (Real)a.lam;
    p.cv = (Real)(a.R / (a.gamma - 1.0));
    p.inv_cv = (Real)((a.gamma - 1.0) / a.R);
    p.wall_T = (Real)a.wall_T;
    return p;
}

// Primitive quantities of a conserved state, computed once per point: 1/rho,
// velocity u = m/rho, |u|^2, pressure p = (gamma-1)(rho E - rho |u|^2/2), E = rho E/rho.
template <typename Real>
struct Prim {
    Real rinv, u[3], uu, p, E;
};

template <typename Real>
__device__ __forceinline__ Prim<Real> primitives(const Real U[5], const Phys<Real>& ph) {
    Prim<Real> s;
    s.rinv = Real(1) / U[0];
    s.u[0] = U[1] * s.rinv;
    s.u[1] = U[2] * s.rinv;
    s.u[2] = U[3] * s.rinv;
    s.uu = s.u[0] * s.u[0] + s.u[1] * s.u[1] + s.u[2] * s.u[2];
    s.p = ph.gm1 * (U[4] - Real(0.5) * U[0] * s.uu);
    s.E = U[4] * s.rinv;
    return s;
}

// Viscous flux F_v(U, G)[c][j] for a conserved state U (primitives s) and a
// conserved-variable gradient G[c][j] = dU_c/dx_j; linear in G.  Row 0 is zero.
template <typename Real>
__device__ __forceinline__ void viscous_flux(const Prim<Real>& s, const Real G[5][3], const Phys<Real>& ph,
                                             Real F[5][3]) {
    const Real rinv = s.rinv;
    const Real u0 = s.u[0], u1 = s.u[1], u2 = s.u[2];
    Real gu[3][3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        gu[0][j] = (G[1][j] - u0 * G[0][j]) * rinv;
        gu[1][j] = (G[2][j] - u1 * G[0][j]) * rinv;
        gu[2][j] = (G[3][j] - u2 * G[0][j]) * rinv;
    }
    const Real div = gu[0][0] + gu[1][1] + gu[2][2];
    const Real mu = ph.mu;
    const Real two_thirds_div = Real(2.0 / 3.0) * div;
    Real tau[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            tau[a][j] = mu * (gu[a][j] + gu[j][a] - (a == j ? two_thirds_div : Real(0)));
    const Real lam_cv = ph.lam * ph.inv_cv;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        // dT/dx_j = ((d(rho E)/dx_j - E drho/dx_j)/rho - u . du/dx_j) / c_v
        const Real gE = (G[4][j] - s.E * G[0][j]) * rinv;
        const Real gT = gE - (u0 * gu[0][j] + u1 * gu[1][j] + u2 * gu[2][j]);
        F[0][j] = Real(0);
        F[1][j] = tau[0][j];
        F[2][j] = tau[1][j];
        F[3][j] = tau[2][j];
        F[4][j] = tau[j][0] * u0 + tau[j][1] * u1 + tau[j][2] * u2 + lam_cv * gT;
    }
}

// F -= F_v(U, G): the viscous flux subtracted in place (rows 1..4).
template <typename Real>
__device__ __forceinline__ void subtract_viscous_flux(const Prim<Real>& s, const Real G[5][3], const Phys<Real>& ph,
                                                      Real F[5][3]) {
    const Real rinv = s.rinv;
    Real gu[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int j = 0; j < 3; ++j) gu[a][j] = (G[1 + a][j] - s.u[a] * G[0][j]) * rinv;
    const Real dd = Real(2.0 / 3.0) * (gu[0][0] + gu[1][1] + gu[2][2]);
    const Real lam_cv = ph.lam * ph.inv_cv;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const Real gT = (G[4][j] - s.E * G[0][j]) * rinv - (s.u[0] * gu[0][j] + s.u[1] * gu[1][j] + s.u[2] * gu[2][j]);
        Real tu = 0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const Real t = ph.mu * (gu[a][j] + gu[j][a] - (a == j ? dd : Real(0)));   // tau_aj = tau_ja
            F[1 + a][j] -= t;
            tu += t * s.u[a];
        }
        F[4][j] -= tu + lam_cv * gT;
    }
}

// F_v(U, G) . n, the viscous flux in direction n (five values, the first zero).
template <typename Real>
__device__ __forceinline__ void viscous_flux_normal(const Prim<Real>& s, const Real G[5][3], const Real n[3],
                                                    const Phys<Real>& ph, Real Fn[5]) {
    const Real rinv = s.rinv;
    Real gu[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int j = 0; j < 3; ++j) gu[a][j] = (G[1 + a][j] - s.u[a] * G[0][j]) * rinv;
    const Real div = gu[0][0] + gu[1][1] + gu[2][2];
    Real tn[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        // (grad u + grad u^T) n - 2/3 div n
        const Real gun = gu[a][0] * n[0] + gu[a][1] * n[1] + gu[a][2] * n[2];
        const Real gtn = gu[0][a] * n[0] + gu[1][a] * n[1] + gu[2][a] * n[2];
        tn[a] = ph.mu * (gun + gtn - Real(2.0 / 3.0) * div * n[a]);
    }
    Real gTn = 0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const Real gT = (G[4][j] - s.E * G[0][j]) * rinv - (s.u[0] * gu[0][j] + s.u[1] * gu[1][j] + s.u[2] * gu[2][j]);
        gTn += gT * n[j];
    }
    Fn[0] = Real(0);
    Fn[1] = tn[0];
    Fn[2] = tn[1];
    Fn[3] = tn[2];
    Fn[4] = s.u[0] * tn[0] + s.u[1] * tn[1] + s.u[2] * tn[2] + ph.lam * ph.inv_cv * gTn;
}

// F_v(U, j (x) n) for a rank-one gradient (the symmetry term of the interior
// penalty method, with j = U^- - U^+): du_a/dx_k = w_a n_k, w_a = (j_{1+a} - u_a j_0)/rho,
// dT/dx_k = t n_k with t = ((j_4 - E j_0)/rho - u . w)/c_v.
template <typename Real>
__device__ __forceinline__ void viscous_flux_rank1(const Prim<Real>& s, const Real jmp[5], const Real n[3],
                                                   const Phys<Real>& ph, Real F[5][3]) {
    Real w[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) w[a] = (jmp[1 + a] - s.u[a] * jmp[0]) * s.rinv;
    const Real div = w[0] * n[0] + w[1] * n[1] + w[2] * n[2];
    const Real t = ((jmp[4] - s.E * jmp[0]) * s.rinv - (s.u[0] * w[0] + s.u[1] * w[1] + s.u[2] * w[2])) * ph.inv_cv;
    const Real un = s.u[0] * n[0] + s.u[1] * n[1] + s.u[2] * n[2];
    const Real uw = s.u[0] * w[0] + s.u[1] * w[1] + s.u[2] * w[2];
    const Real mu = ph.mu, dd = Real(2.0 / 3.0) * div;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        F[0][j] = Real(0);
#pragma unroll
        for (int a = 0; a < 3; ++a) F[1 + a][j] = mu * (w[a] * n[j] + w[j] * n[a] - (a == j ? dd : Real(0)));
        // (tau u)_j = mu (w_j (u.n) + n_j (u.w) - 2/3 div u_j)
        F[4][j] = mu * (w[j] * un + n[j] * uw - dd * s.u[j]) + ph.lam * t * n[j];
    }
}

// Convective flux F_c(U)[c][j].
template <typename Real>
__device__ __forceinline__ void convective_flux(const Real U[5], const Prim<Real>& s, Real F[5][3]) {
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        F[0][j] = U[1 + j];
        F[1][j] = U[1] * s.u[j] + (j == 0 ? s.p : Real(0));
        F[2][j] = U[2] * s.u[j] + (j == 1 ? s.p : Real(0));
        F[3][j] = U[3] * s.u[j] + (j == 2 ? s.p : Real(0));
        F[4][j] = (U[4] + s.p) * s.u[j];
    }
}

// F_c(U) . n and the LLF wave speed |u| + c, c = sqrt(|gamma p / rho|).
template <typename Real>
__device__ __forceinline__ Real convective_normal(const Real U[5], const Prim<Real>& s, const Real n[3],
                                                  const Phys<Real>& ph, Real Fn[5]) {
    const Real un = s.u[0] * n[0] + s.u[1] * n[1] + s.u[2] * n[2];
    Fn[0] = U[0] * un;
    Fn[1] = U[1] * un + s.p * n[0];
    Fn[2] = U[2] * un + s.p * n[1];
    Fn[3] = U[3] * un + s.p * n[2];
    Fn[4] = (U[4] + s.p) * un;
    return sqrt(s.uu) + sqrt(fabs(ph.gamma * s.p * s.rinv));
}

// Exterior state at an isothermal no-slip wall: rho+ = rho-, u+ = -u-,
// T+ = 2 T_wall - T-, E+ = c_v T+ + |u|^2/2 (gradients are copied by the caller).
template <typename Real>
__device__ __forceinline__ void wall_mirror(const Real Um[5], const Prim<Real>& s, const Phys<Real>& ph, Real Up[5]) {
    const Real rho = Um[0];
    const Real ke = Real(0.5) * rho * s.uu;
    const Real T = s.p * s.rinv / ph.R;
    const Real Tp = Real(2) * ph.wall_T - T;
    Up[0] = rho;
    Up[1] = -Um[1];
    Up[2] = -Um[2];
    Up[3] = -Um[3];
    Up[4] = rho * ph.cv * Tp + ke;
}

}  // namespace dgns
