// Hand-written vector-Jacobian products (reverse mode) of the pointwise physics
// of dg_common.h.  Each *_vjp function takes the cotangent of the forward
// function's outputs and ADDS the cotangents of its inputs into the given
// accumulators (U-bar through the primitive quantities, G-bar, jump-bar).
//
// Forward functions (paper Sec. 2.1 and 2.2.2): primitives, convective_normal
// (F_c.n and the Lax-Friedrichs wave speed), convective_flux, viscous_flux_normal
// (F_v.n), subtract_viscous_flux (F -= F_v), viscous_flux_rank1 (F_v(U, j (x) n)),
// wall_mirror.
#pragma once

#include "dg_common.h"

namespace dgns {

// Cotangents of the primitive quantities of one state.
template <typename Real>
struct PrimBar {
    Real rinv, u[3], uu, p, E;
};

template <typename Real>
__device__ __forceinline__ void zero(PrimBar<Real>& b) {
    b.rinv = b.uu = b.p = b.E = 0;
    b.u[0] = b.u[1] = b.u[2] = 0;
}

// primitives(U) reversed: Ub += (d prim / d U)^T pb.
template <typename Real>
__device__ __forceinline__ void primitives_vjp(const Real U[5], const Prim<Real>& s, const Phys<Real>& ph,
                                               PrimBar<Real> pb, Real Ub[5]) {
    // p = gm1 (U4 - U0 uu / 2)
    Ub[4] += ph.gm1 * pb.p;
    Ub[0] -= Real(0.5) * ph.gm1 * s.uu * pb.p;
    pb.uu -= Real(0.5) * ph.gm1 * U[0] * pb.p;
    // uu = u.u
#pragma unroll
    for (int a = 0; a < 3; ++a) pb.u[a] += Real(2) * s.u[a] * pb.uu;
    // E = U4 rinv
    Ub[4] += s.rinv * pb.E;
    pb.rinv += U[4] * pb.E;
    // u_a = U_{1+a} rinv
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        Ub[1 + a] += s.rinv * pb.u[a];
        pb.rinv += U[1 + a] * pb.u[a];
    }
    // rinv = 1/U0
    Ub[0] -= s.rinv * s.rinv * pb.rinv;
}

// convective_normal reversed: Fnb = cotangent of F_c.n, lamb = cotangent of |u| + c.
template <typename Real>
__device__ __forceinline__ void convective_normal_vjp(const Real U[5], const Prim<Real>& s, const Real n[3],
                                                      const Phys<Real>& ph, const Real Fnb[5], Real lamb,
                                                      PrimBar<Real>& pb, Real Ub[5]) {
    const Real un = s.u[0] * n[0] + s.u[1] * n[1] + s.u[2] * n[2];
    Ub[0] += Fnb[0] * un;
    Real unb = Fnb[0] * U[0] + Fnb[4] * (U[4] + s.p);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        Ub[1 + a] += Fnb[1 + a] * un;
        unb += Fnb[1 + a] * U[1 + a];
        pb.p += Fnb[1 + a] * n[a];
    }
    pb.p += Fnb[4] * un;
    Ub[4] += Fnb[4] * un;
#pragma unroll
    for (int a = 0; a < 3; ++a) pb.u[a] += unb * n[a];
    // lambda = sqrt(uu) + sqrt(|x|), x = gamma p rinv
    if (lamb != Real(0)) {
        if (s.uu > Real(0)) pb.uu += lamb * Real(0.5) / sqrt(s.uu);
        const Real x = ph.gamma * s.p * s.rinv;
        const Real ax = fabs(x);
        if (ax > Real(0)) {
            const Real xb = lamb * Real(0.5) / sqrt(ax) * (x < Real(0) ? Real(-1) : Real(1));
            pb.p += ph.gamma * s.rinv * xb;
            pb.rinv += ph.gamma * s.p * xb;
        }
    }
}

// convective_flux reversed: Fb[c][j] cotangent of F_c(U)[c][j].
template <typename Real>
__device__ __forceinline__ void convective_flux_vjp(const Real U[5], const Prim<Real>& s, const Real Fb[5][3],
                                                    PrimBar<Real>& pb, Real Ub[5]) {
    Real Hb = 0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        Ub[1 + j] += Fb[0][j];
        // F[1+a][j] = m_a u_j + p delta_aj
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            Ub[1 + a] += Fb[1 + a][j] * s.u[j];
            pb.u[j] += Fb[1 + a][j] * U[1 + a];
        }
        pb.p += Fb[1 + j][j];
        // F[4][j] = (rho E + p) u_j
        Hb += Fb[4][j] * s.u[j];
        pb.u[j] += Fb[4][j] * (U[4] + s.p);
    }
    Ub[4] += Hb;
    pb.p += Hb;
}

// Reverse of the velocity and temperature gradients shared by the viscous fluxes:
//   gu[a][j] = (G[1+a][j] - u_a G[0][j]) rinv
//   gT_j     = (G[4][j] - E G[0][j]) rinv - sum_a u_a gu[a][j]      (times 1/c_v outside)
// given gub[a][j] and gTb[j]; adds into Gb and the primitive cotangents.
template <typename Real>
__device__ __forceinline__ void gradients_vjp(const Prim<Real>& s, const Real G[5][3], const Real (&gu)[3][3],
                                              Real (&gub)[3][3], const Real gTb[3], PrimBar<Real>& pb, Real Gb[5][3]) {
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        Gb[4][j] += gTb[j] * s.rinv;
        pb.E -= gTb[j] * G[0][j] * s.rinv;
        Gb[0][j] -= gTb[j] * s.E * s.rinv;
        pb.rinv += gTb[j] * (G[4][j] - s.E * G[0][j]);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            pb.u[a] -= gTb[j] * gu[a][j];
            gub[a][j] -= gTb[j] * s.u[a];
        }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            Gb[1 + a][j] += gub[a][j] * s.rinv;
            pb.u[a] -= gub[a][j] * G[0][j] * s.rinv;
            Gb[0][j] -= gub[a][j] * s.u[a] * s.rinv;
            pb.rinv += gub[a][j] * (G[1 + a][j] - s.u[a] * G[0][j]);
        }
}

template <typename Real>
__device__ __forceinline__ void velocity_gradient(const Prim<Real>& s, const Real G[5][3], Real (&gu)[3][3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int j = 0; j < 3; ++j) gu[a][j] = (G[1 + a][j] - s.u[a] * G[0][j]) * s.rinv;
}

// Full viscous flux F_v(U, G)[c][j] reversed, for a cotangent Fb of F_v.
template <typename Real>
__device__ __forceinline__ void viscous_flux_vjp(const Prim<Real>& s, const Real G[5][3], const Phys<Real>& ph,
                                                 const Real Fb[5][3], PrimBar<Real>& pb, Real Gb[5][3]) {
    Real gu[3][3];
    velocity_gradient(s, G, gu);
    const Real dd = Real(2.0 / 3.0) * (gu[0][0] + gu[1][1] + gu[2][2]);
    Real taub[3][3], gTb[3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int j = 0; j < 3; ++j) taub[a][j] = Fb[1 + a][j];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        // F[4][j] = sum_a tau[j][a] u_a + lam/c_v gT_j
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const Real tja = ph.mu * (gu[j][a] + gu[a][j] - (a == j ? dd : Real(0)));
            taub[j][a] += Fb[4][j] * s.u[a];
            pb.u[a] += Fb[4][j] * tja;
        }
        gTb[j] = ph.lam * ph.inv_cv * Fb[4][j];
    }
    // tau = mu (gu + gu^T - 2/3 tr(gu) I)
    Real gub[3][3];
    Real trb = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) trb += taub[a][a];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            gub[a][j] = ph.mu * (taub[a][j] + taub[j][a]) - (a == j ? Real(2.0 / 3.0) * ph.mu * trb : Real(0));
    gradients_vjp(s, G, gu, gub, gTb, pb, Gb);
}

// viscous_flux_normal reversed: Fnb cotangent of F_v(U, G).n.
template <typename Real>
__device__ __forceinline__ void viscous_flux_normal_vjp(const Prim<Real>& s, const Real G[5][3], const Real n[3],
                                                        const Phys<Real>& ph, const Real Fnb[5], PrimBar<Real>& pb,
                                                        Real Gb[5][3]) {
    Real gu[3][3];
    velocity_gradient(s, G, gu);
    const Real div = gu[0][0] + gu[1][1] + gu[2][2];
    Real tn[3], tnb[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const Real gun = gu[a][0] * n[0] + gu[a][1] * n[1] + gu[a][2] * n[2];
        const Real gtn = gu[0][a] * n[0] + gu[1][a] * n[1] + gu[2][a] * n[2];
        tn[a] = ph.mu * (gun + gtn - Real(2.0 / 3.0) * div * n[a]);
    }
    // Fn4 = u . tn + lam/c_v gT.n
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        tnb[a] = Fnb[1 + a] + Fnb[4] * s.u[a];
        pb.u[a] += Fnb[4] * tn[a];
    }
    Real gTb[3];
    const Real gTnb = ph.lam * ph.inv_cv * Fnb[4];
#pragma unroll
    for (int j = 0; j < 3; ++j) gTb[j] = gTnb * n[j];
    Real gub[3][3];
    Real divb = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) divb -= Real(2.0 / 3.0) * ph.mu * tnb[a] * n[a];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            gub[a][j] = ph.mu * (tnb[a] * n[j] + tnb[j] * n[a]) + (a == j ? divb : Real(0));
    gradients_vjp(s, G, gu, gub, gTb, pb, Gb);
}

// viscous_flux_rank1 reversed: Fb cotangent of F_v(U, j (x) n); adds into the
// primitive cotangents of U and into jb (cotangent of the jump j).
template <typename Real>
__device__ __forceinline__ void viscous_flux_rank1_vjp(const Prim<Real>& s, const Real jmp[5], const Real n[3],
                                                       const Phys<Real>& ph, const Real Fb[5][3], PrimBar<Real>& pb,
                                                       Real jb[5]) {
    const Real mu = ph.mu;
    Real w[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) w[a] = (jmp[1 + a] - s.u[a] * jmp[0]) * s.rinv;
    const Real div = w[0] * n[0] + w[1] * n[1] + w[2] * n[2];
    const Real dd = Real(2.0 / 3.0) * div;
    const Real un = s.u[0] * n[0] + s.u[1] * n[1] + s.u[2] * n[2];
    const Real uw = s.u[0] * w[0] + s.u[1] * w[1] + s.u[2] * w[2];
    Real wb[3] = {0, 0, 0};
    Real ddb = 0, unb = 0, uwb = 0, tb = 0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            // F[1+a][j] = mu (w_a n_j + w_j n_a - delta_aj dd)
            wb[a] += mu * Fb[1 + a][j] * n[j];
            wb[j] += mu * Fb[1 + a][j] * n[a];
        }
        ddb -= mu * Fb[1 + j][j];
        // F[4][j] = mu (w_j un + n_j uw - dd u_j) + lam t n_j
        wb[j] += mu * Fb[4][j] * un;
        unb += mu * Fb[4][j] * w[j];
        uwb += mu * Fb[4][j] * n[j];
        ddb -= mu * Fb[4][j] * s.u[j];
        pb.u[j] -= mu * dd * Fb[4][j];
        tb += ph.lam * Fb[4][j] * n[j];
    }
    const Real divb = Real(2.0 / 3.0) * ddb;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        wb[a] += divb * n[a];
        pb.u[a] += unb * n[a] + uwb * w[a];
        wb[a] += uwb * s.u[a];
    }
    // t = ((j4 - E j0) rinv - u.w) / c_v
    const Real t0 = tb * ph.inv_cv;
    jb[4] += t0 * s.rinv;
    pb.E -= t0 * jmp[0] * s.rinv;
    jb[0] -= t0 * s.E * s.rinv;
    pb.rinv += t0 * (jmp[4] - s.E * jmp[0]);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        pb.u[a] -= t0 * w[a];
        wb[a] -= t0 * s.u[a];
    }
    // w_a = (j_{1+a} - u_a j0) rinv
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        jb[1 + a] += wb[a] * s.rinv;
        pb.u[a] -= wb[a] * jmp[0] * s.rinv;
        jb[0] -= wb[a] * s.u[a] * s.rinv;
        pb.rinv += wb[a] * (jmp[1 + a] - s.u[a] * jmp[0]);
    }
}

// wall_mirror reversed: Upb cotangent of the exterior state; adds into the
// interior state's primitive cotangents and Ub.
//   Up0 = U0, Up_{1+a} = -U_{1+a}, Up4 = 2 c_v T_w U0 - (c_v/R) p + U0 uu / 2
template <typename Real>
__device__ __forceinline__ void wall_mirror_vjp(const Real U[5], const Prim<Real>& s, const Phys<Real>& ph,
                                                const Real Upb[5], PrimBar<Real>& pb, Real Ub[5]) {
    Ub[0] += Upb[0] + Upb[4] * (Real(2) * ph.cv * ph.wall_T + Real(0.5) * s.uu);
#pragma unroll
    for (int a = 0; a < 3; ++a) Ub[1 + a] -= Upb[1 + a];
    pb.p -= ph.cv / ph.R * Upb[4];
    pb.uu += Real(0.5) * U[0] * Upb[4];
}

}  // namespace dgns
