// Diagnostics of the Taylor-Green and channel runs (Sec. 5.2.3) and the gradient of
// the kinetic energy, evaluated per cell with sum factorisation (Sec. 2.3), float64.
//
// diag_kernel, one workgroup per cell, writes the cell's nine partial sums
//   [0] int |u|^2/2            [1] int grad u : grad u      [2] -int u.(L_m - u L_rho)/rho
//   [3..7] int U_c (k+1 rule)  [8] cell volume (n_q rule)
// with u = m/rho and the broken (cell-wise) gradient at the n_q^3 Gauss points.  The
// values and reference gradients of rho and m (and the values of L_rho, L_m) come from
// the same z / y / x sweeps as the operator's cell term, processed in chunks of P
// planes; the totals use the mass-point interpolation of the inverse mass matrix.
//
// ke_vjp_kernel writes Ubar = dK/dU for K = int |u|^2/2: the point values
// g = (-|u|^2/rho, u/rho) w|J| are tested against the basis functions by the
// transposed sweeps.
#pragma once

#include "op_impl.h"

namespace dgns {

constexpr int kDiagSums = 9;

template <int N, int Q>
struct DiagSizes {
    static constexpr int N2 = N * N, N3 = N2 * N, Q2 = Q * Q;
    static constexpr int P = Q2 >= 128 ? 1 : (128 / Q2 < Q ? 128 / Q2 : Q);   // planes per chunk
    static constexpr int Z = 12 * Q * N2;     // Z0 [8][Q][N^2] (rho, m, L_rho, L_m), Z1 [4][Q][N^2]
    static constexpr int Y = 16 * P * Q * N;  // Y00 [8][P][Q][N], Y10 [4][P][Q][N], Y01 [4][P][Q][N]
    static constexpr int WORK = CMax<Z + Y, 10 * N3>::v;
};

// Deterministic sum of M per-thread values over the workgroup (fixed tree order).
template <int M>
__device__ __forceinline__ void block_sums(double (&v)[M], double* red) {
    const int tid = threadIdx.x, nth = blockDim.x;
#pragma unroll
    for (int m = 0; m < M; ++m) red[m * nth + tid] = v[m];
    __syncthreads();
    for (int s = nth / 2; s > 0; s >>= 1) {
        if (tid < s)
#pragma unroll
            for (int m = 0; m < M; ++m) red[m * nth + tid] += red[m * nth + tid + s];
        __syncthreads();
    }
#pragma unroll
    for (int m = 0; m < M; ++m) v[m] = red[m * nth];
    __syncthreads();
}

constexpr int kDiagBlock = 128;

template <int N, int Q, bool GEN>
__global__ void __launch_bounds__(kDiagBlock)
diag_kernel(OpArgs a, const double* L, double* partial, KTab<N, Q, double> tb, MTab<N, double> mt) {
    using DS = DiagSizes<N, Q>;
    constexpr int N2 = N * N, N3 = N2 * N, Q2 = Q * Q, Q3 = Q2 * Q, P = DS::P;
    __shared__ double sX[9 * N3];    // U (5 components), then L_rho, L_m (4)
    __shared__ double sW[DS::WORK];
    __shared__ double red[kDiagSums * kDiagBlock];
    __shared__ KTab<N, Q, double> lt;
    __shared__ MTab<N, double> lm;
    const int64_t e = blockIdx.x;
    const int tid = threadIdx.x, nth = blockDim.x;
    const int64_t cs = a.ncell * N3;
    for (int i = tid; i < 9 * N3; i += nth) {
        const int c = i / N3, j = i % N3;
        double v = 0;
        if (c < 5) v = a.U[c * cs + e * N3 + j];
        else if (L) v = L[(c - 5) * cs + e * N3 + j];
        sX[i] = v;
    }
    copy_table<KTab<N, Q, double>, double>(tb, lt);
    copy_table<MTab<N, double>, double>(mt, lm);
    double Jc[9], detJ = 1;
    if constexpr (!GEN) {
#pragma unroll
        for (int m = 0; m < 9; ++m) Jc[m] = a.cell_metric[e * 10 + m];
        detJ = a.cell_metric[e * 10 + 9];
    }
    double acc[kDiagSums];
#pragma unroll
    for (int m = 0; m < kDiagSums; ++m) acc[m] = 0;
    __syncthreads();

    // the 8 interpolated components: rho, m (sX 0..3) and L_rho, L_m (sX 5..8)
    double* Z = sW;
    double* Yb = sW + DS::Z;
    // z-sweep: Z0[c] = S_z X_c (c < 8), Z1[c] = D_z X_c (c < 4)      layout [c][pz][a1 a0]
    for (int it = tid; it < 8 * N2; it += nth) {
        const int c = it / N2, r = it % N2, src = c < 4 ? c : c + 1;
        double v[N];
#pragma unroll
        for (int i = 0; i < N; ++i) v[i] = sX[src * N3 + i * N2 + r];
#pragma unroll
        for (int pz = 0; pz < Q; ++pz) {
            double z0 = 0, z1 = 0;
#pragma unroll
            for (int i = 0; i < N; ++i) {
                z0 += lt.S[pz][i] * v[i];
                z1 += lt.D[pz][i] * v[i];
            }
            Z[(c * Q + pz) * N2 + r] = z0;
            if (c < 4) Z[((8 + c) * Q + pz) * N2 + r] = z1;
        }
    }
    __syncthreads();

    for (int pz0 = 0; pz0 < Q; pz0 += P) {
        // y-sweep of P planes: Y00 = S_y Z0 (8), Y10 = D_y Z0 (4), Y01 = S_y Z1 (4)   layout [kind c][pl][py][a0]
        for (int it = tid; it < 8 * P * N; it += nth) {
            const int a0 = it % N, pl = (it / N) % P, c = it / (N * P), pz = pz0 + pl;
            if (pz >= Q) continue;
            double z0[N], z1[N];
#pragma unroll
            for (int i = 0; i < N; ++i) {
                z0[i] = Z[(c * Q + pz) * N2 + i * N + a0];
                z1[i] = c < 4 ? Z[((8 + c) * Q + pz) * N2 + i * N + a0] : 0.0;
            }
#pragma unroll
            for (int py = 0; py < Q; ++py) {
                double y00 = 0, y10 = 0, y01 = 0;
#pragma unroll
                for (int i = 0; i < N; ++i) {
                    y00 += lt.S[py][i] * z0[i];
                    y10 += lt.D[py][i] * z0[i];
                    y01 += lt.S[py][i] * z1[i];
                }
                Yb[((c * P + pl) * Q + py) * N + a0] = y00;
                if (c < 4) {
                    Yb[(((8 + c) * P + pl) * Q + py) * N + a0] = y10;
                    Yb[(((12 + c) * P + pl) * Q + py) * N + a0] = y01;
                }
            }
        }
        __syncthreads();
        // points of the chunk: x contraction and the integrands
        for (int it = tid; it < P * Q2; it += nth) {
            const int px = it % Q, py = (it / Q) % Q, pl = it / Q2, pz = pz0 + pl;
            if (pz >= Q) continue;
            double v[8], g[4][3];
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                double s = 0, dx = 0, dy = 0, dz = 0;
#pragma unroll
                for (int i = 0; i < N; ++i) {
                    const double y00 = Yb[((c * P + pl) * Q + py) * N + i];
                    s += lt.S[px][i] * y00;
                    if (c < 4) {
                        dx += lt.D[px][i] * y00;
                        dy += lt.S[px][i] * Yb[(((8 + c) * P + pl) * Q + py) * N + i];
                        dz += lt.S[px][i] * Yb[(((12 + c) * P + pl) * Q + py) * N + i];
                    }
                }
                v[c] = s;
                if (c < 4) {
                    g[c][0] = dx;
                    g[c][1] = dy;
                    g[c][2] = dz;
                }
            }
            double J[9], jxw;
            if constexpr (GEN) {
                const int p = px + Q * (py + Q * pz);
                const double* gm = a.cell_metric + e * 10 * Q3 + p;
#pragma unroll
                for (int m = 0; m < 9; ++m) J[m] = gm[m * Q3];
                jxw = gm[9 * Q3];
            } else {
#pragma unroll
                for (int m = 0; m < 9; ++m) J[m] = Jc[m];
                jxw = detJ * lt.w[px] * lt.w[py] * lt.w[pz];
            }
            const double rinv = 1.0 / v[0];
            const double u[3] = {v[1] * rinv, v[2] * rinv, v[3] * rinv};
            double gg = 0;
#pragma unroll
            for (int al = 0; al < 3; ++al)
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    double gm_ = 0, gr = 0;
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        gm_ += J[d * 3 + j] * g[1 + al][d];
                        gr += J[d * 3 + j] * g[0][d];
                    }
                    const double du = (gm_ - u[al] * gr) * rinv;
                    gg += du * du;
                }
            acc[0] += 0.5 * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) * jxw;
            acc[1] += gg * jxw;
            if (L) {
                double r = 0;
#pragma unroll
                for (int al = 0; al < 3; ++al) r += u[al] * (v[5 + al] - u[al] * v[4]) * rinv;
                acc[2] -= r * jxw;
            }
            acc[8] += jxw;
        }
        __syncthreads();
    }

    // conserved totals with the k+1 rule: values at the mass points, times |J| w
    double* t0 = sW;
    double* t1 = sW + 5 * N3;
    sweep_nn<N, double, false>(lm.Sm, sX, t0, 0);
    __syncthreads();
    sweep_nn<N, double, false>(lm.Sm, t0, t1, 1);
    __syncthreads();
    sweep_nn<N, double, false>(lm.Sm, t1, t0, 2);
    __syncthreads();
    for (int p = tid; p < N3; p += nth) {
        double jxw;
        if constexpr (GEN) jxw = a.mass_jxw[e * N3 + p];
        else jxw = detJ * lm.wm[p % N] * lm.wm[(p / N) % N] * lm.wm[p / N2];
#pragma unroll
        for (int c = 0; c < 5; ++c) acc[3 + c] += t0[c * N3 + p] * jxw;
    }
    block_sums<kDiagSums>(acc, red);
    if (tid < kDiagSums) {
        double s = 0;
#pragma unroll
        for (int m = 0; m < kDiagSums; ++m)
            if (m == tid) s = acc[m];
        partial[e * kDiagSums + tid] = s;
    }
}

template <int N, int Q, bool GEN>
__global__ void __launch_bounds__(kDiagBlock)
ke_vjp_kernel(OpArgs a, double* Ub, KTab<N, Q, double> tb) {
    constexpr int N2 = N * N, N3 = N2 * N, Q2 = Q * Q, Q3 = Q2 * Q;
    // values of rho, m at all n_q^3 points: X -> Z [4][Q][N^2] -> Y [4][Q][Q][N] -> G [4][Q^3]
    constexpr int SZ = 4 * Q * N2, SY = 4 * Q2 * N, SG = 4 * Q3;
    __shared__ double sX[4 * N3];
    __shared__ double sA[CMax<SZ, SG>::v];
    __shared__ double sB[CMax<SY, 4 * N2 * Q>::v];
    __shared__ KTab<N, Q, double> lt;
    const int64_t e = blockIdx.x;
    const int tid = threadIdx.x, nth = blockDim.x;
    const int64_t cs = a.ncell * N3;
    for (int i = tid; i < 4 * N3; i += nth) sX[i] = a.U[(i / N3) * cs + e * N3 + i % N3];
    copy_table<KTab<N, Q, double>, double>(tb, lt);
    __syncthreads();
    // forward: Z = S_z X, Y = S_y Z, G = S_x Y
    for (int it = tid; it < 4 * N2; it += nth) {
        const int c = it / N2, r = it % N2;
        for (int pz = 0; pz < Q; ++pz) {
            double s = 0;
#pragma unroll
            for (int i = 0; i < N; ++i) s += lt.S[pz][i] * sX[c * N3 + i * N2 + r];
            sA[(c * Q + pz) * N2 + r] = s;
        }
    }
    __syncthreads();
    for (int it = tid; it < 4 * Q * N; it += nth) {
        const int a0 = it % N, pz = (it / N) % Q, c = it / (N * Q);
        for (int py = 0; py < Q; ++py) {
            double s = 0;
#pragma unroll
            for (int i = 0; i < N; ++i) s += lt.S[py][i] * sA[(c * Q + pz) * N2 + i * N + a0];
            sB[((c * Q + pz) * Q + py) * N + a0] = s;
        }
    }
    __syncthreads();
    // point values and the integrand's derivative g = d(|u|^2/2)/d(rho, m) w|J|
    for (int p = tid; p < Q3; p += nth) {
        const int px = p % Q, py = (p / Q) % Q, pz = p / Q2;
        double v[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            double s = 0;
#pragma unroll
            for (int i = 0; i < N; ++i) s += lt.S[px][i] * sB[((c * Q + pz) * Q + py) * N + i];
            v[c] = s;
        }
        double jxw;
        if constexpr (GEN) jxw = a.cell_metric[(e * 10 + 9) * Q3 + p];
        else jxw = a.cell_metric[e * 10 + 9] * lt.w[px] * lt.w[py] * lt.w[pz];
        const double r = 1.0 / v[0];
        const double u0 = v[1] * r, u1 = v[2] * r, u2 = v[3] * r;
        const double wr = jxw * r;
        // |u|^2/2 = |m|^2 / (2 rho^2): d/dm = u / rho, d/drho = -|u|^2 / rho
        sA[p] = -(u0 * u0 + u1 * u1 + u2 * u2) * wr;
        sA[Q3 + p] = u0 * wr;
        sA[2 * Q3 + p] = u1 * wr;
        sA[3 * Q3 + p] = u2 * wr;
    }
    __syncthreads();
    // transposed: Bx = S_x^T G [4][pz][py][a0], By = S_y^T Bx [4][pz][a1][a0], Ub = S_z^T By
    for (int it = tid; it < 4 * Q2 * N; it += nth) {
        const int a0 = it % N, py = (it / N) % Q, pz = (it / (N * Q)) % Q, c = it / (N * Q2);
        double s = 0;
        for (int px = 0; px < Q; ++px) s += lt.S[px][a0] * sA[c * Q3 + (pz * Q + py) * Q + px];
        sB[((c * Q + pz) * Q + py) * N + a0] = s;
    }
    __syncthreads();
    // By [4][Q][N^2] goes to sA: the point values G are dead
    for (int it = tid; it < 4 * Q * N2; it += nth) {
        const int a0 = it % N, a1 = (it / N) % N, pz = (it / N2) % Q, c = it / (N2 * Q);
        double s = 0;
        for (int py = 0; py < Q; ++py) s += lt.S[py][a1] * sB[((c * Q + pz) * Q + py) * N + a0];
        sA[(c * Q + pz) * N2 + a1 * N + a0] = s;
    }
    __syncthreads();
    for (int it = tid; it < 5 * N3; it += nth) {
        const int c = it / N3, i = it % N3, a2 = i / N2, r = i % N2;
        double s = 0;
        if (c < 4)
            for (int pz = 0; pz < Q; ++pz) s += lt.S[pz][a2] * sA[(c * Q + pz) * N2 + r];
        Ub[c * cs + e * N3 + i] = s;
    }
}

// Channel statistics (Sec. 5.3: averages over the homogeneous directions x, z).  Per
// cell and wall-normal Gauss point p_y, the |det J| w weighted sums over the (p_x, p_z)
// points of [1, rho, u, v, w, uu, vv, ww, uv], u = (rho u)/rho, written to
// partial[(e * Q + p_y) * kStats + m].  Values at the points by the z / y / x sweeps;
// each thread sums one (p_y, p_z) line over p_x, then one (p_y, m) over p_z (fixed order).
constexpr int kStats = 9;

template <int N, int Q, bool GEN>
__global__ void __launch_bounds__(kDiagBlock)
chan_stats_kernel(OpArgs a, double* partial, KTab<N, Q, double> tb) {
    constexpr int N2 = N * N, N3 = N2 * N, Q2 = Q * Q, Q3 = Q2 * Q;
    __shared__ double sX[4 * N3];          // rho, m
    __shared__ double sA[4 * Q * N2];      // z-swept [c][pz][a1 a0]
    __shared__ double sB[4 * Q2 * N];      // y-swept [c][pz][py][a0]
    __shared__ double sP[kStats * Q2];     // line sums [m][py][pz]
    __shared__ KTab<N, Q, double> lt;
    const int64_t e = blockIdx.x;
    const int tid = threadIdx.x, nth = blockDim.x;
    const int64_t cs = a.ncell * N3;
    for (int i = tid; i < 4 * N3; i += nth) sX[i] = a.U[(i / N3) * cs + e * N3 + i % N3];
    copy_table<KTab<N, Q, double>, double>(tb, lt);
    __syncthreads();
    for (int it = tid; it < 4 * N2; it += nth) {
        const int c = it / N2, r = it % N2;
        for (int pz = 0; pz < Q; ++pz) {
            double s = 0;
#pragma unroll
            for (int i = 0; i < N; ++i) s += lt.S[pz][i] * sX[c * N3 + i * N2 + r];
            sA[(c * Q + pz) * N2 + r] = s;
        }
    }
    __syncthreads();
    for (int it = tid; it < 4 * Q * N; it += nth) {
        const int a0 = it % N, pz = (it / N) % Q, c = it / (N * Q);
        for (int py = 0; py < Q; ++py) {
            double s = 0;
#pragma unroll
            for (int i = 0; i < N; ++i) s += lt.S[py][i] * sA[(c * Q + pz) * N2 + i * N + a0];
            sB[((c * Q + pz) * Q + py) * N + a0] = s;
        }
    }
    __syncthreads();
    const double detJ = GEN ? 1.0 : a.cell_metric[e * 10 + 9];
    for (int it = tid; it < Q2; it += nth) {
        const int py = it % Q, pz = it / Q;
        double acc[kStats];
#pragma unroll
        for (int m = 0; m < kStats; ++m) acc[m] = 0;
        for (int px = 0; px < Q; ++px) {
            double v[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                double s = 0;
#pragma unroll
                for (int i = 0; i < N; ++i) s += lt.S[px][i] * sB[((c * Q + pz) * Q + py) * N + i];
                v[c] = s;
            }
            const int p = px + Q * (py + Q * pz);
            const double jxw = GEN ? a.cell_metric[(e * 10 + 9) * Q3 + p] : detJ * lt.w[px] * lt.w[py] * lt.w[pz];
            const double r = 1.0 / v[0];
            const double u0 = v[1] * r, u1 = v[2] * r, u2 = v[3] * r;
            acc[0] += jxw;
            acc[1] += v[0] * jxw;
            acc[2] += u0 * jxw;
            acc[3] += u1 * jxw;
            acc[4] += u2 * jxw;
            acc[5] += u0 * u0 * jxw;
            acc[6] += u1 * u1 * jxw;
            acc[7] += u2 * u2 * jxw;
            acc[8] += u0 * u1 * jxw;
        }
#pragma unroll
        for (int m = 0; m < kStats; ++m) sP[(m * Q + py) * Q + pz] = acc[m];
    }
    __syncthreads();
    for (int it = tid; it < kStats * Q; it += nth) {
        const int m = it / Q, py = it % Q;
        double s = 0;
        for (int pz = 0; pz < Q; ++pz) s += sP[(m * Q + py) * Q + pz];
        partial[(e * Q + py) * kStats + m] = s;
    }
}

// Wall shear stress of the channel (Sec. 5.3, u_tau = sqrt(tau_w / rho)).  Workgroup w
// takes the wall cell w of [the cells (i, k) of row j = 0, whose face xi_1 = 0 is the lower
// wall | the cells of row j = n1 - 1, face xi_1 = 1 the upper wall] and sums over its wall
// face's n_q^2 points, weighted by dA w, the shear mu du_1/dn with n the wall normal into
// the fluid (+x_2 at the lower wall, -x_2 at the upper), the density and 1:
// partial[3 w + {0, 1, 2}].  du_1/dx_2 = (d(rho u_1)/dx_2 - u_1 drho/dx_2)/rho from the
// cell's polynomial, the physical derivative through the cell's J^{-1} at the face point.
constexpr int kWallSums = 3;

template <int N, int Q, bool GEN>
__global__ void __launch_bounds__(64) chan_wall_shear_kernel(OpArgs a, double* partial, KTab<N, Q, double> tb) {
    constexpr int N2 = N * N, N3 = N2 * N, Q2 = Q * Q;
    __shared__ double sX[2 * N3];   // rho, rho u_1
    __shared__ double red[kWallSums * 64];
    const int n0 = a.n[0], n1 = a.n[1], n2 = a.n[2];
    const int w = blockIdx.x, tid = threadIdx.x;
    const int top = w >= n0 * n2 ? 1 : 0;
    const int wl = w - top * n0 * n2, i = wl % n0, kk = wl / n0, j = top ? n1 - 1 : 0;
    const int64_t e = i + (int64_t)n0 * (j + (int64_t)n1 * kk);
    const int64_t cs = a.ncell * N3;
    for (int m = tid; m < 2 * N3; m += blockDim.x) sX[m] = a.U[(m / N3) * cs + e * N3 + m % N3];
    __syncthreads();
    const int s = top;
    // face point number r = q0 + Q q2 (tangential axes x_0, x_2); face id of the wall face
    const int64_t fid = (j + s) + (int64_t)(n1 + 1) * (i + (int64_t)n0 * kk);
    double acc[kWallSums] = {0, 0, 0};
    for (int r = tid; r < Q2; r += blockDim.x) {
        const int q0 = r % Q, q2 = r / Q;
        double v[2] = {0, 0}, g[2][3] = {{0, 0, 0}, {0, 0, 0}};
        for (int a2 = 0; a2 < N; ++a2)
            for (int a1 = 0; a1 < N; ++a1)
                for (int a0 = 0; a0 < N; ++a0) {
                    const double p0 = tb.S[q0][a0], p1 = tb.fv[s][a1], p2 = tb.S[q2][a2];
                    const double d0 = tb.D[q0][a0], d1 = tb.fd[s][a1], d2 = tb.D[q2][a2];
                    for (int c = 0; c < 2; ++c) {
                        const double x = sX[c * N3 + a0 + N * (a1 + N * a2)];
                        v[c] += p0 * p1 * p2 * x;
                        g[c][0] += d0 * p1 * p2 * x;
                        g[c][1] += p0 * d1 * p2 * x;
                        g[c][2] += p0 * p1 * d2 * x;
                    }
                }
        double Ji[9], dAw;
        if constexpr (GEN) {
            const double* fd = a.face_data[1] + fid * 22 * Q2 + r;
            dAw = fd[3 * Q2];
            const int own = s ? 4 : 13;   // the cell is the lower side of the upper wall face
            for (int m = 0; m < 9; ++m) Ji[m] = fd[(own + m) * Q2];
        } else {
            const double* cm = a.cell_metric + e * 10;
            for (int m = 0; m < 9; ++m) Ji[m] = cm[m];
            const double l = sqrt(cm[3] * cm[3] + cm[4] * cm[4] + cm[5] * cm[5]);
            dAw = cm[9] * l * tb.w[q0] * tb.w[q2];
        }
        // d/dx_2 = sum_d (dxi_d / dx_2) d/dxi_d
        const double drho = Ji[1] * g[0][0] + Ji[4] * g[0][1] + Ji[7] * g[0][2];
        const double dm = Ji[1] * g[1][0] + Ji[4] * g[1][1] + Ji[7] * g[1][2];
        const double u = v[1] / v[0];
        const double dudy = (dm - u * drho) / v[0];
        acc[0] += dAw * a.mu * (s ? -dudy : dudy);
        acc[1] += dAw * v[0];
        acc[2] += dAw;
    }
    for (int m = 0; m < kWallSums; ++m) red[m * 64 + tid] = acc[m];
    __syncthreads();
    if (tid < kWallSums) {
        double t = 0;
        for (int l = 0; l < 64; ++l) t += red[tid * 64 + l];
        partial[(int64_t)w * kWallSums + tid] = t;
    }
}

template <int N, int Q, bool GEN>
inline int launch_wall_shear_t(const OpArgs& a, const Tables1D& t, double* partial, hipStream_t st) {
    KTab<N, Q, double> kt;
    MTab<N, double> mt;
    fill_tables<N, Q, double>(t, kt, mt);
    hipLaunchKernelGGL((chan_wall_shear_kernel<N, Q, GEN>), dim3((unsigned)(2 * a.n[0] * a.n[2])), dim3(64), 0, st, a,
                       partial, kt);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int N, int Q, bool GEN>
inline int launch_chan_stats_t(const OpArgs& a, const Tables1D& t, double* partial, hipStream_t st) {
    KTab<N, Q, double> kt;
    MTab<N, double> mt;
    fill_tables<N, Q, double>(t, kt, mt);
    hipLaunchKernelGGL((chan_stats_kernel<N, Q, GEN>), dim3((unsigned)a.ncell), dim3(kDiagBlock), 0, st, a, partial, kt);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int N, int Q, bool GEN>
inline int launch_diag_t(const OpArgs& a, const Tables1D& t, const double* L, double* partial, hipStream_t st) {
    KTab<N, Q, double> kt;
    MTab<N, double> mt;
    fill_tables<N, Q, double>(t, kt, mt);
    hipLaunchKernelGGL((diag_kernel<N, Q, GEN>), dim3((unsigned)a.ncell), dim3(kDiagBlock), 0, st, a, L, partial, kt, mt);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// diag_kernel for the high degrees (k >= 8), where a cell's U and L do not fit in LDS: the
// same nine partial sums, one quadrature plane along xi_2 at a time.  Per plane the z sweep
// reads the coefficient lines of rho, m (and L_rho, L_m) from global memory, then the y and x
// sweeps and the integrands as above; the conserved totals take a second pass, one plane of
// mass points at a time (the k+1 rule of the inverse mass matrix).  Tables from the device
// copy of Tables1D.
constexpr int kDiagHdBlock = 256;

template <int N, int Q>
struct DiagHdSizes {
    static constexpr int N2 = N * N;
    static constexpr int Z = 12 * N2;      // Z0 [8][a1 a0], Z1 [4][a1 a0] of one plane
    static constexpr int Y = 16 * Q * N;   // Y00 [8][py][a0], Y10 [4][py][a0], Y01 [4][py][a0]
    static constexpr int WORK = CMax<Z + Y, 10 * N2>::v;   // mass pass: [5][a1 a0] twice
};

template <int N, int Q, bool GEN>
__global__ void __launch_bounds__(kDiagHdBlock)
diag_hd_kernel(OpArgs a, const double* L, double* partial) {
    using DS = DiagHdSizes<N, Q>;
    constexpr int N2 = N * N, N3 = N2 * N, Q2 = Q * Q, Q3 = Q2 * Q;
    __shared__ double sW[DS::WORK];
    __shared__ double red[kDiagSums * kDiagHdBlock];
    __shared__ double S[Q][N], D[Q][N], w[Q], Sm[N][N], wm[N];
    const Tables1D* t = a.tab_dev;
    const int64_t e = blockIdx.x;
    const int tid = threadIdx.x, nth = blockDim.x;
    const int64_t cs = a.ncell * N3;
    for (int i = tid; i < Q * N; i += nth) {
        S[i / N][i % N] = t->S[i / N][i % N];
        D[i / N][i % N] = t->D[i / N][i % N];
    }
    for (int i = tid; i < N2; i += nth) Sm[i / N][i % N] = t->Sm[i / N][i % N];
    if (tid < Q) w[tid] = t->w[tid];
    if (tid < N) wm[tid] = t->wm[tid];
    double Jc[9], detJ = 1;
    if constexpr (!GEN) {
#pragma unroll
        for (int m = 0; m < 9; ++m) Jc[m] = a.cell_metric[e * 10 + m];
        detJ = a.cell_metric[e * 10 + 9];
    }
    double acc[kDiagSums];
#pragma unroll
    for (int m = 0; m < kDiagSums; ++m) acc[m] = 0;
    __syncthreads();

    // interpolated components c < 8: rho, m (rows 0..3 of U), L_rho, L_m (rows 0..3 of L)
    double* Z = sW;
    double* Yb = sW + DS::Z;
    for (int pz = 0; pz < Q; ++pz) {
        // z: Z0[c] = (S_z X_c)(pz), Z1[c] = (D_z X_c)(pz) for c < 4     [c][a1 a0]
        for (int it = tid; it < 8 * N2; it += nth) {
            const int c = it / N2, r = it % N2;
            double z0 = 0, z1 = 0;
            if (c < 4 || L) {
                const double* x = (c < 4 ? a.U + c * cs : L + (c - 4) * cs) + e * N3 + r;
#pragma unroll 4
                for (int i = 0; i < N; ++i) {
                    const double v = x[i * N2];
                    z0 += S[pz][i] * v;
                    z1 += D[pz][i] * v;
                }
            }
            Z[c * N2 + r] = z0;
            if (c < 4) Z[(8 + c) * N2 + r] = z1;
        }
        __syncthreads();
        // y: Y00 = S_y Z0 (8), Y10 = D_y Z0 (4), Y01 = S_y Z1 (4)     [kind c][py][a0]
        for (int it = tid; it < 8 * Q * N; it += nth) {
            const int a0 = it % N, py = (it / N) % Q, c = it / (N * Q);
            double y00 = 0, y10 = 0, y01 = 0;
#pragma unroll 4
            for (int i = 0; i < N; ++i) {
                const double z0 = Z[c * N2 + i * N + a0];
                y00 += S[py][i] * z0;
                if (c < 4) {
                    y10 += D[py][i] * z0;
                    y01 += S[py][i] * Z[(8 + c) * N2 + i * N + a0];
                }
            }
            Yb[(c * Q + py) * N + a0] = y00;
            if (c < 4) {
                Yb[((8 + c) * Q + py) * N + a0] = y10;
                Yb[((12 + c) * Q + py) * N + a0] = y01;
            }
        }
        __syncthreads();
        // points of the plane: x contraction and the integrands
        for (int it = tid; it < Q2; it += nth) {
            const int px = it % Q, py = it / Q;
            double v[8], g[4][3];
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                double sv = 0, dx = 0, dy = 0, dz = 0;
#pragma unroll 4
                for (int i = 0; i < N; ++i) {
                    const double y00 = Yb[(c * Q + py) * N + i];
                    sv += S[px][i] * y00;
                    if (c < 4) {
                        dx += D[px][i] * y00;
                        dy += S[px][i] * Yb[((8 + c) * Q + py) * N + i];
                        dz += S[px][i] * Yb[((12 + c) * Q + py) * N + i];
                    }
                }
                v[c] = sv;
                if (c < 4) {
                    g[c][0] = dx;
                    g[c][1] = dy;
                    g[c][2] = dz;
                }
            }
            double J[9], jxw;
            if constexpr (GEN) {
                const double* gm = a.cell_metric + e * 10 * Q3 + px + Q * (py + Q * pz);
#pragma unroll
                for (int m = 0; m < 9; ++m) J[m] = gm[m * Q3];
                jxw = gm[9 * Q3];
            } else {
#pragma unroll
                for (int m = 0; m < 9; ++m) J[m] = Jc[m];
                jxw = detJ * w[px] * w[py] * w[pz];
            }
            const double rinv = 1.0 / v[0];
            const double u[3] = {v[1] * rinv, v[2] * rinv, v[3] * rinv};
            double gg = 0;
#pragma unroll
            for (int al = 0; al < 3; ++al)
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    double gm_ = 0, gr = 0;
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        gm_ += J[d * 3 + j] * g[1 + al][d];
                        gr += J[d * 3 + j] * g[0][d];
                    }
                    const double du = (gm_ - u[al] * gr) * rinv;
                    gg += du * du;
                }
            acc[0] += 0.5 * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) * jxw;
            acc[1] += gg * jxw;
            if (L) {
                double r = 0;
#pragma unroll
                for (int al = 0; al < 3; ++al) r += u[al] * (v[5 + al] - u[al] * v[4]) * rinv;
                acc[2] -= r * jxw;
            }
            acc[8] += jxw;
        }
        __syncthreads();
    }

    // conserved totals with the k+1 rule, one plane pm of mass points at a time
    double* A = sW;            // S_m along xi_2   [c][a1 a0]
    double* B = sW + 5 * N2;   // then along xi_1  [c][p1][a0]
    for (int pm = 0; pm < N; ++pm) {
        for (int it = tid; it < 5 * N2; it += nth) {
            const int c = it / N2, r = it % N2;
            const double* x = a.U + c * cs + e * N3 + r;
            double sv = 0;
#pragma unroll 4
            for (int i = 0; i < N; ++i) sv += Sm[pm][i] * x[i * N2];
            A[c * N2 + r] = sv;
        }
        __syncthreads();
        for (int it = tid; it < 5 * N2; it += nth) {
            const int a0 = it % N, p1 = (it / N) % N, c = it / N2;
            double sv = 0;
#pragma unroll 4
            for (int i = 0; i < N; ++i) sv += Sm[p1][i] * A[c * N2 + i * N + a0];
            B[c * N2 + p1 * N + a0] = sv;
        }
        __syncthreads();
        for (int it = tid; it < N2; it += nth) {
            const int p0 = it % N, p1 = it / N;
            double jxw;
            if constexpr (GEN) jxw = a.mass_jxw[e * N3 + p0 + N * (p1 + N * pm)];
            else jxw = detJ * wm[p0] * wm[p1] * wm[pm];
#pragma unroll
            for (int c = 0; c < 5; ++c) {
                double sv = 0;
#pragma unroll 4
                for (int i = 0; i < N; ++i) sv += Sm[p0][i] * B[c * N2 + p1 * N + i];
                acc[3 + c] += sv * jxw;
            }
        }
        __syncthreads();
    }
    block_sums<kDiagSums>(acc, red);
    if (tid < kDiagSums) {
        double sv = 0;
#pragma unroll
        for (int m = 0; m < kDiagSums; ++m)
            if (m == tid) sv = acc[m];
        partial[e * kDiagSums + tid] = sv;
    }
}

template <int N, int Q, bool GEN>
inline int launch_diag_hd_t(const OpArgs& a, const double* L, double* partial, hipStream_t st) {
    hipLaunchKernelGGL((diag_hd_kernel<N, Q, GEN>), dim3((unsigned)a.ncell), dim3(kDiagHdBlock), 0, st, a, L,
                       partial);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int N, int Q, bool GEN>
inline int launch_ke_vjp_t(const OpArgs& a, const Tables1D& t, double* Ub, hipStream_t st) {
    KTab<N, Q, double> kt;
    MTab<N, double> mt;
    fill_tables<N, Q, double>(t, kt, mt);
    hipLaunchKernelGGL((ke_vjp_kernel<N, Q, GEN>), dim3((unsigned)a.ncell), dim3(kDiagBlock), 0, st, a, Ub, kt);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace dgns
