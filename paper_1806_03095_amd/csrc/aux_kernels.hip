// Memory-bound and setup kernels around the DG operator: the low-storage
// Runge-Kutta stage update (paper Sec. 2.4), the kinetic-energy / dissipation
// diagnostics (Sec. 5.2.3) and the L2 projection of the initial states of
// Sec. 5.2.1 (Taylor-Green) and Sec. 5.3.1 (channel).

#include "dg_common.h"
#include "dg_kernels.h"
#include "dgns.h"

namespace dgns {

// Workgroups of 256 threads for a streaming kernel over n items: one item per thread.
// Measured on vectors of 672 MB, a full grid moves a copy at 6.2 TB/s and the RK
// stage update at 5.55 TB/s, against 4.9 and 4.6 TB/s for a grid of 16,384
// workgroups striding over the vector.  The kernels keep their grid-stride loops,
// which only matter past 2^30 workgroups.
static inline int64_t stream_blocks(int64_t n) {
    int64_t blocks = (n + 255) / 256;
    if (blocks > (int64_t(1) << 30)) blocks = int64_t(1) << 30;
    return blocks < 1 ? 1 : blocks;
}

// ------------------------------------------------------------------ LSRK update
// dU <- A dU + dt L;  U <- U + B dU.  With A == 0 the old dU is not read (it may
// hold anything, including NaN, on the first stage).
template <bool FIRST>
__global__ void __launch_bounds__(256) rk_update_kernel(double* __restrict__ U, double* __restrict__ dU,
                                                        const double* __restrict__ L, int64_t n2, double A,
                                                        double B, double dt) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    double2* U2 = reinterpret_cast<double2*>(U);
    double2* dU2 = reinterpret_cast<double2*>(dU);
    const double2* L2 = reinterpret_cast<const double2*>(L);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += stride) {
        const double2 l = L2[i];
        double2 d;
        if (FIRST) {
            d.x = rk_increment(true, A, 0.0, dt, l.x);
            d.y = rk_increment(true, A, 0.0, dt, l.y);
        } else {
            const double2 o = dU2[i];
            d.x = rk_increment(false, A, o.x, dt, l.x);
            d.y = rk_increment(false, A, o.y, dt, l.y);
        }
        double2 u = U2[i];
        u.x = rk_advance(u.x, B, d.x);
        u.y = rk_advance(u.y, B, d.y);
        dU2[i] = d;
        U2[i] = u;
    }
}

__global__ void rk_update_tail(double* U, double* dU, const double* L, int64_t i, double A, double B, double dt,
                               int first) {
    const double d = rk_increment(first != 0, A, first ? 0.0 : dU[i], dt, L[i]);
    dU[i] = d;
    U[i] = rk_advance(U[i], B, d);
}

int launch_rk_update(double* U, double* dU, const double* L, int64_t n, double A, double B, double dt,
                     hipStream_t st) {
    const int64_t n2 = n / 2;
    if (n2 > 0) {
        int64_t blocks = stream_blocks(n2);
        if (A == 0.0)
            hipLaunchKernelGGL(rk_update_kernel<true>, dim3((unsigned)blocks), dim3(256), 0, st, U, dU, L, n2, A, B, dt);
        else
            hipLaunchKernelGGL(rk_update_kernel<false>, dim3((unsigned)blocks), dim3(256), 0, st, U, dU, L, n2, A, B, dt);
    }
    if (n % 2)
        hipLaunchKernelGGL(rk_update_tail, dim3(1), dim3(1), 0, st, U, dU, L, n - 1, A, B, dt, A == 0.0 ? 1 : 0);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// dU <- A dU + dt L;  U_out <- U_in + B dU, with L possibly aliasing U_out (each entry of
// L is read before the same entry of U_out is written, by the same thread).
__global__ void __launch_bounds__(256) rk_update_to_kernel(const double* U_in, double* U_out, double* dU,
                                                           const double* L, int64_t n, double A, double B,
                                                           double dt, int first) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double l = L[i];
        const double d = rk_increment(first != 0, A, first ? 0.0 : dU[i], dt, l);
        dU[i] = d;
        U_out[i] = rk_advance(U_in[i], B, d);
    }
}

int launch_rk_update_to(const double* U_in, double* U_out, double* dU, const double* L, int64_t n, double A, double B,
                        double dt, hipStream_t st) {
    if (n <= 0) return 0;
    const int64_t blocks = stream_blocks(n);
    hipLaunchKernelGGL(rk_update_to_kernel, dim3((unsigned)blocks), dim3(256), 0, st, U_in, U_out, dU, L, n, A, B, dt,
                       A == 0.0 ? 1 : 0);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// ------------------------------------------------------------------ diagnostics
// Totals of the nine per-cell partial sums that diag_kernel (diag_impl.h) writes:
// [0] int |u|^2/2, [1] int grad u : grad u, [2] -int u.(L_m - u L_rho)/rho,
// [3..7] int U (k+1 rule), [8] volume.
constexpr int kDiag = 9;

__device__ inline double block_sum(double v, double* red) {
    const int tid = threadIdx.x;
    red[tid] = v;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (tid < s) red[tid] += red[tid + s];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// Totals of the per-cell partial sums: workgroup m sums quantity m over all cells in
// a fixed order (deterministic).
__global__ void __launch_bounds__(1024) diag_total_kernel(const double* partial, int64_t ncell, double* total) {
    __shared__ double red[1024];
    const int m = blockIdx.x;
    double s = 0;
    for (int64_t e = threadIdx.x; e < ncell; e += blockDim.x) s += partial[e * kDiag + m];
    const double r = block_sum(s, red);
    if (threadIdx.x == 0) total[m] = r;
}

int launch_diag_total(const double* partial, int64_t ncell, double* total, hipStream_t st) {
    hipLaunchKernelGGL(diag_total_kernel, dim3(kDiag), dim3(1024), 0, st, partial, ncell, total);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// The eight diagnostics from the nine totals, as dgns_diagnostics forms them on the host:
// e_k = T0 / V, eps = nu T1 / V, -de_k/dt = T2 / V (NaN without L), the conserved totals.
__global__ void diag_finalize_kernel(const double* total, double nu, int has_L, double* out8) {
    const int i = threadIdx.x;
    if (i >= 8) return;
    const double V = total[8];
    double r;
    if (i == 0) r = total[0] / V;
    else if (i == 1) r = nu * total[1] / V;
    else if (i == 2) r = has_L ? total[2] / V : __builtin_nan("");
    else r = total[i];
    out8[i] = r;
}

int launch_diag_finalize(const double* total, double nu, int has_L, double* out8, hipStream_t st) {
    hipLaunchKernelGGL(diag_finalize_kernel, dim3(1), dim3(64), 0, st, total, nu, has_L, out8);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Totals of the channel statistics over each plane of cells: thread (j, p, m) sums
// quantity m at wall-normal point p over the cells (i, j, k) of row j in a fixed order.
constexpr int kChanStats = 9;
__global__ void __launch_bounds__(256) chan_stats_total_kernel(const double* partial, int n0, int n1, int n2, int q,
                                                             double* total) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n1 * q * kChanStats) return;
    const int m = t % kChanStats, p = (t / kChanStats) % q, j = t / (kChanStats * q);
    double s = 0;
    for (int k = 0; k < n2; ++k)
        for (int i = 0; i < n0; ++i) {
            const int64_t e = i + (int64_t)n0 * (j + (int64_t)n1 * k);
            s += partial[(e * q + p) * kChanStats + m];
        }
    total[t] = s;
}

int launch_chan_stats_total(const double* partial, const int n[3], int q, double* total, hipStream_t st) {
    const int nt = n[1] * q * kChanStats;
    hipLaunchKernelGGL(chan_stats_total_kernel, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, st, partial, n[0], n[1],
                       n[2], q, total);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// ------------------------------------------------------------------ initial states
__device__ inline void initial_state(int ic, const double* q, double gamma, double R, const double x[3], double U[5]) {
    double rho, u[3], p;
    if (ic == DGNS_IC_TAYLOR_GREEN) {
        const double U0 = q[0], L = q[1], M = q[2], rho0 = q[3];
        const double c0 = U0 / M, T0 = c0 * c0 / (gamma * R), p0 = rho0 * R * T0;
        const double x1 = x[0] / L, x2 = x[1] / L, x3 = x[2] / L;
        u[0] = U0 * sin(x1) * cos(x2) * cos(x3);
        u[1] = -U0 * cos(x1) * sin(x2) * cos(x3);
        u[2] = 0.0;
        p = p0 + rho0 * U0 * U0 / 16.0 * (cos(2.0 * x1) + cos(2.0 * x2)) * (cos(2.0 * x3) + 2.0);
        rho = p / (R * T0);
    } else if (ic == DGNS_IC_CHANNEL) {
        const double umax = q[0], M = q[1], pw = q[2];
        const double c = umax / M, T0 = c * c / (gamma * R);
        rho = 1.0;
        u[0] = umax * (1.0 - pow(fabs(x[1]), pw));
        u[1] = u[2] = 0.0;
        p = rho * R * T0;
    } else {
        rho = q[0];
        u[0] = q[1];
        u[1] = q[2];
        u[2] = q[3];
        p = q[4];
    }
    U[0] = rho;
    U[1] = rho * u[0];
    U[2] = rho * u[1];
    U[3] = rho * u[2];
    U[4] = p / (gamma - 1.0) + 0.5 * rho * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
}

// out_i = sum_p phi_i(x_p) |det J| w_p U0(x(x_p)) with the n_q rule (before M^{-1}).
// The components go in passes of cp (all five where their [cp][Q^3] point values fit
// the dynamic LDS, fewer at the largest n_q); the point values are recomputed per pass.
__global__ void __launch_bounds__(256) ic_rhs_kernel(OpArgs a, const Tables1D* __restrict__ tp, const double* geo, int ic,
                                                     const double* icp_d, double* out, int gen, int cp) {
    extern __shared__ double sv[];   // [cp][Q^3]
    const Tables1D& t = *tp;
    const int N = t.n, Q = t.q, N3 = N * N * N, Q3 = Q * Q * Q;
    const int64_t e = blockIdx.x;
    const int64_t cs = a.ncell * N3;
    double q[8];
    for (int m = 0; m < 8; ++m) q[m] = icp_d[m];
    for (int c0 = 0; c0 < 5; c0 += cp) {
        const int nc = 5 - c0 < cp ? 5 - c0 : cp;
        for (int p = threadIdx.x; p < Q3; p += blockDim.x) {
            const int p0 = p % Q, p1 = (p / Q) % Q, p2 = p / (Q * Q);
            double x[3] = {0, 0, 0};
            for (int i = 0; i < N3; ++i) {
                const int a0 = i % N, a1 = (i / N) % N, a2 = i / (N * N);
                const double g = t.Sg[p0][a0] * t.Sg[p1][a1] * t.Sg[p2][a2];
                for (int c = 0; c < 3; ++c) x[c] += g * geo[(e * 3 + c) * N3 + i];
            }
            double U[5];
            initial_state(ic, q, a.gamma, a.R, x, U);
            const double jxw =
                gen ? a.cell_metric[(e * 10 + 9) * Q3 + p] : a.cell_metric[e * 10 + 9] * t.w[p0] * t.w[p1] * t.w[p2];
            for (int c = 0; c < nc; ++c) sv[c * Q3 + p] = U[c0 + c] * jxw;
        }
        __syncthreads();
        for (int it = threadIdx.x; it < nc * N3; it += blockDim.x) {
            const int c = it / N3, i = it % N3;
            const int a0 = i % N, a1 = (i / N) % N, a2 = i / (N * N);
            double s = 0;
            for (int p = 0; p < Q3; ++p) {
                const int p0 = p % Q, p1 = (p / Q) % Q, p2 = p / (Q * Q);
                s += t.S[p0][a0] * t.S[p1][a1] * t.S[p2][a2] * sv[c * Q3 + p];
            }
            out[(c0 + c) * cs + e * N3 + i] = s;
        }
        __syncthreads();
    }
}

int launch_ic_rhs(const OpArgs& a, const Tables1D& t, const Tables1D* t_dev, const double* geo_nodes, int ic,
                  const double* icp, double* out, bool gen, hipStream_t st) {
    const size_t per = sizeof(double) * t.q * t.q * t.q;
    int cp = (int)((64 * 1024) / per);
    cp = cp < 1 ? 1 : (cp > 5 ? 5 : cp);
    hipLaunchKernelGGL(ic_rhs_kernel, dim3((unsigned)a.ncell), dim3(256), per * cp, st, a, t_dev, geo_nodes, ic, icp,
                       out, gen ? 1 : 0, cp);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

__global__ void channel_perturb_kernel(double* U, const double* X, const double* noise, int64_t n, double umax,
                                       double pw, double amp, double gamma, double R) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double rho = U[i];
    double u[3] = {U[n + i] / rho, U[2 * n + i] / rho, U[3 * n + i] / rho};
    const double T = (gamma - 1.0) * (U[4 * n + i] - 0.5 * rho * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2])) / (rho * R);
    const double base = umax * (1.0 - pow(fabs(X[n + i]), pw));
    for (int c = 0; c < 3; ++c) u[c] += amp * base * noise[c * n + i];
    for (int c = 0; c < 3; ++c) U[(1 + c) * n + i] = rho * u[c];
    U[4 * n + i] = rho * (R / (gamma - 1.0) * T + 0.5 * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]));
}

int launch_channel_perturb(double* U, const double* node_x, const double* noise, int64_t ncell, int n3, double umax,
                           double power, double amp, double gamma, double R, hipStream_t st) {
    const int64_t n = ncell * n3;
    hipLaunchKernelGGL(channel_perturb_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, U, node_x, noise, n,
                       umax, power, amp, gamma, R);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace dgns

namespace dgns {

// ------------------------------------------------------------------ adjoint helpers
__global__ void __launch_bounds__(256) fill_kernel(double* __restrict__ y, int64_t n, double v) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) y[i] = v;
}

int launch_fill(double* y, int64_t n, double v, hipStream_t st) {
    const int64_t blocks = stream_blocks(n);
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks), dim3(256), 0, st, y, n, v);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

__global__ void __launch_bounds__(256) axpby_kernel(double* __restrict__ y, const double* __restrict__ x, int64_t n,
                                                    double a, double b) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) y[i] = a * y[i] + b * x[i];
}

int launch_axpby(double* y, const double* x, int64_t n, double a, double b, hipStream_t st) {
    const int64_t blocks = stream_blocks(n);
    hipLaunchKernelGGL(axpby_kernel, dim3((unsigned)blocks), dim3(256), 0, st, y, x, n, a, b);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Ubar_i = sum_q w|J| phi_i(x_q) (-|u|^2, u_1, u_2, u_3, 0)/rho: the gradient of
// K = int |u|^2/2 (n_q rule, u = m/rho) with respect to the coefficients U_i.
}  // namespace dgns
