// Launchers of the DG kernels (one translation unit per polynomial degree).
// Each returns 0 on success, 1 if the (degree, n_q) pair has no compiled kernel,
// -1 if the launch failed.
#pragma once

#include "dg_common.h"

namespace dgns {

int launch_operator_k1(const OpArgs& a, const Tables1D& t, bool fp32, bool gen, hipStream_t st);
int launch_inverse_mass_k1(const double* R, double* L, int64_t ncell, const double* cm, const double* mj,
                            const Tables1D& t, bool fp32, bool gen, hipStream_t st);
int launch_operator_k2(const OpArgs& a, const Tables1D& t, bool fp32, bool gen, hipStream_t st);
int launch_inverse_mass_k2(const double* R, double* L, int64_t ncell, const double* cm, const double* mj,
                            const Tables1D& t, bool fp32, bool gen, hipStream_t st);
int launch_operator_k3(const OpArgs& a, const Tables1D& t, bool fp32, bool gen, hipStream_t st);
int launch_inverse_mass_k3(const double* R, double* L, int64_t ncell, const double* cm, const double* mj,
                            const Tables1D& t, bool fp32, bool gen, hipStream_t st);
int launch_operator_k4(const OpArgs& a, const Tables1D& t, bool fp32, bool gen, hipStream_t st);
int launch_inverse_mass_k4(const double* R, double* L, int64_t ncell, const double* cm, const double* mj,
                            const Tables1D& t, bool fp32, bool gen, hipStream_t st);
int launch_operator_k5(const OpArgs& a, const Tables1D& t, bool fp32, bool gen, hipStream_t st);
int launch_inverse_mass_k5(const double* R, double* L, int64_t ncell, const double* cm, const double* mj,
                            const Tables1D& t, bool fp32, bool gen, hipStream_t st);
int launch_operator_k6(const OpArgs& a, const Tables1D& t, bool fp32, bool gen, hipStream_t st);
int launch_inverse_mass_k6(const double* R, double* L, int64_t ncell, const double* cm, const double* mj,
                            const Tables1D& t, bool fp32, bool gen, hipStream_t st);
int launch_operator_k7(const OpArgs& a, const Tables1D& t, bool fp32, bool gen, hipStream_t st);
int launch_inverse_mass_k7(const double* R, double* L, int64_t ncell, const double* cm, const double* mj,
                            const Tables1D& t, bool fp32, bool gen, hipStream_t st);

// Adjoint of the residual, Ubar = (dR/dU)^T Rbar (float64; degrees 1..5).
int launch_adjoint_k1(const OpArgs& a, const double* Rb, const Tables1D& t, bool gen, hipStream_t st);
int launch_adjoint_k2(const OpArgs& a, const double* Rb, const Tables1D& t, bool gen, hipStream_t st);
int launch_adjoint_k3(const OpArgs& a, const double* Rb, const Tables1D& t, bool gen, hipStream_t st);
int launch_adjoint_k4(const OpArgs& a, const double* Rb, const Tables1D& t, bool gen, hipStream_t st);
int launch_adjoint_k5(const OpArgs& a, const double* Rb, const Tables1D& t, bool gen, hipStream_t st);
int launch_adjoint_k6(const OpArgs& a, const double* Rb, const Tables1D& t, bool gen, hipStream_t st);
int launch_adjoint_k7(const OpArgs& a, const double* Rb, const Tables1D& t, bool gen, hipStream_t st);

// (degree, n_q) pairs with compiled operator kernels
constexpr int kSupported[][2] = {{1, 2}, {1, 3}, {2, 3}, {2, 4}, {2, 5}, {3, 4}, {3, 5}, {3, 6}, {3, 7}, {4, 5},
                                 {4, 6}, {4, 7}, {4, 9}, {5, 6}, {5, 8}, {6, 7}, {6, 10}, {7, 8}, {7, 11}};

// Degrees 8..15 (hd_impl.h: the cell streamed through LDS plane by plane): n_q = k+1, and
// the 3/2 rule where its n_q^2 face points fit one pass of 256 threads (k <= 10).
constexpr int kSupportedHd[][2] = {{8, 9},  {8, 13},  {9, 10},  {9, 14},  {10, 11}, {10, 16},
                                   {11, 12}, {12, 13}, {13, 14}, {14, 15}, {15, 16}};
int launch_operator_hd1(const OpArgs& a, int k, int q, bool fp32, bool gen, hipStream_t st);   // k = 8..11
// The streamed kernels at lower degrees where they measured faster (op_hd0.hip).
bool streamed_preferred(int k, int q, bool fp32, const double force[3]);
// whether the streamed kernels can serve (k, n_q, precision) for some body force: the
// context then sizes the face buffer for their scratch as well
bool streamed_possible(int k, int q, bool fp32);
int launch_operator_hd0(const OpArgs& a, int k, int q, bool fp32, bool gen, hipStream_t st);
int launch_operator_hd2(const OpArgs& a, int k, int q, bool fp32, bool gen, hipStream_t st);   // k = 12..15
int launch_inverse_mass_hd1(const double* R, double* L, int64_t ncell, const double* cm, const double* mj,
                            const Tables1D* t_dev, int k, bool fp32, bool gen, hipStream_t st);
int launch_inverse_mass_hd2(const double* R, double* L, int64_t ncell, const double* cm, const double* mj,
                            const Tables1D* t_dev, int k, bool fp32, bool gen, hipStream_t st);

// LSRK stage update dU <- A dU + dt L; U <- U + B dU (A == 0: dU <- dt L).
int launch_rk_update(double* U, double* dU, const double* L, int64_t n, double A, double B, double dt, hipStream_t st);

// The same update into another buffer: dU <- A dU + dt L; U_out <- U_in + B dU.  L may
// alias U_out (each entry is read before it is written).
int launch_rk_update_to(const double* U_in, double* U_out, double* dU, const double* L, int64_t n, double A, double B,
                        double dt, hipStream_t st);

// Per-cell diagnostic partial sums (nine per cell, see diag_impl.h), float64.
int launch_diagnostics_k1(const OpArgs& a, const Tables1D& t, const double* L, double* partial, bool gen, hipStream_t st);
int launch_diagnostics_k2(const OpArgs& a, const Tables1D& t, const double* L, double* partial, bool gen, hipStream_t st);
int launch_diagnostics_k3(const OpArgs& a, const Tables1D& t, const double* L, double* partial, bool gen, hipStream_t st);
int launch_diagnostics_k4(const OpArgs& a, const Tables1D& t, const double* L, double* partial, bool gen, hipStream_t st);
int launch_diagnostics_k5(const OpArgs& a, const Tables1D& t, const double* L, double* partial, bool gen, hipStream_t st);
int launch_diagnostics_k6(const OpArgs& a, const Tables1D& t, const double* L, double* partial, bool gen, hipStream_t st);
int launch_diagnostics_k7(const OpArgs& a, const Tables1D& t, const double* L, double* partial, bool gen, hipStream_t st);

// Deterministic totals of the nine per-cell partial sums.
// Diagnostics at degrees 8..11 and 12..15 (diag_impl.h: diag_hd_kernel, one quadrature
// plane at a time); 1 if the pair has no kernel.
int launch_diagnostics_hd1(const OpArgs& a, int k, int q, const double* L, double* partial, bool gen, hipStream_t st);
int launch_diagnostics_hd2(const OpArgs& a, int k, int q, const double* L, double* partial, bool gen, hipStream_t st);
int launch_diag_total(const double* partial, int64_t ncell, double* total, hipStream_t st);

// out8 (device) = the eight diagnostics from the nine totals (device).
int launch_diag_finalize(const double* total, double nu, int has_L, double* out8, hipStream_t st);

// Channel statistics: per cell and wall-normal Gauss point, nine weighted sums (see
// diag_impl.h); then their totals over each plane of cells (n[1] * n_q * 9 values).
int launch_chan_stats_k1(const OpArgs& a, const Tables1D& t, double* partial, bool gen, hipStream_t st);
int launch_chan_stats_k2(const OpArgs& a, const Tables1D& t, double* partial, bool gen, hipStream_t st);
int launch_chan_stats_k3(const OpArgs& a, const Tables1D& t, double* partial, bool gen, hipStream_t st);
int launch_chan_stats_k4(const OpArgs& a, const Tables1D& t, double* partial, bool gen, hipStream_t st);
int launch_chan_stats_k5(const OpArgs& a, const Tables1D& t, double* partial, bool gen, hipStream_t st);
int launch_chan_stats_k6(const OpArgs& a, const Tables1D& t, double* partial, bool gen, hipStream_t st);
int launch_chan_stats_k7(const OpArgs& a, const Tables1D& t, double* partial, bool gen, hipStream_t st);
int launch_chan_stats_total(const double* partial, const int n[3], int q, double* total, hipStream_t st);

// Wall shear of the channel: per wall cell (lower row, then upper row) the dA w weighted
// sums of mu du_1/dn, rho and 1 over its wall face (3 per wall cell).
int launch_wall_shear_k1(const OpArgs& a, const Tables1D& t, double* partial, bool gen, hipStream_t st);
int launch_wall_shear_k2(const OpArgs& a, const Tables1D& t, double* partial, bool gen, hipStream_t st);
int launch_wall_shear_k3(const OpArgs& a, const Tables1D& t, double* partial, bool gen, hipStream_t st);
int launch_wall_shear_k4(const OpArgs& a, const Tables1D& t, double* partial, bool gen, hipStream_t st);
int launch_wall_shear_k5(const OpArgs& a, const Tables1D& t, double* partial, bool gen, hipStream_t st);
int launch_wall_shear_k6(const OpArgs& a, const Tables1D& t, double* partial, bool gen, hipStream_t st);
int launch_wall_shear_k7(const OpArgs& a, const Tables1D& t, double* partial, bool gen, hipStream_t st);

// L2 projection right-hand side of an analytic initial state, U_rhs = (phi_i, U0).
int launch_ic_rhs(const OpArgs& a, const Tables1D& t, const Tables1D* t_dev, const double* geo_nodes, int ic,
                  const double* icp, double* out, bool gen, hipStream_t st);

// y <- a y + b x (n doubles).
int launch_axpby(double* y, const double* x, int64_t n, double a, double b, hipStream_t st);

// Ubar = gradient of int |u|^2/2 (n_q rule) with respect to U, float64.
int launch_ke_vjp_k1(const OpArgs& a, const Tables1D& t, double* Ub, bool gen, hipStream_t st);
int launch_ke_vjp_k2(const OpArgs& a, const Tables1D& t, double* Ub, bool gen, hipStream_t st);
int launch_ke_vjp_k3(const OpArgs& a, const Tables1D& t, double* Ub, bool gen, hipStream_t st);
int launch_ke_vjp_k4(const OpArgs& a, const Tables1D& t, double* Ub, bool gen, hipStream_t st);
int launch_ke_vjp_k5(const OpArgs& a, const Tables1D& t, double* Ub, bool gen, hipStream_t st);
int launch_ke_vjp_k6(const OpArgs& a, const Tables1D& t, double* Ub, bool gen, hipStream_t st);
int launch_ke_vjp_k7(const OpArgs& a, const Tables1D& t, double* Ub, bool gen, hipStream_t st);

// y <- v (n doubles), a kernel rather than a memset so that it may be captured in graphs.
int launch_fill(double* y, int64_t n, double v, hipStream_t st);

// Channel perturbation at the nodes: u_a += amp * u1_lam(x2) * noise_a, T kept.
int launch_channel_perturb(double* U, const double* node_x, const double* noise, int64_t ncell, int n3,
                           double umax, double power, double amp, double gamma, double R, hipStream_t st);

}  // namespace dgns
