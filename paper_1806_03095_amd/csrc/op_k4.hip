// Operator (and adjoint) kernels of polynomial degree 4: the supported n_q values.
#include "adj_impl.h"
#include "diag_impl.h"
#include "minv_impl.h"
#include "dg_kernels.h"

namespace dgns {

int launch_operator_k4(const OpArgs& a, const Tables1D& t, bool fp32, bool gen, hipStream_t st) {
    switch (t.q) {
        case 5: return fp32 ? (gen ? launch_op_t<5, 5, float, true>(a, t, st) : launch_op_t<5, 5, float, false>(a, t, st))
                       : (gen ? launch_op_t<5, 5, double, true>(a, t, st) : launch_op_t<5, 5, double, false>(a, t, st));
        case 6: return fp32 ? (gen ? launch_op_t<5, 6, float, true>(a, t, st) : launch_op_t<5, 6, float, false>(a, t, st))
                       : (gen ? launch_op_t<5, 6, double, true>(a, t, st) : launch_op_t<5, 6, double, false>(a, t, st));
        case 7: return fp32 ? (gen ? launch_op_t<5, 7, float, true>(a, t, st) : launch_op_t<5, 7, float, false>(a, t, st))
                       : (gen ? launch_op_t<5, 7, double, true>(a, t, st) : launch_op_t<5, 7, double, false>(a, t, st));
        case 9: return fp32 ? (gen ? launch_op_t<5, 9, float, true>(a, t, st) : launch_op_t<5, 9, float, false>(a, t, st))
                       : (gen ? launch_op_t<5, 9, double, true>(a, t, st) : launch_op_t<5, 9, double, false>(a, t, st));
        default: return 1;
    }
}

int launch_inverse_mass_k4(const double* R, double* L, int64_t ncell, const double* cm, const double* mj,
                            const Tables1D& t, bool fp32, bool gen, hipStream_t st) {
    return fp32 ? (gen ? launch_minv_t<5, float, true>(R, L, ncell, cm, mj, t, st)
                       : launch_minv_t<5, float, false>(R, L, ncell, cm, mj, t, st))
                : (gen ? launch_minv_t<5, double, true>(R, L, ncell, cm, mj, t, st)
                       : launch_minv_t<5, double, false>(R, L, ncell, cm, mj, t, st));
}

int launch_adjoint_k4(const OpArgs& a, const double* Rb, const Tables1D& t, bool gen, hipStream_t st) {
    switch (t.q) {
        case 5: return gen ? launch_adjoint_t<5, 5, true>(a, Rb, t, st) : launch_adjoint_t<5, 5, false>(a, Rb, t, st);
        case 6: return gen ? launch_adjoint_t<5, 6, true>(a, Rb, t, st) : launch_adjoint_t<5, 6, false>(a, Rb, t, st);
        case 7: return gen ? launch_adjoint_t<5, 7, true>(a, Rb, t, st) : launch_adjoint_t<5, 7, false>(a, Rb, t, st);
        case 9: return gen ? launch_adjoint_t<5, 9, true>(a, Rb, t, st) : launch_adjoint_t<5, 9, false>(a, Rb, t, st);
        default: return 1;
    }
}

int launch_diagnostics_k4(const OpArgs& a, const Tables1D& t, const double* L, double* partial, bool gen, hipStream_t st) {
    switch (t.q) {
        case 5: return gen ? launch_diag_t<5, 5, true>(a, t, L, partial, st) : launch_diag_t<5, 5, false>(a, t, L, partial, st);
        case 6: return gen ? launch_diag_t<5, 6, true>(a, t, L, partial, st) : launch_diag_t<5, 6, false>(a, t, L, partial, st);
        case 7: return gen ? launch_diag_t<5, 7, true>(a, t, L, partial, st) : launch_diag_t<5, 7, false>(a, t, L, partial, st);
        case 9: return gen ? launch_diag_t<5, 9, true>(a, t, L, partial, st) : launch_diag_t<5, 9, false>(a, t, L, partial, st);
        default: return 1;
    }
}

int launch_chan_stats_k4(const OpArgs& a, const Tables1D& t, double* partial, bool gen, hipStream_t st) {
    switch (t.q) {
        case 5: return gen ? launch_chan_stats_t<5, 5, true>(a, t, partial, st) : launch_chan_stats_t<5, 5, false>(a, t, partial, st);
        case 6: return gen ? launch_chan_stats_t<5, 6, true>(a, t, partial, st) : launch_chan_stats_t<5, 6, false>(a, t, partial, st);
        case 7: return gen ? launch_chan_stats_t<5, 7, true>(a, t, partial, st) : launch_chan_stats_t<5, 7, false>(a, t, partial, st);
        case 9: return gen ? launch_chan_stats_t<5, 9, true>(a, t, partial, st) : launch_chan_stats_t<5, 9, false>(a, t, partial, st);
        default: return 1;
    }
}

int launch_wall_shear_k4(const OpArgs& a, const Tables1D& t, double* partial, bool gen, hipStream_t st) {
    switch (t.q) {
        case 5: return gen ? launch_wall_shear_t<5, 5, true>(a, t, partial, st) : launch_wall_shear_t<5, 5, false>(a, t, partial, st);
        case 6: return gen ? launch_wall_shear_t<5, 6, true>(a, t, partial, st) : launch_wall_shear_t<5, 6, false>(a, t, partial, st);
        case 7: return gen ? launch_wall_shear_t<5, 7, true>(a, t, partial, st) : launch_wall_shear_t<5, 7, false>(a, t, partial, st);
        case 9: return gen ? launch_wall_shear_t<5, 9, true>(a, t, partial, st) : launch_wall_shear_t<5, 9, false>(a, t, partial, st);
        default: return 1;
    }
}

int launch_ke_vjp_k4(const OpArgs& a, const Tables1D& t, double* Ub, bool gen, hipStream_t st) {
    switch (t.q) {
        case 5: return gen ? launch_ke_vjp_t<5, 5, true>(a, t, Ub, st) : launch_ke_vjp_t<5, 5, false>(a, t, Ub, st);
        case 6: return gen ? launch_ke_vjp_t<5, 6, true>(a, t, Ub, st) : launch_ke_vjp_t<5, 6, false>(a, t, Ub, st);
        case 7: return gen ? launch_ke_vjp_t<5, 7, true>(a, t, Ub, st) : launch_ke_vjp_t<5, 7, false>(a, t, Ub, st);
        case 9: return gen ? launch_ke_vjp_t<5, 9, true>(a, t, Ub, st) : launch_ke_vjp_t<5, 9, false>(a, t, Ub, st);
        default: return 1;
    }
}

}  // namespace dgns
