// Operator (and adjoint) kernels of polynomial degree 6: the supported n_q values.
#include "op_impl.h"
#include "diag_impl.h"
#include "minv_impl.h"
#include "dg_kernels.h"

namespace dgns {

int launch_operator_k6(const OpArgs& a, const Tables1D& t, bool fp32, bool gen, hipStream_t st) {
    switch (t.q) {
        case 7: return fp32 ? (gen ? launch_op_t<7, 7, float, true>(a, t, st) : launch_op_t<7, 7, float, false>(a, t, st))
                       : (gen ? launch_op_t<7, 7, double, true>(a, t, st) : launch_op_t<7, 7, double, false>(a, t, st));
        case 10: return fp32 ? (gen ? launch_op_t<7, 10, float, true>(a, t, st) : launch_op_t<7, 10, float, false>(a, t, st))
                       : (gen ? launch_op_t<7, 10, double, true>(a, t, st) : launch_op_t<7, 10, double, false>(a, t, st));
        default: return 1;
    }
}

int launch_inverse_mass_k6(const double* R, double* L, int64_t ncell, const double* cm, const double* mj,
                            const Tables1D& t, bool fp32, bool gen, hipStream_t st) {
    return fp32 ? (gen ? launch_minv_t<7, float, true>(R, L, ncell, cm, mj, t, st)
                       : launch_minv_t<7, float, false>(R, L, ncell, cm, mj, t, st))
                : (gen ? launch_minv_t<7, double, true>(R, L, ncell, cm, mj, t, st)
                       : launch_minv_t<7, double, false>(R, L, ncell, cm, mj, t, st));
}

// The adjoint's LDS work area exceeds one workgroup's 160 KB at this degree.
int launch_adjoint_k6(const OpArgs&, const double*, const Tables1D&, bool, hipStream_t) { return 1; }

int launch_diagnostics_k6(const OpArgs& a, const Tables1D& t, const double* L, double* partial, bool gen, hipStream_t st) {
    switch (t.q) {
        case 7: return gen ? launch_diag_t<7, 7, true>(a, t, L, partial, st) : launch_diag_t<7, 7, false>(a, t, L, partial, st);
        case 10: return gen ? launch_diag_t<7, 10, true>(a, t, L, partial, st) : launch_diag_t<7, 10, false>(a, t, L, partial, st);
        default: return 1;
    }
}

int launch_chan_stats_k6(const OpArgs& a, const Tables1D& t, double* partial, bool gen, hipStream_t st) {
    switch (t.q) {
        case 7: return gen ? launch_chan_stats_t<7, 7, true>(a, t, partial, st) : launch_chan_stats_t<7, 7, false>(a, t, partial, st);
        case 10: return gen ? launch_chan_stats_t<7, 10, true>(a, t, partial, st) : launch_chan_stats_t<7, 10, false>(a, t, partial, st);
        default: return 1;
    }
}

int launch_wall_shear_k6(const OpArgs& a, const Tables1D& t, double* partial, bool gen, hipStream_t st) {
    switch (t.q) {
        case 7: return gen ? launch_wall_shear_t<7, 7, true>(a, t, partial, st) : launch_wall_shear_t<7, 7, false>(a, t, partial, st);
        case 10: return gen ? launch_wall_shear_t<7, 10, true>(a, t, partial, st) : launch_wall_shear_t<7, 10, false>(a, t, partial, st);
        default: return 1;
    }
}

int launch_ke_vjp_k6(const OpArgs& a, const Tables1D& t, double* Ub, bool gen, hipStream_t st) {
    switch (t.q) {
        case 7: return gen ? launch_ke_vjp_t<7, 7, true>(a, t, Ub, st) : launch_ke_vjp_t<7, 7, false>(a, t, Ub, st);
        case 10: return gen ? launch_ke_vjp_t<7, 10, true>(a, t, Ub, st) : launch_ke_vjp_t<7, 10, false>(a, t, Ub, st);
        default: return 1;
    }
}

}  // namespace dgns
