// Operator (and adjoint) kernels of polynomial degree 7: the supported n_q values.
#include "op_impl.h"
#include "diag_impl.h"
#include "minv_impl.h"
#include "dg_kernels.h"

namespace dgns {

int launch_operator_k7(const OpArgs& a, const Tables1D& t, bool fp32, bool gen, hipStream_t st) {
    switch (t.q) {
        case 8: return fp32 ? (gen ? launch_op_t<8, 8, float, true>(a, t, st) : launch_op_t<8, 8, float, false>(a, t, st))
                       : (gen ? launch_op_t<8, 8, double, true>(a, t, st) : launch_op_t<8, 8, double, false>(a, t, st));
        case 11: return fp32 ? (gen ? launch_op_t<8, 11, float, true>(a, t, st) : launch_op_t<8, 11, float, false>(a, t, st))
                       : (gen ? launch_op_t<8, 11, double, true>(a, t, st) : launch_op_t<8, 11, double, false>(a, t, st));
        default: return 1;
    }
}

int launch_inverse_mass_k7(const double* R, double* L, int64_t ncell, const double* cm, const double* mj,
                            const Tables1D& t, bool fp32, bool gen, hipStream_t st) {
    return fp32 ? (gen ? launch_minv_t<8, float, true>(R, L, ncell, cm, mj, t, st)
                       : launch_minv_t<8, float, false>(R, L, ncell, cm, mj, t, st))
                : (gen ? launch_minv_t<8, double, true>(R, L, ncell, cm, mj, t, st)
                       : launch_minv_t<8, double, false>(R, L, ncell, cm, mj, t, st));
}

// The adjoint's LDS work area exceeds one workgroup's 160 KB at this degree.
int launch_adjoint_k7(const OpArgs&, const double*, const Tables1D&, bool, hipStream_t) { return 1; }

int launch_diagnostics_k7(const OpArgs& a, const Tables1D& t, const double* L, double* partial, bool gen, hipStream_t st) {
    switch (t.q) {
        case 8: return gen ? launch_diag_t<8, 8, true>(a, t, L, partial, st) : launch_diag_t<8, 8, false>(a, t, L, partial, st);
        case 11: return gen ? launch_diag_t<8, 11, true>(a, t, L, partial, st) : launch_diag_t<8, 11, false>(a, t, L, partial, st);
        default: return 1;
    }
}

int launch_chan_stats_k7(const OpArgs& a, const Tables1D& t, double* partial, bool gen, hipStream_t st) {
    switch (t.q) {
        case 8: return gen ? launch_chan_stats_t<8, 8, true>(a, t, partial, st) : launch_chan_stats_t<8, 8, false>(a, t, partial, st);
        case 11: return gen ? launch_chan_stats_t<8, 11, true>(a, t, partial, st) : launch_chan_stats_t<8, 11, false>(a, t, partial, st);
        default: return 1;
    }
}

int launch_wall_shear_k7(const OpArgs& a, const Tables1D& t, double* partial, bool gen, hipStream_t st) {
    switch (t.q) {
        case 8: return gen ? launch_wall_shear_t<8, 8, true>(a, t, partial, st) : launch_wall_shear_t<8, 8, false>(a, t, partial, st);
        case 11: return gen ? launch_wall_shear_t<8, 11, true>(a, t, partial, st) : launch_wall_shear_t<8, 11, false>(a, t, partial, st);
        default: return 1;
    }
}

int launch_ke_vjp_k7(const OpArgs& a, const Tables1D& t, double* Ub, bool gen, hipStream_t st) {
    switch (t.q) {
        case 8: return gen ? launch_ke_vjp_t<8, 8, true>(a, t, Ub, st) : launch_ke_vjp_t<8, 8, false>(a, t, Ub, st);
        case 11: return gen ? launch_ke_vjp_t<8, 11, true>(a, t, Ub, st) : launch_ke_vjp_t<8, 11, false>(a, t, Ub, st);
        default: return 1;
    }
}

}  // namespace dgns
