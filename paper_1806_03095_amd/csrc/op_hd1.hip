// High-degree operator kernels (hd_impl.h), degrees 8..11.
#include "diag_impl.h"
#include "hd_impl.h"

namespace dgns {

template <int N, int Q>
static int op_hd(const OpArgs& a, bool fp32, bool gen, hipStream_t st) {
    return fp32 ? (gen ? launch_op_hd_t<N, Q, float, true>(a, st) : launch_op_hd_t<N, Q, float, false>(a, st))
                : (gen ? launch_op_hd_t<N, Q, double, true>(a, st) : launch_op_hd_t<N, Q, double, false>(a, st));
}

template <int N, int Q>
static int diag_hd(const OpArgs& a, const double* L, double* partial, bool gen, hipStream_t st) {
    return gen ? launch_diag_hd_t<N, Q, true>(a, L, partial, st) : launch_diag_hd_t<N, Q, false>(a, L, partial, st);
}

template <int N>
static int minv_hd(const double* R, double* L, int64_t ncell, const double* cm, const double* mj, const Tables1D* t,
                   bool fp32, bool gen, hipStream_t st) {
    return fp32 ? (gen ? launch_minv_hd_t<N, float, true>(R, L, ncell, cm, mj, t, st)
                       : launch_minv_hd_t<N, float, false>(R, L, ncell, cm, mj, t, st))
                : (gen ? launch_minv_hd_t<N, double, true>(R, L, ncell, cm, mj, t, st)
                       : launch_minv_hd_t<N, double, false>(R, L, ncell, cm, mj, t, st));
}

int launch_operator_hd1(const OpArgs& a, int k, int q, bool fp32, bool gen, hipStream_t st) {
    if (k == 8 && q == 9) return op_hd<9, 9>(a, fp32, gen, st);
    if (k == 8 && q == 13) return op_hd<9, 13>(a, fp32, gen, st);
    if (k == 9 && q == 10) return op_hd<10, 10>(a, fp32, gen, st);
    if (k == 9 && q == 14) return op_hd<10, 14>(a, fp32, gen, st);
    if (k == 10 && q == 11) return op_hd<11, 11>(a, fp32, gen, st);
    if (k == 10 && q == 16) return op_hd<11, 16>(a, fp32, gen, st);
    if (k == 11 && q == 12) return op_hd<12, 12>(a, fp32, gen, st);
    return 1;
}

int launch_inverse_mass_hd1(const double* R, double* L, int64_t ncell, const double* cm, const double* mj,
                            const Tables1D* t, int k, bool fp32, bool gen, hipStream_t st) {
    switch (k) {
        case 8: return minv_hd<9>(R, L, ncell, cm, mj, t, fp32, gen, st);
        case 9: return minv_hd<10>(R, L, ncell, cm, mj, t, fp32, gen, st);
        case 10: return minv_hd<11>(R, L, ncell, cm, mj, t, fp32, gen, st);
        case 11: return minv_hd<12>(R, L, ncell, cm, mj, t, fp32, gen, st);
        default: return 1;
    }
}

int launch_diagnostics_hd1(const OpArgs& a, int k, int q, const double* L, double* partial, bool gen,
                          hipStream_t st) {
    if (k == 8 && q == 9) return diag_hd<9, 9>(a, L, partial, gen, st);
    if (k == 8 && q == 13) return diag_hd<9, 13>(a, L, partial, gen, st);
    if (k == 9 && q == 10) return diag_hd<10, 10>(a, L, partial, gen, st);
    if (k == 9 && q == 14) return diag_hd<10, 14>(a, L, partial, gen, st);
    if (k == 10 && q == 11) return diag_hd<11, 11>(a, L, partial, gen, st);
    if (k == 10 && q == 16) return diag_hd<11, 16>(a, L, partial, gen, st);
    if (k == 11 && q == 12) return diag_hd<12, 12>(a, L, partial, gen, st);
    return 1;
}

}  // namespace dgns
