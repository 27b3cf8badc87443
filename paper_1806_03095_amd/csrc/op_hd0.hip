// The streamed kernels of hd_impl.h at two lower (degree, n_q) pairs where they measured
// faster than the resident ones in float64 without a body force: k = 6, n_q = 10
// (1686 -> 1600 us at 18^3) and k = 7, n_q = 11 (1839 -> 1532 us at 16^3).
#include "hd_impl.h"

namespace dgns {

template <int N, int Q>
static int op_hd(const OpArgs& a, bool gen, hipStream_t st) {
    return gen ? launch_op_hd_t<N, Q, double, true>(a, st) : launch_op_hd_t<N, Q, double, false>(a, st);
}

bool streamed_possible(int k, int q, bool fp32) {
    return k >= 8 || (!fp32 && ((k == 6 && q == 10) || (k == 7 && q == 11)));
}

bool streamed_preferred(int k, int q, bool fp32, const double force[3]) {
    return !fp32 && force[0] == 0 && force[1] == 0 && force[2] == 0 && ((k == 6 && q == 10) || (k == 7 && q == 11));
}

int launch_operator_hd0(const OpArgs& a, int k, int q, bool fp32, bool gen, hipStream_t st) {
    if (fp32) return 1;
    if (k == 6 && q == 10) return op_hd<7, 10>(a, gen, st);
    if (k == 7 && q == 11) return op_hd<8, 11>(a, gen, st);
    return 1;
}

}  // namespace dgns
