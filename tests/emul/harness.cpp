// CPU harness around the operator kernel templates (test infrastructure only).
// Compiled with g++ (and AddressSanitizer) against tests/emul/hip/hip_runtime.h;
// see that file for how a workgroup is emulated.
//
// usage: harness <in.bin> <out.bin>
//   in.bin : dgns_params, dgns_box_mesh, uint32 terms, int32 mode, then U (n_dof float64)
//            and, for mode 2, Rbar (n_dof float64)
//   mode   : 0 residual R, 1 operator L = M^{-1} R, 2 residual adjoint Ubar = (dR/dU)^T Rbar,
//            3 standalone inverse mass M^{-1} U, 4 channel-statistics partial sums,
//            5 wall-shear partial sums
//   out.bin: R, L, Ubar or M^{-1} U (n_dof float64); mode 4: n_cells * n_q * 9 float64;
//            mode 5: 2 n0 n2 * 3 float64 (lower-wall cells, then upper)
#include <cstdio>
#include <string>
#include <vector>

#include "adj_impl.h"
#include "diag_impl.h"
#include "hd_impl.h"
#include "minv_impl.h"
#include "setup.h"

using namespace dgns;

// The high-degree launcher's fused Runge-Kutta stage calls the stand-alone update (in
// aux_kernels.hip, not part of this harness); the harness never runs a stage.
int dgns::launch_rk_update_to(const double*, double*, double*, const double*, int64_t, double, double, double,
                              hipStream_t) {
    return -1;
}

namespace {

template <int N, int Q>
int run_adj(const OpArgs& a, const double* Rb, const Tables1D& t, int gen) {
    if constexpr (N <= 6) return gen ? launch_adjoint_t<N, Q, true>(a, Rb, t, nullptr) : launch_adjoint_t<N, Q, false>(a, Rb, t, nullptr);
    return -4;
}

template <int N, int Q>
int run(const OpArgs& a, const Tables1D& t, int fp32, int gen) {
    if (fp32) return gen ? launch_op_t<N, Q, float, true>(a, t, nullptr) : launch_op_t<N, Q, float, false>(a, t, nullptr);
    return gen ? launch_op_t<N, Q, double, true>(a, t, nullptr) : launch_op_t<N, Q, double, false>(a, t, nullptr);
}

template <int N, int Q>
int run_hd(const OpArgs& a, int fp32, int gen) {
    if (fp32) return gen ? launch_op_hd_t<N, Q, float, true>(a, nullptr) : launch_op_hd_t<N, Q, float, false>(a, nullptr);
    return gen ? launch_op_hd_t<N, Q, double, true>(a, nullptr) : launch_op_hd_t<N, Q, double, false>(a, nullptr);
}

template <int N>
int run_minv_hd(const OpArgs& a, int fp32, int gen) {
    if (fp32)
        return gen ? launch_minv_hd_t<N, float, true>(a.U, a.out, a.ncell, a.cell_metric, a.mass_jxw, a.tab_dev, nullptr)
                   : launch_minv_hd_t<N, float, false>(a.U, a.out, a.ncell, a.cell_metric, a.mass_jxw, a.tab_dev, nullptr);
    return gen ? launch_minv_hd_t<N, double, true>(a.U, a.out, a.ncell, a.cell_metric, a.mass_jxw, a.tab_dev, nullptr)
               : launch_minv_hd_t<N, double, false>(a.U, a.out, a.ncell, a.cell_metric, a.mass_jxw, a.tab_dev, nullptr);
}

template <int N, int Q>
int run_diag_hd(const OpArgs& a, const double* L, int gen) {
    return gen ? launch_diag_hd_t<N, Q, true>(a, L, a.out, nullptr) : launch_diag_hd_t<N, Q, false>(a, L, a.out, nullptr);
}

template <int N, int Q>
int run_stats(const OpArgs& a, const Tables1D& t, int gen) {
    return gen ? launch_chan_stats_t<N, Q, true>(a, t, a.out, nullptr) : launch_chan_stats_t<N, Q, false>(a, t, a.out, nullptr);
}

template <int N, int Q>
int run_wall(const OpArgs& a, const Tables1D& t, int gen) {
    return gen ? launch_wall_shear_t<N, Q, true>(a, t, a.out, nullptr) : launch_wall_shear_t<N, Q, false>(a, t, a.out, nullptr);
}

template <int N>
int run_minv(const OpArgs& a, const Tables1D& t, int fp32, int gen) {
    const double* R = a.U;
    double* L = a.out;
    if (fp32)
        return gen ? launch_minv_t<N, float, true>(R, L, a.ncell, a.cell_metric, a.mass_jxw, t, nullptr)
                   : launch_minv_t<N, float, false>(R, L, a.ncell, a.cell_metric, a.mass_jxw, t, nullptr);
    return gen ? launch_minv_t<N, double, true>(R, L, a.ncell, a.cell_metric, a.mass_jxw, t, nullptr)
               : launch_minv_t<N, double, false>(R, L, a.ncell, a.cell_metric, a.mass_jxw, t, nullptr);
}

}  // namespace

int main(int argc, char** argv) {
    if (argc != 3) return 2;
    FILE* f = std::fopen(argv[1], "rb");
    if (!f) return 3;
    dgns_params prm;
    dgns_box_mesh msh;
    uint32_t terms;
    int32_t fuse;
    if (std::fread(&prm, sizeof prm, 1, f) != 1 || std::fread(&msh, sizeof msh, 1, f) != 1 ||
        std::fread(&terms, 4, 1, f) != 1 || std::fread(&fuse, 4, 1, f) != 1)
        return 4;
    HostSetup hs;
    std::string e;
    int rc = build_setup(prm, msh, hs, e);
    if (rc) {
        std::fprintf(stderr, "setup: %s\n", e.c_str());
        return 5;
    }
    const int64_t ndof = 5 * hs.ncell * hs.n3;
    const int64_t nout = fuse == 4 ? hs.ncell * prm.n_q * kStats
                                   : (fuse == 5 ? (int64_t)2 * msh.n[0] * msh.n[2] * kWallSums
                                                : (fuse == 6 ? hs.ncell * kDiagSums : ndof));
    std::vector<double> U(ndof), out(nout, -12345.0), Rb;
    // face buffer of the split evaluation: six lifted blocks [2][5][N^2] per cell (sized
    // for float64, enough for float32), followed by the streamed cell kernel's scratch
    // [n_q][2][5][N^2] per cell as the library sizes it where those kernels can run (here
    // always, so that any case may run them); filled with a value that would show if read
    // unwritten
    const int64_t nfw_hd = (int64_t)hs.ncell * 10 * prm.n_q * (prm.degree + 1) * (prm.degree + 1);
    std::vector<double> fw(hs.ncell * 6 * 10 * (prm.degree + 1) * (prm.degree + 1) + nfw_hd, 1e300);
    if ((int64_t)std::fread(U.data(), 8, ndof, f) != ndof) return 6;
    if (fuse == 2 || fuse == 6) {
        Rb.resize(ndof);
        if ((int64_t)std::fread(Rb.data(), 8, ndof, f) != ndof) return 6;
    }
    std::fclose(f);
    OpArgs a;
    std::memset(&a, 0, sizeof a);
    a.U = U.data();
    a.out = out.data();
    a.ncell = hs.ncell;
    for (int d = 0; d < 3; ++d) {
        a.n[d] = msh.n[d];
        a.periodic[d] = msh.periodic[d] ? 1 : 0;
        a.face_data[d] = hs.face[d].empty() ? nullptr : hs.face[d].data();
        a.tau_face[d] = hs.tau[d].data();
        a.force[d] = prm.body_force[d];
    }
    a.cell_metric = hs.metric.data();
    a.mass_jxw = hs.mass_jxw.empty() ? nullptr : hs.mass_jxw.data();
    a.gamma = prm.gamma;
    a.R = prm.R;
    a.mu = prm.mu;
    a.lam = prm.lambda;
    a.wall_T = prm.wall_T;
    a.terms = terms;
    a.fuse_minv = fuse == 1 ? 1 : 0;
    a.fw = fw.data();
    a.tab_dev = &hs.tab;
    const int k = prm.degree, q = prm.n_q, fp32 = prm.precision, gen = hs.gen ? 1 : 0;
    rc = -4;
#define EMU_CASE(K, Q_) \
    if (k == K && q == Q_)                                                                                   \
        rc = fuse == 2 ? run_adj<K + 1, Q_>(a, Rb.data(), hs.tab, gen)                                        \
                       : (fuse == 3 ? run_minv<K + 1>(a, hs.tab, fp32, gen)                                  \
                                    : (fuse == 4 ? run_stats<K + 1, Q_>(a, hs.tab, gen)                   \
                                                 : (fuse == 5 ? run_wall<K + 1, Q_>(a, hs.tab, gen)          \
                                                              : run<K + 1, Q_>(a, hs.tab, fp32, gen))));
    EMU_CASES
#ifdef EMU_HD_CASES
    // degrees >= 8: modes 0 (residual), 1 (operator), 3 (stand-alone inverse mass) and 6
    // (diagnostics partial sums [n_cells][9] of U with the second input as L)
#define EMU_HD_CASE(K, Q_) \
    if (k == K && q == Q_)  \
        rc = fuse == 3 ? run_minv_hd<K + 1>(a, fp32, gen)                                               \
                       : (fuse == 6 ? run_diag_hd<K + 1, Q_>(a, Rb.data(), gen)                         \
                                    : (fuse <= 1 ? run_hd<K + 1, Q_>(a, fp32, gen) : -4));
    EMU_HD_CASES
#endif
    if (rc != 0) {
        std::fprintf(stderr, "no emulated kernel for k=%d nq=%d\n", k, q);
        return 7;
    }
    f = std::fopen(argv[2], "wb");
    std::fwrite(out.data(), 8, nout, f);
    std::fclose(f);
    return 0;
}
