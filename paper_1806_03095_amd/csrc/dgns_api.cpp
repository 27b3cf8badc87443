// Host side of the library: the C ABI of include/dgns.h, context lifetime, the
// 1D rules and bases, mesh and geometry setup, and kernel launches.
//
// Geometry (paper Sec. 2.2.1, 2.2.3 eq. IntegralsReferenceSpace): each cell is the
// image of [0,1]^3 under the degree-k interpolant of the box map at its LGL
// points; J = dx/dxi, and the metric terms J^{-1}, |det J| w at every quadrature
// point, the face normal and |det J| |J^{-T} n_xi| w at every face point.
// Penalty (eq. TauIP_Element): tau_e = nu (k+1)^2 (A_interior/2 + A_boundary)/V_e,
// interior faces take the max over both cells.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "dg_common.h"
#include "dg_kernels.h"
#include "dgns.h"
#include "setup.h"

using namespace dgns;

namespace {

thread_local std::string g_err = "no error";

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                              \
    do {                                                                                           \
        hipError_t _e = (expr);                                                                    \
        if (_e != hipSuccess) return fail(DGNS_EHIP, "%s: %s", #expr, hipGetErrorString(_e));      \
    } while (0)

}  // namespace

// ---------------------------------------------------------------- context
constexpr int kMaxRkStages = 16;
constexpr int kWallSumsHost = 3;   // per wall cell: dA w (mu du_1/dn, rho, 1)

struct dgns_ctx {
    dgns_params prm;
    dgns_box_mesh msh;
    hipStream_t stream = nullptr;
    bool gen = false;   // per-point metric (curved / stretched meshes)
    bool fp32 = false;
    int k = 0, n = 0, q = 0;
    int64_t ncell = 0, n3 = 0, ndof = 0;
    double h_min = 0;
    Tables1D tab;
    std::vector<double> geo;      // [E][3][N3] geometry nodes (LGL)
    std::vector<double> node_x;   // [3][E][N3] coordinates of the basis nodes
    double* d_metric = nullptr;
    double* d_face[3] = {nullptr, nullptr, nullptr};
    double* d_tau[3] = {nullptr, nullptr, nullptr};
    double* d_mass_jxw = nullptr;
    double* d_partial = nullptr;
    double* d_total = nullptr;
    Tables1D* d_tab = nullptr;
    double* d_scratch = nullptr;   // n_dof doubles, allocated on the first operator VJP
    double* d_stats = nullptr;     // channel statistics partial sums and totals, on first use
    double* d_wall = nullptr;      // wall-shear partial sums, on first use
    // running sums of the time-averaged channel statistics (dgns_channel_stats_*)
    int64_t stats_samples = 0;
    std::vector<double> stats_sum;  // n[1] * n_q rows of [y, rho, u, v, w, uu, vv, ww, uv]
    double tau_sum = 0, rho_w_sum = 0;
    double* noalloc = nullptr;     // this device's copy of the static workspace below
    double* d_fw = nullptr;        // face buffer of the split evaluation (six lifted blocks per cell)
    // 2N-storage Runge-Kutta scheme of dgns_rk_step (Williamson form), default below
    int rk_s = 0;
    double rk_A[kMaxRkStages], rk_B[kMaxRkStages], rk_c[kMaxRkStages];
};

// Workspace of dgns_diagnostics_noalloc: the per-cell partial sums and their totals
// live in this file-scope device array instead of memory the library allocates, so that
// the entry point never allocates.  Every GPU the library runs on holds its own copy
// until the process ends; host code must use the address hipGetSymbolAddress returns for
// the current device (kept per device below), never the array's name.
constexpr int64_t kNoAllocMaxCells = 262144;                      // 64^3 cells
constexpr int64_t kNoAllocDoubles = 9 * kNoAllocMaxCells + 16;    // partials + totals (18.9 MB)
static __device__ __align__(256) double scratch[kNoAllocDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
double* g_noalloc_ptr[kMaxDevices] = {};

// Address of this device's copy of the workspace, looked up once per device.
int noalloc_workspace(double** out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(DGNS_EUNSUPPORTED, "device index %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void* p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_noalloc_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_noalloc_ptr[dev];
    return 0;
}

template <typename T>
int upload(const std::vector<T>& h, T** d) {
    HIP_TRY(hipMalloc((void**)d, sizeof(T) * std::max<size_t>(1, h.size())));
    if (!h.empty()) HIP_TRY(hipMemcpy(*d, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice));
    return 0;
}

void free_ctx(dgns_ctx* c) {
    hipFree(c->d_metric);
    for (int d = 0; d < 3; ++d) {
        hipFree(c->d_face[d]);
        hipFree(c->d_tau[d]);
    }
    hipFree(c->d_mass_jxw);
    hipFree(c->d_partial);
    hipFree(c->d_total);
    hipFree(c->d_tab);
    hipFree(c->d_scratch);
    hipFree(c->d_stats);
    hipFree(c->d_wall);
    hipFree(c->d_fw);
}

OpArgs make_args(const dgns_ctx* c, const double* U, double* out, unsigned terms, int fuse) {
    OpArgs a;
    std::memset(&a, 0, sizeof a);
    a.U = U;
    a.out = out;
    a.ncell = c->ncell;
    for (int d = 0; d < 3; ++d) {
        a.n[d] = c->msh.n[d];
        a.periodic[d] = c->msh.periodic[d] ? 1 : 0;
        a.face_data[d] = c->d_face[d];
        a.tau_face[d] = c->d_tau[d];
        a.force[d] = c->prm.body_force[d];
    }
    a.cell_metric = c->d_metric;
    a.mass_jxw = c->d_mass_jxw;
    a.gamma = c->prm.gamma;
    a.R = c->prm.R;
    a.mu = c->prm.mu;
    a.lam = c->prm.lambda;
    a.wall_T = c->prm.wall_T;
    a.terms = terms;
    a.fuse_minv = fuse;
    a.fw = c->d_fw;
    a.tab_dev = c->d_tab;
    return a;
}

int dispatch_operator(const dgns_ctx* c, const OpArgs& a) {
    int rc = 1;
    if (streamed_preferred(c->k, c->q, c->fp32, c->prm.body_force)) {
        rc = launch_operator_hd0(a, c->k, c->q, c->fp32, c->gen, c->stream);
        if (rc != 0) return fail(DGNS_EHIP, "operator launch failed: %s", hipGetErrorString(hipGetLastError()));
        return 0;
    }
    switch (c->k) {
        case 1: rc = launch_operator_k1(a, c->tab, c->fp32, c->gen, c->stream); break;
        case 2: rc = launch_operator_k2(a, c->tab, c->fp32, c->gen, c->stream); break;
        case 3: rc = launch_operator_k3(a, c->tab, c->fp32, c->gen, c->stream); break;
        case 4: rc = launch_operator_k4(a, c->tab, c->fp32, c->gen, c->stream); break;
        case 5: rc = launch_operator_k5(a, c->tab, c->fp32, c->gen, c->stream); break;
        case 6: rc = launch_operator_k6(a, c->tab, c->fp32, c->gen, c->stream); break;
        case 7: rc = launch_operator_k7(a, c->tab, c->fp32, c->gen, c->stream); break;
        case 8: case 9: case 10: case 11: rc = launch_operator_hd1(a, c->k, c->q, c->fp32, c->gen, c->stream); break;
        case 12: case 13: case 14: case 15: rc = launch_operator_hd2(a, c->k, c->q, c->fp32, c->gen, c->stream); break;
    }
    if (rc == 1) return fail(DGNS_EUNSUPPORTED, "no operator kernel for degree %d, n_q %d", c->k, c->q);
    if (rc != 0) return fail(DGNS_EHIP, "operator launch failed: %s", hipGetErrorString(hipGetLastError()));
    return 0;
}

int dispatch_minv(const dgns_ctx* c, const double* R, double* L) {
    int rc = 1;
    const double* cm = c->d_metric;
    const double* mj = c->d_mass_jxw;
    switch (c->k) {
        case 1: rc = launch_inverse_mass_k1(R, L, c->ncell, cm, mj, c->tab, c->fp32, c->gen, c->stream); break;
        case 2: rc = launch_inverse_mass_k2(R, L, c->ncell, cm, mj, c->tab, c->fp32, c->gen, c->stream); break;
        case 3: rc = launch_inverse_mass_k3(R, L, c->ncell, cm, mj, c->tab, c->fp32, c->gen, c->stream); break;
        case 4: rc = launch_inverse_mass_k4(R, L, c->ncell, cm, mj, c->tab, c->fp32, c->gen, c->stream); break;
        case 5: rc = launch_inverse_mass_k5(R, L, c->ncell, cm, mj, c->tab, c->fp32, c->gen, c->stream); break;
        case 6: rc = launch_inverse_mass_k6(R, L, c->ncell, cm, mj, c->tab, c->fp32, c->gen, c->stream); break;
        case 7: rc = launch_inverse_mass_k7(R, L, c->ncell, cm, mj, c->tab, c->fp32, c->gen, c->stream); break;
        case 8: case 9: case 10: case 11:
            rc = launch_inverse_mass_hd1(R, L, c->ncell, cm, mj, c->d_tab, c->k, c->fp32, c->gen, c->stream);
            break;
        case 12: case 13: case 14: case 15:
            rc = launch_inverse_mass_hd2(R, L, c->ncell, cm, mj, c->d_tab, c->k, c->fp32, c->gen, c->stream);
            break;
    }
    if (rc == 1) return fail(DGNS_EUNSUPPORTED, "no inverse-mass kernel for degree %d", c->k);
    if (rc != 0) return fail(DGNS_EHIP, "inverse-mass launch failed: %s", hipGetErrorString(hipGetLastError()));
    return 0;
}

// Per-cell diagnostic partial sums into partial (9 n_cells doubles), then their totals
// into total (9 doubles); by default the context's buffers.
int dispatch_diagnostics(const dgns_ctx* c, const OpArgs& a, const double* L, double* partial = nullptr,
                         double* total = nullptr) {
    if (!partial) partial = c->d_partial;
    if (!total) total = c->d_total;
    int rc = 1;
    switch (c->k) {
        case 1: rc = launch_diagnostics_k1(a, c->tab, L, partial, c->gen, c->stream); break;
        case 2: rc = launch_diagnostics_k2(a, c->tab, L, partial, c->gen, c->stream); break;
        case 3: rc = launch_diagnostics_k3(a, c->tab, L, partial, c->gen, c->stream); break;
        case 4: rc = launch_diagnostics_k4(a, c->tab, L, partial, c->gen, c->stream); break;
        case 5: rc = launch_diagnostics_k5(a, c->tab, L, partial, c->gen, c->stream); break;
        case 6: rc = launch_diagnostics_k6(a, c->tab, L, partial, c->gen, c->stream); break;
        case 7: rc = launch_diagnostics_k7(a, c->tab, L, partial, c->gen, c->stream); break;
        case 8: case 9: case 10: case 11:
            rc = launch_diagnostics_hd1(a, c->k, c->q, L, partial, c->gen, c->stream);
            break;
        case 12: case 13: case 14: case 15:
            rc = launch_diagnostics_hd2(a, c->k, c->q, L, partial, c->gen, c->stream);
            break;
    }
    if (rc == 0) rc = launch_diag_total(partial, c->ncell, total, c->stream);
    if (rc == 1) return fail(DGNS_EUNSUPPORTED, "no diagnostics kernel for degree %d, n_q %d", c->k, c->q);
    if (rc != 0) return fail(DGNS_EHIP, "diagnostics launch failed: %s", hipGetErrorString(hipGetLastError()));
    return 0;
}

int dispatch_ke_vjp(const dgns_ctx* c, const OpArgs& a, double* Ub) {
    int rc = 1;
    switch (c->k) {
        case 1: rc = launch_ke_vjp_k1(a, c->tab, Ub, c->gen, c->stream); break;
        case 2: rc = launch_ke_vjp_k2(a, c->tab, Ub, c->gen, c->stream); break;
        case 3: rc = launch_ke_vjp_k3(a, c->tab, Ub, c->gen, c->stream); break;
        case 4: rc = launch_ke_vjp_k4(a, c->tab, Ub, c->gen, c->stream); break;
        case 5: rc = launch_ke_vjp_k5(a, c->tab, Ub, c->gen, c->stream); break;
        case 6: rc = launch_ke_vjp_k6(a, c->tab, Ub, c->gen, c->stream); break;
        case 7: rc = launch_ke_vjp_k7(a, c->tab, Ub, c->gen, c->stream); break;
    }
    if (rc == 1) return fail(DGNS_EUNSUPPORTED, "no kinetic-energy kernel for degree %d, n_q %d", c->k, c->q);
    if (rc != 0) return fail(DGNS_EHIP, "kinetic energy VJP launch failed");
    return 0;
}

int dispatch_adjoint(const dgns_ctx* c, const OpArgs& a, const double* Rb) {
    if (c->fp32) return fail(DGNS_EUNSUPPORTED, "the adjoint is float64 only");
    int rc = 1;
    switch (c->k) {
        case 1: rc = launch_adjoint_k1(a, Rb, c->tab, c->gen, c->stream); break;
        case 2: rc = launch_adjoint_k2(a, Rb, c->tab, c->gen, c->stream); break;
        case 3: rc = launch_adjoint_k3(a, Rb, c->tab, c->gen, c->stream); break;
        case 4: rc = launch_adjoint_k4(a, Rb, c->tab, c->gen, c->stream); break;
        case 5: rc = launch_adjoint_k5(a, Rb, c->tab, c->gen, c->stream); break;
        default: break;
    }
    if (rc == 1) return fail(DGNS_EUNSUPPORTED, "no adjoint kernel for degree %d, n_q %d", c->k, c->q);
    if (rc != 0) return fail(DGNS_EHIP, "adjoint launch failed: %s", hipGetErrorString(hipGetLastError()));
    return 0;
}

bool aligned8(const void* p) { return ((uintptr_t)p & 7u) == 0; }

// [a, a + na) and [b, b + nb) share an element
bool overlap(const double* a, int64_t na, const double* b, int64_t nb) { return a < b + nb && b < a + na; }

}  // namespace

static void rk_default(dgns_ctx* c);

// ---------------------------------------------------------------- C ABI
extern "C" {

const char* dgns_last_error(void) { return g_err.c_str(); }

int dgns_create(const dgns_params* prm, const dgns_box_mesh* msh, void* stream, dgns_ctx** out) {
    if (!prm || !msh || !out) return fail(DGNS_EINVAL, "null argument");
    *out = nullptr;
    if (prm->degree < 1 || prm->degree > 15) return fail(DGNS_EINVAL, "degree %d outside 1..15", prm->degree);
    if (prm->n_q < 1 || prm->n_q > kMaxQ) return fail(DGNS_EINVAL, "n_q %d outside 1..%d", prm->n_q, kMaxQ);
    if (prm->basis != DGNS_BASIS_LGL && prm->basis != DGNS_BASIS_GL) return fail(DGNS_EINVAL, "unknown basis");
    if (prm->precision != DGNS_FP64 && prm->precision != DGNS_FP32) return fail(DGNS_EINVAL, "unknown precision");
    if (!(prm->gamma > 1) || !(prm->R > 0) || !(prm->mu >= 0) || !(prm->lambda >= 0) || !(prm->rho_ref > 0))
        return fail(DGNS_EINVAL, "fluid parameters out of range");
    if (msh->kind < 0 || msh->kind > 2) return fail(DGNS_EINVAL, "unknown mesh kind");
    for (int d = 0; d < 3; ++d) {
        if (msh->n[d] < 1) return fail(DGNS_EINVAL, "n[%d] = %d < 1", d, msh->n[d]);
        if (!(msh->hi[d] > msh->lo[d])) return fail(DGNS_EINVAL, "empty box in direction %d", d);
    }
    bool wall = !msh->periodic[0] || !msh->periodic[1] || !msh->periodic[2];
    if (wall && !(prm->wall_T > 0)) return fail(DGNS_EINVAL, "walls need wall_T > 0");
    const int64_t ncell = (int64_t)msh->n[0] * msh->n[1] * msh->n[2];
    if (ncell > 2147483647LL) return fail(DGNS_EINVAL, "too many cells");
    bool ok = false;
    for (const auto& kq : kSupported) ok |= (kq[0] == prm->degree && kq[1] == prm->n_q);
    for (const auto& kq : kSupportedHd) ok |= (kq[0] == prm->degree && kq[1] == prm->n_q);
    if (!ok) return fail(DGNS_EUNSUPPORTED, "no kernel for degree %d with n_q %d", prm->degree, prm->n_q);
    if (prm->degree >= 8 && (prm->body_force[0] != 0 || prm->body_force[1] != 0 || prm->body_force[2] != 0))
        return fail(DGNS_EUNSUPPORTED, "body forces are supported for degrees up to 7");

    dgns_ctx* c = new dgns_ctx();
    rk_default(c);
    c->prm = *prm;
    c->msh = *msh;
    c->stream = (hipStream_t)stream;
    c->k = prm->degree;
    c->n = prm->degree + 1;
    c->q = prm->n_q;
    c->fp32 = prm->precision == DGNS_FP32;
    c->gen = msh->kind != DGNS_MESH_AFFINE;
    c->ncell = ncell;
    c->n3 = (int64_t)c->n * c->n * c->n;
    c->ndof = 5 * ncell * c->n3;
    int rc = 0;
    {
        HostSetup hs;
        std::string err;
        rc = build_setup(*prm, *msh, hs, err);
        if (rc != 0) {
            fail(rc, "%s", err.c_str());
        } else {
            c->tab = hs.tab;
            c->h_min = hs.h_min;
            c->geo.swap(hs.geo);
            c->node_x.swap(hs.node_x);
            rc = upload(hs.metric, &c->d_metric);
            for (int d = 0; d < 3 && rc == 0; ++d) {
                rc = upload(hs.tau[d], &c->d_tau[d]);
                if (rc == 0 && c->gen) rc = upload(hs.face[d], &c->d_face[d]);
            }
            if (rc == 0 && c->gen) rc = upload(hs.mass_jxw, &c->d_mass_jxw);
        }
    }
    if (rc == 0) {
        std::vector<Tables1D> tv(1, c->tab);
        rc = upload(tv, &c->d_tab);
    }
    if (rc == 0) rc = noalloc_workspace(&c->noalloc);
    if (rc == 0) {
        // the face buffer of the kernels that evaluate each face once: six blocks of
        // 2 x 5 (k+1)^2 values per cell (float64 size, which also covers float32); where the
        // streamed kernels may run, followed by their per-cell scratch of z-swept planes,
        // [n_q][2][5][(k+1)^2] values per cell
        int64_t nfw = ncell * 6 * 10 * (int64_t)c->n * c->n;
        if (streamed_possible(c->k, c->q, c->fp32)) nfw += ncell * 10 * (int64_t)c->q * c->n * c->n;
        if (hipMalloc((void**)&c->d_fw, sizeof(double) * nfw) != hipSuccess) {
            c->d_fw = nullptr;
            rc = fail(DGNS_ENOMEM, "face buffer (%lld doubles)", (long long)nfw);
        }
    }
    if (rc == 0) {
        hipError_t e1 = hipMalloc((void**)&c->d_partial, sizeof(double) * 9 * ncell);
        hipError_t e2 = hipMalloc((void**)&c->d_total, sizeof(double) * 9);
        if (e1 != hipSuccess || e2 != hipSuccess) rc = fail(DGNS_ENOMEM, "diagnostics buffers");
    }
    if (rc != 0) {
        free_ctx(c);
        delete c;
        return rc;
    }
    *out = c;
    return DGNS_OK;
}

int dgns_destroy(dgns_ctx* c) {
    if (!c) return DGNS_OK;
    hipStreamSynchronize(c->stream);
    free_ctx(c);
    delete c;
    return DGNS_OK;
}

int dgns_sizes(const dgns_ctx* c, int64_t* n_cells, int64_t* nodes_per_cell, int64_t* n_dof) {
    if (!c) return fail(DGNS_EINVAL, "null context");
    if (n_cells) *n_cells = c->ncell;
    if (nodes_per_cell) *nodes_per_cell = c->n3;
    if (n_dof) *n_dof = c->ndof;
    return DGNS_OK;
}

int dgns_set_stream(dgns_ctx* c, void* stream) {
    if (!c) return fail(DGNS_EINVAL, "null context");
    c->stream = (hipStream_t)stream;
    return DGNS_OK;
}

int dgns_apply_residual(dgns_ctx* c, const double* U, double* R, unsigned term_mask) {
    if (!c || !U || !R) return fail(DGNS_EINVAL, "null argument");
    if (!aligned8(U) || !aligned8(R)) return fail(DGNS_EINVAL, "vectors must be 8-byte aligned");
    if (overlap(U, c->ndof, R, c->ndof)) return fail(DGNS_EINVAL, "U and R overlap");
    if (term_mask & ~DGNS_TERM_ALL) return fail(DGNS_EINVAL, "unknown term bits");
    return dispatch_operator(c, make_args(c, U, R, term_mask, 0));
}

int dgns_apply_inverse_mass(dgns_ctx* c, const double* R, double* L) {
    if (!c || !R || !L) return fail(DGNS_EINVAL, "null argument");
    if (!aligned8(R) || !aligned8(L)) return fail(DGNS_EINVAL, "vectors must be 8-byte aligned");
    if (R != L && overlap(R, c->ndof, L, c->ndof)) return fail(DGNS_EINVAL, "R and L partially overlap");
    return dispatch_minv(c, R, L);
}

int dgns_apply_operator(dgns_ctx* c, const double* U, double* L, double t) {
    (void)t;
    if (!c || !U || !L) return fail(DGNS_EINVAL, "null argument");
    if (!aligned8(U) || !aligned8(L)) return fail(DGNS_EINVAL, "vectors must be 8-byte aligned");
    if (overlap(U, c->ndof, L, c->ndof)) return fail(DGNS_EINVAL, "U and L overlap");
    return dispatch_operator(c, make_args(c, U, L, DGNS_TERM_ALL, 1));
}

// Carpenter & Kennedy (1994), five stages, fourth order, 2N storage: the default scheme.
static const double kRkA[5] = {0.0, -567301805773.0 / 1357537059087.0, -2404267990393.0 / 2016746695238.0,
                               -3550918686646.0 / 2091501179385.0, -1275806237668.0 / 842570457699.0};
static const double kRkB[5] = {1432997174477.0 / 9575080441755.0, 5161836677717.0 / 13612068292357.0,
                               1720146321549.0 / 2090206949498.0, 3134564353537.0 / 4481467310338.0,
                               2277821191437.0 / 14882151754819.0};

// Stage times of a 2N scheme: stage i evaluates L at U_0 + sum_{l < i} B_l dU_l with
// dU_l = sum_{j <= l} (prod_{m = j+1..l} A_m) dt k_j, so c_i = sum_{l < i} B_l sum_{j <= l} prod A.
static void rk_stage_times(int s, const double* A, const double* B, double* cc) {
    for (int i = 0; i < s; ++i) {
        double ci = 0;
        for (int l = 0; l < i; ++l) {
            double w = 0;
            for (int j = 0; j <= l; ++j) {
                double p = 1;
                for (int m = j + 1; m <= l; ++m) p *= A[m];
                w += p;
            }
            ci += B[l] * w;
        }
        cc[i] = ci;
    }
}

static void rk_default(dgns_ctx* c) {
    c->rk_s = 5;
    for (int i = 0; i < 5; ++i) {
        c->rk_A[i] = kRkA[i];
        c->rk_B[i] = kRkB[i];
    }
    rk_stage_times(5, c->rk_A, c->rk_B, c->rk_c);
}

int dgns_set_rk_scheme(dgns_ctx* c, int stages, const double* A, const double* B, const double* cc) {
    if (!c) return fail(DGNS_EINVAL, "null context");
    if (stages == 0 && !A && !B && !cc) {
        rk_default(c);
        return DGNS_OK;
    }
    if (!A || !B) return fail(DGNS_EINVAL, "null coefficient array");
    if (stages < 1 || stages > kMaxRkStages) return fail(DGNS_EINVAL, "stages %d outside 1..%d", stages, kMaxRkStages);
    if (A[0] != 0.0) return fail(DGNS_EINVAL, "A[0] must be 0 (the first stage does not read dU)");
    for (int i = 0; i < stages; ++i)
        if (!std::isfinite(A[i]) || !std::isfinite(B[i]) || (cc && !std::isfinite(cc[i])))
            return fail(DGNS_EINVAL, "coefficient %d is not finite", i);
    c->rk_s = stages;
    for (int i = 0; i < stages; ++i) {
        c->rk_A[i] = A[i];
        c->rk_B[i] = B[i];
    }
    if (cc)
        for (int i = 0; i < stages; ++i) c->rk_c[i] = cc[i];
    else
        rk_stage_times(stages, c->rk_A, c->rk_B, c->rk_c);
    return DGNS_OK;
}

int dgns_get_rk_scheme(const dgns_ctx* c, int* stages, double* A, double* B, double* cc) {
    if (!c || !stages) return fail(DGNS_EINVAL, "null argument");
    *stages = c->rk_s;
    for (int i = 0; i < c->rk_s; ++i) {
        if (A) A[i] = c->rk_A[i];
        if (B) B[i] = c->rk_B[i];
        if (cc) cc[i] = c->rk_c[i];
    }
    return DGNS_OK;
}

int dgns_rk_step(dgns_ctx* c, double* U, double* work, double t, double dt) {
    (void)t;
    if (!c || !U || !work) return fail(DGNS_EINVAL, "null argument");
    if (!aligned8(U) || !aligned8(work)) return fail(DGNS_EINVAL, "vectors must be 8-byte aligned");
    if (overlap(U, c->ndof, work, 2 * c->ndof)) return fail(DGNS_EINVAL, "U and work overlap");
    if (!std::isfinite(dt)) return fail(DGNS_EINVAL, "dt is not finite");
    double* dU = work;
    double* U2 = work + c->ndof;
    const int s = c->rk_s;
    // Stages 1..s-1 fuse the update into the operator kernel, alternating the state
    // between U and U2 (a stage cannot overwrite the U its neighbours still read):
    // U -> U2 -> U -> ...  The last stage writes L into the other buffer and updates
    // the state in place; after an odd number of fused stages the state ends in U2 and
    // is copied back.
    const double* src = U;
    double* dst = U2;
    for (int i = 0; i < s - 1; ++i) {
        OpArgs a = make_args(c, src, nullptr, DGNS_TERM_ALL, 1);
        a.rk.dU = dU;
        a.rk.U_out = dst;
        a.rk.A = c->rk_A[i];
        a.rk.B = c->rk_B[i];
        a.rk.dt = dt;
        int rc = dispatch_operator(c, a);
        if (rc) return rc;
        double* next = const_cast<double*>(src);
        src = dst;
        dst = next;
    }
    double* state = const_cast<double*>(src);
    int rc = dispatch_operator(c, make_args(c, state, dst, DGNS_TERM_ALL, 1));
    if (rc) return rc;
    if (launch_rk_update(state, dU, dst, c->ndof, c->rk_A[s - 1], c->rk_B[s - 1], dt, c->stream) != 0)
        return fail(DGNS_EHIP, "rk update launch failed");
    if (state != U) HIP_TRY(hipMemcpyAsync(U, state, sizeof(double) * c->ndof, hipMemcpyDeviceToDevice, c->stream));
    return DGNS_OK;
}

int dgns_rk_stage_update(dgns_ctx* c, double* U, double* dU, const double* L, int stage, double dt) {
    if (!c || !U || !dU || !L) return fail(DGNS_EINVAL, "null argument");
    if (stage < 0 || stage >= c->rk_s) return fail(DGNS_EINVAL, "stage %d outside 0..%d", stage, c->rk_s - 1);
    if (!std::isfinite(dt)) return fail(DGNS_EINVAL, "dt is not finite");
    if (!aligned8(U) || !aligned8(dU) || !aligned8(L)) return fail(DGNS_EINVAL, "vectors must be 8-byte aligned");
    const int64_t n = c->ndof;
    if (overlap(U, n, dU, n) || overlap(U, n, L, n) || overlap(dU, n, L, n))
        return fail(DGNS_EINVAL, "U, dU and L must not overlap");
    if (launch_rk_update(U, dU, L, n, c->rk_A[stage], c->rk_B[stage], dt, c->stream) != 0)
        return fail(DGNS_EHIP, "rk update launch failed");
    return DGNS_OK;
}

int dgns_compute_dt(const dgns_ctx* c, double Cr, double D, double e, double f, double umax, double mach,
                    double* dt) {
    if (!c || !dt) return fail(DGNS_EINVAL, "null argument");
    if (!(umax > 0) || !(mach > 0) || !(Cr > 0)) return fail(DGNS_EINVAL, "umax, mach and Cr must be positive");
    const double k = c->k;
    const double nu = c->prm.mu / c->prm.rho_ref;
    const double dtc = Cr / std::pow(k, e) * c->h_min / (umax + umax / mach);
    const double dtv = (nu > 0 && D > 0) ? D / std::pow(k, f) * c->h_min * c->h_min / nu : INFINITY;
    *dt = std::min(dtc, dtv);
    return DGNS_OK;
}

int dgns_diagnostics(dgns_ctx* c, const double* U, const double* L, double* out8) {
    if (!c || !U || !out8) return fail(DGNS_EINVAL, "null argument");
    if (!aligned8(U) || (L && !aligned8(L))) return fail(DGNS_EINVAL, "vectors must be 8-byte aligned");
    OpArgs a = make_args(c, U, nullptr, 0, 0);
    int rc = dispatch_diagnostics(c, a, L);
    if (rc) return rc;
    double tot[9];
    HIP_TRY(hipMemcpyAsync(tot, c->d_total, sizeof tot, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    const double V = tot[8];
    const double nu = c->prm.mu / c->prm.rho_ref;
    double r[8];
    r[0] = tot[0] / V;
    r[1] = nu * tot[1] / V;
    r[2] = L ? tot[2] / V : NAN;
    for (int i = 0; i < 5; ++i) r[3 + i] = tot[3 + i];
    for (int i = 0; i < 8; ++i)
        if (i != 2 || L)
            if (!std::isfinite(r[i])) return fail(DGNS_ENONFINITE, "diagnostic %d is not finite", i);
    for (int i = 0; i < 8; ++i) out8[i] = r[i];   // written only on success
    return DGNS_OK;
}

int dgns_diagnostics_noalloc(dgns_ctx* c, const double* U, const double* L, double* out8) {
    if (!c || !U || !out8) return fail(DGNS_EINVAL, "null argument");
    if (!aligned8(U) || (L && !aligned8(L)) || !aligned8(out8)) return fail(DGNS_EINVAL, "vectors must be 8-byte aligned");
    if (c->ncell > kNoAllocMaxCells)
        return fail(DGNS_EINVAL, "mesh of %lld cells; the allocation-free diagnostics hold at most %lld",
                    (long long)c->ncell, (long long)kNoAllocMaxCells);
    if (overlap(out8, 8, U, c->ndof) || (L && overlap(out8, 8, L, c->ndof)))
        return fail(DGNS_EINVAL, "out8 overlaps an input");
    if (!c->noalloc) return fail(DGNS_EHIP, "no workspace address for this context");
    double* partial = c->noalloc;
    double* total = c->noalloc + 9 * kNoAllocMaxCells;
    OpArgs a = make_args(c, U, nullptr, 0, 0);
    int rc = dispatch_diagnostics(c, a, L, partial, total);
    if (rc) return rc;
    if (launch_diag_finalize(total, c->prm.mu / c->prm.rho_ref, L ? 1 : 0, out8, c->stream) != 0)
        return fail(DGNS_EHIP, "diagnostics finalize launch failed");
    return DGNS_OK;
}

int dgns_apply_residual_vjp(dgns_ctx* c, const double* U, const double* Rbar, double* Ubar, unsigned term_mask) {
    if (!c || !U || !Rbar || !Ubar) return fail(DGNS_EINVAL, "null argument");
    if (!aligned8(U) || !aligned8(Rbar) || !aligned8(Ubar)) return fail(DGNS_EINVAL, "vectors must be 8-byte aligned");
    if (overlap(Ubar, c->ndof, U, c->ndof) || overlap(Ubar, c->ndof, Rbar, c->ndof))
        return fail(DGNS_EINVAL, "Ubar overlaps an input");
    if (term_mask & ~DGNS_TERM_ALL) return fail(DGNS_EINVAL, "unknown term bits");
    return dispatch_adjoint(c, make_args(c, U, Ubar, term_mask, 0), Rbar);
}

static int channel_profiles(dgns_ctx* c, const double* U, std::vector<double>& res);
static int channel_wall_shear(dgns_ctx* c, const double* U, double out3[3]);

int dgns_channel_statistics(dgns_ctx* c, const double* U, double* out) {
    if (!c || !U || !out) return fail(DGNS_EINVAL, "null argument");
    if (!aligned8(U)) return fail(DGNS_EINVAL, "U must be 8-byte aligned");
    std::vector<double> res;
    int rc = channel_profiles(c, U, res);
    if (rc) return rc;
    std::copy(res.begin(), res.end(), out);   // written only on success
    return DGNS_OK;
}

int dgns_channel_wall_shear(dgns_ctx* c, const double* U, double* out3) {
    if (!c || !U || !out3) return fail(DGNS_EINVAL, "null argument");
    if (!aligned8(U)) return fail(DGNS_EINVAL, "U must be 8-byte aligned");
    double r[3];
    int rc = channel_wall_shear(c, U, r);
    if (rc) return rc;
    for (int m = 0; m < 3; ++m) out3[m] = r[m];
    return DGNS_OK;
}

int dgns_channel_stats_reset(dgns_ctx* c) {
    if (!c) return fail(DGNS_EINVAL, "null context");
    c->stats_samples = 0;
    c->stats_sum.clear();
    c->tau_sum = c->rho_w_sum = 0;
    return DGNS_OK;
}

int dgns_channel_stats_sample(dgns_ctx* c, const double* U) {
    if (!c || !U) return fail(DGNS_EINVAL, "null argument");
    if (!aligned8(U)) return fail(DGNS_EINVAL, "U must be 8-byte aligned");
    std::vector<double> res;
    double w[3];
    int rc = channel_profiles(c, U, res);
    if (!rc) rc = channel_wall_shear(c, U, w);
    if (rc) return rc;
    if (c->stats_sum.empty()) c->stats_sum.assign(res.size(), 0.0);
    for (size_t m = 0; m < res.size(); ++m) c->stats_sum[m] += res[m];
    c->tau_sum += w[0];
    c->rho_w_sum += w[1];
    ++c->stats_samples;
    return DGNS_OK;
}

int dgns_channel_stats_result(dgns_ctx* c, double* profiles, double* scalars) {
    if (!c || !profiles || !scalars) return fail(DGNS_EINVAL, "null argument");
    if (c->stats_samples < 1) return fail(DGNS_EINVAL, "no samples");
    const double ns = (double)c->stats_samples;
    const double tau = c->tau_sum / ns, rho_w = c->rho_w_sum / ns;
    if (!(tau > 0) || !(rho_w > 0)) return fail(DGNS_ENONFINITE, "mean wall shear %g is not positive", tau);
    const double u_tau = std::sqrt(tau / rho_w), nu = c->prm.mu / c->prm.rho_ref;
    const int64_t rows = (int64_t)c->stats_sum.size() / 9;
    std::vector<double> out(rows * 8);
    const double ylo = c->msh.lo[1];
    for (int64_t r = 0; r < rows; ++r) {
        const double* a = c->stats_sum.data() + r * 9;
        const double y = a[0] / ns, rho = a[1] / ns, u = a[2] / ns, v = a[3] / ns, w = a[4] / ns;
        const double uu = a[5] / ns, vv = a[6] / ns, ww = a[7] / ns, uv = a[8] / ns;
        double* o = out.data() + r * 8;
        o[0] = y;
        o[1] = (y - ylo) * u_tau / nu;
        o[2] = u / u_tau;
        o[3] = std::sqrt(std::max(uu - u * u, 0.0)) / u_tau;
        o[4] = std::sqrt(std::max(vv - v * v, 0.0)) / u_tau;
        o[5] = std::sqrt(std::max(ww - w * w, 0.0)) / u_tau;
        o[6] = (uv - u * v) / (u_tau * u_tau);
        o[7] = rho;
    }
    std::copy(out.begin(), out.end(), profiles);
    scalars[0] = u_tau;
    scalars[1] = tau;
    scalars[2] = rho_w;
    scalars[3] = ns;
    return DGNS_OK;
}

}  // extern "C"

// Plane averages at the wall-normal Gauss points (see dgns_channel_statistics), on the host.
static int channel_profiles(dgns_ctx* c, const double* U, std::vector<double>& res_out) {
    if (c->msh.kind == DGNS_MESH_CURVED)
        return fail(DGNS_EUNSUPPORTED, "channel statistics need planes of constant y (affine or channel mesh)");
    const int q = c->q, n1 = c->msh.n[1];
    const int64_t np = c->ncell * q * 9, nt = (int64_t)n1 * q * 9;
    if (!c->d_stats && hipMalloc((void**)&c->d_stats, sizeof(double) * (np + nt)) != hipSuccess) {
        c->d_stats = nullptr;
        return fail(DGNS_ENOMEM, "channel statistics buffer (%lld doubles)", (long long)(np + nt));
    }
    OpArgs a = make_args(c, U, nullptr, 0, 0);
    int rc = 1;
    switch (c->k) {
        case 1: rc = launch_chan_stats_k1(a, c->tab, c->d_stats, c->gen, c->stream); break;
        case 2: rc = launch_chan_stats_k2(a, c->tab, c->d_stats, c->gen, c->stream); break;
        case 3: rc = launch_chan_stats_k3(a, c->tab, c->d_stats, c->gen, c->stream); break;
        case 4: rc = launch_chan_stats_k4(a, c->tab, c->d_stats, c->gen, c->stream); break;
        case 5: rc = launch_chan_stats_k5(a, c->tab, c->d_stats, c->gen, c->stream); break;
        case 6: rc = launch_chan_stats_k6(a, c->tab, c->d_stats, c->gen, c->stream); break;
        case 7: rc = launch_chan_stats_k7(a, c->tab, c->d_stats, c->gen, c->stream); break;
    }
    if (rc == 1) return fail(DGNS_EUNSUPPORTED, "no statistics kernel for degree %d, n_q %d", c->k, c->q);
    if (rc == 0) rc = launch_chan_stats_total(c->d_stats, c->msh.n, q, c->d_stats + np, c->stream);
    if (rc != 0) return fail(DGNS_EHIP, "channel statistics launch failed");
    std::vector<double> tot(nt);
    HIP_TRY(hipMemcpyAsync(tot.data(), c->d_stats + np, sizeof(double) * nt, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    // y of the wall-normal points: the geometry interpolant of cell row j along xi_1
    // (y depends on xi_1 alone on these meshes), read from the first cell of the row
    const int N = c->n;
    std::vector<double> res(nt);
    for (int j = 0; j < n1; ++j) {
        const int64_t e = (int64_t)c->msh.n[0] * j;
        const double* g = c->geo.data() + (e * 3 + 1) * c->n3;
        for (int p = 0; p < q; ++p) {
            double y = 0;
            for (int i = 0; i < N; ++i) y += g[N * i] * c->tab.Sg[p][i];
            const double* t = tot.data() + ((int64_t)j * q + p) * 9;
            double* o = res.data() + ((int64_t)j * q + p) * 9;
            o[0] = y;
            for (int m = 1; m < 9; ++m) o[m] = t[m] / t[0];
            for (int m = 0; m < 9; ++m)
                if (!std::isfinite(o[m])) return fail(DGNS_ENONFINITE, "statistic %d at row %d, point %d is not finite", m, j, p);
        }
    }
    res_out.swap(res);
    return DGNS_OK;
}

// Mean wall shear over both walls in x_2: {tau_w, rho_w, wall area} (area-weighted means).
static int channel_wall_shear(dgns_ctx* c, const double* U, double out3[3]) {
    if (c->msh.periodic[1]) return fail(DGNS_EUNSUPPORTED, "the wall shear needs walls in direction 1");
    if (c->msh.kind == DGNS_MESH_CURVED)
        return fail(DGNS_EUNSUPPORTED, "the wall shear needs planar walls of constant x_2 (affine or channel mesh)");
    const int64_t nw = 2 * (int64_t)c->msh.n[0] * c->msh.n[2];
    if (!c->d_wall && hipMalloc((void**)&c->d_wall, sizeof(double) * kWallSumsHost * nw) != hipSuccess) {
        c->d_wall = nullptr;
        return fail(DGNS_ENOMEM, "wall shear buffer");
    }
    OpArgs a = make_args(c, U, nullptr, 0, 0);
    int rc = 1;
    switch (c->k) {
        case 1: rc = launch_wall_shear_k1(a, c->tab, c->d_wall, c->gen, c->stream); break;
        case 2: rc = launch_wall_shear_k2(a, c->tab, c->d_wall, c->gen, c->stream); break;
        case 3: rc = launch_wall_shear_k3(a, c->tab, c->d_wall, c->gen, c->stream); break;
        case 4: rc = launch_wall_shear_k4(a, c->tab, c->d_wall, c->gen, c->stream); break;
        case 5: rc = launch_wall_shear_k5(a, c->tab, c->d_wall, c->gen, c->stream); break;
        case 6: rc = launch_wall_shear_k6(a, c->tab, c->d_wall, c->gen, c->stream); break;
        case 7: rc = launch_wall_shear_k7(a, c->tab, c->d_wall, c->gen, c->stream); break;
    }
    if (rc == 1) return fail(DGNS_EUNSUPPORTED, "no wall-shear kernel for degree %d, n_q %d", c->k, c->q);
    if (rc != 0) return fail(DGNS_EHIP, "wall shear launch failed");
    std::vector<double> part(kWallSumsHost * nw);
    HIP_TRY(hipMemcpyAsync(part.data(), c->d_wall, sizeof(double) * part.size(), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    double t[3] = {0, 0, 0};
    for (int64_t w = 0; w < nw; ++w)
        for (int m = 0; m < 3; ++m) t[m] += part[w * kWallSumsHost + m];   // fixed order: deterministic
    out3[0] = t[0] / t[2];
    out3[1] = t[1] / t[2];
    out3[2] = t[2];
    for (int m = 0; m < 3; ++m)
        if (!std::isfinite(out3[m])) return fail(DGNS_ENONFINITE, "wall shear sum %d is not finite", m);
    return DGNS_OK;
}

extern "C" {

static int ensure_scratch(dgns_ctx* c) {
    if (c->d_scratch) return 0;
    if (hipMalloc((void**)&c->d_scratch, sizeof(double) * c->ndof) != hipSuccess) {
        c->d_scratch = nullptr;
        return fail(DGNS_ENOMEM, "operator VJP scratch (%lld doubles)", (long long)c->ndof);
    }
    return 0;
}

int dgns_apply_operator_vjp(dgns_ctx* c, const double* U, const double* Lbar, double* Ubar) {
    if (!c || !U || !Lbar || !Ubar) return fail(DGNS_EINVAL, "null argument");
    if (!aligned8(U) || !aligned8(Lbar) || !aligned8(Ubar)) return fail(DGNS_EINVAL, "vectors must be 8-byte aligned");
    if (overlap(Ubar, c->ndof, U, c->ndof) || overlap(Ubar, c->ndof, Lbar, c->ndof))
        return fail(DGNS_EINVAL, "Ubar overlaps an input");
    int rc = ensure_scratch(c);
    if (rc) return rc;
    // L = M^{-1} R(U): Ubar = (dR/dU)^T M^{-T} Lbar, and M is symmetric
    rc = dispatch_minv(c, Lbar, c->d_scratch);
    if (rc) return rc;
    return dispatch_adjoint(c, make_args(c, U, Ubar, DGNS_TERM_ALL, 0), c->d_scratch);
}

int dgns_rk_step_vjp(dgns_ctx* c, const double* U_n, double t, double dt, const double* Ubar_np1, double* Ubar_n,
                     double* work) {
    (void)t;
    if (!c || !U_n || !Ubar_np1 || !Ubar_n || !work) return fail(DGNS_EINVAL, "null argument");
    if (!aligned8(U_n) || !aligned8(Ubar_np1) || !aligned8(Ubar_n) || !aligned8(work))
        return fail(DGNS_EINVAL, "vectors must be 8-byte aligned");
    const int64_t n = c->ndof;
    const int s = c->rk_s;
    const int64_t nw = (int64_t)(s + 4) * n;
    if (overlap(work, nw, U_n, n) || overlap(work, nw, Ubar_np1, n) || overlap(work, nw, Ubar_n, n) ||
        overlap(Ubar_n, n, U_n, n) || (Ubar_n != Ubar_np1 && overlap(Ubar_n, n, Ubar_np1, n)))
        return fail(DGNS_EINVAL, "overlapping arguments");
    if (!std::isfinite(dt)) return fail(DGNS_EINVAL, "dt is not finite");
    double* X = work;               // stage inputs U_1..U_{s-1} (U_0 = U_n)
    double* dU = work + (int64_t)(s - 1) * n;
    double* L = dU + n;
    double* dUb = L + n;
    double* Rb = dUb + n;
    double* T = Rb + n;
    // forward recomputation of the stage inputs
    for (int i = 0; i < s - 1; ++i) {
        const double* src = i == 0 ? U_n : X + (int64_t)(i - 1) * n;
        double* Ui = X + (int64_t)i * n;
        HIP_TRY(hipMemcpyAsync(Ui, src, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream));
        int rc = dispatch_operator(c, make_args(c, src, L, DGNS_TERM_ALL, 1));
        if (rc) return rc;
        if (launch_rk_update(Ui, dU, L, n, c->rk_A[i], c->rk_B[i], dt, c->stream) != 0)
            return fail(DGNS_EHIP, "rk update launch failed");
    }
    // reverse sweep over the stages
    if (Ubar_n != Ubar_np1)
        HIP_TRY(hipMemcpyAsync(Ubar_n, Ubar_np1, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream));
    if (launch_fill(dUb, n, 0.0, c->stream) != 0) return fail(DGNS_EHIP, "fill launch failed");
    for (int i = s - 1; i >= 0; --i) {
        const double* Xi = i == 0 ? U_n : X + (int64_t)(i - 1) * n;
        // U_i = U_{i-1} + B_i dU_i  ->  dUbar_i += B_i Ubar_i
        if (launch_axpby(dUb, Ubar_n, n, 1.0, c->rk_B[i], c->stream) != 0) return fail(DGNS_EHIP, "axpby launch failed");
        // K_i = L(U_{i-1}), dU_i = A_i dU_{i-1} + dt K_i  ->  Ubar_{i-1} += dt (dL/dU)^T dUbar_i
        int rc = dispatch_minv(c, dUb, Rb);
        if (rc) return rc;
        rc = dispatch_adjoint(c, make_args(c, Xi, T, DGNS_TERM_ALL, 0), Rb);
        if (rc) return rc;
        if (launch_axpby(Ubar_n, T, n, 1.0, dt, c->stream) != 0) return fail(DGNS_EHIP, "axpby launch failed");
        //  dUbar_{i-1} = A_i dUbar_i
        if (launch_axpby(dUb, dUb, n, c->rk_A[i], 0.0, c->stream) != 0) return fail(DGNS_EHIP, "axpby launch failed");
    }
    return DGNS_OK;
}

int dgns_kinetic_energy(dgns_ctx* c, const double* U, double* ke) {
    if (!c || !U || !ke) return fail(DGNS_EINVAL, "null argument");
    if (!aligned8(U)) return fail(DGNS_EINVAL, "U must be 8-byte aligned");
    OpArgs a = make_args(c, U, nullptr, 0, 0);
    int rc = dispatch_diagnostics(c, a, nullptr);
    if (rc) return rc;
    double tot[9];
    HIP_TRY(hipMemcpyAsync(tot, c->d_total, sizeof tot, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (!std::isfinite(tot[0])) return fail(DGNS_ENONFINITE, "kinetic energy is not finite");
    *ke = tot[0];
    return DGNS_OK;
}

int dgns_kinetic_energy_vjp(dgns_ctx* c, const double* U, double* Ubar) {
    if (!c || !U || !Ubar) return fail(DGNS_EINVAL, "null argument");
    if (!aligned8(U) || !aligned8(Ubar)) return fail(DGNS_EINVAL, "vectors must be 8-byte aligned");
    if (overlap(U, c->ndof, Ubar, c->ndof)) return fail(DGNS_EINVAL, "U and Ubar overlap");
    return dispatch_ke_vjp(c, make_args(c, U, nullptr, 0, 0), Ubar);
}

int dgns_project_ic(dgns_ctx* c, int ic, const double* icp, const double* noise, double* U) {
    if (!c || !icp || !U) return fail(DGNS_EINVAL, "null argument");
    if (ic < 0 || ic > 2) return fail(DGNS_EINVAL, "unknown initial condition %d", ic);
    if (!aligned8(U) || (noise && !aligned8(noise))) return fail(DGNS_EINVAL, "vectors must be 8-byte aligned");
    double q[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const int np = ic == DGNS_IC_UNIFORM ? 5 : 4;
    for (int i = 0; i < np; ++i) q[i] = icp[i];
    double *d_geo = nullptr, *d_q = nullptr, *d_x = nullptr;
    std::vector<double> qv(q, q + 8);
    int rc = upload(c->geo, &d_geo);
    if (!rc) rc = upload(qv, &d_q);
    if (!rc) {
        OpArgs a = make_args(c, nullptr, nullptr, 0, 0);
        if (launch_ic_rhs(a, c->tab, c->d_tab, d_geo, ic, d_q, U, c->gen, c->stream) != 0)
            rc = fail(DGNS_EHIP, "ic launch failed");
    }
    if (!rc) rc = dispatch_minv(c, U, U);
    if (!rc && ic == DGNS_IC_CHANNEL && noise) {
        rc = upload(c->node_x, &d_x);
        if (!rc && launch_channel_perturb(U, d_x, noise, c->ncell, (int)c->n3, q[0], q[2], q[3], c->prm.gamma,
                                          c->prm.R, c->stream) != 0)
            rc = fail(DGNS_EHIP, "perturbation launch failed");
    }
    hipStreamSynchronize(c->stream);
    hipFree(d_geo);
    hipFree(d_q);
    hipFree(d_x);
    return rc;
}

}  // extern "C"
