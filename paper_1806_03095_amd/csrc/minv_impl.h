// Stand-alone inverse mass matrix of the DG operator (Sec. 2.2.3, 2.3): L = M^{-1} R per
// cell and conserved field, with M the mass matrix of the k+1 point Gauss rule, applied
// as the tensor product of the inverse 1D interpolation matrices and the diagonal of
// |J| w at the mass points.  The operator kernel applies the same inverse in LDS on its
// own residual (op_impl.h); this kernel serves the stand-alone entry point.
#pragma once

#include "op_impl.h"

namespace dgns {

// Standalone inverse mass.  A workgroup of 256 threads takes RPB consecutive (component,
// cell) blocks, one contiguous run of RPB N^3 values; each thread owns LPT lines of N
// values per axis.  The x-lines are loaded straight from memory (consecutive threads on
// consecutive lines, so a wave covers one contiguous run) and swept in registers; the
// sweeps along xi_1 and xi_2 (then the diagonal scaling and the transposed sweeps back)
// read a line from LDS into registers and write it back in place, so that one barrier
// per change of axis suffices; the last x sweep stores straight to memory.  Two lines
// per thread for N <= 6 double the bytes in flight per workgroup (measured 3-11% faster
// on vectors past the last-level cache; staging whole runs through LDS with coalesced
// loads was 10-20% slower).  In place allowed: a workgroup reads all of its blocks
// before it writes them.
constexpr int kMinvLineBlock = 256;

template <int N>
struct MinvPlan {
    static constexpr int LPT = N <= 6 ? 2 : 1;                  // lines per thread and axis
    static constexpr int RPB = LPT * kMinvLineBlock / (N * N);  // blocks per workgroup
};

template <int N, bool TRANS, typename Real>
__device__ __forceinline__ void apply_line(const Real (&M)[N][N], Real (&v)[N]) {
    Real t[N];
#pragma unroll
    for (int o = 0; o < N; ++o) {
        Real acc = 0;
#pragma unroll
        for (int m = 0; m < N; ++m) acc += (TRANS ? M[m][o] : M[o][m]) * v[m];
        t[o] = acc;
    }
#pragma unroll
    for (int o = 0; o < N; ++o) v[o] = t[o];
}

// One sweep of the standalone inverse mass over the thread's lines along one axis:
// AX 0 lines (a1, a2), AX 1 lines (a0, a2), AX 2 lines (a0, a1); the line's values are
// strided by 1, N, N^2 within the block.
template <int N, int AX, bool TRANS, typename Real>
__device__ __forceinline__ void minv_sweep(const Real (&M)[N][N], Real* blk, int ln) {
    constexpr int N2 = N * N;
    const int base = AX == 0 ? ln * N : (AX == 1 ? (ln / N) * N2 + ln % N : ln);
    constexpr int st = AX == 0 ? 1 : (AX == 1 ? N : N2);
    Real v[N];
#pragma unroll
    for (int m = 0; m < N; ++m) v[m] = blk[base + m * st];
    apply_line<N, TRANS>(M, v);
#pragma unroll
    for (int m = 0; m < N; ++m) blk[base + m * st] = v[m];
}

template <int N, typename Real, bool GEN>
__global__ void __launch_bounds__(kMinvLineBlock)
inverse_mass_line_kernel(const double* R, double* L, int64_t ncell, const double* cell_metric,
                           const double* mass_jxw, MTab<N, Real> mt) {
    constexpr int N2 = N * N, N3 = N2 * N, LPT = MinvPlan<N>::LPT, RPB = MinvPlan<N>::RPB;
    constexpr int B = kMinvLineBlock;
    __shared__ Real buf[RPB * N3];
    __shared__ Real lwm[N];
    const int tid = threadIdx.x;
    if (tid < N) lwm[tid] = mt.wm[tid];
    const MTab<N, Real>* tp = &mt;
    if constexpr (N > 7) {
        __shared__ MTab<N, Real> lmt;
        copy_table<MTab<N, Real>, Real>(mt, lmt);
        tp = &lmt;
        __syncthreads();
    }
    const auto& Smi = tp->Smi;
    const int64_t row0 = (int64_t)blockIdx.x * RPB;
    const int rows = 5 * ncell - row0 < RPB ? (int)(5 * ncell - row0) : RPB;
    Real v[LPT][N];
#pragma unroll
    for (int j = 0; j < LPT; ++j) {
        const int line = tid + j * B;
        if (line < rows * N2) {
            const double* src = R + row0 * N3 + (int64_t)line * N;
#pragma unroll
            for (int m = 0; m < N; ++m) v[j][m] = (Real)src[m];
        }
    }
#pragma unroll
    for (int j = 0; j < LPT; ++j) {
        const int line = tid + j * B;
        if (line < rows * N2) {
            apply_line<N, true>(Smi, v[j]);
#pragma unroll
            for (int m = 0; m < N; ++m) buf[line * N + m] = v[j][m];
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < LPT; ++j) {
        const int line = tid + j * B;
        if (line < rows * N2) minv_sweep<N, 1, true>(Smi, buf + (line / N2) * N3, line % N2);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < LPT; ++j) {
        const int line = tid + j * B;
        if (line < rows * N2) {
            const int lb = line / N2, ln = line % N2, z0 = ln % N, z1 = ln / N;
            Real* blk = buf + lb * N3;
            Real w[N];
#pragma unroll
            for (int m = 0; m < N; ++m) w[m] = blk[m * N2 + ln];
            apply_line<N, true>(Smi, w);
            const int64_t e = (row0 + lb) % ncell;
            if constexpr (GEN) {
                const double* jw = mass_jxw + e * N3 + ln;
#pragma unroll
                for (int m = 0; m < N; ++m) w[m] = w[m] / (Real)jw[m * N2];
            } else {
                const Real f = Real(1) / ((Real)cell_metric[e * 10 + 9] * lwm[z0] * lwm[z1]);
#pragma unroll
                for (int m = 0; m < N; ++m) w[m] = w[m] * (f / tp->wm[m]);
            }
            apply_line<N, false>(Smi, w);
#pragma unroll
            for (int m = 0; m < N; ++m) blk[m * N2 + ln] = w[m];
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < LPT; ++j) {
        const int line = tid + j * B;
        if (line < rows * N2) minv_sweep<N, 1, false>(Smi, buf + (line / N2) * N3, line % N2);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < LPT; ++j) {
        const int line = tid + j * B;
        if (line < rows * N2) {
#pragma unroll
            for (int m = 0; m < N; ++m) v[j][m] = buf[line * N + m];
            apply_line<N, false>(Smi, v[j]);
            double* dst = L + row0 * N3 + (int64_t)line * N;
#pragma unroll
            for (int m = 0; m < N; ++m) dst[m] = (double)v[j][m];
        }
    }
}

template <int N, typename Real, bool GEN>
inline int launch_minv_t(const double* R, double* L, int64_t ncell, const double* cm, const double* mj,
                         const Tables1D& t, hipStream_t st) {
    MTab<N, Real> mt;
    for (int i = 0; i < N; ++i) {
        for (int j = 0; j < N; ++j) {
            mt.Sm[i][j] = (Real)t.Sm[i][j];
            mt.Smi[i][j] = (Real)t.Smi[i][j];
        }
        mt.wm[i] = (Real)t.wm[i];
    }
    constexpr int RPB = MinvPlan<N>::RPB;
    const int64_t grid = (5 * ncell + RPB - 1) / RPB;
    hipLaunchKernelGGL((inverse_mass_line_kernel<N, Real, GEN>), dim3((unsigned)grid), dim3(kMinvLineBlock), 0, st, R,
                       L, ncell, cm, mj, mt);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace dgns
