// Host-side checks of the operator kernel's LDS plan for every compiled (degree, n_q)
// and both precisions (and of the face kernel's where the face terms have a kernel of
// their own): the work area holds every phase, the regions that two phases use
// at once do not overlap, the fused trace phase covers its items, and the whole
// footprint fits a compute unit's LDS.  Prints one line per kernel and "all ok" when
// every check holds; exits non-zero otherwise.
#include <cstdio>

#include "dg_kernels.h"
#include "op_impl.h"

using namespace dgns;

static int g_fail = 0;

static void check(bool ok, int k, int q, const char* prec, const char* what) {
    if (!ok) {
        std::printf("FAIL k=%d n_q=%d %s: %s\n", k, q, prec, what);
        ++g_fail;
    }
}

// [a0, a0 + n0) and [a1, a1 + n1) share no element
static bool disjoint(int a0, int n0, int a1, int n1) { return a0 + n0 <= a1 || a1 + n1 <= a0; }

// The face kernel of the split evaluation: one pass of face points (their results wait in
// registers), OUT then T1 within the three-face layout, the single-face layout inside it,
// and the footprint (sU, work area, tables) within a compute unit.
template <int N, int Q, typename Real>
void face_plan(int k, const char* prec) {
    using FB = FaceBlock<N, Q, Real>;
    using F = typename FB::FS;
    using F1 = typename FB::FS1;
    check(FB::threads == 64 || FB::threads == 128 || FB::threads == 256, k, Q, prec, "face block size");
    check(FB::one_pass && F::ALIAS && F1::ALIAS, k, Q, prec, "face kernel: one face point per thread");
    check(F::OUT_OFF == 0 && F::T1_OFF == F::OUT && F::OUT + F::T1 <= F::TOTAL, k, Q, prec, "face kernel: OUT then T1");
    check(F::TR_OFF == F::SW && F::SW + F::TR <= F::TOTAL, k, Q, prec, "face kernel: traces after the swept traces");
    check(F1::TOTAL <= F::TOTAL && F1::OUT_OFF == 0 && F1::T1_OFF == F1::OUT, k, Q, prec, "face kernel: wall face layout");
    check(FB::lds <= 160 * 1024, k, Q, prec, "face kernel LDS footprint");
    std::printf("k=%d n_q=%d %s: face kernel B=%d work=%d LDS=%d B\n", k, Q, prec, FB::threads, F::TOTAL, FB::lds);
}

template <int N, int Q, typename Real>
void plan() {
    constexpr int B = OpBlock<N, Q, Real>::threads;
    constexpr bool fused = OpBlock<N, Q, Real>::fused;
    constexpr bool split = OpBlock<N, Q, Real>::split;
    using S = OpSizes<N, Q, B, (int)sizeof(Real), fused, split>;
    using F = FaceSizes<N, Q, B, S::NF, fused>;
    const int k = N - 1, N3 = N * N * N;
    const char* prec = sizeof(Real) == 8 ? "fp64" : "fp32";
    check(B == 64 || B == 128 || B == 256, k, Q, prec, "block size");
    if constexpr (split) {
        // the operator kernel stages the six lifted face blocks, then runs the cell chunks,
        // body force and mass-matrix sweeps in the same work area
        check(S::P >= 1 && S::P <= Q, k, Q, prec, "planes per chunk");
        check(S::WORK >= S::CELL && S::WORK >= 60 * N * N && S::WORK >= 10 * N3, k, Q, prec, "work area (split)");
        const int bytes = (S::WORK + 10 * N3 + S::TABLES) * (int)sizeof(Real);
        check(bytes <= 160 * 1024, k, Q, prec, "LDS footprint");
        std::printf("k=%d n_q=%d %s: split, B=%d P=%d work=%d LDS=%d B\n", k, Q, prec, B, S::P, S::WORK, bytes);
        face_plan<N, Q, Real>(k, prec);
        return;
    }
    check(S::NF == 1 || S::NF == 3, k, Q, prec, "faces per group");
    check(S::P >= 1 && S::P <= Q, k, Q, prec, "planes per chunk");
    // the work area holds the cell chunk, the face group and the 2 x 5 N^3 of the mass
    // matrix and body-force sweeps
    check(S::WORK >= S::CELL && S::WORK >= F::TOTAL && S::WORK >= 10 * N3, k, Q, prec, "work area");
    if (F::ALIAS) {
        // SW | TR, then OUT | T1, then W | T1 (W written over OUT while T1 is read)
        check(S::NF * Q * Q <= B, k, Q, prec, "one pass of face points");
        check(F::TR_OFF == F::SW && F::SW + F::TR <= F::TOTAL, k, Q, prec, "traces after the swept traces");
        check(F::OUT_OFF == 0 && F::T1_OFF == F::OUT && F::OUT + F::T1 <= F::TOTAL, k, Q, prec, "OUT then T1");
        check(disjoint(F::OUT_OFF, F::W, F::T1_OFF, F::T1), k, Q, prec, "W clear of T1");
    } else {
        // R1 = {SW, T1} and R2 = {TR, OUT, W}: each phase reads one region and writes the other
        check(F::R1 >= F::SW && F::R1 >= F::T1, k, Q, prec, "region 1");
        check(F::R2 >= F::TR && F::R2 >= F::OUT && F::R2 >= F::W, k, Q, prec, "region 2");
        check(F::TR_OFF == F::R1 && F::OUT_OFF == F::R1 && F::T1_OFF == 0, k, Q, prec, "split offsets");
        check(F::R1 + F::R2 == F::TOTAL, k, Q, prec, "split total");
    }
    if (F::FUSED_TRACE) {
        // items of one side fill whole waves and the two sides fit the padded span
        constexpr int per_side = S::NF * 5 * N, span = (per_side + 63) / 64 * 64;
        check(span % 64 == 0 && per_side <= span, k, Q, prec, "fused trace items");
        check(F::TR == 0, k, Q, prec, "fused traces take no LDS");
    } else {
        check(F::TR == S::NF * 20 * N * N, k, Q, prec, "stored traces");
    }
    const int bytes = (S::WORK + 10 * N3 + S::TABLES) * (int)sizeof(Real);
    check(bytes <= 160 * 1024, k, Q, prec, "LDS footprint");
    std::printf("k=%d n_q=%d %s: B=%d NF=%d P=%d fused traces=%d work=%d LDS=%d B\n", k, Q, prec, B, S::NF, S::P,
                (int)fused, S::WORK, bytes);
}

template <int N, int Q>
void both() {
    plan<N, Q, double>();
    plan<N, Q, float>();
}

template <size_t I = 0>
void all() {
    constexpr size_t n = sizeof(kSupported) / sizeof(kSupported[0]);
    if constexpr (I < n) {
        both<kSupported[I][0] + 1, kSupported[I][1]>();
        all<I + 1>();
    }
}

int main() {
    all();
    if (g_fail) return 1;
    std::printf("all ok\n");
    return 0;
}
