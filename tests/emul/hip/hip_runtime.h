// Test-only stand-in for <hip/hip_runtime.h> that lets the kernel templates of
// paper_1806_03095_amd/csrc compile as ordinary host C++ (g++), so that their
// indexing and arithmetic can be checked on the CPU against the oracle.
//
// Each workgroup is emulated by ONE thread (blockDim.x == 1): every cooperative
// loop "for (it = threadIdx.x; it < n; it += blockDim.x)" then visits all of its
// items, and __syncthreads() is a no-op.  Because the kernels only exchange data
// between phases separated by barriers, this sequential execution computes the
// same values as the parallel one.  __shared__ arrays become static locals.
#pragma once

#include <cmath>
#include <cstdint>
#include <cstring>

struct dim3 {
    unsigned x, y, z;
    dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
struct EmuIdx {
    unsigned x = 0, y = 0, z = 0;
};
inline EmuIdx threadIdx;
inline EmuIdx blockIdx;
inline EmuIdx blockDim{1, 1, 1};
inline EmuIdx gridDim{1, 1, 1};

typedef void* hipStream_t;
typedef int hipError_t;
constexpr hipError_t hipSuccess = 0;
inline hipError_t hipGetLastError() { return hipSuccess; }
inline const char* hipGetErrorString(hipError_t) { return "emulated"; }

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(x)
#define __shared__ static
#define __restrict__
#define __syncthreads() ((void)0)

using std::fabs;
using std::sqrt;

#define hipLaunchKernelGGL(kernel, grid, block, shm, stream, ...)            \
    do {                                                                      \
        const dim3 _g(grid);                                                  \
        for (unsigned _b = 0; _b < _g.x; ++_b) {                              \
            blockIdx.x = _b;                                                  \
            threadIdx.x = 0;                                                  \
            blockDim.x = 1;                                                   \
            kernel(__VA_ARGS__);                                              \
        }                                                                     \
    } while (0)
