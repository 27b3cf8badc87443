// Test-only stand-in for <hip/hip_runtime.h> that lets the kernel templates of
// paper_1806_03095_amd/csrc compile as ordinary host C++ (g++), so that their
// indexing and arithmetic can be checked on the CPU against the oracle.
//
// Each workgroup is emulated by blockDim.x host threads (the block size the
// launch asks for) that run the kernel body concurrently: threadIdx is
// thread-local, __shared__ arrays become static locals (one copy shared by the
// threads of the block), and __syncthreads() is a barrier of those threads.
// Workgroups run one after another.  A kernel whose threads do not all reach the
// same barriers deadlocks here, which the test's time limit reports.
#pragma once

#include <cmath>
#include <condition_variable>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <thread>
#include <vector>

struct dim3 {
    unsigned x, y, z;
    dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
struct EmuIdx {
    unsigned x = 0, y = 0, z = 0;
};
inline thread_local EmuIdx threadIdx;
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
#define amdgpu_waves_per_eu(...)   // AMDGPU register-allocation attribute: meaningless on the host
#define __shared__ static
#define __restrict__
// Reusable barrier of the emulated workgroup's threads.
struct EmuBarrier {
    std::mutex m;
    std::condition_variable cv;
    unsigned n = 1, count = 0, gen = 0;
    void reset(unsigned nthreads) {
        n = nthreads;
        count = 0;
    }
    void wait() {
        std::unique_lock<std::mutex> lock(m);
        const unsigned g = gen;
        if (++count == n) {
            count = 0;
            ++gen;
            cv.notify_all();
        } else {
            cv.wait(lock, [&] { return gen != g; });
        }
    }
};
inline EmuBarrier emu_barrier;
#define __syncthreads() emu_barrier.wait()

using std::fabs;
using std::sqrt;

#define hipLaunchKernelGGL(kernel, grid, block, shm, stream, ...)                  \
    do {                                                                            \
        const dim3 _g = dim3(grid), _blk = dim3(block);                             \
        blockDim.x = _blk.x;                                                        \
        for (unsigned _b = 0; _b < _g.x; ++_b) {                                    \
            blockIdx.x = _b;                                                        \
            emu_barrier.reset(_blk.x);                                              \
            std::vector<std::thread> _th;                                           \
            for (unsigned _t = 0; _t < _blk.x; ++_t)                                \
                _th.emplace_back([&, _t] {                                          \
                    threadIdx.x = _t;                                               \
                    kernel(__VA_ARGS__);                                            \
                });                                                                 \
            for (auto& _x : _th) _x.join();                                         \
        }                                                                           \
    } while (0)
