// TEST INFRASTRUCTURE, not part of the library. A host stand-in for the HIP runtime
// header, used only by tests/test_host_mass_flux.py: it lets g++ compile the library's
// mass-flux kernel source unchanged and run each kernel as a host function over its
// launch grid, one block and thread after another, so that AddressSanitizer can check
// every access. The library itself is built with hipcc for gfx950 only.
#pragma once
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
using std::min;
using std::max;
struct dim3 {
    unsigned x, y, z;
    dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
extern thread_local dim3 threadIdx, blockIdx, blockDim, gridDim;
#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(x)
#define __shared__ static
typedef int hipError_t;
typedef void* hipStream_t;
typedef void* hipEvent_t;
enum { hipSuccess = 0 };
inline hipError_t hipGetLastError() { return 0; }
inline int __double2loint(double v) { int64_t b; memcpy(&b, &v, 8); return (int)(b & 0xffffffff); }
inline int __double2hiint(double v) { int64_t b; memcpy(&b, &v, 8); return (int)(b >> 32); }
inline double __hiloint2double(int hi, int lo) { int64_t b = ((int64_t)hi << 32) | (uint32_t)lo; double v; memcpy(&v, &b, 8); return v; }
#define __builtin_amdgcn_update_dpp(old, src, ctrl, rm, bm, bc) (src)
#define __builtin_amdgcn_readfirstlane(x) (x)
inline unsigned long long __ballot(int) { return 0; }
inline void __syncthreads() {}
#define hipLaunchKernelGGL(k, g, b, sh, s, ...)                                                   \
    do {                                                                                         \
        const dim3 G_(g), B_(b);                                                                 \
        gridDim = G_;                                                                            \
        blockDim = B_;                                                                           \
        for (unsigned bz = 0; bz < G_.z; ++bz)                                                   \
            for (unsigned by = 0; by < G_.y; ++by)                                               \
                for (unsigned bx = 0; bx < G_.x; ++bx)                                           \
                    for (unsigned tz = 0; tz < B_.z; ++tz)                                       \
                        for (unsigned ty = 0; ty < B_.y; ++ty)                                   \
                            for (unsigned tx = 0; tx < B_.x; ++tx) {                             \
                                blockIdx = dim3(bx, by, bz);                                     \
                                threadIdx = dim3(tx, ty, tz);                                    \
                                k(__VA_ARGS__);                                                  \
                            }                                                                    \
    } while (0)
