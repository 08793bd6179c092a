// Device helpers shared by the kernels: ghost-cell index mapping, the one-fluid heat
// capacity, the mixed-cell test, the 3x3x3 gather and deterministic block sums.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "geom.h"
#include "kernels.h"

namespace pcv {

// Ghost rule per axis: periodic wrap, or outflow = copy of the nearest interior cell.
// Positions within one period of the domain (all that the stencils reach on grids of
// at least three cells) wrap with one correction; the loops only run on smaller grids.
__device__ __forceinline__ int wrap(int i, int n, int bc) {
    if (bc == 0) {
        if (i < 0) i += n;
        else if (i >= n) i -= n;
        if (i < 0 || i >= n) {
            while (i < 0) i += n;
            while (i >= n) i -= n;
        }
        return i;
    }
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

// One-fluid volumetric heat capacity C_p = C_pl c + C_pg (1 - c) (eq. c_vol_avg).
__device__ __forceinline__ double cp_of(const Dom& d, double c) { return d.cp_l * c + d.cp_g * (1.0 - c); }

// Mixed cell: eps < c < 1 - eps (section 3.1).
__device__ __forceinline__ bool mixed(const Dom& d, double c) { return c > d.eps && c < 1.0 - d.eps; }

// The 3x3x3 volume fractions around (x, y, z) (ghost positions allowed), fully
// unrolled so that they stay in registers: c27[(dz+1)*9 + (dy+1)*3 + (dx+1)].
__device__ __forceinline__ void gather27(const Dom& d, const double* __restrict__ c, int x, int y, int z,
                                         double (&c27)[27]) {
    int xs[3], ys[3], zs[3];
#pragma unroll
    for (int o = 0; o < 3; ++o) {
        xs[o] = wrap(x + o - 1, d.n[0], d.bc[0]);
        ys[o] = wrap(y + o - 1, d.n[1], d.bc[1]);
        zs[o] = d.ndim == 2 ? 0 : wrap(z + o - 1, d.n[2], d.bc[2]);
    }
#pragma unroll
    for (int dz = 0; dz < 3; ++dz)
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {
            const long row = ((long)zs[dz] * d.n[1] + ys[dy]) * d.n[0];
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) c27[dz * 9 + dy * 3 + dx] = c[row + xs[dx]];
        }
}

// Wavefront sum (result in lane 63) with DPP row shifts and row broadcasts, which
// move data between lanes inside the VALU instead of through LDS. Each step moves the
// two 32-bit halves of the double; lanes without a source read 0. The order of the
// additions is fixed, so the sum is deterministic.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    const int nlo = __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xf, 0xf, false);
    const int nhi = __builtin_amdgcn_update_dpp(0, hi, CTRL, 0xf, 0xf, false);
    return __hiloint2double(nhi, nlo);
}

__device__ __forceinline__ double wave_sum_lane63(double v) {
    v += dpp_move<0x111>(v);  // row_shr:1
    v += dpp_move<0x112>(v);  // row_shr:2
    v += dpp_move<0x114>(v);  // row_shr:4
    v += dpp_move<0x118>(v);  // row_shr:8: lane 15 of each row holds the row sum
    v += dpp_move<0x142>(v);  // row_bcast:15: row r gets lane 15 of row r-1
    v += dpp_move<0x143>(v);  // row_bcast:31: rows 2, 3 get lane 31
    return v;
}

// Sum of 8 per-thread values over a block of NWAVES wavefronts; thread q < 8 writes
// the total of quantity q to out[q * stride]. Fixed shapes, so deterministic. Bit q of
// skip (uniform over the wavefront) says that quantity q is +0 in every lane: its
// wavefront sum, +0, is then not computed.
template <int NWAVES>
__device__ __forceinline__ void block_sum8(const double (&v)[8], double* out, long stride, unsigned skip = 0) {
    __shared__ double red[8][NWAVES];
    const int tid = threadIdx.y * blockDim.x + threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    skip = __builtin_amdgcn_readfirstlane(skip);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        double s = 0.0;
        if (!(skip >> q & 1u)) s = wave_sum_lane63(v[q]);
        if (lane == 63) red[q][wave] = s;
    }
    __syncthreads();
    if (tid < 8) {
        double s = red[tid][0];
#pragma unroll
        for (int w = 1; w < NWAVES; ++w) s += red[tid][w];
        out[tid * stride] = s;
    }
}

// A pointer read from memory (a table of per-domain arguments) is generic to the
// compiler, which then accesses it with flat instructions: each counts as a
// vector-memory and as an LDS operation, so that every wait for one kind also waits for
// the other. Passed through a global-address-space pointer, which the empty asm keeps
// from being folded away, it is accessed with global instructions, like a kernel
// argument. The pointer must be wavefront-uniform and held in scalar registers.
template <typename T>
__device__ __forceinline__ T* in_global(T* p) {
    using G = __attribute__((address_space(1))) T*;
    G g = (G)p;
    __asm__("" : "+s"(g));
    return (T*)g;
}

// Bit of the mixed-cell mask for cell x of the row starting at word rowword.
__device__ __forceinline__ bool mask_bit(const uint64_t* __restrict__ mask, long rowword, int x) {
    return (mask[rowword + (x >> 6)] >> (x & 63)) & 1ull;
}

// Index of face f along axis of the face row through transverse cell coordinates.
__device__ __forceinline__ long face_at(const Dom& d, int axis, int x, int y, int z, int f) {
    if (axis == 0) return ((long)z * d.n[1] + y) * (d.n[0] + 1) + f;
    if (axis == 1) return ((long)z * (d.n[1] + 1) + f) * d.n[0] + x;
    return ((long)f * d.n[1] + y) * d.n[0] + x;
}

}  // namespace pcv
