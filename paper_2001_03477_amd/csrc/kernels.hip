// Small HIP kernels around the advection step: checksum column sums, field
// conversions and checks, and batched cell geometry for testing and reuse.
#include <hip/hip_runtime.h>

#include "common.h"

namespace pcv {

namespace {

// A thread's share of a column of nb block partials: sixteen strided accumulators while
// sixteen loads fit, then four, then one (loads in flight for long columns such as the
// per-cell-block partials of step 2), combined in a fixed tree.
__device__ __forceinline__ double column_partial(const double* __restrict__ P, int nb) {
    double v[16] = {};
    int b = threadIdx.x;
    for (; b + 15 * 256 < nb; b += 16 * 256)
#pragma unroll
        for (int u = 0; u < 16; ++u) v[u] += P[b + u * 256];
    for (; b + 3 * 256 < nb; b += 4 * 256)
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] += P[b + u * 256];
    for (; b < nb; b += 256) v[0] += P[b];
#pragma unroll
    for (int w = 8; w > 0; w >>= 1)
#pragma unroll
        for (int u = 0; u < w; ++u) v[u] += v[u + w];
    return v[0];
}

// Column sums of the quantity-major partial tables: block (q, slot) adds the nb[slot]
// block partials of quantity q in a fixed order (column_partial per thread, then a
// fixed tree).
__global__ void __launch_bounds__(256)
k_colsum(const double* __restrict__ part, long stride, int nb0, int nb1, int nb2, int nb3,
         double* __restrict__ colsum) {
    __shared__ double sm[256];
    const int q = blockIdx.x, slot = blockIdx.y;
    const int nb = slot == 0 ? nb0 : (slot == 1 ? nb1 : (slot == 2 ? nb2 : nb3));
    const double* P = part + ((long)slot * kPartialWidth + q) * stride;
    sm[threadIdx.x] = column_partial(P, nb);
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) colsum[slot * kPartialWidth + q] = sm[0];
}

// k_colsum for many domains: block (q, slot, i) sums quantity q of slot of domain i in
// the same order as k_colsum.
__global__ void __launch_bounds__(256) k_colsum_batch(const ColsumArgs* __restrict__ cs) {
    __shared__ double sm[256];
    const ColsumArgs c = cs[blockIdx.z];
    const int q = blockIdx.x, slot = blockIdx.y;
    const int nb = c.nb[slot];
    const double* P = c.part + ((long)slot * kPartialWidth + q) * c.stride;
    sm[threadIdx.x] = column_partial(P, nb);
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) c.colsum[slot * kPartialWidth + q] = sm[0];
}

__global__ void k_energy_from_T(Dom d, const double* __restrict__ c, const double* __restrict__ T,
                                double* __restrict__ e) {
    const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id < d.ncell) e[id] = cp_of(d, c[id]) * T[id];
}

__global__ void k_T_from_energy(Dom d, const double* __restrict__ c, const double* __restrict__ e,
                                double* __restrict__ T) {
    const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id < d.ncell) T[id] = e[id] / cp_of(d, c[id]);
}

__global__ void k_check(const double* __restrict__ x, long n, int check_range, unsigned int* flags) {
    unsigned int f = 0;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const double v = x[i];
        if (!isfinite(v)) f |= 1u;
        else if (check_range && (v < 0.0 || v > 1.0)) f |= 2u;
    }
    if (f) atomicOr(flags, f);
}

// max |x| over the block first, then one atomic per block
__global__ void __launch_bounds__(256) k_maxabs(const double* __restrict__ x, long n, unsigned long long* maxbits) {
    __shared__ double sm[4];
    double m = 0.0;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        m = fmax(m, fabs(x[i]));
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_down(m, off, 64));
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        m = fmax(fmax(sm[0], sm[1]), fmax(sm[2], sm[3]));
        if (m > 0.0) atomicMax(maxbits, (unsigned long long)__double_as_longlong(m));
    }
}

__global__ void k_to_float(long n, const double* __restrict__ in, float* __restrict__ out) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        out[i] = (float)in[i];
}

__global__ void k_periodic_faces(Dom d, int axis, const double* __restrict__ vel, unsigned int* flags) {
    // the transverse extent of the face planes of `axis`
    const int ta = axis == 0 ? 1 : 0, tb = axis == 2 ? 1 : 2;
    const long nt = (long)d.n[ta] * (d.ndim == 2 && tb == 2 ? 1 : d.n[tb]);
    for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < nt; t += (long)gridDim.x * blockDim.x) {
        int p[3] = {0, 0, 0};
        p[ta] = (int)(t % d.n[ta]);
        p[tb] = (int)(t / d.n[ta]);
        int q[3] = {p[0], p[1], p[2]};
        q[axis] = d.n[axis];
        if (vel[face_at(d, axis, p[0], p[1], p[2], 0)] != vel[face_at(d, axis, q[0], q[1], q[2], d.n[axis])])
            atomicOr(flags, 4u);
    }
}

__global__ void k_geom_volume(int n, const double* m, const double* a, double* out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = volume(m[3 * i], m[3 * i + 1], m[3 * i + 2], a[i]);
}
__global__ void k_geom_alpha(int n, const double* m, const double* c, double* out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = alpha_of(m[3 * i], m[3 * i + 1], m[3 * i + 2], c[i]);
}
__global__ void k_geom_slab(int n, const double* m, const double* a, const int* axis, const double* lam,
                            double* out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = slab(m[3 * i], m[3 * i + 1], m[3 * i + 2], a[i], axis[i], lam[i]);
}
__global__ void k_geom_normal(int n, const double* c27, int method, double* m) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double loc[27];
    for (int q = 0; q < 27; ++q) loc[q] = c27[27 * (long)i + q];
    const Normal r = normal27(loc, method);
    m[3 * i] = r.m[0];
    m[3 * i + 1] = r.m[1];
    m[3 * i + 2] = r.m[2];
}
__global__ void k_geom_weno5(int n, const double* v, double eps, double* out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double* p = v + 5 * (long)i;
    out[i] = weno5(p[0], p[1], p[2], p[3], p[4], eps);
}

dim3 linear_grid(long n, int bs) { return dim3((unsigned)((n + bs - 1) / bs)); }

}  // namespace

hipError_t launch_colsum(const double* part, long part_stride, const int* nb, double* colsum, hipStream_t s) {
    hipLaunchKernelGGL(k_colsum, dim3(kPartialWidth, kSlots), dim3(256), 0, s, part, part_stride, nb[0], nb[1],
                       nb[2], nb[3], colsum);
    return hipGetLastError();
}

hipError_t launch_colsum_batch(int nd, const ColsumArgs* cs, hipStream_t s) {
    hipLaunchKernelGGL(k_colsum_batch, dim3(kPartialWidth, kSlots, nd), dim3(256), 0, s, cs);
    return hipGetLastError();
}

hipError_t launch_energy_from_T(const Dom& d, const double* c, const double* T, double* e, hipStream_t s) {
    hipLaunchKernelGGL(k_energy_from_T, linear_grid(d.ncell, 256), dim3(256), 0, s, d, c, T, e);
    return hipGetLastError();
}

hipError_t launch_T_from_energy(const Dom& d, const double* c, const double* e, double* T, hipStream_t s) {
    hipLaunchKernelGGL(k_T_from_energy, linear_grid(d.ncell, 256), dim3(256), 0, s, d, c, e, T);
    return hipGetLastError();
}

hipError_t launch_check(const double* x, long n, int check_range, unsigned int* flags, hipStream_t s) {
    long nb = (n + 255) / 256;
    if (nb > 4096) nb = 4096;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_check, dim3((unsigned)nb), dim3(256), 0, s, x, n, check_range, flags);
    return hipGetLastError();
}

hipError_t launch_maxabs(const double* x, long n, unsigned long long* maxbits, hipStream_t s) {
    long nb = (n + 255) / 256;
    if (nb > 1024) nb = 1024;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_maxabs, dim3((unsigned)nb), dim3(256), 0, s, x, n, maxbits);
    return hipGetLastError();
}

hipError_t launch_to_float(long n, const double* in, float* out, hipStream_t s) {
    long nb = (n + 255) / 256;
    if (nb > 8192) nb = 8192;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_to_float, dim3((unsigned)nb), dim3(256), 0, s, n, in, out);
    return hipGetLastError();
}

hipError_t launch_periodic_faces(const Dom& d, int axis, const double* vel, unsigned int* flags,
                                 hipStream_t s) {
    hipLaunchKernelGGL(k_periodic_faces, dim3(256), dim3(256), 0, s, d, axis, vel, flags);
    return hipGetLastError();
}

hipError_t launch_geom_volume(int n, const double* m, const double* a, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_geom_volume, linear_grid(n, 256), dim3(256), 0, s, n, m, a, out);
    return hipGetLastError();
}
hipError_t launch_geom_alpha(int n, const double* m, const double* c, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_geom_alpha, linear_grid(n, 256), dim3(256), 0, s, n, m, c, out);
    return hipGetLastError();
}
hipError_t launch_geom_slab(int n, const double* m, const double* a, const int* axis, const double* lam,
                            double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_geom_slab, linear_grid(n, 256), dim3(256), 0, s, n, m, a, axis, lam, out);
    return hipGetLastError();
}
hipError_t launch_geom_normal(int n, const double* c27, int method, double* m, hipStream_t s) {
    hipLaunchKernelGGL(k_geom_normal, linear_grid(n, 256), dim3(256), 0, s, n, c27, method, m);
    return hipGetLastError();
}
hipError_t launch_geom_weno5(int n, const double* v, double eps, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_geom_weno5, linear_grid(n, 256), dim3(256), 0, s, n, v, eps, out);
    return hipGetLastError();
}

}  // namespace pcv
