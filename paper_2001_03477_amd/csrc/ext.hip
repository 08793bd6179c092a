// Liquid-velocity extension (section 3.3.1, eq. press_inv) on gfx950.
//
// The one-fluid velocity u carries the phase-change source m'' (1/rho_g - 1/rho_l)
// delta_Gamma in its divergence. The liquid velocity u_l = u + u~ removes it: on a
// sub-domain made of the mixed cells and their first and second gas neighbours (face
// steps through gas), with walls towards the liquid and a fixed pressure at the third
// gas neighbours (and at outflow boundaries), the Poisson problem
//   sum over non-wall faces of (phi_j - phi_i) / rho_f = S a_i,  S = m'' (1/rho_g - 1/rho_l),
// (phi = dt p~ / h, a_i the PLIC plane area in cell units, rho_f the mean of the two
// cells' rho(c)) is solved, and u~_f = -(phi_R - phi_L) / rho_f on the faces of the
// sub-domain.
//
// The steps: labels by three dilation passes; the unknowns compacted in cell order
// (block counts, one scan, scatter); the operator assembled per unknown (six neighbour
// slots); conjugate gradients on the symmetric positive definite form with the
// diagonal as preconditioner, every dot product a fixed-order reduction over block
// partials (deterministic); the face corrections. All floating point is double
// precision.
#include <hip/hip_runtime.h>

#include "common.h"
#include "ext.h"

namespace pcv {

namespace {

constexpr int kNeighbours = 6;

// Cell coordinates of the linear cell index id, in 32-bit unsigned arithmetic (the
// extension takes at most 2^31 - 1 cells).
__device__ __forceinline__ void cell_xyz(const Dom& d, long id, int& x, int& y, int& z) {
    const unsigned ui = (unsigned)id, nx = (unsigned)d.n[0], ny = (unsigned)d.n[1];
    x = (int)(ui % nx);
    const unsigned r = ui / nx;
    y = (int)(r % ny);
    z = (int)(r / ny);
}

// Face neighbour of cell (x, y, z) along axis in direction step (-1 or 1): its index,
// or -1 beyond an outflow boundary; periodic axes wrap.
__device__ __forceinline__ long neighbour(const Dom& d, int x, int y, int z, int axis, int step) {
    int q[3] = {x, y, z};
    const int n = d.n[axis];
    q[axis] += step;
    if (q[axis] < 0 || q[axis] >= n) {
        if (d.bc[axis] != 0) return -1;
        q[axis] = q[axis] < 0 ? q[axis] + n : q[axis] - n;
    }
    return ((long)q[2] * d.n[1] + q[1]) * d.n[0] + q[0];
}

__device__ __forceinline__ double rho_of(double rho_l, double rho_g, double c) {
    return rho_l * c + rho_g * (1.0 - c);
}

__device__ __forceinline__ bool unknown(int8_t l) { return l >= 0 && l <= 2; }

// dV/dalpha of the lower half (0 <= a <= S/2) of the volume function, regime by
// regime (the derivatives of the closed forms of geom.h).
__device__ double dvol_lower(const Sorted3& s, double a) {
    const double m1 = s.m1, m2 = s.m2, m3 = s.m3;
    if (a <= 0.0) return 0.0;
    if (a < m1) return a * a / (2.0 * m1 * m2 * m3);
    const double dq = 6.0 * a - 3.0 * m1;
    if (a < m2) return dq / (6.0 * m2 * m3);
    const double m12 = m1 + m2;
    if (m12 <= m3) {
        if (a < m12) {
            const double t = a - m2;
            return (dq - 3.0 * t * t / m1) / (6.0 * m2 * m3);
        }
        return 1.0 / m3;
    }
    const double t2 = a - m2;
    if (a < m3) return (dq - 3.0 * t2 * t2 / m1) / (6.0 * m2 * m3);
    const double t3 = a - m3;
    return (dq - 3.0 * (t2 * t2 + t3 * t3) / m1) / (6.0 * m2 * m3);
}

// Area of the plane m.x = alpha inside the unit cube: |m|_2 dV/dalpha.
__device__ double plane_area(double mx, double my, double mz, double alpha) {
    double a = alpha;
    if (mx < 0.0) a -= mx;
    if (my < 0.0) a -= my;
    if (mz < 0.0) a -= mz;
    const Sorted3 s = sort_abs(mx, my, mz);
    const double S = s.m1 + s.m2 + s.m3;
    if (a <= 0.0 || a >= S) return 0.0;
    const double dv = a <= 0.5 * S ? dvol_lower(s, a) : dvol_lower(s, S - a);
    return sqrt(mx * mx + my * my + mz * mz) * dv;
}

__global__ void __launch_bounds__(kExtBlock) k_ext_init(Dom d, const double* __restrict__ c, int8_t* __restrict__ lab) {
    for (long i = (long)blockIdx.x * kExtBlock + threadIdx.x; i < d.ncell; i += (long)gridDim.x * kExtBlock) {
        const double v = c[i];
        lab[i] = mixed(d, v) ? 0 : (v >= 1.0 - d.eps ? -1 : kExtFar);
    }
}

// Gas cells not yet labelled with a face neighbour of label k - 1 take label k. Cells
// labelled in this pass are only read for the value k - 1, which they never had, so
// the pass does not depend on the order of the threads.
__global__ void __launch_bounds__(kExtBlock) k_ext_dilate(Dom d, int8_t* __restrict__ lab, int k) {
    for (long i = (long)blockIdx.x * kExtBlock + threadIdx.x; i < d.ncell; i += (long)gridDim.x * kExtBlock) {
        if (lab[i] != kExtFar) continue;
        int x, y, z;
        cell_xyz(d, i, x, y, z);
        bool hit = false;
        for (int a = 0; a < d.ndim; ++a)
            for (int st = -1; st <= 1; st += 2) {
                const long j = neighbour(d, x, y, z, a, st);
                if (j >= 0 && lab[j] == k - 1) hit = true;
            }
        if (hit) lab[i] = (int8_t)k;
    }
}

// Unknowns of each run of kExtCells cells (one block walks its run in kExtBlock-cell
// pieces).
__global__ void __launch_bounds__(kExtBlock) k_ext_count(Dom d, const int8_t* __restrict__ lab, int* __restrict__ counts) {
    __shared__ int s_n[kExtBlock / 64];
    int nw = 0;
    for (int piece = 0; piece < kExtCells / kExtBlock; ++piece) {
        const long i = (long)blockIdx.x * kExtCells + piece * kExtBlock + threadIdx.x;
        nw += __popcll(__ballot(i < d.ncell && unknown(lab[i])));
    }
    if ((threadIdx.x & 63) == 0) s_n[threadIdx.x >> 6] = nw;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int w = 0; w < kExtBlock / 64; ++w) t += s_n[w];
        counts[blockIdx.x] = t;
    }
}

// Exclusive offsets of the run counts (one block walks them in chunks) and the total.
__global__ void __launch_bounds__(kExtScanBlock) k_ext_scan(const int* __restrict__ counts, int nb, int* __restrict__ offs,
                                                            int* __restrict__ total) {
    __shared__ int s_v[kExtScanBlock];
    int carry = 0;
    for (int base = 0; base < nb; base += kExtScanBlock) {
        const int i = base + (int)threadIdx.x;
        const int v = i < nb ? counts[i] : 0;
        s_v[threadIdx.x] = v;
        __syncthreads();
        // inclusive scan in LDS (Hillis-Steele)
        for (int off = 1; off < kExtScanBlock; off <<= 1) {
            const int add = threadIdx.x >= (unsigned)off ? s_v[threadIdx.x - off] : 0;
            __syncthreads();
            s_v[threadIdx.x] += add;
            __syncthreads();
        }
        if (i < nb) offs[i] = carry + s_v[threadIdx.x] - v;
        carry += s_v[kExtScanBlock - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = carry;
}

// list[offset + rank] = cell for the unknowns of each run, in cell order; map[cell] =
// its index (or -1).
__global__ void __launch_bounds__(kExtBlock) k_ext_scatter(Dom d, const int8_t* __restrict__ lab, const int* __restrict__ offs,
                                                           int* __restrict__ list, int* __restrict__ map) {
    __shared__ int s_n[kExtBlock / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int base = offs[blockIdx.x];
    for (int piece = 0; piece < kExtCells / kExtBlock; ++piece) {
        const long i = (long)blockIdx.x * kExtCells + piece * kExtBlock + threadIdx.x;
        const bool u = i < d.ncell && unknown(lab[i]);
        const unsigned long long b = __ballot(u);
        if (lane == 0) s_n[w] = __popcll(b);
        __syncthreads();
        int pos = base;
        for (int k = 0; k < w; ++k) pos += s_n[k];
        pos += __popcll(b & __lanemask_lt());
        if (i < d.ncell) {
            map[i] = u ? pos : -1;
            if (u) list[pos] = (int)i;
        }
        for (int k = 0; k < kExtBlock / 64; ++k) base += s_n[k];
        __syncthreads();  // s_n is rewritten by the next piece
    }
}

__global__ void __launch_bounds__(kExtBlock) k_ext_assemble(Dom d, const double* __restrict__ c, const double* __restrict__ mdot,
                                                            double rho_g, double S, int nu, const int8_t* __restrict__ lab,
                                                            const int* __restrict__ map, const int* __restrict__ list,
                                                            int* __restrict__ nbr, double* __restrict__ coef,
                                                            double* __restrict__ dg, double* __restrict__ g) {
    const int i = blockIdx.x * kExtBlock + threadIdx.x;
    if (i >= nu) return;
    const long id = list[i];
    int x, y, z;
    cell_xyz(d, id, x, y, z);
    const double ci = c[id];
    const double ri = rho_of(d.rho_l, rho_g, ci);
    double diag = 0.0;
    int slot = 0;
    for (int a = 0; a < d.ndim; ++a)
        for (int st = -1; st <= 1; st += 2, ++slot) {
            int nb = -1;
            double cf = 0.0;
            const long j = neighbour(d, x, y, z, a, st);
            if (j < 0) {  // outflow boundary: fixed pressure, the ghost is a copy
                diag -= 1.0 / ri;
            } else if (lab[j] != -1) {  // (liquid: a wall, no flux)
                const double f = 1.0 / (0.5 * (ri + rho_of(d.rho_l, rho_g, c[j])));
                diag -= f;
                if (unknown(lab[j])) {
                    nb = map[j];
                    cf = f;
                }
            }
            nbr[(long)i * kNeighbours + slot] = nb;
            coef[(long)i * kNeighbours + slot] = cf;
        }
    for (; slot < kNeighbours; ++slot) {
        nbr[(long)i * kNeighbours + slot] = -1;
        coef[(long)i * kNeighbours + slot] = 0.0;
    }
    double b = 0.0;
    const double m = mdot[id];
    if (lab[id] == 0 && m != 0.0) {
        double c27[27];
        gather27(d, c, x, y, z, c27);
        const Normal nm = normal27(c27, d.normal);
        const double alpha = alpha_of(nm.m[0], nm.m[1], nm.m[2], ci);
        b = m * S * plane_area(nm.m[0], nm.m[1], nm.m[2], alpha);
    }
    // the symmetric positive definite form: (-A) phi = -b
    dg[i] = -diag;
    g[i] = -b;
}

// Two partial sums of a block (thread 0 writes part[2 blk], part[2 blk + 1]).
__device__ __forceinline__ void block_sum2(double a, double b, double* part) {
    __shared__ double s_a[kExtBlock / 64], s_b[kExtBlock / 64];
    const double wa = wave_sum_lane63(a), wb = wave_sum_lane63(b);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 63) {
        s_a[w] = wa;
        s_b[w] = wb;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double ta = s_a[0], tb = s_b[0];
        for (int k = 1; k < kExtBlock / 64; ++k) {
            ta += s_a[k];
            tb += s_b[k];
        }
        part[2 * blockIdx.x] = ta;
        part[2 * blockIdx.x + 1] = tb;
    }
}

__global__ void __launch_bounds__(kExtBlock) k_cg_start(int nu, const double* __restrict__ g, const double* __restrict__ dg,
                                                        double* __restrict__ x, double* __restrict__ r,
                                                        double* __restrict__ z, double* __restrict__ p,
                                                        double* __restrict__ part) {
    const int i = blockIdx.x * kExtBlock + threadIdx.x;
    double rz = 0.0, rr = 0.0;
    if (i < nu) {
        const double ri = g[i];
        const double zi = dg[i] > 0.0 ? ri / dg[i] : 0.0;  // a cell with walls only: no unknown
        x[i] = 0.0;
        r[i] = ri;
        z[i] = zi;
        p[i] = zi;
        rz = ri * zi;
        rr = ri * ri;
    }
    block_sum2(rz, rr, part);
}

// The new direction p = z + beta p_old (at the unknown and, recomputed, at its
// neighbours: p_old and p are separate buffers), q = M p (M the symmetric positive
// definite operator) and the partials of p . q.
__global__ void __launch_bounds__(kExtBlock) k_cg_spmv(int nu, const double* __restrict__ scal, const int* __restrict__ nbr,
                                                       const double* __restrict__ coef, const double* __restrict__ dg,
                                                       const double* __restrict__ z, const double* __restrict__ p_old,
                                                       double* __restrict__ p, double* __restrict__ q,
                                                       double* __restrict__ part) {
    const int i = blockIdx.x * kExtBlock + threadIdx.x;
    double pq = 0.0;
    if (i < nu) {
        const double be = scal[kCgBeta];
        const double pi = fma(be, p_old[i], z[i]);  // the same rounding as at the neighbours
        double s = dg[i] * pi;
#pragma unroll
        for (int k = 0; k < kNeighbours; ++k) {
            const int j = nbr[(long)i * kNeighbours + k];
            if (j >= 0) s -= coef[(long)i * kNeighbours + k] * fma(be, p_old[j], z[j]);
        }
        p[i] = pi;
        q[i] = s;
        pq = pi * s;
    }
    block_sum2(pq, 0.0, part);
}

// Fixed-order sums of nb pairs of block partials: every thread of the block gets the
// same totals (the same order in every block and in k_cg_reduce).
__device__ __forceinline__ void sum_pairs(const double* __restrict__ part, int nb, double& ta, double& tb) {
    double a = 0.0, b = 0.0;
    for (int k = threadIdx.x; k < nb; k += kExtBlock) {
        a += part[2 * k];
        b += part[2 * k + 1];
    }
    __shared__ double s_a[kExtBlock / 64], s_b[kExtBlock / 64];
    const double wa = wave_sum_lane63(a), wb = wave_sum_lane63(b);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 63) {
        s_a[w] = wa;
        s_b[w] = wb;
    }
    __syncthreads();
    ta = s_a[0];
    tb = s_b[0];
    for (int k = 1; k < kExtBlock / 64; ++k) {
        ta += s_a[k];
        tb += s_b[k];
    }
}

// alpha = rz / p.q from the product's partials (each block sums them itself), then
// x += alpha p, r -= alpha q, z = r / diag and the partials of r . z, r . r.
__global__ void __launch_bounds__(kExtBlock) k_cg_update(int nu, const double* __restrict__ scal,
                                                         const double* __restrict__ part_pq, int nb,
                                                         const double* __restrict__ p, const double* __restrict__ q,
                                                         const double* __restrict__ dg, double* __restrict__ x,
                                                         double* __restrict__ r, double* __restrict__ z,
                                                         double* __restrict__ part) {
    double pq, unused;
    sum_pairs(part_pq, nb, pq, unused);
    const double al = pq > 0.0 ? scal[kCgRz] / pq : 0.0;
    const int i = blockIdx.x * kExtBlock + threadIdx.x;
    double rz = 0.0, rr = 0.0;
    if (i < nu) {
        x[i] += al * p[i];
        const double ri = r[i] - al * q[i];
        const double zi = dg[i] > 0.0 ? ri / dg[i] : 0.0;
        r[i] = ri;
        z[i] = zi;
        rz = ri * zi;
        rr = ri * ri;
    }
    block_sum2(rz, rr, part);
}

// Sums the nb pairs of partials in a fixed order and updates the scalars: mode 0 after
// the start (rz, rr, gg = rr, beta = 0), otherwise after the update (beta = rz' / rz,
// rz = rz', rr).
__global__ void __launch_bounds__(kExtBlock) k_cg_reduce(const double* __restrict__ part, int nb, double* __restrict__ scal,
                                                         int mode) {
    double ta, tb;
    sum_pairs(part, nb, ta, tb);
    if (threadIdx.x != 0) return;
    if (mode == 0) {
        scal[kCgRz] = ta;
        scal[kCgRr] = tb;
        scal[kCgGg] = tb;
        scal[kCgBeta] = 0.0;
    } else {
        scal[kCgBeta] = scal[kCgRz] > 0.0 ? ta / scal[kCgRz] : 0.0;
        scal[kCgRz] = ta;
        scal[kCgRr] = tb;
    }
}

// The correction of face i of axis; returns the new velocity.
template <typename T>
__device__ __forceinline__ double face_update(const Dom& d, int axis, long i, const double* __restrict__ c, double rho_g,
                                              const int8_t* __restrict__ lab, const int* __restrict__ map,
                                              const double* __restrict__ phi, T* __restrict__ vel,
                                              double* __restrict__ du) {
    const long nx = d.n[0], ny = d.n[1];
    // the face's coordinates in 32-bit unsigned arithmetic (far cheaper than 64-bit
    // division): the extension takes at most 2^31 - 1 cells, so fewer than 2^32 faces
    const unsigned ui = (unsigned)i, ux = (unsigned)nx, uy = (unsigned)ny;
    int q[3], f;
    if (axis == 0) {
        f = (int)(ui % (ux + 1u));
        const unsigned r = ui / (ux + 1u);
        q[1] = (int)(r % uy);
        q[2] = (int)(r / uy);
    } else if (axis == 1) {
        q[0] = (int)(ui % ux);
        const unsigned r = ui / ux;
        f = (int)(r % (uy + 1u));
        q[2] = (int)(r / (uy + 1u));
    } else {
        q[0] = (int)(ui % ux);
        const unsigned r = ui / ux;
        q[1] = (int)(r % uy);
        f = (int)(r / uy);
    }
    const int n = d.n[axis];
    const bool per = d.bc[axis] == 0;
    long L = -1, R = -1;
    {
        int qa[3] = {q[0], q[1], q[2]};
        if (f >= 1 || per) {
            qa[axis] = f >= 1 ? f - 1 : n - 1;
            L = ((long)qa[2] * ny + qa[1]) * nx + qa[0];
        }
        if (f < n || per) {
            qa[axis] = f < n ? f : 0;
            R = ((long)qa[2] * ny + qa[1]) * nx + qa[0];
        }
    }
    const int8_t lL = L >= 0 ? lab[L] : kExtFar, lR = R >= 0 ? lab[R] : kExtFar;
    const bool inL = L >= 0 && unknown(lL), inR = R >= 0 && unknown(lR);
    double v = 0.0;
    if ((inL || inR) && lL != -1 && lR != -1) {
        const double rL = rho_of(d.rho_l, rho_g, c[L >= 0 ? L : R]);
        const double rR = rho_of(d.rho_l, rho_g, c[R >= 0 ? R : L]);
        const double pL = inL ? phi[map[L]] : 0.0;
        const double pR = inR ? phi[map[R]] : 0.0;
        v = -(pR - pL) / (0.5 * (rL + rR));
    }
    const double u0 = (double)vel[i];
    if (du) du[i] = v;
    if (v == 0.0) return u0;
    const double u1 = u0 + v;
    vel[i] = (T)u1;
    return u1;
}

// Face f of axis between cells L = f - 1 and R = f (periodic axes: face n is face 0):
// the stored velocity becomes u + u~ in place, du (if not null) receives u~, and the
// largest |u + u~| of the block goes into *maxbits (atomic max of the bit pattern of a
// non-negative double).
template <typename T>
__global__ void __launch_bounds__(kExtBlock) k_ext_faces(Dom d, int axis, long nf, const double* __restrict__ c,
                                                         double rho_g, const int8_t* __restrict__ lab,
                                                         const int* __restrict__ map, const double* __restrict__ phi,
                                                         T* __restrict__ vel, double* __restrict__ du,
                                                         unsigned long long* __restrict__ maxbits) {
    __shared__ double s_m[kExtBlock / 64];
    double mx = 0.0;
    // grid-stride over the faces: few blocks, so that few atomics meet on *maxbits
    for (long i = (long)blockIdx.x * kExtBlock + threadIdx.x; i < nf; i += (long)gridDim.x * kExtBlock)
        mx = fmax(mx, fabs(face_update(d, axis, i, c, rho_g, lab, map, phi, vel, du)));
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_down(mx, off, 64));
    if ((threadIdx.x & 63) == 0) s_m[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kExtBlock / 64; ++w) mx = fmax(mx, s_m[w]);
        if (mx > 0.0) atomicMax(maxbits, (unsigned long long)__double_as_longlong(mx));
    }
}


constexpr int kExtFaceBlocks = 2048;  // grid of the face pass (eight blocks per compute unit)

int blocks_for(long n) { return (int)((n + kExtBlock - 1) / kExtBlock); }
int runs_for(long n) { return (int)((n + kExtCells - 1) / kExtCells); }

}  // namespace

ExtLayout ext_layout(const Dom& d, long max_faces) {
    ExtLayout L;
    const size_t n = (size_t)d.ncell;
    const size_t nb = (size_t)blocks_for(d.ncell);
    const size_t nr = (size_t)runs_for(d.ncell);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = (off + bytes + 255) & ~(size_t)255;
        return at;
    };
    L.lab = take(n);
    L.map = take(n * sizeof(int));
    L.list = take(n * sizeof(int));
    L.counts = take(nr * sizeof(int));
    L.offs = take(nr * sizeof(int));
    L.total = take(sizeof(int));
    L.nbr = take(n * kNeighbours * sizeof(int));
    L.coef = take(n * kNeighbours * sizeof(double));
    L.dg = take(n * sizeof(double));
    L.g = take(n * sizeof(double));
    for (int k = 0; k < 6; ++k) L.vec[k] = take(n * sizeof(double));
    L.part = take(2 * nb * sizeof(double));
    L.part2 = take(2 * nb * sizeof(double));
    L.scal = take(kCgScalars * sizeof(double));
    L.du = take((size_t)max_faces * sizeof(double));
    L.bytes = off;
    return L;
}

ExtIO ext_views(const ExtLayout& L, void* ws) {
    char* b = (char*)ws;
    ExtIO io;
    io.lab = (int8_t*)(b + L.lab);
    io.map = (int*)(b + L.map);
    io.list = (int*)(b + L.list);
    io.counts = (int*)(b + L.counts);
    io.offs = (int*)(b + L.offs);
    io.total = (int*)(b + L.total);
    io.nbr = (int*)(b + L.nbr);
    io.coef = (double*)(b + L.coef);
    io.dg = (double*)(b + L.dg);
    io.g = (double*)(b + L.g);
    io.x = (double*)(b + L.vec[0]);
    io.r = (double*)(b + L.vec[1]);
    io.z = (double*)(b + L.vec[2]);
    io.p = (double*)(b + L.vec[3]);
    io.q = (double*)(b + L.vec[4]);
    io.p2 = (double*)(b + L.vec[5]);
    io.part = (double*)(b + L.part);
    io.part2 = (double*)(b + L.part2);
    io.scal = (double*)(b + L.scal);
    io.du = (double*)(b + L.du);
    return io;
}

hipError_t launch_ext_labels(const Dom& d, const double* c, const ExtIO& io, hipStream_t s) {
    const int nb = blocks_for(d.ncell);
    const int ng = nb < 8192 ? nb : 8192;  // grid-stride kernels
    const int nr = runs_for(d.ncell);
    hipLaunchKernelGGL(k_ext_init, dim3(ng), dim3(kExtBlock), 0, s, d, c, io.lab);
    for (int k = 1; k <= 3; ++k) hipLaunchKernelGGL(k_ext_dilate, dim3(ng), dim3(kExtBlock), 0, s, d, io.lab, k);
    hipLaunchKernelGGL(k_ext_count, dim3(nr), dim3(kExtBlock), 0, s, d, io.lab, io.counts);
    hipLaunchKernelGGL(k_ext_scan, dim3(1), dim3(kExtScanBlock), 0, s, io.counts, nr, io.offs, io.total);
    hipLaunchKernelGGL(k_ext_scatter, dim3(nr), dim3(kExtBlock), 0, s, d, io.lab, io.offs, io.list, io.map);
    return hipGetLastError();
}

hipError_t launch_ext_assemble(const Dom& d, const double* c, const double* mdot, double rho_g, int nu,
                               const ExtIO& io, hipStream_t s) {
    if (nu <= 0) return hipSuccess;
    const double S = 1.0 / rho_g - 1.0 / d.rho_l;
    hipLaunchKernelGGL(k_ext_assemble, dim3(blocks_for(nu)), dim3(kExtBlock), 0, s, d, c, mdot, rho_g, S, nu,
                       io.lab, io.map, io.list, io.nbr, io.coef, io.dg, io.g);
    return hipGetLastError();
}

hipError_t launch_cg_start(int nu, const ExtIO& io, hipStream_t s) {
    const int nb = blocks_for(nu);
    hipLaunchKernelGGL(k_cg_start, dim3(nb), dim3(kExtBlock), 0, s, nu, io.g, io.dg, io.x, io.r, io.z, io.p, io.part);
    hipLaunchKernelGGL(k_cg_reduce, dim3(1), dim3(kExtBlock), 0, s, io.part, nb, io.scal, 0);
    return hipGetLastError();
}

hipError_t launch_cg_iteration(int nu, int iter, const ExtIO& io, hipStream_t s) {
    const int nb = blocks_for(nu);
    // the direction of iteration iter (1, 2, ...) goes to p2 for odd iter, p for even;
    // the first reads the start's p = z (with beta = 0)
    double* p_new = (iter & 1) ? io.p2 : io.p;
    const double* p_old = (iter & 1) ? io.p : io.p2;
    hipLaunchKernelGGL(k_cg_spmv, dim3(nb), dim3(kExtBlock), 0, s, nu, io.scal, io.nbr, io.coef, io.dg, io.z, p_old,
                       p_new, io.q, io.part);
    hipLaunchKernelGGL(k_cg_update, dim3(nb), dim3(kExtBlock), 0, s, nu, io.scal, io.part, nb, p_new, io.q, io.dg,
                       io.x, io.r, io.z, io.part2);
    hipLaunchKernelGGL(k_cg_reduce, dim3(1), dim3(kExtBlock), 0, s, io.part2, nb, io.scal, 2);
    return hipGetLastError();
}

hipError_t launch_ext_faces(const Dom& d, int axis, const double* c, double rho_g, void* vel, int mixed, double* du,
                            unsigned long long* maxbits, const ExtIO& io, hipStream_t s) {
    long nf;
    if (axis == 0) nf = (long)(d.n[0] + 1) * d.n[1] * d.n[2];
    else if (axis == 1) nf = (long)d.n[0] * (d.n[1] + 1) * d.n[2];
    else nf = (long)d.n[0] * d.n[1] * (d.n[2] + 1);
    const int nb = blocks_for(nf) < kExtFaceBlocks ? blocks_for(nf) : kExtFaceBlocks;
    if (mixed)
        hipLaunchKernelGGL(k_ext_faces<float>, dim3(nb), dim3(kExtBlock), 0, s, d, axis, nf, c, rho_g, io.lab,
                           io.map, io.x, (float*)vel, du, maxbits);
    else
        hipLaunchKernelGGL(k_ext_faces<double>, dim3(nb), dim3(kExtBlock), 0, s, d, axis, nf, c, rho_g, io.lab,
                           io.map, io.x, (double*)vel, du, maxbits);
    return hipGetLastError();
}

}  // namespace pcv
