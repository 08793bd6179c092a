// HIP kernels of the advection step on gfx950: the step prologue, the direction
// sweeps (section 3.3.1 with the energy fluxes of section 3.4.1), step 2 with the
// latent correction (section 3.3.2, section 3.4.1), the checksum reduction, and
// small field utilities.
//
// All floating point is double precision and is compiled without contraction, so
// that every value that feeds a decision (mixed-cell test, donor side, the normal
// estimator's candidate selection, the dilatation flag) is evaluated exactly as
// specified. Reductions are deterministic: fixed-shape block trees and a fixed-order
// second pass.
#include <hip/hip_runtime.h>

#include "geom.h"
#include "kernels.h"

namespace pcv {

namespace {

constexpr int kBX = 64;  // one wavefront along x
constexpr int kBY = 4;   // four wavefronts per block

__device__ __forceinline__ int wrap(int i, int n, int bc) {
    if (bc == 0) {
        while (i < 0) i += n;
        while (i >= n) i -= n;
        return i;
    }
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

// Linear index of the (ghost-mapped) cell at (x, y, z).
__device__ __forceinline__ long cell_index(const Dom& d, int x, int y, int z) {
    const int i = wrap(x, d.n[0], d.bc[0]);
    const int j = wrap(y, d.n[1], d.bc[1]);
    const int k = d.ndim == 2 ? 0 : wrap(z, d.n[2], d.bc[2]);
    return ((long)k * d.n[1] + j) * d.n[0] + i;
}

__device__ __forceinline__ long face_index(const Dom& d, int axis, int x, int y, int z) {
    if (axis == 0) return ((long)z * d.n[1] + y) * (d.n[0] + 1) + x;
    if (axis == 1) return ((long)z * (d.n[1] + 1) + y) * d.n[0] + x;
    return ((long)z * d.n[1] + y) * d.n[0] + x;
}

__device__ __forceinline__ double cp_of(const Dom& d, double c) {
    return d.cp_l * c + d.cp_g * (1.0 - c);
}

__device__ __forceinline__ bool mixed(const Dom& d, double c) {
    return c > d.eps && c < 1.0 - d.eps;
}

__device__ void gather27(const Dom& d, const double* __restrict__ c, int x, int y, int z, double* c27) {
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx)
                c27[(dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)] = c[cell_index(d, x + dx, y + dy, z + dz)];
}

// Sum of 8 per-thread values over the block (256 threads), written by thread 0.
__device__ void block_sum8(const double (&v)[8], double* out) {
    __shared__ double red[8][kBX * kBY / 64];
    const int tid = threadIdx.y * blockDim.x + threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    for (int q = 0; q < 8; ++q) {
        double s = v[q];
        for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
        if (lane == 0) red[q][wave] = s;
    }
    __syncthreads();
    if (tid < 8) {
        double s = 0.0;
        for (int w = 0; w < kBX * kBY / 64; ++w) s += red[tid][w];
        out[tid] = s;
    }
}

// Liquid volume flux Phi and energy flux E through the face of `axis` whose right
// cell is at pos, for face CFL number lam (section 3.3.1 and section 3.4.1).
__device__ void face_flux(const Dom& d, int axis, const double* __restrict__ c,
                          const double* __restrict__ e, double lam, const int* pos, double& Phi,
                          double& E) {
    Phi = 0.0;
    E = 0.0;
    if (lam == 0.0) return;
    int dp[3] = {pos[0], pos[1], pos[2]};
    if (lam > 0.0) dp[axis] -= 1;
    const double cd = c[cell_index(d, dp[0], dp[1], dp[2])];
    const double L = fabs(lam);
    double F;
    if (mixed(d, cd)) {
        double c27[27];
        gather27(d, c, dp[0], dp[1], dp[2], c27);
        const Normal nm = normal27(c27, d.normal);
        const double alpha = alpha_of(nm.m[0], nm.m[1], nm.m[2], cd);
        F = slab(nm.m[0], nm.m[1], nm.m[2], alpha, axis, lam);
    } else {
        F = L * cd;
    }
    double T[5];
    for (int s = 0; s < 5; ++s) {
        int q[3] = {pos[0], pos[1], pos[2]};
        q[axis] += lam > 0.0 ? (s - 3) : (2 - s);
        const long id = cell_index(d, q[0], q[1], q[2]);
        T[s] = e[id] / cp_of(d, c[id]);
    }
    const double Tf = weno5(T[0], T[1], T[2], T[3], T[4], d.weno_eps);
    const double sg = lam > 0.0 ? 1.0 : -1.0;
    Phi = sg * F;
    E = sg * ((d.cp_l * F + d.cp_g * (L - F)) * Tf);
}

__global__ void __launch_bounds__(kBX* kBY)
k_prologue(Dom d, const double* __restrict__ c, const double* __restrict__ e,
           uint8_t* __restrict__ cc, double* __restrict__ ec) {
    const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= d.ncell) return;
    const double cv = c[id];
    const double T = e[id] / cp_of(d, cv);
    const bool liquid = cv >= 0.5;
    cc[id] = liquid ? 1 : 0;
    ec[id] = (liquid ? d.cp_l : d.cp_g) * T;
}

template <int AX>
__global__ void __launch_bounds__(kBX* kBY)
k_sweep(Dom d, const double* __restrict__ c, const double* __restrict__ e,
        const uint8_t* __restrict__ cc, const double* __restrict__ ec,
        const double* __restrict__ vel, double kfac, double* __restrict__ c_out,
        double* __restrict__ e_out, double* __restrict__ part) {
    const int x = blockIdx.x * kBX + threadIdx.x;
    const int y = blockIdx.y * kBY + threadIdx.y;
    const int z = blockIdx.z;
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (x < d.n[0] && y < d.n[1]) {
        int pos[3] = {x, y, z};
        int posR[3] = {x, y, z};
        posR[AX] += 1;
        const double lamL = vel[face_index(d, AX, pos[0], pos[1], pos[2])] * kfac;
        const double lamR = vel[face_index(d, AX, posR[0], posR[1], posR[2])] * kfac;
        double PhiL, EL, PhiR, ER;
        face_flux(d, AX, c, e, lamL, pos, PhiL, EL);
        face_flux(d, AX, c, e, lamR, posR, PhiR, ER);
        const long id = ((long)z * d.n[1] + y) * d.n[0] + x;
        const double dl = lamR - lamL;
        const double flag = (double)cc[id];
        double cn = c[id] - (PhiR - PhiL) + flag * dl;
        double en = e[id] - (ER - EL) + ec[id] * dl;
        acc[4] = flag * dl;
        acc[5] = ec[id] * dl;
        if (cn < 0.0 || cn > 1.0) {
            const double T = en / cp_of(d, cn);
            const double cl = cn < 0.0 ? 0.0 : 1.0;
            const double el = en + (d.cp_l - d.cp_g) * (cl - cn) * T;
            acc[0] = cl - cn;
            acc[1] = el - en;
            cn = cl;
            en = el;
        }
        c_out[id] = cn;
        e_out[id] = en;
        if (d.bc[AX] == 1) {
            if (pos[AX] == 0) {
                acc[2] -= PhiL;
                acc[3] -= EL;
            }
            if (pos[AX] == d.n[AX] - 1) {
                acc[2] += PhiR;
                acc[3] += ER;
            }
        }
        acc[6] = cn;
        acc[7] = en;
    }
    const long blk = ((long)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    block_sum8(acc, part + blk * kPartialWidth);
}

// Step 2, first pass: the reconstruction and the moved plane constant of every mixed
// cell with a non-zero mass flux (section 3.3.2): rec = (m, alpha~, alpha*).
__global__ void __launch_bounds__(kBX* kBY)
k_phase_recon(Dom d, const double* __restrict__ c, const double* __restrict__ mdot, double dt_h,
              double* __restrict__ rec) {
    const int x = blockIdx.x * kBX + threadIdx.x;
    const int y = blockIdx.y * kBY + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= d.n[0] || y >= d.n[1]) return;
    const long id = ((long)z * d.n[1] + y) * d.n[0] + x;
    const double md = mdot[id];
    const double cv = c[id];
    if (md == 0.0 || !mixed(d, cv)) return;
    double c27[27];
    gather27(d, c, x, y, z, c27);
    const Normal nm = normal27(c27, d.normal);
    const double alpha = alpha_of(nm.m[0], nm.m[1], nm.m[2], cv);
    const double dd = -(md / d.rho_l) * dt_h;
    const double norm2 = sqrt(nm.m[0] * nm.m[0] + nm.m[1] * nm.m[1] + nm.m[2] * nm.m[2]);
    double* r = rec + 5 * id;
    r[0] = nm.m[0];
    r[1] = nm.m[1];
    r[2] = nm.m[2];
    r[3] = alpha;
    r[4] = alpha + norm2 * dd;
}

// Step 2, second pass: a moving cell takes V(m, alpha*) (the motion capped at the cell
// bounds); a pure cell that a neighbour's plane advances into (liquid for
// evaporation, gas for condensation) takes the volume the extended plane sweeps in
// it, averaged over those neighbours; then the latent correction
// Delta e = Delta c (C_pl - C_pg) T_Gamma (section 3.4.1).
__global__ void __launch_bounds__(kBX* kBY)
k_phase_apply(Dom d, const double* __restrict__ c, const double* __restrict__ e,
              const double* __restrict__ mdot, double dt_h, const double* __restrict__ rec,
              double* __restrict__ c_out, double* __restrict__ e_out, double* __restrict__ part) {
    const int x = blockIdx.x * kBX + threadIdx.x;
    const int y = blockIdx.y * kBY + threadIdx.y;
    const int z = blockIdx.z;
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (x < d.n[0] && y < d.n[1]) {
        const long id = ((long)z * d.n[1] + y) * d.n[0] + x;
        const double cj = c[id];
        double cnew = cj;
        if (mixed(d, cj)) {
            if (mdot[id] != 0.0) {
                const double* r = rec + 5 * id;
                cnew = volume(r[0], r[1], r[2], r[4]);
            }
        } else {
            const double want = cj >= 1.0 - d.eps ? -1.0 : 1.0;
            double sum = 0.0;
            int cnt = 0;
            const int pos[3] = {x, y, z};
            for (int k = 0; k < d.ndim; ++k)
                for (int s = -1; s <= 1; s += 2) {
                    int q[3] = {pos[0], pos[1], pos[2]};
                    q[k] += s;
                    if (d.bc[k] == 1 && (q[k] < 0 || q[k] >= d.n[k])) continue;
                    const long nid = cell_index(d, q[0], q[1], q[2]);
                    const double mdn = mdot[nid];
                    if (mdn == 0.0 || !mixed(d, c[nid])) continue;
                    const double dd = -(mdn / d.rho_l) * dt_h;
                    const double motion = dd > 0.0 ? 1.0 : -1.0;
                    if (motion != want) continue;
                    const double* r = rec + 5 * nid;
                    const double mo = -s * r[k];
                    const double swept = volume(r[0], r[1], r[2], r[3] - mo) - volume(r[0], r[1], r[2], r[4] - mo);
                    sum += swept;
                    ++cnt;
                }
            if (cnt) cnew = cj - sum / cnt;
        }
        const double dc = cnew - cj;
        const double de = (dc * (d.cp_l - d.cp_g)) * d.T_gamma;
        const double enew = e[id] + de;
        c_out[id] = cnew;
        e_out[id] = enew;
        acc[0] = dc;
        acc[1] = de;
        acc[6] = cnew;
        acc[7] = enew;
    }
    const long blk = ((long)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    block_sum8(acc, part + blk * kPartialWidth);
}

// Fixed-order reduction of the per-block partials of the stages that ran.
__global__ void __launch_bounds__(256)
k_reduce(const double* __restrict__ part, int nblocks, int slot_mask, int last_slot, double hv,
         double* __restrict__ stats) {
    __shared__ double sm[256];
    // quantity q of slot s is column q of the slot's [nblocks][8] table
    double out[10];
    for (int o = 0; o < 10; ++o) out[o] = 0.0;
    for (int s = 0; s < kSlots; ++s) {
        if (!(slot_mask & (1 << s)) && s != last_slot) continue;
        const double* P = part + (long)s * nblocks * kPartialWidth;
        for (int q = 0; q < kPartialWidth; ++q) {
            double v = 0.0;
            for (int b = threadIdx.x; b < nblocks; b += 256) v += P[(long)b * kPartialWidth + q];
            sm[threadIdx.x] = v;
            __syncthreads();
            for (int w = 128; w > 0; w >>= 1) {
                if (threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
                __syncthreads();
            }
            const double tot = sm[0];
            __syncthreads();
            if (s == last_slot && q >= 6) out[q - 6] = tot;  // vol, energy
            if (!(slot_mask & (1 << s))) continue;
            if (s < 3) {
                if (q == 0) out[2] += tot;
                if (q == 1) out[3] += tot;
                if (q == 2) out[6] += tot;
                if (q == 3) out[7] += tot;
                if (q == 4) out[8] += tot;
                if (q == 5) out[9] += tot;
            } else {
                if (q == 0) out[4] += tot;
                if (q == 1) out[5] += tot;
            }
        }
    }
    if (threadIdx.x == 0)
        for (int o = 0; o < 10; ++o) stats[o] = out[o] * hv;
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

__global__ void k_maxabs(const double* __restrict__ x, long n, unsigned long long* maxbits) {
    double m = 0.0;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        m = fmax(m, fabs(x[i]));
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_down(m, off, 64));
    if ((threadIdx.x & 63) == 0 && m > 0.0)
        atomicMax(maxbits, (unsigned long long)__double_as_longlong(m));
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
        if (vel[face_index(d, axis, p[0], p[1], p[2])] != vel[face_index(d, axis, q[0], q[1], q[2])])
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

Launch cell_launch(const Dom& d) {
    Launch L;
    L.block = dim3(kBX, kBY, 1);
    L.grid = dim3((d.n[0] + kBX - 1) / kBX, (d.n[1] + kBY - 1) / kBY, d.ndim == 2 ? 1 : d.n[2]);
    L.nblocks = (int)(L.grid.x * L.grid.y * L.grid.z);
    return L;
}

hipError_t launch_prologue(const Dom& d, const double* c, const double* e, uint8_t* cc, double* ec,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_prologue, linear_grid(d.ncell, 256), dim3(256), 0, s, d, c, e, cc, ec);
    return hipGetLastError();
}

hipError_t launch_sweep(const Dom& d, int axis, const double* c, const double* e, const uint8_t* cc,
                        const double* ec, const double* vel, double kfac, double* c_out,
                        double* e_out, double* part, hipStream_t s) {
    const Launch L = cell_launch(d);
    if (axis == 0)
        hipLaunchKernelGGL(k_sweep<0>, L.grid, L.block, 0, s, d, c, e, cc, ec, vel, kfac, c_out, e_out, part);
    else if (axis == 1)
        hipLaunchKernelGGL(k_sweep<1>, L.grid, L.block, 0, s, d, c, e, cc, ec, vel, kfac, c_out, e_out, part);
    else
        hipLaunchKernelGGL(k_sweep<2>, L.grid, L.block, 0, s, d, c, e, cc, ec, vel, kfac, c_out, e_out, part);
    return hipGetLastError();
}

hipError_t launch_phase(const Dom& d, const double* c, const double* e, const double* mdot, double dt,
                        double h, double* rec, double* c_out, double* e_out, double* part,
                        hipStream_t s) {
    const Launch L = cell_launch(d);
    const double dt_h = dt / h;
    hipLaunchKernelGGL(k_phase_recon, L.grid, L.block, 0, s, d, c, mdot, dt_h, rec);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k_phase_apply, L.grid, L.block, 0, s, d, c, e, mdot, dt_h, rec, c_out, e_out, part);
    return hipGetLastError();
}

hipError_t launch_reduce(const double* part, int nblocks, int slot_mask, int last_slot, double hv,
                         double* stats, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(256), 0, s, part, nblocks, slot_mask, last_slot, hv, stats);
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
    if (nb > 4096) nb = 4096;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_maxabs, dim3((unsigned)nb), dim3(256), 0, s, x, n, maxbits);
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
