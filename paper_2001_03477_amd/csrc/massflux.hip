// Mass-transfer rate from the PLIC reconstruction (section 3.2) on gfx950, in three
// launches over the grid:
//   1. k_mf_plane: every mixed cell's plane as a unit normal n = m / |m|_2 (liquid
//      towards gas) and its distance d = alpha / |m|_2 from the cell origin, the
//      corner nearest the domain origin (eq. plane_m, eq. cell_d);
//   2. k_mf_pure: every pure cell within two cells of a mixed cell takes the plane of
//      the neighbouring mixed cell whose normal is most collinear with the translation
//      dx from that cell's origin to the pure cell's centre, xi = |n . dx|, and stores
//      its distance |d - n . dx| h (eq. dint_trans) and the normal gradient into its
//      phase (T - T_Gamma) / distance (eq. grad_n_T);
//   3. k_mf_mdot: every mixed cell averages those gradients over the pure cells of its
//      5x5(x5) block, per phase, with weights gamma = xi / |dx|^2 relative to its own
//      plane (eq. normTgrad), and m'' = (k_g G_g + k_l G_l) / h_fg (eq. mdot_calc, both
//      gradients taken into their phase).
// One thread per cell, x across the wavefront. The mixed cells are read from the
// state's bitmask, so a pure cell far from the interface costs the mask words of its
// block. The collinearity and the distance are evaluated without contraction in a
// fixed order, so that the choice of plane does not depend on rounding.
#include <hip/hip_runtime.h>

#include "common.h"

namespace pcv {

namespace {

// Collinearities within this band count as equal (the first candidate in the scan
// order is kept); nodes closer than this to the selected plane (cell units) give no
// gradient.
constexpr double kMfTie = 1e-12;
constexpr double kMfMinDist = 1e-6;
constexpr int kMfR = 2;  // first and second neighbours

// Row (z ny + y) and x of the block position (x+ox, y+oy, z+oz): periodic axes wrap,
// positions beyond an outflow boundary do not exist (false). Small periodic axes wrap
// repeatedly.
__device__ __forceinline__ bool mf_pos(const Dom& d, int x, int y, int z, int ox, int oy, int oz, long& row,
                                       int& xx) {
    int q[3] = {x + ox, y + oy, z + oz};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int n = d.n[a];
        if (q[a] >= 0 && q[a] < n) continue;
        if ((a == 2 && d.ndim == 2) || d.bc[a] == 1) return false;
        while (q[a] < 0) q[a] += n;
        while (q[a] >= n) q[a] -= n;
    }
    row = (long)q[2] * d.n[1] + q[1];
    xx = q[0];
    return true;
}

// n . dx in the order x, y, z, without contraction.
__device__ __forceinline__ double mf_dot(const double* n, double dx0, double dx1, double dx2) {
#pragma clang fp contract(off)
    double s = n[0] * dx0;
    s += n[1] * dx1;
    s += n[2] * dx2;
    return s;
}

__global__ void __launch_bounds__(256) k_mf_plane(Dom d, const double* __restrict__ c, const uint64_t* __restrict__ mask,
                                                  double* __restrict__ plane) {
    const int x = blockIdx.x * 64 + threadIdx.x;
    const int y = blockIdx.y * 4 + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= d.n[0] || y >= d.n[1]) return;
    const long row = (long)z * d.n[1] + y;
    if (!mask_bit(mask, row * d.wpr, x)) return;
    const long id = row * d.n[0] + x;
    double c27[27];
    gather27(d, c, x, y, z, c27);
    const Normal nm = normal27(c27, d.normal);
    const double alpha = alpha_of(nm.m[0], nm.m[1], nm.m[2], c[id]);
    double norm;
    {
#pragma clang fp contract(off)
        norm = sqrt(nm.m[0] * nm.m[0] + nm.m[1] * nm.m[1] + nm.m[2] * nm.m[2]);
    }
    plane[4 * id + 0] = nm.m[0] / norm;
    plane[4 * id + 1] = nm.m[1] / norm;
    plane[4 * id + 2] = nm.m[2] / norm;
    plane[4 * id + 3] = alpha / norm;
}

__global__ void __launch_bounds__(256) k_mf_pure(Dom d, const double* __restrict__ c, const double* __restrict__ e,
                                                 const uint64_t* __restrict__ mask,
                                                 const double* __restrict__ plane, double h, double* __restrict__ q,
                                                 double* __restrict__ dist) {
    const int x = blockIdx.x * 64 + threadIdx.x;
    const int y = blockIdx.y * 4 + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= d.n[0] || y >= d.n[1]) return;
    const long row = (long)z * d.n[1] + y;
    const long id = row * d.n[0] + x;
    double qv = __builtin_nan(""), dv = __builtin_nan("");
    if (!mask_bit(mask, row * d.wpr, x)) {
        const int rz = d.ndim == 2 ? 0 : kMfR;
        bool found = false;
        double best = 0.0, dbest = 0.0;
        for (int oz = -rz; oz <= rz; ++oz)
            for (int oy = -kMfR; oy <= kMfR; ++oy)
                for (int ox = -kMfR; ox <= kMfR; ++ox) {
                    long mrow;
                    int mx;
                    if (!mf_pos(d, x, y, z, ox, oy, oz, mrow, mx) || !mask_bit(mask, mrow * d.wpr, mx)) continue;
                    const long mid = mrow * d.n[0] + mx;
                    // from the mixed cell's origin to this cell's centre
                    const double dx0 = -ox + 0.5, dx1 = -oy + 0.5, dx2 = d.ndim == 2 ? 0.0 : -oz + 0.5;
                    const double* pn = plane + 4 * mid;
                    const double p0 = pn[0], p1 = pn[1], p2 = pn[2], pd = pn[3];
                    const double nv[3] = {p0, p1, p2};
                    const double s = mf_dot(nv, dx0, dx1, dx2);
                    const double xi = fabs(s);
                    if (!found || xi > best + kMfTie) {
                        found = true;
                        best = xi;
                        dbest = pd - s;
                    }
                }
        if (found) {
            dv = fabs(dbest) * h;
            if (fabs(dbest) > kMfMinDist) {
                const double cv = c[id];
                const double T = e[id] / cp_of(d, cv);
                qv = (T - d.T_gamma) / dv;
            }
        }
    }
    q[id] = qv;
    if (dist) dist[id] = dv;
}

__global__ void __launch_bounds__(256) k_mf_mdot(Dom d, const double* __restrict__ c, const uint64_t* __restrict__ mask,
                                                 const double* __restrict__ plane,
                                                 const double* __restrict__ q, double k_l, double k_g, double h_fg,
                                                 double* __restrict__ mdot) {
    const int x = blockIdx.x * 64 + threadIdx.x;
    const int y = blockIdx.y * 4 + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= d.n[0] || y >= d.n[1]) return;
    const long row = (long)z * d.n[1] + y;
    const long id = row * d.n[0] + x;
    double out = 0.0;
    if (mask_bit(mask, row * d.wpr, x)) {
        const int rz = d.ndim == 2 ? 0 : kMfR;
        const double nv[3] = {plane[4 * id + 0], plane[4 * id + 1], plane[4 * id + 2]};
        double wg = 0.0, wl = 0.0, gg = 0.0, gl = 0.0;
        for (int oz = -rz; oz <= rz; ++oz)
            for (int oy = -kMfR; oy <= kMfR; ++oy)
                for (int ox = -kMfR; ox <= kMfR; ++ox) {
                    long prow;
                    int px;
                    if (!mf_pos(d, x, y, z, ox, oy, oz, prow, px)) continue;
                    const long pid = prow * d.n[0] + px;
                    const double qp = q[pid];
                    if (qp != qp) continue;  // mixed, or no gradient
                    const double dx0 = ox + 0.5, dx1 = oy + 0.5, dx2 = d.ndim == 2 ? 0.0 : oz + 0.5;
                    double gam;
                    {
#pragma clang fp contract(off)
                        const double xi = fabs(mf_dot(nv, dx0, dx1, dx2));
                        const double r2 = dx0 * dx0 + dx1 * dx1 + dx2 * dx2;
                        gam = xi / r2;
                    }
                    if (c[pid] >= 0.5) {
                        wl += gam;
                        gl += gam * qp;
                    } else {
                        wg += gam;
                        gg += gam * qp;
                    }
                }
        const double Gg = wg > 0.0 ? gg / wg : 0.0;
        const double Gl = wl > 0.0 ? gl / wl : 0.0;
        out = (k_g * Gg + k_l * Gl) / h_fg;
    }
    mdot[id] = out;
}

}  // namespace

hipError_t launch_mass_flux(const Dom& d, const MassFluxIO& io, hipStream_t s) {
    const Launch L = cell_launch(d);
    hipLaunchKernelGGL(k_mf_plane, L.grid, L.block, 0, s, d, io.c, io.mask, io.plane);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k_mf_pure, L.grid, L.block, 0, s, d, io.c, io.e, io.mask, io.plane, io.h, io.q,
                       io.dist);
    err = hipGetLastError();
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k_mf_mdot, L.grid, L.block, 0, s, d, io.c, io.mask, io.plane, io.q, io.k_l,
                       io.k_g, io.h_fg, io.mdot);
    return hipGetLastError();
}

}  // namespace pcv
