// Implicit energy diffusion with the interface temperature imposed (section 3.4.2, eqs.
// T_diff_disc and mod_branchesT) on gfx950.
//
// Each node belongs to the liquid when c >= 1/2, else to the gas, and diffuses with
// its phase's constant conductivity k_p and volumetric heat capacity C_p. Towards a
// face neighbour of the same phase the gradient is the difference over h; towards one
// of the other phase the interface is a boundary at distance theta with T = T_Gamma, the
// gradient is (T_Gamma - T_i) / theta and the node's control width along that axis
// becomes (h + theta) / 2 (both sides irregular: (theta_L + theta_R) / 2). Outflow walls
// are adiabatic; periodic axes wrap. theta: the height of the six-cell column centred on
// the face when it is bounded by pure cells of the two phases, else the crossing of
// 1/2 by the linear interpolation of the node phase's indicator between the two nodes;
// capped to [1e-3 h, h]. Backward Euler:
//   (1 + sum coef) T_i - sum over same-phase sides of coef T_j
//       = T*_i + sum over interface sides of coef T_Gamma,
//   coef = (dt k_p / C_p) / (width h * w h), w = h (node side) or theta (interface side),
// solved by BiCGSTAB with the diagonal as preconditioner. The system is not symmetric
// (the widths differ between a node and its neighbour). Every dot product is a
// fixed-order reduction over the partials of a fixed grid (deterministic).
#include <hip/hip_runtime.h>

#include "common.h"
#include "diffusion.h"

#include <mutex>

namespace pcv {

namespace {

constexpr int kSides = 6;
constexpr int kMarch = 8;  // cells per column of a product block along z
constexpr double kEpsTheta = 1e-3;

// Coordinates of cell base + t: the block-uniform base is divided once, the lane's
// offset t (< the block size) carried forward without divisions.
__device__ __forceinline__ void cell_at(const Dom& d, long base, int t, int (&q)[3]) {
    const long nx = d.n[0], ny = d.n[1];
    int x = (int)(base % nx);
    const long r = base / nx;
    int y = (int)(r % ny);
    int z = (int)(r / ny);
    x += t;
    while (x >= d.n[0]) {
        x -= d.n[0];
        if (++y == d.n[1]) {
            y = 0;
            ++z;
        }
    }
    q[0] = x;
    q[1] = y;
    q[2] = z;
}

// Grid-stride loop over the cells in runs of kDiffBlock (the same cells per block in
// every launch, so the block partials are deterministic): i is the lane's cell, q its
// coordinates.
#define FOR_CELLS(d, i, q)                                                                          \
    for (long base_ = (long)blockIdx.x * kDiffBlock; base_ < (d).ncell; base_ += (long)gridDim.x * kDiffBlock) \
        if (const long i = base_ + threadIdx.x; i < (d).ncell)                                         \
            if (int q[3]; (cell_at((d), base_, (int)threadIdx.x, q), true))

__device__ __forceinline__ long cell_id(const Dom& d, const int (&q)[3]) {
    return ((long)q[2] * d.n[1] + q[1]) * d.n[0] + q[0];
}

// Cell off steps along axis from q: periodic wrap, outflow copy (clamped).
__device__ __forceinline__ long column_cell(const Dom& d, const int (&q)[3], int axis, int off) {
    int r[3] = {q[0], q[1], q[2]};
    const int n = d.n[axis];
    int v = r[axis] + off;
    if (v < 0 || v >= n) {
        if (d.bc[axis] == 0) v = ((v % n) + n) % n;
        else v = v < 0 ? 0 : n - 1;
    }
    r[axis] = v;
    return cell_id(d, r);
}

// Face neighbour: index, or -1 beyond an outflow boundary.
__device__ __forceinline__ long face_neighbour(const Dom& d, const int (&q)[3], int axis, int step) {
    const int n = d.n[axis];
    const int v = q[axis] + step;
    if ((v < 0 || v >= n) && d.bc[axis] != 0) return -1;
    return column_cell(d, q, axis, step);
}

// Distance (cell units) from node q (indicator of its phase fi) to the interface
// towards its neighbour j along axis in direction step.
__device__ double theta_of(const Dom& d, const double* __restrict__ c, const int (&q)[3], bool liquid, int axis,
                           int step, long j) {
    double f[6];
#pragma unroll
    for (int o = 0; o < 6; ++o) {
        const double v = c[column_cell(d, q, axis, (o - 2) * step)];
        f[o] = liquid ? v : 1.0 - v;
    }
    double t;
    if (f[0] >= 1.0 - d.eps && f[5] <= d.eps) {
        double sum = 0.0;
#pragma unroll
        for (int o = 0; o < 6; ++o) sum += f[o];
        t = sum - 2.5;
    } else {
        const double fi = f[2];
        const double fj = liquid ? c[j] : 1.0 - c[j];
        t = (fi - 0.5) / (fi - fj);
    }
    return fmin(fmax(t, kEpsTheta), 1.0);
}

__global__ void __launch_bounds__(kDiffBlock) k_diff_assemble(Dom d, const double* __restrict__ c,
                                                              const double* __restrict__ e, double h, double dt,
                                                              double k_l, double k_g, uint8_t* __restrict__ kindo,
                                                              double* __restrict__ diag, double* __restrict__ off,
                                                              double* __restrict__ b, double* __restrict__ x) {
    FOR_CELLS(d, i, q) {
        const double ci = c[i];
        const bool liquid = ci >= 0.5;
        const double a = dt * (liquid ? k_l : k_g) / (liquid ? d.cp_l : d.cp_g);
        const double Ts = e[i] / cp_of(d, ci);
        double dg = 1.0, rhs = Ts;
        bool iface = false;
        unsigned walls = 0;  // bit slot: that side is an outflow wall
        double ok[kSides];
        int slot = 0;
        for (int axis = 0; axis < d.ndim; ++axis) {
            // kinds: 0 wall, 1 node, 2 interface; w in cell units
            int sk[2];
            double w[2];
            for (int s = 0; s < 2; ++s) {
                const int step = s == 0 ? -1 : 1;
                const long j = face_neighbour(d, q, axis, step);
                if (j < 0) {
                    sk[s] = 0;
                    w[s] = 1.0;
                } else if ((c[j] >= 0.5) == liquid) {
                    sk[s] = 1;
                    w[s] = 1.0;
                } else {
                    sk[s] = 2;
                    w[s] = theta_of(d, c, q, liquid, axis, step, j);
                }
            }
            const double width = 0.5 * (w[0] + w[1]);
            for (int s = 0; s < 2; ++s, ++slot) {
                double o = 0.0;
                if (sk[s] != 0) {
                    const double coef = a / (width * h * w[s] * h);
                    dg += coef;
                    if (sk[s] == 1) o = -coef;
                    else rhs += coef * d.T_gamma;
                }
                if (sk[s] == 0) walls |= 1u << slot;
                if (sk[s] == 2) iface = true;
                ok[slot] = o;
            }
        }
        // a row without an interface side is its phase's regular row (RowConst) with
        // the wall sides left out; the others are stored
        kindo[i] = (uint8_t)((liquid ? 1 : 0) | (iface ? 2 : 0) | walls << 2);
        if (iface) {
            for (int q2 = 0; q2 < kSides; ++q2) off[(long)q2 * d.ncell + i] = q2 < slot ? ok[q2] : 0.0;
            diag[i] = dg;
        }
        b[i] = rhs;
        x[i] = Ts;  // initial guess: the temperature before the step
    }
}

// y_i = diag_i x_i + sum over sides of off_side(i) x_neighbour (zero coefficients for
// walls and interface sides). Rows without an interface side take their phase's
// coefficient on every side that is not a wall, and the diagonal 1 plus those
// coefficients summed in side order (the same values the assembly computes); the others
// the stored ones.
// The coefficient of a regular row of the phase in bit 0 of its kind, chosen between the
// two values rather than indexed by the lane's kind (an indexed read of the argument
// structure would be a memory load per lane, waited for with everything in flight).
__device__ __forceinline__ double phase_coef(const Rows& m, uint8_t k) { return (k & 1) ? m.rc.c[1] : m.rc.c[0]; }

__device__ __forceinline__ double row_diag(const Rows& m, long i, uint8_t k, int sides) {
    if (k & 2) return m.diag[i];
    const double c = phase_coef(m, k);
    double dg = 1.0;
    for (int slot = 0; slot < sides; ++slot)
        if (!(k >> (2 + slot) & 1)) dg += c;
    return dg;
}

// Up to three partial sums per block of kDiffBlock threads (tid the linear thread
// index; thread 0..2 writes part[3 blk + k]).
__device__ __forceinline__ void block_sum3(double a, double b, double c3, double* part, int tid, long blk) {
    __shared__ double s[3][kDiffBlock / 64];
    const double wa = wave_sum_lane63(a), wb = wave_sum_lane63(b), wc = wave_sum_lane63(c3);
    const int lane = tid & 63, w = tid >> 6;
    if (lane == 63) {
        s[0][w] = wa;
        s[1][w] = wb;
        s[2][w] = wc;
    }
    __syncthreads();
    if (tid < 3) {
        double t = s[tid][0];
        for (int k = 1; k < kDiffBlock / 64; ++k) t += s[tid][k];
        part[3 * blk + tid] = t;
    }
}
__device__ __forceinline__ void block_sum3(double a, double b, double c3, double* part) {
    block_sum3(a, b, c3, part, (int)threadIdx.x, (long)blockIdx.x);
}

// Neighbour position along an axis of n cells: periodic wrap, outflow clamp (the
// clamped value is never used: wall sides have no coefficient).
__device__ __forceinline__ int nb_pos(int v, int n, int bc) {
    if (v >= 0 && v < n) return v;
    if (bc == 0) return v < 0 ? v + n : v - n;
    return v < 0 ? 0 : n - 1;
}

// The products over columns: a thread owns the column (x, y) of a block of 64 x 4
// columns and marches over kMarch cells along z, keeping x at z - 1, z, z + 1 in
// registers; the x and y neighbours are rows of the same block (coalesced, in cache).
// Per row the diagonal first, then the sides in the order x-, x+, y-, y+, z-, z+. MODE 0: start
// (r = b - A x, rhat = r, p = v = 0; partials rhat.r, r.r, b.b); 1: y = A x with the
// partial rhat.y; 2: y = A x with the partials y.s, y.y; 4: one damped Jacobi step
// y = x + w (b - A x) / diag (the preconditioner's level 0, no partials).
template <int MODE>
__global__ void __launch_bounds__(kDiffBlock) k_bi_march(Dom d, Rows m, const double* __restrict__ xin,
                                                         double* __restrict__ y, const double* __restrict__ rh,
                                                         const double* __restrict__ sv, const double* __restrict__ b,
                                                         double* __restrict__ rhw, double* __restrict__ p,
                                                         double* __restrict__ v, double* __restrict__ part,
                                                         double w) {
    const int nx = d.n[0], ny = d.n[1], nz = d.n[2];
    const int x = blockIdx.x * 64 + threadIdx.x, yy = blockIdx.y * 4 + threadIdx.y;
    const int z0 = blockIdx.z * kMarch, z1 = z0 + kMarch < nz ? z0 + kMarch : nz;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    if (x < nx && yy < ny) {
        const long plane = (long)nx * ny;
        const long col = (long)yy * nx + x;
        const long xm = (long)yy * nx + nb_pos(x - 1, nx, d.bc[0]), xp = (long)yy * nx + nb_pos(x + 1, nx, d.bc[0]);
        const long ym = (long)nb_pos(yy - 1, ny, d.bc[1]) * nx + x, yp = (long)nb_pos(yy + 1, ny, d.bc[1]) * nx + x;
        const bool three = d.ndim == 3;
        // the vector read beside x: b (residual, relaxation), rhat or s (dot products)
        const double* __restrict__ dop = MODE == 1 ? rh : (MODE == 2 ? sv : b);
        double xprev = three ? xin[nb_pos(z0 - 1, nz, d.bc[2]) * plane + col] : 0.0;
        double xcur = xin[z0 * plane + col];
        double xnext = three ? xin[nb_pos(z0 + 1, nz, d.bc[2]) * plane + col] : 0.0;
        // plane z's in-plane neighbours, kind and dop, and x at z + 1, loaded one step ahead
        double n0 = xin[z0 * plane + xm], n1 = xin[z0 * plane + xp], n2 = xin[z0 * plane + ym],
               n3 = xin[z0 * plane + yp];
        uint8_t kn = m.kind[z0 * plane + col];
        double dn = dop[z0 * plane + col];
        // fully unrolled, so that the values carried from step to step are renamed
        // registers rather than moved ones (a move of a value still being loaded waits for it)
#pragma unroll
        for (int t = 0; t < kMarch; ++t) {
            const int z = z0 + t;
            if (z >= z1) break;
            const long zb = z * plane;
            const long i = zb + col;
            const double nbv[6] = {n0, n1, n2, n3, xprev, xnext};
            const uint8_t k = kn;
            const double di = dn;
            // The next step's loads are issued at every step (the last step repeats its own
            // plane, in cache): with a fixed number of loads per step the compiler waits for
            // each value by its count, not for every load in flight.
            {
                const long zn = (z + 1 < z1 ? z + 1 : z) * plane;
                n0 = xin[zn + xm];
                n1 = xin[zn + xp];
                n2 = xin[zn + ym];
                n3 = xin[zn + yp];
                kn = m.kind[zn + col];
                dn = dop[zn + col];
            }
            const double xnn = three ? xin[nb_pos(z + 2 < z1 ? z + 2 : z1, nz, d.bc[2]) * plane + col] : 0.0;
            const int sides = 2 * d.ndim;
            // Each branch uses up its own loads: a stored (interface) row's diagonal or
            // coefficients read in one branch and used after the join would make every
            // step wait there for all loads in flight.
            double dg, yi;
            if (k & 2) {
                dg = m.diag[i];
                yi = dg * xcur;
                for (int slot = 0; slot < sides; ++slot) {
                    const double o = m.off[(long)slot * d.ncell + i];
                    if (o != 0.0) yi += o * nbv[slot];
                }
            } else {
                dg = row_diag(m, i, k, sides);
                yi = dg * xcur;
                const double o = -phase_coef(m, k);
                for (int slot = 0; slot < sides; ++slot)
                    if (!(k >> (2 + slot) & 1)) yi += o * nbv[slot];
            }
            if (MODE == 4) {
                y[i] = xcur + w * (di - yi) / dg;
            } else if (MODE == 0) {
                const double ri = di - yi;
                y[i] = ri;  // r
                rhw[i] = ri;
                p[i] = 0.0;
                v[i] = 0.0;
                s0 += ri * ri;
                s1 += ri * ri;
                s2 += di * di;
            } else {
                y[i] = yi;
                if (MODE == 2) {
                    s0 += yi * di;
                    s1 += yi * yi;
                } else {
                    s0 += di * yi;
                }
            }
            xprev = xcur;
            xcur = xnext;
            xnext = xnn;
        }
    }
    if (MODE < 4) {
        const long blk = ((long)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
        block_sum3(s0, s1, s2, part, (int)(threadIdx.y * 64 + threadIdx.x), blk);
    }
}

#define GRID_STRIDE(i, n) for (long i = (long)blockIdx.x * kDiffBlock + threadIdx.x; i < (n); i += (long)gridDim.x * kDiffBlock)

// p = r + beta (p - omega v) (then ph = M^-1 p by the preconditioner).
__global__ void __launch_bounds__(kDiffBlock) k_bi_dir(Dom d, const double* __restrict__ scal,
                                                       const double* __restrict__ r, const double* __restrict__ v,
                                                       double* __restrict__ p) {
    const double be = scal[kBiBeta], om = scal[kBiOmega];
    GRID_STRIDE(i, d.ncell) p[i] = r[i] + be * (p[i] - om * v[i]);
}

// s = r - alpha v (then sh = M^-1 s by the preconditioner).
__global__ void __launch_bounds__(kDiffBlock) k_bi_half(Dom d, const double* __restrict__ scal,
                                                        const double* __restrict__ r, const double* __restrict__ v,
                                                        double* __restrict__ s) {
    const double al = scal[kBiAlpha];
    GRID_STRIDE(i, d.ncell) s[i] = r[i] - al * v[i];
}

// x += alpha ph + omega sh, r = s - omega t; partials (rhat.r, r.r, 0).
__global__ void __launch_bounds__(kDiffBlock) k_bi_update(Dom d, const double* __restrict__ scal,
                                                          const double* __restrict__ ph, const double* __restrict__ sh,
                                                          const double* __restrict__ s,
                                                          const double* __restrict__ t, const double* __restrict__ rh,
                                                          double* __restrict__ x, double* __restrict__ r,
                                                          double* __restrict__ part) {
    const double al = scal[kBiAlpha], om = scal[kBiOmega];
    double s0 = 0.0, s1 = 0.0;
    GRID_STRIDE(i, d.ncell) {
        const double si = s[i];
        x[i] += al * ph[i] + om * sh[i];
        const double ri = si - om * t[i];
        r[i] = ri;
        s0 += rh[i] * ri;
        s1 += ri * ri;
    }
    block_sum3(s0, s1, 0.0, part);
}

// Fixed-order sums of the nb triples of partials, then the scalars: mode 0 after the
// start (rho, rr, bb; alpha = omega = 1), 1 after A ph (alpha = rho / rhat.v), 2 after
// A sh (omega = t.s / t.t), 3 after the update (beta = (rho' / rho)(alpha / omega), rho,
// rr). A zero denominator leaves the step at zero (the iteration then stalls and the
// host reports no convergence).
__global__ void __launch_bounds__(kDiffBlock) k_bi_reduce(const double* __restrict__ part, int nb, double* __restrict__ scal,
                                                          int mode) {
    // four interleaved accumulators per quantity (more loads in flight), then a fixed tree
    double acc[3][4] = {};
    int k = threadIdx.x;
    for (; k + 3 * kDiffBlock < nb; k += 4 * kDiffBlock)
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int q = 0; q < 3; ++q) acc[q][u] += part[3 * (k + u * kDiffBlock) + q];
    for (; k < nb; k += kDiffBlock)
#pragma unroll
        for (int q = 0; q < 3; ++q) acc[q][0] += part[3 * k + q];
    const double a = (acc[0][0] + acc[0][1]) + (acc[0][2] + acc[0][3]);
    const double b = (acc[1][0] + acc[1][1]) + (acc[1][2] + acc[1][3]);
    const double c3 = (acc[2][0] + acc[2][1]) + (acc[2][2] + acc[2][3]);
    __shared__ double s[3][kDiffBlock / 64];
    const double wa = wave_sum_lane63(a), wb = wave_sum_lane63(b), wc = wave_sum_lane63(c3);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 63) {
        s[0][w] = wa;
        s[1][w] = wb;
        s[2][w] = wc;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double t0 = s[0][0], t1 = s[1][0], t2 = s[2][0];
    for (int k = 1; k < kDiffBlock / 64; ++k) {
        t0 += s[0][k];
        t1 += s[1][k];
        t2 += s[2][k];
    }
    if (mode == 0) {
        scal[kBiRho] = t0;
        scal[kBiRr] = t1;
        scal[kBiBb] = t2;
        scal[kBiAlpha] = 1.0;
        scal[kBiOmega] = 1.0;
        scal[kBiBeta] = 0.0;
    } else if (mode == 1) {
        scal[kBiAlpha] = t0 != 0.0 ? scal[kBiRho] / t0 : 0.0;
    } else if (mode == 2) {
        scal[kBiOmega] = t1 != 0.0 ? t0 / t1 : 0.0;
    } else {
        const double rho = scal[kBiRho];
        scal[kBiBeta] = (rho != 0.0 && scal[kBiOmega] != 0.0) ? (t0 / rho) * (scal[kBiAlpha] / scal[kBiOmega]) : 0.0;
        scal[kBiRho] = t0;
        scal[kBiRr] = t1;
    }
}

// Multigrid preconditioner M^-1: one V(0,2) cycle over levels of 2 x 2 x 2 aggregates
// (unsmoothed aggregation: piecewise constant prolongation P, restriction R = P^T,
// Galerkin coarse operators R A P, built once per call): on each level the right-hand
// side is restricted as it is, the level below returns its correction, and two damped
// Jacobi steps (weight kMgOmega) start from the prolongated correction; the coarsest
// level takes kMgCoarseSweeps steps from zero. (Measured on the C3 bubble's operator:
// 13 iterations against 12 with a V(1,1) cycle, whose residual and pre-smoothing passes
// over the cells cost more than the iteration saved.) Every kernel is a fixed function
// of its inputs (no atomics), so the preconditioner, like the rest of the solve, is
// deterministic.
constexpr double kMgOmega = 0.8;
constexpr int kMgCoarseSweeps = 4;

// A level's cells per axis, boundary rule per axis, dimension.
struct MgGeom {
    int n[3];
    int bc[3];
    int ndim;
    long ncell;
};

MgGeom mg_geom(const Dom& d, const int* n) {
    MgGeom g;
    for (int a = 0; a < 3; ++a) {
        g.n[a] = n[a];
        g.bc[a] = d.bc[a];
    }
    g.ndim = d.ndim;
    g.ncell = (long)n[0] * n[1] * n[2];
    return g;
}

dim3 mg_grid(const MgGeom& g) { return dim3((g.n[0] + 63) / 64, (g.n[1] + 3) / 4, g.n[2]); }

// The launch covers a level with blocks of 64 x 4 cells per plane (q: the thread's cell).
#define MG_CELL(g, q, i)                                                                            \
    const int q[3] = {(int)(blockIdx.x * 64 + threadIdx.x), (int)(blockIdx.y * 4 + threadIdx.y),  \
                      (int)blockIdx.z};                                                             \
    if (q[0] >= (g).n[0] || q[1] >= (g).n[1]) return;                                               \
    const long i = ((long)q[2] * (g).n[1] + q[1]) * (g).n[0] + q[0];

__device__ __forceinline__ long mg_index(const MgGeom& g, const int (&q)[3]) {
    return ((long)q[2] * g.n[1] + q[1]) * g.n[0] + q[0];
}

// Level 0, first Jacobi step from zero (single-level preconditioner): x0 = w b / diag.
__global__ void __launch_bounds__(kDiffBlock) k_mg_first0(Dom d, Rows m, const double* __restrict__ b,
                                                          double* __restrict__ x0) {
    GRID_STRIDE(i, d.ncell) x0[i] = kMgOmega * b[i] / row_diag(m, i, m.kind[i], 2 * d.ndim);
}

// Level 0: one Jacobi step from the prolongated coarse correction x = P xc (read at the
// cell and its neighbours through their aggregates): y = x + w (b - A x) / diag.
// The coarse index of the aggregate holding the neighbour of fine cell q on side S (the
// cell's own aggregate beyond an outflow boundary, where the coefficient is zero).
template <int S>
__device__ __forceinline__ long mg_coarse_nb(const MgGeom& fg, const MgGeom& cg, const int (&q)[3]) {
    constexpr int axis = S >> 1;
    int r[3] = {q[0], q[1], q[2]};
    int v = r[axis] + ((S & 1) ? 1 : -1);
    if (v < 0 || v >= fg.n[axis]) v = fg.bc[axis] != 0 ? r[axis] : (v < 0 ? v + fg.n[axis] : v - fg.n[axis]);
    r[axis] = v;
    return ((long)(r[2] >> 1) * cg.n[1] + (r[1] >> 1)) * cg.n[0] + (r[0] >> 1);
}

// Level 0: one Jacobi step from the prolongated coarse correction x = P xc (read at the
// cell and its neighbours through their aggregates): y = x + w (b - A x) / diag. The
// seven coarse values are loaded before they are summed (in side order).
__global__ void __launch_bounds__(kDiffBlock) k_mg_psmooth0(Dom d, Rows m, MgGeom fg, MgGeom cg,
                                                            const double* __restrict__ xc,
                                                            const double* __restrict__ b, double* __restrict__ y) {
    MG_CELL(fg, q, i)
    const uint8_t k = m.kind[i];
    const int sides = 2 * d.ndim;
    const long ic = ((long)(q[2] >> 1) * cg.n[1] + (q[1] >> 1)) * cg.n[0] + (q[0] >> 1);
    const long jc[6] = {mg_coarse_nb<0>(fg, cg, q), mg_coarse_nb<1>(fg, cg, q), mg_coarse_nb<2>(fg, cg, q),
                        mg_coarse_nb<3>(fg, cg, q), sides > 4 ? mg_coarse_nb<4>(fg, cg, q) : ic,
                        sides > 4 ? mg_coarse_nb<5>(fg, cg, q) : ic};
    double xn[6];
#pragma unroll
    for (int s = 0; s < 6; ++s) xn[s] = xc[jc[s]];
    const double xi = xc[ic], bi = b[i];
    const double dg = row_diag(m, i, k, sides);
    double ax = dg * xi;
    if (k & 2) {
#pragma unroll
        for (int s = 0; s < 6; ++s)
            if (s < sides) ax += m.off[(long)s * d.ncell + i] * xn[s];
    } else {
        const double o = -phase_coef(m, k);
#pragma unroll
        for (int s = 0; s < 6; ++s)
            if (s < sides && !(k >> (2 + s) & 1)) ax += o * xn[s];
    }
    y[i] = xi + kMgOmega * (bi - ax) / dg;
}

// Index of the neighbour of cell q on side S of a level (the cell itself beyond an
// outflow boundary, where the coefficient is zero).
template <int S>
__device__ __forceinline__ long mg_nb_idx(const MgGeom& g, const int (&q)[3]) {
    constexpr int axis = S >> 1;
    int r[3] = {q[0], q[1], q[2]};
    int v = r[axis] + ((S & 1) ? 1 : -1);
    if (v < 0 || v >= g.n[axis]) v = g.bc[axis] != 0 ? r[axis] : (v < 0 ? v + g.n[axis] : v - g.n[axis]);
    r[axis] = v;
    return mg_index(g, r);
}

// The six neighbour indices of cell q on a level (2D: the last two are the cell itself).
__device__ __forceinline__ void mg_nbs(const MgGeom& g, const int (&q)[3], long i, long (&j)[6]) {
    j[0] = mg_nb_idx<0>(g, q);
    j[1] = mg_nb_idx<1>(g, q);
    j[2] = mg_nb_idx<2>(g, q);
    j[3] = mg_nb_idx<3>(g, q);
    j[4] = g.ndim == 3 ? mg_nb_idx<4>(g, q) : i;
    j[5] = g.ndim == 3 ? mg_nb_idx<5>(g, q) : i;
}

// (A x)_i on a coarse level, the values loaded before they are summed (in side order).
__device__ __forceinline__ double mg_apply_row(const MgGeom& g, const double* __restrict__ diag,
                                               const double* __restrict__ off, const double* __restrict__ x,
                                               const int (&q)[3], long i) {
    long j[6];
    mg_nbs(g, q, i, j);
    double xn[6], o[6];
#pragma unroll
    for (int s = 0; s < 6; ++s) {
        xn[s] = x[j[s]];
        o[s] = off[(long)s * g.ncell + i];
    }
    double y = diag[i] * x[i];
#pragma unroll
    for (int s = 0; s < 6; ++s)
        if (s < 2 * g.ndim) y += o[s] * xn[s];
    return y;
}

// Coarse level, first Jacobi step from zero: x = w b / diag.
__global__ void __launch_bounds__(kDiffBlock) k_mg_first(MgGeom g, const double* __restrict__ diag,
                                                         const double* __restrict__ b, double* __restrict__ x) {
    MG_CELL(g, q, i)
    x[i] = kMgOmega * b[i] / diag[i];
}

// Coarse level, one damped Jacobi step: y = x + w (b - A x) / diag.
__global__ void __launch_bounds__(kDiffBlock) k_mg_smooth(MgGeom g, const double* __restrict__ diag,
                                                          const double* __restrict__ off, const double* __restrict__ x,
                                                          const double* __restrict__ b, double* __restrict__ y) {
    MG_CELL(g, q, i)
    y[i] = x[i] + kMgOmega * (b[i] - mg_apply_row(g, diag, off, x, q, i)) / diag[i];
}

// Coarse level: one Jacobi step from the prolongated correction x = P xc:
// y = x + w (b - A x) / diag.
__global__ void __launch_bounds__(kDiffBlock) k_mg_psmooth(MgGeom g, MgGeom cg, const double* __restrict__ diag,
                                                           const double* __restrict__ off,
                                                           const double* __restrict__ xc,
                                                           const double* __restrict__ b, double* __restrict__ y) {
    MG_CELL(g, q, i)
    const long ic = ((long)(q[2] >> 1) * cg.n[1] + (q[1] >> 1)) * cg.n[0] + (q[0] >> 1);
    const long jc[6] = {mg_coarse_nb<0>(g, cg, q), mg_coarse_nb<1>(g, cg, q), mg_coarse_nb<2>(g, cg, q),
                        mg_coarse_nb<3>(g, cg, q), g.ndim == 3 ? mg_coarse_nb<4>(g, cg, q) : ic,
                        g.ndim == 3 ? mg_coarse_nb<5>(g, cg, q) : ic};
    double xn[6], o[6];
#pragma unroll
    for (int s = 0; s < 6; ++s) {
        xn[s] = xc[jc[s]];
        o[s] = off[(long)s * g.ncell + i];
    }
    const double xi = xc[ic], dg = diag[i];
    double ax = dg * xi;
#pragma unroll
    for (int s = 0; s < 6; ++s)
        if (s < 2 * g.ndim) ax += o[s] * xn[s];
    y[i] = xi + kMgOmega * (b[i] - ax) / dg;
}

// Restriction: bc_I = sum of rf over the aggregate I (fixed order z, y, x).
__global__ void __launch_bounds__(kDiffBlock) k_mg_restrict(MgGeom fg, MgGeom cg, const double* __restrict__ rf,
                                                            double* __restrict__ bc) {
    MG_CELL(cg, q, I)
    double sum = 0.0;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                const int f[3] = {2 * q[0] + dx, 2 * q[1] + dy, 2 * q[2] + dz};
                if (f[0] < fg.n[0] && f[1] < fg.n[1] && f[2] < fg.n[2]) sum += rf[mg_index(fg, f)];
            }
    bc[I] = sum;
}

// Coarse operator entries of one fine row (diagonal dg, side coefficients o[s]) of a cell
// f of the aggregate I = f / 2: a side whose neighbour lies in I adds to the diagonal,
// the others to I's coefficient on that side (the neighbour then lies in the aggregate
// beyond that side, across a periodic wrap too).
__device__ __forceinline__ void mg_accumulate(const MgGeom& fg, const int (&f)[3], double dg, const double (&o)[6],
                                              const int (&I)[3], double& cd, double (&co)[6]) {
    cd += dg;
    for (int s = 0; s < 2 * fg.ndim; ++s) {
        if (o[s] == 0.0) continue;
        const int axis = s >> 1;
        int v = f[axis] + ((s & 1) ? 1 : -1);
        if (v < 0 || v >= fg.n[axis]) v = v < 0 ? v + fg.n[axis] : v - fg.n[axis];  // nonzero: periodic
        if ((v >> 1) == I[axis]) cd += o[s];
        else co[s] += o[s];
    }
}

// Level 1 from the cells' operator (Rows), one thread per coarse cell, the fine rows of
// the aggregate in the order z, y, x and each row's sides in side order.
__global__ void __launch_bounds__(kDiffBlock) k_mg_build0(Dom d, Rows m, MgGeom fg, MgGeom cg,
                                                          double* __restrict__ cdiag, double* __restrict__ coff) {
    MG_CELL(cg, I, ic)
    double cd = 0.0, co[6] = {0, 0, 0, 0, 0, 0};
    const int sides = 2 * d.ndim;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                const int f[3] = {2 * I[0] + dx, 2 * I[1] + dy, 2 * I[2] + dz};
                if (f[0] >= fg.n[0] || f[1] >= fg.n[1] || f[2] >= fg.n[2]) continue;
                const long i = mg_index(fg, f);
                const uint8_t k = m.kind[i];
                double o[6] = {0, 0, 0, 0, 0, 0};
                for (int s = 0; s < sides; ++s)
                    o[s] = (k & 2) ? m.off[(long)s * d.ncell + i] : ((k >> (2 + s) & 1) ? 0.0 : -phase_coef(m, k));
                mg_accumulate(fg, f, row_diag(m, i, k, sides), o, I, cd, co);
            }
    cdiag[ic] = cd;
    for (int s = 0; s < 6; ++s) coff[(long)s * cg.ncell + ic] = co[s];
}

// Level l + 1 from level l's explicit operator.
__global__ void __launch_bounds__(kDiffBlock) k_mg_build(MgGeom fg, const double* __restrict__ fdiag,
                                                         const double* __restrict__ foff, MgGeom cg,
                                                         double* __restrict__ cdiag, double* __restrict__ coff) {
    MG_CELL(cg, I, ic)
    double cd = 0.0, co[6] = {0, 0, 0, 0, 0, 0};
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                const int f[3] = {2 * I[0] + dx, 2 * I[1] + dy, 2 * I[2] + dz};
                if (f[0] >= fg.n[0] || f[1] >= fg.n[1] || f[2] >= fg.n[2]) continue;
                const long i = mg_index(fg, f);
                double o[6] = {0, 0, 0, 0, 0, 0};
                for (int s = 0; s < 2 * fg.ndim; ++s) o[s] = foff[(long)s * fg.ncell + i];
                mg_accumulate(fg, f, fdiag[i], o, I, cd, co);
            }
    cdiag[ic] = cd;
    for (int s = 0; s < 6; ++s) coff[(long)s * cg.ncell + ic] = co[s];
}

// e = C_p(c) T^{n+1}; T_out (if not null) = T^{n+1}.
__global__ void __launch_bounds__(kDiffBlock) k_diff_finish(Dom d, const double* __restrict__ c,
                                                            const double* __restrict__ x, double* __restrict__ e,
                                                            double* __restrict__ T_out) {
    GRID_STRIDE(i, d.ncell) {
        e[i] = cp_of(d, c[i]) * x[i];
        if (T_out) T_out[i] = x[i];
    }
}

dim3 march_grid(const Dom& d) {
    const int nz = d.ndim == 3 ? d.n[2] : 1;
    return dim3((d.n[0] + 63) / 64, (d.n[1] + 3) / 4, (nz + kMarch - 1) / kMarch);
}

int grid_for(long n) {
    const long nb = (n + kDiffBlock - 1) / kDiffBlock;
    return (int)(nb < kDiffGrid ? nb : kDiffGrid);
}

}  // namespace

// Scratch of pcvof_diffuse_static. In host code `scratch` names a host-side stand-in,
// not device memory: only the address from hipGetSymbolAddress is ever used.
static __device__ __align__(256) unsigned char scratch[kDiffStaticBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

hipError_t diff_static_scratch(int device, void** ptr, size_t* bytes) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) {
            const hipError_t e2 = hipSetDevice(cur);
            if (e == hipSuccess) e = e2;
        }
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[device] = p;
    }
    *ptr = g_scratch_ptr[device];
    *bytes = kDiffStaticBytes;
    return hipSuccess;
}

DiffLayout diff_layout(const Dom& d) {
    DiffLayout L;
    const size_t n = (size_t)d.ncell;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = (off + bytes + 255) & ~(size_t)255;
        return at;
    };
    L.kind = take(n);
    L.diag = take(n * sizeof(double));
    L.off = take(kSides * n * sizeof(double));
    L.b = take(n * sizeof(double));
    for (int k = 0; k < 9; ++k) L.vec[k] = take(n * sizeof(double));
    const dim3 mg = march_grid(d);
    const size_t nm = (size_t)mg.x * mg.y * mg.z;
    L.part = take(3 * (nm > (size_t)kDiffGrid ? nm : (size_t)kDiffGrid) * sizeof(double));
    L.scal = take(kBiScalars * sizeof(double));
    // the preconditioner: level-0 iterate, then the coarse levels (every axis halved,
    // rounding up, while the longest is above 8 cells)
    L.mgx0 = take(n * sizeof(double));
    int nl[3] = {d.n[0], d.n[1], d.ndim == 3 ? d.n[2] : 1};
    L.mg_levels = 1;
    for (int a = 0; a < 3; ++a) L.mg_n[0][a] = nl[a];
    auto longest = [&]() {
        int m = 1;
        for (int a = 0; a < d.ndim; ++a) m = nl[a] > m ? nl[a] : m;
        return m;
    };
    while (L.mg_levels < kMgMaxLevels && longest() > 8) {
        for (int a = 0; a < d.ndim; ++a) nl[a] = (nl[a] + 1) / 2;
        const int l = L.mg_levels++;
        for (int a = 0; a < 3; ++a) L.mg_n[l][a] = nl[a];
        const size_t nc = (size_t)nl[0] * nl[1] * nl[2];
        L.mg_diag[l] = take(nc * sizeof(double));
        L.mg_off[l] = take(kSides * nc * sizeof(double));
        L.mg_b[l] = take(nc * sizeof(double));
        L.mg_x[l] = take(nc * sizeof(double));
        L.mg_y[l] = take(nc * sizeof(double));
    }
    L.bytes = off;
    return L;
}

DiffIO diff_views(const DiffLayout& L, void* ws) {
    char* p = (char*)ws;
    DiffIO io;
    io.kind = (uint8_t*)(p + L.kind);
    io.diag = (double*)(p + L.diag);
    io.off = (double*)(p + L.off);
    io.b = (double*)(p + L.b);
    double* v[9];
    for (int k = 0; k < 9; ++k) v[k] = (double*)(p + L.vec[k]);
    io.x = v[0];
    io.r = v[1];
    io.rh = v[2];
    io.p = v[3];
    io.v = v[4];
    io.s = v[5];
    io.t = v[6];
    io.ph = v[7];
    io.sh = v[8];
    io.part = (double*)(p + L.part);
    io.scal = (double*)(p + L.scal);
    io.rows.kind = io.kind;
    io.rows.diag = io.diag;
    io.rows.off = io.off;
    io.mgx0 = (double*)(p + L.mgx0);
    io.mg_levels = L.mg_levels;
    for (int l = 0; l < L.mg_levels; ++l) {
        MgLevel& v = io.mg[l];
        for (int a = 0; a < 3; ++a) v.n[a] = L.mg_n[l][a];
        v.ncell = (long)v.n[0] * v.n[1] * v.n[2];
        v.diag = v.off = v.b = v.x = v.y = nullptr;
        if (l > 0) {
            v.diag = (double*)(p + L.mg_diag[l]);
            v.off = (double*)(p + L.mg_off[l]);
            v.b = (double*)(p + L.mg_b[l]);
            v.x = (double*)(p + L.mg_x[l]);
            v.y = (double*)(p + L.mg_y[l]);
        }
    }
    return io;
}

namespace {

// z = M^-1 in: one V(0,2) cycle. Level l > 0 (right-hand side b_l restricted from the
// level above): b_{l+1} = R b_l, the level below's correction xc, then y = P xc + w D^-1
// (b_l - A P xc) and x_l = y + w D^-1 (b_l - A y); the coarsest level: Jacobi steps from
// zero. Level 0 the same on the cells' operator with b_0 = in and z = x_0. With a single
// level, two Jacobi steps from zero.
void mg_vcycle(const Dom& d, const DiffIO& io, const double* in, double* z, hipStream_t s) {
    const dim3 mg = march_grid(d);
    const dim3 blk(64, 4);
    const double* dn = nullptr;
    double* dw = nullptr;
    const int L = io.mg_levels;
    if (L == 1) {
        hipLaunchKernelGGL(k_mg_first0, dim3(grid_for(d.ncell)), dim3(kDiffBlock), 0, s, d, io.rows, in, io.mgx0);
    } else {
        MgGeom g[kMgMaxLevels];
        for (int l = 0; l < L; ++l) g[l] = mg_geom(d, io.mg[l].n);
        hipLaunchKernelGGL(k_mg_restrict, mg_grid(g[1]), blk, 0, s, g[0], g[1], in, io.mg[1].b);
        for (int l = 1; l + 1 < L; ++l)
            hipLaunchKernelGGL(k_mg_restrict, mg_grid(g[l + 1]), blk, 0, s, g[l], g[l + 1], (const double*)io.mg[l].b,
                               io.mg[l + 1].b);
        // coarsest: Jacobi steps from zero, alternating between x and y
        const MgLevel& c = io.mg[L - 1];
        hipLaunchKernelGGL(k_mg_first, mg_grid(g[L - 1]), blk, 0, s, g[L - 1], (const double*)c.diag,
                           (const double*)c.b, c.x);
        double* cur = c.x;
        double* oth = c.y;
        for (int k = 1; k < kMgCoarseSweeps; ++k) {
            hipLaunchKernelGGL(k_mg_smooth, mg_grid(g[L - 1]), blk, 0, s, g[L - 1], (const double*)c.diag,
                               (const double*)c.off, (const double*)cur, (const double*)c.b, oth);
            double* t = cur;
            cur = oth;
            oth = t;
        }
        const double* below = cur;  // the level below's correction
        for (int l = L - 2; l >= 1; --l) {
            const MgLevel& v = io.mg[l];
            hipLaunchKernelGGL(k_mg_psmooth, mg_grid(g[l]), blk, 0, s, g[l], g[l + 1], (const double*)v.diag,
                               (const double*)v.off, below, (const double*)v.b, v.y);
            hipLaunchKernelGGL(k_mg_smooth, mg_grid(g[l]), blk, 0, s, g[l], (const double*)v.diag,
                               (const double*)v.off, (const double*)v.y, (const double*)v.b, v.x);
            below = v.x;
        }
        hipLaunchKernelGGL(k_mg_psmooth0, mg_grid(g[0]), blk, 0, s, d, io.rows, g[0], g[1], below, in, io.mgx0);
    }
    hipLaunchKernelGGL(k_bi_march<4>, mg, blk, 0, s, d, io.rows, (const double*)io.mgx0, z, dn, dn, in, dw, dw, dw,
                       dw, kMgOmega);
}

}  // namespace

// The neighbour coefficient of each phase's regular row, computed as the assembly
// computes it (width and distances of one cell on every side).
RowConst row_const(double h, double dt, double k_l, double k_g, double cp_l, double cp_g) {
    RowConst rc;
    for (int p = 0; p < 2; ++p) {
        const double a = dt * (p ? k_l : k_g) / (p ? cp_l : cp_g);
        const double width = 0.5 * (1.0 + 1.0);
        rc.c[p] = a / (width * h * 1.0 * h);
    }
    return rc;
}

hipError_t launch_diff_start(const Dom& d, const double* c, const double* e, double h, double dt, double k_l,
                             double k_g, DiffIO& io, hipStream_t s) {
    const int ng = grid_for(d.ncell);
    io.rows.rc = row_const(h, dt, k_l, k_g, d.cp_l, d.cp_g);
    hipLaunchKernelGGL(k_diff_assemble, dim3(ng), dim3(kDiffBlock), 0, s, d, c, e, h, dt, k_l, k_g, io.kind, io.diag,
                       io.off, io.b, io.x);
    // the coarse operators of the preconditioner
    for (int l = 1; l < io.mg_levels; ++l) {
        const MgGeom fg = mg_geom(d, io.mg[l - 1].n), cg = mg_geom(d, io.mg[l].n);
        if (l == 1)
            hipLaunchKernelGGL(k_mg_build0, mg_grid(cg), dim3(64, 4), 0, s, d, io.rows, fg, cg, io.mg[1].diag,
                               io.mg[1].off);
        else
            hipLaunchKernelGGL(k_mg_build, mg_grid(cg), dim3(64, 4), 0, s, fg, (const double*)io.mg[l - 1].diag,
                               (const double*)io.mg[l - 1].off, cg, io.mg[l].diag, io.mg[l].off);
    }
    const dim3 mg = march_grid(d);
    const int nm = (int)(mg.x * mg.y * mg.z);
    hipLaunchKernelGGL(k_bi_march<0>, mg, dim3(64, 4), 0, s, d, io.rows, io.x, io.r, (const double*)nullptr,
                       (const double*)nullptr, io.b, io.rh, io.p, io.v, io.part, 0.0);
    hipLaunchKernelGGL(k_bi_reduce, dim3(1), dim3(kDiffBlock), 0, s, io.part, nm, io.scal, 0);
    return hipGetLastError();
}

hipError_t launch_diff_iteration(const Dom& d, const DiffIO& io, hipStream_t s) {
    const int ng = grid_for(d.ncell);
    hipLaunchKernelGGL(k_bi_dir, dim3(ng), dim3(kDiffBlock), 0, s, d, io.scal, io.r, io.v, io.p);
    mg_vcycle(d, io, io.p, io.ph, s);
    const dim3 mg = march_grid(d);
    const int nm = (int)(mg.x * mg.y * mg.z);
    hipLaunchKernelGGL(k_bi_march<1>, mg, dim3(64, 4), 0, s, d, io.rows, io.ph, io.v, io.rh, (const double*)nullptr,
                       (const double*)nullptr, (double*)nullptr, (double*)nullptr, (double*)nullptr, io.part, 0.0);
    hipLaunchKernelGGL(k_bi_reduce, dim3(1), dim3(kDiffBlock), 0, s, io.part, nm, io.scal, 1);
    hipLaunchKernelGGL(k_bi_half, dim3(ng), dim3(kDiffBlock), 0, s, d, io.scal, io.r, io.v, io.s);
    mg_vcycle(d, io, io.s, io.sh, s);
    hipLaunchKernelGGL(k_bi_march<2>, mg, dim3(64, 4), 0, s, d, io.rows, io.sh, io.t, io.rh, (const double*)io.s,
                       (const double*)nullptr, (double*)nullptr, (double*)nullptr, (double*)nullptr, io.part, 0.0);
    hipLaunchKernelGGL(k_bi_reduce, dim3(1), dim3(kDiffBlock), 0, s, io.part, nm, io.scal, 2);
    hipLaunchKernelGGL(k_bi_update, dim3(ng), dim3(kDiffBlock), 0, s, d, io.scal, io.ph, io.sh, io.s, io.t, io.rh,
                       io.x, io.r, io.part);
    hipLaunchKernelGGL(k_bi_reduce, dim3(1), dim3(kDiffBlock), 0, s, io.part, ng, io.scal, 3);
    return hipGetLastError();
}

hipError_t launch_diff_finish(const Dom& d, const double* c, double* e, double* T_out, const DiffIO& io,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_diff_finish, dim3(grid_for(d.ncell)), dim3(kDiffBlock), 0, s, d, c, io.x, e, T_out);
    return hipGetLastError();
}

}  // namespace pcv
