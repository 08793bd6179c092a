// The advection step on gfx950: the direction sweeps (section 3.3.1, with the
// conservative energy fluxes of section 3.4.1) and step 2 with its latent correction
// (section 3.3.2, section 3.4.1).
//
// A sweep is one launch over tiles of faces. Each wavefront first finds the faces of
// its rows (x sweep) or columns (y, z sweeps) with a mixed cell on either side, from
// the mixed-cell mask of the input, then reconstructs the mixed upwind donors of those
// faces with all of its lanes (normal, plane constant, liquid volume of the upwind
// face-flux region) into a table in LDS, and then streams over its cells: WENO5 face
// temperatures, face fluxes (the table for mixed donors, |lambda| c for pure ones),
// the cell update, the clip, the checksum partials and the mask of the output. The
// geometry of one wavefront overlaps with the streaming of the others on the same
// SIMD. All floating point is double precision.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>

#include <type_traits>

#include "common.h"
#include "geom32.h"

namespace pcv {

namespace {

struct SweepArgs {
    const double* c;
    const double* e;
    const uint64_t* mask;  // mixed cells of c
    int first;             // (here, not last: this order spills fewer scalar registers)
    uint64_t* mask_out;    // mixed cells of c_out
    uint8_t* cc;       // written by the first sweep of a step, read by the others
    void* ec;          // double, or float in the mixed-precision mode
    const void* vel;   // double, or float in the mixed-precision mode
    double kfac;
    double* fgeo;          // overflow of the y / z blocks' LDS flux tables, face layout of vel
    double* c_out;
    double* e_out;
    double* part;        // quantity-major partial table of this stage
    long part_stride;
};

// Mask of the mixed cells of c, after the fractions were set from outside.
__global__ void __launch_bounds__(256) k_classify(Dom d, const double* __restrict__ c, uint64_t* __restrict__ mask) {
    const int x = blockIdx.x * 64 + threadIdx.x;
    const int y = blockIdx.y * 4 + threadIdx.y;
    const int z = blockIdx.z;
    const bool mx = x < d.n[0] && y < d.n[1] && mixed(d, c[((long)z * d.n[1] + y) * d.n[0] + x]);
    const unsigned long long bits = __ballot(mx);
    if (threadIdx.x == 0 && y < d.n[1]) mask[((long)z * d.n[1] + y) * d.wpr + blockIdx.x] = bits;
}

// Liquid volume, in cell units, of the upwind region of the donor cell at (x, y, z)
// (ghost positions allowed: they map like every other read) crossing a face of a
// sweep along AX with CFL number lam; cd is the donor's fraction (mixed). The plane is
// reconstructed from the donor's own 3x3x3 block, so a periodic face computed from
// either side, or a ghost donor beyond an outflow boundary, gives the same value.
// Weymouth-Yue sweeps: the donor slab of width |lam| next to the face. Lagrangian-
// explicit sweeps: the donor is stretched by s = 1 + (lam_R - lam_L) (its own faces),
// and the flux is s times the liquid of its slab of width |lam| / s.
template <int AX>
__device__ double donor_fraction(const Dom& d, const double* __restrict__ c, int x, int y, int z, double cd,
                                 double lam, double s) {
    double c27[27];
    gather27(d, c, x, y, z, c27);
    const Normal nm = normal27(c27, d.normal);
    const double alpha = alpha_of(nm.m[0], nm.m[1], nm.m[2], cd);
    if (d.split) return s * slab(nm.m[0], nm.m[1], nm.m[2], alpha, AX, lam / s);
    return slab(nm.m[0], nm.m[1], nm.m[2], alpha, AX, lam);
}

// Face position f (between cells f-1 and f) of an axis with n cells beyond the domain:
// periodic axes wrap (face n is face 0), outflow axes repeat the boundary face, so a
// ghost donor has the same velocity on both faces and is not stretched.
__device__ __forceinline__ int face_wrap(int f, int n, int bc) {
    if (bc == 0) return f < 0 ? f + n : (f > n ? f - n : f);
    return f < 0 ? 0 : (f > n ? n : f);
}

// Stretch s = 1 + (lam_R - lam_L) of the donor of a face with CFL number lam, given
// the CFL number lo of the donor's other face (the face before it when lam > 0, after
// it otherwise).
__device__ __forceinline__ double donor_stretch(double lam, double lo) {
    return lam > 0.0 ? 1.0 + (lam - lo) : 1.0 + (lo - lam);
}

// Mixed-precision mode: face velocities and e_c are stored in single precision; the
// donor's normal, plane constant and slab volume are evaluated in single precision,
// except that the plane constant and the slab volume stay in double precision for
// fractions within kMixedFp64Band of 0 or 1. The flux is kept inside the bounds of an
// exact slab volume, [max(0, c_D - (1 - |lam|)), min(|lam|, c_D)]. Fractions,
// energies, fluxes and all sums stay in double precision.
constexpr double kMixedFp64Band = 1e-3;

template <bool MP>
struct Prec {
    using T = double;
};
template <>
struct Prec<true> {
    using T = float;
};

// Stored values in their storage type: prefetched values stay in it until they are
// used, so that the conversion does not wait for the load.
template <bool MP>
__device__ __forceinline__ typename Prec<MP>::T vel_at(const SweepArgs& a, long i) {
    return ((const typename Prec<MP>::T*)a.vel)[i];
}
template <bool MP>
__device__ __forceinline__ typename Prec<MP>::T ec_at(const SweepArgs& a, long i) {
    return ((const typename Prec<MP>::T*)a.ec)[i];
}

template <int AX, bool MP>
__device__ double donor_flux(const Dom& d, const double* __restrict__ c, int x, int y, int z, double cd,
                             double lam, double s) {
    if (!MP) return donor_fraction<AX>(d, c, x, y, z, cd, lam, s);
    double c27[27];
    gather27(d, c, x, y, z, c27);
    float c27f[27];
#pragma unroll
    for (int q = 0; q < 27; ++q) c27f[q] = (float)c27[q];
    const NormalF nm = normal27_f(c27f, d.normal);
    const double lw = d.split ? lam / s : lam;  // slab width (Lagrangian-explicit: |lam| / s)
    const double L = fabs(lw);
    double F;
    if (fmin(cd, 1.0 - cd) < kMixedFp64Band) {
        const double alpha = alpha_of(nm.m[0], nm.m[1], nm.m[2], cd);
        F = slab(nm.m[0], nm.m[1], nm.m[2], alpha, AX, lw);
    } else {
        const float alpha = alpha_of_f(nm.m[0], nm.m[1], nm.m[2], (float)cd, (float)(1.0 - cd));
        F = (double)slab_f(nm.m[0], nm.m[1], nm.m[2], alpha, AX, (float)lw);
    }
    F = fmin(fmax(F, fmax(0.0, cd - (1.0 - L))), fmin(L, cd));
    return d.split ? s * F : F;
}

// Linear index of the block (row of the partial tables).
__device__ __forceinline__ int block_linear() {
    return (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
}

// Cell update of a sweep (section 3.3.1 with the split dilatation term, and the
// conservative energy update of section 3.4.1), the clip into [0,1] keeping T, and the
// step prologue when first: c_c = [c >= 1/2], e_c = C_p(c_c) T. Returns the new c.
template <bool MP>
__device__ __forceinline__ double update_cell(const Dom& d, const SweepArgs& a, long id, double cv, double ev,
                                              double Tv, double lamL, double lamR, double PhiL, double PhiR,
                                              double EL, double ER, uint8_t cc_in, double ec_in,
                                              double (&acc)[8]) {
    double flag, ecv;
    if (a.first) {
        const bool liquid = cv >= 0.5;
        flag = liquid ? 1.0 : 0.0;
        using T = typename Prec<MP>::T;
        const T ecs = (T)((liquid ? d.cp_l : d.cp_g) * Tv);  // every sweep uses the stored value
        ecv = (double)ecs;
        a.cc[id] = liquid ? 1 : 0;
        ((T*)a.ec)[id] = ecs;
    } else {
        flag = (double)cc_in;
        ecv = ec_in;
    }
    if (d.split) {  // Lagrangian-explicit sweeps: c' = s c - (PhiR - PhiL), likewise e
        flag = cv;
        ecv = ev;
    }
    const double dl = lamR - lamL;
    double cn = cv - (PhiR - PhiL) + flag * dl;
    double en = ev - (ER - EL) + ecv * dl;
    acc[4] += flag * dl;
    acc[5] += ecv * dl;
    if (cn < 0.0 || cn > 1.0) {
        const double T = en / cp_of(d, cn);
        const double cl = cn < 0.0 ? 0.0 : 1.0;
        const double el = en + (d.cp_l - d.cp_g) * (cl - cn) * T;
        acc[0] += cl - cn;
        acc[1] += el - en;
        cn = cl;
        en = el;
    }
    a.c_out[id] = cn;
    a.e_out[id] = en;
    acc[6] += cn;
    acc[7] += en;
    return cn;
}

// Volume and energy fluxes through a face with CFL number lam, given the liquid volume
// F of the upwind region and the WENO5 face temperature Tf: Phi = sgn(lam) F and
// E = sgn(lam) [C_pl F + C_pg (|lam| - F)] Tf (section 3.4.1, eq. disc_et_adv). With the
// non-conservative energy flux (eq. disc_et_adv_noncons) E = lam Tf, which each cell
// scales by its own heat capacity (cell_energy_flux).
__device__ __forceinline__ void face_energy(const Dom& d, double lam, double F, double Tf, double& Phi,
                                            double& E) {
    const double L = fabs(lam);
    const double sg = lam > 0.0 ? 1.0 : -1.0;
    Phi = sg * F;
    if (d.ncons)
        E = lam * Tf;
    else
        E = sg * ((d.cp_l * F + d.cp_g * (L - F)) * Tf);
}

// The energy fluxes through the left and right faces of a cell with fraction cv as the
// cell sees them: as computed (conservative), or scaled by the cell's own heat capacity
// (non-conservative).
__device__ __forceinline__ void cell_energy_flux(const Dom& d, double cv, double& EL, double& ER) {
    if (d.ncons) {
        const double k = cp_of(d, cv);
        EL *= k;
        ER *= k;
    }
}

// Longest column chunk of the y and z sweeps, and the number of donor fluxes a y / z
// wavefront keeps in LDS (fluxes beyond it go to a face array in global memory,
// written and read back by the same wavefront).
constexpr int TCH = 64;
constexpr int kMinChunk = 8;
constexpr int TFCAP = 255;
static_assert(TCH <= 64 && ((TCH + 1) << 6) <= 65536, "work items fit 16 bits");
static_assert(TFCAP <= 255, "saturated list positions fit 8 bits");

// x sweep: a wavefront walks XR rows (XR = 1, 2, 4 or 8, chosen per domain) of one
// sub-row range [x0, x1) (x0 a multiple of 64, at most XKMAX chunks of 64 cells) chunk
// by chunk, one cell per lane. Lane l computes the right face of its cell and takes the
// left face from lane l - 1; lane 0 takes it from lane 63 of the previous chunk, or, at
// the start of a row, from the row's first face, which the wavefront computes for all
// of its rows at once. Fractions, energies and temperatures are staged in a ring of two
// 64-position LDS slots (chunk j holds positions x0 - 2 + 64 j .. + 63), so that each
// position is loaded and divided once per row; the chunk after the current one is
// staged before its faces are computed (the WENO5 stencil of the last lane reaches 3
// cells ahead) and loaded one chunk earlier. The output mask words are the chunks
// (64 cells). Before the walk the wavefront lists the faces of all its rows with a mixed
// cell on either side (in walk order: first faces, then row by row, chunk by chunk) and
// reconstructs their mixed donors 64 at a time; the walk recomputes each face's list
// position from the same mask words, so no per-face index is stored.
constexpr int XW = 64;
constexpr int XWAVES = 4;
constexpr int XRMAX = 8;     // rows per wavefront
constexpr int XKMAX = 8;     // chunks per sub-row (512 cells; face offsets fit 11 bits)
// Donor fluxes per wavefront kept in LDS (more go to fgeo, whose reads wait for all of
// the wavefront's loads). 384 with 512-cell sub-rows fits the LDS of 256 with 1024-cell
// ones; measured at 512^3, where eight rows of a wavefront list up to several hundred
// faces, the x sweep took 1.785 instead of 1.822 ms.
constexpr int XFCAP = 384;
constexpr int XRING = 128;   // staged positions per wavefront (two chunks)

// Plan of an x sweep: rows per wavefront, chunks per sub-row range, ranges per row. The
// kernels take rows and chunks packed into one int (rows | chunks << 8).
struct XPlan {
    int rows, chunks, splits;
};
// The given rows per wavefront, ranges as long as allowed.
inline XPlan x_plan_rows(int nx, int rows) {
    const int kt = (nx + XW - 1) / XW;
    const int ch = kt < XKMAX ? kt : XKMAX;
    return {rows, ch, (kt + ch - 1) / ch};
}
inline long x_waves(const XPlan& p, int ny, int nz) { return (long)p.splits * ((ny + p.rows - 1) / p.rows) * nz; }
// Single-domain rule: 8 rows per wavefront if that leaves at least 16,384 wavefronts, else 4
// rows if that leaves 4,096, else 2 if 2,048, else one row, with shorter ranges while fewer
// than 2,048 wavefronts. (Measured: 8 rows at 512^3, 4 at 256^3 and 128^3 were the fastest;
// one row per wavefront at 128^3 took 50 instead of 35 µs per x sweep: every wavefront then
// pays the first-face pass, a staging-only chunk and the geometry latency for one short row.)
inline XPlan x_plan_rule(int nx, int ny, int nz) {
    const int rows[3] = {8, 4, 2};
    const long need[3] = {16384, 4096, 2048};
    for (int i = 0; i < 3; ++i) {
        const XPlan p = x_plan_rows(nx, rows[i]);
        if (x_waves(p, ny, nz) >= need[i]) return p;
    }
    XPlan p = x_plan_rows(nx, 1);
    const int kt = (nx + XW - 1) / XW;
    while (p.chunks > 1 && x_waves(p, ny, nz) < 2048) {
        p.chunks = (p.chunks + 1) >> 1;
        p.splits = (kt + p.chunks - 1) / p.chunks;
    }
    return p;
}
inline int x_plan_pack(const XPlan& p) { return p.rows | (p.chunks << 8); }

// Mixed bit of cell x (ghost positions mapped) in row R of the input mask.
__device__ __forceinline__ bool mask64(const Dom& d, const uint64_t* __restrict__ mask, int R, int x) {
    const int xm = wrap(x, d.n[0], d.bc[0]);
    return (mask[(long)R * d.wpr + (xm >> 6)] >> (xm & 63)) & 1ull;
}

// Whether the right face of this lane's cell x0 + 64 k + lane (own: x < x1) has a mixed
// cell on either side: w0 is the mask word of the chunk, w1 the next word of the row (0
// past the row's end), gbit the bit of the ghost cell right of the last cell (cell 0 on
// periodic axes, the last cell on outflow ones).
__device__ __forceinline__ bool x_face_need(int nx, uint64_t w0, uint64_t w1, int x, int lane, bool own,
                                            bool gbit) {
    bool right;
    if (x + 1 == nx)
        right = gbit;
    else if (lane < 63)
        right = (w0 >> (lane + 1)) & 1ull;
    else
        right = w1 & 1ull;
    return own && (((w0 >> lane) & 1ull) || right);
}

// A wavefront-uniform 64-bit value moved into scalar registers (each half zero-extended).
__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)v);
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Orders a wavefront's LDS accesses: the compiler keeps them on their side of it, and
// the LDS executes a wavefront's accesses in order.
__device__ __forceinline__ void wave_lds_order() {
    __builtin_amdgcn_wave_barrier();
    __asm__ volatile("" ::: "memory");
}

// Flux of the listed face at list position q: from the wavefront's LDS table below cap,
// else from the global face array at g. The global read is waited for inside its own
// branch: merged with the LDS read into one generic load, or waited for where the two
// branches join, it would make every face wait for all of the wavefront's loads in
// flight, the prefetches of the next faces included.
__device__ __forceinline__ double listed_flux(const double* tab, unsigned q, unsigned cap, const double* g) {
    double F;
    if (q < cap) {
        F = tab[q];
    } else {
        F = *g;
        __builtin_amdgcn_s_waitcnt(0);
    }
    return F;
}

// A tile of a sweep: block coordinates in the domain's own launch grid and the row
// of the partial tables it writes.
struct TileAt {
    int bx, by, bz;
    int blk;
};

template <bool MP>
__device__ __forceinline__ void sweep_x_body(const Dom& d, const SweepArgs& a, const TileAt& tl, int plan) {
    // one record per wavefront, so that every table is one base address plus a constant
    struct WaveLds {
        double c[XRING], e[XRING], T[XRING];
        double F[XFCAP];                      // liquid flux of listed faces, by position
        double first[3][XRMAX];               // Phi, E, lambda of each row's carried face
        uint64_t mw[XRMAX * (XKMAX + 1)];     // input mask words of the rows
        uint64_t bal[XRMAX * XKMAX];          // listed faces of each chunk (ballot)
        unsigned short work[128];             // listed faces not yet reconstructed (ring)
    };
    __shared__ WaveLds s_x[XWAVES];
    using T = typename Prec<MP>::T;
    const int lane = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.y);
    WaveLds& W = s_x[wave];
    const int nx = d.n[0];
    const int prows = plan & 0xff, pchunks = plan >> 8;  // rows per wavefront, chunks per range
    const int x0 = tl.bx * pchunks * XW;
    const int x1 = min(nx, x0 + pchunks * XW);
    const int K = (x1 - x0 + XW - 1) / XW;
    const int y0 = (tl.by * XWAVES + wave) * prows;
    const int nrows = max(0, min(prows, d.n[1] - y0));  // uniform over the wavefront
    const int R0 = tl.bz * d.n[1] + y0;                    // row index (z ny + y) of row 0
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};

    // Geometry: list the faces (item = row << 11 | face offset from x0) and reconstruct
    // the mixed donors of the listed faces 64 at a time (position q of the list: flux in
    // s_F[q], or in fgeo at the face beyond XFCAP).
    unsigned nwork = 0, ndone = 0;
    auto append = [&](bool need, unsigned item) {
        const unsigned long long bal = __ballot(need);
        if (need) W.work[(nwork + (unsigned)__popcll(bal & __lanemask_lt())) & 127] = (unsigned short)item;
        nwork += (unsigned)__popcll(bal);
    };
    auto reconstruct = [&]() {  // items ndone .. min(nwork, ndone + 64) - 1
        wave_lds_order();
        const unsigned q = ndone + lane;
        if (q < nwork) {
            const unsigned it = W.work[q & 127];
            const int r = it >> 11, f = x0 + (int)(it & 2047);
            const int R = R0 + r;
            const double lam = vel_at<MP>(a, (long)R * (nx + 1) + f) * a.kfac;
            const int xd = lam > 0.0 ? f - 1 : f;
            const double cd = a.c[(long)R * nx + wrap(xd, nx, d.bc[0])];
            if (lam != 0.0 && mixed(d, cd)) {
                double s = 1.0;
                if (d.split) {
                    const int fo = face_wrap(lam > 0.0 ? f - 1 : f + 1, nx, d.bc[0]);
                    s = donor_stretch(lam, vel_at<MP>(a, (long)R * (nx + 1) + fo) * a.kfac);
                }
                const double F = donor_flux<0, MP>(d, a.c, xd, y0 + r, tl.bz, cd, lam, s);
                if (q < XFCAP)
                    W.F[q] = F;
                else
                    a.fgeo[(long)R * (nx + 1) + f] = F;
            }
        }
        ndone = min(nwork, ndone + XW);
        wave_lds_order();
    };
    const bool need0 = lane < nrows && (mask64(d, a.mask, R0 + lane, x0 - 1) || mask64(d, a.mask, R0 + lane, x0));
    const unsigned pos0 = (unsigned)__popcll(__ballot(need0) & __lanemask_lt());  // list position
    append(need0, (unsigned)lane << 11);
    const unsigned nfirst = nwork;
    // the mask words x0 / 64 .. x0 / 64 + K of each row (0 past the row's end), and the
    // bits of the rows' ghost cells right of their last cells
    for (int i = lane; i < nrows * (XKMAX + 1); i += XW) {
        const int r = i / (XKMAX + 1), w = (x0 >> 6) + (i - r * (XKMAX + 1));
        W.mw[i] = w < d.wpr ? a.mask[(long)(R0 + r) * d.wpr + w] : 0ull;
    }
    const uint64_t gbits = __ballot(lane < nrows && mask64(d, a.mask, R0 + lane, nx));
    wave_lds_order();
    for (int r = 0; r < nrows; ++r) {
        const bool gbit = (gbits >> r) & 1ull;
        for (int k = 0; k < K; ++k) {
            const int x = x0 + 64 * k + lane;
            const uint64_t w0 = W.mw[r * (XKMAX + 1) + k], w1 = W.mw[r * (XKMAX + 1) + k + 1];
            const bool need = x_face_need(nx, w0, w1, x, lane, x < x1, gbit);
            const uint64_t bal = __ballot(need);
            if (lane == 0) W.bal[r * XKMAX + k] = bal;
            append(need, ((unsigned)r << 11) | (unsigned)(64 * k + lane + 1));
            while (nwork - ndone >= (unsigned)XW) reconstruct();
        }
    }
    if (nwork > ndone) reconstruct();
    if (nwork > XFCAP) __threadfence_block();  // fgeo entries are read back by other lanes

    // The first face (x0) of each row: lane r computes it for row r.
    if (lane < nrows) {
        const int R = R0 + lane;
        const long rb = (long)R * nx;
        const double lam = vel_at<MP>(a, (long)R * (nx + 1) + x0) * a.kfac;
        double Phi = 0.0, E = 0.0;
        if (lam != 0.0) {
            const int b = lam > 0.0 ? x0 - 3 : x0 + 2, st = lam > 0.0 ? 1 : -1;
            double Ts[5];
#pragma unroll
            for (int i = 0; i < 5; ++i) {
                const long id = rb + wrap(b + i * st, nx, d.bc[0]);
                Ts[i] = a.e[id] / cp_of(d, a.c[id]);
            }
            const double Tf = weno5(Ts[0], Ts[1], Ts[2], Ts[3], Ts[4], d.weno_eps);
            const double cd = a.c[rb + wrap(lam > 0.0 ? x0 - 1 : x0, nx, d.bc[0])];
            double F = fabs(lam) * cd;
            if (mixed(d, cd)) F = W.F[pos0];
            face_energy(d, lam, F, Tf, Phi, E);
        }
        W.first[0][lane] = Phi;
        W.first[1][lane] = E;
        W.first[2][lane] = lam;
    }

    // The walk. Prefetched registers: the next chunk to stage (c, e) and the next step's
    // face velocity and frozen fields (in their storage type).
    double pc = 0.0, pe = 0.0;
    T pu = 0, pec = 0;
    uint8_t pcc = 0;
    // Positions x0 - 2 + 64 j + lane of row R. The stencils read staged positions up to
    // (x1 - x0) + 4 only, so lanes past that load nothing (their slots are never read): the
    // chunk that wraps round a periodic row then fetches its few cells, not 64.
    auto load_chunk = [&](int R, int j) {
        if (64 * j + lane <= (x1 - x0) + 4) {
            const long id = (long)R * nx + wrap(x0 - 2 + 64 * j + lane, nx, d.bc[0]);
            pc = a.c[id];
            pe = a.e[id];
        }
    };
    auto load_step = [&](int R, int k) {  // right face and frozen fields of cell x0 + 64 k + lane
        const int x = x0 + 64 * k + lane;
        if (x < x1) {
            pu = vel_at<MP>(a, (long)R * (nx + 1) + x + 1);
            if (!a.first) {
                pcc = a.cc[(long)R * nx + x];
                pec = ec_at<MP>(a, (long)R * nx + x);
            }
        }
    };
    unsigned pos_base = nfirst;  // list position of the next step's first listed face
    // The stencils of a row's faces read staged positions up to (x1 - x0) + 4, so chunk K is
    // staged only if that reaches it.
    const int klast = (x1 - x0) + 4 >= XW * K ? K : K - 1;
    if (nrows > 0) load_chunk(R0, 0);
    for (int r = 0; r < nrows; ++r) {
        const int R = R0 + r;
        const long rb = (long)R * nx;
        for (int j = 0; j <= K; ++j) {
            if (j <= klast) {  // stage chunk j
                const int q = (64 * j + lane) & (XRING - 1);
                const double cj = pc, ej = pe;
                W.c[q] = cj;
                W.e[q] = ej;
                W.T[q] = ej / cp_of(d, cj);
            }
            if (j < klast)
                load_chunk(R, j + 1);
            else if (j == klast && r + 1 < nrows)
                load_chunk(R + 1, 0);
            const double u = (double)pu, ec_own = (double)pec;
            const uint8_t cc_own = pcc;
            if (j < K) load_step(R, j);
            wave_lds_order();
            if (j == 0) continue;
            // step k = j - 1: cell x = x0 + 64 k + lane (staged position p), right face x + 1
            const int k = j - 1;
            const int x = x0 + 64 * k + lane;
            const bool own = x < x1;
            const int p = 64 * k + lane + 2;
            const uint64_t bal = uniform64(W.bal[r * XKMAX + k]);
            const unsigned pos = pos_base + (unsigned)__popcll(bal & __lanemask_lt());
            pos_base += (unsigned)__popcll(bal);
            double Phi = 0.0, E = 0.0, lam = 0.0;
            if (own) {
                lam = u * a.kfac;
                if (lam != 0.0) {
                    const double cd = lam > 0.0 ? W.c[p & (XRING - 1)] : W.c[(p + 1) & (XRING - 1)];
                    // upwind stencil selected first (cells x-2 .. x+2, or x+3 .. x-1 mirrored),
                    // so that one WENO5 evaluation serves both signs
                    const int b = lam > 0.0 ? p - 2 : p + 3, st = lam > 0.0 ? 1 : -1;
                    const double Tf = weno5(W.T[b & (XRING - 1)], W.T[(b + st) & (XRING - 1)],
                                            W.T[(b + 2 * st) & (XRING - 1)],
                                            W.T[(b + 3 * st) & (XRING - 1)],
                                            W.T[(b + 4 * st) & (XRING - 1)], d.weno_eps);
                    double F = fabs(lam) * cd;
                    if (mixed(d, cd)) F = listed_flux(W.F, pos, XFCAP, a.fgeo + (long)R * (nx + 1) + x + 1);
                    face_energy(d, lam, F, Tf, Phi, E);
                }
            }
            // the left face of cell l is the face of lane l - 1; lane 0 reads the row's
            // carried face (its first face, then lane 63's face of the previous chunk)
            double PhiL = __shfl_up(Phi, 1, 64), EL = __shfl_up(E, 1, 64), lamL = __shfl_up(lam, 1, 64);
            if (lane == 0) {
                PhiL = W.first[0][r];
                EL = W.first[1][r];
                lamL = W.first[2][r];
            }
            wave_lds_order();
            if (lane == XW - 1) {
                W.first[0][r] = Phi;
                W.first[1][r] = E;
                W.first[2][r] = lam;
            }
            bool mx = false;
            if (own) {
                const int pq = p & (XRING - 1);
                const double cv = W.c[pq];
                double ELc = EL, ERc = E;
                cell_energy_flux(d, cv, ELc, ERc);
                const double cn = update_cell<MP>(d, a, rb + x, cv, W.e[pq], W.T[pq], lamL, lam, PhiL,
                                                  Phi, ELc, ERc, cc_own, ec_own, acc);
                mx = mixed(d, cn);
                if (d.bc[0] == 1) {
                    if (x == 0) {
                        acc[2] -= PhiL;
                        acc[3] -= ELc;
                    }
                    if (x == nx - 1) {
                        acc[2] += Phi;
                        acc[3] += ERc;
                    }
                }
            }
            // mask of the output: the chunk is one word
            const unsigned long long bits = __ballot(mx);
            if (lane == 0) a.mask_out[(long)R * d.wpr + (x0 >> 6) + k] = bits;
            wave_lds_order();
        }
    }
    block_sum8<XWAVES>(acc, a.part + tl.blk, a.part_stride);
}

// y and z sweeps: each thread owns one column along the sweep axis (x across the
// wavefront, so every load is coalesced) and marches over a chunk of it, keeping the
// fractions, energies and temperatures of cells f-3 .. f+2 in registers; each face
// flux is computed once and used by both neighbours.
template <int AX, bool MP>
__device__ __forceinline__ void sweep_t_body(const Dom& d, const SweepArgs& a, int chunk, const TileAt& tl) {
    constexpr int TA = AX == 1 ? 2 : 1;  // the transverse axis other than x
    __shared__ unsigned short s_work[4][128];  // listed faces not yet reconstructed (ring)
    __shared__ uint64_t s_mw[4][TCH + 2];      // input mask words of cells s0 - 1 .. s1
    __shared__ uint8_t s_idx[4][TCH + 1][64];  // list position of each listed face (at most TFCAP)
    __shared__ double s_F[4][TFCAP];           // liquid flux of listed faces, by list position
    const int lane = threadIdx.x, tr = threadIdx.y;
    const int bx = tl.bx, by = tl.by, bz = tl.bz;
    const int x = bx * 64 + lane;
    const int t = by * 4 + tr;
    const int nt = (d.ndim == 2 && TA == 2) ? 1 : d.n[TA];
    const bool ok = x < d.n[0] && t < nt;
    const int ns = d.n[AX];
    const int s0 = bz * chunk;
    const int s1 = min(s0 + chunk, ns);
    const long plane = (long)d.n[0] * d.n[1];
    const long base = ok ? (AX == 1 ? (long)t * plane + x : (long)t * d.n[0] + x) : 0;
    const long stride = AX == 1 ? d.n[0] : plane;
    const long fbase = ok ? (AX == 1 ? (long)t * (d.n[1] + 1) * d.n[0] + x : (long)t * d.n[0] + x) : 0;
    const long fstride = AX == 1 ? d.n[0] : plane;
    auto cell_id = [&](int cell) { return base + (long)wrap(cell, ns, d.bc[AX]) * stride; };

    // Geometry: the faces s0 .. s1 of the wavefront's columns with a mixed cell on either
    // side, in face order and lane order (item = face offset:lane). The 64 columns of a
    // wavefront are one mask word per cell of the sweep axis, so the words of
    // cells s0-1 .. s1 are staged in LDS and a face's list is the lanes of (w_j | w_j+1).
    // The mixed donors of the listed faces are reconstructed 64 at a time (list position
    // q: flux in s_F[q] below TFCAP, else in fgeo at the face); s_idx keeps each listed
    // face's position, saturated at TFCAP.
    const uint64_t okmask = __ballot(ok);
    const int nface = s1 - s0 + 1;
    for (int j = lane; j <= nface; j += 64) {
        uint64_t w = 0ull;
        if (t < nt) {
            const int cell = wrap(s0 - 1 + j, ns, d.bc[AX]);
            const long row = AX == 1 ? (long)t * d.n[1] + cell : (long)cell * d.n[1] + t;
            w = a.mask[row * d.wpr + bx];
        }
        s_mw[tr][j] = w;
    }
    wave_lds_order();
    auto listed = [&](int j) { return uniform64(s_mw[tr][j] | s_mw[tr][j + 1]) & okmask; };
    unsigned nwork = 0, ndone = 0;
    auto reconstruct = [&]() {  // items ndone .. min(nwork, ndone + 64) - 1
        wave_lds_order();
        const unsigned q = ndone + lane;
        if (q < nwork) {
            const unsigned it = s_work[tr][q & 127];
            const int fl = it >> 6, l = it & 63;
            const int xw = bx * 64 + l;
            const long bw = AX == 1 ? (long)t * plane + xw : (long)t * d.n[0] + xw;
            const long fw = AX == 1 ? (long)t * (d.n[1] + 1) * d.n[0] + xw : (long)t * d.n[0] + xw;
            const int f = s0 + fl;
            const double lam = vel_at<MP>(a, fw + (long)f * fstride) * a.kfac;
            const int sd = lam > 0.0 ? f - 1 : f;
            const double cd = a.c[bw + (long)wrap(sd, ns, d.bc[AX]) * stride];
            if (lam != 0.0 && mixed(d, cd)) {
                double sf = 1.0;
                if (d.split) {
                    const int fo = face_wrap(lam > 0.0 ? f - 1 : f + 1, ns, d.bc[AX]);
                    sf = donor_stretch(lam, vel_at<MP>(a, fw + (long)fo * fstride) * a.kfac);
                }
                const double F = AX == 1 ? donor_flux<1, MP>(d, a.c, xw, sd, t, cd, lam, sf)
                                         : donor_flux<2, MP>(d, a.c, xw, t, sd, cd, lam, sf);
                if (q < TFCAP)
                    s_F[tr][q] = F;
                else
                    a.fgeo[fw + (long)f * fstride] = F;
            }
        }
        ndone = min(nwork, ndone + 64u);
        wave_lds_order();
    };
    for (int j = 0; j < nface; ++j) {
        const uint64_t bal = listed(j);
        if ((bal >> lane) & 1ull) {
            const unsigned q = nwork + (unsigned)__popcll(bal & __lanemask_lt());
            s_work[tr][q & 127] = (unsigned short)((j << 6) | lane);
            s_idx[tr][j][lane] = (uint8_t)min(q, (unsigned)TFCAP);
        }
        nwork += (unsigned)__popcll(bal);
        while (nwork - ndone >= 64u) reconstruct();
    }
    if (nwork > ndone) reconstruct();
    // the overflow fluxes are read back by other lanes of this wavefront
    if (nwork > TFCAP) __threadfence_block();
    // Register ring of cells f-3 .. f+4 in slots (k + j) % 8, where k counts the faces
    // of the chunk and j = 0..7 the cells from f-3: cells f-3 .. f+2 are the WENO and
    // update window, cells f+3, f+4 are loads in flight; at each face the load of cell
    // f+5 is issued into the slot of cell f-3 (three faces ahead, so that many loads
    // stay in flight per wavefront). Face velocities and the frozen fields of the cell
    // to update use rings of VR slots, loaded VR faces ahead: four in the mixed mode,
    // two in double precision, where that keeps the kernel within 128 registers per lane
    // (four wavefronts per SIMD instead of three). The loop is unrolled eight times so
    // that every slot is a compile-time register.
    constexpr int R = 8;
    constexpr int VR = MP ? 4 : 2;
    static_assert(R % VR == 0, "the unrolled loop keeps the ring slots fixed");
    double cr[R], er[R], Tw[R];
    typename Prec<MP>::T vr[VR], ecr[VR];  // storage type until used
    uint8_t ccr[VR];
#pragma unroll
    for (int j = 0; j < R; ++j) {
        cr[j] = 0.0;
        er[j] = 0.0;
        Tw[j] = 0.0;
        if (ok) {
            const long id = cell_id(s0 - 3 + j);
            cr[j] = a.c[id];
            er[j] = a.e[id];
        }
    }
#pragma unroll
    for (int j = 0; j < VR; ++j) {
        vr[j] = 0.0;
        ecr[j] = 0.0;
        ccr[j] = 0;
        const int f = s0 + j;
        if (ok && f <= s1) {
            vr[j] = vel_at<MP>(a, fbase + (long)f * fstride);
            // cell f-1 is updated at face f; the first face updates nothing
            if (!a.first && j > 0) {
                ccr[j] = a.cc[base + (long)(f - 1) * stride];
                ecr[j] = ec_at<MP>(a, base + (long)(f - 1) * stride);
            }
        }
    }
#pragma unroll
    for (int j = 0; j < 5; ++j) Tw[j] = ok ? er[j] / cp_of(d, cr[j]) : 0.0;
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    double PhiP = 0.0, EP = 0.0, lamP = 0.0;
    auto step = [&](auto kc, int f) {
        constexpr int K = decltype(kc)::value;
        constexpr int J0 = K % R, J1 = (K + 1) % R, J2 = (K + 2) % R, J3 = (K + 3) % R, J4 = (K + 4) % R,
                      J5 = (K + 5) % R;
        constexpr int V = K % VR;
        Tw[J5] = ok ? er[J5] / cp_of(d, cr[J5]) : 0.0;
        const double lam = ok ? (double)vr[V] * a.kfac : 0.0;
        double Phi = 0.0, E = 0.0;
        if (lam != 0.0) {
            const double cd = lam > 0.0 ? cr[J2] : cr[J3];
            double F = fabs(lam) * cd;
            if (mixed(d, cd)) {
                const unsigned idx = s_idx[tr][f - s0][lane];
                F = listed_flux(s_F[tr], idx, TFCAP, a.fgeo + fbase + (long)f * fstride);
            }
            // upwind stencil selected first, so that one WENO5 evaluation serves both signs
            const bool pos = lam > 0.0;
            const double Tf = weno5(pos ? Tw[J0] : Tw[J5], pos ? Tw[J1] : Tw[J4], pos ? Tw[J2] : Tw[J3],
                                    pos ? Tw[J3] : Tw[J2], pos ? Tw[J4] : Tw[J1], d.weno_eps);
            face_energy(d, lam, F, Tf, Phi, E);
        }
        bool mx = false;
        if (ok && f > s0) {
            const int cell = f - 1;
            const long id = base + (long)cell * stride;
            double EL = EP, ER = E;
            cell_energy_flux(d, cr[J2], EL, ER);
            const double cn = update_cell<MP>(d, a, id, cr[J2], er[J2], Tw[J2], lamP, lam, PhiP, Phi, EL, ER,
                                              ccr[V], (double)ecr[V], acc);
            mx = mixed(d, cn);
            if (d.bc[AX] == 1) {
                if (cell == 0) {
                    acc[2] -= PhiP;
                    acc[3] -= EL;
                }
                if (cell == ns - 1) {
                    acc[2] += Phi;
                    acc[3] += ER;
                }
            }
        }
        if (f > s0) {  // mask of the output: the wavefront's 64 cells are one word
            const unsigned long long bits = __ballot(mx);
            if (lane == 0 && t < nt) {
                const long row = AX == 1 ? (long)t * d.n[1] + (f - 1) : (long)(f - 1) * d.n[1] + t;
                a.mask_out[row * d.wpr + bx] = bits;
            }
        }
        PhiP = Phi;
        EP = E;
        lamP = lam;
        // loads ahead into the slots just released
        if (ok) {
            if (f + 5 - 2 <= s1) {  // cell f+5 enters the window at face f+3
                const long id = cell_id(f + 5);
                cr[J0] = a.c[id];
                er[J0] = a.e[id];
            }
            if (f + VR <= s1) {
                vr[V] = vel_at<MP>(a, fbase + (long)(f + VR) * fstride);
                if (!a.first) {
                    ccr[V] = a.cc[base + (long)(f + VR - 1) * stride];
                    ecr[V] = ec_at<MP>(a, base + (long)(f + VR - 1) * stride);
                }
            }
        }
    };
    using std::integral_constant;
    for (int f = s0; f <= s1; f += R) {
        step(integral_constant<int, 0>{}, f);
        if (f + 1 > s1) break;
        step(integral_constant<int, 1>{}, f + 1);
        if (f + 2 > s1) break;
        step(integral_constant<int, 2>{}, f + 2);
        if (f + 3 > s1) break;
        step(integral_constant<int, 3>{}, f + 3);
        if (f + 4 > s1) break;
        step(integral_constant<int, 4>{}, f + 4);
        if (f + 5 > s1) break;
        step(integral_constant<int, 5>{}, f + 5);
        if (f + 6 > s1) break;
        step(integral_constant<int, 6>{}, f + 6);
        if (f + 7 > s1) break;
        step(integral_constant<int, 7>{}, f + 7);
    }
    block_sum8<4>(acc, a.part + tl.blk, a.part_stride);
}

// Kernel entry points. The x sweeps ask for five wavefronts per SIMD and the y / z
// sweeps for four (every variant fits without spilling).
__device__ __forceinline__ TileAt own_tile() {
    return {(int)blockIdx.x, (int)blockIdx.y, (int)blockIdx.z, block_linear()};
}
// Tile of a y / z sweep block, with the blocks of every whole aligned group of 64
// transposed as 8 x 8. The hardware deals consecutive blocks to the eight XCDs in turn
// (block 8 m + k of a group runs on XCD k), so the transpose hands XCD k the consecutive
// tiles 8 k .. 8 k + 7 of the group: neighbouring column blocks along x, which read the
// same cache lines of the mask words, of the c_c bytes and of the geometry halos, now
// through one L2. A trailing partial group keeps its order. The tile's partial-table
// row is its own linear index, as without the transpose. (Measured: y and z sweeps
// 3-4% faster at 512^3, 1-2% at 128^3 and 256^3; the x sweeps, whose blocks share
// little, gained at 256^3 only and keep the plain order.)
__device__ __forceinline__ TileAt xcd_tile() {
    const int b = block_linear();
    const int n = (int)(gridDim.x * gridDim.y * gridDim.z);
    const int L = (b | 63) < n ? (b & ~63) | ((b & 7) << 3) | ((b >> 3) & 7) : b;
    const int gx = (int)gridDim.x, gy = (int)gridDim.y;
    const int r = L / gx;
    return {L - r * gx, r % gy, r / gy, L};
}
__global__ void __launch_bounds__(XW* XWAVES) __attribute__((amdgpu_waves_per_eu(5, 8)))
k_sweep_x(Dom d, SweepArgs a, int plan) {
    sweep_x_body<false>(d, a, own_tile(), plan);
}
__global__ void __launch_bounds__(XW* XWAVES) __attribute__((amdgpu_waves_per_eu(5, 8)))
k_sweep_x_mixed(Dom d, SweepArgs a, int plan) {
    sweep_x_body<true>(d, a, own_tile(), plan);
}
template <int AX>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8)))
k_sweep_t(Dom d, SweepArgs a, int chunk) {
    sweep_t_body<AX, false>(d, a, chunk, xcd_tile());
}
template <int AX>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8)))
k_sweep_t_mixed(Dom d, SweepArgs a, int chunk) {
    sweep_t_body<AX, true>(d, a, chunk, xcd_tile());
}

// Batched sweeps: one launch advances the same sweep of many independent domains,
// one block per entry of a table of tiles (domain, tile coordinates in the domain's
// own launch grid, partial-table row). Each domain's Dom and SweepArgs come from
// device arrays, read into scalar registers; a tile computes exactly what the block
// of the single-domain launch with the same coordinates computes. (Blocks that loop
// over several tiles would keep the tables' fields live across the loop: 40 to 65
// more vector registers per lane and one wavefront per SIMD less.)
// A structure every lane of the block reads at the same address, moved into scalar
// registers one 32-bit word at a time (so that its fields do not occupy vector
// registers in the sweep bodies).
template <typename S>
__device__ __forceinline__ S uniform_load(const S* p) {
    static_assert(sizeof(S) % 4 == 0, "whole words");
    constexpr int kWords = (int)(sizeof(S) / 4);
    const unsigned* src = (const unsigned*)p;
    unsigned w[kWords];
#pragma unroll
    for (int i = 0; i < kWords; ++i) w[i] = __builtin_amdgcn_readfirstlane(src[i]);
    S out;
    memcpy(&out, w, sizeof(S));
    return out;
}

// The domain's arrays, addressed as global memory (the pointers come from a table).
__device__ __forceinline__ SweepArgs global_args(SweepArgs a) {
    a.c = in_global(a.c);
    a.e = in_global(a.e);
    a.mask = in_global(a.mask);
    a.mask_out = in_global(a.mask_out);
    a.cc = in_global(a.cc);
    a.ec = in_global(a.ec);
    a.vel = in_global(a.vel);
    a.fgeo = in_global(a.fgeo);
    a.c_out = in_global(a.c_out);
    a.e_out = in_global(a.e_out);
    a.part = in_global(a.part);
    return a;
}

template <bool MP>
__device__ __forceinline__ void sweep_x_tiles(const Dom* __restrict__ doms, const SweepArgs* __restrict__ args,
                                              const BatchTile* __restrict__ tiles, int ntiles) {
    const int t = blockIdx.x;
    if (t >= ntiles) return;
    const BatchTile bt = uniform_load(tiles + t);
    const Dom d = uniform_load(doms + bt.dom);
    const SweepArgs a = global_args(uniform_load(args + bt.dom));
    sweep_x_body<MP>(d, a, TileAt{bt.bx, bt.by, bt.bz, bt.blk}, bt.chunk);
}
template <int AX, bool MP>
__device__ __forceinline__ void sweep_t_tiles(const Dom* __restrict__ doms, const SweepArgs* __restrict__ args,
                                              const BatchTile* __restrict__ tiles, int ntiles) {
    const int t = blockIdx.x;
    if (t >= ntiles) return;
    const BatchTile bt = uniform_load(tiles + t);
    const Dom d = uniform_load(doms + bt.dom);
    const SweepArgs a = global_args(uniform_load(args + bt.dom));
    sweep_t_body<AX, MP>(d, a, bt.chunk, TileAt{bt.bx, bt.by, bt.bz, bt.blk});
}
__global__ void __launch_bounds__(XW* XWAVES) __attribute__((amdgpu_waves_per_eu(5, 8)))
k_sweep_x_batch(const Dom* doms, const SweepArgs* args, const BatchTile* tiles, int ntiles) {
    sweep_x_tiles<false>(doms, args, tiles, ntiles);
}
__global__ void __launch_bounds__(XW* XWAVES) __attribute__((amdgpu_waves_per_eu(5, 8)))
k_sweep_x_batch_mixed(const Dom* doms, const SweepArgs* args, const BatchTile* tiles, int ntiles) {
    sweep_x_tiles<true>(doms, args, tiles, ntiles);
}
template <int AX>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8)))
k_sweep_t_batch(const Dom* doms, const SweepArgs* args, const BatchTile* tiles, int ntiles) {
    sweep_t_tiles<AX, false>(doms, args, tiles, ntiles);
}
template <int AX>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8)))
k_sweep_t_batch_mixed(const Dom* doms, const SweepArgs* args, const BatchTile* tiles, int ntiles) {
    sweep_t_tiles<AX, true>(doms, args, tiles, ntiles);
}

}  // namespace

Launch cell_launch(const Dom& d) {
    Launch L;
    L.block = dim3(64, 4, 1);
    L.grid = dim3((d.n[0] + 63) / 64, (d.n[1] + 3) / 4, d.ndim == 2 ? 1 : d.n[2]);
    L.nblocks = (int)(L.grid.x * L.grid.y * L.grid.z);
    return L;
}

// Launch shape of a sweep. x: the rule's rows of one sub-row range per wavefront, four
// wavefronts per block (grid: sub-row ranges, row groups, planes; *chunk = the packed
// plan). y, z: 64 x 4 columns
// per block marching over a chunk of the sweep axis; the chunk is the longest of C, C / 2,
// ... 8 cells that still gives >= 4096 blocks (four rounds of blocks at four wavefronts
// per SIMD on 256 CUs; fewer, longer columns leave the last round partly idle), where C
// is TCH for mixed-precision y sweeps and TCH / 2 otherwise (the faster choice measured
// at 512^3: longer columns halve the halo reads, but the double-precision sweeps and the
// z sweeps, whose columns cross a plane per cell, gain nothing from them).
Launch sweep_launch(const Dom& d, int axis, bool mixed, int* chunk) {
    Launch L;
    L.block = dim3(64, 4, 1);
    const int nz = d.ndim == 2 ? 1 : d.n[2];
    if (axis == 0) {
        const XPlan p = x_plan_rule(d.n[0], d.n[1], nz);
        L.grid = dim3(p.splits, (d.n[1] + XWAVES * p.rows - 1) / (XWAVES * p.rows), nz);
        *chunk = x_plan_pack(p);
    } else {
        const int nt = axis == 1 ? nz : d.n[1];
        const long bxy = (long)((d.n[0] + 63) / 64) * ((nt + 3) / 4);
        const int ns = d.n[axis];
        int ch = mixed && axis == 1 ? TCH : TCH / 2;
        while (ch > 8 && bxy * ((ns + ch - 1) / ch) < 4096) ch >>= 1;
        *chunk = ch;
        L.grid = dim3((d.n[0] + 63) / 64, (nt + 3) / 4, (ns + ch - 1) / ch);
    }
    L.nblocks = (int)(L.grid.x * L.grid.y * L.grid.z);
    return L;
}

int max_sweep_tiles(const Dom& d, int axis) {
    // x: the rule's plan or one row per wavefront (the most blocks a batch may choose);
    // y / z: the shortest chunk a batch may choose (kMinChunk)
    if (axis == 0) return std::max(sweep_tiles(d, 0, false, 0, 0, nullptr), sweep_tiles(d, 0, false, 1, 0, nullptr));
    return sweep_tiles(d, axis, false, kMinChunk, 0, nullptr);
}

int max_partial_blocks(const Dom& d) {
    int m = std::max(cell_launch(d).nblocks, phase_launch(d).nblocks);
    for (int a = 0; a < d.ndim; ++a) m = std::max(m, max_sweep_tiles(d, a));
    return m;
}

hipError_t launch_classify(const Dom& d, const double* c, uint64_t* mask, hipStream_t s) {
    const Launch L = cell_launch(d);
    hipLaunchKernelGGL(k_classify, L.grid, L.block, 0, s, d, c, mask);
    return hipGetLastError();
}

// With events, the launch goes through hipExtLaunchKernelGGL, which records them with
// the kernel's own dispatch (so that they time the kernel alone).
template <bool MP>
void launch_sweep_kernel(const Dom& d, int axis, const Launch& L, int chunk, const SweepArgs& a, hipStream_t s,
                         hipEvent_t e0, hipEvent_t e1) {
    if (e0 && e1) {
        if (axis == 0)
            hipExtLaunchKernelGGL(MP ? k_sweep_x_mixed : k_sweep_x, L.grid, L.block, 0, s, e0, e1, 0, d, a, chunk);
        else if (axis == 1)
            hipExtLaunchKernelGGL(MP ? k_sweep_t_mixed<1> : k_sweep_t<1>, L.grid, L.block, 0, s, e0, e1, 0, d, a,
                                  chunk);
        else
            hipExtLaunchKernelGGL(MP ? k_sweep_t_mixed<2> : k_sweep_t<2>, L.grid, L.block, 0, s, e0, e1, 0, d, a,
                                  chunk);
        return;
    }
    if (axis == 0)
        hipLaunchKernelGGL(MP ? k_sweep_x_mixed : k_sweep_x, L.grid, L.block, 0, s, d, a, chunk);
    else if (axis == 1)
        hipLaunchKernelGGL(MP ? k_sweep_t_mixed<1> : k_sweep_t<1>, L.grid, L.block, 0, s, d, a, chunk);
    else
        hipLaunchKernelGGL(MP ? k_sweep_t_mixed<2> : k_sweep_t<2>, L.grid, L.block, 0, s, d, a, chunk);
}

size_t sweep_args_bytes() { return sizeof(SweepArgs); }

int max_chunk() { return TCH; }
int min_chunk() { return kMinChunk; }

void sweep_args_pack(const SweepIO& io, void* out) {
    SweepArgs a{io.c,    io.e,     io.mask,  io.first, io.mask_out, io.cc,   io.ec,
                io.vel,  io.kfac,  io.fgeo,  io.c_out, io.e_out,    io.part, io.part_stride};
    memcpy(out, &a, sizeof a);
}

hipError_t launch_sweep_batch(int axis, int mixed, const Dom* doms, const void* args, const BatchTile* tiles,
                              int ntiles, hipStream_t s) {
    const SweepArgs* a = (const SweepArgs*)args;
    const dim3 g(ntiles > 0 ? ntiles : 1), b(64, 4, 1);
    if (axis == 0)
        hipLaunchKernelGGL(mixed ? k_sweep_x_batch_mixed : k_sweep_x_batch, g, b, 0, s, doms, a, tiles, ntiles);
    else if (axis == 1)
        hipLaunchKernelGGL(mixed ? k_sweep_t_batch_mixed<1> : k_sweep_t_batch<1>, g, b, 0, s, doms, a, tiles, ntiles);
    else
        hipLaunchKernelGGL(mixed ? k_sweep_t_batch_mixed<2> : k_sweep_t_batch<2>, g, b, 0, s, doms, a, tiles, ntiles);
    return hipGetLastError();
}

int sweep_tiles(const Dom& d, int axis, bool mixed, int chunk, int dom, BatchTile* out) {
    int ch = 0;
    Launch L = sweep_launch(d, axis, mixed, &ch);
    if (axis == 0 && chunk > 0) {  // chunk: rows per wavefront
        const XPlan p = x_plan_rows(d.n[0], chunk);
        L.grid = dim3(p.splits, (d.n[1] + XWAVES * p.rows - 1) / (XWAVES * p.rows), L.grid.z);
        ch = x_plan_pack(p);
    } else if (axis != 0) {
        ch = chunk > 0 ? chunk : ch;
        L.grid.z = (d.n[axis] + ch - 1) / ch;
    }
    int k = 0;
    for (unsigned z = 0; z < L.grid.z; ++z)
        for (unsigned y = 0; y < L.grid.y; ++y)
            for (unsigned x = 0; x < L.grid.x; ++x, ++k)
                if (out) out[k] = BatchTile{dom, (int)x, (int)y, (int)z, k, ch};
    return k;
}

hipError_t launch_sweep(const Dom& d, int axis, const SweepIO& io, hipStream_t s) {
    int chunk = 0;
    const Launch L = sweep_launch(d, axis, io.mixed != 0, &chunk);
    SweepArgs a{io.c,    io.e,     io.mask,  io.first, io.mask_out, io.cc,   io.ec,
                io.vel,  io.kfac,  io.fgeo,  io.c_out, io.e_out,    io.part, io.part_stride};
    if (io.mixed)
        launch_sweep_kernel<true>(d, axis, L, chunk, a, s, io.ev_start, io.ev_stop);
    else
        launch_sweep_kernel<false>(d, axis, L, chunk, a, s, io.ev_start, io.ev_stop);
    *io.nblocks = L.nblocks;
    return hipGetLastError();
}


}  // namespace pcv
