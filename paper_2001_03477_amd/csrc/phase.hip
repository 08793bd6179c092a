// Step 2 of the two-step advection (section 3.3.2) on gfx950: the interface of every
// mixed cell with a mass flux moves by Delta d = -(m'' / rho_l) dt / h along its
// normal, alpha* = alpha~ + |m|_2 Delta d, and the latent correction
// Delta e = Delta c (C_pl - C_pg) T_Gamma of section 3.4.1 follows every change of
// the volume fraction.
//
// Only cells at the interface can change: the mixed cells and their face neighbours.
// Both launches therefore work on the mixed-cell bitmask of the state, one lane per
// 64-bit mask word (a row segment of 63 or 64 cells), and visit only the set bits:
//   1. k_phase_recon: the plane record (m, alpha~, alpha*) of every mixed cell with a
//      non-zero mass flux;
//   2. k_phase_apply: each mixed cell takes V(m, alpha*) (the motion capped at the
//      cell's bounds), each pure face neighbour that a plane advances into takes the
//      volume that plane sweeps in it, averaged over those neighbours. The fractions
//      and energies are updated in place (a cell reads no neighbour's fraction or
//      energy), and the lane writes its word of the new state's mask in the same
//      layout as the input's.
// A wavefront's 64 lanes hold 64 consecutive mask words, so the mask is read
// coalesced. The cells to visit (the set bits of the wavefront's words) are then
// numbered across the wavefront and dealt to its lanes 64 at a time, so that a word
// with many interface cells (a row that grazes the interface) is shared by the whole
// wavefront instead of looping in one lane: the cost is the mask plus the interface
// cells, not the grid.
#include <hip/hip_runtime.h>

#include "common.h"

namespace pcv {

namespace {

constexpr int kPhaseBlock = 256;

// Word k of the mask row (z, y), located from the flat word index gw (rows of wpr
// words).
struct Seg {
    long row;   // z * ny + y
    int y, z;
    int k;      // word of the row
    int x0;     // first cell
    int n;      // cells in the segment (0: no segment)
};

__device__ __forceinline__ Seg seg_of(const Dom& d, long gw) {
    Seg s;
    const long nrows = (long)(d.ndim == 2 ? 1 : d.n[2]) * d.n[1];
    s.row = gw / d.wpr;
    s.k = (int)(gw - s.row * d.wpr);
    s.z = (int)(s.row / d.n[1]);
    s.y = (int)(s.row - (long)s.z * d.n[1]);
    s.x0 = s.k * 64;
    s.n = (s.row < nrows && s.x0 < d.n[0]) ? min(64, d.n[0] - s.x0) : 0;
    return s;
}

// The bits of a segment of n cells (1 <= n <= 64).
__device__ __forceinline__ uint64_t seg_bits(int n) { return n == 64 ? ~0ull : (1ull << n) - 1ull; }

// Bit of cell x in the mask row starting at word rowword.
__device__ __forceinline__ uint64_t bit_at(const uint64_t* __restrict__ mask, long rowword, int x) {
    return (mask[rowword + (x >> 6)] >> (x & 63)) & 1ull;
}

// Mask word k of the row (z, y) shifted by one cell along axis (1 or 2) in direction
// sg: the word of the neighbouring row (wrapped on periodic axes), or 0 beyond an
// outflow boundary or along the missing axis of a 2D grid.
__device__ __forceinline__ uint64_t row_word(const Dom& d, const uint64_t* __restrict__ mask, const Seg& s,
                                             int axis, int sg) {
    if (axis >= d.ndim) return 0ull;
    int y = s.y, z = s.z;
    int& q = axis == 1 ? y : z;
    const int n = d.n[axis];
    q += sg;
    if (q < 0 || q >= n) {
        if (d.bc[axis] == 1) return 0ull;
        q = q < 0 ? q + n : q - n;
    }
    return mask[((long)z * d.n[1] + y) * d.wpr + s.k];
}

// Mixed bit of the x neighbour of the segment's first (sg = -1) or last (sg = +1)
// cell: in the neighbouring word of the row, wrapped on a periodic x axis, 0 beyond an
// outflow boundary.
__device__ __forceinline__ uint64_t edge_bit(const Dom& d, const uint64_t* __restrict__ mask, const Seg& s,
                                             int sg) {
    int x = sg < 0 ? s.x0 - 1 : s.x0 + s.n;
    if (x < 0 || x >= d.n[0]) {
        if (d.bc[0] == 1) return 0ull;
        x = x < 0 ? x + d.n[0] : x - d.n[0];
    }
    return bit_at(mask, s.row * d.wpr, x);
}

// The set bits of the 64 lanes' words, numbered lane by lane and, within a word, in bit
// order: entry t of the wavefront's list is a bit of the first lane j whose inclusive
// prefix count exceeds t.
struct WaveList {
    int excl;   // entries before this lane's word
    int total;  // entries of the wavefront (uniform)
};

__device__ __forceinline__ WaveList wave_list(uint64_t w) {
    const int lane = threadIdx.x & 63;
    const int pop = __popcll(w);
    int incl = pop;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
    }
    return {incl - pop, __shfl(incl, 63, 64)};
}

// Entry t of the list: the lane j whose word holds it and the bit's rank in that word.
// Every lane of the wavefront must take part (the search reads other lanes).
__device__ __forceinline__ int wave_list_at(const WaveList& L, int t, int* rank) {
    int j = 0;
#pragma unroll
    for (int step = 32; step; step >>= 1) {
        // lanes 0 .. j+step-1 hold entries below t when the next lane's count does
        const int next = __shfl(L.excl, j + step, 64);
        if (j + step < 64 && next <= t) j += step;
    }
    *rank = t - __shfl(L.excl, j, 64);
    return j;
}

// Position of the set bit of rank k (0-based) of w.
__device__ __forceinline__ int nth_bit(uint64_t w, int k) {
    int pos = 0;
#pragma unroll
    for (int half = 32; half; half >>= 1) {
        const int c = __popcll(w & ((1ull << half) - 1ull));
        if (k >= c) {
            k -= c;
            w >>= half;
            pos += half;
        }
    }
    return pos;
}

__device__ __forceinline__ uint64_t shfl64(uint64_t v, int j) {
    const unsigned lo = __shfl((unsigned)v, j, 64), hi = __shfl((unsigned)(v >> 32), j, 64);
    return ((uint64_t)hi << 32) | lo;
}

__global__ void __launch_bounds__(kPhaseBlock)
k_phase_recon(Dom d, const double* __restrict__ c, const uint64_t* __restrict__ mask,
              const double* __restrict__ mdot, double dt_h, double* __restrict__ rec) {
    const int lane = threadIdx.x & 63;
    const long gw = (long)blockIdx.x * kPhaseBlock + threadIdx.x;
    const Seg s = seg_of(d, gw);
    // only the segment's own cells (bits beyond them are not cells of this word)
    const uint64_t w = s.n ? mask[gw] & seg_bits(s.n) : 0ull;
    const WaveList L = wave_list(w);
    for (int base = 0; base < L.total; base += 64) {
        const int t = base + lane;
        int rank;
        const int j = wave_list_at(L, t, &rank);
        const uint64_t wj = shfl64(w, j);
        if (t >= L.total) continue;
        const Seg sj = seg_of(d, gw - lane + j);
        const int x = sj.x0 + nth_bit(wj, rank);
        const long id = sj.row * d.n[0] + x;
        const double md = mdot[id];
        if (md == 0.0) continue;
        double c27[27];
        gather27(d, c, x, sj.y, sj.z, c27);
        const Normal nm = normal27(c27, d.normal);
        const double alpha = alpha_of(nm.m[0], nm.m[1], nm.m[2], c[id]);
        const double dd = -(md / d.rho_l) * dt_h;
        const double norm2 = sqrt(nm.m[0] * nm.m[0] + nm.m[1] * nm.m[1] + nm.m[2] * nm.m[2]);
        double* r = rec + 5 * id;
        r[0] = nm.m[0];
        r[1] = nm.m[1];
        r[2] = nm.m[2];
        r[3] = alpha;
        r[4] = alpha + norm2 * dd;
    }
}

__global__ void __launch_bounds__(kPhaseBlock)
k_phase_apply(Dom d, double* __restrict__ c, double* __restrict__ e, const uint64_t* __restrict__ mask,
              const double* __restrict__ mdot, double dt_h, const double* __restrict__ rec,
              uint64_t* __restrict__ mask_out, double* __restrict__ part, long part_stride) {
    constexpr int kWaves = kPhaseBlock / 64;
    // per word of the block: its mixed bits and the mixed bits of the six face
    // neighbours of its cells; the new state's mixed bits
    __shared__ uint64_t s_bits[7][kPhaseBlock];
    __shared__ unsigned long long s_out[kPhaseBlock];
    const int lane = threadIdx.x & 63;
    const long gw = (long)blockIdx.x * kPhaseBlock + threadIdx.x;
    const Seg s = seg_of(d, gw);
    uint64_t todo = 0ull;
    {
        uint64_t w = 0ull, nb[6] = {0ull, 0ull, 0ull, 0ull, 0ull, 0ull};
        if (s.n) {
            const uint64_t valid = seg_bits(s.n);
            w = mask[gw] & valid;
            nb[0] = ((w << 1) | edge_bit(d, mask, s, -1)) & valid;                    // x-
            nb[1] = ((w >> 1) | (edge_bit(d, mask, s, +1) << (s.n - 1))) & valid;     // x+
            nb[2] = row_word(d, mask, s, 1, -1) & valid;                                   // y-
            nb[3] = row_word(d, mask, s, 1, +1) & valid;                                   // y+
            nb[4] = row_word(d, mask, s, 2, -1) & valid;                                   // z-
            nb[5] = row_word(d, mask, s, 2, +1) & valid;                                   // z+
            todo = w | nb[0] | nb[1] | nb[2] | nb[3] | nb[4] | nb[5];
        }
        s_bits[0][threadIdx.x] = w;
#pragma unroll
        for (int j = 0; j < 6; ++j) s_bits[1 + j][threadIdx.x] = nb[j];
        s_out[threadIdx.x] = 0ull;
    }
    __syncthreads();
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const WaveList L = wave_list(todo);
    const int wbase = threadIdx.x - lane;  // the wavefront's first word in the block
    for (int base = 0; base < L.total; base += 64) {
        const int t = base + lane;
        int rank;
        const int j = wave_list_at(L, t, &rank);
        const uint64_t tj = shfl64(todo, j);
        if (t >= L.total) continue;
        const int sw = wbase + j;
        const Seg sj = seg_of(d, gw - lane + j);
        const int b = nth_bit(tj, rank);
        const int x = sj.x0 + b;
        const long id = sj.row * d.n[0] + x;
        const double cj = c[id];
        double cnew = cj;
        if ((s_bits[0][sw] >> b) & 1ull) {
            if (mdot[id] != 0.0) {
                const double* r = rec + 5 * id;
                cnew = volume(r[0], r[1], r[2], r[4]);
            }
        } else {
            // the neighbours visited in the fixed order x-, x+, y-, y+, z-, z+
            const double want = cj >= 1.0 - d.eps ? -1.0 : 1.0;
            const int pos[3] = {x, sj.y, sj.z};
            double sum = 0.0;
            int cnt = 0;
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                if (!((s_bits[1 + k][sw] >> b) & 1ull)) continue;
                const int ax = k >> 1, sg = (k & 1) ? 1 : -1;
                int q[3] = {pos[0], pos[1], pos[2]};
                q[ax] += sg;
                const long nid = ((long)wrap(q[2], d.ndim == 2 ? 1 : d.n[2], d.bc[2]) * d.n[1] +
                                  wrap(q[1], d.n[1], d.bc[1])) * d.n[0] + wrap(q[0], d.n[0], d.bc[0]);
                const double mdn = mdot[nid];
                if (mdn == 0.0) continue;
                const double dd = -(mdn / d.rho_l) * dt_h;
                const double motion = dd > 0.0 ? 1.0 : -1.0;
                if (motion != want) continue;
                const double* r = rec + 5 * nid;
                const double mo = -sg * r[ax];
                sum += volume(r[0], r[1], r[2], r[3] - mo) - volume(r[0], r[1], r[2], r[4] - mo);
                ++cnt;
            }
            if (cnt) cnew = cj - sum / cnt;
        }
        const double dc = cnew - cj;
        if (dc != 0.0) {
            const double de = (dc * (d.cp_l - d.cp_g)) * d.T_gamma;
            c[id] = cnew;
            e[id] = e[id] + de;
            acc[0] += dc;
            acc[1] += de;
        }
        if (mixed(d, cnew)) atomicOr(&s_out[sw], 1ull << b);
    }
    __syncthreads();
    if (s.n) mask_out[gw] = s_out[threadIdx.x];
    // the step totals come from the last sweep's sums plus these changes
    block_sum8<kWaves>(acc, part + blockIdx.x, part_stride, 0xFCu);
}

}  // namespace

Launch phase_launch(const Dom& d) {
    Launch L;
    const long words = (long)(d.ndim == 2 ? 1 : d.n[2]) * d.n[1] * d.wpr;
    L.block = dim3(kPhaseBlock, 1, 1);
    L.grid = dim3((unsigned)((words + kPhaseBlock - 1) / kPhaseBlock), 1, 1);
    L.nblocks = (int)L.grid.x;
    return L;
}

hipError_t launch_phase(const Dom& d, const PhaseIO& io, hipStream_t s) {
    const double dt_h = io.dt / io.h;
    const Launch L = phase_launch(d);
    hipLaunchKernelGGL(k_phase_recon, L.grid, L.block, 0, s, d, io.c, io.mask, io.mdot, dt_h, io.rec);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k_phase_apply, L.grid, L.block, 0, s, d, io.c, io.e, io.mask, io.mdot, dt_h,
                       io.rec, io.mask_out, io.part, io.part_stride);
    if (io.nblocks) *io.nblocks = L.nblocks;
    return hipGetLastError();
}

}  // namespace pcv
