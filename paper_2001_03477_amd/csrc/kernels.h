// Internal interface between the C-ABI layer and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pcv {

// Everything a kernel needs to know about a domain, passed by value.
struct Dom {
    int ndim;
    int n[3];      // cells per axis
    int bc[3];     // 0 periodic, 1 outflow
    long ncell;
    double cp_l, cp_g, rho_l, T_gamma, eps, weno_eps;
    int normal;
    int wpr;       // words per row of the mixed-cell masks: ceil(n[0] / 64)
    int ncons;     // 1: non-conservative energy flux (cells scale lambda T_f by their C_p)
    int split;     // 1: Lagrangian-explicit sweeps (donor stretched by 1 + lam_R - lam_L)
};

// Mixed-cell mask of a state: one bit per cell, rows of wpr = ceil(nx / 64) 64-bit words,
// word k of a row holding cells 64k .. 64k + 63 (bit = offset).

// Per-block partial sums written by every stage kernel: 8 doubles per block.
// Sweeps: clip_v, clip_e, bnd_v, bnd_e, src_v, src_e, tot_v, tot_e.
// Phase change: phase_v, phase_e, 0, 0, 0, 0, 0, 0 (the step's totals are the last
// sweep's plus these changes).
constexpr int kPartialWidth = 8;
constexpr int kSlots = 4;  // 3 sweeps + phase change

struct Launch {
    dim3 grid, block;
    int nblocks;
};
Launch cell_launch(const Dom& d);

// Largest number of blocks of any stage kernel (rows of the partial tables).
int max_partial_blocks(const Dom& d);

struct SweepIO {
    const double* c;
    const double* e;
    const uint64_t* mask;      // mixed cells of c
    uint64_t* mask_out;        // mixed cells of c_out
    uint8_t* cc;
    void* ec;                  // double, or float when mixed
    int first;                 // also freeze c_c and e_c of the step (the prologue)
    int mixed;                 // mixed-precision mode (single-precision geometry and storage)
    const void* vel;           // double, or float when mixed
    double kfac;               // lambda_f = vel_f * kfac
    double* fgeo;              // face array (layout of vel) for donor fluxes beyond the LDS tables
    double* c_out;
    double* e_out;
    double* part;              // partials: quantity q of block b at part[q * part_stride + b]
    long part_stride;
    int* nblocks;              // out: blocks of the sweep kernel
    hipEvent_t ev_start = nullptr;  // if set: events recorded with the kernel's dispatch
    hipEvent_t ev_stop = nullptr;
};
// Mask of the mixed cells of c, after the fractions were set.
hipError_t launch_classify(const Dom& d, const double* c, uint64_t* mask, hipStream_t s);

// A direction sweep is one launch (geometry of the mixed donors inside each tile).
hipError_t launch_sweep(const Dom& d, int axis, const SweepIO& io, hipStream_t s);

// Batched sweeps of many domains. A tile is one block of a domain's single-domain
// sweep launch: its coordinates in that launch grid, its row in the domain's partial
// table (blk) and, for y / z sweeps, the column chunk.
struct BatchTile {
    int dom, bx, by, bz, blk, chunk;  // chunk: y / z column chunk; x: the packed plan
};
// Tiles of a domain's sweep along axis (chunk <= 0: the single-domain rule; else, for
// y / z, the given column chunk, at most the longest supported, and for x the given rows
// per wavefront, 1, 2, 4 or 8); writes them to out (if not null) and returns their
// number. The tiles' blk rows stay below max_partial_blocks.
int sweep_tiles(const Dom& d, int axis, bool mixed, int chunk, int dom, BatchTile* out);
// Most tiles of any choice of sweep_tiles along axis.
int max_sweep_tiles(const Dom& d, int axis);
// The device form of a sweep's arguments (the batched kernels read one per domain).
size_t sweep_args_bytes();
void sweep_args_pack(const SweepIO& io, void* out);
// One launch over the ntiles tiles of a sweep along axis (one block per tile).
hipError_t launch_sweep_batch(int axis, int mixed, const Dom* doms, const void* args, const BatchTile* tiles,
                              int ntiles, hipStream_t s);
// Longest and shortest column chunks of the y / z sweeps (sweep_tiles accepts the
// powers of two between them).
int max_chunk();
int min_chunk();

struct PhaseIO {
    double* c;                 // updated in place
    double* e;                 // updated in place
    const uint64_t* mask;      // mixed cells of c
    uint64_t* mask_out;        // mixed cells after the step
    const double* mdot;
    double dt, h;
    double* rec;
    double* part;              // quantity 0: sum of Delta c, 1: sum of Delta e (per block)
    long part_stride;
    int* nblocks;              // out: blocks (partial rows); may be null
};
// Step 2: reconstruction of the moving cells, then the shift of the interface cells,
// in place, one lane per mask word.
Launch phase_launch(const Dom& d);
hipError_t launch_phase(const Dom& d, const PhaseIO& io, hipStream_t s);

// colsum[slot * 8 + q] = sum over the nb[slot] blocks of quantity q of slot.
hipError_t launch_colsum(const double* part, long part_stride, const int* nb, double* colsum, hipStream_t s);
// The same for many domains in one launch: domain i uses cs[i].
struct ColsumArgs {
    const double* part;
    long stride;
    int nb[4];
    double* colsum;
};
hipError_t launch_colsum_batch(int nd, const ColsumArgs* cs, hipStream_t s);

hipError_t launch_energy_from_T(const Dom& d, const double* c, const double* T, double* e, hipStream_t s);
hipError_t launch_T_from_energy(const Dom& d, const double* c, const double* e, double* T, hipStream_t s);
// flags[0] |= 1 (non-finite), 2 (outside [0,1] when check_range)
hipError_t launch_check(const double* x, long n, int check_range, unsigned int* flags, hipStream_t s);
// *maxbits = max over |x| as the bit pattern of a non-negative double (atomic max)
hipError_t launch_maxabs(const double* x, long n, unsigned long long* maxbits, hipStream_t s);
// flags |= 4 when the two boundary faces of a periodic axis differ
hipError_t launch_periodic_faces(const Dom& d, int axis, const double* vel, unsigned int* flags,
                                 hipStream_t s);

hipError_t launch_geom_volume(int n, const double* m, const double* a, double* out, hipStream_t s);
hipError_t launch_geom_alpha(int n, const double* m, const double* c, double* out, hipStream_t s);
hipError_t launch_geom_slab(int n, const double* m, const double* a, const int* axis, const double* lam,
                            double* out, hipStream_t s);
hipError_t launch_geom_normal(int n, const double* c27, int method, double* m, hipStream_t s);
hipError_t launch_geom_weno5(int n, const double* v, double eps, double* out, hipStream_t s);
// out[i] = (float)in[i]
hipError_t launch_to_float(long n, const double* in, float* out, hipStream_t s);

// Mass-transfer rate from the PLIC reconstruction (section 3.2) of a state (fractions
// c, energies e, mixed-cell mask): plane records (4 doubles per cell, mixed cells),
// the pure cells' normal gradients q (NaN where none), optional distances, and m''.
struct MassFluxIO {
    const double* c;
    const double* e;
    const uint64_t* mask;
    double* plane;
    double* q;
    double* dist;   // may be null
    double* mdot;
    double h, k_l, k_g, h_fg;
};
hipError_t launch_mass_flux(const Dom& d, const MassFluxIO& io, hipStream_t s);

}  // namespace pcv
