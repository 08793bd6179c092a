// Internal interface of the liquid-velocity extension (section 3.3.1, eq. press_inv)
// between the C-ABI layer and its HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "kernels.h"

namespace pcv {

// Views into the caller's extension workspace (ext_layout gives the offsets). Sizes
// are for the worst case of every cell in the sub-domain; nu of them are used.
struct ExtIO {
    int8_t* lab;      // per cell: 0 mixed, 1..3 gas layers, -1 liquid, kExtFar other gas
    int* map;         // per cell: index among the unknowns, or -1
    int* list;        // per unknown: its cell
    int* counts;      // per run of kExtCells cells: number of unknowns; then exclusive offsets
    int* offs;
    int* total;       // number of unknowns
    int* nbr;         // per unknown, 6 slots: neighbouring unknown or -1
    double* coef;     // per unknown, 6 slots: 1 / rho_f of that neighbour
    double* dg;       // per unknown: sum of 1 / rho_f over its non-wall faces (diagonal)
    double* g;        // per unknown: right-hand side of the symmetric positive system
    double *x, *r, *z, *p, *q, *p2;  // conjugate-gradient vectors (p2, p: directions of odd, even iterations)
    double* part;     // per block: two partial sums (start, product)
    double* part2;    // per block: two partial sums (update)
    double* scal;     // scalars of the iteration (kCg*)
    double* du;       // face buffer: u~ of one axis (for host output)
};

constexpr int kExtFar = 100;
constexpr int kExtBlock = 256;
constexpr int kExtCells = 4096;     // cells per run of the compaction
constexpr int kExtScanBlock = 1024;
enum { kCgRz = 0, kCgAlpha = 1, kCgBeta = 2, kCgRr = 3, kCgGg = 4, kCgScalars = 8 };

struct ExtLayout {
    size_t lab, map, list, counts, offs, total, nbr, coef, dg, g, vec[6], part, part2, scal, du, bytes;
};
ExtLayout ext_layout(const Dom& d, long max_faces);
ExtIO ext_views(const ExtLayout& L, void* ws);

// Labels of the cells, then the unknowns in cell order (list, map, *total).
hipError_t launch_ext_labels(const Dom& d, const double* c, const ExtIO& io, hipStream_t s);
// Operator and right-hand side over the nu unknowns: S = 1/rho_g - 1/rho_l.
hipError_t launch_ext_assemble(const Dom& d, const double* c, const double* mdot, double rho_g, int nu,
                               const ExtIO& io, hipStream_t s);
// Conjugate gradients with the diagonal as preconditioner: start (x = 0), then one
// iteration; scal[kCgRr] and scal[kCgGg] hold |r|^2 and |g|^2 after each.
hipError_t launch_cg_start(int nu, const ExtIO& io, hipStream_t s);
hipError_t launch_cg_iteration(int nu, int iter, const ExtIO& io, hipStream_t s);
// The stored velocity of axis (float when mixed) becomes u + u~ in place; du (may be
// null) receives u~ per face; *maxbits (zeroed by the caller) the largest |u + u~| as
// the bit pattern of a non-negative double.
hipError_t launch_ext_faces(const Dom& d, int axis, const double* c, double rho_g, void* vel, int mixed, double* du,
                            unsigned long long* maxbits, const ExtIO& io, hipStream_t s);

}  // namespace pcv
