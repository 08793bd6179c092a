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
    int* counts;      // per block of cells: number of unknowns; then exclusive offsets
    int* offs;
    int* total;       // number of unknowns
    int* nbr;         // per unknown, 6 slots: neighbouring unknown or -1
    double* coef;     // per unknown, 6 slots: 1 / rho_f of that neighbour
    double* dg;       // per unknown: sum of 1 / rho_f over its non-wall faces (diagonal)
    double* g;        // per unknown: right-hand side of the symmetric positive system
    double *x, *r, *z, *p, *q;  // conjugate-gradient vectors
    double* part;     // per block: two partial sums
    double* scal;     // scalars of the iteration (kCg*)
    double* ul;       // face buffer: u + u~ of one axis
    double* du;       // face buffer: u~ of one axis
};

constexpr int kExtFar = 100;
constexpr int kExtBlock = 256;
enum { kCgRz = 0, kCgAlpha = 1, kCgBeta = 2, kCgRr = 3, kCgGg = 4, kCgScalars = 8 };

struct ExtLayout {
    size_t lab, map, list, counts, offs, total, nbr, coef, dg, g, vec[5], part, scal, ul, du, bytes;
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
hipError_t launch_cg_iteration(int nu, const ExtIO& io, hipStream_t s);
// u + u~ (into io.ul) and u~ (into du_out, or io.du when du_out is null) on the faces
// of axis; vel is the stored velocity (float when mixed).
hipError_t launch_ext_faces(const Dom& d, int axis, const double* c, double rho_g, const void* vel, int mixed,
                            double* du_out, const ExtIO& io, hipStream_t s);

}  // namespace pcv
