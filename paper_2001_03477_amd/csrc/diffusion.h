// Internal interface of the implicit energy diffusion with the interface temperature
// imposed (section 3.4.2) between the C-ABI layer and its HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

#include "kernels.h"

namespace pcv {

constexpr int kDiffBlock = 256;
constexpr int kDiffGrid = 2048;  // blocks of the grid-stride kernels (and partials per reduction)
enum { kBiRho = 0, kBiAlpha = 1, kBiOmega = 2, kBiBeta = 3, kBiRr = 4, kBiBb = 5, kBiScalars = 8 };

// Views into the caller's diffusion workspace (diff_layout gives the offsets).
struct DiffIO {
    double* diag;   // per cell: diagonal of the backward-Euler operator
    double* off;    // 6 slots x cells (slot-major): coefficient of the face neighbour (0: wall or interface)
    double* b;      // per cell: right-hand side (T* and the T_Gamma terms)
    double *x, *r, *rh, *p, *v, *s, *t, *ph, *sh;  // BiCGSTAB vectors (x: T^{n+1})
    double* part;   // 3 partial sums per block of the fixed grid
    double* scal;   // kBi* scalars
};

struct DiffLayout {
    size_t diag, off, b, vec[9], part, scal, bytes;
};
DiffLayout diff_layout(const Dom& d);
DiffIO diff_views(const DiffLayout& L, void* ws);

// Operator, right-hand side and x = T* from the state (c, e); BiCGSTAB start:
// scal[kBiRr] = |r|^2, scal[kBiBb] = |b|^2.
hipError_t launch_diff_start(const Dom& d, const double* c, const double* e, double h, double dt, double k_l,
                             double k_g, const DiffIO& io, hipStream_t s);
// One BiCGSTAB iteration (scal[kBiRr] updated).
hipError_t launch_diff_iteration(const Dom& d, const DiffIO& io, hipStream_t s);
// e = C_p(c) T^{n+1}; T_out (may be null) = T^{n+1}.
hipError_t launch_diff_finish(const Dom& d, const double* c, double* e, double* T_out, const DiffIO& io,
                              hipStream_t s);

}  // namespace pcv
