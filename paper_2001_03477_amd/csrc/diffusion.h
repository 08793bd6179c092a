// Internal interface of the implicit energy diffusion with the interface temperature
// imposed (section 3.4.2) between the C-ABI layer and its HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "kernels.h"

namespace pcv {

constexpr int kDiffBlock = 256;
constexpr int kDiffGrid = 2048;  // blocks of the grid-stride kernels (and partials per reduction)
enum { kBiRho = 0, kBiAlpha = 1, kBiOmega = 2, kBiBeta = 3, kBiRr = 4, kBiBb = 5, kBiScalars = 8 };

// Neighbour coefficient of a phase's regular row (a node of that phase whose sides are
// nodes of the same phase or walls); index 0 gas, 1 liquid.
struct RowConst {
    double c[2];
};
// The operator: per cell a kind byte (bit 0 liquid, bit 1 stored row, bits 2 to 7 the
// wall sides), the stored rows' diagonal and coefficients, the regular rows' constants.
struct Rows {
    const uint8_t* kind;
    const double* diag;
    const double* off;
    RowConst rc;
};

// Multigrid preconditioner: levels of 2 x 2 x 2 aggregates (2 x 2 in 2D) down to at most
// 8 cells along the shortest axis; level l > 0 holds an explicit seven-point operator
// (diagonal, six neighbour coefficients slot-major in the sides' order x-, x+, y-, y+,
// z-, z+) and its vectors (right-hand side b, iterate x, scratch y).
constexpr int kMgMaxLevels = 12;
struct MgLevel {
    int n[3];
    long ncell;
    double *diag, *off, *b, *x, *y;
};

// Views into the caller's diffusion workspace (diff_layout gives the offsets).
struct DiffIO {
    uint8_t* kind;  // per cell: bit 0 liquid, bit 1 row stored (an interface side), bits 2-7 wall sides
    double* diag;   // per cell: diagonal of the backward-Euler operator (stored rows)
    double* off;    // 6 slots x cells (slot-major): coefficient of the face neighbour (0: wall or interface)
    double* b;      // per cell: right-hand side (T* and the T_Gamma terms)
    double *x, *r, *rh, *p, *v, *s, *t, *ph, *sh;  // BiCGSTAB vectors (x: T^{n+1})
    double* part;   // 3 partial sums per block of the fixed grid
    double* scal;   // kBi* scalars
    Rows rows;      // the operator as the kernels read it (rc set by launch_diff_start)
    double* mgx0;                // level-0 iterate of the V-cycle
    int mg_levels;               // levels including the cells' own (1: Jacobi steps only)
    MgLevel mg[kMgMaxLevels];    // mg[l], l >= 1: the coarse levels
};

struct DiffLayout {
    size_t kind, diag, off, b, vec[9], part, scal, mgx0, bytes;
    int mg_levels;
    int mg_n[kMgMaxLevels][3];
    size_t mg_diag[kMgMaxLevels], mg_off[kMgMaxLevels], mg_b[kMgMaxLevels], mg_x[kMgMaxLevels], mg_y[kMgMaxLevels];
};
DiffLayout diff_layout(const Dom& d);
DiffIO diff_views(const DiffLayout& L, void* ws);

// Operator, right-hand side and x = T* from the state (c, e), the coarse operators of the
// multigrid preconditioner; BiCGSTAB start: scal[kBiRr] = |r|^2, scal[kBiBb] = |b|^2.
hipError_t launch_diff_start(const Dom& d, const double* c, const double* e, double h, double dt, double k_l,
                             double k_g, DiffIO& io, hipStream_t s);
// One BiCGSTAB iteration (scal[kBiRr] updated).
hipError_t launch_diff_iteration(const Dom& d, const DiffIO& io, hipStream_t s);
// The diffusion's scratch for callers that cannot allocate: a file-scope device array
// of kDiffStaticBytes on every GPU the library runs on (held until the process ends).
// Its address on `device`, looked up once per device with that device current.
constexpr size_t kDiffStaticBytes = size_t(256) << 20;
hipError_t diff_static_scratch(int device, void** ptr, size_t* bytes);

// e = C_p(c) T^{n+1}; T_out (may be null) = T^{n+1}.
hipError_t launch_diff_finish(const Dom& d, const double* c, double* e, double* T_out, const DiffIO& io,
                              hipStream_t s);

}  // namespace pcv
