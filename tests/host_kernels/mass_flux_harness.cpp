// TEST INFRASTRUCTURE (tests/test_host_mass_flux.py). Runs the library's mass-flux
// kernels (section 3.2) on the host over their exact launch grid, each buffer in an
// allocation of exactly the size the library's workspace gives it, so that
// AddressSanitizer reports any access outside it. Input: a binary file of the grid,
// the parameters, c and e; output: m'' and the distances.
#include "hip/hip_runtime.h"
thread_local dim3 threadIdx, blockIdx, blockDim, gridDim;
#include "../../paper_2001_03477_amd/csrc/massflux.hip"  // the library source, unchanged

namespace pcv {
Launch cell_launch(const Dom& d) {  // as in sweep.hip
    Launch L;
    L.block = dim3(64, 4, 1);
    L.grid = dim3((d.n[0] + 63) / 64, (d.n[1] + 3) / 4, d.ndim == 2 ? 1 : d.n[2]);
    L.nblocks = (int)(L.grid.x * L.grid.y * L.grid.z);
    return L;
}
}  // namespace pcv

template <typename T>
static T* alloc(size_t n) {
    T* p = (T*)malloc(n * sizeof(T));
    if (!p) abort();
    for (size_t i = 0; i < n * sizeof(T); ++i) ((unsigned char*)p)[i] = 0xA5;  // garbage, like device memory
    return p;
}

int main(int argc, char** argv) {
    FILE* f = fopen(argv[1], "rb");
    int hdr[8];
    double par[8];
    if (fread(hdr, sizeof hdr, 1, f) != 1 || fread(par, sizeof par, 1, f) != 1) return 2;
    pcv::Dom d;
    d.ndim = hdr[0];
    d.n[0] = hdr[1]; d.n[1] = hdr[2]; d.n[2] = hdr[3];
    d.bc[0] = hdr[4]; d.bc[1] = hdr[5]; d.bc[2] = hdr[6];
    d.normal = hdr[7];
    d.ncell = (long)d.n[0] * d.n[1] * d.n[2];
    d.cp_l = par[0]; d.cp_g = par[1]; d.rho_l = 1.0; d.T_gamma = par[2]; d.eps = 1e-12; d.weno_eps = 1e-6;
    d.wpr = (d.n[0] + 63) / 64;
    d.ncons = 0; d.split = 0;
    const double h = par[3], k_l = par[4], k_g = par[5], h_fg = par[6];
    const size_t N = (size_t)d.ncell;
    double* c = alloc<double>(N);
    double* e = alloc<double>(N);
    if (fread(c, 8, N, f) != N || fread(e, 8, N, f) != N) return 3;
    fclose(f);
    // the classification mask after set_vof (64 cells per word, one word per 64-cell block row)
    const size_t words = (size_t)d.n[2] * d.n[1] * d.wpr;
    uint64_t* mask = alloc<uint64_t>(words);
    for (int z = 0; z < d.n[2]; ++z)
        for (int y = 0; y < d.n[1]; ++y)
            for (int bx = 0; bx < (d.n[0] + 63) / 64; ++bx) {
                uint64_t bits = 0;
                for (int l = 0; l < 64; ++l) {
                    const int x = bx * 64 + l;
                    if (x < d.n[0]) {
                        const double cv = c[((size_t)z * d.n[1] + y) * d.n[0] + x];
                        if (cv > d.eps && cv < 1.0 - d.eps) bits |= 1ull << l;
                    }
                }
                mask[((size_t)z * d.n[1] + y) * d.wpr + bx] = bits;
            }
    // workspace sizes of capi.cpp: rec 5N doubles, fgeo the largest face count, mdot N;
    // the caller's distance array N
    size_t maxf = 1;
    const size_t nx = d.n[0], ny = d.n[1], nz = d.n[2];
    const size_t fc[3] = {nz * ny * (nx + 1), nz * (ny + 1) * nx, (nz + 1) * ny * nx};
    for (int a = 0; a < 3; ++a) maxf = std::max(maxf, a < d.ndim ? fc[a] : (size_t)1);
    double* rec = alloc<double>(5 * N);
    double* fgeo = alloc<double>(maxf);
    double* mdot = alloc<double>(N);
    double* dist = alloc<double>(N);
    pcv::MassFluxIO io;
    io.c = c; io.e = e; io.mask = mask;
    io.plane = rec; io.q = fgeo; io.dist = dist; io.mdot = mdot;
    io.h = h; io.k_l = k_l; io.k_g = k_g; io.h_fg = h_fg;
    const pcv::Launch L = pcv::cell_launch(d);
    fprintf(stderr, "grid %u x %u x %u, block %u x %u\n", L.grid.x, L.grid.y, L.grid.z, L.block.x, L.block.y);
    if (pcv::launch_mass_flux(d, io, nullptr) != 0) return 4;
    FILE* o = fopen(argv[2], "wb");
    fwrite(mdot, 8, N, o);
    fwrite(dist, 8, N, o);
    fclose(o);
    return 0;
}
