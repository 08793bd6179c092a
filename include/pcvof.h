/*
 * pcvof -- geometric PLIC-VOF advection with conservative thermal-energy
 * advection and the two-step phase-change shift, on AMD Instinct MI355X (gfx950).
 *
 * One call to pcvof_advect_step advances the volume fraction c and the thermal
 * energy e = C_p T (C_p = rho c_p per unit volume, eq. c_vol_avg) of a uniform
 * Cartesian MAC grid by one time step:
 *   - step 1 of the paper's VOF scheme (section 3.3.1): ndim direction-split
 *     geometric sweeps with the given divergence-free liquid velocity; each sweep
 *     reconstructs a plane m.x = alpha per mixed cell (section 3.2, eq. plane_m),
 *     takes the liquid volume of the upwind face-flux region of the donor cell, and
 *     carries the heat capacity of the fluxed liquid and gas volumes at the WENO5
 *     face temperature (section 3.4.1, eq. disc_et_adv);
 *   - step 2 (section 3.3.2, eq. vof_step2_full): the interface shift by
 *     Delta d = -(m''/rho_l) dt / h in mixed cells, with the capped motion carried
 *     into the neighbours the interface moves into, and the latent energy correction
 *     Delta e = Delta c (C_pl - C_pg) T_Gamma (section 3.4.1).
 * Around the step: pcvof_extend_velocity turns a one-fluid velocity into the liquid
 * velocity of step 1 (section 3.3.1, eq. press_inv), pcvof_diffuse takes one implicit
 * energy-diffusion step with T_Gamma at the interface (section 3.4.2), and
 * pcvof_compute_mass_flux would give m'' from the reconstruction (section 3.2; its
 * kernels are switched off in this version).
 *
 * Layout. Cell arrays are [nz][ny][nx] doubles, x fastest. MAC face velocities:
 * u [nz][ny][nx+1] on x-faces, v [nz][ny+1][nx] on y-faces, w [nz+1][ny][nx] on
 * z-faces (face i lies between cells i-1 and i). For a periodic axis the last face
 * must equal the first. 2D grids have ndim = 2, nz = 1 and no w.
 *
 * Ownership. The caller owns all memory: a 256-byte aligned device workspace of
 * pcvof_workspace_bytes() bytes (for instance a torch uint8 tensor), the workspaces
 * the extension and the diffusion take per call, and the HIP
 * stream (for instance torch.cuda.current_stream().cuda_stream). The library never
 * allocates device memory, never keeps pointers passed to set_/get_ calls, and
 * enqueues all work on the given stream. Calls with mem = PCVOF_MEM_DEVICE copy
 * asynchronously on the stream; calls with mem = PCVOF_MEM_HOST return after the
 * copy has completed.
 *
 * Errors. Every call returns a status (0 = PCVOF_OK, negative = error) and never
 * throws or exits; pcvof_last_error() gives a message for the calling thread.
 */
#ifndef PCVOF_H
#define PCVOF_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    PCVOF_OK = 0,
    PCVOF_ERR_ARG = -1,        /* invalid argument (null pointer, bad size, bad enum) */
    PCVOF_ERR_CFL = -2,        /* max |u_f| * |u_scale| * dt / h above params.cfl_max */
    PCVOF_ERR_NONFINITE = -3,  /* NaN or Inf in an input field */
    PCVOF_ERR_BOUNDS = -4,     /* volume fraction outside [0, 1] */
    PCVOF_ERR_WORKSPACE = -5,  /* workspace too small or misaligned */
    PCVOF_ERR_HIP = -6,        /* a HIP runtime call failed */
    PCVOF_ERR_STATE = -7       /* call out of order (e.g. step before set_vof) */
};

enum { PCVOF_MEM_HOST = 0, PCVOF_MEM_DEVICE = 1 };
enum { PCVOF_BC_PERIODIC = 0, PCVOF_BC_OUTFLOW = 1 };
enum { PCVOF_NORMAL_YOUNGS = 0, PCVOF_NORMAL_MYC = 1, PCVOF_NORMAL_CC = 2 };
/* Arithmetic of the advection step. FP64: everything in double precision. MIXED: the
   face velocities and the frozen energy coefficient e_c are stored in single
   precision (velocities are converted when set), and the interface normal, plane
   constant and upwind slab volume of mixed donors are evaluated in single precision,
   except that the plane constant and slab volume stay in double precision for
   fractions within 1e-3 of 0 or 1; fluxes are kept within the bounds of an exact slab
   volume. Volume fractions, energies, flux differences, clipping, step 2 and all
   checksums stay in double precision, so volume and energy remain conserved to
   round-off; the fractions differ from the FP64 result at the level of single
   precision rounding of the geometry. The mixed-cell threshold of this mode is
   max(eps_mixed, 1e-6): single-precision rounding of the fluxes leaves fractions of
   order 1e-8 in cells the FP64 path leaves pure, and those are not interface cells. */
enum { PCVOF_PREC_FP64 = 0, PCVOF_PREC_MIXED = 1 };
/* Energy flux of the sweeps (section 3.4.1). CONSERVATIVE (eq. disc_et_adv): the face
   carries the fluxed heat capacity of the geometric liquid and gas volumes times the
   WENO5 face temperature, E_f = sgn(lambda) [C_pl F + C_pg (|lambda| - F)] T_f, so that
   the energy is conserved and a uniform temperature stays uniform.
   NONCONSERVATIVE (eq. disc_et_adv_noncons, the approximation the paper argues
   against): the face carries lambda T_f and each cell multiplies the difference of its
   two faces by its own heat capacity C_p(c) of the current sweep; energy is then not
   conserved (stats.energy no longer obeys the bookkeeping identity) and temperatures
   near the interface drift. Provided as an ablation of the conservative scheme. */
enum { PCVOF_EFLUX_CONSERVATIVE = 0, PCVOF_EFLUX_NONCONSERVATIVE = 1 };
/* Direction-split scheme of the sweeps (section 3.3 names both). WY: the Eulerian-
   implicit sweeps of Weymouth and Yue that the paper builds on; the face flux is the
   liquid of the donor slab of width |lambda| and the dilatation terms use c_c and e_c
   frozen over the step, so volume and energy are conserved in a divergence-free field.
   LE: the Lagrangian-explicit sweeps of Li (CIAM); every point of the donor moves with
   the velocity interpolated linearly between the donor's two faces, which stretches
   the donor by s = 1 + (lambda_R - lambda_L): the face flux is s times the liquid of the
   donor slab of width |lambda| / s, and the dilatation terms use the current c and e
   (c' = s c - (Phi_R - Phi_L)). Fractions then stay in [0, 1] without clipping, but the
   dilatation terms do not cancel over the sweeps of a step: volume and energy are not
   conserved (stats.vol_src and stats.energy_src report the change). Beyond an outflow
   boundary the ghost donor is not stretched (s = 1). Provided as an ablation. */
enum { PCVOF_SPLIT_WY = 0, PCVOF_SPLIT_LE = 1 };

typedef struct {
    int ndim;        /* 2 or 3 */
    int nx, ny, nz;  /* cells per axis (nz == 1 when ndim == 2), each >= 1 */
    double h;        /* cubic cell edge, > 0 */
    int bc[3];       /* per axis x, y, z: PCVOF_BC_PERIODIC or PCVOF_BC_OUTFLOW
                        (outflow: ghost cells copy the nearest interior cell) */
} pcvof_grid;

typedef struct {
    double cp_l, cp_g;  /* volumetric heat capacities rho c_p of liquid and gas, > 0 */
    double rho_l;       /* liquid density used by the phase-change shift, > 0 */
    double T_gamma;     /* interface (saturation) temperature */
    double eps_mixed;   /* mixed cell: eps < c < 1 - eps (section 3.1 uses 1e-12) */
    double weno_eps;    /* epsilon of the WENO5 nonlinear weights (1e-6) */
    double cfl_max;     /* largest admissible face CFL number (0.5) */
    int normal;         /* PCVOF_NORMAL_*: interface normal estimator (MYC per section 3.2) */
    int precision;      /* PCVOF_PREC_* */
    int energy_flux;    /* PCVOF_EFLUX_* (CONSERVATIVE is the paper's scheme) */
    int split;          /* PCVOF_SPLIT_* (WY is the paper's scheme) */
} pcvof_params;

/* Checksums of one step (cell volume hv = h^ndim). The change of total volume obeys
   vol(n+1) - vol(n) = -vol_bnd_out + vol_src + vol_clip + vol_phase, and likewise for
   the energy, up to round-off. */
typedef struct {
    double vol, energy;                  /* hv * sum c, hv * sum e after the step */
    double vol_clip, energy_clip;        /* sweep clipping of c into [0,1] (T kept) */
    double vol_phase, energy_phase;      /* step 2 change of c, and its latent correction */
    double vol_bnd_out, energy_bnd_out;  /* net outflow through outflow boundaries */
    double vol_src, energy_src;          /* split dilatation terms c_c dlam, e_c dlam */
    double max_cfl;                      /* max |lambda_f| used by the step */
} pcvof_stats;

typedef struct pcvof_handle pcvof_handle;

/* Bytes of device workspace a domain needs (0 on invalid arguments). */
size_t pcvof_workspace_bytes(const pcvof_grid* grid, const pcvof_params* params);

/* Binds a domain to a caller-owned device workspace (256-byte aligned, at least
   pcvof_workspace_bytes) and a HIP stream (NULL = the null stream). */
int pcvof_create(const pcvof_grid* grid, const pcvof_params* params, void* d_workspace,
                 size_t workspace_bytes, void* hip_stream, pcvof_handle** out);
int pcvof_destroy(pcvof_handle* h);

/* Field input. set_vof checks 0 <= c <= 1 and finiteness (PCVOF_ERR_BOUNDS /
   PCVOF_ERR_NONFINITE, synchronising). set_energy sets e directly; set_temperature
   sets e = C_p(c) T and needs c first. set_velocity copies the three MAC face arrays
   (w ignored in 2D), checks finiteness and periodic face equality, and records
   max |u_f| for the CFL check (synchronising). set_mass_flux sets m'' per cell
   (mass per area and time, positive = evaporation); NULL switches step 2 off. */
int pcvof_set_vof(pcvof_handle* h, const double* c, int mem);
int pcvof_set_energy(pcvof_handle* h, const double* e, int mem);
int pcvof_set_temperature(pcvof_handle* h, const double* T, int mem);
int pcvof_set_velocity(pcvof_handle* h, const double* u, const double* v, const double* w,
                       int mem);
int pcvof_set_mass_flux(pcvof_handle* h, const double* mdot, int mem);

/* Mass-transfer rate from the PLIC reconstruction (section 3.2; eqs. cell_d,
   dint_trans, grad_n_T, normTgrad, mdot_calc), computed from the current fractions and
   temperatures T = e / C_p(c), with T_Gamma = params.T_gamma:
   * every mixed cell's plane gives a unit normal n = m / |m|_2 (liquid towards gas)
     and a distance d = alpha / |m|_2 from the cell's origin (its corner nearest the
     domain origin);
   * every pure cell within two cells of a mixed cell (first and second neighbours,
     5x5(x5) block) takes the plane of the neighbouring mixed cell whose normal is most
     collinear with the translation dx from that cell's origin to the pure cell's
     centre, xi = |n . dx| (first in z, y, x scan order on ties within 1e-12), its
     distance |d - n . dx| h, and the gradient into its phase (T - T_Gamma) / distance
     (none when the distance is below 1e-6 h);
   * every mixed cell averages those gradients over the pure cells of its 5x5(x5)
     block, per phase, with weights xi / |dx|^2 relative to its own plane, and
     m'' = (k_g G_g + k_l G_l) / h_fg (0 for a phase without such cells).
   Positions beyond an outflow boundary are not part of the blocks; periodic axes wrap.
   The result becomes the domain's mass flux, as after pcvof_set_mass_flux (step 2 on;
   0 outside mixed cells). mdot_out (optional) receives m'' per cell, dist_out
   (optional) the distance of every pure cell that has one and NaN elsewhere, both in
   the cell layout, in host (mem = 0) or device (mem = 1) memory. k_l, k_g >= 0,
   h_fg != 0 (PCVOF_ERR_ARG otherwise); needs the fractions and energies
   (PCVOF_ERR_STATE); not inside a step.
   In this version the call validates its arguments and then returns PCVOF_ERR_STATE:
   its GPU kernels are switched off (their first run ended in a memory fault whose
   cause is not found yet). */
int pcvof_compute_mass_flux(pcvof_handle* h, double k_l, double k_g, double h_fg, double* mdot_out,
                            double* dist_out, int mem);

/* Liquid-velocity extension (section 3.3.1, eq. press_inv and the correction after
   it). The stored face velocity u is taken as the one-fluid velocity, whose
   divergence carries the phase-change source m'' (1/rho_g - 1/rho_l) delta_Gamma; the
   call replaces it by the liquid velocity u_l = u + u~, which is divergence-free
   where u carried that source:
   * sub-domain: the mixed cells (eps < c < 1 - eps) and the gas cells that are first
     or second face neighbours of them through gas (shortest path of face steps);
     faces to liquid cells are walls (no correction), the faces to the third gas
     neighbours and faces on outflow boundaries hold a fixed pressure;
   * on it, sum over non-wall faces of (phi_j - phi_i) / rho_f = S a_i with
     S = m'' (1/rho_g - 1/rho_l), a_i the area of the cell's PLIC plane (cell units,
     the step's normal method and alpha from c), rho_f the mean of the two cells'
     rho(c) = rho_l c + rho_g (1 - c) (a ghost beyond an outflow boundary copies its
     cell), phi = 0 on the fixed-pressure side (phi = dt p~ / h: dt and h cancel);
   * u~ = -(phi_R - phi_L) / rho_f on the faces of the sub-domain, zero elsewhere.
   The system is solved by conjugate gradients (diagonal preconditioner, deterministic
   reductions) until |r|_2 <= rel_tol |b|_2 (0 < rel_tol < 1), at most max_iter
   iterations (>= 1). Needs the fractions, the velocity and the mass flux
   (PCVOF_ERR_STATE otherwise); rho_g > 0. d_workspace: device memory of at least
   pcvof_extension_workspace_bytes(h) bytes, 256-byte aligned, owned by the caller, only
   used during the call (PCVOF_ERR_WORKSPACE if smaller or misaligned). du, dv, dw (optional, dw ignored in 2D)
   receive u~ per face in the velocity layouts, in host (mem = 0) or device (mem = 1)
   memory. info (optional) receives the number of unknowns, the iterations and the
   final relative residual. When the iterations do not converge (a part of the
   sub-domain with a source but without a fixed-pressure face has no solution), the
   call returns PCVOF_ERR_STATE and leaves the velocity unchanged. Not inside a step,
   not on a batch domain, at most 2^31 - 1 cells. */
typedef struct {
    long unknowns;
    int iterations;
    double rel_residual;
} pcvof_ext_info;
size_t pcvof_extension_workspace_bytes(pcvof_handle* h);
int pcvof_extend_velocity(pcvof_handle* h, double rho_g, double rel_tol, int max_iter, void* d_workspace,
                          size_t workspace_bytes, double* du, double* dv, double* dw, int mem,
                          pcvof_ext_info* info);

/* Implicit energy diffusion with the interface temperature imposed (section 3.4.2,
   eqs. T_diff_disc and mod_branchesT), one backward-Euler step of length dt on the
   current state:
   * a node is liquid when c >= 1/2, else gas, and diffuses with its phase's constant
     conductivity (k_l, k_g) and volumetric heat capacity (params cp_l, cp_g);
   * towards a face neighbour of the same phase the gradient is the difference over h;
     towards one of the other phase the interface is a boundary at distance theta where
     T = T_Gamma (params T_gamma): the gradient is (T_Gamma - T_i) / theta and the
     node's control width along that axis becomes (h + theta) / 2 ((theta_L + theta_R) / 2
     with the interface on both sides);
   * theta is the height of the six-cell column centred on the face when that column is
     bounded by pure cells of the two phases, else the point where the linear
     interpolation of the node phase's indicator between the two nodes crosses 1/2,
     capped to [1e-3 h, h];
   * outflow boundaries are adiabatic, periodic axes wrap;
   * the temperature before the step is e / C_p(c) (one-fluid C_p), the energy after it
     C_p(c) T^{n+1}.
   The non-symmetric system is solved by BiCGSTAB preconditioned with one multigrid
   V(0,2) cycle (2 x 2 x 2 aggregates, Galerkin coarse operators, damped Jacobi steps;
   deterministic reductions) from T*, until |r|_2 <= rel_tol |b|_2 (0 < rel_tol < 1), at
   most max_iter iterations (>= 1); without convergence PCVOF_ERR_STATE and the energy
   is unchanged. dt > 0, k_l, k_g >= 0 (PCVOF_ERR_ARG otherwise); needs the fractions
   and energies (PCVOF_ERR_STATE); not inside a step, not on a batch domain.
   d_workspace: device memory of at least pcvof_diffusion_workspace_bytes(h) bytes,
   256-byte aligned, owned by the caller, used during the call only (PCVOF_ERR_WORKSPACE
   if smaller or misaligned).
   T_out (optional) receives T^{n+1} in the cell layout, in host (mem = 0) or device
   (mem = 1) memory; info (optional) the iterations and final relative residual
   (unknowns = cells). */
size_t pcvof_diffusion_workspace_bytes(pcvof_handle* h);
int pcvof_diffuse(pcvof_handle* h, double dt, double k_l, double k_g, double rel_tol, int max_iter, void* d_workspace,
                  size_t workspace_bytes, double* T_out, int mem, pcvof_ext_info* info);

/* pcvof_diffuse for callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid allocation): the same operation,
   arguments and results as pcvof_diffuse, without the workspace arguments. It allocates
   nothing: its scratch is one device array of 256 MiB per GPU, part of the library and
   held until the process ends, enough for domains of about 1.7 million cells
   (pcvof_diffusion_workspace_bytes(h) <= 256 MiB); larger domains get
   PCVOF_ERR_WORKSPACE without anything launched. Every call on a GPU shares that GPU's
   array: calls that overlap on one GPU (several host threads, or streams that run at
   the same time) race and give undefined results. The array keeps the last call's
   contents; the call writes every location it reads. */
int pcvof_diffuse_static(pcvof_handle* h, double dt, double k_l, double k_g, double rel_tol, int max_iter,
                         double* T_out, int mem, pcvof_ext_info* info);

/* One time step with face CFL numbers lambda_f = u_f * (u_scale * dt) / h:
   prologue, ndim sweeps in the axis order rotated by the step counter (x,y,z /
   y,z,x / z,x,y), step 2 when a mass flux is set, checksums. Increments the step
   counter. stats may be NULL (no synchronisation); otherwise the call waits for the
   step and fills it. */
int pcvof_advect_step(pcvof_handle* h, double dt, double u_scale, pcvof_stats* stats);

/* The stages of pcvof_advect_step, for staged use and testing. begin_step freezes
   c_c = [c >= 1/2] and e_c = C_p(c_c) T for the sweeps of a step; sweep runs one
   direction sweep (axis 0..ndim-1); phase_change runs step 2 with time step dt;
   end_step reduces the checksums (stats may be NULL) and increments the counter. */
int pcvof_begin_step(pcvof_handle* h);
int pcvof_sweep(pcvof_handle* h, int axis, double dt, double u_scale);
int pcvof_phase_change(pcvof_handle* h, double dt);
int pcvof_end_step(pcvof_handle* h, pcvof_stats* stats);

/* nsteps consecutive pcvof_advect_step calls from one host call, with the velocity
   scale of step k in u_scale[k] (host array of nsteps values; NULL = 1 for all).
   last (nullable) receives the checksums of the final step. */
int pcvof_advect_steps(pcvof_handle* h, int nsteps, double dt, const double* u_scale,
                       pcvof_stats* last);

/* Kernel timing. pcvof_set_profiling takes a mask of kernel classes (bit k = class k,
   PCVOF_PROF_ALL = every class, 0 = off). While a class is selected, each of its
   launches is bracketed by two HIP events recorded on the library's stream (each
   event adds a few microseconds of device time to the stream, so select only the
   classes to be measured). pcvof_get_profile waits for the stream and returns the
   accumulated device time per class since profiling was last enabled. A non-zero
   mask resets the accumulators; 0 keeps them readable. Bits outside
   PCVOF_PROF_ALL give PCVOF_ERR_ARG. */
enum {
    PCVOF_PROF_SWEEP_X = 0,   /* sweep kernels, per axis (each includes the geometry of */
    PCVOF_PROF_SWEEP_Y = 1,   /* the mixed donors of its tiles) */
    PCVOF_PROF_SWEEP_Z = 2,
    PCVOF_PROF_PHASE = 3,     /* step 2 (both of its kernels) */
    PCVOF_PROF_CHECKSUM = 4,  /* column sums of the checksums */
    PCVOF_PROF_CLASSES = 5,
    PCVOF_PROF_ALL = (1 << 5) - 1
};
typedef struct {
    double ms[PCVOF_PROF_CLASSES];     /* total device time, milliseconds */
    long launches[PCVOF_PROF_CLASSES];
} pcvof_profile;
int pcvof_set_profiling(pcvof_handle* h, int classes);
int pcvof_get_profile(pcvof_handle* h, pcvof_profile* out);

/* Field output (same layout as the input). */
int pcvof_get_vof(pcvof_handle* h, double* out, int mem);
int pcvof_get_energy(pcvof_handle* h, double* out, int mem);
int pcvof_get_temperature(pcvof_handle* h, double* out, int mem);

/* Step counter (sets the sweep order); part of the state for checkpoint / resume. */
int pcvof_get_step(pcvof_handle* h, long* step);
int pcvof_set_step(pcvof_handle* h, long step);

const char* pcvof_last_error(void);

/* Batches of independent domains (the same method on each domain, section 3.3 and
   3.4.1). A batch owns nd domain handles ("views") carved out of one caller-owned
   workspace of pcvof_batch_workspace_bytes bytes. Every domain of a batch has the same
   ndim and precision; sizes, boundary conditions and the other parameters may differ.
   Fields are set and read through the views (pcvof_batch_domain) with the usual
   set_/get_ calls; views are destroyed with the batch and must not be stepped on their
   own between batched steps (PCVOF_ERR_STATE).
   pcvof_batch_advect_step advances every domain by one step (its own dt[i], velocity
   scale 1) with one fused launch per direction sweep over the tiles of all domains
   (one block per tile; every tile computes what the single-domain sweep's block
   computes, so results are bitwise those of pcvof_advect_step), step 2 for
   domains with a mass flux, and one checksum launch. Argument tables are cached per
   recurring step state. With use_graph != 0 (and no mass flux in any domain) the
   launches of a step are captured once per cached state into a HIP graph and replayed
   afterwards. stats (nullable) receives nd checksum records and synchronises.
   pcvof_batch_set_tiles sets the rows per wavefront of the x sweep (chunk[0]: 0 = each
   domain's single-domain rule, else 1, 2, 4 or 8) and the column chunk of the y / z sweeps
   (chunk[1], chunk[2]: 0 = each domain's single-domain rule, else a power of two in
   [8, 64]); the fields do not depend on these choices;
   pcvof_batch_autotune times the choices on the current state (reps timed launches per
   choice; the state is not advanced) and keeps the fastest per axis. */
typedef struct pcvof_batch pcvof_batch;
size_t pcvof_batch_workspace_bytes(int nd, const pcvof_grid* grids, const pcvof_params* params);
int pcvof_batch_create(int nd, const pcvof_grid* grids, const pcvof_params* params, void* d_workspace,
                       size_t workspace_bytes, void* hip_stream, pcvof_batch** out);
int pcvof_batch_destroy(pcvof_batch* b);
int pcvof_batch_domain(pcvof_batch* b, int i, pcvof_handle** view);
int pcvof_batch_advect_step(pcvof_batch* b, const double* dt, int use_graph, pcvof_stats* stats);
int pcvof_batch_get_step(pcvof_batch* b, long* step);
int pcvof_batch_set_tiles(pcvof_batch* b, const int* chunk);
int pcvof_batch_get_tiles(pcvof_batch* b, int* chunk, int* ntiles);
int pcvof_batch_autotune(pcvof_batch* b, const double* dt, int reps, int* chosen_chunk);

/* Batched cell geometry on device arrays of n entries (testing and reuse), enqueued
   on the given stream. m holds 3 doubles per entry; the volume functions accept any
   non-zero m, the plane constant is returned in the same scaling as m.
   volume: |{x in [0,1]^3 : m.x <= alpha}|; alpha: inverse of volume for c in (0,1);
   slab: liquid volume (cell units) of the donor region crossing a face in a sweep
   along axis with face CFL number lam (x_axis in [1-lam,1] for lam > 0, [0,|lam|]
   for lam < 0); normal: normal from 27 fractions c27[(dz+1)*9+(dy+1)*3+(dx+1)];
   weno5: face value between v[2] and v[3] from 5 values per entry. */
int pcvof_geom_volume(int n, const double* m, const double* alpha, double* out, void* stream);
int pcvof_geom_alpha(int n, const double* m, const double* c, double* out, void* stream);
int pcvof_geom_slab(int n, const double* m, const double* alpha, const int* axis,
                    const double* lam, double* out, void* stream);
int pcvof_geom_normal(int n, const double* c27, int method, double* m, void* stream);
int pcvof_geom_weno5(int n, const double* v, double eps, double* out, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* PCVOF_H */
