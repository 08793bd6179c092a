/*
 * PCVOF ORACLE -- test infrastructure, not part of the product.
 *
 * A plain, slow, double-precision CPU reference of one time step of the
 * geometric PLIC-VOF advection with conservative thermal-energy advection
 * (paper section 3.3, "Geometric VOF advection for phase change", and section
 * 3.4.1, "Calculating the energy advection term"). Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg may load it. It shares no
 * code with the HIP library.
 *
 * Conventions (paper section 3.2, eq. plane_m): each cell has local coordinates
 * x in [0,1]^3 with the origin at the cell corner nearest the domain origin; the
 * interface is the plane m.x = alpha with |m1|+|m2|+|m3| = 1; the liquid is the
 * side m.x <= alpha, i.e. m points from the liquid into the gas (section 2,
 * interface normal n_Gamma).
 */
#ifndef PCVOF_ORACLE_H
#define PCVOF_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int ndim;          /* 2 or 3; ndim == 2 requires nz == 1 */
    int nx, ny, nz;    /* cells per axis */
    double h;          /* cubic cell edge */
    int bc[3];         /* per axis: 0 periodic, 1 outflow (zero-gradient ghost) */
} or_grid;

typedef struct {
    double cp_l, cp_g;   /* volumetric heat capacities rho*c_p of liquid and gas */
    double rho_l;        /* liquid density (phase-change shift) */
    double T_gamma;      /* interface (saturation) temperature */
    double eps_mixed;    /* mixed-cell threshold eps < c < 1-eps (section 3.1: 1e-12) */
    double weno_eps;     /* WENO5 epsilon of the nonlinear weights */
    int normal;          /* 0 Youngs, 1 mixed Youngs-centred (MYC), 2 centred columns only */
    int energy_flux;     /* 0 conservative fluxes (section 3.4.1, eq. disc_et_adv); 1 the
                            non-conservative approximation of eq. disc_et_adv_noncons */
    int split;           /* 0 Weymouth-Yue Eulerian-implicit sweeps with the frozen c_c, e_c
                            dilatation terms; 1 Lagrangian-explicit sweeps of Li (CIAM, the
                            other scheme section 3.3 names), dilatation with the current c, e */
} or_params;

typedef struct {
    double vol, energy;              /* h^d * sum c, h^d * sum e after the step */
    double vol_clip, energy_clip;    /* sweep clipping of c into [0,1] (energy keeps T) */
    double vol_phase, energy_phase;  /* step-2 change of c and of e (latent correction) */
    double vol_bnd_out, energy_bnd_out; /* net outflow through outflow boundaries */
    double vol_src, energy_src;      /* split dilatation terms cc*dlam, ec*dlam (Lagrangian-
                                        explicit sweeps: c*dlam, e*dlam) */
    double max_cfl;                  /* max |u_f| * u_scale * dt / h over the faces used */
} or_stats;

/* ---- cell geometry ---- */
double or_volume(const double m[3], double alpha);      /* |{x in [0,1]^3 : m.x <= alpha}| */
double or_area(const double m[3], double alpha);        /* area of {m.x = alpha} inside the cube */
double or_alpha(const double m[3], double c);           /* alpha with or_volume(m, alpha) = c */
void   or_normal(const double c27[27], int method, double m[3]);
double or_slab(const double m[3], double alpha, int axis, double lam);
double or_weno5(const double v[5], double eps);

/* Batched helpers for the test suite. */
void or_volume_n(int n, const double* m, const double* alpha, double* out);
void or_area_n(int n, const double* m, const double* alpha, double* out);
void or_alpha_n(int n, const double* m, const double* c, double* out);
void or_slab_n(int n, const double* m, const double* alpha, const int* axis,
               const double* lam, double* out);

/* ---- one time step, and its stages ---- */
/* Frozen split fields of the step: cc = [c >= 1/2], ec = Cp(cc) * T. */
void or_prologue(const or_grid* g, const or_params* p, const double* c, const double* e,
                 double* cc, double* ec);
/* One direction sweep with face CFL numbers lam = vel * kfac; writes c_out, e_out and
   accumulates the sweep's clip, boundary and source terms (cell units) into acc[0..5]:
   vol_clip, energy_clip, vol_bnd_out, energy_bnd_out, vol_src, energy_src. */
int or_sweep(const or_grid* g, const or_params* p, int axis, const double* c, const double* e,
             const double* cc, const double* ec, const double* vel, double kfac,
             double* c_out, double* e_out, double* acc);
/* Step 2 (interface shift for the phase-change source) and the latent correction;
   acc[0..1] += vol_phase, energy_phase (cell units). */
int or_phase_change(const or_grid* g, const or_params* p, const double* c, const double* e,
                    const double* mdot, double dt, double* c_out, double* e_out, double* acc);
/* Full step: prologue, ndim sweeps in the order rotated by step_index, step 2 when mdot
   is not NULL. u, v, w are MAC face velocities (w ignored when ndim == 2). */
int or_step(const or_grid* g, const or_params* p, const double* c, const double* e,
            const double* u, const double* v, const double* w, const double* mdot,
            double dt, double u_scale, long step_index, double* c_out, double* e_out,
            or_stats* st);

/* Mass-transfer rate from the PLIC reconstruction (section 3.2), from the fractions c
   and the cell temperatures T: for every pure cell within two cells (first and second
   neighbours) of a mixed cell, the distance |d_Gamma| (physical units) from its centre
   to the plane of the neighbouring mixed cell whose normal is most collinear with the
   translation to that centre, and its normal gradient (T - T_Gamma) / |d_Gamma|; for
   every mixed cell, m'' = (k_g G_g + k_l G_l) / h_fg from the collinearity- and
   distance-weighted averages G of those gradients over its 5x5(x5) block, per phase.
   mdot (every cell; 0 outside mixed cells) and dist (NULL or every cell; NaN where no
   distance is defined). Returns 0, -1 on bad arguments, -2 if out of memory. */
int or_mass_flux(const or_grid* g, const or_params* p, const double* c, const double* T,
                 double k_l, double k_g, double h_fg, double* mdot, double* dist);

#ifdef __cplusplus
}
#endif
#endif
