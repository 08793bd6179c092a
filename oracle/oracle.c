/*
 * PCVOF ORACLE -- test infrastructure, not part of the product.
 *
 * Plain FP64 CPU reference of one step of the paper's geometric VOF advection
 * with conservative thermal-energy advection. Every routine is the plain
 * definition of what it computes, written for a reader to check against the
 * paper; nothing is blocked, fused or reordered for speed. Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load this
 * library. It shares no code with the HIP library.
 *
 * Parity status of each function (what pins it) is listed in the test suite;
 * the mixed Youngs-centred selection rule (or_normal, method 1) follows the
 * published idea of Aulisa et al. in a reading stated below, and its agreement
 * with any other published code is "parity unpinned".
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* Compensated (Neumaier) summation for the step's checksums.                 */
/* ------------------------------------------------------------------------- */
typedef struct { double s, c; } ksum;

static void kadd(ksum* k, double x) {
    double t = k->s + x;
    if (fabs(k->s) >= fabs(x)) k->c += (k->s - t) + x;
    else k->c += (x - t) + k->s;
    k->s = t;
}
static double kval(const ksum* k) { return k->s + k->c; }

/* ------------------------------------------------------------------------- */
/* Cell geometry: the unit cube cut by the half-space m.x <= alpha.           */
/* Section 3.2 (eq. plane_m) defines the plane; section 3.3.2 uses c = f(alpha,m). */
/* ------------------------------------------------------------------------- */

/* Area of {(u,v) in [0,1]^2 : a*u + b*v <= beta}: the unit square is clipped by
   the half-plane one edge at a time (Sutherland-Hodgman) and the area of the
   resulting polygon is taken with the shoelace formula. */
static double clipped_square_area(double a, double b, double beta) {
    static const double sq[4][2] = {{0.0, 0.0}, {1.0, 0.0}, {1.0, 1.0}, {0.0, 1.0}};
    double poly[8][2];
    int n = 0;
    for (int k = 0; k < 4; ++k) {
        const double* P = sq[k];
        const double* Q = sq[(k + 1) % 4];
        double fP = a * P[0] + b * P[1] - beta;
        double fQ = a * Q[0] + b * Q[1] - beta;
        if (fP <= 0.0) {
            poly[n][0] = P[0];
            poly[n][1] = P[1];
            ++n;
        }
        if ((fP <= 0.0) != (fQ <= 0.0)) {
            double t = fP / (fP - fQ);
            poly[n][0] = P[0] + t * (Q[0] - P[0]);
            poly[n][1] = P[1] + t * (Q[1] - P[1]);
            ++n;
        }
    }
    double s = 0.0;
    for (int k = 0; k < n; ++k) {
        int l = (k + 1) % n;
        s += poly[k][0] * poly[l][1] - poly[l][0] * poly[k][1];
    }
    return 0.5 * fabs(s);
}

/* Reflect the cube so that every normal component is non-negative: x_i -> 1-x_i
   for m_i < 0 turns m.x <= alpha into |m|.x' <= alpha + sum_{m_i<0} |m_i|. */
static double reflect(const double m_in[3], double alpha, double m[3]) {
    double a = alpha;
    for (int i = 0; i < 3; ++i) {
        if (m_in[i] < 0.0) {
            m[i] = -m_in[i];
            a += m[i];
        } else {
            m[i] = m_in[i];
        }
    }
    return a;
}

/* Clipped areas of the six cube faces: A0[i] on the face x_i = 0, A1[i] on x_i = 1
   (reflected frame, m >= 0). */
static void face_areas(const double m[3], double a, double A0[3], double A1[3]) {
    for (int i = 0; i < 3; ++i) {
        int j = (i + 1) % 3, k = (i + 2) % 3;
        A0[i] = clipped_square_area(m[j], m[k], a);
        A1[i] = clipped_square_area(m[j], m[k], a - m[i]);
    }
}

/* Volume of {x in [0,1]^3 : m.x <= alpha} for any non-zero m, by the divergence
   theorem applied to the clipped polyhedron with the reference point at the
   reflected origin: V = (1/3) * sum over boundary faces of (x.n) * area. Faces on
   x_i = 0 contribute nothing, faces on x_i = 1 contribute their clipped area, and
   the cut face (on the plane, x.n = a/|m|) has the area that closes the vector
   area of the surface: A_cut * n = sum_i (A0_i - A1_i) e_i. */
double or_volume(const double m_in[3], double alpha) {
    double m[3];
    double a = reflect(m_in, alpha, m);
    double S = m[0] + m[1] + m[2];
    if (a <= 0.0) return 0.0;
    if (a >= S) return 1.0;
    double A0[3], A1[3];
    face_areas(m, a, A0, A1);
    double nn = m[0] * m[0] + m[1] * m[1] + m[2] * m[2];
    double far = A1[0] + A1[1] + A1[2];
    double cut = m[0] * (A0[0] - A1[0]) + m[1] * (A0[1] - A1[1]) + m[2] * (A0[2] - A1[2]);
    return (far + (a / nn) * cut) / 3.0;
}

/* Area of the interface polygon {m.x = alpha} inside the unit cube, from the same
   vector-area closure: A_cut = sum_i m_i (A0_i - A1_i) / |m|_2. */
double or_area(const double m_in[3], double alpha) {
    double m[3];
    double a = reflect(m_in, alpha, m);
    double S = m[0] + m[1] + m[2];
    if (a <= 0.0 || a >= S) return 0.0;
    double A0[3], A1[3];
    face_areas(m, a, A0, A1);
    double cut = m[0] * (A0[0] - A1[0]) + m[1] * (A0[1] - A1[1]) + m[2] * (A0[2] - A1[2]);
    return cut / sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
}

/* Reflected plane constant a in [0, S] with V(a) = v (reflected frame, m >= 0):
   bisection on the monotone volume function until the bracket cannot shrink
   further. */
static double bisect_alpha(const double m[3], double v) {
    double lo = 0.0, hi = m[0] + m[1] + m[2];
    double mid = 0.5 * (lo + hi);
    for (int it = 0; it < 200; ++it) {
        mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (or_volume(m, mid) < v) lo = mid;
        else hi = mid;
    }
    return mid;
}

/* Plane constant for a given volume fraction (section 3.2: "alpha is obtained by
   geometrical volume calculations"; the inverse of c = f(alpha, m) of section 3.3.2).
   The cube is centrally symmetric, so V(a) + V(S - a) = 1 in the reflected frame:
   above one half the complementary volume 1 - c (exact in floating point) is
   inverted instead, where the volume function is small and evaluated to full
   relative precision, and the plane is reflected, a = S - a(1 - c). Inverting V = c
   directly near c = 1 would resolve a only to the absolute rounding of V (about
   1e-16) divided by its slope, the vanishing area of a corner plane. */
double or_alpha(const double m_in[3], double c) {
    double m[3];
    double shift = reflect(m_in, 0.0, m); /* alpha_reflected = alpha + shift */
    double S = m[0] + m[1] + m[2];
    if (c <= 0.0) return 0.0 - shift;
    if (c >= 1.0) return S - shift;
    if (c > 0.5) return (S - bisect_alpha(m, 1.0 - c)) - shift;
    return bisect_alpha(m, c) - shift;
}

/* ------------------------------------------------------------------------- */
/* Interface normal from the 3x3x3 block of volume fractions around a cell.   */
/* c27[(dz+1)*9 + (dy+1)*3 + (dx+1)], offsets in {-1,0,1}.                    */
/* ------------------------------------------------------------------------- */
static double c27_at(const double* c27, int a, int oa, int t1, int o1, int t2, int o2) {
    int off[3] = {0, 0, 0};
    off[a] = oa;
    off[t1] = o1;
    off[t2] = o2;
    return c27[(off[2] + 1) * 9 + (off[1] + 1) * 3 + (off[0] + 1)];
}

static void transverse(int a, int* t1, int* t2) {
    *t1 = (a == 0) ? 1 : 0;
    *t2 = (a == 2) ? 1 : 2;
}

/* Youngs' gradient: for each axis, the (1,2,1) x (1,2,1)-weighted sum of the
   central differences over the 3x3 transverse block, summed with the second
   transverse offset outermost. */
static void youngs_gradient(const double* c27, double g[3]) {
    static const double w[3] = {1.0, 2.0, 1.0};
    for (int a = 0; a < 3; ++a) {
        int t1, t2;
        transverse(a, &t1, &t2);
        double acc = 0.0;
        for (int o2 = -1; o2 <= 1; ++o2)
            for (int o1 = -1; o1 <= 1; ++o1) {
                double d = c27_at(c27, a, 1, t1, o1, t2, o2) - c27_at(c27, a, -1, t1, o1, t2, o2);
                acc = acc + (w[o1 + 1] * w[o2 + 1]) * d;
            }
        g[a] = acc;
    }
}

/* Decisions of the normal estimator use a tie band: gradients of magnitude up to
   NORMAL_TIE count as zero and candidates within NORMAL_TIE count as equal (lowest
   axis first), so that round-off differences of the inputs cannot change which
   formula is used (symmetric configurations tie exactly). */
static const double NORMAL_TIE = 1e-12;

/* Centred-columns candidate for column axis d: the liquid heights of the 3-cell
   columns along d at the four transverse neighbours give the transverse slopes
   m_t = (H(t=-1) - H(t=+1)) / 2; the column component is +1 when the liquid lies
   towards -d (Youngs' gradient along d negative), -1 when it lies towards +d, and the
   candidate is invalid when that gradient is zero (within the tie band). Returns
   validity; comp holds the unnormalised components and *L their l1 norm. */
static int cc_candidate(const double* c27, const double g[3], int d, double comp[3], double* L) {
    int t1, t2;
    transverse(d, &t1, &t2);
    if (fabs(g[d]) <= NORMAL_TIE) return 0;
    double H[2][2];
    for (int s = 0; s < 2; ++s) {
        int o = s == 0 ? -1 : 1;
        H[0][s] = (c27_at(c27, d, -1, t1, o, t2, 0) + c27_at(c27, d, 0, t1, o, t2, 0)) +
                  c27_at(c27, d, 1, t1, o, t2, 0);
        H[1][s] = (c27_at(c27, d, -1, t1, 0, t2, o) + c27_at(c27, d, 0, t1, 0, t2, o)) +
                  c27_at(c27, d, 1, t1, 0, t2, o);
    }
    comp[d] = g[d] < 0.0 ? 1.0 : -1.0;
    comp[t1] = 0.5 * (H[0][0] - H[0][1]);
    comp[t2] = 0.5 * (H[1][0] - H[1][1]);
    *L = (fabs(comp[0]) + fabs(comp[1])) + fabs(comp[2]);
    return 1;
}

/* method 0: Youngs, m = -g / |g|_1 (a zero gradient gives m = (1,0,0)).
   method 1: mixed Youngs-centred (the normal named in section 3.2, after Aulisa et
   al.). Reading: among the valid centred-columns candidates take the one whose own
   (column-axis) component |m_d| = 1/L_d is largest, lowest axis on ties. Columns
   that fail to bracket the interface flatten that candidate, which shows as an own
   component larger than every component of Youngs' normal; in that case, or when no
   candidate is valid, Youngs' normal is used, otherwise the centred-columns one.
   Zero tests and comparisons use the tie band NORMAL_TIE.
   method 2: the best centred-columns candidate alone (Youngs when none is valid). */
void or_normal(const double c27[27], int method, double m[3]) {
    double g[3];
    youngs_gradient(c27, g);
    double LY = (fabs(g[0]) + fabs(g[1])) + fabs(g[2]);
    double my[3] = {1.0, 0.0, 0.0};
    int flat = LY <= NORMAL_TIE;
    if (!flat) {
        for (int i = 0; i < 3; ++i) my[i] = -g[i] / LY;
    }
    if (method == 0 || flat) {
        memcpy(m, my, sizeof my);
        return;
    }
    int best = -1;
    double best_own = 0.0, best_comp[3] = {0, 0, 0}, best_L = 1.0;
    for (int d = 0; d < 3; ++d) {
        double comp[3], L;
        if (!cc_candidate(c27, g, d, comp, &L)) continue;
        double own = 1.0 / L;
        if (best < 0 || own > best_own + NORMAL_TIE) {
            best = d;
            best_own = own;
            best_L = L;
            memcpy(best_comp, comp, sizeof comp);
        }
    }
    if (best < 0) {
        memcpy(m, my, sizeof my);
        return;
    }
    if (method == 1) {
        double ymax = fabs(my[0]);
        if (fabs(my[1]) > ymax) ymax = fabs(my[1]);
        if (fabs(my[2]) > ymax) ymax = fabs(my[2]);
        if (best_own > ymax + NORMAL_TIE) {
            memcpy(m, my, sizeof my);
            return;
        }
    }
    for (int i = 0; i < 3; ++i) m[i] = best_comp[i] / best_L;
}

/* Liquid volume, in units of the cell volume, of the region of the donor cell that
   crosses the face during the step (the upwind face-flux region of the direction-
   split geometric schemes cited in section 3.3, reused for the heat capacity in
   section 3.4.1). For lam > 0 the donor is on the left and the region is
   x_axis in [1-lam, 1]; for lam < 0 the donor is on the right and the region is
   x_axis in [0, |lam|]. The region is mapped affinely onto the unit cube. */
double or_slab(const double m[3], double alpha, int axis, double lam) {
    double L = fabs(lam);
    if (L == 0.0) return 0.0;
    double mm[3] = {m[0], m[1], m[2]};
    double a = alpha;
    if (lam > 0.0) a = alpha - m[axis] * (1.0 - L);
    mm[axis] = m[axis] * L;
    return L * or_volume(mm, a);
}

/* Fifth-order WENO face value (Jiang and Shu; the scheme cited in section 3.4.1)
   at the face between v[2] and v[3] from the left-biased stencil v[0..4]. */
double or_weno5(const double v[5], double eps) {
    double q0 = (2.0 * v[0] - 7.0 * v[1] + 11.0 * v[2]) / 6.0;
    double q1 = (-v[1] + 5.0 * v[2] + 2.0 * v[3]) / 6.0;
    double q2 = (2.0 * v[2] + 5.0 * v[3] - v[4]) / 6.0;
    double s0a = v[0] - 2.0 * v[1] + v[2], s0b = v[0] - 4.0 * v[1] + 3.0 * v[2];
    double s1a = v[1] - 2.0 * v[2] + v[3], s1b = v[1] - v[3];
    double s2a = v[2] - 2.0 * v[3] + v[4], s2b = 3.0 * v[2] - 4.0 * v[3] + v[4];
    double b0 = 13.0 / 12.0 * s0a * s0a + 0.25 * s0b * s0b;
    double b1 = 13.0 / 12.0 * s1a * s1a + 0.25 * s1b * s1b;
    double b2 = 13.0 / 12.0 * s2a * s2a + 0.25 * s2b * s2b;
    double a0 = 0.1 / ((eps + b0) * (eps + b0));
    double a1 = 0.6 / ((eps + b1) * (eps + b1));
    double a2 = 0.3 / ((eps + b2) * (eps + b2));
    return (a0 * q0 + a1 * q1 + a2 * q2) / (a0 + a1 + a2);
}

void or_volume_n(int n, const double* m, const double* alpha, double* out) {
    for (int i = 0; i < n; ++i) out[i] = or_volume(m + 3 * i, alpha[i]);
}
void or_area_n(int n, const double* m, const double* alpha, double* out) {
    for (int i = 0; i < n; ++i) out[i] = or_area(m + 3 * i, alpha[i]);
}
void or_alpha_n(int n, const double* m, const double* c, double* out) {
    for (int i = 0; i < n; ++i) out[i] = or_alpha(m + 3 * i, c[i]);
}
void or_slab_n(int n, const double* m, const double* alpha, const int* axis, const double* lam,
               double* out) {
    for (int i = 0; i < n; ++i) out[i] = or_slab(m + 3 * i, alpha[i], axis[i], lam[i]);
}

/* ------------------------------------------------------------------------- */
/* Grid access with ghost cells.                                              */
/* ------------------------------------------------------------------------- */
static int ncell(const or_grid* g, int a) { return a == 0 ? g->nx : (a == 1 ? g->ny : g->nz); }

/* Ghost rule per axis: periodic wrap, or outflow = copy of the nearest interior
   cell. The z axis of a 2D grid (one plane) wraps onto that plane. */
static int map_index(const or_grid* g, int a, int i) {
    int n = ncell(g, a);
    if (a == 2 && g->ndim == 2) return 0;
    if (g->bc[a] == 0) return ((i % n) + n) % n;
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

static long cell_id(const or_grid* g, int x, int y, int z) {
    int i = map_index(g, 0, x), j = map_index(g, 1, y), k = map_index(g, 2, z);
    return ((long)k * g->ny + j) * g->nx + i;
}

/* Face velocity index along axis a at face position f (between cells f-1 and f)
   with transverse cell coordinates. MAC layouts: u [nz][ny][nx+1],
   v [nz][ny+1][nx], w [nz+1][ny][nx]. */
static long face_id(const or_grid* g, int a, int x, int y, int z) {
    if (a == 0) return ((long)z * g->ny + y) * (g->nx + 1) + x;
    if (a == 1) return ((long)z * (g->ny + 1) + y) * g->nx + x;
    return ((long)z * g->ny + y) * g->nx + x;
}

static double cp_of(const or_params* p, double c) { return p->cp_l * c + p->cp_g * (1.0 - c); }

static void gather27(const or_grid* g, const double* c, int x, int y, int z, double* c27) {
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx)
                c27[(dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)] = c[cell_id(g, x + dx, y + dy, z + dz)];
}

static int is_mixed(const or_params* p, double c) { return c > p->eps_mixed && c < 1.0 - p->eps_mixed; }

static int check_grid(const or_grid* g) {
    if (!g || (g->ndim != 2 && g->ndim != 3)) return -1;
    if (g->nx < 1 || g->ny < 1 || g->nz < 1) return -1;
    if (g->ndim == 2 && g->nz != 1) return -1;
    if (!(g->h > 0.0)) return -1;
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Step stages.                                                               */
/* ------------------------------------------------------------------------- */

/* Before the sweeps (section 3.4.1): e_t = C_p T with C_p = C_pl c + C_pg (1-c), so
   T^n = e / C_p(c^n). The split dilatation terms of the conservative direction-split
   scheme use c_c = [c^n >= 1/2] frozen over the step; the energy carries the
   matching e_c = C_p(c_c) T^n, so that a uniform temperature stays uniform. */
void or_prologue(const or_grid* g, const or_params* p, const double* c, const double* e,
                 double* cc, double* ec) {
    long n = (long)g->nx * g->ny * g->nz;
    for (long i = 0; i < n; ++i) {
        double T = e[i] / cp_of(p, c[i]);
        double flag = c[i] >= 0.5 ? 1.0 : 0.0;
        cc[i] = flag;
        ec[i] = (flag == 1.0 ? p->cp_l : p->cp_g) * T;
    }
}

/* CFL number of the face at position f along axis a (between cells f-1 and f) of the
   face row through pos. Faces beyond the domain: periodic axes wrap (face n is face
   0); outflow axes repeat the boundary face, so a ghost cell's two faces carry the
   same velocity. */
static double face_lam(const or_grid* g, int a, const double* vel, double kfac, const int* pos, int f) {
    int n = ncell(g, a);
    if (g->bc[a] == 0) {
        while (f < 0) f += n;
        while (f > n) f -= n;
    } else {
        f = f < 0 ? 0 : (f > n ? n : f);
    }
    int q[3] = {pos[0], pos[1], pos[2]};
    q[a] = f;
    return vel[face_id(g, a, q[0], q[1], q[2])] * kfac;
}

/* Face flux of one sweep: the liquid volume F through the face (section 3.3) and the
   energy flux E = sgn(lam) [C_pl F + C_pg (|lam| - F)] T_f, i.e. the fluxed heat
   capacity weighted by the fluxed liquid and gas volumes times the WENO5 face
   temperature (section 3.4.1, eq. disc_et_adv). With the non-conservative energy flux
   (eq. disc_et_adv_noncons) the face carries only lam T_f; each cell multiplies it by
   its own heat capacity in or_sweep. Position (x,y,z) is the cell right of the face.

   Weymouth-Yue sweeps: F is the liquid in the donor's slab of width |lam| next to the
   face. Lagrangian-explicit sweeps (Li): every point of the donor moves with the
   velocity interpolated linearly between its two faces, so the donor is stretched by
   s = 1 + (lam_R - lam_L) and the part that crosses the face is the slab of width
   |lam| / s next to it, whose liquid volume is multiplied by s. A pure donor gives
   |lam| c_D in both schemes. */
static void face_flux(const or_grid* g, const or_params* p, int a, const double* c,
                      const double* e, const double* vel, double kfac, double lam, int x,
                      int y, int z, double* Phi, double* E) {
    *Phi = 0.0;
    *E = 0.0;
    if (lam == 0.0) return;
    int pos[3] = {x, y, z};
    int dpos[3] = {x, y, z};
    if (lam > 0.0) dpos[a] -= 1;
    long d = cell_id(g, dpos[0], dpos[1], dpos[2]);
    double cd = c[d], L = fabs(lam), F;
    if (is_mixed(p, cd)) {
        double c27[27], m[3];
        gather27(g, c, dpos[0], dpos[1], dpos[2], c27);
        or_normal(c27, p->normal, m);
        double alpha = or_alpha(m, cd);
        if (p->split == 1) {
            /* the donor's faces are dpos[a] and dpos[a] + 1 */
            double lamL = face_lam(g, a, vel, kfac, pos, dpos[a]);
            double lamR = face_lam(g, a, vel, kfac, pos, dpos[a] + 1);
            double s = 1.0 + (lamR - lamL);
            F = s * or_slab(m, alpha, a, lam / s);
        } else {
            F = or_slab(m, alpha, a, lam);
        }
    } else {
        F = L * cd;
    }
    double T[5];
    for (int s = 0; s < 5; ++s) {
        int q[3] = {pos[0], pos[1], pos[2]};
        /* lam > 0: cells f-3 .. f+1; lam < 0: cells f+2 .. f-2 (mirrored) */
        q[a] += lam > 0.0 ? (s - 3) : (2 - s);
        long id = cell_id(g, q[0], q[1], q[2]);
        T[s] = e[id] / cp_of(p, c[id]);
    }
    double Tf = or_weno5(T, p->weno_eps);
    double sg = lam > 0.0 ? 1.0 : -1.0;
    *Phi = sg * F;
    if (p->energy_flux == 1)
        *E = lam * Tf;
    else
        *E = sg * ((p->cp_l * F + p->cp_g * (L - F)) * Tf);
}

int or_sweep(const or_grid* g, const or_params* p, int a, const double* c, const double* e,
             const double* cc, const double* ec, const double* vel, double kfac,
             double* c_out, double* e_out, double* acc) {
    if (check_grid(g) || a < 0 || a >= g->ndim) return -1;
    ksum s_clip = {0, 0}, s_eclip = {0, 0}, s_bnd = {0, 0}, s_ebnd = {0, 0};
    ksum s_src = {0, 0}, s_esrc = {0, 0};
    int n[3] = {g->nx, g->ny, g->nz};
    for (int z = 0; z < n[2]; ++z)
        for (int y = 0; y < n[1]; ++y)
            for (int x = 0; x < n[0]; ++x) {
                int pos[3] = {x, y, z};
                int posR[3] = {x, y, z};
                posR[a] += 1;
                double lamL = vel[face_id(g, a, pos[0], pos[1], pos[2])] * kfac;
                double lamR = vel[face_id(g, a, posR[0], posR[1], posR[2])] * kfac;
                double PhiL, EL, PhiR, ER;
                face_flux(g, p, a, c, e, vel, kfac, lamL, pos[0], pos[1], pos[2], &PhiL, &EL);
                face_flux(g, p, a, c, e, vel, kfac, lamR, posR[0], posR[1], posR[2], &PhiR, &ER);
                long id = cell_id(g, x, y, z);
                if (p->energy_flux == 1) {
                    /* eq. disc_et_adv_noncons: the cell's own heat capacity (of the
                       current sweep's state) times the temperature fluxes */
                    double k = cp_of(p, c[id]);
                    EL *= k;
                    ER *= k;
                }
                double dl = lamR - lamL;
                /* dilatation term: the frozen c_c, e_c (Weymouth-Yue), or the cell's own
                   current c, e, i.e. c' = s c - (PhiR - PhiL) (Lagrangian-explicit) */
                double fc = p->split == 1 ? c[id] : cc[id];
                double fe = p->split == 1 ? e[id] : ec[id];
                double cn = c[id] - (PhiR - PhiL) + fc * dl;
                double en = e[id] - (ER - EL) + fe * dl;
                kadd(&s_src, fc * dl);
                kadd(&s_esrc, fe * dl);
                if (cn < 0.0 || cn > 1.0) {
                    /* clip into [0,1] keeping the cell temperature */
                    double T = en / cp_of(p, cn);
                    double cl = cn < 0.0 ? 0.0 : 1.0;
                    double el = en + (p->cp_l - p->cp_g) * (cl - cn) * T;
                    kadd(&s_clip, cl - cn);
                    kadd(&s_eclip, el - en);
                    cn = cl;
                    en = el;
                }
                c_out[id] = cn;
                e_out[id] = en;
                if (g->bc[a] == 1) {
                    if (pos[a] == 0) {
                        kadd(&s_bnd, -PhiL);
                        kadd(&s_ebnd, -EL);
                    }
                    if (pos[a] == n[a] - 1) {
                        kadd(&s_bnd, PhiR);
                        kadd(&s_ebnd, ER);
                    }
                }
            }
    acc[0] += kval(&s_clip);
    acc[1] += kval(&s_eclip);
    acc[2] += kval(&s_bnd);
    acc[3] += kval(&s_ebnd);
    acc[4] += kval(&s_src);
    acc[5] += kval(&s_esrc);
    return 0;
}

/* Step 2 (section 3.3.2). In every mixed cell of c~ with a non-zero mass flux the
   reconstructed plane is moved along its unit normal by
   Delta d = -(m''/rho_l) dt / h (cell units), i.e. alpha* = alpha~ + |m|_2 Delta d,
   and the cell's new fraction is V(m, alpha*), which caps the motion at the cell
   bounds (c = 0 or 1 once the plane has left the cell). The part of the motion that
   leaves the cell is accounted for in the neighbours the interface moves into: a
   pure face neighbour on the side the plane advances into (a liquid cell when the
   liquid evaporates, a gas cell when vapour condenses) receives the volume that the
   moving plane, extended into it, sweeps there,
       V(m, alpha~ - m.o) - V(m, alpha* - m.o)     (o: offset of the neighbour),
   averaged over all the moving planes of its mixed face neighbours with that sign of
   m''. Every cell whose fraction changed then gets the latent correction
   Delta e = Delta c (C_pl - C_pg) T_Gamma (section 3.4.1). */
int or_phase_change(const or_grid* g, const or_params* p, const double* c, const double* e,
                    const double* mdot, double dt, double* c_out, double* e_out, double* acc) {
    if (check_grid(g)) return -1;
    long ntot = (long)g->nx * g->ny * g->nz;
    /* per moving cell: m[3], alpha~, alpha*, motion sign (+1 condensation, -1 evaporation) */
    double* rec = (double*)calloc((size_t)ntot * 6, sizeof(double));
    if (!rec) return -2;
    int n[3] = {g->nx, g->ny, g->nz};
    for (int z = 0; z < n[2]; ++z)
        for (int y = 0; y < n[1]; ++y)
            for (int x = 0; x < n[0]; ++x) {
                long id = cell_id(g, x, y, z);
                double* r = rec + 6 * id;
                c_out[id] = c[id];
                if (mdot[id] == 0.0 || !is_mixed(p, c[id])) continue;
                double c27[27];
                gather27(g, c, x, y, z, c27);
                or_normal(c27, p->normal, r);
                r[3] = or_alpha(r, c[id]);
                double dd = -(mdot[id] / p->rho_l) * (dt / g->h);
                double nm = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
                r[4] = r[3] + nm * dd;
                r[5] = dd > 0.0 ? 1.0 : -1.0;
                c_out[id] = or_volume(r, r[4]);
            }
    for (int z = 0; z < n[2]; ++z)
        for (int y = 0; y < n[1]; ++y)
            for (int x = 0; x < n[0]; ++x) {
                long id = cell_id(g, x, y, z);
                double cj = c[id];
                double want; /* motion sign that advances into this cell */
                if (cj >= 1.0 - p->eps_mixed) want = -1.0;
                else if (cj <= p->eps_mixed) want = 1.0;
                else continue;
                double sum = 0.0;
                int cnt = 0;
                for (int k = 0; k < g->ndim; ++k)
                    for (int s = -1; s <= 1; s += 2) {
                        /* neighbour i at offset s e_k; this cell sits at o = -s e_k from i */
                        int q[3] = {x, y, z};
                        q[k] += s;
                        if (g->bc[k] == 1 && (q[k] < 0 || q[k] >= n[k])) continue;
                        long nid = cell_id(g, q[0], q[1], q[2]);
                        const double* r = rec + 6 * nid;
                        if (r[5] != want) continue;
                        double mo = -s * r[k];
                        double swept = or_volume(r, r[3] - mo) - or_volume(r, r[4] - mo);
                        sum += swept;
                        ++cnt;
                    }
                if (cnt) c_out[id] = cj - sum / cnt;
            }
    ksum s_ph = {0, 0}, s_eph = {0, 0};
    for (long i = 0; i < ntot; ++i) {
        double dc = c_out[i] - c[i];
        double de = (dc * (p->cp_l - p->cp_g)) * p->T_gamma;
        e_out[i] = e[i] + de;
        kadd(&s_ph, dc);
        kadd(&s_eph, de);
    }
    acc[0] += kval(&s_ph);
    acc[1] += kval(&s_eph);
    free(rec);
    return 0;
}

int or_step(const or_grid* g, const or_params* p, const double* c, const double* e,
            const double* u, const double* v, const double* w, const double* mdot,
            double dt, double u_scale, long step_index, double* c_out, double* e_out,
            or_stats* st) {
    if (check_grid(g) || step_index < 0) return -1;
    long n = (long)g->nx * g->ny * g->nz;
    double* cc = (double*)malloc((size_t)n * sizeof(double));
    double* ec = (double*)malloc((size_t)n * sizeof(double));
    double* ca = (double*)malloc((size_t)n * sizeof(double));
    double* ea = (double*)malloc((size_t)n * sizeof(double));
    double* cb = (double*)malloc((size_t)n * sizeof(double));
    double* eb = (double*)malloc((size_t)n * sizeof(double));
    if (!cc || !ec || !ca || !ea || !cb || !eb) {
        free(cc); free(ec); free(ca); free(ea); free(cb); free(eb);
        return -2;
    }
    memset(st, 0, sizeof *st);
    double kfac = (u_scale * dt) / g->h;
    or_prologue(g, p, c, e, cc, ec);
    memcpy(ca, c, (size_t)n * sizeof(double));
    memcpy(ea, e, (size_t)n * sizeof(double));
    double acc[6] = {0, 0, 0, 0, 0, 0};
    const double* vels[3] = {u, v, w};
    long nfaces[3] = {(long)g->nz * g->ny * (g->nx + 1), (long)g->nz * (g->ny + 1) * g->nx,
                      (long)(g->nz + 1) * g->ny * g->nx};
    double maxcfl = 0.0;
    for (int s = 0; s < g->ndim; ++s) {
        int a = (int)((step_index + s) % g->ndim);
        or_sweep(g, p, a, ca, ea, cc, ec, vels[a], kfac, cb, eb, acc);
        for (long f = 0; f < nfaces[a]; ++f) {
            double l = fabs(vels[a][f] * kfac);
            if (l > maxcfl) maxcfl = l;
        }
        double* t;
        t = ca; ca = cb; cb = t;
        t = ea; ea = eb; eb = t;
    }
    double hv = g->ndim == 3 ? g->h * g->h * g->h : g->h * g->h;
    double pc[2] = {0, 0};
    if (mdot) {
        or_phase_change(g, p, ca, ea, mdot, dt, cb, eb, pc);
        double* t;
        t = ca; ca = cb; cb = t;
        t = ea; ea = eb; eb = t;
    }
    ksum sv = {0, 0}, se = {0, 0};
    for (long i = 0; i < n; ++i) {
        kadd(&sv, ca[i]);
        kadd(&se, ea[i]);
    }
    memcpy(c_out, ca, (size_t)n * sizeof(double));
    memcpy(e_out, ea, (size_t)n * sizeof(double));
    st->vol = kval(&sv) * hv;
    st->energy = kval(&se) * hv;
    st->vol_clip = acc[0] * hv;
    st->energy_clip = acc[1] * hv;
    st->vol_bnd_out = acc[2] * hv;
    st->energy_bnd_out = acc[3] * hv;
    st->vol_src = acc[4] * hv;
    st->energy_src = acc[5] * hv;
    st->vol_phase = pc[0] * hv;
    st->energy_phase = pc[1] * hv;
    st->max_cfl = maxcfl;
    free(cc); free(ec); free(ca); free(ea); free(cb); free(eb);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Mass-transfer rate from the PLIC reconstruction (section 3.2).             */
/* ------------------------------------------------------------------------- */

/* Candidates whose collinearity differs by at most this much count as equal (the
   first in the scan order is kept), and pure cells whose node lies closer than this
   to the selected plane (cell units) give no finite-difference gradient. */
#define MASS_FLUX_TIE 1e-12
#define MASS_FLUX_MIN_DIST 1e-6

/* Stencil position (x+ox, y+oy, z+oz) of the 5x5(x5) neighbourhood: periodic axes
   wrap, positions beyond an outflow boundary do not exist (returns -1). */
static long stencil_id(const or_grid* g, int x, int y, int z, int ox, int oy, int oz) {
    int q[3] = {x + ox, y + oy, z + oz};
    for (int a = 0; a < 3; ++a) {
        int n = ncell(g, a);
        if (q[a] >= 0 && q[a] < n) continue;
        if (a == 2 && g->ndim == 2) return -1;
        if (g->bc[a] == 1) return -1;
        q[a] = ((q[a] % n) + n) % n;
    }
    return ((long)q[2] * g->ny + q[1]) * g->nx + q[0];
}

/* Translation from the origin of a cell (its corner nearest the domain origin) to the
   centre (node) of the cell at stencil offset (ox, oy, oz), in cell units; 2D grids
   have no z component. */
static void node_offset(const or_grid* g, int ox, int oy, int oz, double dx[3]) {
    dx[0] = ox + 0.5;
    dx[1] = oy + 0.5;
    dx[2] = g->ndim == 2 ? 0.0 : oz + 0.5;
}

/* n . dx in the fixed order x, y, z. */
static double dot3(const double n[3], const double dx[3]) {
    double s = n[0] * dx[0];
    s += n[1] * dx[1];
    s += n[2] * dx[2];
    return s;
}

int or_mass_flux(const or_grid* g, const or_params* p, const double* c, const double* T,
                 double k_l, double k_g, double h_fg, double* mdot, double* dist) {
    if (check_grid(g) || !(h_fg != 0.0)) return -1;
    const long n = (long)g->nx * g->ny * g->nz;
    const int R = 2;                       /* first and second neighbours */
    const int rz = g->ndim == 2 ? 0 : R;
    /* Plane of every mixed cell (eq. plane_m, eq. cell_d): unit normal n = m/|m|_2
       (liquid towards gas) and distance d = alpha/|m|_2 from the cell origin. */
    double* pn = (double*)calloc((size_t)n * 4, sizeof(double));
    double* q = (double*)malloc((size_t)n * sizeof(double));
    if (!pn || !q) {
        free(pn);
        free(q);
        return -2;
    }
    for (int z = 0; z < g->nz; ++z)
        for (int y = 0; y < g->ny; ++y)
            for (int x = 0; x < g->nx; ++x) {
                long id = ((long)z * g->ny + y) * g->nx + x;
                if (!is_mixed(p, c[id])) continue;
                double c27[27], m[3];
                gather27(g, c, x, y, z, c27);
                or_normal(c27, p->normal, m);
                double alpha = or_alpha(m, c[id]);
                double norm = sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
                pn[4 * id + 0] = m[0] / norm;
                pn[4 * id + 1] = m[1] / norm;
                pn[4 * id + 2] = m[2] / norm;
                pn[4 * id + 3] = alpha / norm;
            }
    /* Pure cells within two cells of a mixed cell: the distance to the plane of the
       neighbouring mixed cell whose normal is most collinear with the translation to
       the pure cell's node, xi = |n . dx| (eq. dint_trans; ties keep the first in the
       scan order), and the finite-difference normal gradient into the pure cell's phase,
       (T - T_Gamma) / d_Gamma (eq. grad_n_T). */
    for (long i = 0; i < n; ++i) {
        q[i] = NAN;
        if (dist) dist[i] = NAN;
    }
    for (int z = 0; z < g->nz; ++z)
        for (int y = 0; y < g->ny; ++y)
            for (int x = 0; x < g->nx; ++x) {
                long id = ((long)z * g->ny + y) * g->nx + x;
                if (is_mixed(p, c[id])) continue;
                int found = 0;
                double best = 0.0, dbest = 0.0;
                for (int oz = -rz; oz <= rz; ++oz)
                    for (int oy = -R; oy <= R; ++oy)
                        for (int ox = -R; ox <= R; ++ox) {
                            long mid = stencil_id(g, x, y, z, ox, oy, oz);
                            if (mid < 0 || !is_mixed(p, c[mid])) continue;
                            double dx[3];
                            node_offset(g, -ox, -oy, -oz, dx);  /* from the mixed cell's origin */
                            double xi = fabs(dot3(pn + 4 * mid, dx));
                            if (!found || xi > best + MASS_FLUX_TIE) {
                                found = 1;
                                best = xi;
                                dbest = pn[4 * mid + 3] - dot3(pn + 4 * mid, dx);
                            }
                        }
                if (!found) continue;
                double d = fabs(dbest) * g->h;
                if (dist) dist[id] = d;
                if (fabs(dbest) > MASS_FLUX_MIN_DIST) q[id] = (T[id] - p->T_gamma) / d;
            }
    /* Mixed cells: per phase, the weighted average of the pure neighbours' gradients in
       the 5x5(x5) block, chi = gamma / sum gamma with gamma = xi / |dx|^2 relative to the
       mixed cell's own plane (eq. normTgrad), and m'' = (k_g G_g + k_l G_l) / h_fg
       (eq. mdot_calc with both gradients taken into their phase). */
    for (int z = 0; z < g->nz; ++z)
        for (int y = 0; y < g->ny; ++y)
            for (int x = 0; x < g->nx; ++x) {
                long id = ((long)z * g->ny + y) * g->nx + x;
                mdot[id] = 0.0;
                if (!is_mixed(p, c[id])) continue;
                double wsum[2] = {0.0, 0.0}, gsum[2] = {0.0, 0.0};
                for (int oz = -rz; oz <= rz; ++oz)
                    for (int oy = -R; oy <= R; ++oy)
                        for (int ox = -R; ox <= R; ++ox) {
                            long pid = stencil_id(g, x, y, z, ox, oy, oz);
                            if (pid < 0 || is_mixed(p, c[pid]) || isnan(q[pid])) continue;
                            double dx[3];
                            node_offset(g, ox, oy, oz, dx);
                            double xi = fabs(dot3(pn + 4 * id, dx));
                            double r2 = dx[0] * dx[0] + dx[1] * dx[1] + dx[2] * dx[2];
                            double gam = xi / r2;
                            int ph = c[pid] >= 0.5 ? 1 : 0; /* 1 liquid, 0 gas */
                            wsum[ph] += gam;
                            gsum[ph] += gam * q[pid];
                        }
                double Gg = wsum[0] > 0.0 ? gsum[0] / wsum[0] : 0.0;
                double Gl = wsum[1] > 0.0 ? gsum[1] / wsum[1] : 0.0;
                mdot[id] = (k_g * Gg + k_l * Gl) / h_fg;
            }
    free(pn);
    free(q);
    return 0;
}
