// Cell geometry of the PLIC reconstruction (section 3.2, eq. plane_m) in closed form:
// the volume of the unit cube below the plane m.x = alpha, its inverse, the liquid
// volume of a sweep's upwind face-flux region, the interface normal and the WENO5
// face value (section 3.4.1). Double precision, usable on host and device.
//
// The volume function is homogeneous of degree 0 in (m, alpha), so no routine here
// needs |m|_1 = 1. Reflecting the axes with m_i < 0 (x_i -> 1 - x_i) and sorting the
// magnitudes gives 0 <= m1 <= m2 <= m3 with sum S; by central symmetry only
// alpha <= S/2 is needed (V(alpha) = 1 - V(S - alpha)), where the cube cut by the
// plane is, with m12 = m1 + m2:
//   alpha <  m1            : a corner tetrahedron          V = a^3 / (6 m1 m2 m3)
//   m1 <= alpha < m2       : a truncated tetrahedron       V = (3a^2 - 3a m1 + m1^2) / (6 m2 m3)
//   m2 <= alpha < min(m12, m3): two corners cut off
//       V = ((3a^2 - 3a m1 + m1^2) - (a - m2)^3 / m1) / (6 m2 m3)
//   m12 <= alpha <= m3     : the plane crosses all four edges along x3
//       V = (a - m12/2) / m3
//   m3 <= alpha < m12      : three corners cut off
//       V = ((3a^2 - 3a m1 + m1^2) - ((a - m2)^3 + (a - m3)^3) / m1) / (6 m2 m3)
// These are the inclusion-exclusion sums over the cube's vertices, divided through by
// the vanishing factors so that every regime stays well conditioned when components
// of m go to zero (each regime is empty when its divisor is zero).
#pragma once

#include <math.h>

#if defined(__HIPCC__)
#define PCV_HD __host__ __device__ __forceinline__
#else
#define PCV_HD static inline
#endif

namespace pcv {

struct Sorted3 {
    double m1, m2, m3;  // 0 <= m1 <= m2 <= m3
};

PCV_HD Sorted3 sort_abs(double a, double b, double c) {
    a = fabs(a);
    b = fabs(b);
    c = fabs(c);
    double lo = fmin(a, b), hi = fmax(a, b);
    double m1 = fmin(lo, c);
    double t = fmax(lo, c);
    double m2 = fmin(t, hi);
    double m3 = fmax(t, hi);
    return {m1, m2, m3};
}

// V for 0 <= a <= S/2 (lower half).
PCV_HD double vol_lower(const Sorted3& s, double a) {
    const double m1 = s.m1, m2 = s.m2, m3 = s.m3;
    if (a <= 0.0) return 0.0;
    if (a < m1) return a * a * a / (6.0 * m1 * m2 * m3);
    const double q = 3.0 * a * a - 3.0 * a * m1 + m1 * m1;
    if (a < m2) return q / (6.0 * m2 * m3);
    const double m12 = m1 + m2;
    if (m12 <= m3) {
        if (a < m12) {
            const double t = a - m2;
            return (q - t * t * t / m1) / (6.0 * m2 * m3);
        }
        return (a - 0.5 * m12) / m3;
    }
    const double t2 = a - m2;
    if (a < m3) return (q - t2 * t2 * t2 / m1) / (6.0 * m2 * m3);
    const double t3 = a - m3;
    return (q - (t2 * t2 * t2 + t3 * t3 * t3) / m1) / (6.0 * m2 * m3);
}

// |{x in [0,1]^3 : m.x <= alpha}| for any non-zero m.
PCV_HD double volume(double mx, double my, double mz, double alpha) {
    double a = alpha;
    if (mx < 0.0) a -= mx;
    if (my < 0.0) a -= my;
    if (mz < 0.0) a -= mz;
    const Sorted3 s = sort_abs(mx, my, mz);
    const double S = s.m1 + s.m2 + s.m3;
    if (a <= 0.0) return 0.0;
    if (a >= S) return 1.0;
    // one evaluation of the lower half for both halves (a single inlined copy, so that
    // lanes on either side of S / 2 run the same instructions)
    const bool up = !(a <= 0.5 * S);
    const double v = vol_lower(s, up ? S - a : a);
    return up ? 1.0 - v : v;
}

// Cube root of x > 0: a single-precision estimate refined by one Halley step in double
// precision (cubic convergence takes the ~1e-7 relative error of the estimate below
// rounding). Arguments outside the single-precision normal range use the library cbrt.
PCV_HD double cbrt_pos(double x) {
    if (!(x > 1e-36 && x < 1e36)) return cbrt(x);
    const double r = (double)cbrtf((float)x);
    const double r3 = r * r * r;
    return r * (r3 + 2.0 * x) / (2.0 * r3 + x);
}

// Inverse of vol_lower for 0 < v <= 1/2: closed forms in the tetrahedron,
// truncated-tetrahedron and four-edge regimes; Halley iterations (cubic convergence)
// on the cubic regimes, started from the chord between the regime's end points and
// kept inside the regime's bracket. A step below 1e-8 of the bracket leaves an error
// far below rounding, so at most three iterations run (six are allowed).
PCV_HD double alpha_lower(const Sorted3& s, double v) {
    const double m1 = s.m1, m2 = s.m2, m3 = s.m3;
    const double m12 = m1 + m2;
    const double d6 = 6.0 * m2 * m3;
    if (m1 > 0.0) {
        const double v1 = m1 * m1 / d6;
        if (v < v1) return cbrt_pos(6.0 * m1 * m2 * m3 * v);
    }
    if (!(m2 > 0.0)) return m3 * v;  // m1 = m2 = 0: a slab
    const double v2 = (3.0 * m2 * m2 - 3.0 * m2 * m1 + m1 * m1) / d6;  // V(m2)
    if (v < v2) return 0.5 * m1 + sqrt(fmax(2.0 * m2 * m3 * v - m1 * m1 / 12.0, 0.0));
    // the cubic regimes (m1 > 0 here: with m1 = 0 the truncated and four-edge regimes
    // meet at V = m2 / (2 m3)); the volumes at the bracket ends are the regime bounds
    // already known: V(m2) = v2, V(m12) or V(m3) = v3, V(S/2) = 1/2
    double lo, hi, vlo, vhi;
    int three;  // number of corners cut off in the cubic regime
    if (m12 <= m3) {
        const double v3 = 0.5 * m12 / m3;
        if (v >= v3) return m3 * v + 0.5 * m12;
        lo = m2;
        hi = m12;
        vlo = v2;
        vhi = v3;
        three = 0;
    } else {
        // V(m3): two corners cut off, (q(m3) - (m3 - m2)^3 / m1) / (6 m2 m3)
        const double t = m3 - m2;
        const double v3 = ((3.0 * m3 * m3 - 3.0 * m3 * m1 + m1 * m1) - t * t * t / m1) / d6;
        if (v < v3) {
            lo = m2;
            hi = m3;
            vlo = v2;
            vhi = v3;
            three = 0;
        } else {
            lo = m3;
            hi = 0.5 * (m1 + m2 + m3);
            vlo = v3;
            vhi = 0.5;
            three = 1;
        }
    }
    const double inv_m1 = 1.0 / m1;
    const double inv_d2 = 1.0 / (2.0 * m2 * m3);
    double a = (vhi > vlo) ? lo + (hi - lo) * ((v - vlo) / (vhi - vlo)) : lo;
    const double tol = 1e-8 * (hi - lo);
    for (int it = 0; it < 6; ++it) {
        // f = V(a) - v and its first two derivatives (V is cubic in the regime)
        const double t2 = a - m2;
        const double q = 3.0 * a * a - 3.0 * a * m1 + m1 * m1;
        double cub = t2 * t2 * t2, sq = t2 * t2, lin = t2;
        if (three) {
            const double t3 = a - m3;
            cub += t3 * t3 * t3;
            sq += t3 * t3;
            lin += t3;
        }
        const double f = (q - cub * inv_m1) * (inv_d2 / 3.0) - v;
        const double fp = ((2.0 * a - m1) - sq * inv_m1) * inv_d2;
        const double fpp = (2.0 - 2.0 * lin * inv_m1) * inv_d2;
        double an = a - 2.0 * f * fp / (2.0 * fp * fp - f * fpp);
        an = fmin(fmax(an, lo), hi);
        const double step = an - a;
        a = an;
        if (fabs(step) <= tol) break;
    }
    return a;
}

// Plane constant alpha with volume(m, alpha) = c, 0 < c < 1, in the scaling of m.
PCV_HD double alpha_of(double mx, double my, double mz, double c) {
    double shift = 0.0;
    if (mx < 0.0) shift += mx;
    if (my < 0.0) shift += my;
    if (mz < 0.0) shift += mz;
    const Sorted3 s = sort_abs(mx, my, mz);
    const double S = s.m1 + s.m2 + s.m3;
    // one inversion of the lower half for both halves (a single inlined copy)
    const bool up = !(c <= 0.5);
    const double la = alpha_lower(s, up ? 1.0 - c : c);
    const double a = up ? S - la : la;
    return a + shift;
}

// Liquid volume, in cell units, of the donor region crossing a face during a sweep
// along `axis` with face CFL number lam: x_axis in [1-lam, 1] of the left donor for
// lam > 0, x_axis in [0, |lam|] of the right donor for lam < 0, mapped affinely onto
// the unit cube.
PCV_HD double slab(double mx, double my, double mz, double alpha, int axis, double lam) {
    const double L = fabs(lam);
    if (L == 0.0) return 0.0;
    double m[3] = {mx, my, mz};
    double a = alpha;
    if (lam > 0.0) a = alpha - m[axis] * (1.0 - L);
    m[axis] = m[axis] * L;
    return L * volume(m[0], m[1], m[2], a);
}

// Fifth-order WENO face value (Jiang-Shu) between v2 and v3 from the left-biased
// stencil v0..v4: candidate parabolas of the three sub-stencils, smoothness
// indicators, weights d_k / (eps + beta_k)^2 normalised with one division.
PCV_HD double weno5(double v0, double v1, double v2, double v3, double v4, double eps) {
    const double q0 = (2.0 * v0 - 7.0 * v1 + 11.0 * v2) * (1.0 / 6.0);
    const double q1 = (-v1 + 5.0 * v2 + 2.0 * v3) * (1.0 / 6.0);
    const double q2 = (2.0 * v2 + 5.0 * v3 - v4) * (1.0 / 6.0);
    const double s0a = v0 - 2.0 * v1 + v2, s0b = v0 - 4.0 * v1 + 3.0 * v2;
    const double s1a = v1 - 2.0 * v2 + v3, s1b = v1 - v3;
    const double s2a = v2 - 2.0 * v3 + v4, s2b = 3.0 * v2 - 4.0 * v3 + v4;
    const double k = 13.0 / 12.0;
    const double b0 = eps + (k * s0a * s0a + 0.25 * s0b * s0b);
    const double b1 = eps + (k * s1a * s1a + 0.25 * s1b * s1b);
    const double b2 = eps + (k * s2a * s2a + 0.25 * s2b * s2b);
    const double t0 = b0 * b0, t1 = b1 * b1, t2 = b2 * b2;
    const double w0 = 0.1 * (t1 * t2), w1 = 0.6 * (t0 * t2), w2 = 0.3 * (t0 * t1);
    return (w0 * q0 + w1 * q1 + w2 * q2) / (w0 + w1 + w2);
}

// Interface normal from the 3x3x3 fractions around a cell, c27[(dz+1)*9+(dy+1)*3+(dx+1)].
// Every operation that feeds a decision is evaluated in a fixed order, without
// contraction (the rest of the library contracts multiply-adds into FMAs), so that
// identical inputs always give identical normals, and every
// decision uses the tie band kNormalTie (gradients up to it count as zero, candidates
// within it as equal, lowest axis first), so that round-off differences of the inputs
// cannot switch formulas; symmetric configurations produce exact ties.
//   Youngs: g_a = sum over the transverse block, second transverse offset outermost,
//   of (1,2,1)x(1,2,1)-weighted central differences; m = -g / |g|_1, (1,0,0) if g = 0.
//   Centred columns along d (valid when g_d != 0): transverse components
//   (H(-1) - H(+1)) / 2 from the 3-cell column sums H at the four transverse
//   neighbours, column component +1 if g_d < 0 else -1, normalised by its l1 norm L_d.
//   Mixed Youngs-centred (method 1): the valid candidate with the largest own
//   component 1/L_d (lowest axis on ties) unless that exceeds Youngs' largest
//   component, which signals columns that do not bracket the interface; then Youngs.
//   Method 2: the best centred-columns candidate (Youngs if none is valid).
struct Normal {
    double m[3];
};

constexpr double kNormalTie = 1e-12;

PCV_HD double c27_at(const double* c27, int a, int oa, int t1, int o1, int t2, int o2) {
    const int ox = a == 0 ? oa : (t1 == 0 ? o1 : o2);
    const int oy = a == 1 ? oa : (t1 == 1 ? o1 : o2);
    const int oz = a == 2 ? oa : (t1 == 2 ? o1 : o2);
    return c27[(oz + 1) * 9 + (oy + 1) * 3 + (ox + 1)];
}

PCV_HD Normal normal27(const double* c27, int method) {
#pragma clang fp contract(off)
    double g[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int t1 = (a == 0) ? 1 : 0;
        const int t2 = (a == 2) ? 1 : 2;
        double acc = 0.0;
#pragma unroll
        for (int o2 = -1; o2 <= 1; ++o2) {
            const double w2 = (o2 == 0) ? 2.0 : 1.0;
#pragma unroll
            for (int o1 = -1; o1 <= 1; ++o1) {
                const double w1 = (o1 == 0) ? 2.0 : 1.0;
                const double d = c27_at(c27, a, 1, t1, o1, t2, o2) - c27_at(c27, a, -1, t1, o1, t2, o2);
                acc = acc + (w1 * w2) * d;
            }
        }
        g[a] = acc;
    }
    const double LY = (fabs(g[0]) + fabs(g[1])) + fabs(g[2]);
    Normal y = {{1.0, 0.0, 0.0}};
    const bool flat = LY <= kNormalTie;
    if (!flat) {
        y.m[0] = -g[0] / LY;
        y.m[1] = -g[1] / LY;
        y.m[2] = -g[2] / LY;
    }
    if (method == 0 || flat) return y;
    int best = -1;
    double best_own = 0.0, best_L = 1.0;
    double best_c[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if (fabs(g[d]) <= kNormalTie) continue;
        const int t1 = (d == 0) ? 1 : 0;
        const int t2 = (d == 2) ? 1 : 2;
        double H[2][2];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int o = s == 0 ? -1 : 1;
            H[0][s] = (c27_at(c27, d, -1, t1, o, t2, 0) + c27_at(c27, d, 0, t1, o, t2, 0)) +
                      c27_at(c27, d, 1, t1, o, t2, 0);
            H[1][s] = (c27_at(c27, d, -1, t1, 0, t2, o) + c27_at(c27, d, 0, t1, 0, t2, o)) +
                      c27_at(c27, d, 1, t1, 0, t2, o);
        }
        double comp[3];
        comp[d] = g[d] < 0.0 ? 1.0 : -1.0;
        comp[t1] = 0.5 * (H[0][0] - H[0][1]);
        comp[t2] = 0.5 * (H[1][0] - H[1][1]);
        const double L = (fabs(comp[0]) + fabs(comp[1])) + fabs(comp[2]);
        const double own = 1.0 / L;
        if (best < 0 || own > best_own + kNormalTie) {
            best = d;
            best_own = own;
            best_L = L;
            best_c[0] = comp[0];
            best_c[1] = comp[1];
            best_c[2] = comp[2];
        }
    }
    if (best < 0) return y;
    if (method == 1) {
        double ymax = fabs(y.m[0]);
        if (fabs(y.m[1]) > ymax) ymax = fabs(y.m[1]);
        if (fabs(y.m[2]) > ymax) ymax = fabs(y.m[2]);
        if (best_own > ymax + kNormalTie) return y;
    }
    Normal r;
    r.m[0] = best_c[0] / best_L;
    r.m[1] = best_c[1] / best_L;
    r.m[2] = best_c[2] / best_L;
    return r;
}

}  // namespace pcv
