// Single-precision cell geometry for the mixed-precision mode: the same closed forms
// as geom.h (PLIC plane of section 3.2, eq. plane_m; volume, inverse and upwind slab
// volume) evaluated in float. The caller keeps double precision for the plane
// constant where the fraction is close to 0 or 1 and for every accumulation.
#pragma once

#include "geom.h"

namespace pcv {

struct Sorted3f {
    float m1, m2, m3;  // 0 <= m1 <= m2 <= m3
};

PCV_HD Sorted3f sort_abs_f(float a, float b, float c) {
    a = fabsf(a);
    b = fabsf(b);
    c = fabsf(c);
    const float lo = fminf(a, b), hi = fmaxf(a, b);
    const float m1 = fminf(lo, c);
    const float t = fmaxf(lo, c);
    return {m1, fminf(t, hi), fmaxf(t, hi)};
}

// V for 0 <= a <= S/2 (the regimes of geom.h).
PCV_HD float vol_lower_f(const Sorted3f& s, float a) {
    const float m1 = s.m1, m2 = s.m2, m3 = s.m3;
    if (a <= 0.0f) return 0.0f;
    if (a < m1) return a * a * a / (6.0f * m1 * m2 * m3);
    const float q = 3.0f * a * a - 3.0f * a * m1 + m1 * m1;
    if (a < m2) return q / (6.0f * m2 * m3);
    const float m12 = m1 + m2;
    if (m12 <= m3) {
        if (a < m12) {
            const float t = a - m2;
            return (q - t * t * t / m1) / (6.0f * m2 * m3);
        }
        return (a - 0.5f * m12) / m3;
    }
    const float t2 = a - m2;
    if (a < m3) return (q - t2 * t2 * t2 / m1) / (6.0f * m2 * m3);
    const float t3 = a - m3;
    return (q - (t2 * t2 * t2 + t3 * t3 * t3) / m1) / (6.0f * m2 * m3);
}

PCV_HD float volume_f(float mx, float my, float mz, float alpha) {
    float a = alpha;
    if (mx < 0.0f) a -= mx;
    if (my < 0.0f) a -= my;
    if (mz < 0.0f) a -= mz;
    const Sorted3f s = sort_abs_f(mx, my, mz);
    const float S = s.m1 + s.m2 + s.m3;
    if (a <= 0.0f) return 0.0f;
    if (a >= S) return 1.0f;
    const bool up = !(a <= 0.5f * S);  // one inlined copy for both halves
    const float v = vol_lower_f(s, up ? S - a : a);
    return up ? 1.0f - v : v;
}

// Inverse of vol_lower_f for 0 < v <= 1/2: closed forms, and Halley iterations on the
// cubic regimes (as in geom.h).
PCV_HD float alpha_lower_f(const Sorted3f& s, float v) {
    const float m1 = s.m1, m2 = s.m2, m3 = s.m3;
    const float m12 = m1 + m2;
    const float d6 = 6.0f * m2 * m3;
    if (m1 > 0.0f && v < m1 * m1 / d6) return cbrtf(6.0f * m1 * m2 * m3 * v);
    if (!(m2 > 0.0f)) return m3 * v;
    const float v2 = (3.0f * m2 * m2 - 3.0f * m2 * m1 + m1 * m1) / d6;  // V(m2)
    if (v < v2) return 0.5f * m1 + sqrtf(fmaxf(2.0f * m2 * m3 * v - m1 * m1 / 12.0f, 0.0f));
    // cubic regimes: the bracket ends' volumes are the regime bounds (see alpha_lower)
    float lo, hi, vlo, vhi;
    int three;
    if (m12 <= m3) {
        const float v3 = 0.5f * m12 / m3;
        if (v >= v3) return m3 * v + 0.5f * m12;
        lo = m2;
        hi = m12;
        vlo = v2;
        vhi = v3;
        three = 0;
    } else {
        const float t = m3 - m2;
        const float v3 = ((3.0f * m3 * m3 - 3.0f * m3 * m1 + m1 * m1) - t * t * t / m1) / d6;  // V(m3)
        if (v < v3) {
            lo = m2;
            hi = m3;
            vlo = v2;
            vhi = v3;
            three = 0;
        } else {
            lo = m3;
            hi = 0.5f * (m1 + m2 + m3);
            vlo = v3;
            vhi = 0.5f;
            three = 1;
        }
    }
    const float inv_m1 = 1.0f / m1;
    const float inv_d2 = 1.0f / (2.0f * m2 * m3);
    float a = (vhi > vlo) ? lo + (hi - lo) * ((v - vlo) / (vhi - vlo)) : lo;
    const float tol = 1e-4f * (hi - lo);
    for (int it = 0; it < 4; ++it) {
        const float t2 = a - m2;
        const float q = 3.0f * a * a - 3.0f * a * m1 + m1 * m1;
        float cub = t2 * t2 * t2, sq = t2 * t2, lin = t2;
        if (three) {
            const float t3 = a - m3;
            cub += t3 * t3 * t3;
            sq += t3 * t3;
            lin += t3;
        }
        const float f = (q - cub * inv_m1) * (inv_d2 / 3.0f) - v;
        const float fp = ((2.0f * a - m1) - sq * inv_m1) * inv_d2;
        const float fpp = (2.0f - 2.0f * lin * inv_m1) * inv_d2;
        float an = a - 2.0f * f * fp / (2.0f * fp * fp - f * fpp);
        an = fminf(fmaxf(an, lo), hi);
        const float step = an - a;
        a = an;
        if (fabsf(step) <= tol) break;
    }
    return a;
}

// Plane constant for fraction c with cbar = 1 - c taken in double precision by the
// caller (so that fractions close to 1 keep their gas volume).
PCV_HD float alpha_of_f(float mx, float my, float mz, float c, float cbar) {
    float shift = 0.0f;
    if (mx < 0.0f) shift += mx;
    if (my < 0.0f) shift += my;
    if (mz < 0.0f) shift += mz;
    const Sorted3f s = sort_abs_f(mx, my, mz);
    const float S = s.m1 + s.m2 + s.m3;
    const bool up = !(c <= 0.5f);  // one inlined copy for both halves
    const float la = alpha_lower_f(s, up ? cbar : c);
    const float a = up ? S - la : la;
    return a + shift;
}

PCV_HD float slab_f(float mx, float my, float mz, float alpha, int axis, float lam) {
    const float L = fabsf(lam);
    if (L == 0.0f) return 0.0f;
    float m[3] = {mx, my, mz};
    float a = alpha;
    if (lam > 0.0f) a = alpha - m[axis] * (1.0f - L);
    m[axis] = m[axis] * L;
    return L * volume_f(m[0], m[1], m[2], a);
}

// Normal from the 3x3x3 fractions (the estimators of normal27 in geom.h) in float,
// with a tie band suited to single precision.
struct NormalF {
    float m[3];
};

constexpr float kNormalTieF = 1e-6f;

PCV_HD float c27f_at(const float* c27, int a, int oa, int t1, int o1, int t2, int o2) {
    const int ox = a == 0 ? oa : (t1 == 0 ? o1 : o2);
    const int oy = a == 1 ? oa : (t1 == 1 ? o1 : o2);
    const int oz = a == 2 ? oa : (t1 == 2 ? o1 : o2);
    return c27[(oz + 1) * 9 + (oy + 1) * 3 + (ox + 1)];
}

PCV_HD NormalF normal27_f(const float* c27, int method) {
    float g[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int t1 = (a == 0) ? 1 : 0;
        const int t2 = (a == 2) ? 1 : 2;
        float acc = 0.0f;
#pragma unroll
        for (int o2 = -1; o2 <= 1; ++o2) {
            const float w2 = (o2 == 0) ? 2.0f : 1.0f;
#pragma unroll
            for (int o1 = -1; o1 <= 1; ++o1) {
                const float w1 = (o1 == 0) ? 2.0f : 1.0f;
                acc += (w1 * w2) * (c27f_at(c27, a, 1, t1, o1, t2, o2) - c27f_at(c27, a, -1, t1, o1, t2, o2));
            }
        }
        g[a] = acc;
    }
    const float LY = fabsf(g[0]) + fabsf(g[1]) + fabsf(g[2]);
    NormalF y = {{1.0f, 0.0f, 0.0f}};
    const bool flat = LY <= kNormalTieF;
    if (!flat) {
        const float inv = 1.0f / LY;
        y.m[0] = -g[0] * inv;
        y.m[1] = -g[1] * inv;
        y.m[2] = -g[2] * inv;
    }
    if (method == 0 || flat) return y;
    int best = -1;
    float best_own = 0.0f, best_L = 1.0f;
    float best_c[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if (fabsf(g[d]) <= kNormalTieF) continue;
        const int t1 = (d == 0) ? 1 : 0;
        const int t2 = (d == 2) ? 1 : 2;
        float H[2][2];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int o = s == 0 ? -1 : 1;
            H[0][s] = c27f_at(c27, d, -1, t1, o, t2, 0) + c27f_at(c27, d, 0, t1, o, t2, 0) +
                      c27f_at(c27, d, 1, t1, o, t2, 0);
            H[1][s] = c27f_at(c27, d, -1, t1, 0, t2, o) + c27f_at(c27, d, 0, t1, 0, t2, o) +
                      c27f_at(c27, d, 1, t1, 0, t2, o);
        }
        float comp[3];
        comp[d] = g[d] < 0.0f ? 1.0f : -1.0f;
        comp[t1] = 0.5f * (H[0][0] - H[0][1]);
        comp[t2] = 0.5f * (H[1][0] - H[1][1]);
        const float L = fabsf(comp[0]) + fabsf(comp[1]) + fabsf(comp[2]);
        const float own = 1.0f / L;
        if (best < 0 || own > best_own + kNormalTieF) {
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
        const float ymax = fmaxf(fabsf(y.m[0]), fmaxf(fabsf(y.m[1]), fabsf(y.m[2])));
        if (best_own > ymax + kNormalTieF) return y;
    }
    const float inv = 1.0f / best_L;
    NormalF r;
    r.m[0] = best_c[0] * inv;
    r.m[1] = best_c[1] * inv;
    r.m[2] = best_c[2] * inv;
    return r;
}

}  // namespace pcv
