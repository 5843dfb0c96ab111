// crmath.h -- correctly rounded binary64 exp, log, log1p, pow and u^(1/a),
// the elementary functions of the bitexact setting (Section 4.2, exact
// reproducibility across platforms: with bitexact on, every library function
// call of every sampler is one whose result does not depend on the platform).
// A correctly rounded function has exactly one admissible result, so a draw
// made with these is the same on any hardware and equal, bit for bit, to any
// other correctly rounded evaluation of the same formula.
//
// Method: each function is evaluated in triple-double arithmetic (three
// binary64 words h + m + l) to a relative error below about 2^-140, then
// rounded once to binary64 with the correctly rounded three-term sum of
// Boldo and Melquiond ("Emulation of FMA and correctly rounded sums: proved
// algorithms using rounding to odd", IEEE Trans. Computers 57(4), 2008),
// whose inner sum is rounded to odd.  The triple-double building blocks are
// error-free transformations (Knuth's TwoSum, the fused-multiply-add product)
// followed by a renormalisation, in the manner of Lauter ("Basic building
// blocks for a triple-double intermediate format", INRIA RR-5702, 2005).
// The result is correct whenever the exact value lies farther than the
// evaluation error from a rounding boundary; for exp, log and log1p the
// published searches for hardest-to-round binary64 arguments (Lefevre and
// Muller) put every non-exact value much farther than 2^-140 relative from a
// midpoint, and the exact cases (exp(0), log(1), ...) are taken apart.  pow
// and u^(1/a) have two arguments and no such exhaustive search; a result
// that is itself exactly a binary64 midpoint (an integer power of a short
// operand) is rounded from the 2^-140 evaluation.
//
// Reductions.  exp: x = k ln2/64 + r with k = round(64 x/ln2), |r| <= ln2/128,
// exp(x) = 2^(k div 64) 2^((k mod 64)/64) exp(r), exp(r) by its Taylor
// polynomial of degree 14.  log: x = 2^e m with m in [sqrt(1/2), sqrt(2)),
// c = an 8-bit approximation of 1/m from a 128-entry table, r = m c - 1
// (exact, |r| < 2^-7), log(x) = e ln2 - log(c) + log1p(r), log1p(r) by its
// series to degree 21.  The tables and constants come from decimal
// arithmetic (gen_crmath_tables.py).  Everything here is plain binary64
// arithmetic with explicit fma, so the host and device builds agree bit for
// bit.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace rp {
namespace crm {

#include "crmath_tables.inc"

#define CRM_FN __host__ __device__ inline

struct TD {
    double h, m, l;
};

CRM_FN uint64_t bits_of(double x)
{
    uint64_t u;
    __builtin_memcpy(&u, &x, 8);
    return u;
}
CRM_FN double from_bits(uint64_t u)
{
    double x;
    __builtin_memcpy(&x, &u, 8);
    return x;
}

// s + e == a + b exactly (Knuth)
CRM_FN void two_sum(double a, double b, double &s, double &e)
{
    s = a + b;
    const double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}
// p + e == a b exactly (no underflow)
CRM_FN void two_prod(double a, double b, double &p, double &e)
{
    p = a * b;
    e = fma(a, b, -p);
}

// The four doubles as a triple-double: one exact VecSum pass, a second pass
// over its errors, the last two error words rounded into one (a relative
// error near 2^-159 of the largest partial sum).
CRM_FN TD renorm(double a, double b, double c, double d)
{
    double s, e1, e2, e3;
    two_sum(c, d, s, e3);
    two_sum(b, s, s, e2);
    two_sum(a, s, s, e1);
    double t, f1, f2;
    two_sum(e2, e3, t, f2);
    two_sum(e1, t, t, f1);
    const double u = f1 + f2;
    double h, g, m, l;
    two_sum(s, t, h, g);
    two_sum(g, u, m, l);
    return TD{h, m, l};
}

CRM_FN TD td_add(const TD &a, const TD &b)
{
    double s0, e0, s1, e1;
    two_sum(a.h, b.h, s0, e0);
    two_sum(a.m, b.m, s1, e1);
    return renorm(s0, s1, e0, e1 + (a.l + b.l));
}

CRM_FN TD td_add_d(const TD &a, double b)
{
    double s0, e0;
    two_sum(a.h, b, s0, e0);
    return renorm(s0, a.m, e0, a.l);
}

CRM_FN TD td_mul(const TD &a, const TD &b)
{
    double p0, q0, p1, q1, p2, q2;
    two_prod(a.h, b.h, p0, q0);
    two_prod(a.h, b.m, p1, q1);
    two_prod(a.m, b.h, p2, q2);
    double s1, e1, e2;
    two_sum(p1, p2, s1, e1);
    two_sum(s1, q0, s1, e2);
    const double lo = ((a.h * b.l + a.m * b.m) + a.l * b.h) + ((q1 + q2) + (e1 + e2));
    return renorm(p0, s1, lo, 0.0);
}

CRM_FN TD td_mul_d(const TD &a, double b)
{
    double p0, q0, p1, q1;
    two_prod(a.h, b, p0, q0);
    two_prod(a.m, b, p1, q1);
    double s1, e1;
    two_sum(p1, q0, s1, e1);
    return renorm(p0, s1, a.l * b + q1, e1);
}

// a / b by three steps of long division, each remainder formed exactly
CRM_FN TD td_div_d(const TD &a, double b)
{
    const double q0 = a.h / b;
    double p, e;
    two_prod(q0, b, p, e);
    TD r = renorm(a.h - p, -e, a.m, a.l);  // a.h - p is exact (remainder of a rounded quotient)
    const double q1 = r.h / b;
    two_prod(q1, b, p, e);
    r = renorm(r.h - p, -e, r.m, r.l);
    const double q2 = r.h / b;
    return renorm(q0, q1, q2, 0.0);
}

CRM_FN TD td_of(const double *t) { return TD{t[0], t[1], t[2]}; }

// ---------------------------------------------------------------------------
// RN(a + b + c) (Boldo and Melquiond): the low part of a + b + c rounded to
// odd, then one rounding to nearest.  No underflow or overflow inside.
CRM_FN double round_odd_sum(double x, double y)
{
    double s, e;
    two_sum(x, y, s, e);
    if (e != 0.0 && (bits_of(s) & 1) == 0) {
        // s is even and the exact sum lies between s and its neighbour on
        // e's side, which is odd
        const bool away = (s > 0.0) == (e > 0.0);
        s = from_bits(away ? bits_of(s) + 1 : bits_of(s) - 1);
    }
    return s;
}

CRM_FN double rn3(double a, double b, double c)
{
    double uh, ul, th, tl;
    two_sum(b, c, uh, ul);
    two_sum(a, uh, th, tl);
    const double v = round_odd_sum(tl, ul);
    return th + v;
}

// RN(2^k (y.h + y.m + y.l)) for y.h in about [0.7, 1.42]: binary scaling of
// the rounded value in the normal range, rounding on the subnormal grid
// below it, overflow to +inf above.
CRM_FN double round_scaled(const TD &y, int k)
{
    // at k = -1022 the values y >= 1 are normal, and the grid of [1, 2) scaled
    // by 2^-1022 is the subnormal spacing 2^-1074 as well
    if (k >= -1021 || (k == -1022 && y.h >= 1.0)) {
        const double r = rn3(y.h, y.m, y.l);
        if (k > 1024) return HUGE_VAL;
        return ldexp(r, k);  // exact, or +inf when 2^k r overflows
    }
    const int s = k + 1074;  // y 2^s counts units of 2^-1074, below 2^52 here
    if (s < -1) return 0.0;  // below 1.42 / 4 units: rounds to 0
    const double hs = ldexp(y.h, s), ms = ldexp(y.m, s), ls = ldexp(y.l, s);
    const double M = 0x1p52;  // M + v has unit spacing for 0 <= v < 2^52
    double a, b, c, d;
    two_sum(M, hs, a, b);
    two_sum(b, ms, c, d);
    const double q = rn3(a, c, d + ls) - M;
    return ldexp(q, -1074);
}

// ---------------------------------------------------------------------------
// exp(x) for a triple-double x with |x.h| <= 746: 2^k y with y = 2^(j/64) exp(r)
CRM_FN TD exp_td(const TD &x, int &k_out)
{
    const double kd = rint(x.h * CRM_INV_LN2_64);
    const int k = (int)kd;
    const int j = k & 63;
    k_out = (k - j) / 64;
    // r = x - k ln2/64: k c1 is exact (36-bit c1, |k| < 2^17) and x.h - k c1
    // is exact (the two are within a factor of two of each other, or k = 0)
    const double r0 = x.h - kd * CRM_LN2_64[0];
    double p2, e2, p3, e3;
    two_prod(kd, CRM_LN2_64[1], p2, e2);
    two_prod(kd, CRM_LN2_64[2], p3, e3);
    const double low = x.l - (e3 + kd * CRM_LN2_64[3]);
    TD r = renorm(r0, x.m, -p2, -e2);
    r = td_add(r, renorm(-p3, low, 0.0, 0.0));
    // exp(r) = sum_{i <= 14} r^i / i!, Horner from the top: binary64 for the
    // terms of degree >= 11, double-double for 6..10, triple-double below
    double sd = CRM_INV_FACT[14][0];
    for (int i = 13; i >= 11; i--) sd = fma(sd, r.h, CRM_INV_FACT[i][0]);
    // double-double stage: (dh, dl) = (dh, dl) r + c_i
    double dh = sd, dl = 0.0;
    for (int i = 10; i >= 6; i--) {
        double ph, pl;
        two_prod(dh, r.h, ph, pl);
        pl = pl + (dh * r.m + dl * r.h);
        double sh, se;
        two_sum(CRM_INV_FACT[i][0], ph, sh, se);
        se = se + (CRM_INV_FACT[i][1] + pl);
        two_sum(sh, se, dh, dl);
    }
    TD q{dh, dl, 0.0};
    for (int i = 5; i >= 0; i--) q = td_add(td_mul(q, r), td_of(CRM_INV_FACT[i]));
    return td_mul(q, td_of(CRM_EXP_T[j]));
}

// log1p(r) for |r| < 2^-7 (r exact): r q_1 with q_i = 1/i - r q_{i+1} up to
// degree 21; binary64 for i >= 15, double-double for 7..14, triple-double
// below
CRM_FN TD log1p_series(double r)
{
    double sd = CRM_INV_INT[21][0];
    for (int i = 20; i >= 15; i--) sd = CRM_INV_INT[i][0] - r * sd;
    double dh = sd, dl = 0.0;
    for (int i = 14; i >= 7; i--) {
        double ph, pl;
        two_prod(dh, r, ph, pl);
        pl = pl + dl * r;
        double sh, se;
        two_sum(CRM_INV_INT[i][0], -ph, sh, se);
        se = se + (CRM_INV_INT[i][1] - pl);
        two_sum(sh, se, dh, dl);
    }
    TD q{dh, dl, 0.0};
    for (int i = 6; i >= 1; i--) {
        const TD t = td_mul_d(q, -r);
        q = td_add(t, td_of(CRM_INV_INT[i]));
    }
    return td_mul_d(q, r);
}

// log(x) for finite x > 0
CRM_FN TD log_td(double x)
{
    int e = 0;
    if (x < 0x1p-1022) {
        x *= 0x1p64;
        e = -64;
    }
    const uint64_t u = bits_of(x);
    e += (int)((u >> 52) & 0x7ff) - 1023;
    double m = from_bits((u & 0x000fffffffffffffull) | 0x3ff0000000000000ull);  // [1, 2)
    const int i = (int)((u >> 45) & 127);
    if (i >= 53) {
        m *= 0.5;
        e += 1;
    }
    const double c = CRM_LOG_C[i];
    const double r = fma(m, c, -1.0);  // exact: |r| < 2^-7 with c of 8 bits
    TD s = log1p_series(r);
    if (c != 1.0) s = td_add(s, td_of(CRM_LOG_L[i]));
    if (e != 0) {
        const double ed = (double)e;
        double p2, e2, p3, e3;
        two_prod(ed, CRM_LN2[1], p2, e2);
        two_prod(ed, CRM_LN2[2], p3, e3);
        const TD E = renorm(ed * CRM_LN2[0], p2, p3, e2 + (e3 + ed * CRM_LN2[3]));  // e c1 exact
        s = td_add(E, s);
    }
    return s;
}

// ---------------------------------------------------------------------------
CRM_FN double cr_exp(double x)
{
    if (x != x) return x + x;
    if (x > 710.0) return HUGE_VAL;
    if (x < -746.0) return 0.0;
    if (x == 0.0) return 1.0;
    int k;
    const TD y = exp_td(TD{x, 0.0, 0.0}, k);
    return round_scaled(y, k);
}

CRM_FN double cr_log(double x)
{
    if (x != x) return x + x;
    if (x < 0.0) return __builtin_nan("");
    if (x == 0.0) return -HUGE_VAL;
    if (x == HUGE_VAL) return x;
    if (x == 1.0) return 0.0;
    const TD y = log_td(x);
    return rn3(y.h, y.m, y.l);
}

CRM_FN double cr_log1p(double x)
{
    if (x != x) return x + x;
    if (x < -1.0) return __builtin_nan("");
    if (x == -1.0) return -HUGE_VAL;
    if (x == HUGE_VAL) return x;
    if (fabs(x) < 0x1p-54) return x;  // x - x^2/2 rounds to x (also for +-0 and subnormals)
    TD y;
    if (fabs(x) < 0x1p-7) {
        y = log1p_series(x);
    } else {
        double a, b;
        two_sum(1.0, x, a, b);  // 1 + x = a + b exactly
        y = log_td(a);
        if (b != 0.0) {
            // log(a + b) = log(a) + t - t^2/2 + ..., t = b/a, |t| <= 2^-53
            const double t0 = b / a;
            const double t1 = fma(-t0, a, b) / a;
            y = td_add(y, renorm(t0, t1, -0.5 * t0 * t0, 0.0));
        }
    }
    return rn3(y.h, y.m, y.l);
}

CRM_FN bool is_int(double y) { return rint(y) == y; }
CRM_FN bool is_odd_int(double y) { return is_int(y) && fabs(y) < 0x1p53 && (((int64_t)y) & 1) != 0; }

// |x|^y for finite x != 0 and finite y != 0 (the sign is the caller's)
CRM_FN double pow_pos(double ax, double y)
{
    if (ax == 1.0) return 1.0;
    if (y == 1.0) return ax;
    if (y == 2.0) return ax * ax;
    if (y == 0.5) return sqrt(ax);
    if (y == -1.0) return 1.0 / ax;
    const TD t = td_mul_d(log_td(ax), y);
    if (t.h > 710.0) return HUGE_VAL;
    if (t.h < -746.0) return 0.0;
    int k;
    const TD r = exp_td(t, k);
    return round_scaled(r, k);
}

// x^y with the special values of C99 (F.9.4.4)
CRM_FN double cr_pow(double x, double y)
{
    if (y == 0.0) return 1.0;
    if (x == 1.0) return 1.0;
    if (x != x || y != y) return x + y;
    const double ax = fabs(x);
    if (y == HUGE_VAL || y == -HUGE_VAL) {
        if (ax == 1.0) return 1.0;
        return ((ax < 1.0) == (y < 0.0)) ? HUGE_VAL : 0.0;
    }
    const bool odd = is_odd_int(y);
    if (x == 0.0) {
        if (y < 0.0) return odd ? copysign(HUGE_VAL, x) : HUGE_VAL;
        return odd ? x : 0.0;
    }
    if (ax == HUGE_VAL) {
        const double v = y < 0.0 ? 0.0 : HUGE_VAL;
        return (x < 0.0 && odd) ? -v : v;
    }
    if (x < 0.0) {
        if (!is_int(y)) return __builtin_nan("");
        const double v = pow_pos(ax, y);
        return odd ? -v : v;
    }
    return pow_pos(x, y);
}

// u^(1/a) for u >= 0 and a > 0 finite: exp(log(u)/a) with the quotient taken
// in triple-double (no rounding of 1/a)
CRM_FN double cr_powinv(double u, double a)
{
    if (u != u || a != a) return u + a;
    if (u < 0.0 || a <= 0.0) return __builtin_nan("");
    if (u == 0.0 || u == 1.0 || a == 1.0) return u;
    if (u == HUGE_VAL) return u;
    if (a == HUGE_VAL) return 1.0;
    const TD t = td_div_d(log_td(u), a);
    if (t.h > 710.0) return HUGE_VAL;
    if (t.h < -746.0) return 0.0;
    int k;
    const TD r = exp_td(t, k);
    return round_scaled(r, k);
}

#undef CRM_FN

}  // namespace crm
}  // namespace rp
