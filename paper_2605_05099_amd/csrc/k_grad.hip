// k_grad.hip -- implicit-reparameterization backward for gamma and beta.
//
// A draw z = F^{-1}(u; theta) moves with its parameter while u = F(z; theta)
// stays fixed, so dz/dtheta = -(dF/dtheta)(z; theta) / f(z; theta).  The
// kernels evaluate that ratio in binary32 at the binary32 sample and
// parameters, with an estimate of the rounding error; elements whose
// estimate is too large are evaluated again in binary64 (parameters
// promoted exactly).  g_theta = g_z * dz/dtheta is rounded once to binary32.
// The normalising constants Gamma(alpha) and B(a, b) cancel between
// numerator and density, so neither is ever formed.
//
// Gamma(alpha, 1), P = regularized lower incomplete gamma, Q = 1 - P:
//   z < alpha + 1: P = e^{-z} sum_n z^{alpha+n} / Gamma(alpha+n+1), so
//       dz/dalpha = -z sum_n t_n (ln z - psi(alpha+n+1)),
//       t_0 = 1/alpha, t_n = t_{n-1} z / (alpha+n);
//   z >= alpha + 1: Gamma(alpha, z) = e^{-z} z^alpha h(alpha, z) with h the
//       Legendre continued fraction, so dz/dalpha = z (h (ln z - psi(alpha)) + dh/dalpha);
//       h and dh/dalpha come from one modified-Lentz pass in forward-mode
//       dual numbers.
// Beta(a, b), I = regularized incomplete beta:
//   z < (a+1)/(a+b+2): I = z^a (1-z)^b h(a, b, z) / (a B(a, b)), h the
//       incomplete-beta continued fraction; otherwise I = 1 - I_{1-z}(b, a).
//       Differentiating the logarithm of the prefactor gives the psi terms
//       below; dh/da, dh/db again come from dual numbers.
// z = 0 (and z = 1 for beta) give 0, the limit of the formulas; a parameter
// that is not > 0, or a sample outside the support, gives NaN.
#include <hip/hip_runtime.h>

#include "rp_internal.h"

namespace rp {

namespace {

// Arithmetic of one precision.  R = double: the reference evaluation (1/a
// from the hardware reciprocal and two Newton steps, about full binary64
// precision; the platform log).  R = float: the bulk evaluation (hardware
// reciprocal and logarithm, about an ulp each; log(1 - x) by log(u) x /
// (1 - u), u = 1 - x, which keeps its relative accuracy for small x).
template <class R>
struct Ar;
template <>
struct Ar<double> {
    static constexpr double kTiny = 1e-300;
    // stopping tolerance 2^-36: the result is rounded to binary32 (relative
    // spacing 2^-23), so a truncation error of a few times 2^-36, even after
    // the slowest geometric tails, stays three orders below that rounding
    static constexpr double kEps = 0x1p-36;
    static RP_HD double rcp(double a)
    {
#if defined(__HIP_DEVICE_COMPILE__)
        double r = __builtin_amdgcn_rcp(a);
        double e = __fma_rn(-a, r, 1.0);
        r = __fma_rn(r, e, r);
        e = __fma_rn(-a, r, 1.0);
        return __fma_rn(r, e, r);
#else
        return 1.0 / a;
#endif
    }
    static constexpr int kMaxIter = 1 << 16;
    static constexpr bool kNoise = false;  // derivative stopping test without a noise floor
    static RP_HD double lg(double x) { return log(x); }
    static RP_HD double lg1m(double x) { return log1p(-x); }
    static RP_HD double div(double x, double y) { return x / y; }
};
template <>
struct Ar<float> {
    static constexpr float kTiny = 1e-30f;
    // truncation below 2^-21 relative, a few binary32 ulps: the factors of
    // the continued fractions settle within an ulp or two of 1 (the
    // hardware reciprocal is exact to an ulp), never closer
    static constexpr float kEps = 0x1p-21f;
    static constexpr int kMaxIter = 4096;  // not converged: binary64 instead
    static constexpr bool kNoise = true;
    static RP_HD float rcp(float a)
    {
#if defined(__HIP_DEVICE_COMPILE__)
        return __builtin_amdgcn_rcpf(a);
#else
        return 1.0f / a;
#endif
    }
    static RP_HD float lg(float x)
    {
#if defined(__HIP_DEVICE_COMPILE__)
        return __builtin_amdgcn_logf(x) * 0x1.62e430p-1f;
#else
        return logf(x);
#endif
    }
    static RP_HD float div(float x, float y) { return x * rcp(y); }
    static RP_HD float lg1m(float x)
    {
        const float u = 1.0f - x;
        if (u == 1.0f) return -x;
        return lg(u) * div(x, 1.0f - u);
    }
};

// psi(x), x > 0: for x < 10 shift by ten, psi(x) = psi(x + 10) - sum_{i<10}
// 1/(x + i), the sum formed as one quotient N/D (D = prod (x + i), N
// accumulated alongside) so that every lane runs the same ten multiply-adds
// and one reciprocal; then the asymptotic series ln x - 1/(2x) - sum_k B_2k /
// (2k x^2k) (Bernoulli numbers 1/6, -1/30, 1/42, -1/30, 5/66, -691/2730),
// truncation error below 1e-15 for x >= 10.
template <class R>
RP_HD R digamma(R x)
{
    R num = 0, den = 1;
#pragma unroll
    for (int i = 0; i < 10; i++) {
        const R t = x + (R)i;
        num = num * t + den;
        den = den * t;
    }
    const bool shift = x < (R)10;
    const R r = shift ? -num * Ar<R>::rcp(den) : (R)0;
    x = shift ? x + (R)10 : x;
    const R i1 = Ar<R>::rcp(x), i2 = i1 * i1;
    const R s = i2 * ((R)(1.0 / 12.0) - i2 * ((R)(1.0 / 120.0) - i2 * ((R)(1.0 / 252.0) - i2 * ((R)(1.0 / 240.0) - i2 * ((R)(1.0 / 132.0) - i2 * (R)(691.0 / 32760.0))))));
    return r + Ar<R>::lg(x) - (R)0.5 * i1 - s;
}

// psi(x + y) - psi(x) for x, y > 0 without the cancellation of the two
// values: for x < 10 shift by ten, the difference gaining the positive
// terms y / ((x + i)(x + y + i)), i < 10; for x >= 10 the difference of
// the asymptotic series, its leading term log1p(y / x).
template <class R>
RP_HD R digamma_diff(R x, R y)
{
    R acc = 0;
    if (x < (R)10) {
#pragma unroll
        for (int i = 0; i < 10; i++) acc += Ar<R>::div(y, (x + (R)i) * (x + y + (R)i));
        x = x + (R)10;
    }
    const R q = Ar<R>::div(y, x);
    const R l = Ar<R>::lg1m(-q);  // log1p(q) = log(1 - (-q))
    const R u = x + y;
    const R i1 = Ar<R>::rcp(x), j1 = Ar<R>::rcp(u);
    const R i2 = i1 * i1, j2 = j1 * j1;
    // (1/(2x) - 1/(2u)) = y / (2 x u)
    const R half = Ar<R>::div(y, (R)2 * x * u);
    auto ser = [](R t2) {
        return t2 * ((R)(1.0 / 12.0) - t2 * ((R)(1.0 / 120.0) - t2 * ((R)(1.0 / 252.0) - t2 * ((R)(1.0 / 240.0) - t2 * ((R)(1.0 / 132.0) - t2 * (R)(691.0 / 32760.0))))));
    };
    return acc + l + half - (ser(j2) - ser(i2));
}

// value and derivatives with respect to up to two parameters
template <class R>
struct Dual {
    R v, a, b;
};
template <class R>
RP_HD Dual<R> dmul(Dual<R> x, Dual<R> y)
{
    return {x.v * y.v, x.a * y.v + x.v * y.a, x.b * y.v + x.v * y.b};
}
template <class R>
RP_HD Dual<R> dadd(Dual<R> x, Dual<R> y)
{
    return {x.v + y.v, x.a + y.a, x.b + y.b};
}
template <class R>
RP_HD Dual<R> dinv(Dual<R> x)
{
    const R r = Ar<R>::rcp(x.v), r2 = -r * r;
    return {r, x.a * r2, x.b * r2};
}
template <class R>
RP_HD Dual<R> dconst(R v)
{
    return {v, (R)0, (R)0};
}

template <class R>
RP_HD Dual<R> guard(Dual<R> x)
{
    if (fabs(x.v) < Ar<R>::kTiny) x.v = Ar<R>::kTiny;
    return x;
}

// Gamma(alpha, z) e^z z^{-alpha} and its alpha-derivative (z >= alpha + 1):
// 1/(z+1-alpha -) 1(1-alpha)/(z+3-alpha -) 2(2-alpha)/(z+5-alpha -) ...
// iters: the steps taken.
template <class R>
RP_HD Dual<R> gamma_cf(R al, R z, int &iters)
{
    Dual<R> bq = {z + (R)1 - al, (R)-1, (R)0};
    Dual<R> c = dconst((R)1 / Ar<R>::kTiny);
    Dual<R> d = dinv(bq);
    Dual<R> h = d;
    int i = 1;
    for (; i < Ar<R>::kMaxIter; i++) {
        const Dual<R> an = {-(R)i * ((R)i - al), (R)i, (R)0};
        bq.v += (R)2;
        d = guard(dadd(dmul(an, d), bq));
        c = guard(dadd(bq, dmul(an, dinv(c))));
        d = dinv(d);
        const Dual<R> del = dmul(d, c);
        h = dmul(h, del);
        // binary32: del.a settles at the rounding level of its two products
        const R floor = Ar<R>::kNoise ? fabs(d.a * c.v) + fabs(d.v * c.a) : (R)0;
        if (fabs(del.v - (R)1) < Ar<R>::kEps && fabs(del.a) < Ar<R>::kEps * (fabs(h.a / h.v) + floor) + (R)1e-18) break;
    }
    iters = i;
    return h;
}

// dz/dalpha for Gamma(alpha, 1).  cond (when not null) receives an estimate
// of the result's relative rounding error in units of the precision's
// epsilon: the magnitudes that cancel in the result times the operations
// their errors pass through.
template <class R>
RP_HD R gamma_dz_dalpha(R z, R al, R *cond = nullptr)
{
    if (cond) *cond = (R)0;
    if (!(al > (R)0) || !(z >= (R)0) || z == (R)INFINITY) return (R)NAN;
    if (z == (R)0) return (R)0;
    const R lz = Ar<R>::lg(z);
    if (z < al + (R)1) {
        R t = Ar<R>::rcp(al);
        R psi = digamma(al + (R)1);
        R s = t * (lz - psi), sabs = fabs(s), mag = fabs(t) * (fabs(lz) + fabs(psi));
        int n = 1;
        for (; n < Ar<R>::kMaxIter; n++) {
            const R an = al + (R)n;
            const R ia = Ar<R>::rcp(an);
            t = t * z * ia;
            psi = psi + ia;
            const R term = t * (lz - psi);
            s += term;
            sabs += fabs(term);
            mag += fabs(t) * (fabs(lz) + fabs(psi));
            if (fabs(term) < Ar<R>::kEps * (R)0.25 * sabs) break;
        }
        if (cond) *cond = n < Ar<R>::kMaxIter ? mag * (R)(n + 16) / fabs(s) : (R)INFINITY;
        return -z * s;
    }
    int iters;
    const Dual<R> h = gamma_cf(al, z, iters);
    const R pa = digamma(al);
    const R r = h.v * (lz - pa) + h.a;
    if (cond)
        *cond = iters < Ar<R>::kMaxIter ? (fabs(h.v) * (fabs(lz) + fabs(pa)) + fabs(h.a)) * (R)(iters + 16) / fabs(r)
                                        : (R)INFINITY;
    return z * r;
}

// Incomplete-beta continued fraction h(p, q, x) and its derivatives with
// respect to p (.a) and q (.b):
// 1/(1+) d1/(1+) d2/(1+) ...,  d_{2m+1} = -(p+m)(p+q+m) x / ((p+2m)(p+2m+1)),
// d_{2m} = m (q-m) x / ((p+2m-1)(p+2m)).
template <class R>
RP_HD Dual<R> beta_cf(R p, R q, R x, int &iters)
{
    const Dual<R> P = {p, (R)1, (R)0}, Qd = {q, (R)0, (R)1};
    const Dual<R> one = dconst((R)1);
    Dual<R> c = one;
    // first numerator d_1 = -(p+q) x / (p+1)
    Dual<R> d1 = dmul(dmul(dadd(P, Qd), dconst(-x)), dinv(dadd(P, one)));
    Dual<R> d = dinv(guard(dadd(one, d1)));
    Dual<R> h = d;
    int m = 1;
    for (; m < Ar<R>::kMaxIter; m++) {
        const R fm = (R)m, m2 = (R)2 * fm;
        // even step
        Dual<R> num = dmul(dconst(fm * x), dadd(Qd, dconst(-fm)));
        Dual<R> den = dmul(dadd(P, dconst(m2 - (R)1)), dadd(P, dconst(m2)));
        Dual<R> aa = dmul(num, dinv(den));
        d = dinv(guard(dadd(one, dmul(aa, d))));
        c = guard(dadd(one, dmul(aa, dinv(c))));
        h = dmul(h, dmul(d, c));
        // odd step
        num = dmul(dmul(dadd(P, dconst(fm)), dadd(dadd(P, Qd), dconst(fm))), dconst(-x));
        den = dmul(dadd(P, dconst(m2)), dadd(P, dconst(m2 + (R)1)));
        aa = dmul(num, dinv(den));
        d = dinv(guard(dadd(one, dmul(aa, d))));
        c = guard(dadd(one, dmul(aa, dinv(c))));
        const Dual<R> del = dmul(d, c);
        h = dmul(h, del);
        const R floor = Ar<R>::kNoise ? fabs(d.a * c.v) + fabs(d.v * c.a) + fabs(d.b * c.v) + fabs(d.v * c.b) : (R)0;
        if (fabs(del.v - (R)1) < Ar<R>::kEps &&
            fabs(del.a) + fabs(del.b) < Ar<R>::kEps * ((fabs(h.a) + fabs(h.b)) / fabs(h.v) + floor) + (R)1e-18)
            break;
    }
    iters = m;
    return h;
}

// dz/da, dz/db for Beta(a, b); cond as for gamma_dz_dalpha (the larger of
// the two results' estimates)
template <class R>
RP_HD void beta_dz_dab(R z, R a, R b, R &ga, R &gb, R *cond = nullptr)
{
    if (cond) *cond = (R)0;
    if (!(a > (R)0) || !(b > (R)0) || !(z >= (R)0) || !(z <= (R)1)) {
        ga = gb = (R)NAN;
        return;
    }
    if (z == (R)0 || z == (R)1) {
        ga = gb = (R)0;
        return;
    }
    const R lz = Ar<R>::lg(z), l1z = Ar<R>::lg1m(z);
    const R w = z * ((R)1 - z);
    // one continued fraction for both sides of the symmetry switch (a
    // wavefront mixing the two then runs a single loop), arguments swapped
    // on the upper side: h(b, a, 1 - z) with .a = d/db and .b = d/da
    const bool lower = z < Ar<R>::div(a + (R)1, a + b + (R)2);
    int iters;
    const Dual<R> h = beta_cf(lower ? a : b, lower ? b : a, lower ? z : (R)1 - z, iters);
    // the digamma combinations as differences (psi(s) + 1/s = psi(s + 1)):
    //   psi(a+b) - psi(a+1), psi(a+b) - psi(b), psi(a+b) - psi(a), psi(a+b) - psi(b+1)
    auto dd = [](R x, R t) { return t >= x ? digamma_diff(x, t - x) : -digamma_diff(t, x - t); };
    const R ab = a + b;
    R ra, rb, ma, mb, da, db;
    if (lower) {
        da = dd(a + (R)1, ab);
        db = digamma_diff(b, a);
        ra = h.v * (lz + da) + h.a;
        rb = h.v * (l1z + db) + h.b;
        ma = fabs(h.v) * (fabs(lz) + fabs(da)) + fabs(h.a);
        mb = fabs(h.v) * (fabs(l1z) + fabs(db)) + fabs(h.b);
        const R f = Ar<R>::div(w, a);
        ga = -f * ra;
        gb = -f * rb;
    } else {
        da = digamma_diff(a, b);
        db = dd(b + (R)1, ab);
        ra = h.v * (lz + da) + h.b;
        rb = h.v * (l1z + db) + h.a;
        ma = fabs(h.v) * (fabs(lz) + fabs(da)) + fabs(h.b);
        mb = fabs(h.v) * (fabs(l1z) + fabs(db)) + fabs(h.a);
        const R f = Ar<R>::div(w, b);
        ga = f * ra;
        gb = f * rb;
    }
    if (cond) {
        const R ca = ma / fabs(ra), cb = mb / fabs(rb);
        *cond = iters < Ar<R>::kMaxIter ? (ca > cb ? ca : cb) * (R)(2 * iters + 16) : (R)INFINITY;
    }
}

// ---------------------------------------------------------------------------
// Work keys.  The cost of an element is the length of its series or
// continued fraction, which varies by more than an order of magnitude over
// the parameter range; a wavefront runs as long as its slowest lane.  Each
// block therefore loads a tile of elements, orders it by a 6-bit key that
// predicts the loop length, and gives every wavefront 64 consecutive
// elements in that order.  The key only changes which lanes evaluate which
// elements together, never a result.

// Gamma: the series (z < alpha + 1) needs about n terms where the term ratio
// product falls below 2^-38, n ln((alpha + n/2) / z) = 26, solved by a few
// fixed-point steps; the continued fraction (z >= alpha + 1 > 1) converges
// more slowly the smaller z is.
// a / b from the hardware reciprocal: keys need no correctly rounded quotient
__device__ __forceinline__ float qdiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }

__device__ __forceinline__ int gamma_key(float zf, float af)
{
    if (!(af > 0.f) || !(zf > 0.f) || !(zf < INFINITY)) return 0;
    if (zf < af + 1.f) {
        float nn = 8.f;
#pragma unroll
        for (int k = 0; k < 4; k++) nn = fminf(qdiv(26.f, fmaxf(__logf(qdiv(af + 0.5f * nn, zf)), 1e-3f)), 4096.f);
        return min(31, (int)(4.f * __log2f(nn + 1.f)));
    }
    return 32 + min(31, max(0, (int)(4.f * __log2f(zf))));
}

// Beta: after the symmetry switch the continued fraction runs at x < (p+1) /
// (p+q+2).  Its partial numerators tend to -x/4, and with them the error
// ratio per step to rho(x) = (1 - sqrt(1-x)) / (1 + sqrt(1-x)); the first
// numerator is about r = x (p+q+2) / (p+1), so the pair count is predicted
// from rho(r): ln(2^-36) / (2 ln rho).
__device__ __forceinline__ int beta_key(float zf, float af, float bf)
{
    if (!(af > 0.f) || !(bf > 0.f) || !(zf > 0.f) || !(zf < 1.f)) return 0;
    const bool sw = !(zf < qdiv(af + 1.f, af + bf + 2.f));
    const float p = sw ? bf : af, q = sw ? af : bf, x = sw ? 1.f - zf : zf;
    const float r = fminf(qdiv(x * (p + q + 2.f), p + 1.f), 0.999999f);
    const float sq = sqrtf(1.f - r);
    const float rho = qdiv(1.f - sq, 1.f + sq);
    const float nn = 1.f + qdiv(12.5f, fmaxf(-__logf(fmaxf(rho, 1e-30f)), 1e-6f));
    return min(63, max(0, (int)(8.f * __log2f(nn))));
}

constexpr int kGradBlock = 256;

// The per-element evaluations out of line, so the tile bookkeeping and the
// series/continued-fraction loops do not share one register allocation.
struct D2 {
    double a, b;
};
__device__ __noinline__ double gamma_elem(double z, double al) { return gamma_dz_dalpha(z, al); }
__device__ __forceinline__ D2 beta_elem(double z, double a, double b)
{
    D2 r;
    beta_dz_dab(z, a, b, r.a, r.b);
    return r;
}

// The binary32 bulk: the same formulas in binary32 (hardware reciprocal and
// logarithm), accepted when the estimate of its rounding error (cond, in
// units of 2^-24) is at most kCond; the others are evaluated again in
// binary64.  On the [4096, 1024] workload the accepted binary32 results are
// within 5e-6 (gamma) and 8e-6 (beta) relative of the binary64 ones, and
// about 1 % (gamma) and 6 % (beta) of the elements take binary64.
constexpr float kCondGamma = 3000.f, kCondBeta = 300.f;
constexpr int kFbCap = 256;  // binary64 list of a tile (LDS); more go at once
struct F2 {
    float a, b;
    bool ok;
};
// This file is built with binary32 subnormals flushed to zero: a subnormal
// input, or a result below 2^-100 in magnitude (whose terms could have
// underflowed), goes to binary64.
constexpr float kF32Small = 0x1p-100f;
__device__ __forceinline__ bool subnormal(float x)
{
    const uint32_t u = __float_as_uint(x) & 0x7fffffffu;
    return u != 0u && u < 0x00800000u;
}
__device__ __noinline__ F2 gamma_elem32(float z, float al)
{
    if (subnormal(z) || subnormal(al)) return {0.f, 0.f, false};
    float c;
    const float r = gamma_dz_dalpha<float>(z, al, &c);
    return {r, 0.f, c <= kCondGamma && !(fabsf(r) < kF32Small && r != 0.f)};
}
__device__ __noinline__ F2 beta_elem32(float z, float a, float b)
{
    if (subnormal(z) || subnormal(a) || subnormal(b)) return {0.f, 0.f, false};
    F2 r;
    float c;
    beta_dz_dab<float>(z, a, b, r.a, r.b, &c);
    r.ok = c <= kCondBeta && !(fabsf(r.a) < kF32Small && r.a != 0.f) && !(fabsf(r.b) < kF32Small && r.b != 0.f);
    return r;
}

// One tile of TILE elements per iteration: coalesced loads into LDS, a
// counting sort of the element indices by key, evaluation in key order
// (results back into LDS at the element's own slot), coalesced stores.
// Inputs are read in full before any output of the tile is written, so the
// outputs may alias the inputs.
template <bool BETA, int TILE>
__global__ __launch_bounds__(kGradBlock, BETA ? 4 : 5) void k_grad_sorted(const float *z, const float *pa, const float *pb,
                                                            const float *gz, float *ga, float *gb, uint64_t n)
{
    constexpr int K = TILE / kGradBlock;
    __shared__ float s_z[TILE], s_a[TILE], s_b[BETA ? TILE : 1], s_g[TILE];
    __shared__ uint16_t s_perm[TILE], s_fb[kFbCap];
    __shared__ uint32_t s_cnt[64], s_nfb;
    const int tid = threadIdx.x;
    for (uint64_t base = (uint64_t)blockIdx.x * TILE; base < n; base += (uint64_t)gridDim.x * TILE) {
        const int cnt = (int)((n - base) < (uint64_t)TILE ? (n - base) : (uint64_t)TILE);
        if (tid < 64) s_cnt[tid] = 0;
        if (tid == 0) s_nfb = 0;
        __syncthreads();
        float zf[K], af[K], bf[K], gf[K];
        if (cnt == TILE) {  // all loads of a full tile in flight together
#pragma unroll
            for (int k = 0; k < K; k++) {
                const uint64_t i = base + k * kGradBlock + tid;
                zf[k] = z[i];
                af[k] = pa[i];
                bf[k] = BETA ? pb[i] : 0.f;
                gf[k] = gz[i];
            }
        } else {
#pragma unroll
            for (int k = 0; k < K; k++) {
                const int e = k * kGradBlock + tid;
                const uint64_t i = base + (e < cnt ? e : 0);
                zf[k] = z[i];
                af[k] = pa[i];
                bf[k] = BETA ? pb[i] : 0.f;
                gf[k] = gz[i];
            }
        }
        int key[K];
        uint32_t rank[K];
#pragma unroll
        for (int k = 0; k < K; k++) {
            const int e = k * kGradBlock + tid;
            if (e < cnt) {
                s_z[e] = zf[k];
                s_a[e] = af[k];
                if (BETA) s_b[e] = bf[k];
                s_g[e] = gf[k];
                key[k] = BETA ? beta_key(zf[k], af[k], bf[k]) : gamma_key(zf[k], af[k]);
                rank[k] = atomicAdd(&s_cnt[key[k]], 1u);
            }
        }
        __syncthreads();
        if (tid < 64) {  // exclusive scan of the 64 bucket sizes (one wavefront)
            const uint32_t c = s_cnt[tid];
            uint32_t v = c;
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const uint32_t u = __shfl_up(v, d, 64);
                if (tid >= d) v += u;
            }
            s_cnt[tid] = v - c;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < K; k++) {
            const int e = k * kGradBlock + tid;
            if (e < cnt) s_perm[s_cnt[key[k]] + rank[k]] = (uint16_t)e;
        }
        __syncthreads();
        // binary32 pass in key order; elements whose error estimate is too
        // large are listed for the binary64 pass
#pragma unroll 1
        for (int k = 0; k < K; k++) {
            const int q = k * kGradBlock + tid;
            if (q < cnt) {
                const int e = s_perm[q];
                const F2 d = BETA ? beta_elem32(s_z[e], s_a[e], s_b[e]) : gamma_elem32(s_z[e], s_a[e]);
                if (d.ok) {
                    const double g = (double)s_g[e];
                    s_a[e] = (float)(g * (double)d.a);
                    if (BETA) s_b[e] = (float)(g * (double)d.b);
                } else {
                    const uint32_t slot = atomicAdd(&s_nfb, 1u);
                    if (slot < (uint32_t)kFbCap) {
                        s_fb[slot] = (uint16_t)e;
                    } else {  // list full (not met on the workload): at once
                        const double g = (double)s_g[e];
                        if (BETA) {
                            const D2 dd = beta_elem((double)s_z[e], (double)s_a[e], (double)s_b[e]);
                            s_a[e] = (float)(g * dd.a);
                            s_b[e] = (float)(g * dd.b);
                        } else {
                            s_a[e] = (float)(g * gamma_elem((double)s_z[e], (double)s_a[e]));
                        }
                    }
                }
            }
        }
        __syncthreads();
        const int nfb = (int)(s_nfb < (uint32_t)kFbCap ? s_nfb : (uint32_t)kFbCap);
#pragma unroll 1
        for (int q = tid; q < nfb; q += kGradBlock) {
            const int e = s_fb[q];
            const double g = (double)s_g[e];
            if (BETA) {
                const D2 d = beta_elem((double)s_z[e], (double)s_a[e], (double)s_b[e]);
                s_a[e] = (float)(g * d.a);
                s_b[e] = (float)(g * d.b);
            } else {
                const double d = gamma_elem((double)s_z[e], (double)s_a[e]);
                s_a[e] = (float)(g * d);
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < K; k++) {
            const int e = k * kGradBlock + tid;
            if (e < cnt) {
                ga[base + e] = s_a[e];
                if (BETA) gb[base + e] = s_b[e];
            }
        }
        __syncthreads();
    }
}

constexpr int kGammaTile = 2048, kBetaTile = 1024;

unsigned grid_for(uint64_t n, int tile)
{
    const uint64_t b = (n + tile - 1) / tile;
    return (unsigned)(b < 4096 ? b : 4096);
}
bool aligned4(const void *p) { return ((uintptr_t)p & 3) == 0; }

}  // namespace

}  // namespace rp

using namespace rp;

extern "C" int rp_gamma_grad(const float *d_z, const float *d_alpha, const float *d_gz, float *d_galpha, uint64_t n,
                             void *hip_stream)
{
    if (n == 0) return RP_OK;
    if (!d_z || !d_alpha || !d_gz || !d_galpha) return fail(RP_ENULL, "rp_gamma_grad: NULL device pointer");
    if (!aligned4(d_z) || !aligned4(d_alpha) || !aligned4(d_gz) || !aligned4(d_galpha))
        return fail(RP_EINVAL, "rp_gamma_grad: pointers not aligned to 4 bytes");
    hipLaunchKernelGGL((k_grad_sorted<false, kGammaTile>), dim3(grid_for(n, kGammaTile)), dim3(kGradBlock), 0,
                       (hipStream_t)hip_stream, d_z, d_alpha, (const float *)nullptr, d_gz, d_galpha, (float *)nullptr, n);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? RP_OK : fail(RP_EDEVICE, "rp_gamma_grad launch: %s", hipGetErrorString(e));
}

extern "C" int rp_gamma_grad_host(const float *z, const float *alpha, const float *gz, float *galpha, uint64_t n)
{
    if (n == 0) return RP_OK;
    if (!z || !alpha || !gz || !galpha) return fail(RP_ENULL, "rp_gamma_grad_host: NULL pointer");
    for (uint64_t i = 0; i < n; i++)
        galpha[i] = (float)((double)gz[i] * gamma_dz_dalpha<double>((double)z[i], (double)alpha[i]));
    return RP_OK;
}

extern "C" int rp_beta_grad_host(const float *z, const float *a, const float *b, const float *gz, float *ga, float *gb,
                                 uint64_t n)
{
    if (n == 0) return RP_OK;
    if (!z || !a || !b || !gz || !ga || !gb) return fail(RP_ENULL, "rp_beta_grad_host: NULL pointer");
    for (uint64_t i = 0; i < n; i++) {
        double da, db;
        beta_dz_dab<double>((double)z[i], (double)a[i], (double)b[i], da, db);
        ga[i] = (float)((double)gz[i] * da);
        gb[i] = (float)((double)gz[i] * db);
    }
    return RP_OK;
}

extern "C" int rp_beta_grad(const float *d_z, const float *d_a, const float *d_b, const float *d_gz, float *d_ga,
                            float *d_gb, uint64_t n, void *hip_stream)
{
    if (n == 0) return RP_OK;
    if (!d_z || !d_a || !d_b || !d_gz || !d_ga || !d_gb) return fail(RP_ENULL, "rp_beta_grad: NULL device pointer");
    if (!aligned4(d_z) || !aligned4(d_a) || !aligned4(d_b) || !aligned4(d_gz) || !aligned4(d_ga) || !aligned4(d_gb))
        return fail(RP_EINVAL, "rp_beta_grad: pointers not aligned to 4 bytes");
    hipLaunchKernelGGL((k_grad_sorted<true, kBetaTile>), dim3(grid_for(n, kBetaTile)), dim3(kGradBlock), 0,
                       (hipStream_t)hip_stream, d_z, d_a, d_b, d_gz, d_ga, d_gb, n);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? RP_OK : fail(RP_EDEVICE, "rp_beta_grad launch: %s", hipGetErrorString(e));
}
