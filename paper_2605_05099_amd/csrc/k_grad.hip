// k_grad.hip -- implicit-reparameterization backward for gamma and beta.
//
// A draw z = F^{-1}(u; theta) moves with its parameter while u = F(z; theta)
// stays fixed, so dz/dtheta = -(dF/dtheta)(z; theta) / f(z; theta).  The
// kernels evaluate that ratio in binary64 at the binary32 sample and
// parameters (promoted exactly) and return g_theta = g_z * dz/dtheta rounded
// once to binary32.  The normalising constants Gamma(alpha) and B(a, b)
// cancel between numerator and density, so neither is ever formed.
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

// 1/a to full binary64 precision without the correctly rounded division
// sequence: the hardware reciprocal (about 23 good bits) and two Newton
// steps r <- r + r (1 - a r).  a is finite, nonzero and not subnormal here.
RP_HD double rcp(double a)
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

// psi(x), x > 0: for x < 10 shift by ten, psi(x) = psi(x + 10) - sum_{i<10}
// 1/(x + i), the sum formed as one quotient N/D (D = prod (x + i), N
// accumulated alongside) so that every lane runs the same ten multiply-adds
// and one reciprocal; then the asymptotic series ln x - 1/(2x) - sum_k B_2k /
// (2k x^2k) (Bernoulli numbers 1/6, -1/30, 1/42, -1/30, 5/66, -691/2730),
// truncation error below 1e-15 for x >= 10.
RP_HD double digamma(double x)
{
    double num = 0.0, den = 1.0;
#pragma unroll
    for (int i = 0; i < 10; i++) {
        const double t = x + (double)i;
        num = num * t + den;
        den = den * t;
    }
    const bool shift = x < 10.0;
    const double r = shift ? -num * rcp(den) : 0.0;
    x = shift ? x + 10.0 : x;
    const double i1 = rcp(x), i2 = i1 * i1;
    const double s = i2 * (1.0 / 12.0 - i2 * (1.0 / 120.0 - i2 * (1.0 / 252.0 - i2 * (1.0 / 240.0 - i2 * (1.0 / 132.0 - i2 * (691.0 / 32760.0))))));
    return r + log(x) - 0.5 * i1 - s;
}

// value and derivatives with respect to up to two parameters
struct Dual {
    double v, a, b;
};
RP_HD Dual dmul(Dual x, Dual y) { return {x.v * y.v, x.a * y.v + x.v * y.a, x.b * y.v + x.v * y.b}; }
RP_HD Dual dadd(Dual x, Dual y) { return {x.v + y.v, x.a + y.a, x.b + y.b}; }
RP_HD Dual dinv(Dual x)
{
    const double r = rcp(x.v), r2 = -r * r;
    return {r, x.a * r2, x.b * r2};
}
RP_HD Dual dconst(double v) { return {v, 0.0, 0.0}; }

constexpr double kTiny = 1e-300;
// Stopping tolerance 2^-36: the result is rounded to binary32 (relative
// spacing 2^-23), so a relative truncation error of a few times 2^-36, even
// after the slowest geometric tails, stays three orders below the output
// rounding.  Tighter stopping only adds iterations.
constexpr double kEps = 0x1p-36;
constexpr int kMaxIter = 1 << 16;

RP_HD Dual guard(Dual x)
{
    if (fabs(x.v) < kTiny) x.v = kTiny;
    return x;
}

// Gamma(alpha, z) e^z z^{-alpha} and its alpha-derivative (z >= alpha + 1):
// 1/(z+1-alpha -) 1(1-alpha)/(z+3-alpha -) 2(2-alpha)/(z+5-alpha -) ...
RP_HD Dual gamma_cf(double al, double z)
{
    Dual bq = {z + 1.0 - al, -1.0, 0.0};
    Dual c = dconst(1.0 / kTiny);
    Dual d = dinv(bq);
    Dual h = d;
    for (int i = 1; i < kMaxIter; i++) {
        const Dual an = {-(double)i * ((double)i - al), (double)i, 0.0};
        bq.v += 2.0;
        d = guard(dadd(dmul(an, d), bq));
        c = guard(dadd(bq, dmul(an, dinv(c))));
        d = dinv(d);
        const Dual del = dmul(d, c);
        h = dmul(h, del);
        if (fabs(del.v - 1.0) < kEps && fabs(del.a) < kEps * fabs(h.a / h.v) + 1e-18) break;
    }
    return h;
}

RP_HD double gamma_dz_dalpha(double z, double al)
{
    if (!(al > 0.0) || !(z >= 0.0) || z == INFINITY) return NAN;
    if (z == 0.0) return 0.0;
    const double lz = log(z);
    if (z < al + 1.0) {
        double t = rcp(al);
        double psi = digamma(al + 1.0);
        double s = t * (lz - psi), sabs = fabs(s);
        for (int n = 1; n < kMaxIter; n++) {
            const double an = al + (double)n;
            const double ia = rcp(an);
            t = t * z * ia;
            psi = psi + ia;
            const double term = t * (lz - psi);
            s += term;
            sabs += fabs(term);
            if (fabs(term) < kEps * 0.25 * sabs) break;
        }
        return -z * s;
    }
    const Dual h = gamma_cf(al, z);
    return z * (h.v * (lz - digamma(al)) + h.a);
}

// Incomplete-beta continued fraction h(p, q, x) and its derivatives with
// respect to p (.a) and q (.b):
// 1/(1+) d1/(1+) d2/(1+) ...,  d_{2m+1} = -(p+m)(p+q+m) x / ((p+2m)(p+2m+1)),
// d_{2m} = m (q-m) x / ((p+2m-1)(p+2m)).
RP_HD Dual beta_cf(double p, double q, double x)
{
    const Dual P = {p, 1.0, 0.0}, Qd = {q, 0.0, 1.0};
    const Dual one = dconst(1.0);
    Dual c = one;
    // first numerator d_1 = -(p+q) x / (p+1)
    Dual d1 = dmul(dmul(dadd(P, Qd), dconst(-x)), dinv(dadd(P, one)));
    Dual d = dinv(guard(dadd(one, d1)));
    Dual h = d;
    for (int m = 1; m < kMaxIter; m++) {
        const double fm = (double)m, m2 = 2.0 * fm;
        // even step
        Dual num = dmul(dconst(fm * x), dadd(Qd, dconst(-fm)));
        Dual den = dmul(dadd(P, dconst(m2 - 1.0)), dadd(P, dconst(m2)));
        Dual aa = dmul(num, dinv(den));
        d = dinv(guard(dadd(one, dmul(aa, d))));
        c = guard(dadd(one, dmul(aa, dinv(c))));
        h = dmul(h, dmul(d, c));
        // odd step
        num = dmul(dmul(dadd(P, dconst(fm)), dadd(dadd(P, Qd), dconst(fm))), dconst(-x));
        den = dmul(dadd(P, dconst(m2)), dadd(P, dconst(m2 + 1.0)));
        aa = dmul(num, dinv(den));
        d = dinv(guard(dadd(one, dmul(aa, d))));
        c = guard(dadd(one, dmul(aa, dinv(c))));
        const Dual del = dmul(d, c);
        h = dmul(h, del);
        if (fabs(del.v - 1.0) < kEps && fabs(del.a) + fabs(del.b) < kEps * (fabs(h.a) + fabs(h.b)) / fabs(h.v) + 1e-18)
            break;
    }
    return h;
}

RP_HD void beta_dz_dab(double z, double a, double b, double &ga, double &gb)
{
    if (!(a > 0.0) || !(b > 0.0) || !(z >= 0.0) || !(z <= 1.0)) {
        ga = gb = NAN;
        return;
    }
    if (z == 0.0 || z == 1.0) {
        ga = gb = 0.0;
        return;
    }
    const double lz = log(z), l1z = log1p(-z);
    const double pab = digamma(a + b), pa = digamma(a), pb = digamma(b);
    const double w = z * (1.0 - z);
    // one continued fraction for both sides of the symmetry switch (a
    // wavefront mixing the two then runs a single loop), arguments swapped
    // on the upper side: h(b, a, 1 - z) with .a = d/db and .b = d/da
    const bool lower = z < (a + 1.0) / (a + b + 2.0);
    const Dual h = beta_cf(lower ? a : b, lower ? b : a, lower ? z : 1.0 - z);
    if (lower) {
        ga = -(w / a) * (h.v * (lz - 1.0 / a - pa + pab) + h.a);
        gb = -(w / a) * (h.v * (l1z - pb + pab) + h.b);
    } else {
        ga = (w / b) * (h.v * (lz - pa + pab) + h.b);
        gb = (w / b) * (h.v * (l1z - 1.0 / b - pb + pab) + h.a);
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
    __shared__ uint16_t s_perm[TILE];
    __shared__ uint32_t s_cnt[64];
    const int tid = threadIdx.x;
    for (uint64_t base = (uint64_t)blockIdx.x * TILE; base < n; base += (uint64_t)gridDim.x * TILE) {
        const int cnt = (int)((n - base) < (uint64_t)TILE ? (n - base) : (uint64_t)TILE);
        if (tid < 64) s_cnt[tid] = 0;
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
#pragma unroll 1
        for (int k = 0; k < K; k++) {
            const int q = k * kGradBlock + tid;
            if (q < cnt) {
                const int e = s_perm[q];
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
