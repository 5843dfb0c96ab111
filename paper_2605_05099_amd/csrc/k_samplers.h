// k_samplers.h -- lane-per-substream samplers: fused moments, gamma, beta.
// Included by fill.hip (one translation unit shares the constant tables).
//
// Each lane runs the serial definition of its substream: normals by the
// ziggurat (zig_serial), uniforms from the top 53 bits, Marsaglia-Tsang gamma
// (Section 3.1, "Gamma and related distributions") with the shape < 1 boost,
// beta as X / (X + Y).  Floating point is evaluated exactly as written
// (-ffp-contract=off), so the decisions and values match the serial
// definition; only log/exp may differ from another library by an ulp.
#pragma once

// ---------------------------------------------------------------------------
// serial word streams for the counter / LCG engines (lane-per-substream use)
struct LanePhilox32 {
    uint64_t clo, chi, key, b0, b1;
    uint32_t ph;
    bool have;
    __device__ void load(const FillArgs &a, uint64_t i)
    {
        clo = a.words[i];
        chi = a.words[a.n + i];
        key = a.words[2 * a.n + i];
        ph = a.phase[i];
        have = false;
    }
    __device__ uint64_t next()
    {
        if (!have) {
            philox4x32(clo, chi, key, b0, b1);
            have = true;
        }
        const uint64_t w = ph ? b1 : b0;
        if (++ph == 2) {
            ph = 0;
            clo += 1;
            chi += (clo == 0) ? 1u : 0u;
            have = false;
        }
        return w;
    }
    __device__ void store(const FillArgs &a, uint64_t i) const
    {
        a.words[i] = clo;
        a.words[a.n + i] = chi;
        a.phase[i] = ph;
    }
};

struct LanePhilox64 {
    uint64_t c[4], k0, k1, b[4];
    uint32_t ph;
    bool have;
    __device__ void load(const FillArgs &a, uint64_t i)
    {
#pragma unroll
        for (int k = 0; k < 4; k++) c[k] = a.words[(uint64_t)k * a.n + i];
        k0 = a.words[4 * a.n + i];
        k1 = a.words[5 * a.n + i];
        ph = a.phase[i];
        have = false;
    }
    __device__ uint64_t next()
    {
        if (!have) {
            philox4x64(c, k0, k1, b);
            have = true;
        }
        uint64_t w = b[0];
        w = (ph == 1) ? b[1] : w;
        w = (ph == 2) ? b[2] : w;
        w = (ph == 3) ? b[3] : w;
        if (++ph == 4) {
            ph = 0;
            uint64_t carry = 1;
#pragma unroll
            for (int k = 0; k < 4; k++) {
                c[k] += carry;
                carry = (carry && c[k] == 0) ? 1u : 0u;
            }
            have = false;
        }
        return w;
    }
    __device__ void store(const FillArgs &a, uint64_t i) const
    {
#pragma unroll
        for (int k = 0; k < 4; k++) a.words[(uint64_t)k * a.n + i] = c[k];
        a.phase[i] = ph;
    }
};

struct LanePcg {
    u128 s, inc;
    __device__ void load(const FillArgs &a, uint64_t i)
    {
        s = u128{a.words[i], a.words[a.n + i]};
        inc = u128{a.words[2 * a.n + i], a.words[3 * a.n + i]};
    }
    __device__ uint64_t next()
    {
        const uint64_t w = pcg_dxsm(s);
        s = pcg_step(s, inc);
        return w;
    }
    __device__ void store(const FillArgs &a, uint64_t i) const
    {
        a.words[i] = s.lo;
        a.words[a.n + i] = s.hi;
    }
};

// ---------------------------------------------------------------------------
// U^(1/a) for the gamma boost (a < 1), U = k 2^-53.  log U is formed to about
// 2^-70 absolute with the table log: U = 2^e m, m in [1, 2), c = table point
// near m, log U = e ln2 + log c + log1p((m - c)/c); then t = log(U)/a as a
// pair of doubles and the result exp(t_hi) (1 + t_lo).  Its error is about an
// ulp whatever the size of |t|, where a plain exp(log(U)/a) would lose
// |t| ulps.
__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e)
{
    s = a + b;
    const double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

__device__ double boost_pow(double u, double a)
{
    if (u == 0.0) return 0.0;
    int ex;
    double m = frexp(u, &ex);  // u = m 2^ex, m in [0.5, 1)
    m = m * 2.0;
    ex -= 1;
    const int i = (int)(((uint64_t)__double_as_longlong(m) >> 44) & 0xff);
    const double c = RP_LOG_C[i], ic = RP_LOG_INV[i];
    const double num = m - c;  // exact: m and c are within a factor of 2
    const double rh = num * ic;
    const double rl = __fma_rn(-rh, c, num) * ic;
    const double p = (rh * rh) * (-0.5 + rh * (1.0 / 3.0 + rh * (-0.25 + rh * (0.2 + rh * (-1.0 / 6.0 + rh * (1.0 / 7.0))))));
    double sh, sl, t;
    two_sum((double)ex * RP_LN2_HI, RP_LOG_HI[i], sh, sl);
    two_sum(sh, rh, sh, t);
    sl = sl + t + (((double)ex * RP_LN2_LO + RP_LOG_LO[i]) + (rl + p));
    const double lh = sh + sl;
    const double ll = sl - (lh - sh);
    const double th = lh / a;
    const double tl = (__fma_rn(-th, a, lh) + ll) / a;
    const double eh = exp(th);
    if (eh == 0.0) return 0.0;  // also keeps 0 * inf away when a is tiny
    return eh + eh * tl;
}

// The rejection loops accept with probability above 0.95 (Marsaglia-Tsang)
// per attempt; the bound only guarantees that a lane exits.
static constexpr int kMaxAttempts = 1 << 20;

template <class E>
__device__ double mt_gamma(E &eng, const ZigLds *zt, double a)
{
    const double d = a - 1.0 / 3.0;
    const double c = 1.0 / sqrt(9.0 * d);
    for (int it = 0; it < kMaxAttempts; it++) {
        double x, v;
        int guard = 0;
        do {
            x = zig_serial<RP_NORM>(zt, eng);
            v = 1.0 + c * x;
        } while (v <= 0.0 && ++guard < kMaxAttempts);
        v = v * v * v;
        const double u = u01_53(eng.next());
        const double x2 = x * x;
        if (u < 1.0 - 0.0331 * (x2 * x2)) return d * v;
        if (log(u) < 0.5 * x2 + d * ((1.0 - v) + log(v))) return d * v;
    }
    return d;
}

template <class E>
__device__ double gamma_one(E &eng, const ZigLds *zt, double a)
{
    if (a < 1.0) {
        const double g = mt_gamma(eng, zt, a + 1.0);
        const double u = u01_53(eng.next());
        return g * boost_pow(u, a);
    }
    return mt_gamma(eng, zt, a);
}

template <class E>
__device__ double beta_one(E &eng, const ZigLds *zt, double a, double b)
{
    const double x = gamma_one(eng, zt, a);
    const double y = gamma_one(eng, zt, b);
    const double t = x + y;
    if (t == 0.0) return a / (a + b);
    return x / t;
}

// ---------------------------------------------------------------------------

template <class E>
__global__ __launch_bounds__(256) void k_norm_moments(SampArgs s)
{
    __shared__ ZigLds zt;
    load_zig<RP_NORM>(&zt);
    __syncthreads();
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= s.count) return;
    E eng;
    eng.load(s.f, i);
    double a = 0.0, q = 0.0;
    for (uint64_t t = 0; t < s.f.per_stream; t++) {
        const double x = zig_serial<RP_NORM>(&zt, eng);
        a = a + x;
        q = q + x * x;
    }
    s.sum[i] = a;
    s.sumsq[i] = q;
    eng.store(s.f, i);
}

template <class E, bool BETA>
__global__ __launch_bounds__(256) void k_gamma_elem(SampArgs s)
{
    __shared__ ZigLds zt;
    load_zig<RP_NORM>(&zt);
    __syncthreads();
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= s.count) return;
    E eng;
    eng.load(s.f, i);
    const double pa = (double)s.pa[i];
    const double pb = BETA ? (double)s.pb[i] : 1.0;
    if (!(pa > 0.0) || !(pb > 0.0)) {
        s.z[i] = __builtin_nanf("");
        return;
    }
    const double v = BETA ? beta_one(eng, &zt, pa, pb) : gamma_one(eng, &zt, pa);
    s.z[i] = (float)v;
    eng.store(s.f, i);
}


// Row i of z (count rows of per_stream = d values) holds the next d normals
// of substream i rounded to binary32.  With d a multiple of 4 each lane
// writes its row as 16-byte pieces.
template <class E>
__global__ __launch_bounds__(256) void k_norm_rows(SampArgs s)
{
    __shared__ ZigLds zt;
    load_zig<RP_NORM>(&zt);
    __syncthreads();
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= s.count) return;
    E eng;
    eng.load(s.f, i);
    const uint64_t d = s.f.per_stream;
    float *row = s.z + i * d;
    if ((d & 3) == 0) {
        for (uint64_t t = 0; t < d; t += 4) {
            float4 v;
            v.x = (float)zig_serial<RP_NORM>(&zt, eng);
            v.y = (float)zig_serial<RP_NORM>(&zt, eng);
            v.z = (float)zig_serial<RP_NORM>(&zt, eng);
            v.w = (float)zig_serial<RP_NORM>(&zt, eng);
            *(float4 *)(row + t) = v;
        }
    } else {
        for (uint64_t t = 0; t < d; t++) row[t] = (float)zig_serial<RP_NORM>(&zt, eng);
    }
    if (s.advance) eng.store(s.f, i);
}

template <class E>
static int launch_moments_e(const SampArgs &s, hipStream_t st)
{
    const uint64_t blocks = (s.count + 255) / 256;
    hipLaunchKernelGGL((k_norm_moments<E>), dim3((unsigned)blocks), dim3(256), 0, st, s);
    return RP_OK;
}

template <class E>
static int launch_elem_e(const SampArgs &s, bool beta, hipStream_t st)
{
    const uint64_t blocks = (s.count + 255) / 256;
    if (beta)
        hipLaunchKernelGGL((k_gamma_elem<E, true>), dim3((unsigned)blocks), dim3(256), 0, st, s);
    else
        hipLaunchKernelGGL((k_gamma_elem<E, false>), dim3((unsigned)blocks), dim3(256), 0, st, s);
    return RP_OK;
}

int launch_moments(int engine, const SampArgs &s, hipStream_t st)
{
    switch (engine) {
    case RP_X256PP: launch_moments_e<LaneX256>(s, st); break;
    case RP_PCG64: launch_moments_e<LanePcg>(s, st); break;
    case RP_PHILOX4X32: launch_moments_e<LanePhilox32>(s, st); break;
    case RP_PHILOX: launch_moments_e<LanePhilox64>(s, st); break;
    case RP_SFC64: launch_moments_e<LaneSfc64>(s, st); break;
    case RP_RANLUX: launch_moments_e<LaneRanlux>(s, st); break;
    default: return fail(RP_EINVAL, "unknown engine");
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? RP_OK : fail(RP_EDEVICE, "moments launch: %s", hipGetErrorString(e));
}

int launch_norm_rows(int engine, const SampArgs &s, hipStream_t st)
{
    const dim3 grid((unsigned)((s.count + 255) / 256)), block(256);
    switch (engine) {
    case RP_X256PP: hipLaunchKernelGGL(k_norm_rows<LaneX256>, grid, block, 0, st, s); break;
    case RP_PCG64: hipLaunchKernelGGL(k_norm_rows<LanePcg>, grid, block, 0, st, s); break;
    case RP_PHILOX4X32: hipLaunchKernelGGL(k_norm_rows<LanePhilox32>, grid, block, 0, st, s); break;
    case RP_PHILOX: hipLaunchKernelGGL(k_norm_rows<LanePhilox64>, grid, block, 0, st, s); break;
    case RP_SFC64: hipLaunchKernelGGL(k_norm_rows<LaneSfc64>, grid, block, 0, st, s); break;
    case RP_RANLUX: hipLaunchKernelGGL(k_norm_rows<LaneRanlux>, grid, block, 0, st, s); break;
    default: return fail(RP_EINVAL, "unknown engine");
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? RP_OK : fail(RP_EDEVICE, "normal rows launch: %s", hipGetErrorString(e));
}

int launch_gamma_elem(int engine, const SampArgs &s, bool beta, hipStream_t st)
{
    switch (engine) {
    case RP_X256PP: launch_elem_e<LaneX256>(s, beta, st); break;
    case RP_PCG64: launch_elem_e<LanePcg>(s, beta, st); break;
    case RP_PHILOX4X32: launch_elem_e<LanePhilox32>(s, beta, st); break;
    case RP_PHILOX: launch_elem_e<LanePhilox64>(s, beta, st); break;
    case RP_SFC64: launch_elem_e<LaneSfc64>(s, beta, st); break;
    case RP_RANLUX: launch_elem_e<LaneRanlux>(s, beta, st); break;
    default: return fail(RP_EINVAL, "unknown engine");
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? RP_OK : fail(RP_EDEVICE, "gamma launch: %s", hipGetErrorString(e));
}
