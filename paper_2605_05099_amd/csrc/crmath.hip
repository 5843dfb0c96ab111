// crmath.hip -- the correctly rounded functions of crmath.h as library calls,
// evaluated on the host (rp_crmath_host) or on the device (rp_crmath).  The
// two builds run the same binary64 operations, so they agree bit for bit.
#include <hip/hip_runtime.h>

#include "crmath.h"
#include "rp_internal.h"

namespace rp {

namespace {

__host__ __device__ inline double cr_eval(int fn, double x, double y)
{
    switch (fn) {
    case RP_CR_EXP: return crm::cr_exp(x);
    case RP_CR_LOG: return crm::cr_log(x);
    case RP_CR_LOG1P: return crm::cr_log1p(x);
    case RP_CR_POW: return crm::cr_pow(x, y);
    default: return crm::cr_powinv(x, y);
    }
}

__global__ __launch_bounds__(256) void k_crmath(int fn, const double *x, const double *y, double *out, uint64_t n)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        out[i] = cr_eval(fn, x[i], y ? y[i] : 0.0);
}

int check(const char *who, int fn, const double *x, const double *y, double *out)
{
    if (fn < RP_CR_EXP || fn > RP_CR_POWINV) return fail(RP_EINVAL, "%s: unknown function %d", who, fn);
    if (!x || !out) return fail(RP_ENULL, "%s: NULL argument or output", who);
    if ((fn == RP_CR_POW || fn == RP_CR_POWINV) && !y) return fail(RP_ENULL, "%s: NULL second argument", who);
    return RP_OK;
}

}  // namespace

}  // namespace rp

using namespace rp;

extern "C" int rp_crmath_host(int fn, const double *x, const double *y, double *out, uint64_t n)
{
    const int rc = check("rp_crmath_host", fn, x, y, out);
    if (rc) return rc;
    for (uint64_t i = 0; i < n; i++) out[i] = cr_eval(fn, x[i], y ? y[i] : 0.0);
    return RP_OK;
}

extern "C" int rp_crmath(int fn, const double *d_x, const double *d_y, double *d_out, uint64_t n, void *hip_stream)
{
    const int rc = check("rp_crmath", fn, d_x, d_y, d_out);
    if (rc) return rc;
    if (n == 0) return RP_OK;
    const uint64_t blocks = std::min<uint64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_crmath, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)hip_stream, fn, d_x,
                       (fn == RP_CR_POW || fn == RP_CR_POWINV) ? d_y : nullptr, d_out, n);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(RP_EDEVICE, "rp_crmath launch: %s", hipGetErrorString(e));
    return RP_OK;
}
