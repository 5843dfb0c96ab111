// k_mvn.hip -- multivariate normal rows (Section 3.1, "Multivariate normal
// distribution"): X = mu + Z L^T for n rows of d standard normals Z, with L
// the lower-triangular Cholesky factor of the covariance, and its backward
// grad_mu = sum_rows G, grad_L = tril(G^T Z).
//
// Row i of Z is the next d normals of substream i (binary64 ziggurat draws
// rounded to binary32).  Z is generated into a stream-ordered workspace by
// the lane-per-row kernel, then contracted on the matrix cores with
// v_mfma_f32_32x32x2f32 (binary32 in, binary32 accumulate).  The backward
// regenerates the same Z from the substream states the forward started from,
// so nothing of size n x d is kept between the two.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <limits>
#include <vector>

#include "rp_internal.h"

namespace rp {

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kKT = 32;         // backward k (rows of G and Z) per LDS stage
constexpr int kTile = 128;      // rows of a block tile
constexpr int kLdT = kTile + 4; // backward LDS row stride (floats), rows indexed by k

__device__ __forceinline__ float4 load4(const float *M, uint64_t rows, uint64_t cols, uint64_t r, uint64_t c,
                                        bool vec)
{
    float4 v = {0.f, 0.f, 0.f, 0.f};
    if (r >= rows) return v;
    const float *p = M + r * cols + c;
    if (vec && c + 3 < cols) return *(const float4 *)p;
    if (c < cols) v.x = p[0];
    if (c + 1 < cols) v.y = p[1];
    if (c + 2 < cols) v.z = p[2];
    if (c + 3 < cols) v.w = p[3];
    return v;
}

// Blocks are dealt round-robin to the 8 XCDs; renumber them so that each XCD
// works through a contiguous range of tiles (tiles that share operand rows
// then share that XCD's L2).
__device__ __forceinline__ unsigned xcd_tile(unsigned b, unsigned nb)
{
    return (nb % 8 == 0) ? (b % 8) * (nb / 8) + b / 8 : b;
}

// One 32x32 output tile of C += A B per lane-pair of operands, lane l giving
// A[l % 32][k] and B[k][l % 32] for the k of its half (l / 32); the result
// element v of lane l is C[8 (v / 4) + 4 (l / 32) + v % 4][l % 32].
__device__ __forceinline__ int acc_row(int v, int h) { return 8 * (v >> 2) + 4 * h + (v & 3); }

// ---------------------------------------------------------------------------
// Whether the factor has an entry above the diagonal that is not +0 (*flag
// = 1; NaN and -0 count) or is lower triangular (0).  For a lower factor
// column c of X needs only k <= c, so each column tile of the forward stops
// its k loop after its own last column (half the products at large d); the
// skipped products are exact zeros.
__global__ void k_upper_clear(int *flag) { *flag = 0; }

__global__ __launch_bounds__(256) void k_upper_scan(const float *L, int d, int *flag)
{
    const uint64_t dd = (uint64_t)d, total = dd * dd;
    bool nz = false;
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t r = e / dd, c = e - r * dd;
        if (c > r && __float_as_uint(L[e]) != 0u) nz = true;
    }
    if (__syncthreads_or(nz) && threadIdx.x == 0) atomicOr(flag, 1);
}

// forward: block tile 128 rows x BN columns, 4 waves as 2 x 2, wave tile
// 64 x BN/2 (2 x BN/64 MFMA tiles).  Each lane half takes four consecutive k
// of an eight-k step, so operand fragments are single 16-byte LDS reads.
// The k loop runs in stages of kFK with two LDS buffers (one barrier a
// stage): the global loads of stage t + 2 are in flight while stage t + 1 is
// written and stage t is contracted.
//
// With a lower factor, column tile c of X needs the k tiles up to its own
// last column, so its cost grows with c.  Block (row tile r, pair p) does
// column tiles p and nct - 1 - p of row tile r one after the other, so every
// block carries about the same number of k stages (blocks of unequal length
// leave the compute units that drew the long ones working alone at the end).
// upper: the flag of k_upper_scan.
constexpr int kFK = 16;          // forward k per LDS stage
constexpr int kFLd = kFK + 4;    // forward LDS row stride (floats), rows indexed by m / n
constexpr int kFCpr = kFK / 4;   // threads per operand row of a stage (16 bytes each)
constexpr int kFRpp = 256 / kFCpr;  // operand rows per pass of the block

template <int BN>
__global__ __launch_bounds__(256, 3) void k_mvn_fwd(const float *Z, const float *L, const float *mu, float *X,
                                                 uint64_t n, int d, unsigned ncol_tiles, int vec, const int *upper)
{
    constexpr int TN = BN / 64;
    constexpr int NA = kTile / kFRpp, NB = BN / kFRpp;
    __shared__ __align__(16) float As[2][kTile * kFLd];
    __shared__ __align__(16) float Bs[2][BN * kFLd];
    const unsigned npair = (ncol_tiles + 1) / 2;
    const unsigned wp = xcd_tile(blockIdx.x, gridDim.x);
    const unsigned rt = wp / npair, pr = wp % npair;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int h = lane >> 5, l32 = lane & 31;
    const int wr = wave >> 1, wc = wave & 1;
    const int lr = tid / kFCpr, lc = 4 * (tid % kFCpr);
    const uint64_t dd = (uint64_t)d;
    const uint64_t row0 = (uint64_t)rt * kTile;
    const bool tri = __builtin_amdgcn_readfirstlane(*upper) == 0;
#pragma unroll 1
    for (int q = 0; q < 2; q++) {
        const unsigned ct = q == 0 ? pr : ncol_tiles - 1 - pr;
        if (q == 1 && ct == pr) break;
        const int col0 = (int)ct * BN;
        f32x16 acc[2][TN];
#pragma unroll
        for (int a = 0; a < 2; a++)
#pragma unroll
            for (int b = 0; b < TN; b++)
#pragma unroll
                for (int v = 0; v < 16; v++) acc[a][b][v] = 0.f;
        int nk = (d + kFK - 1) / kFK;
        if (tri) {
            const int last = (col0 + BN + kFK - 1) / kFK;  // k tiles holding columns < col0 + BN
            nk = nk < last ? nk : last;
        }
        // unconditional 16-byte loads when the whole tile is inside Z and L
        const bool full = vec && row0 + kTile <= n && d % kFK == 0 && col0 + BN <= d;
        const float *pa = Z + (row0 + lr) * dd + lc;
        const float *pb = L + (uint64_t)(col0 + lr) * dd + lc;
        float4 ra[NA], rb[NB];
        auto gload = [&](int kt) {
            const uint64_t k0 = (uint64_t)kt * kFK;
            if (full) {
#pragma unroll
                for (int r = 0; r < NA; r++) ra[r] = *(const float4 *)(pa + (uint64_t)(r * kFRpp) * dd + k0);
#pragma unroll
                for (int r = 0; r < NB; r++) rb[r] = *(const float4 *)(pb + (uint64_t)(r * kFRpp) * dd + k0);
            } else {
#pragma unroll
                for (int r = 0; r < NA; r++) ra[r] = load4(Z, n, dd, row0 + lr + r * kFRpp, k0 + lc, vec);
#pragma unroll
                for (int r = 0; r < NB; r++)
                    rb[r] = load4(L, dd, dd, (uint64_t)(col0 + lr + r * kFRpp), k0 + lc, vec);
            }
        };
        auto swrite = [&](int buf) {
#pragma unroll
            for (int r = 0; r < NA; r++) *(float4 *)&As[buf][(lr + r * kFRpp) * kFLd + lc] = ra[r];
#pragma unroll
            for (int r = 0; r < NB; r++) *(float4 *)&Bs[buf][(lr + r * kFRpp) * kFLd + lc] = rb[r];
        };
        // with a triangular factor, the k steps past a 32-column sub-tile's
        // last column multiply zeros: the sub-tile skips them
        int jlast[TN];
#pragma unroll
        for (int b = 0; b < TN; b++) jlast[b] = tri ? col0 + wc * (BN / 2) + b * 32 + 31 : d;
        auto compute = [&](int buf, int kt) {
#pragma unroll
            for (int s = 0; s < kFK / 8; s++) {
                const int k8 = kt * kFK + 8 * s;  // first k of this step
                float4 af[2], bf[TN];
#pragma unroll
                for (int a = 0; a < 2; a++)
                    af[a] = *(const float4 *)&As[buf][(wr * 64 + a * 32 + l32) * kFLd + 8 * s + 4 * h];
#pragma unroll
                for (int b = 0; b < TN; b++)
                    bf[b] = *(const float4 *)&Bs[buf][(wc * (BN / 2) + b * 32 + l32) * kFLd + 8 * s + 4 * h];
#pragma unroll
                for (int a = 0; a < 2; a++)
#pragma unroll
                    for (int b = 0; b < TN; b++) {
                        if (k8 > jlast[b]) continue;  // wave-uniform
                        acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[a].x, bf[b].x, acc[a][b], 0, 0, 0);
                        acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[a].y, bf[b].y, acc[a][b], 0, 0, 0);
                        acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[a].z, bf[b].z, acc[a][b], 0, 0, 0);
                        acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[a].w, bf[b].w, acc[a][b], 0, 0, 0);
                    }
            }
        };
        gload(0);
        swrite(0);
        __syncthreads();
        if (nk > 1) gload(1);
        for (int kt = 0; kt < nk; kt++) {
            compute(kt & 1, kt);
            if (kt + 1 < nk) {
                swrite((kt + 1) & 1);
                __syncthreads();
                if (kt + 2 < nk) gload(kt + 2);
            }
        }
        // element v of a lane's MFMA tile is row 8 (v / 4) + 4 h + v % 4: the
        // store pointer steps by one row, and by five after every fourth
        const bool rows_full = row0 + kTile <= n;
#pragma unroll
        for (int b = 0; b < TN; b++) {
            const int j = col0 + wc * (BN / 2) + b * 32 + l32;
            if (j >= d) continue;
            const float m = mu[j];
            const uint64_t i0 = row0 + (uint64_t)(wr * 64 + 4 * h);
            float *p = X + i0 * dd + j;
#pragma unroll
            for (int a = 0; a < 2; a++)
#pragma unroll
                for (int v = 0; v < 16; v++) {
                    const int r = a * 32 + acc_row(v, 0);
                    if (rows_full || i0 + r < n) *p = acc[a][b][v] + m;
                    p += ((v & 3) == 3) ? 5 * dd : dd;
                }
        }
        __syncthreads();  // the next tile of the pair rewrites both LDS buffers
    }
}

// ---------------------------------------------------------------------------
// backward, split over the rows: block (tile t, slice s) accumulates
// sum_{i in slice s} G[i][a] Z[i][b] for the 128 x 128 tile t of the lower
// triangle (tiles with ta >= tb), and, in the tiles with tb = 0, the column
// sums of G over the slice.
__global__ __launch_bounds__(256) void k_mvn_bwd(const float *G, const float *Z, uint64_t n, int d, uint64_t slice,
                                                 float *part, float *gmu_part, int vec)
{
    __shared__ __align__(16) float Gs[kKT * kLdT];
    __shared__ __align__(16) float Zs[kKT * kLdT];
    unsigned t = blockIdx.x, ta = 0;
    while (t > ta) {
        t -= ta + 1;
        ta++;
    }
    const unsigned tb = t;
    const int a0 = (int)ta * kTile, b0 = (int)tb * kTile;
    const uint64_t i0 = (uint64_t)blockIdx.y * slice;
    uint64_t i1 = i0 + slice;
    if (i1 > n) i1 = n;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int h = lane >> 5, l32 = lane & 31;
    const int wr = wave >> 1, wc = wave & 1;
    const uint64_t dd = (uint64_t)d;
    f32x16 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int b = 0; b < 2; b++)
#pragma unroll
            for (int v = 0; v < 16; v++) acc[a][b][v] = 0.f;
    float colsum = 0.f;
    float4 rg[4], rz[4];
    const uint64_t nk = (i1 > i0) ? (i1 - i0 + kKT - 1) / kKT : 0;
#pragma unroll
    for (int r = 0; r < 4; r++) {
        const int u = tid + 256 * r;
        rg[r] = load4(G, i1, dd, i0 + (u >> 5), a0 + 4 * (u & 31), vec);
        rz[r] = load4(Z, i1, dd, i0 + (u >> 5), b0 + 4 * (u & 31), vec);
    }
    for (uint64_t kt = 0; kt < nk; kt++) {
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const int u = tid + 256 * r;
            *(float4 *)&Gs[(u >> 5) * kLdT + 4 * (u & 31)] = rg[r];
            *(float4 *)&Zs[(u >> 5) * kLdT + 4 * (u & 31)] = rz[r];
        }
        __syncthreads();
        if (kt + 1 < nk) {
            const uint64_t k0 = i0 + (kt + 1) * kKT;
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int u = tid + 256 * r;
                rg[r] = load4(G, i1, dd, k0 + (u >> 5), a0 + 4 * (u & 31), vec);
                rz[r] = load4(Z, i1, dd, k0 + (u >> 5), b0 + 4 * (u & 31), vec);
            }
        }
        if (tb == 0 && tid < kTile) {
#pragma unroll 8
            for (int k = 0; k < kKT; k++) colsum += Gs[k * kLdT + tid];
        }
#pragma unroll
        for (int k = 0; k < kKT; k += 2) {
            float af[2], bf[2];
#pragma unroll
            for (int a = 0; a < 2; a++) af[a] = Gs[(k + h) * kLdT + wr * 64 + a * 32 + l32];
#pragma unroll
            for (int b = 0; b < 2; b++) bf[b] = Zs[(k + h) * kLdT + wc * 64 + b * 32 + l32];
#pragma unroll
            for (int a = 0; a < 2; a++)
#pragma unroll
                for (int b = 0; b < 2; b++)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[a], bf[b], acc[a][b], 0, 0, 0);
        }
    }
    float *P = part + (uint64_t)blockIdx.y * dd * dd;
#pragma unroll
    for (int b = 0; b < 2; b++) {
        const int j = b0 + wc * 64 + b * 32 + l32;
        if (j >= d) continue;
#pragma unroll
        for (int a = 0; a < 2; a++)
#pragma unroll
            for (int v = 0; v < 16; v++) {
                const int i = a0 + wr * 64 + a * 32 + acc_row(v, h);
                if (i < d) P[(uint64_t)i * dd + j] = acc[a][b][v];
            }
    }
    if (tb == 0 && tid < kTile && a0 + tid < d) gmu_part[(uint64_t)blockIdx.y * dd + a0 + tid] = colsum;
}

// The per-slice partials are summed in binary64 in two passes, so that the
// reduction has parallelism even when there are few elements (d = 64: 4096
// elements, 2048 slices).  Elements of the combined array are the d x d
// entries of the grad_L partials followed by the d entries of the grad_mu
// partials.  Pass 1: block (x, y) sums slices 64 y .. 64 y + 63 of elements
// 64 x .. 64 x + 63, four threads per element.  Pass 2: the group sums of an
// element, in group order.  Entries above the diagonal of grad_L are 0.
constexpr int kRedGroup = 64;

__global__ __launch_bounds__(256) void k_mvn_reduce1(const float *part, const float *gmu_part, int nslices, int d,
                                                     double *sums)
{
    __shared__ double red[4][64];
    const uint64_t dd = (uint64_t)d, total = dd * dd, all = total + dd;
    const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
    const uint64_t e = (uint64_t)blockIdx.x * 64 + lane;
    const int k0 = (int)blockIdx.y * kRedGroup;
    const int k1 = nslices < k0 + kRedGroup ? nslices : k0 + kRedGroup;
    double acc = 0.0;
    const bool gmu = e >= total;
    if (e < all && (gmu || e / dd >= e % dd)) {
        const float *src = gmu ? gmu_part + (e - total) : part + e;
        const uint64_t stride = gmu ? dd : total;
        for (int k = k0 + q; k < k1; k += 4) acc += (double)src[(uint64_t)k * stride];
    }
    red[q][lane] = acc;
    __syncthreads();
    if (q == 0 && e < all) sums[(uint64_t)blockIdx.y * all + e] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
}

__global__ __launch_bounds__(256) void k_mvn_reduce2(const double *sums, int ngroups, int d, float *gL, float *gmu)
{
    const uint64_t dd = (uint64_t)d, total = dd * dd, all = total + dd;
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < all;
         e += (uint64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        if (e >= total || e / dd >= e % dd)
            for (int g = 0; g < ngroups; g++) s += sums[(uint64_t)g * all + e];
        if (e < total) gL[e] = (float)s;
        else gmu[e - total] = (float)s;
    }
}

int hip_fail(hipError_t e, const char *what) { return fail(RP_EDEVICE, "%s: %s", what, hipGetErrorString(e)); }

bool al16(const void *p) { return ((uintptr_t)p & 15) == 0; }
bool al4(const void *p) { return ((uintptr_t)p & 3) == 0; }

// Keep freed stream-ordered allocations cached in the device's default pool.
int keep_pool(hipStream_t)
{
    static bool done[64] = {false};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return RP_OK;
    if (done[dev]) return RP_OK;
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
        uint64_t thr = UINT64_MAX;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
    }
    done[dev] = true;
    return RP_OK;
}

int gen_rows(rp_streams *s, float *z, int d, uint64_t n, bool advance, hipStream_t st)
{
    SampArgs a{};
    a.f.words = s->d_words;
    a.f.phase = s->d_phase;
    a.f.n = s->n;
    a.f.flags = settings_flags(s);
    a.f.per_stream = (uint64_t)d;
    a.count = n;
    a.z = z;
    a.advance = advance ? 1 : 0;
    return launch_norm_rows(s->engine, a, st);
}

int check_common(const char *who, rp_streams *s, int d, uint64_t n)
{
    if (!s) return fail(RP_ENULL, "%s: NULL streams", who);
    if (d < 1 || d > 65536) return fail(RP_EINVAL, "%s: d = %d (1..65536)", who, d);
    if (n > s->n) return fail(RP_EINVAL, "%s: %llu rows but only %llu substreams", who, (unsigned long long)n,
                              (unsigned long long)s->n);
    return RP_OK;
}

}  // namespace

}  // namespace rp

using namespace rp;

extern "C" int rp_mvn(rp_streams *s, const float *d_mu, const float *d_L, int d, uint64_t n, float *d_X,
                      void *hip_stream)
{
    int rc = check_common("rp_mvn", s, d, n);
    if (rc) return rc;
    if (n == 0) return RP_OK;
    if (!d_mu || !d_L || !d_X) return fail(RP_ENULL, "rp_mvn: NULL device pointer");
    if (!al4(d_mu) || !al4(d_L) || !al4(d_X)) return fail(RP_EINVAL, "rp_mvn: pointers not aligned to 4 bytes");
    rc = ensure_device_tables();
    if (rc) return rc;
    hipStream_t st = (hipStream_t)hip_stream;
    keep_pool(st);
    float *z = nullptr;
    const uint64_t zbytes = (n * (uint64_t)d * sizeof(float) + 255) & ~(uint64_t)255;
    hipError_t e = hipMallocAsync((void **)&z, zbytes + 256, st);
    if (e != hipSuccess) return fail(RP_ENOMEM, "rp_mvn: workspace of %llu floats: %s",
                                     (unsigned long long)(n * (uint64_t)d), hipGetErrorString(e));
    int *upper = (int *)((char *)z + zbytes);
    hipLaunchKernelGGL(k_upper_clear, dim3(1), dim3(1), 0, st, upper);
    {
        const uint64_t total = (uint64_t)d * (uint64_t)d;
        const uint64_t blocks = std::min<uint64_t>((total + 255) / 256, 1024);
        hipLaunchKernelGGL(k_upper_scan, dim3((unsigned)blocks), dim3(256), 0, st, d_L, d, upper);
    }
    rc = gen_rows(s, z, d, n, true, st);
    if (rc == RP_OK) {
        const int vec = (d % 4 == 0) && al16(d_L) && al16(z) ? 1 : 0;
        const uint64_t nrt = (n + kTile - 1) / kTile;
        if (d <= 64) {
            const unsigned nct = 1;
            hipLaunchKernelGGL(k_mvn_fwd<64>, dim3((unsigned)nrt), dim3(256), 0, st, z, d_L, d_mu, d_X, n, d, nct,
                               vec, (const int *)upper);
        } else {
            const unsigned nct = (unsigned)((d + 127) / 128), npair = (nct + 1) / 2;
            hipLaunchKernelGGL(k_mvn_fwd<128>, dim3((unsigned)(nrt * npair)), dim3(256), 0, st, z, d_L, d_mu, d_X,
                               n, d, nct, vec, (const int *)upper);
        }
        e = hipGetLastError();
        if (e != hipSuccess) rc = hip_fail(e, "rp_mvn launch");
    }
    (void)hipFreeAsync(z, st);
    return rc;
}

extern "C" int rp_mvn_backward(rp_streams *s, const float *d_G, int d, uint64_t n, float *d_gmu, float *d_gL,
                               void *hip_stream)
{
    int rc = check_common("rp_mvn_backward", s, d, n);
    if (rc) return rc;
    if (!d_G || !d_gmu || !d_gL) return fail(RP_ENULL, "rp_mvn_backward: NULL device pointer");
    if (!al4(d_G) || !al4(d_gmu) || !al4(d_gL)) return fail(RP_EINVAL, "rp_mvn_backward: pointers not aligned");
    rc = ensure_device_tables();
    if (rc) return rc;
    hipStream_t st = (hipStream_t)hip_stream;
    keep_pool(st);
    // split the rows so that the lower-triangle tiles times the slices give
    // about 2048 blocks
    const uint64_t nt = (uint64_t)(d + kTile - 1) / kTile;
    const uint64_t ntl = nt * (nt + 1) / 2;
    uint64_t nsl = (2048 + ntl - 1) / ntl;
    const uint64_t max_sl = (n + kKT - 1) / kKT;
    if (nsl > max_sl) nsl = max_sl;
    if (nsl < 1) nsl = 1;
    uint64_t slice = (n + nsl - 1) / nsl;
    slice = (slice + kKT - 1) / kKT * kKT;
    if (slice == 0) slice = kKT;
    nsl = (n + slice - 1) / slice;
    if (nsl == 0) nsl = 1;
    const uint64_t dd = (uint64_t)d;
    const uint64_t zf = n * dd, pf = nsl * dd * dd, gf = nsl * dd;
    const uint64_t ngroups = n ? (nsl + kRedGroup - 1) / kRedGroup : 0, all = dd * dd + dd;
    // floats: Z, the slice partials of grad_L and grad_mu; then the group sums (binary64)
    const uint64_t fl = (zf + 3) / 4 * 4 + pf + gf;
    const uint64_t sum_off = (fl * sizeof(float) + 255) / 256 * 256;
    float *ws = nullptr;
    hipError_t e = hipMallocAsync((void **)&ws, sum_off + ngroups * all * sizeof(double) + 256, st);
    if (e != hipSuccess) return fail(RP_ENOMEM, "rp_mvn_backward: workspace: %s", hipGetErrorString(e));
    float *z = ws;
    float *part = ws + ((zf + 3) & ~3ull);
    float *gpart = part + pf;
    double *sums = (double *)((char *)ws + sum_off);
    rc = n ? gen_rows(s, z, d, n, false, st) : RP_OK;
    if (rc == RP_OK) {
        const int vec = (d % 4 == 0) && al16(d_G) && al16(z) ? 1 : 0;
        if (n) hipLaunchKernelGGL(k_mvn_bwd, dim3((unsigned)ntl, (unsigned)nsl), dim3(256), 0, st, d_G, z, n, d,
                                  slice, part, gpart, vec);
        if (ngroups)
            hipLaunchKernelGGL(k_mvn_reduce1, dim3((unsigned)((all + 63) / 64), (unsigned)ngroups), dim3(256), 0, st,
                               part, gpart, (int)nsl, d, sums);
        uint64_t blocks = (all + 255) / 256;
        if (blocks > 4096) blocks = 4096;
        hipLaunchKernelGGL(k_mvn_reduce2, dim3((unsigned)blocks), dim3(256), 0, st, sums, (int)ngroups, d, d_gL,
                           d_gmu);
        e = hipGetLastError();
        if (e != hipSuccess) rc = hip_fail(e, "rp_mvn_backward launch");
    }
    (void)hipFreeAsync(ws, st);
    return rc;
}

// Pivoted Cholesky (the paper's fallback for semidefinite covariances,
// with LAPACK dpstrf's rule): step j pivots on the largest diagonal entry of
// the remaining Schur complement and stops when it is at most
// tol = d eps max_i Sigma_ii; column j of L is formed left-looking from the
// permuted Sigma and the earlier columns.  A = P L (row perm[k] of A is row
// k of L), so Sigma = A A^T.  A trailing diagonal entry below -tol means
// Sigma is not semidefinite.
extern "C" int rp_mvn_factor(const double *Sigma, int d, double *A, int *rank)
{
    if (!Sigma || !A || !rank) return fail(RP_ENULL, "rp_mvn_factor: NULL pointer");
    if (d < 1) return fail(RP_EINVAL, "rp_mvn_factor: d = %d", d);
    const size_t D = (size_t)d;
    for (size_t i = 0; i < D; i++)
        for (size_t j = 0; j <= i; j++)
            if (!std::isfinite(Sigma[i * D + j])) return fail(RP_EINVAL, "rp_mvn_factor: Sigma is not finite");
    // the plain factorization first (its failure is not an error here)
    std::vector<double> L(D * D, 0.0), S(D * D);
    bool pd = true;
    for (size_t i = 0; i < D && pd; i++) {
        for (size_t j = 0; j <= i; j++) {
            double s = Sigma[i * D + j];
            for (size_t k = 0; k < j; k++) s -= L[i * D + k] * L[j * D + k];
            if (i == j) {
                if (!(s > 0.0)) {
                    pd = false;
                    break;
                }
                L[i * D + i] = std::sqrt(s);
            } else {
                L[i * D + j] = s / L[j * D + j];
            }
        }
    }
    if (pd) {
        std::copy(L.begin(), L.end(), A);
        *rank = d;
        return RP_OK;
    }
    for (size_t i = 0; i < D; i++)
        for (size_t j = 0; j <= i; j++) S[i * D + j] = S[j * D + i] = Sigma[i * D + j];
    std::fill(L.begin(), L.end(), 0.0);
    std::vector<size_t> perm(D);
    std::vector<double> diag(D);
    double dmax = S[0];
    for (size_t i = 1; i < D; i++) dmax = std::max(dmax, S[i * D + i]);
    const double tol = (double)d * std::numeric_limits<double>::epsilon() * dmax;
    for (size_t i = 0; i < D; i++) perm[i] = i;
    size_t r = D;
    double rest = 0.0;
    for (size_t j = 0; j < D; j++) {
        size_t p = j;
        for (size_t i = j; i < D; i++) {
            double v = S[i * D + i];
            for (size_t k = 0; k < j; k++) v -= L[i * D + k] * L[i * D + k];
            diag[i] = v;
            if (v > diag[p]) p = i;
        }
        if (!(diag[p] > tol)) {
            r = j;
            rest = diag[j];
            for (size_t i = j + 1; i < D; i++) rest = std::min(rest, diag[i]);
            break;
        }
        if (p != j) {
            for (size_t c = 0; c < D; c++) std::swap(S[j * D + c], S[p * D + c]);
            for (size_t c = 0; c < D; c++) std::swap(S[c * D + j], S[c * D + p]);
            for (size_t c = 0; c < j; c++) std::swap(L[j * D + c], L[p * D + c]);
            std::swap(perm[j], perm[p]);
        }
        const double ljj = std::sqrt(diag[p]);
        L[j * D + j] = ljj;
        for (size_t i = j + 1; i < D; i++) {
            double s = S[i * D + j];
            for (size_t k = 0; k < j; k++) s -= L[i * D + k] * L[j * D + k];
            L[i * D + j] = s / ljj;
        }
    }
    if (r < D && rest < -tol)
        return fail(RP_ENOTSPD, "rp_mvn_factor: covariance is not positive semidefinite (trailing diagonal %g)",
                    rest);
    for (size_t k = 0; k < D; k++)
        for (size_t c = 0; c < D; c++) A[perm[k] * D + c] = L[k * D + c];
    *rank = (int)r;
    return RP_OK;
}

// Cholesky-Banachiewicz in binary64 on the host, reading the lower triangle
// of Sigma (row-major d x d) and writing L with zeros above the diagonal.
extern "C" int rp_cholesky(const double *Sigma, int d, double *L)
{
    if (!Sigma || !L) return fail(RP_ENULL, "rp_cholesky: NULL pointer");
    if (d < 1) return fail(RP_EINVAL, "rp_cholesky: d = %d", d);
    const size_t D = (size_t)d;
    for (size_t i = 0; i < D; i++) {
        for (size_t j = 0; j <= i; j++) {
            double s = Sigma[i * D + j];
            for (size_t k = 0; k < j; k++) s -= L[i * D + k] * L[j * D + k];
            if (i == j) {
                if (!(s > 0.0) || !std::isfinite(s))
                    return fail(RP_ENOTSPD, "rp_cholesky: leading minor %zu is not positive definite", i + 1);
                L[i * D + i] = std::sqrt(s);
            } else {
                L[i * D + j] = s / L[j * D + j];
            }
        }
        for (size_t j = i + 1; j < D; j++) L[i * D + j] = 0.0;
    }
    return RP_OK;
}
