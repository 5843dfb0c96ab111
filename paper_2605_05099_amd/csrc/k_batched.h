// k_batched.h -- batched gamma / beta over many parameter sets with uneven
// counts.  Included by fill.hip after k_samplers.h.
//
// Set j draws count[j] values from substream j (the serial definition: one
// scalar stream per set) into out[offset_j ...], offset_j = sum_{k<j} count[k].
// One launch sequence, recorded once in a HIP graph by the plan:
//   k_bat_prep     clear the bucket histogram and the work-queue head
//   k_bat_reduce   per-block sums of the counts, histogram of the sort keys
//   k_bat_top      exclusive scans of the block sums and of the histogram
//   k_bat_apply    per-set offsets; counting-sort scatter of set indices
//   k_batched      persistent generator: each wave pops a group of 64 * spl
//                  sorted sets from the atomic queue, one set per lane at a
//                  time, until the queue is empty
// Sorting puts the longest sets first (and, within equal counts, sets of the
// same kind together: shape < 1 needs the boost), so the 64 sets of a group
// have nearly equal work and the last groups to be popped are the shortest.

namespace bat {
constexpr int kItems = 4;                       // counts per thread in the scan
constexpr int kScanBlock = 256;
constexpr int kPerBlock = kItems * kScanBlock;  // counts per scan block
constexpr int kCountKeys = 4096;                // counts >= 4095 share the top key
constexpr int kBuckets = 2 * kCountKeys;

__device__ __forceinline__ int64_t clamp_count(int64_t c) { return c > 0 ? c : 0; }

// Sort key: longest first, then sets that need the shape < 1 boost after the
// ones that do not.
template <bool BETA>
__device__ __forceinline__ uint32_t sort_key(int64_t c, double pa, double pb)
{
    const int64_t ce = c < kCountKeys - 1 ? c : kCountKeys - 1;
    const bool boost = BETA ? (pa < 1.0 || pb < 1.0) : (pa < 1.0);
    return (uint32_t)((kCountKeys - 1 - ce) * 2 + (boost ? 1 : 0));
}

// Exclusive scan over the block of 64-bit values; `total` gets the block sum.
__device__ __forceinline__ int64_t block_exclusive_scan(int64_t v, int64_t &total, int64_t *lds)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    int64_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) lds[wid] = x;
    __syncthreads();
    int64_t pre = 0, tot = 0;
    for (int w = 0; w < nw; w++) {
        const int64_t s = lds[w];
        pre += (w < wid) ? s : 0;
        tot += s;
    }
    __syncthreads();
    total = tot;
    return pre + x - v;
}
}  // namespace bat

__global__ __launch_bounds__(256) void k_bat_prep(BatchArgs a)
{
    for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < (uint32_t)bat::kBuckets; k += gridDim.x * blockDim.x)
        a.hist[k] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) *a.queue = 0;
}

__global__ void k_bat_queue_reset(uint32_t *q) { *q = 0; }

int launch_queue_reset(const BatchArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL(k_bat_queue_reset, dim3(1), dim3(1), 0, st, a.queue);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? RP_OK : fail(RP_EDEVICE, "queue reset launch: %s", hipGetErrorString(e));
}

template <bool BETA>
__global__ __launch_bounds__(bat::kScanBlock) void k_bat_reduce(BatchArgs a)
{
    __shared__ uint32_t h[bat::kBuckets];
    __shared__ int64_t lds[bat::kScanBlock / 64];
    for (int k = threadIdx.x; k < bat::kBuckets; k += blockDim.x) h[k] = 0;
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * bat::kPerBlock + (uint64_t)threadIdx.x * bat::kItems;
    int64_t sum = 0;
#pragma unroll
    for (int k = 0; k < bat::kItems; k++) {
        const uint64_t j = base + k;
        if (j < a.n_sets) {
            const int64_t c = bat::clamp_count(a.count[j]);
            sum += c;
            atomicAdd(&h[bat::sort_key<BETA>(c, a.pa[j], BETA ? a.pb[j] : 1.0)], 1u);
        }
    }
    int64_t total;
    (void)bat::block_exclusive_scan(sum, total, lds);
    if (threadIdx.x == 0) a.block_sums[blockIdx.x] = total;
    for (int k = threadIdx.x; k < bat::kBuckets; k += blockDim.x)
        if (h[k]) atomicAdd(&a.hist[k], h[k]);
}

// One block: exclusive scans of the block sums (in place) and of the
// histogram (in place: bucket k then holds the first position of key k).
__global__ __launch_bounds__(1024) void k_bat_top(BatchArgs a, uint64_t nblocks)
{
    __shared__ int64_t lds[1024 / 64];
    int64_t carry = 0;
    for (uint64_t base = 0; base < nblocks; base += blockDim.x) {
        const uint64_t i = base + threadIdx.x;
        const int64_t v = i < nblocks ? a.block_sums[i] : 0;
        int64_t tot;
        const int64_t ex = bat::block_exclusive_scan(v, tot, lds);
        if (i < nblocks) a.block_sums[i] = carry + ex;
        carry += tot;
    }
    carry = 0;
    for (int base = 0; base < bat::kBuckets; base += blockDim.x) {
        const int i = base + threadIdx.x;
        const int64_t v = i < bat::kBuckets ? a.hist[i] : 0;
        int64_t tot;
        const int64_t ex = bat::block_exclusive_scan(v, tot, lds);
        if (i < bat::kBuckets) a.hist[i] = (uint32_t)(carry + ex);
        carry += tot;
    }
}

template <bool BETA>
__global__ __launch_bounds__(bat::kScanBlock) void k_bat_apply(BatchArgs a)
{
    __shared__ int64_t lds[bat::kScanBlock / 64];
    const uint64_t base = (uint64_t)blockIdx.x * bat::kPerBlock + (uint64_t)threadIdx.x * bat::kItems;
    int64_t c[bat::kItems];
    int64_t sum = 0;
#pragma unroll
    for (int k = 0; k < bat::kItems; k++) {
        const uint64_t j = base + k;
        c[k] = j < a.n_sets ? bat::clamp_count(a.count[j]) : 0;
        sum += c[k];
    }
    int64_t total;
    int64_t off = bat::block_exclusive_scan(sum, total, lds) + a.block_sums[blockIdx.x];
#pragma unroll
    for (int k = 0; k < bat::kItems; k++) {
        const uint64_t j = base + k;
        if (j < a.n_sets) {
            a.offsets[j] = off;
            const uint32_t key = bat::sort_key<BETA>(c[k], a.pa[j], BETA ? a.pb[j] : 1.0);
            a.order[atomicAdd(&a.hist[key], 1u)] = (uint32_t)j;
        }
        off += c[k];
    }
}

// Persistent generator.  Lane l of a wave that popped group g works through
// the sorted positions g*64*spl + s*64 + l, s = 0 .. spl-1, moving to its next
// set as soon as the current one is done.
template <class E, bool BETA, bool BX = false>
__global__ __launch_bounds__(256) void k_batched(BatchArgs a)
{
    __shared__ ZigLds zt;
    __shared__ LogLds lt;
    load_zig<RP_NORM>(&zt, a.f.flags);
    load_logt(&lt);
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const uint64_t n = a.n_sets;
    const uint64_t group = 64ull * (uint64_t)a.spl;
    for (;;) {
        uint32_t g = 0;
        if (lane == 0) g = atomicAdd(a.queue, 1u);
        g = __shfl(g, 0, 64);
        const uint64_t first = (uint64_t)g * group;
        if (first >= n) break;
        int s = 0;
        uint64_t idx = first + lane;
        bool valid = false, bad = false;
        uint32_t j = 0;
        int64_t cnt = 0, t = 0;
        double *out = nullptr;
        E eng;
        GamMachine<BETA, false, BX> gm;
        for (;;) {
            if (s < a.spl && !valid) {
                // open the next set of this lane (or skip past the end)
                idx = first + (uint64_t)s * 64 + lane;
                if (idx < n) {
                    j = a.order[idx];
                    cnt = bat::clamp_count(a.count[j]);
                    out = a.out + a.offsets[j];
                    const double pa = a.pa[j];
                    const double pb = BETA ? a.pb[j] : 1.0;
                    bad = !(pa > 0.0) || !(pb > 0.0);
                    if (!bad) {
                        eng.load(a.f, j);
                        gm.set(pa, pb);
                    }
                    valid = true;
                    t = 0;
                } else {
                    s = a.spl;
                }
            }
            if (!valid) break;
            if (t < cnt) {
                if (bad) {
                    out[t++] = __builtin_nan("");
                } else {
                    double v;
                    if (gm.step(eng, &zt, &lt, v)) out[t++] = v;
                }
            } else {
                if (!bad) eng.store(a.f, j);
                valid = false;
                s++;
            }
        }
    }
}

template <class E>
static int launch_batched_e(const BatchArgs &a, bool beta, unsigned grid, unsigned block, hipStream_t st)
{
    const bool bx = (a.f.flags & kFlagBitexact) != 0;
    if (beta && bx)
        hipLaunchKernelGGL((k_batched<E, true, true>), dim3(grid), dim3(block), 0, st, a);
    else if (beta)
        hipLaunchKernelGGL((k_batched<E, true, false>), dim3(grid), dim3(block), 0, st, a);
    else if (bx)
        hipLaunchKernelGGL((k_batched<E, false, true>), dim3(grid), dim3(block), 0, st, a);
    else
        hipLaunchKernelGGL((k_batched<E, false, false>), dim3(grid), dim3(block), 0, st, a);
    return RP_OK;
}

int launch_batched_gen(int engine, const BatchArgs &a, bool beta, unsigned grid, unsigned block, hipStream_t st)
{
    switch (engine) {
    case RP_X256PP: launch_batched_e<LaneX256>(a, beta, grid, block, st); break;
    case RP_X256SS: launch_batched_e<LaneX256SS>(a, beta, grid, block, st); break;
    case RP_SQUARES: launch_batched_e<LaneSquares>(a, beta, grid, block, st); break;
    case RP_XORO128: launch_batched_e<LaneXoro128>(a, beta, grid, block, st); break;
    case RP_XS128: launch_batched_e<LaneXs128>(a, beta, grid, block, st); break;
    case RP_CHACHA20: launch_batched_e<LaneChacha>(a, beta, grid, block, st); break;
    case RP_PCG64: launch_batched_e<LanePcg>(a, beta, grid, block, st); break;
    case RP_PHILOX4X32: launch_batched_e<LanePhilox32>(a, beta, grid, block, st); break;
    case RP_PHILOX: launch_batched_e<LanePhilox64>(a, beta, grid, block, st); break;
    case RP_SFC64: launch_batched_e<LaneSfc64>(a, beta, grid, block, st); break;
    case RP_CWG128: launch_batched_e<LaneCwg128>(a, beta, grid, block, st); break;
    case RP_X256PPS: launch_batched_e<LaneX256Simd>(a, beta, grid, block, st); break;
    case RP_X256SSS: launch_batched_e<LaneX256SSSimd>(a, beta, grid, block, st); break;
    case RP_SFC64S: launch_batched_e<LaneSfc64Simd>(a, beta, grid, block, st); break;
    case RP_RANLUX: launch_batched_e<LaneRanlux>(a, beta, grid, block, st); break;
    default: return fail(RP_EINVAL, "unknown engine");
    }
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? RP_OK : fail(RP_EDEVICE, "batched launch: %s", hipGetErrorString(e));
}

int launch_batched_setup(const BatchArgs &a, bool beta, hipStream_t st)
{
    const uint64_t nb = (a.n_sets + bat::kPerBlock - 1) / bat::kPerBlock;
    hipLaunchKernelGGL(k_bat_prep, dim3(8), dim3(256), 0, st, a);
    if (beta) {
        hipLaunchKernelGGL(k_bat_reduce<true>, dim3((unsigned)nb), dim3(bat::kScanBlock), 0, st, a);
        hipLaunchKernelGGL(k_bat_top, dim3(1), dim3(1024), 0, st, a, nb);
        hipLaunchKernelGGL(k_bat_apply<true>, dim3((unsigned)nb), dim3(bat::kScanBlock), 0, st, a);
    } else {
        hipLaunchKernelGGL(k_bat_reduce<false>, dim3((unsigned)nb), dim3(bat::kScanBlock), 0, st, a);
        hipLaunchKernelGGL(k_bat_top, dim3(1), dim3(1024), 0, st, a, nb);
        hipLaunchKernelGGL(k_bat_apply<false>, dim3((unsigned)nb), dim3(bat::kScanBlock), 0, st, a);
    }
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? RP_OK : fail(RP_EDEVICE, "batched setup launch: %s", hipGetErrorString(e));
}

int batched_blocks_for_scan(uint64_t n_sets) { return (int)((n_sets + bat::kPerBlock - 1) / bat::kPerBlock); }
int batched_buckets() { return bat::kBuckets; }
