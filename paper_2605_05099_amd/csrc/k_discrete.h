// k_discrete.h -- batched permutations and samples (Section 3.2): one
// instance per substream, one lane per instance.  Every draw is a 32-bit
// bounded integer by Lemire's method on the substream's 32-bit items (low
// half first, a half left over at the end of the call dropped), so each
// instance equals the serial definition on its substream.  Included by
// fill.hip (lane engines, FillArgs).

// 32-bit items of a lane engine
template <class E>
struct Items32 {
    E &eng;
    bool have = false;
    uint32_t hi = 0;
    __device__ explicit Items32(E &e) : eng(e) {}
    __device__ uint32_t next()
    {
        if (have) {
            have = false;
            return hi;
        }
        const uint64_t w = eng.next();
        hi = (uint32_t)(w >> 32);
        have = true;
        return (uint32_t)w;
    }
    // uniform on {0 .. b-1}, b >= 1: Lemire's multiply, with the threshold
    // (2^32 - b) mod b formed only when the low half is below b
    __device__ uint32_t bounded(uint32_t b)
    {
        eng.reserve(1);
        uint64_t p = (uint64_t)next() * b;
        uint32_t low = (uint32_t)p;
        if (low < b) {
            const uint32_t thr = (0u - b) % b;
            while (low < thr) {
                eng.reserve(1);
                p = (uint64_t)next() * b;
                low = (uint32_t)p;
            }
        }
        return (uint32_t)(p >> 32);
    }
};

// Fisher-Yates (Durstenfeld): row starts as the identity; for j from n-1
// down to 1, swap entries j and r, r uniform on {0 .. j}.  f.per_stream = n.
template <class E>
__global__ __launch_bounds__(256) void k_permutations(FillArgs f)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= f.n) return;
    const uint32_t n = (uint32_t)f.per_stream;
    uint32_t *row = (uint32_t *)f.out + i * (uint64_t)n;
    for (uint32_t q = 0; q < n; q++) row[q] = q;
    E eng;
    eng.load(f, i);
    Items32<E> it(eng);
    for (uint32_t j = n - 1; j >= 1; j--) {
        const uint32_t r = it.bounded(j + 1);
        const uint32_t t = row[j];
        row[j] = row[r];
        row[r] = t;
    }
    eng.store(f, i);
}

// Rows of at most CAP entries (512: 64 KiB, two blocks per CU; 1024:
// 128 KiB of gfx950's 160 KiB, one block): the 64 rows of a one-wavefront
// block live in LDS as 16-bit entries, so the swaps are LDS accesses
// instead of dependent reads of HBM; the identity is written and the
// finished rows are stored cooperatively (consecutive lanes on consecutive
// entries).
template <class E, uint32_t CAP>
__global__ __launch_bounds__(64) void k_permutations_lds(FillArgs f)
{
    __shared__ uint16_t rows[64 * CAP];
    const uint32_t n = (uint32_t)f.per_stream;
    const int lane = (int)threadIdx.x;
    const uint64_t id0 = (uint64_t)blockIdx.x * 64;
    const uint64_t i = id0 + (uint64_t)lane;
    for (uint32_t q = (uint32_t)lane; q < 64 * n; q += 64) rows[q] = (uint16_t)(q % n);
    wave_sync();
    if (i < f.n) {
        uint16_t *row = rows + (uint32_t)lane * n;
        E eng;
        eng.load(f, i);
        Items32<E> it(eng);
        for (uint32_t j = n - 1; j >= 1; j--) {
            const uint32_t r = it.bounded(j + 1);
            const uint16_t t = row[j];
            row[j] = row[r];
            row[r] = t;
        }
        eng.store(f, i);
    }
    wave_sync();
    uint32_t *out = (uint32_t *)f.out;
    const uint32_t rows_here = f.n - id0 < 64 ? (uint32_t)(f.n - id0) : 64u;
    for (uint32_t rr = 0; rr < rows_here; rr++)
        for (uint32_t q = (uint32_t)lane; q < n; q += 64) out[(id0 + rr) * n + q] = rows[rr * n + q];
}

// k distinct elements of {0 .. n-1} per substream (f.per_stream = k,
// f.bound = n).  k <= n/2: Floyd's algorithm, for j from n-k to n-1 draw t
// on {0 .. j} and append t, or j when t is already in the sample; the
// membership test uses an open-addressing table of 2^tbits >= 2k entries
// per substream (f.words-independent workspace `tab`, cleared here).
// k > n/2: reservoir (Vitter's algorithm R), the row itself being the
// reservoir.
static constexpr uint32_t kEmpty = 0xffffffffu;

template <class E>
__global__ __launch_bounds__(256) void k_sample(FillArgs f, uint32_t *tab, int tbits)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= f.n) return;
    const uint32_t k = (uint32_t)f.per_stream, n = (uint32_t)f.bound;
    uint32_t *row = (uint32_t *)f.out + i * (uint64_t)k;
    E eng;
    eng.load(f, i);
    Items32<E> it(eng);
    if (2 * (uint64_t)k <= n) {
        const uint32_t cap = 1u << tbits, mask = cap - 1;
        uint32_t *h = tab + i * (uint64_t)cap;
        for (uint32_t q = 0; q < cap; q++) h[q] = kEmpty;
        for (uint32_t c = 0; c < k; c++) {
            const uint32_t j = n - k + c;
            const uint32_t t = it.bounded(j + 1);
            // look t up; insert the appended value (t, or j if t is present;
            // j itself is never present: every earlier value is below j)
            uint32_t s = (t * 0x9E3779B1u) >> (32 - tbits);
            bool seen = false;
            while (h[s] != kEmpty) {
                if (h[s] == t) {
                    seen = true;
                    break;
                }
                s = (s + 1) & mask;
            }
            const uint32_t v = seen ? j : t;
            if (seen) {
                s = (v * 0x9E3779B1u) >> (32 - tbits);
                while (h[s] != kEmpty) s = (s + 1) & mask;
            }
            h[s] = v;
            row[c] = v;
        }
    } else {
        for (uint32_t q = 0; q < k; q++) row[q] = q;
        for (uint32_t v = k; v < n; v++) {
            const uint32_t j = it.bounded(v + 1);
            if (j < k) row[j] = v;
        }
    }
    eng.store(f, i);
}

template <class E>
static void launch_discrete_e(bool perm, const FillArgs &f, uint32_t *tab, int tbits, hipStream_t st)
{
    const dim3 grid((unsigned)((f.n + 255) / 256)), block(256);
    const dim3 grid64((unsigned)((f.n + 63) / 64));
    if (perm && f.per_stream <= 512) hipLaunchKernelGGL((k_permutations_lds<E, 512>), grid64, dim3(64), 0, st, f);
    else if (perm && f.per_stream <= 1024)
        hipLaunchKernelGGL((k_permutations_lds<E, 1024>), grid64, dim3(64), 0, st, f);
    else if (perm) hipLaunchKernelGGL(k_permutations<E>, grid, block, 0, st, f);
    else hipLaunchKernelGGL(k_sample<E>, grid, block, 0, st, f, tab, tbits);
}

int launch_discrete(int engine, bool perm, const FillArgs &f, uint32_t *tab, int tbits, hipStream_t st)
{
    switch (engine) {
    case RP_X256PP: launch_discrete_e<LaneX256>(perm, f, tab, tbits, st); break;
    case RP_X256SS: launch_discrete_e<LaneX256SS>(perm, f, tab, tbits, st); break;
    case RP_PCG64: launch_discrete_e<LanePcg>(perm, f, tab, tbits, st); break;
    case RP_PHILOX4X32: launch_discrete_e<LanePhilox32>(perm, f, tab, tbits, st); break;
    case RP_PHILOX: launch_discrete_e<LanePhilox64>(perm, f, tab, tbits, st); break;
    case RP_SFC64: launch_discrete_e<LaneSfc64>(perm, f, tab, tbits, st); break;
    case RP_CWG128: launch_discrete_e<LaneCwg128>(perm, f, tab, tbits, st); break;
    case RP_X256PPS: launch_discrete_e<LaneX256Simd>(perm, f, tab, tbits, st); break;
    case RP_X256SSS: launch_discrete_e<LaneX256SSSimd>(perm, f, tab, tbits, st); break;
    case RP_SFC64S: launch_discrete_e<LaneSfc64Simd>(perm, f, tab, tbits, st); break;
    case RP_RANLUX: launch_discrete_e<LaneRanlux>(perm, f, tab, tbits, st); break;
    case RP_SQUARES: launch_discrete_e<LaneSquares>(perm, f, tab, tbits, st); break;
    case RP_XORO128: launch_discrete_e<LaneXoro128>(perm, f, tab, tbits, st); break;
    case RP_XS128: launch_discrete_e<LaneXs128>(perm, f, tab, tbits, st); break;
    case RP_CHACHA20: launch_discrete_e<LaneChacha>(perm, f, tab, tbits, st); break;
    default: return fail(RP_EINVAL, "unknown engine");
    }
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? RP_OK : fail(RP_EDEVICE, "permutation / sample launch: %s", hipGetErrorString(e));
}
