// rp_internal.h -- structures shared by the host core and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/rp.h"
#include "engines.h"

struct rp_rng {
    int engine = RP_X256PP;
    uint64_t st[32] = {0};  // state words, Table 3 order (32 for the SIMD engines)
    uint32_t phase = 0;     // words used from the current block (block engines)
    uint64_t seed = 0;      // last seed given to rp_seed (base for substreams)
    std::vector<uint32_t> key;
    std::string err;
    bool full_mantissa = true;  // U(0,1) by method 1 (53/24 bits); false: method 2 (52/23)
    bool squeeze = true;        // ziggurat wedge tests decided by the squeeze where it can
    bool bitexact = false;      // every exp / log / log1p / pow of a sampler correctly rounded
};

struct rp_streams {
    int engine = RP_X256PP;
    uint64_t n = 0;
    int nwords = 0;            // state words per substream
    uint64_t *d_words = nullptr;  // SoA: word k of substream i at [k * n + i]
    uint32_t *d_phase = nullptr;  // n entries
    int device = 0;
    bool full_mantissa = true;    // taken from the base stream at creation
    bool squeeze = true;          // taken from the base stream at creation
    bool bitexact = false;        // taken from the base stream at creation
};

namespace rp {

// ---- host core -------------------------------------------------------------
int state_words(int engine);
int block_words(int engine);
void set_error(const char *fmt, ...);
void set_error_rng(rp_rng *rng, const char *fmt, ...);
int fail(int code, const char *fmt, ...);

// ranlux++ multiplier A = a^2048 mod m and its power table (host)
const uint64_t *ranlux_A();
const uint32_t *ranlux_B();

// PCG64 power tables: A^k and G_k = 1 + A + ... + A^(k-1) (mod 2^128)
struct PcgAffine {
    u128 mult, plus;  // s -> mult * s + plus * inc
};

// device-side constant tables (uploaded once per device)
int ensure_device_tables();

// internal bits of FillArgs::flags (above the public per-call flags)
constexpr int kFlagNoSqueeze = 1 << 16;  // wedge tests evaluate f(x) every time
constexpr int kFlagBitexact = 1 << 17;   // correctly rounded elementary functions

// the FillArgs flag bits a substream set's settings imply
inline int settings_flags(const rp_streams *s)
{
    return (s->squeeze ? 0 : kFlagNoSqueeze) | (s->bitexact ? kFlagBitexact : 0);
}

// ---- kernel launchers (fill.hip) -------------------------------------------
struct FillArgs {
    uint64_t *words;   // SoA state
    uint32_t *phase;
    uint64_t n;        // substreams
    uint64_t per_stream;
    void *out;
    uint64_t bound;    // Lemire bound (0 = full range)
    uint64_t thresh;   // Lemire threshold (2^w - b) mod b
    int flags;
    double xp[4];      // transform parameters of rp_fill_law (host-formed)
};

int launch_fill(int engine, int dist, int dtype, const FillArgs &a, hipStream_t stream);
// rp_fill_law: the base fill of the law with its transform fused at the store
int launch_fill_law(int engine, int law, bool f32, const FillArgs &a, hipStream_t stream);
// rp_fill_law for the laws of several base draws per value (k_samplers.h)
int launch_fill_mix(int engine, int law, bool f32, const FillArgs &a, hipStream_t stream);

// lane-per-substream samplers (k_samplers.h)
struct SampArgs {
    FillArgs f;           // substream states (f.n = substreams, f.per_stream for moments)
    uint64_t count;       // lanes: substreams (moments) or elements
    const float *pa;      // per-element shape (gamma) or a (beta)
    const float *pb;      // per-element b (beta)
    float *z;             // per-element result
    double *sum, *sumsq;  // per-substream moments
    int advance;          // rows of normals: store the advanced states
};
// batched gamma / beta (k_batched.h)
struct BatchArgs {
    FillArgs f;              // substream states (set j uses substream j)
    const double *pa, *pb;   // per-set shape (gamma) or a, b (beta)
    const int64_t *count;    // per-set counts (negative counts as 0)
    uint64_t n_sets;
    double *out;             // sum of counts values, set-major
    int64_t *offsets;        // scratch: n_sets exclusive prefix sums
    uint32_t *order;         // scratch: n_sets sorted set indices
    uint32_t *hist;          // scratch: sort-key histogram / bucket cursors
    int64_t *block_sums;     // scratch: one per scan block
    uint32_t *queue;         // scratch: work-queue head
    int spl;                 // sets per lane per popped group
};
int launch_batched_setup(const BatchArgs &a, bool beta, hipStream_t stream);
int launch_batched_gen(int engine, const BatchArgs &a, bool beta, unsigned grid, unsigned block, hipStream_t stream);
int launch_queue_reset(const BatchArgs &a, hipStream_t stream);
int batched_blocks_for_scan(uint64_t n_sets);
int batched_buckets();

// serial split of one stream (k_serial.h)
constexpr int kSerJt = 304;
struct SerialArgs {
    uint64_t base[9];      // engine state words at the start (Table 3 order)
    uint32_t phase;        // words used from the current block
    uint32_t lanes;        // generator lanes
    uint64_t C;            // words per lane (a multiple of the block size)
    uint64_t words;        // words generated: positions 0 .. words-1
    uint64_t jt[kSerJt];   // jump data, engine specific
    FillArgs fa;           // out, bound, thresh, flags
    uint64_t n;            // outputs wanted
    uint64_t units;        // attempts start at units 0 .. units-1 (words or halves)
    uint64_t *wbuf;        // generated words (rejection samplers)
    uint8_t *cexit;        // per chunk: exclusive prefix map within its block
    uint32_t *ccount;
    uint8_t *bexit;        // per block: the block's map
    uint32_t *bcount;
    uint8_t *bentry;       // per block: entry offset and output base
    uint64_t *bbase;
    uint64_t *result;      // end unit of the n-th output, outputs available, overflow
    uint64_t nchunks, nblocks;
};
int launch_serial_fixed(int engine, int dist, int dtype, const SerialArgs &a, hipStream_t stream);
int launch_serial_stitch(int engine, int dist, int dtype, const SerialArgs &a, hipStream_t stream);
int serial_chunk_units();
int serial_entries();
int serial_chunks_per_block();

int launch_moments(int engine, const SampArgs &s, hipStream_t stream);
// batched permutations (perm) or samples (k_discrete.h); f.per_stream = n or
// k, f.bound = n for samples; tab: 2^tbits entries per substream (Floyd)
int launch_discrete(int engine, bool perm, const FillArgs &f, uint32_t *tab, int tbits, hipStream_t stream);
int launch_gamma_elem(int engine, const SampArgs &s, bool beta, hipStream_t stream);
// rows of normals: z[i * d + t] = t-th normal of substream i, binary32
int launch_norm_rows(int engine, const SampArgs &s, hipStream_t stream);

}  // namespace rp
