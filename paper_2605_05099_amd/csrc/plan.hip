// plan.hip -- batched gamma / beta: plan object, graph capture and autotuner.
//
// A plan owns the scratch of the batched launch sequence (per-set offsets,
// sorted set order, key histogram, scan block sums, queue head), the launch
// configuration of the persistent generator, and the HIP graph that records
// the whole sequence for one set of arguments.  A call whose arguments match
// the recorded ones replays the graph with one hipGraphLaunch; otherwise the
// sequence is recorded again first.  No memset node is recorded: the queue
// head and histogram are cleared by a kernel at the start of the sequence.
#include <hip/hip_runtime.h>

#include "rp_internal.h"

using namespace rp;

struct rp_plan {
    int device = 0;
    int cus = 256;
    hipStream_t cap = nullptr;  // private stream used for capture and tuning
    // scratch
    uint64_t cap_sets = 0, cap_blocks = 0;
    int64_t *offsets = nullptr;
    uint32_t *order = nullptr;
    int64_t *block_sums = nullptr;
    uint32_t *hist = nullptr;   // kBuckets entries followed by the queue head
    // generator configuration
    int block = 256, blocks_per_cu = 8, spl = 1;
    bool tuned = false;
    // recorded graph and the arguments it was recorded with
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // every pointer the recorded kernels read or write is part of the key, so
    // a new set whose state arrays reuse an old address is never served by a
    // graph that holds the old set's other array
    struct Key {
        int beta, engine, device, block, blocks_per_cu, spl;
        const void *words, *phase, *pa, *pb, *count, *out;
        uint64_t n_sets, n_streams;
        bool operator==(const Key &o) const
        {
            return beta == o.beta && engine == o.engine && device == o.device && block == o.block &&
                   blocks_per_cu == o.blocks_per_cu && spl == o.spl && words == o.words && phase == o.phase &&
                   pa == o.pa && pb == o.pb && count == o.count && out == o.out && n_sets == o.n_sets &&
                   n_streams == o.n_streams;
        }
    } key{};
    bool have_key = false;
};

namespace {

int hip_fail(hipError_t e, const char *what)
{
    return fail(RP_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

void drop_graph(rp_plan *p)
{
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->exec = nullptr;
    p->graph = nullptr;
    p->have_key = false;
}

void free_scratch(rp_plan *p)
{
    (void)hipFree(p->offsets);
    (void)hipFree(p->order);
    (void)hipFree(p->block_sums);
    (void)hipFree(p->hist);
    p->offsets = nullptr;
    p->order = nullptr;
    p->block_sums = nullptr;
    p->hist = nullptr;
    p->cap_sets = p->cap_blocks = 0;
}

int ensure_scratch(rp_plan *p, uint64_t n_sets)
{
    if (n_sets <= p->cap_sets && p->hist) return RP_OK;
    drop_graph(p);  // the recorded graph points at the old buffers
    free_scratch(p);
    const uint64_t nb = (uint64_t)batched_blocks_for_scan(n_sets);
    hipError_t e = hipMalloc((void **)&p->offsets, n_sets * sizeof(int64_t));
    if (e == hipSuccess) e = hipMalloc((void **)&p->order, n_sets * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc((void **)&p->block_sums, nb * sizeof(int64_t));
    if (e == hipSuccess) e = hipMalloc((void **)&p->hist, (batched_buckets() + 64) * sizeof(uint32_t));
    if (e != hipSuccess) {
        free_scratch(p);
        return fail(RP_ENOMEM, "batched plan scratch for %llu sets: %s", (unsigned long long)n_sets,
                    hipGetErrorString(e));
    }
    p->cap_sets = n_sets;
    p->cap_blocks = nb;
    return RP_OK;
}

BatchArgs make_args(rp_plan *p, rp_streams *s, const double *pa, const double *pb, const int64_t *count,
                    uint64_t n_sets, double *out, int spl)
{
    BatchArgs a{};
    a.f.words = s->d_words;
    a.f.phase = s->d_phase;
    a.f.n = s->n;
    a.f.flags = settings_flags(s);
    a.pa = pa;
    a.pb = pb;
    a.count = count;
    a.n_sets = n_sets;
    a.out = out;
    a.offsets = p->offsets;
    a.order = p->order;
    a.hist = p->hist;
    a.block_sums = p->block_sums;
    a.queue = p->hist + batched_buckets();
    a.spl = spl;
    return a;
}

int validate(const char *who, rp_streams *s, const double *pa, const double *pb, bool beta, const int64_t *count,
             uint64_t n_sets, double *out, rp_plan *p)
{
    if (!s || !p) return fail(RP_ENULL, "%s: NULL streams or plan", who);
    if (n_sets == 0) return 1;
    if (!pa || !count || !out || (beta && !pb)) return fail(RP_ENULL, "%s: NULL device pointer", who);
    if (n_sets > s->n) return fail(RP_EINVAL, "%s: %llu sets but only %llu substreams", who,
                                   (unsigned long long)n_sets, (unsigned long long)s->n);
    if (n_sets > 0xFFFFFFFFull) return fail(RP_EINVAL, "%s: more than 2^32 - 1 sets", who);
    if ((uintptr_t)pa % 8 || (uintptr_t)count % 8 || (uintptr_t)out % 8 || (beta && (uintptr_t)pb % 8))
        return fail(RP_EINVAL, "%s: pointers not aligned to 8 bytes", who);
    return 0;
}

int record(rp_plan *p, rp_streams *s, const BatchArgs &a, bool beta)
{
    drop_graph(p);
    hipError_t e = hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "batched: begin capture");
    int rc = launch_batched_setup(a, beta, p->cap);
    const unsigned grid = (unsigned)(p->cus * p->blocks_per_cu);
    if (rc == RP_OK) rc = launch_batched_gen(s->engine, a, beta, grid, (unsigned)p->block, p->cap);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(p->cap, &g);
    if (rc != RP_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "batched: end capture");
    p->graph = g;
    e = hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        drop_graph(p);
        return hip_fail(e, "batched: graph instantiate");
    }
    return RP_OK;
}

int run_batched(const char *who, rp_streams *s, const double *pa, const double *pb, bool beta, const int64_t *count,
                uint64_t n_sets, double *out, rp_plan *p, void *hip_stream)
{
    int rc = validate(who, s, pa, pb, beta, count, n_sets, out, p);
    if (rc) return rc > 0 ? RP_OK : rc;
    rc = ensure_device_tables();
    if (rc) return rc;
    rc = ensure_scratch(p, n_sets);
    if (rc) return rc;
    rp_plan::Key k{beta ? 1 : 0, s->engine, s->device, p->block, p->blocks_per_cu, p->spl,
                   s->d_words, s->d_phase, pa, pb, count, out, n_sets, s->n};
    if (!p->have_key || !(k == p->key)) {
        rc = record(p, s, make_args(p, s, pa, pb, count, n_sets, out, p->spl), beta);
        if (rc) return rc;
        p->key = k;
        p->have_key = true;
    }
    const hipError_t e = hipGraphLaunch(p->exec, (hipStream_t)hip_stream);
    return e == hipSuccess ? RP_OK : hip_fail(e, "batched: graph launch");
}

}  // namespace

extern "C" int rp_plan_create(rp_plan **out)
{
    if (!out) return fail(RP_ENULL, "rp_plan_create: NULL out");
    *out = nullptr;
    rp_plan *p = new rp_plan;
    hipError_t e = hipGetDevice(&p->device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&p->cus, hipDeviceAttributeMultiprocessorCount, p->device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking);
    if (e != hipSuccess) {
        delete p;
        return hip_fail(e, "rp_plan_create");
    }
    *out = p;
    return RP_OK;
}

extern "C" void rp_plan_free(rp_plan *p)
{
    if (!p) return;
    drop_graph(p);
    free_scratch(p);
    if (p->cap) (void)hipStreamDestroy(p->cap);
    delete p;
}

extern "C" int rp_plan_set_config(rp_plan *p, int block, int blocks_per_cu, int sets_per_lane)
{
    if (!p) return fail(RP_ENULL, "rp_plan_set_config: NULL plan");
    if (block < 64 || block > 256 || block % 64 || blocks_per_cu < 1 || blocks_per_cu > 64 || sets_per_lane < 1 ||
        sets_per_lane > 16)
        return fail(RP_EINVAL, "rp_plan_set_config: block %d (64..256, multiple of 64), blocks/CU %d (1..64), "
                               "sets/lane %d (1..16)", block, blocks_per_cu, sets_per_lane);
    p->block = block;
    p->blocks_per_cu = blocks_per_cu;
    p->spl = sets_per_lane;
    return RP_OK;
}

extern "C" int rp_plan_get_config(const rp_plan *p, int *block, int *blocks_per_cu, int *sets_per_lane)
{
    if (!p || !block || !blocks_per_cu || !sets_per_lane) return fail(RP_ENULL, "rp_plan_get_config: NULL argument");
    *block = p->block;
    *blocks_per_cu = p->blocks_per_cu;
    *sets_per_lane = p->spl;
    return p->tuned ? 1 : 0;
}

extern "C" int rp_gamma_batched(rp_streams *s, const double *d_alpha, const int64_t *d_count, uint64_t n_sets,
                                double *d_out, rp_plan *plan, void *hip_stream)
{
    return run_batched("rp_gamma_batched", s, d_alpha, nullptr, false, d_count, n_sets, d_out, plan, hip_stream);
}

extern "C" int rp_beta_batched(rp_streams *s, const double *d_a, const double *d_b, const int64_t *d_count,
                               uint64_t n_sets, double *d_out, rp_plan *plan, void *hip_stream)
{
    return run_batched("rp_beta_batched", s, d_a, d_b, true, d_count, n_sets, d_out, plan, hip_stream);
}

// Times the generator for each candidate configuration on a copy of the
// substreams (the caller's substreams are not advanced) and keeps the
// fastest.  d_out is overwritten.  Synchronous.
extern "C" int rp_plan_autotune(rp_plan *p, rp_streams *s, int beta, const double *d_pa, const double *d_pb,
                                const int64_t *d_count, uint64_t n_sets, double *d_out)
{
    int rc = validate("rp_plan_autotune", s, d_pa, d_pb, beta != 0, d_count, n_sets, d_out, p);
    if (rc) return rc > 0 ? RP_OK : rc;
    rc = ensure_device_tables();
    if (rc) return rc;
    rc = ensure_scratch(p, n_sets);
    if (rc) return rc;
    // inputs may still be in flight on the caller's stream
    hipError_t se = hipDeviceSynchronize();
    if (se != hipSuccess) return hip_fail(se, "rp_plan_autotune: synchronize");
    rp_streams *copy = nullptr;
    rc = rp_streams_duplicate(s, &copy);
    if (rc) return rc;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        rp_streams_free(copy);
        return hip_fail(e, "rp_plan_autotune: events");
    }
    static const int kBlocks[] = {64, 128, 256};
    static const int kPerCu[] = {2, 4, 6, 8, 12, 16};
    static const int kSpl[] = {1, 2};
    float best = 1e30f;
    int bb = p->block, bp = p->blocks_per_cu, bs = p->spl;
    BatchArgs a = make_args(p, copy, d_pa, d_pb, d_count, n_sets, d_out, 1);
    rc = launch_batched_setup(a, beta != 0, p->cap);
    for (int blk : kBlocks) {
        for (int pc : kPerCu) {
            // keep the resident waves per CU in a range that fits: at most
            // 32 waves of 256-thread blocks is 8 blocks
            if (blk * pc > 64 * 32) continue;
            for (int spl : kSpl) {
                if (rc) break;
                a.spl = spl;
                const unsigned grid = (unsigned)(p->cus * pc);
                float ms = 0.0f;
                for (int rep = 0; rep < 3 && rc == RP_OK; rep++) {
                    rc = launch_queue_reset(a, p->cap);
                    if (rc) break;
                    (void)hipEventRecord(e0, p->cap);
                    rc = launch_batched_gen(copy->engine, a, beta != 0, grid, (unsigned)blk, p->cap);
                    (void)hipEventRecord(e1, p->cap);
                    e = hipEventSynchronize(e1);
                    if (e != hipSuccess) {
                        rc = hip_fail(e, "rp_plan_autotune: run");
                        break;
                    }
                    float t = 0.0f;
                    (void)hipEventElapsedTime(&t, e0, e1);
                    if (rep > 0) ms += t;  // first run warms up
                }
                if (rc == RP_OK && ms < best) {
                    best = ms;
                    bb = blk;
                    bp = pc;
                    bs = spl;
                }
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    rp_streams_free(copy);
    if (rc) return rc;
    drop_graph(p);
    p->block = bb;
    p->blocks_per_cu = bp;
    p->spl = bs;
    p->tuned = true;
    return RP_OK;
}
