// Ensembles of circuits of uneven size and depth (the statistics of Sec. IV
// are averages over many random circuit instances), captured once in a HIP
// graph and replayed.
//
// The work of a complex64 register-tile ensemble is cut into items: a run of
// register tiles of one sweep of one instance, or a run of amplitudes of its
// statistics pass.  The items are laid out in one table in the order (round,
// instance, chunk), where the r-th round holds the r-th sweep of every
// instance that has one (then that instance's statistics pass once its
// sweeps are done).  An item of sweep r of instance i needs every item of the
// earlier sweeps of i and nothing else.  Two schedules execute the table:
//
// * round launches (default): one launch per round, whose grid is every item
//   of that round of every instance; kernel boundaries order the rounds, so
//   no item waits and no cross-workgroup fence is needed;
// * persistent (SV_FLAG_BATCH_PERSISTENT): one launch whose resident
//   workgroups take items from a global queue in table order and wait on
//   per-instance completion counters (agent-scope acquire; producers
//   release after their writes).  Items are dequeued in order and only by
//   running workgroups, and every dependency of an item lies earlier in the
//   table, so the earliest unfinished item can always proceed and the waits
//   end; the wait is nevertheless bounded and raises an error flag instead
//   of spinning forever.  On this chip the release of an item costs a
//   write-back of the XCD's L2, so this schedule takes coarse items (256
//   tiles, 2^19 amplitudes of statistics) where the round launches take fine
//   ones (16 tiles, 2^14 amplitudes) for parallelism within a round.
//
// Statistics partial rows are combined per instance in chunk order.
//
// Complex128 ensembles, and circuits whose plan is not made of register
// tiles only, take the plain path: every instance's sweeps and statistics
// pass recorded as ordinary launches in one captured graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "device_common.h"
#include "internal.h"
#include "reduce_common.h"

namespace svi {


// register tiles per work item, and log2 of the amplitudes per statistics
// item (at most; an instance of fewer qubits takes one item), per schedule
constexpr int TPI_ROUND = 16, TPI_PERSISTENT = 256;
constexpr int STAT_BITS_ROUND = 14, STAT_BITS_PERSISTENT = 19;
constexpr int MIN_QUBITS = 14;          // smallest instance of the item tables

struct BRound {                         // one (instance, sweep) run of items
    uint64_t first;                     // table index of its first item
    uint64_t ntiles;                    // tiles (sweep) or amplitudes (statistics)
    const uint8_t *prog;                // sweep program; null for statistics
    int32_t inst;
    int32_t vb;                         // register qubits; 0 for statistics
    int32_t need;                       // items of the instance that precede it
    int32_t nitems;
    int32_t tpi;                        // register tiles per item (multiple of 4)
    int32_t pad;
};

struct BInst {
    cplx<float> *psi;
    double *part;                       // statistics partial rows (16 doubles)
    int32_t n;
    int32_t nchunks;
    int32_t stat_bits;                  // log2 amplitudes per statistics item
    int32_t pad;
};

__global__ void k_zero_u32(unsigned *p, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0u;
}

// Wave-uniform 64-bit value (scalar registers).
__device__ __forceinline__ uint64_t uniform_u64(uint64_t v) {
    return ((uint64_t)__builtin_amdgcn_readfirstlane((unsigned)(v >> 32)) << 32) |
           (uint64_t)(unsigned)__builtin_amdgcn_readfirstlane((unsigned)v);
}

// One item: up to R.tpi register tiles (R.tpi / 4 per wave), or one
// statistics chunk written as a partial row of the instance.
template <int VB>
__device__ __forceinline__ void run_item(const BRound &R, const BInst &I, uint64_t chunk, int lane, int wave,
                                         double *red, unsigned long long *zred) {
    if (R.vb > 0) {
#pragma unroll 1
        for (int i = 0; i < R.tpi / 4; i++) {
            const uint64_t tile = chunk * (uint64_t)R.tpi + wave + 4 * i;
            if (tile >= R.ntiles) break;
            regtile_apply<float, VB>(I.psi, R.prog, tile, lane);
        }
        return;
    }
    // S, sum p ln p, sum ln p, sum u^k (k = 1..10), zero count
    double acc[NSTAT];
#pragma unroll
    for (int q = 0; q < NSTAT; q++) acc[q] = 0.0;
    unsigned zeros = 0;
    const double Nd = ldexp(1.0, I.n);
    const gptr<cpx<float>> src =
        (gptr<cpx<float>>)(reinterpret_cast<cpx<float> *>(I.psi) + (chunk << I.stat_bits));
    constexpr int UNR = 8;   // loads in flight per thread
    const int span = 1 << I.stat_bits;   // a multiple of BLOCK * UNR
    for (int j0 = threadIdx.x; j0 < span; j0 += BLOCK * UNR) {
        cpx<float> buf[UNR];
#pragma unroll
        for (int v = 0; v < UNR; v++) {
            buf[v].re = src[j0 + v * BLOCK].re;
            buf[v].im = src[j0 + v * BLOCK].im;
        }
#pragma unroll
        for (int v = 0; v < UNR; v++) stat_add(acc, zeros, prob_of(buf[v]), Nd);
    }
    block_sum<double, NSTAT>(acc, red);
    zeros = wave_sum(zeros);
    if (lane == 0) zred[threadIdx.x >> 6] = zeros;
    __syncthreads();
    double *row = I.part + chunk * 16;
    if (threadIdx.x < NSTAT) row[threadIdx.x] = red[threadIdx.x];
    if (threadIdx.x == NSTAT) row[NSTAT] = (double)(zred[0] + zred[1] + zred[2] + zred[3]);
}

// Sum of an instance's partial rows for quantity q in chunk order (Neumaier).
__device__ __forceinline__ double combine_rows(const BInst &I, int q) {
    double sum = 0.0, c = 0.0;
    for (int b = 0; b < I.nchunks; b++) {
        const double x = I.part[(uint64_t)b * 16 + q];
        const double t = sum + x;
        if (fabs(sum) >= fabs(x)) c += (sum - t) + x;
        else c += (x - t) + sum;
        sum = t;
    }
    return sum + c;
}

// Round schedule: items [item0, item0 + gridDim.x), one per workgroup.
template <int VB>
__global__ __launch_bounds__(BLOCK) void k_batch_round(const BRound *__restrict__ rounds,
                                                       const uint32_t *__restrict__ item_round, uint64_t item0,
                                                       const BInst *__restrict__ insts) {
    __shared__ double red[4 * NSTAT];
    __shared__ unsigned long long zred[4];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint64_t item = item0 + blockIdx.x;
    const BRound &R = rounds[item_round[item]];
    const BInst I = insts[R.inst];
    run_item<VB>(R, I, item - R.first, lane, wave, red, zred);
}

__global__ void k_batch_combine(const BInst *__restrict__ insts, double *__restrict__ results) {
    const BInst I = insts[blockIdx.x];
    if (threadIdx.x <= NSTAT) results[(uint64_t)blockIdx.x * 16 + threadIdx.x] = combine_rows(I, threadIdx.x);
}

// Persistent schedule.
template <int VB>
__global__ __launch_bounds__(BLOCK) void k_batch_persistent(const BRound *__restrict__ rounds,
                                                            const uint32_t *__restrict__ item_round,
                                                            uint64_t total, const BInst *__restrict__ insts,
                                                            unsigned long long *head, unsigned *err,
                                                            unsigned *done, unsigned *stats_done,
                                                            double *__restrict__ results, unsigned spin_limit) {
    __shared__ unsigned long long s_item;
    __shared__ int s_flag;
    __shared__ double red[4 * NSTAT];
    __shared__ unsigned long long zred[4];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(head, 1ull);
        __syncthreads();
        const uint64_t item = uniform_u64(s_item);
        __syncthreads();
        if (item >= total) break;
        const BRound &R = rounds[item_round[item]];
        const int inst = R.inst;
        if (threadIdx.x == 0) {
            int ok = 1;
            unsigned it = 0;
            while (__hip_atomic_load(&done[inst], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) <
                   (unsigned)R.need) {
                if (++it > spin_limit ||
                    __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
                    ok = 0;
                    atomicExch(err, 1u);
                    break;
                }
                __builtin_amdgcn_s_sleep(4);
            }
            s_flag = ok;
        }
        __syncthreads();
        __threadfence();   // acquire for every wave of the workgroup
        if (!__builtin_amdgcn_readfirstlane(s_flag)) continue;   // item given up (error raised)
        const BInst I = insts[inst];
        run_item<VB>(R, I, item - R.first, lane, wave, red, zred);
        __threadfence();   // release this item's writes
        __syncthreads();
        if (threadIdx.x == 0) {
            __hip_atomic_fetch_add(&done[inst], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            int last = 0;
            if (R.vb == 0) {
                const unsigned t = __hip_atomic_fetch_add(&stats_done[inst], 1u, __ATOMIC_ACQ_REL,
                                                          __HIP_MEMORY_SCOPE_AGENT);
                last = t + 1 == (unsigned)R.nitems;
            }
            s_flag = last;
        }
        __syncthreads();
        if (__builtin_amdgcn_readfirstlane(s_flag)) {
            // the instance's last statistics chunk combines its partial rows
            __threadfence();
            if (threadIdx.x <= NSTAT) results[(uint64_t)inst * 16 + threadIdx.x] = combine_rows(I, threadIdx.x);
        }
        __syncthreads();
    }
}

static void finish_stats(const double *r, int n, sv_stats *o) {
    const double N = std::ldexp(1.0, n);
    const double S = r[0];
    const double lnS = std::log(S);
    o->norm = S;
    o->entropy = lnS - r[1] / S;
    o->zero_count = (int64_t)r[NSTAT];
    o->unif_ce = o->zero_count ? INFINITY : lnS - r[2] / N;
    double Sk = 1.0;
    for (int k = 0; k < 10; k++) {
        Sk *= S;
        o->moments[k] = r[3 + k] / N / Sk;
    }
}

static sv_status batch_graph_of_launches(sv_state **sts, const sv_circuit *cs, int64_t count,
                                         const sv_opts *opts, sv_stats *out);

// A captured ensemble and the device memory it uses.
struct EnsembleGraph {
    std::vector<const void *> key;           // schedule, width, then (state data, plan) per instance
    std::vector<std::shared_ptr<Plan>> plans;   // keep the device programs alive
    hipStream_t stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void *mem = nullptr;                     // tables | counters | results | partials
    double *res = nullptr;
    unsigned *err = nullptr;
    void release() {
        if (stream) (void)hipStreamSynchronize(stream);
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (mem) (void)hipFree(mem);
        if (stream) (void)hipStreamDestroy(stream);
        exec = nullptr;
        graph = nullptr;
        mem = nullptr;
        stream = nullptr;
    }
};

// Item table, device memory and the captured graph of one schedule.
static sv_status build_ensemble(sv_state **sts, const std::vector<std::shared_ptr<Plan>> &plans, int64_t count,
                                int vb, bool persistent, EnsembleGraph *g) {
    g->plans = plans;
    std::vector<BRound> rounds;
    std::vector<BInst> insts(count);
    std::vector<int32_t> items_so_far(count, 0);
    // launches of the round schedule: [first item, end item)
    std::vector<std::pair<uint64_t, uint64_t>> launches;
    const int tpi = persistent ? TPI_PERSISTENT : TPI_ROUND;
    auto stat_bits = [&](int n) { return std::min(n, persistent ? STAT_BITS_PERSISTENT : STAT_BITS_ROUND); };
    uint64_t total = 0;
    size_t nrounds = 0;
    for (int64_t i = 0; i < count; i++) nrounds = std::max(nrounds, plans[i]->ops.size() + 1);
    for (size_t r = 0; r < nrounds; r++) {
        const uint64_t round_first = total;
        for (int64_t i = 0; i < count; i++) {
            const Plan &p = *plans[i];
            BRound R{};
            R.inst = (int32_t)i;
            R.need = items_so_far[i];
            R.tpi = tpi;
            if (r < p.ops.size()) {
                const Op &op = p.ops[r];
                R.vb = op.vbits;
                R.prog = (const uint8_t *)p.dprog + op.prog_off;
                R.ntiles = (1ull << sts[i]->n) >> (LANE_BITS + op.vbits);
                R.nitems = (int32_t)((R.ntiles + tpi - 1) / tpi);
            } else if (r == p.ops.size()) {
                R.vb = 0;
                R.prog = nullptr;
                R.ntiles = 1ull << sts[i]->n;
                R.nitems = 1 << (sts[i]->n - stat_bits(sts[i]->n));
            } else {
                continue;
            }
            R.first = total;
            total += (uint64_t)R.nitems;
            items_so_far[i] += R.nitems;
            rounds.push_back(R);
        }
        if (total > round_first) launches.push_back({round_first, total});
    }
    if (rounds.size() >= (1ull << 32)) return fail(SV_ERANGE, "ensemble too large");
    std::vector<uint32_t> item_round(total);
    for (size_t r = 0; r < rounds.size(); r++)
        for (int32_t k = 0; k < rounds[r].nitems; k++) item_round[rounds[r].first + k] = (uint32_t)r;
    size_t part_rows = 0;
    for (int64_t i = 0; i < count; i++) part_rows += (size_t)1 << (sts[i]->n - stat_bits(sts[i]->n));
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t o_rounds = 0;
    const size_t o_items = al(rounds.size() * sizeof(BRound));
    const size_t o_insts = o_items + al(total * sizeof(uint32_t));
    const size_t o_ctl = o_insts + al((size_t)count * sizeof(BInst));
    const size_t nctl = 4 + 2 * (size_t)count;   // head (2 words), err, pad, done[], stats_done[]
    const size_t o_res = o_ctl + al(nctl * sizeof(unsigned));
    const size_t o_part = o_res + al((size_t)count * 16 * sizeof(double));
    const size_t bytes = o_part + part_rows * 16 * sizeof(double);
    hipError_t e = hipMalloc(&g->mem, bytes);
    if (e != hipSuccess) {
        g->mem = nullptr;
        return e == hipErrorOutOfMemory ? fail(SV_ENOMEM, "no device memory for the ensemble tables")
                                        : hip_fail(e, "hipMalloc");
    }
    uint8_t *m = (uint8_t *)g->mem;
    size_t row0 = 0;
    for (int64_t i = 0; i < count; i++) {
        insts[i].psi = (cplx<float> *)sts[i]->data;
        insts[i].n = sts[i]->n;
        insts[i].stat_bits = stat_bits(sts[i]->n);
        insts[i].nchunks = 1 << (sts[i]->n - insts[i].stat_bits);
        insts[i].part = (double *)(m + o_part) + row0 * 16;
        row0 += insts[i].nchunks;
    }
    SV_HIP(hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking));
    SV_HIP(hipMemcpyAsync(m + o_rounds, rounds.data(), rounds.size() * sizeof(BRound), hipMemcpyHostToDevice,
                          g->stream));
    SV_HIP(hipMemcpyAsync(m + o_items, item_round.data(), total * sizeof(uint32_t), hipMemcpyHostToDevice,
                          g->stream));
    SV_HIP(hipMemcpyAsync(m + o_insts, insts.data(), insts.size() * sizeof(BInst), hipMemcpyHostToDevice,
                          g->stream));
    SV_HIP(hipStreamSynchronize(g->stream));
    const BRound *d_rounds = (const BRound *)(m + o_rounds);
    const uint32_t *d_items = (const uint32_t *)(m + o_items);
    const BInst *d_insts = (const BInst *)(m + o_insts);
    unsigned *ctl = (unsigned *)(m + o_ctl);
    g->err = ctl + 2;
    g->res = (double *)(m + o_res);
    int per_cu = 0, dev = 0, ncu = 0;
    auto kp = vb == 3 ? k_batch_persistent<3> : vb == 4 ? k_batch_persistent<4>
            : vb == 5 ? k_batch_persistent<5> : k_batch_persistent<6>;
    auto kr = vb == 3 ? k_batch_round<3> : vb == 4 ? k_batch_round<4> : vb == 5 ? k_batch_round<5> : k_batch_round<6>;
    if (persistent) {
        SV_HIP(hipGetDevice(&dev));
        SV_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
        SV_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kp, BLOCK, 0));
    }
    SV_HIP(hipStreamBeginCapture(g->stream, hipStreamCaptureModeThreadLocal));
    // counters cleared by a kernel (no memset node in the graph)
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(256), 0, g->stream, ctl, (int)nctl);
    if (persistent) {
        // as many workgroups as can be resident at once
        const unsigned grid = (unsigned)std::max(1, ncu * std::max(1, per_cu));
        hipLaunchKernelGGL(kp, dim3(grid), dim3(BLOCK), 0, g->stream, d_rounds, d_items, total, d_insts,
                           (unsigned long long *)ctl, g->err, ctl + 4, ctl + 4 + count, g->res, 1u << 22);
    } else {
        for (const auto &L : launches) {
            // grids of at most 2^31 - 1 workgroups
            for (uint64_t a = L.first; a < L.second; a += 0x7fffffffull) {
                const uint64_t nb = std::min<uint64_t>(L.second - a, 0x7fffffffull);
                hipLaunchKernelGGL(kr, dim3((unsigned)nb), dim3(BLOCK), 0, g->stream, d_rounds, d_items, a,
                                   d_insts);
            }
        }
        hipLaunchKernelGGL(k_batch_combine, dim3((unsigned)count), dim3(64), 0, g->stream, d_insts, g->res);
    }
    e = hipStreamEndCapture(g->stream, &g->graph);
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    SV_HIP(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
    return SV_OK;
}

}  // namespace svi

using namespace svi;

extern "C" sv_status sv_apply_batch(sv_state **sts, const sv_circuit *cs, int64_t count, const sv_opts *opts,
                                    sv_stats *out) {
    if (count < 0 || (count > 0 && (!sts || !cs || !out))) return fail(SV_EINVAL, "bad batch arguments");
    if (count == 0) return SV_OK;
    const sv_dtype dt = sts[0] ? sts[0]->dt : SV_C64;
    hipStream_t user = sts[0] ? sts[0]->stream : nullptr;
    bool tables = dt == SV_C64;
    for (int64_t i = 0; i < count; i++) {
        if (!sts[i] || !sts[i]->data) return fail(SV_EINVAL, "null state in batch");
        if (sts[i]->dt != dt) return fail(SV_EINVAL, "batch states must share a dtype");
        if (sts[i]->stream != user) return fail(SV_EINVAL, "batch states must share a stream");
        if (cs[i].n != sts[i]->n) return fail(SV_EINVAL, "circuit / state size mismatch in batch");
        if (sts[i]->n < MIN_QUBITS) tables = false;
    }
    if (opts && opts->mode != SV_MODE_AUTO && opts->mode != SV_MODE_REGTILE) tables = false;
    if (opts && (opts->flags & SV_FLAG_BATCH_LAUNCHES)) tables = false;
    if (!tables) return batch_graph_of_launches(sts, cs, count, opts, out);
    const bool persistent = opts && (opts->flags & SV_FLAG_BATCH_PERSISTENT);

    // plans (register tiles from |0..0>, one width for the ensemble) and the
    // captured graph; the last ensemble's graph is kept and replayed when the
    // same states, plans and schedule come again
    static EnsembleGraph *last = nullptr;   // kept for the process
    bool fallback = false;
    auto prepare = [&](int vb) -> sv_status {
        std::vector<std::shared_ptr<Plan>> plans(count);
        std::vector<const void *> key;
        key.push_back((const void *)(intptr_t)(persistent ? 1 : 0));
        key.push_back((const void *)(intptr_t)vb);
        for (int64_t i = 0; i < count; i++) {
            PlanRequest rq{};
            rq.n = sts[i]->n;
            rq.dtype = dt;
            rq.mode = SV_MODE_REGTILE;
            rq.tile = vb;
            rq.from_zero = true;
            rq.force_zero = true;
            SV_TRY(get_plan(sts[i], &cs[i], rq, &plans[i]));
            for (const Op &op : plans[i]->ops)
                if (op.type != OP_REGTILE || op.vbits != vb) {
                    fallback = true;
                    return SV_OK;
                }
            key.push_back(sts[i]->data);
            key.push_back(plans[i].get());
        }
        if (last && last->key == key) return SV_OK;
        if (last) {
            last->release();
            delete last;
            last = nullptr;
        }
        EnsembleGraph *g = new EnsembleGraph();
        const sv_status rc = build_ensemble(sts, plans, count, vb, persistent, g);
        if (rc != SV_OK) {
            g->release();
            delete g;
            return rc;
        }
        g->key = key;
        last = g;
        return SV_OK;
    };
    if (user) SV_HIP(hipStreamSynchronize(user));
    else SV_HIP(hipDeviceSynchronize());
    // width: given, or the fastest of 4..6 timed on this ensemble itself
    // (once per list of instance sizes and schedule; the timing runs write
    // the same outputs as the call)
    static std::map<std::vector<int>, int> *width_of = new std::map<std::vector<int>, int>();
    std::vector<int> shape;
    shape.push_back(persistent ? 1 : 0);
    for (int64_t i = 0; i < count; i++) shape.push_back(sts[i]->n);
    int vb = 6;
    if (opts && opts->mode == SV_MODE_REGTILE && opts->tile_qubits > 0) {
        vb = std::min(6, std::max(3, opts->tile_qubits));
    } else if (width_of->count(shape)) {
        vb = (*width_of)[shape];
    } else {
        float best_ms = -1;
        for (int w = 4; w <= 6; w++) {
            SV_TRY(prepare(w));
            if (fallback) return batch_graph_of_launches(sts, cs, count, opts, out);
            hipEvent_t t0, t1;
            SV_HIP(hipEventCreate(&t0));
            SV_HIP(hipEventCreate(&t1));
            (void)hipEventRecord(t0, last->stream);
            hipError_t e = hipGraphLaunch(last->exec, last->stream);
            (void)hipEventRecord(t1, last->stream);
            if (e == hipSuccess) e = hipEventSynchronize(t1);
            float ms = 0;
            (void)hipEventElapsedTime(&ms, t0, t1);
            (void)hipEventDestroy(t0);
            (void)hipEventDestroy(t1);
            if (e != hipSuccess) return hip_fail(e, "ensemble width timing");
            if (best_ms < 0 || ms < best_ms) {
                best_ms = ms;
                vb = w;
            }
        }
        (*width_of)[shape] = vb;
    }
    SV_TRY(prepare(vb));
    if (fallback) return batch_graph_of_launches(sts, cs, count, opts, out);
    std::vector<double> host((size_t)count * 16);
    unsigned herr = 0;
    hipError_t e = hipGraphLaunch(last->exec, last->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(host.data(), last->res, host.size() * 8, hipMemcpyDeviceToHost, last->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&herr, last->err, 4, hipMemcpyDeviceToHost, last->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(last->stream);
    for (int64_t i = 0; i < count; i++) {
        sts[i]->known_zero = false;
        sts[i]->ck_key.clear();
    }
    if (e != hipSuccess) return hip_fail(e, "ensemble launch");
    if (herr) return fail(SV_EDEVICE, "batch: a dependency wait exceeded its bound");
    for (int64_t i = 0; i < count; i++) finish_stats(&host[16 * i], sts[i]->n, &out[i]);
    return SV_OK;
}

namespace svi {

// Every instance's sweeps and statistics pass as ordinary launches recorded
// in one captured graph (complex128 and non-register-tile plans).
static sv_status batch_graph_of_launches(sv_state **sts, const sv_circuit *cs, int64_t count,
                                         const sv_opts *opts, sv_stats *out) {
    const sv_dtype dt = sts[0]->dt;
    hipStream_t user = sts[0]->stream;
    std::vector<std::shared_ptr<Plan>> plans(count);
    for (int64_t i = 0; i < count; i++) {
        PlanRequest rq{};
        rq.n = sts[i]->n;
        rq.dtype = dt;
        rq.mode = (opts && opts->mode != SV_MODE_AUTO) ? opts->mode : SV_MODE_REGTILE;
        rq.k_max = opts ? opts->k_max : 0;
        rq.tile = opts ? opts->tile_qubits : 0;
        rq.from_zero = true;
        rq.force_zero = true;
        SV_TRY(get_plan(sts[i], &cs[i], rq, &plans[i]));
    }
    static Workspace *res_ws = new Workspace(), *part_ws = new Workspace();   // kept for the process
    SV_TRY(res_ws->reserve((size_t)count * 16 * sizeof(double)));
    SV_TRY(part_ws->reserve((size_t)2049 * 16 * sizeof(double)));
    double *res = (double *)res_ws->ptr;
    double *part = (double *)part_ws->ptr;
    hipStream_t cap;
    SV_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    if (user) SV_HIP(hipStreamSynchronize(user));
    else SV_HIP(hipDeviceSynchronize());
    std::vector<hipStream_t> saved(count);
    for (int64_t i = 0; i < count; i++) {
        saved[i] = sts[i]->stream;
        sts[i]->stream = cap;
    }
    sv_status rc = SV_OK;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) rc = hip_fail(e, "hipStreamBeginCapture");
    for (int64_t i = 0; rc == SV_OK && i < count; i++) {
        rc = run_plan(sts[i], *plans[i]);
        if (rc == SV_OK) rc = batch_stats_enqueue(sts[i], part, res + 16 * i);
    }
    e = hipStreamEndCapture(cap, &graph);
    if (rc == SV_OK && e != hipSuccess) rc = hip_fail(e, "hipStreamEndCapture");
    if (rc == SV_OK) {
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) rc = hip_fail(e, "hipGraphInstantiate");
    }
    if (rc == SV_OK) {
        e = hipGraphLaunch(exec, cap);
        if (e != hipSuccess) rc = hip_fail(e, "hipGraphLaunch");
    }
    std::vector<double> host((size_t)count * 16);
    if (rc == SV_OK) {
        e = hipMemcpyAsync(host.data(), res, host.size() * 8, hipMemcpyDeviceToHost, cap);
        if (e == hipSuccess) e = hipStreamSynchronize(cap);
        if (e != hipSuccess) rc = hip_fail(e, "batch result copy");
    }
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipStreamSynchronize(cap);
    (void)hipStreamDestroy(cap);
    for (int64_t i = 0; i < count; i++) {
        sts[i]->stream = saved[i];
        sts[i]->known_zero = false;
        sts[i]->ck_key.clear();
    }
    if (rc != SV_OK) return rc;
    for (int64_t i = 0; i < count; i++) finish_stats(&host[16 * i], sts[i]->n, &out[i]);
    return SV_OK;
}

}  // namespace svi
