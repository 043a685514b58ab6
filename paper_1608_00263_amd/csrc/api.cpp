// C ABI entry points (include/sv.h): handle management, argument checks,
// plan cache and dispatch.  All device work is enqueued on the handle's
// stream; functions returning host scalars synchronise it.
#include <hip/hip_runtime.h>

#include <cmath>
#include <limits>
#include <cstdio>
#include <cstdlib>
#include <new>

#include "internal.h"

namespace svi {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }

sv_status fail(sv_status st, const std::string &msg) {
    g_err = msg;
    return st;
}

sv_status hip_fail(hipError_t e, const char *what) {
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    g_err = m;
    return e == hipErrorOutOfMemory ? SV_ENOMEM : SV_EDEVICE;
}

sv_status Workspace::reserve(size_t need) {
    if (need <= bytes) return SV_OK;
    if (ptr) {
        SV_HIP(hipDeviceSynchronize());
        SV_HIP(hipFree(ptr));
        ptr = nullptr;
        bytes = 0;
    }
    size_t want = need < ((size_t)1 << 20) ? ((size_t)1 << 20) : need;
    hipError_t e = hipMalloc(&ptr, want);
    if (e != hipSuccess) {
        ptr = nullptr;
        return hip_fail(e, "workspace hipMalloc");
    }
    bytes = want;
    return SV_OK;
}

Workspace::~Workspace() {
    if (ptr) (void)hipFree(ptr);
}

static int max_qubits(sv_dtype dt) { return dt == SV_C64 ? 35 : 34; }

static sv_status check_state(sv_state *st) {
    if (!st) return fail(SV_EINVAL, "null state handle");
    if (!st->data) return fail(SV_ESTATE, "state has no device buffer");
    return SV_OK;
}

static sv_status check_circuit(sv_state *st, const sv_circuit *c) {
    if (!c) return fail(SV_EINVAL, "null circuit");
    if (c->n != st->n) return fail(SV_EINVAL, "circuit qubit count differs from the state's");
    if (c->ngates < 0 || (c->ngates > 0 && !c->gates)) return fail(SV_EINVAL, "bad gate array");
    if (c->nparams < 0 || (c->nparams > 0 && !c->theta)) return fail(SV_EINVAL, "bad theta array");
    if (c->nmats < 0 || (c->nmats > 0 && !c->mats)) return fail(SV_EINVAL, "bad matrix array");
    return SV_OK;
}

static PlanRequest make_request(sv_state *st, const sv_opts *o) {
    PlanRequest rq{};
    rq.n = st->n;
    rq.dtype = st->dt;
    rq.mode = o ? o->mode : SV_MODE_AUTO;
    rq.k_max = o ? o->k_max : 0;
    rq.tile = o ? o->tile_qubits : 0;
    rq.budget = o ? o->sweep_budget : 0;
    rq.force_zero = o && (o->flags & SV_FLAG_FROM_ZERO);
    rq.from_zero = st->known_zero || rq.force_zero;
    rq.no_mfma = o && (o->flags & SV_FLAG_NO_MFMA);
    return rq;
}

// ---------------------------------------------------------------------------
// autotuner
// ---------------------------------------------------------------------------
static std::map<std::string, sv_opts> g_tuned;   // process-wide choices

static std::vector<sv_opts> tune_candidates(const sv_state *st) {
    std::vector<sv_opts> c;
    auto add = [&](int mode, int k, int t, int budget = 0) { c.push_back(sv_opts{mode, k, t, 0, budget, 0}); };
    if (st->n >= 10) {
        // register tiles of each width at the default sweep budget, and the
        // widest also at a smaller budget: lighter sweeps, sometimes one more
        // of them (which is faster depends on the circuit: measured on the
        // 30-qubit depth-40 circuit 42.3 against 43.4 ms in complex64, 95.2
        // against 97.8 ms in complex128, on the 35-qubit one 1.68 against
        // 1.61 s)
        if (st->dt == SV_C64) {
            add(SV_MODE_REGTILE, 0, 4); add(SV_MODE_REGTILE, 0, 5); add(SV_MODE_REGTILE, 0, 6);
            add(SV_MODE_REGTILE, 0, 6, 160);
        } else {
            add(SV_MODE_REGTILE, 0, 3); add(SV_MODE_REGTILE, 0, 4); add(SV_MODE_REGTILE, 0, 5);
            add(SV_MODE_REGTILE, 0, 5, 140);
        }
        add(SV_MODE_FUSED, 2, 0);
        add(SV_MODE_FUSED, 3, 0);
        // complex64 LDS tiles of dense 8x8 blocks are bound by the FP32 VALU
        // (32 multiply-adds per amplitude and block, several blocks per tile):
        // they are not a candidate there
        if (st->dt != SV_C64) add(SV_MODE_TILED, 3, 11);
    } else {
        add(SV_MODE_SPEC, 0, 0);
    }
    return c;
}

static std::string tune_key(const sv_state *st, const sv_circuit *c, bool from_zero) {
    PlanRequest rq{};
    rq.n = st->n;
    rq.dtype = st->dt;
    rq.mode = SV_MODE_AUTO;
    rq.from_zero = from_zero;
    return plan_key(c, rq);
}

static sv_status time_plan(sv_state *st, const Plan &plan, void *psi, float *ms) {
    hipEvent_t a, b;
    SV_HIP(hipEventCreate(&a));
    SV_HIP(hipEventCreate(&b));
    sv_status rc = SV_OK;
    (void)hipEventRecord(a, st->stream);
    for (const Op &op : plan.ops) {
        rc = launch_op(st, plan, op, psi);
        if (rc != SV_OK) break;
    }
    (void)hipEventRecord(b, st->stream);
    hipError_t e = hipEventSynchronize(b);
    if (rc == SV_OK && e != hipSuccess) rc = hip_fail(e, "hipEventSynchronize");
    if (rc == SV_OK) (void)hipEventElapsedTime(ms, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return rc;
}

// A plan cannot run faster than its algorithmic bytes at the HBM peak
// (8 TB/s): a candidate whose bound exceeds the best measured time is not
// timed.
static double plan_floor_ms(const Plan &plan) {
    double b = 0;
    for (const Op &op : plan.ops) b += op.bytes;
    return b / 8.0e9;
}

// Resolve SV_MODE_AUTO to concrete options for (st, c).  May run the
// scratch-state tuning; sets *explore when this call should instead time a
// candidate on the real state.
static sv_status resolve_auto(sv_state *st, const sv_circuit *c, bool from_zero, sv_opts *out, int *explore) {
    *explore = -1;
    const std::string key = tune_key(st, c, from_zero);
    auto it = g_tuned.find(key);
    if (it != g_tuned.end()) { *out = it->second; return SV_OK; }
    std::vector<sv_opts> cand = tune_candidates(st);
    if (cand.size() == 1) { g_tuned[key] = cand[0]; *out = cand[0]; return SV_OK; }
    const size_t bytes = (size_t)state_bytes(st->n, st->dt);
    size_t freeb = 0, total = 0;
    SV_HIP(hipMemGetInfo(&freeb, &total));
    if (freeb > bytes + bytes / 4 + ((size_t)1 << 30)) {
        void *scratch = nullptr;
        SV_HIP(hipMalloc(&scratch, bytes));
        SV_HIP(hipMemsetAsync(scratch, 0, bytes, st->stream));
        int best = -1;
        float best_ms = 0;
        sv_status rc = SV_OK;
        for (size_t i = 0; i < cand.size() && rc == SV_OK; i++) {
            PlanRequest rq = make_request(st, &cand[i]);
            rq.from_zero = from_zero;
            std::shared_ptr<Plan> plan;
            rc = get_plan(st, c, rq, &plan);
            if (rc == SV_OK && best >= 0 && plan_floor_ms(*plan) > best_ms) continue;
            float ms = 0, m1 = 0;
            if (rc == SV_OK) rc = time_plan(st, *plan, scratch, &ms);           // warm
            // best of three: candidates a few percent apart stay ordered
            for (int r = 0; r < 3 && rc == SV_OK; r++) {
                rc = time_plan(st, *plan, scratch, &m1);
                if (r == 0 || m1 < ms) ms = m1;
            }
            if (rc == SV_OK && (best < 0 || ms < best_ms)) { best = (int)i; best_ms = ms; }
        }
        (void)hipStreamSynchronize(st->stream);
        (void)hipFree(scratch);
        if (rc != SV_OK) return rc;
        g_tuned[key] = cand[best];
        *out = cand[best];
        return SV_OK;
    }
    // no room for a scratch state: explore on the real calls
    Tune &t = st->tunes[key];
    if (t.cand.empty()) { t.cand = cand; t.ms.assign(cand.size(), 0.0); }
    while (t.next > 0 && t.next < t.cand.size()) {
        double best_ms = t.ms[0];
        for (size_t i = 1; i < t.next; i++) best_ms = std::min(best_ms, t.ms[i]);
        PlanRequest rq = make_request(st, &t.cand[t.next]);
        rq.from_zero = from_zero;
        std::shared_ptr<Plan> plan;
        SV_TRY(get_plan(st, c, rq, &plan));
        if (plan_floor_ms(*plan) <= best_ms) break;
        t.ms[t.next++] = std::numeric_limits<double>::infinity();   // cannot win: not run
    }
    if (t.next < t.cand.size()) {
        *explore = (int)t.next;
        *out = t.cand[t.next];
        return SV_OK;
    }
    int best = 0;
    for (size_t i = 1; i < t.ms.size(); i++)
        if (t.ms[i] < t.ms[best]) best = (int)i;
    g_tuned[key] = t.cand[best];
    *out = t.cand[best];
    return SV_OK;
}

// Options actually used for a call (AUTO resolved).
static sv_status effective_opts(sv_state *st, const sv_circuit *c, const sv_opts *o, sv_opts *eff,
                                int *explore) {
    *explore = -1;
    sv_opts d{SV_MODE_AUTO, 0, 0, 0};
    if (o) d = *o;
    if (d.mode != SV_MODE_AUTO) { *eff = d; return SV_OK; }
    const bool from_zero = st->known_zero || (d.flags & SV_FLAG_FROM_ZERO);
    sv_opts r;
    SV_TRY(resolve_auto(st, c, from_zero, &r, explore));
    r.flags = d.flags;
    *eff = r;
    return SV_OK;
}

sv_status get_plan(sv_state *st, const sv_circuit *c, PlanRequest rq, std::shared_ptr<Plan> *out) {
    if (rq.mode == SV_MODE_AUTO) rq.mode = SV_MODE_REGTILE;   // only without a handle-level choice
    if (rq.mode < SV_MODE_PLAIN || rq.mode > SV_MODE_REGTILE) return fail(SV_EINVAL, "unknown mode");
    if (rq.k_max < 0 || rq.k_max > 5) return fail(SV_EINVAL, "k_max must be 0..5");
    if (rq.budget != 0 && (rq.budget < 20 || rq.budget > 2000)) return fail(SV_EINVAL, "sweep_budget must be 0 or 20..2000");
    std::string key = plan_key(c, rq);
    auto it = st->plans.find(key);
    if (it != st->plans.end()) {
        *out = it->second;
        return SV_OK;
    }
    auto plan = std::make_shared<Plan>();
    SV_TRY(build_plan(c, rq, plan.get()));
    SV_TRY(upload_plan(st, plan.get()));
    if (st->plans.size() > 64) st->plans.clear();
    st->plans[key] = plan;
    *out = plan;
    return SV_OK;
}

sv_status run_plan(sv_state *st, const Plan &plan) {
    st->ck_key.clear();
    for (const Op &op : plan.ops) SV_TRY(launch_op(st, plan, op, st->data));
    st->known_zero = false;
    return SV_OK;
}

}  // namespace svi

using namespace svi;

extern "C" {

const char *sv_last_error(void) { return g_err.c_str(); }

static sv_status new_state(int n, sv_dtype dt, void *stream, sv_state **out) {
    if (!out) return fail(SV_EINVAL, "null output handle");
    *out = nullptr;
    if (dt != SV_C64 && dt != SV_C128) return fail(SV_EINVAL, "unknown dtype");
    if (n < 1 || n > max_qubits(dt)) {
        char b[96];
        snprintf(b, sizeof b, "n = %d out of range 1..%d", n, max_qubits(dt));
        return fail(SV_ERANGE, b);
    }
    sv_state *st = new (std::nothrow) sv_state();
    if (!st) return fail(SV_ENOMEM, "host allocation failed");
    st->n = n;
    st->dt = dt;
    st->stream = (hipStream_t)stream;
    hipError_t e = hipGetDevice(&st->device);
    if (e != hipSuccess) {
        delete st;
        return hip_fail(e, "hipGetDevice");
    }
    *out = st;
    return SV_OK;
}

sv_status sv_alloc(int n, sv_dtype dt, void *hip_stream, sv_state **out) {
    sv_state *st = nullptr;
    SV_TRY(new_state(n, dt, hip_stream, &st));
    size_t bytes = (size_t)state_bytes(n, dt);
    size_t freeb = 0, total = 0;
    hipError_t e = hipMemGetInfo(&freeb, &total);
    if (e != hipSuccess) {
        delete st;
        return hip_fail(e, "hipMemGetInfo");
    }
    if (bytes > freeb) {
        delete st;
        char b[128];
        snprintf(b, sizeof b, "state needs %zu bytes, %zu free", bytes, freeb);
        return fail(SV_ENOMEM, b);
    }
    e = hipMalloc(&st->data, bytes);
    if (e != hipSuccess) {
        delete st;
        return hip_fail(e, "hipMalloc(state)");
    }
    st->owned = true;
    sv_status rc = sv_reset(st);
    if (rc != SV_OK) {
        sv_free(st);
        return rc;
    }
    *out = st;
    return SV_OK;
}

sv_status sv_attach(int n, sv_dtype dt, void *dev_ptr, void *hip_stream, sv_state **out) {
    if (!dev_ptr) return fail(SV_EINVAL, "null device pointer");
    sv_state *st = nullptr;
    SV_TRY(new_state(n, dt, hip_stream, &st));
    st->data = dev_ptr;
    st->owned = false;
    *out = st;
    return SV_OK;
}

sv_status sv_free(sv_state *st) {
    if (!st) return SV_OK;
    if (st->stream) (void)hipStreamSynchronize(st->stream);
    else (void)hipDeviceSynchronize();
    if (st->owned && st->data) (void)hipFree(st->data);
    delete st;
    return SV_OK;
}

sv_status sv_reset(sv_state *st) {
    SV_TRY(check_state(st));
    SV_TRY(launch_init_zero(st, st->data));
    // only a buffer the library owns stays |0..0> until the next call: the
    // caller may write an attached buffer at any time
    st->known_zero = st->owned;
    st->ck_key.clear();
    return SV_OK;
}

sv_status sv_data(sv_state *st, void **dev_ptr) {
    SV_TRY(check_state(st));
    if (!dev_ptr) return fail(SV_EINVAL, "null output pointer");
    *dev_ptr = st->data;
    st->known_zero = false;   // the caller may write through the pointer
    st->ck_key.clear();
    return SV_OK;
}

sv_status sv_apply_circuit(sv_state *st, const sv_circuit *c, const sv_opts *opts) {
    SV_TRY(check_state(st));
    SV_TRY(check_circuit(st, c));
    if (opts && (opts->flags & SV_FLAG_CHECKPOINTS)) return run_forward_checkpoints(st, c, opts);
    sv_opts eff;
    int explore = -1;
    SV_TRY(effective_opts(st, c, opts, &eff, &explore));
    std::shared_ptr<Plan> plan;
    const bool from_zero = st->known_zero || (eff.flags & SV_FLAG_FROM_ZERO);
    SV_TRY(get_plan(st, c, make_request(st, &eff), &plan));
    if (explore < 0) return run_plan(st, *plan);
    float ms = 0;
    st->ck_key.clear();
    SV_TRY(time_plan(st, *plan, st->data, &ms));
    st->known_zero = false;
    Tune &t = st->tunes[tune_key(st, c, from_zero)];
    t.ms[explore] = ms;
    t.next++;
    return SV_OK;
}

sv_status sv_autotune(sv_state *st, const sv_circuit *c, int from_zero, sv_opts *chosen, int *complete) {
    SV_TRY(check_state(st));
    SV_TRY(check_circuit(st, c));
    sv_opts r;
    int explore = -1;
    SV_TRY(resolve_auto(st, c, from_zero != 0, &r, &explore));
    if (chosen) *chosen = r;
    if (complete) *complete = explore < 0;
    return SV_OK;
}

static int32_t sweep_kind(const Op &op) {
    switch (op.type) {
    case OP_INIT_UNIFORM: case OP_INIT_ZERO: return SV_SWEEP_INIT;
    case OP_PLAIN_1Q: return SV_SWEEP_PLAIN_1Q;
    case OP_PLAIN_CZ: return SV_SWEEP_PLAIN_CZ;
    case OP_SPEC_DENSE: return SV_SWEEP_SPEC_DENSE;
    case OP_SPEC_REAL: return SV_SWEEP_SPEC_REAL;
    case OP_SPEC_DIAG: return SV_SWEEP_SPEC_DIAG;
    case OP_SPEC_CZ: return SV_SWEEP_SPEC_CZ;
    case OP_REGTILE: return SV_SWEEP_REGTILE;
    case OP_LDSTILE: return op.mfma ? SV_SWEEP_LDSTILE_MFMA : SV_SWEEP_LDSTILE;
    default: return 0;
    }
}

sv_status sv_apply_circuit_timed(sv_state *st, const sv_circuit *c, const sv_opts *opts, int64_t cap,
                                 float *op_ms, int32_t *op_kind, double *op_bytes, int64_t *nops) {
    SV_TRY(check_state(st));
    SV_TRY(check_circuit(st, c));
    sv_opts eff;
    int explore = -1;
    SV_TRY(effective_opts(st, c, opts, &eff, &explore));
    std::shared_ptr<Plan> plan;
    SV_TRY(get_plan(st, c, make_request(st, &eff), &plan));
    const size_t m = plan->ops.size();
    st->ck_key.clear();
    std::vector<hipEvent_t> ev(m + 1);
    for (auto &e : ev) SV_HIP(hipEventCreate(&e));
    sv_status rc = SV_OK;
    hipError_t he = hipEventRecord(ev[0], st->stream);
    if (he != hipSuccess) rc = hip_fail(he, "hipEventRecord");
    for (size_t i = 0; rc == SV_OK && i < m; i++) {
        rc = launch_op(st, *plan, plan->ops[i], st->data);
        if (rc == SV_OK) {
            he = hipEventRecord(ev[i + 1], st->stream);
            if (he != hipSuccess) rc = hip_fail(he, "hipEventRecord");
        }
    }
    if (rc == SV_OK) {
        he = hipEventSynchronize(ev[m]);
        if (he != hipSuccess) rc = hip_fail(he, "hipEventSynchronize");
    }
    for (size_t i = 0; rc == SV_OK && i < m && (int64_t)i < cap; i++) {
        float ms = 0;
        he = hipEventElapsedTime(&ms, ev[i], ev[i + 1]);
        if (he != hipSuccess) { rc = hip_fail(he, "hipEventElapsedTime"); break; }
        if (op_ms) op_ms[i] = ms;
        if (op_kind) op_kind[i] = sweep_kind(plan->ops[i]);
        if (op_bytes) op_bytes[i] = plan->ops[i].bytes;
    }
    for (auto &e : ev) (void)hipEventDestroy(e);
    if (rc != SV_OK) return rc;
    st->known_zero = false;
    if (nops) *nops = (int64_t)m;
    return SV_OK;
}

sv_status sv_plan_info(sv_state *st, const sv_circuit *c, const sv_opts *opts, int64_t *sweeps,
                       double *bytes) {
    SV_TRY(check_state(st));
    SV_TRY(check_circuit(st, c));
    sv_opts eff;
    int explore = -1;
    SV_TRY(effective_opts(st, c, opts, &eff, &explore));
    std::shared_ptr<Plan> plan;
    SV_TRY(get_plan(st, c, make_request(st, &eff), &plan));
    if (sweeps) *sweeps = plan->sweeps;
    if (bytes) *bytes = plan->bytes;
    return SV_OK;
}

sv_status sv_cycle_moments(sv_state *st, const sv_circuit *c, const sv_opts *opts, int64_t cap, sv_stats *out,
                           int64_t *ncycles) {
    SV_TRY(check_state(st));
    SV_TRY(check_circuit(st, c));
    if (cap > 0 && !out) return fail(SV_EINVAL, "null statistics output");
    PlanRequest rq = make_request(st, opts);
    rq.from_zero = true;
    rq.force_zero = true;
    if (rq.budget != 0 && (rq.budget < 20 || rq.budget > 2000)) return fail(SV_EINVAL, "sweep_budget must be 0 or 20..2000");
    const std::string key = "cyc:" + plan_key(c, rq);
    std::shared_ptr<Plan> plan;
    auto it = st->plans.find(key);
    if (it != st->plans.end()) {
        plan = it->second;
    } else {
        plan = std::make_shared<Plan>();
        SV_TRY(build_cycle_plan(c, rq, plan.get()));
        SV_TRY(upload_plan(st, plan.get()));
        if (st->plans.size() > 64) st->plans.clear();
        st->plans[key] = plan;
    }
    const int64_t nc = (int64_t)plan->cycle_row.size();
    if (ncycles) *ncycles = nc;
    if (cap < nc) return fail(SV_ERANGE, "per-cycle statistics: cap is smaller than the number of cycles");
    int64_t nrows = 0;
    for (const Op &op : plan->ops) nrows += op.type == OP_STATS;
    SV_TRY(st->ws.reserve((size_t)(2048 + nrows) * 16 * sizeof(double)));
    double *part = (double *)st->ws.ptr;
    double *res = part + (size_t)2048 * 16;
    st->ck_key.clear();
    for (const Op &op : plan->ops) {
        if (op.type == OP_STATS) SV_TRY(batch_stats_enqueue(st, part, res + (size_t)16 * op.q0));
        else SV_TRY(launch_op(st, *plan, op, st->data));
    }
    st->known_zero = false;
    std::vector<double> host((size_t)nrows * 16);
    SV_HIP(hipMemcpyAsync(host.data(), res, host.size() * sizeof(double), hipMemcpyDeviceToHost, st->stream));
    SV_HIP(hipStreamSynchronize(st->stream));
    std::vector<sv_stats> rows((size_t)nrows);
    for (int64_t r = 0; r < nrows; r++) finish_stats_row(st->n, &host[(size_t)16 * r], &rows[(size_t)r]);
    for (int64_t t = 0; t < nc; t++) out[t] = rows[(size_t)plan->cycle_row[(size_t)t]];
    return SV_OK;
}

sv_status sv_pair_stats(sv_state *a, sv_state *b, int32_t nbins, double zmin, double zmax, sv_pair *out,
                        uint64_t *hist) {
    SV_TRY(check_state(a));
    SV_TRY(check_state(b));
    if (!out) return fail(SV_EINVAL, "null output");
    if (a->n != b->n || a->dt != b->dt) return fail(SV_EINVAL, "pair statistics need two states of one size and dtype");
    if (a->stream != b->stream) return fail(SV_EINVAL, "pair statistics need two states on one stream");
    if (nbins < 0 || nbins > 1024) return fail(SV_ERANGE, "nbins out of range 0..1024");
    if (nbins > 0 && (!hist || !std::isfinite(zmin) || !std::isfinite(zmax) || !(zmin < zmax)))
        return fail(SV_EINVAL, "a histogram needs an output array and a finite range zmin < zmax");
    const int n = a->n;
    std::vector<double> thr((size_t)nbins + 1);
    const double dz = nbins > 0 ? (zmax - zmin) / nbins : 0.0;
    for (int j = 0; j <= nbins && nbins > 0; j++) thr[(size_t)j] = std::ldexp(std::exp(zmin + j * dz), -n);
    double r[16] = {0};
    SV_TRY(run_pair_stats(a, b, nbins, thr.data(), r, hist));
    const double N = std::ldexp(1.0, n);
    const double Sa = r[0], Sb = r[1];
    if (nbins > 0 && !(Sa < 4.0 && Sb < 4.0))
        return fail(SV_ERANGE, "sv_pair_stats: a norm of 4 or more has no 64-bit integer histogram masses");
    out->norm_a = Sa;
    out->norm_b = Sb;
    out->overlap_re = r[2];
    out->overlap_im = r[3];
    out->fidelity = (r[2] * r[2] + r[3] * r[3]) / (Sa * Sb);
    out->zero_mass_b = r[9];
    out->zero_a = (int64_t)r[10];
    out->xent = r[9] > 0.0 ? INFINITY : std::log(Sa) - r[7] / Sb;
    out->unif_ce = out->zero_a ? INFINITY : std::log(Sa) - r[8] / N;
    out->delta_h = out->zero_a ? NAN : out->unif_ce - out->xent;
    const double cab = N * r[6] / (Sa * Sb) - 1.0, caa = N * r[4] / (Sa * Sa) - 1.0, cbb = N * r[5] / (Sb * Sb) - 1.0;
    out->corr = (caa > 0.0 && cbb > 0.0) ? cab / std::sqrt(caa * cbb) : NAN;
    return SV_OK;
}

sv_status sv_probs(sv_state *st, uint64_t begin, uint64_t count, int out_f64, void *dev_out) {
    SV_TRY(check_state(st));
    const uint64_t N = 1ull << st->n;
    if (begin > N || count > N - begin) return fail(SV_ERANGE, "probability range outside the state");
    if (count && !dev_out) return fail(SV_EINVAL, "null output buffer");
    return run_probs(st, begin, count, out_f64, dev_out);
}

sv_status sv_moments(sv_state *st, sv_stats *out) {
    SV_TRY(check_state(st));
    if (!out) return fail(SV_EINVAL, "null output");
    return run_stats(st, st->data, out);
}

sv_status sv_sample(sv_state *st, int64_t k, uint64_t seed, uint64_t *out, int out_on_device) {
    SV_TRY(check_state(st));
    if (k < 0 || k > ((int64_t)1 << 31)) return fail(SV_ERANGE, "sample count out of range");
    if (k == 0) return SV_OK;
    if (!out) return fail(SV_EINVAL, "null output");
    uint64_t *dout = out;
    if (!out_on_device) {
        SV_TRY(st->ws2.reserve((size_t)k * 8));
        dout = (uint64_t *)st->ws2.ptr;
    }
    SV_TRY(run_sample(st, st->data, k, seed, dout));
    if (!out_on_device)
        SV_HIP(hipMemcpyAsync(out, dout, (size_t)k * 8, hipMemcpyDeviceToHost, st->stream));
    SV_HIP(hipStreamSynchronize(st->stream));
    return SV_OK;
}

sv_status sv_moments_sample(sv_state *st, sv_stats *stats, int64_t k, uint64_t seed, uint64_t *out,
                            int out_on_device) {
    SV_TRY(check_state(st));
    if (!stats) return fail(SV_EINVAL, "null statistics output");
    if (k < 0 || k > ((int64_t)1 << 31)) return fail(SV_ERANGE, "sample count out of range");
    if (k > 0 && !out) return fail(SV_EINVAL, "null output");
    uint64_t *dout = out;
    if (k > 0 && !out_on_device) {
        SV_TRY(st->ws2.reserve((size_t)k * 8));
        dout = (uint64_t *)st->ws2.ptr;
    }
    SV_TRY(run_stats_sample(st, st->data, stats, k, seed, dout));
    if (k > 0 && !out_on_device)
        SV_HIP(hipMemcpyAsync(out, dout, (size_t)k * 8, hipMemcpyDeviceToHost, st->stream));
    SV_HIP(hipStreamSynchronize(st->stream));
    return SV_OK;
}

sv_status sv_moments_sample_noalloc(sv_state *st, sv_stats *stats, int64_t k, uint64_t seed, uint64_t *dev_out) {
    SV_TRY(check_state(st));
    if (!stats) return fail(SV_EINVAL, "null statistics output");
    if (k < 0 || k > ((int64_t)1 << 31)) return fail(SV_ERANGE, "sample count out of range");
    if (k > 0 && !dev_out) return fail(SV_EINVAL, "null device output");
    SV_TRY(run_stats_sample_noalloc(st, stats, k, seed, dev_out));
    SV_HIP(hipStreamSynchronize(st->stream));
    return SV_OK;
}

sv_status sv_sample_from(const double *probs, uint64_t N, const uint64_t *r64, int64_t k, uint64_t *out,
                         void *hip_stream) {
    if (!probs || !r64 || (k > 0 && !out)) return fail(SV_EINVAL, "null pointer");
    if (N < 1 || N > (1ull << 35)) return fail(SV_ERANGE, "N out of range 1..2^35");
    if (k < 0 || k > ((int64_t)1 << 31)) return fail(SV_ERANGE, "sample count out of range");
    return run_sample_from(probs, N, r64, k, out, (hipStream_t)hip_stream);
}

sv_status sv_cross_entropy(sv_state *st, const uint64_t *samples, int64_t k, double norm, double *ce,
                           double *delta_h, int64_t *zero_samples) {
    SV_TRY(check_state(st));
    if (k <= 0 || !samples || !ce) return fail(SV_EINVAL, "need k > 0 samples and an output");
    if (!(norm <= 0.0 || std::isfinite(norm))) return fail(SV_EINVAL, "norm must be finite");
    for (int64_t i = 0; i < k; i++)
        if (samples[i] >= (1ull << st->n)) return fail(SV_ERANGE, "sv_cross_entropy: a sample is not an n-bit string");
    double S = norm;
    if (!(norm > 0.0)) SV_TRY(run_norm(st, st->data, &S));
    SV_TRY(st->ws2.reserve((size_t)k * 8));
    uint64_t *dx = (uint64_t *)st->ws2.ptr;
    SV_HIP(hipMemcpyAsync(dx, samples, (size_t)k * 8, hipMemcpyHostToDevice, st->stream));
    double sum_log = 0;
    int64_t zeros = 0;
    SV_TRY(run_cross_entropy(st, st->data, dx, k, S, &sum_log, &zeros));
    const double euler_gamma = 0.57721566490153286061;
    *ce = zeros ? INFINITY : std::log(S) - sum_log / (double)k;
    if (delta_h) *delta_h = std::log(std::ldexp(1.0, st->n)) + euler_gamma - *ce;
    if (zero_samples) *zero_samples = zeros;
    return SV_OK;
}

}  // extern "C"
