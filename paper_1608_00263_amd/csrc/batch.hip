// Ensembles of circuits (different qubit counts and depths) simulated in one
// HIP graph: every instance's sweeps and its statistics pass are recorded
// once on a capture stream and the graph is replayed; per-instance results
// stay on the device until one copy at the end.
#include <hip/hip_runtime.h>

#include <cmath>

#include "internal.h"

namespace svi {

sv_status batch_stats_enqueue(sv_state *st, double *part, double *res);   // reduce.hip

}  // namespace svi

using namespace svi;

extern "C" sv_status sv_apply_batch(sv_state **sts, const sv_circuit *cs, int64_t count, const sv_opts *opts,
                                    sv_stats *out) {
    if (count < 0 || (count > 0 && (!sts || !cs || !out))) return fail(SV_EINVAL, "bad batch arguments");
    if (count == 0) return SV_OK;
    const sv_dtype dt = sts[0] ? sts[0]->dt : SV_C64;
    hipStream_t user = sts[0] ? sts[0]->stream : nullptr;
    for (int64_t i = 0; i < count; i++) {
        if (!sts[i] || !sts[i]->data) return fail(SV_EINVAL, "null state in batch");
        if (sts[i]->dt != dt) return fail(SV_EINVAL, "batch states must share a dtype");
        if (sts[i]->stream != user) return fail(SV_EINVAL, "batch states must share a stream");
        if (cs[i].n != sts[i]->n) return fail(SV_EINVAL, "circuit / state size mismatch in batch");
    }
    // plans (built and uploaded before capture), from |0..0>
    std::vector<std::shared_ptr<Plan>> plans(count);
    for (int64_t i = 0; i < count; i++) {
        PlanRequest rq{};
        rq.n = sts[i]->n;
        rq.dtype = dt;
        rq.mode = opts ? opts->mode : SV_MODE_AUTO;
        rq.k_max = opts ? opts->k_max : 0;
        rq.tile = opts ? opts->tile_qubits : 0;
        rq.from_zero = true;
        SV_TRY(get_plan(sts[i], &cs[i], rq, &plans[i]));
    }
    // device results: 16 doubles per instance; partials reused in order
    // kept until the process ends (no static destructor after runtime teardown)
    static Workspace *res_ws = new Workspace(), *part_ws = new Workspace();
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
        const Plan &p = *plans[i];
        if (p.ops.empty() || p.ops[0].type != OP_INIT_UNIFORM) rc = launch_init_zero(sts[i], sts[i]->data);
        if (rc == SV_OK) rc = run_plan(sts[i], p);
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
    }
    if (rc != SV_OK) return rc;
    for (int64_t i = 0; i < count; i++) {
        const double *r = &host[16 * i];
        const double N = std::ldexp(1.0, sts[i]->n);
        const double S = r[0];
        const double lnS = std::log(S);
        sv_stats &o = out[i];
        o.norm = S;
        o.entropy = lnS - r[1] / S;
        o.zero_count = (int64_t)r[13];
        o.unif_ce = o.zero_count ? INFINITY : lnS - r[2] / N;
        double Sk = 1.0;
        for (int k = 0; k < 10; k++) {
            Sk *= S;
            o.moments[k] = r[3 + k] / N / Sk;
        }
    }
    return SV_OK;
}
