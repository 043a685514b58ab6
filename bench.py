"""Benchmark of the hot path on one MI355X.

One step = the whole path over one synthetic input: simulate the 5x6-grid,
30-qubit, depth-40 random circuit of Sec. IV from |0...0> in complex64
(fused register-tile sweeps), compute the output statistics (entropy,
uniform cross entropy, moments 1..10), draw 10^5 samples and evaluate
their cross entropy.  Prints one JSON line.

value      = algorithmic HBM bytes of the step / step time (GB/s); the
             bytes are the sweeps' reads + writes of the state, one state
             read for the statistics and the sampler's bucket weights
             together, and a 16-amplitude run per sample (the cross entropy
             reuses the norm of the statistics);
roofline   = the dominant kernel (register-tile sweep), its algorithmic
             bytes per launch over its event-timed average duration;
circuit_s  = seconds of the same circuit per planning mode (plain per-gate,
             specialised per-gate, fused 2^k blocks, LDS tiles, register
             tiles) in complex64 and complex128;
grad       = adjoint gradient time over forward time on the 5x5, depth-30
             parametrised circuit (10^4 samples) for checkpoint intervals;
cpu_baseline = the FP64 reference timed on this host on a bounded sample.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBPS = 8000.0
PEAK_FP32_MFMA_TFLOPS = 157.3   # dense FP32 matrix peak of the MI355X
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_regtile_c2_traffic.txt")
# sources of the register-tile sweep and its programs: the counter-based
# traffic of the profile summary is reported only while these are unchanged
KERNEL_SOURCES = ["paper_1608_00263_amd/csrc/device_common.h", "paper_1608_00263_amd/csrc/sweeps.hip",
                  "paper_1608_00263_amd/csrc/internal.h", "paper_1608_00263_amd/csrc/plan.cpp"]


def kernel_sha1():
    import hashlib
    h = hashlib.sha1()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def profile_summary(tile):
    """Key-value lines of the committed counter summary of the register-tile
    sweep, or {} when it is missing, for another tile width, or older than
    the kernel sources."""
    try:
        kv = {}
        with open(TRAFFIC_FILE) as fh:
            for line in fh:
                if ":" in line and not line.startswith("#"):
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        if kv.get("source_sha1") != kernel_sha1() or int(kv.get("register_qubits", -1)) != tile:
            return {}
        return kv
    except (OSError, ValueError):
        return {}


def measured_traffic(tile):
    """HBM bytes per register-tile launch from the counter summary, or None."""
    v = profile_summary(tile).get("traffic_bytes_per_launch")
    return float(v) if v is not None else None


def measured_valu_frac(tile):
    """Vector-ALU issue share of the register-tile sweeps from the counter
    summary (instructions over one per CU-cycle at 2.4 GHz), or None."""
    v = profile_summary(tile).get("valu_frac")
    return float(v) if v is not None else None


def log(msg):
    sys.stderr.write("[bench] %s\n" % msg)
    sys.stderr.flush()


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--mode", default="regtile")
    ap.add_argument("--tile", type=int, default=6)
    ap.add_argument("--samples", type=int, default=100000)
    ap.add_argument("--no-modes", action="store_true", help="skip the per-mode circuit timings")
    ap.add_argument("--no-grad", action="store_true", help="skip the adjoint timing")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU baseline")
    ap.add_argument("--no-ensemble", action="store_true", help="skip the ensemble timing")
    ap.add_argument("--no-c5", action="store_true", help="skip the 35-qubit run")
    ap.add_argument("--ensemble", type=int, default=512, help="ensemble instances")
    ap.add_argument("--copy-probe", action="store_true",
                    help="after the timed steps, copy an 8 GiB buffer three times (a plain copy "
                         "kernel of known size, the calibration of the HBM byte counters)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    return ap.parse_args()


def cpu_baseline(circ, budget_s):
    """The FP64 reference on this host: gates of the 30-qubit circuit,
    complex128, one plain sweep per gate, until the time budget is used."""
    import numpy as np
    import oracle
    n = circ.n
    psi = oracle.zero_state(n)
    S = 16.0 * 2 ** n
    done = 0
    t0 = time.perf_counter()
    while done < circ.ngates and time.perf_counter() - t0 < budget_s:
        oracle.apply_circuit(circ, psi, done, done + 1)
        done += 1
    dt = time.perf_counter() - t0
    del psi
    return {"value": round(2 * S * done / dt / 1e9, 3), "unit": "GB/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": "first %d of %d gates of the 5x6 depth-40 circuit, 30 qubits, complex128, "
                      "one plain sweep per gate (%.1f s); GB/s = 2 x 16 GiB x gates / time"
                      % (done, circ.ngates, dt)}


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py measures one GPU: there is no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_1608_00263_amd import circuits as C
    from paper_1608_00263_amd import sv

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    dev_name = torch.cuda.get_device_name(0)
    circ = C.make_circuit(5, 6, 40, seed=2)
    n = circ.n
    S64 = 8.0 * 2 ** n
    args = sv.CircuitArgs(circ)
    st = sv.State(n, "c64")
    m = a.samples

    def step():
        ms, kinds, by = st.apply_timed(circ, a.mode, 0, a.tile, args=args, from_zero=True)
        mom, xs = st.moments_and_sample(m, 1002)
        ce, dh, z = st.cross_entropy(xs, norm=mom["norm"])
        return ms, kinds, by, mom, ce, dh

    log("device %s; circuit 5x6 d40: %d gates" % (dev_name, circ.ngates))
    for i in range(a.warmup):
        step()
        log("warmup %d done" % i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sweep_ms = []
    sweep_bytes = []
    dom_ms = 0.0
    dom_bytes = 0.0
    dom_launches = 0
    last = None
    for i in range(a.steps):
        ms, kinds, by, mom, ce, dh = step()
        sweep_ms.append(float(ms.sum()))
        sweep_bytes.append(float(by.sum()))
        sel = kinds == 8        # register-tile sweeps
        dom_ms += float(ms[sel].sum())
        dom_bytes += float(by[sel].sum())
        dom_launches += int(sel.sum())
        last = (mom, ce, dh, len(ms))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    step_s = (t1 - t0) / a.steps
    mom, ce, dh, nsweeps = last
    step_bytes = sweep_bytes[-1] + S64 + m * 128.0
    value = step_bytes / step_s / 1e9
    achieved = dom_bytes / (dom_ms / 1e3) / 1e9
    floor = sweep_floor(sv, C, st, a.tile if a.mode == "regtile" else 6)
    log("timed %d steps: %.2f ms/step, sweeps %.2f ms, %d sweeps" % (a.steps, step_s * 1e3,
                                                                        np.mean(sweep_ms), nsweeps))
    out = {
        "metric": "HBM GB/s (% peak) of gate sweeps; 30q d40 circuit sec fused vs plain; grad/fwd",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(step_s * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": "random lattice circuit, 5x6 grid = 30 qubits, depth 40 (625 gates), "
                               "complex64 state, statistics + 1e5 samples + their cross entropy",
                   "mode": a.mode, "register_qubits": a.tile, "sweeps": nsweeps},
        "sweep_GBps": round(sweep_bytes[-1] / (np.mean(sweep_ms) / 1e3) / 1e9, 2),
        "sweep_frac_of_peak": round(sweep_bytes[-1] / (np.mean(sweep_ms) / 1e3) / 1e9 / PEAK_HBM_GBPS, 4),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBPS, 4), "traffic": measured_traffic(a.tile if a.mode == "regtile" else -1),
                     "kernel": "k_regtile<float,%d>" % a.tile,
                     "launch_avg_ms": round(dom_ms / max(dom_launches, 1), 4),
                     "bytes_per_launch": round(dom_bytes / max(dom_launches, 1), 1),
                     "valu_frac": measured_valu_frac(a.tile if a.mode == "regtile" else -1),
                     "achievable": floor["GBps"], "frac_of_achievable": round(achieved / floor["GBps"], 4),
                     "achievable_how": floor["how"],
                     "kernel_sources_sha1": kernel_sha1()},
        "results": {"entropy": mom["entropy"], "unif_ce": mom["unif_ce"], "norm": mom["norm"],
                    "M2": mom["M2"], "M10": mom["M10"], "ce": ce, "delta_h": dh},
    }
    if a.copy_probe:
        out["copy_probe"] = copy_probe(torch)
    if not a.no_modes:
        out["circuit_s"] = mode_timings(sv, C, circ, torch)
    if not a.no_grad:
        out["grad"] = grad_timings(sv, C, torch)
    if not a.no_ensemble:
        out["ensemble"] = ensemble_timings(sv, C, torch, a.ensemble)
    if not a.no_c5:
        out["c5"] = c5_run(sv, C, torch)
    st.close()
    del st
    torch.cuda.empty_cache()
    if not a.no_cpu:
        log("cpu baseline (%.0f s budget)" % a.cpu_seconds)
        out["cpu_baseline"] = cpu_baseline(circ, a.cpu_seconds)
    print(json.dumps(out), flush=True)


def sweep_floor(sv, C, st, tile):
    """The second denominator of the roofline: the same register-tile sweep
    kernel with a one-gate program (one X^1/2 on the top qubit, register
    tile rows of 64 contiguous amplitudes), reading and writing the whole
    state; best of five launches."""
    import numpy as np
    one = C.Circuit(n=st.n, gates=C.make_gates([(C.SX, st.n - 1, -1, 1, -1, -1)]))
    best = None
    for _ in range(6):
        ms, kinds, by = st.apply_timed(one, "regtile", 0, tile)
        t = float(ms.sum())
        best = t if best is None else min(best, t)
    gbps = 2.0 * 8.0 * 2 ** st.n / (best / 1e3) / 1e9
    log("one-gate sweep: %.3f ms = %.0f GB/s" % (best, gbps))
    return {"GBps": round(gbps, 1), "how": "k_regtile<float,%d> with a one-gate program, best of 6 launches "
                                           "(%.3f ms for 2 x 8 GiB)" % (tile, best)}


def copy_probe(torch):
    """torch's device copy of 2^30 complex64 (8 GiB read + 8 GiB write), three times."""
    x = torch.empty(1 << 30, dtype=torch.complex64, device="cuda")
    y = torch.empty_like(x)
    x.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / 3
    del x, y
    torch.cuda.empty_cache()
    return {"bytes": 2 * 8.0 * 2 ** 30, "s": round(dt, 5), "GBps": round(2 * 8.0 * 2 ** 30 / dt / 1e9, 1)}


def mode_timings(sv, C, circ, torch):
    res = {}
    for dtype in ("c64", "c128"):
        st = sv.State(circ.n, dtype)
        args = sv.CircuitArgs(circ)
        modes = [("plain", 0, 0, False), ("spec", 0, 0, False), ("fused", 2, 0, False),
                 ("fused", 3, 0, False), ("fused", 4, 0, False), ("fused", 5, 0, False),
                 ("tiled", 3, 12 if dtype == "c64" else 11, False),
                 ("tiled", 4, 13 if dtype == "c64" else 12, False)]
        if dtype == "c64":
            modes += [("fused", 4, 0, True), ("fused", 5, 0, True), ("regtile", 0, 4, False),
                      ("regtile", 0, 5, False), ("regtile", 0, 6, False),
                      # few gates per sweep: more sweeps, each close to streaming
                      ("regtile_b60", 0, 6, False)]
        else:
            modes += [("regtile", 0, 3, False), ("regtile", 0, 4, False), ("regtile", 0, 5, False)]
        modes += [("auto", 0, 0, False)]
        for mode, k, t, nomf in modes:
            budget = 60 if mode.endswith("_b60") else 0
            mode = mode.replace("_b60", "")
            st.apply(circ, mode, k, t, args=args, from_zero=True, no_mfma=nomf, budget=budget)   # plan + warm / tune
            if mode == "auto":
                for _ in range(8):
                    st.apply(circ, mode, k, t, args=args, from_zero=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st.apply(circ, mode, k, t, args=args, from_zero=True, no_mfma=nomf, budget=budget)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            sw, by = st.plan_info(circ, mode, k, t, no_mfma=nomf, from_zero=True, budget=budget)
            key = "%s_%s%s%s%s" % (dtype, mode, ("_k%d" % k if k else "") + ("_t%d" % t if t else ""),
                                   "_valu" if nomf else "", "_b%d" % budget if budget else "")
            res[key] = {"s": round(dt, 4), "sweeps": sw, "GBps": round(by / dt / 1e9, 1),
                        "frac_of_peak": round(by / dt / 1e9 / PEAK_HBM_GBPS, 4)}
            if mode in ("fused", "tiled"):
                tot, mf = dense_block_flops(sv, circ, dtype, mode, k, t, nomf)
                res[key]["dense_TFLOPs"] = round(tot / dt / 1e12, 2)
                if mf:
                    # MFMA block flops over the whole circuit time: a lower
                    # bound on the rate of the matrix cores while they run
                    res[key]["mfma_TFLOPs"] = round(mf / dt / 1e12, 2)
                    res[key]["mfma_frac_of_peak"] = round(mf / dt / 1e12 / PEAK_FP32_MFMA_TFLOPS, 4)
            if mode == "auto":
                res[key]["choice"] = st.autotune(circ, from_zero=True)[:3]
            log("%s: %.3f s, %d sweeps" % (key, dt, sw))
        st.close()
        del st
        torch.cuda.empty_cache()
    return res


def dense_block_flops(sv, circ, dtype, mode, k, t, nomf):
    """Algorithmic flops of the plan's dense 2^k blocks (8 * 2^k per
    amplitude each: a complex 2^k x 2^k matrix on every 2^k-vector), and of
    those that run on MFMA, read from the host description of the plan."""
    import re
    d = sv.host_plan_describe(circ, dtype, mode, k, t, from_zero=True, no_mfma=nomf)
    N = float(2 ** circ.n)
    tot = mf = 0.0
    for blocks, m in re.findall(r"blocks=\[([0-9]*)\][^\n]*mfma=(\d)", d):
        for ch in blocks:
            kk = int(ch)
            f = 8.0 * 2 ** kk * N
            tot += f
            if m == "1" and kk >= 4:
                mf += f
    return tot, mf


def c5_run(sv, C, torch):
    """The 5x7 grid, 35 qubits, depth 40, complex64 in place (256 GiB):
    register-tile sweeps timed per launch, statistics, 10^6 samples and
    their cross entropy."""
    import numpy as np
    torch.cuda.empty_cache()
    free, total = torch.cuda.mem_get_info(0)
    if free < 8 * 2 ** 35 + (4 << 30):
        return {"skipped": "needs 260 GiB of free device memory, %.0f GiB free" % (free / 2 ** 30)}
    circ = C.make_circuit(5, 7, 40, seed=5)
    args = sv.CircuitArgs(circ)
    st = sv.State(35, "c64")
    S = 8.0 * 2 ** 35
    out = {"workload": "5x7 grid, 35 qubits, depth 40 (%d gates), complex64 in place, 1e6 samples"
                       % circ.ngates}
    runs = []
    for rep in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ms, kinds, by = st.apply_timed(circ, "regtile", 0, 6, args=args, from_zero=True)
        torch.cuda.synchronize()
        runs.append((time.perf_counter() - t0, ms, by))
        log("c5 circuit: %.3f s, %d sweeps" % (runs[-1][0], len(ms)))
    dt, ms, by = runs[-1]
    t0 = time.perf_counter()
    m = st.moments()
    t_stats = time.perf_counter() - t0
    t0 = time.perf_counter()
    xs = st.sample(10 ** 6, 1005)
    t_sample = time.perf_counter() - t0
    t0 = time.perf_counter()
    ce, dh, z = st.cross_entropy(xs, norm=m["norm"])
    t_ce = time.perf_counter() - t0
    t0 = time.perf_counter()
    m2, xs2 = st.moments_and_sample(10 ** 6, 1005)
    t_both = time.perf_counter() - t0
    assert (xs2 == xs).all()
    gbps = float(by.sum()) / (float(ms.sum()) / 1e3) / 1e9
    out.update({"circuit_s": round(dt, 4), "sweeps": len(ms), "sweep_ms_avg": round(float(ms.mean()), 3),
                "sweep_GBps": round(gbps, 1), "sweep_frac_of_peak": round(gbps / PEAK_HBM_GBPS, 4),
                "stats_s": round(t_stats, 4), "sample_s": round(t_sample, 4), "ce_s": round(t_ce, 4),
                "stats_and_sample_one_pass_s": round(t_both, 4),
                "norm": m["norm"], "entropy": m["entropy"],
                "entropy_porter_thomas": 35 * math.log(2.0) - 1.0 + 0.5772156649015329,
                "M2": m["M2"], "M3": m["M3"], "ce": ce, "delta_h": dh, "zero_samples": z})
    st.close()
    del st
    torch.cuda.empty_cache()
    return out


def ensemble_timings(sv, C, torch, count, reps=3):
    """The ensemble of Sec. IV circuits (grids 4x5, 4x6, 5x5; depth 20..40):
    one launch per sweep round over all instances (default), the persistent
    work-queue launch, and the ordinary per-instance launches, each captured
    in a graph."""
    import numpy as np
    circs = C.make_ensemble(count)
    args = sv.BatchArgs(circs)
    states = [sv.State(c.n, "c64") for c in circs]
    state_bytes = sum(8.0 * 2 ** c.n for c in circs)
    out = {"workload": "%d instances, grids 4x5/4x6/5x5, depth 20..40, complex64, %.1f GB of states"
                       % (count, state_bytes / 1e9)}
    runs = [("auto", {}), ("regtile_t4", dict(mode="regtile", tile=4)),
            ("regtile_t5", dict(mode="regtile", tile=5)), ("regtile_t6", dict(mode="regtile", tile=6)),
            ("persistent_t5", dict(mode="regtile", tile=5, persistent=True)),
            ("launches_t5", dict(mode="regtile", tile=5, launches=True))]
    for label, kw in runs:
        t0 = time.perf_counter()
        res = sv.apply_batch(states, circs, args=args, **kw)      # plans, width, graph
        first = time.perf_counter() - t0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            res = sv.apply_batch(states, circs, args=args, **kw)
        dt = (time.perf_counter() - t0) / reps
        rec = {"s": round(dt, 4), "first_call_s": round(first, 3),
               "instances_per_s": round(count / dt, 1)}
        if "tile" in kw:
            by = sum(sv.host_plan(c, "c64", "regtile", 0, kw["tile"])["bytes"] for c in circs) + state_bytes
            rec["GBps"] = round(by / dt / 1e9, 1)
        ent = np.array([r["entropy"] for r in res])
        norm = np.array([r["norm"] for r in res])
        rec["max_norm_err"] = float(np.abs(norm - 1).max())
        rec["mean_entropy_gap"] = float(np.mean([math.log(2.0 ** c.n) - e for c, e in zip(circs, ent)]))
        out[label] = rec
        log("ensemble %s: %.3f s (first call %.2f s)" % (label, dt, first))
    for st in states:
        st.close()
    del states
    torch.cuda.empty_cache()
    return out


def grad_timings(sv, C, torch):
    """Adjoint gradient of the 5x5 depth-30 parametrised circuit (every
    non-Hadamard gate a rotation offset, theta ~ N(0, 0.05^2)) on 10^4
    samples of the theta = 0 circuit: backward seconds over forward seconds.
    ready_cN: the backward reuses the output state of the forward (what an
    autograd step does); full_cN: the backward recomputes the forward and
    keeps a state copy every N cycles."""
    import numpy as np
    circ = C.make_circuit(5, 5, 30, seed=4, parametrise=True, theta_seed=4004, theta_std=0.05)
    nominal = circ.with_theta(np.zeros(circ.nparams))
    st = sv.State(circ.n, "c64")
    st.apply(nominal, "regtile", 0, 6, from_zero=True)
    xs = st.sample(10000, 1004)
    args = sv.CircuitArgs(circ)
    st.apply(circ, "auto", args=args, from_zero=True)
    for _ in range(8):
        st.apply(circ, "auto", args=args, from_zero=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        st.apply(circ, "auto", args=args, from_zero=True)
    torch.cuda.synchronize()
    fwd = (time.perf_counter() - t0) / 5
    out = {"workload": "5x5 grid, 25 qubits, depth 30, %d parametrised gates, complex64, 1e4 samples"
                       % circ.nparams, "forward_s": round(fwd, 5)}
    for tile in (4, 5):
        for ck, ready in ((0, True), (0, False), (5, False), (10, False)):
            def once():
                if ready:
                    st.apply(circ, "auto", args=args, from_zero=True)
                    torch.cuda.synchronize()
                t = time.perf_counter()
                r = st.backward(circ, xs, checkpoint_c=ck, tile=tile, state_ready=ready)
                return time.perf_counter() - t, r
            once()
            best = None
            for _ in range(3):
                dt, (loss, g) = once()
                best = dt if best is None else min(best, dt)
            key = "%s_c%d_t%d" % ("ready" if ready else "full", ck, tile)
            out[key] = {"grad_s": round(best, 5), "grad_over_fwd": round(best / fwd, 3), "loss": loss}
            log("grad %s: %.4f s (fwd %.4f s)" % (key, best, fwd))
    st.close()
    return out


if __name__ == "__main__":
    main()
