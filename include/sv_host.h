/*
 * sv_host.h -- host-only diagnostics of the state-vector library (no GPU
 * needed): inspect the sweep plan built for a circuit and replay it on a
 * host copy of the state.
 *
 * The replay interprets the same tile programs (register tiles, LDS tiles,
 * fused 2^k blocks, sign and phase terms) that the GPU kernels execute, in
 * double precision, so that the planner -- gate specialisation, diagonal
 * folding, fusion, sweep grouping and program encoding -- can be checked
 * on a CPU.  It is a test aid, not a simulator: it is slow and the GPU
 * entry points of sv.h never call it.
 */
#ifndef SV_HOST_H_INCLUDED
#define SV_HOST_H_INCLUDED

#include "sv.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Build the plan sv_apply_circuit would use for (c, dt, opts) on a state
 * whose contents are |0...0> when from_zero is set.  Outputs (any may be
 * NULL): number of sweeps, algorithmic bytes, number of sweeps executed on
 * the matrix cores.  SV_EINVAL for an invalid circuit, as sv_apply_circuit. */
sv_status sv_host_plan(const sv_circuit *c, sv_dtype dt, const sv_opts *opts, int from_zero,
                       int64_t *sweeps, double *bytes, int64_t *mfma_sweeps);

/* Replay that plan on psi: 2^c->n complex128 amplitudes (interleaved re, im,
 * host memory), in place.  Matrices are rounded to the precision of dt
 * exactly as on the GPU. */
sv_status sv_host_emulate(const sv_circuit *c, sv_dtype dt, const sv_opts *opts, int from_zero,
                          double *psi);

/* Replay of the plan sv_cycle_moments runs for (c, dt, opts) from |0...0>
 * (n <= 26): probs (host, cap_rows x 2^n doubles, may be NULL) gets
 * |psi_x|^2 at each statistics point of the plan, row by row; cycle_row
 * (host, cap_cycles entries, may be NULL) the row that reports each cycle
 * t = 0..D; *nrows and *ncycles (may be NULL) their numbers.  SV_ERANGE if
 * cap_rows or cap_cycles is too small (the counts are still written). */
sv_status sv_host_cycle_emulate(const sv_circuit *c, sv_dtype dt, const sv_opts *opts, int64_t cap_rows,
                                double *probs, int32_t *cycle_row, int64_t cap_cycles, int64_t *nrows,
                                int64_t *ncycles);

/* Text description of that plan, one line per sweep (kind, tile qubits,
 * gate and term counts), written to buf (NUL-terminated, at most cap
 * bytes, truncated if longer). */
sv_status sv_host_plan_describe(const sv_circuit *c, sv_dtype dt, const sv_opts *opts, int from_zero,
                                char *buf, int64_t cap);

#ifdef __cplusplus
}
#endif

#endif /* SV_HOST_H_INCLUDED */
