/*
 * sv.h -- C ABI of the MI355X (gfx950) state-vector library for the random
 * lattice circuits of Boixo et al., "Characterizing Quantum Supremacy in
 * Near-Term Devices" (arXiv:1608.00263).
 *
 * The library evolves a 2^n amplitude state on one GPU (Sec. II: the output
 * |psi> = U|psi_0> of a random circuit U, psi_0 = |0...0>), and computes the
 * quantities the paper defines on its output distribution p_U(x) = |<x|psi>|^2:
 * probabilities, entropy, cross entropy with the uniform distribution, the
 * normalised moments N^{k-1} sum_x p^k, bit-string samples and their cross
 * entropy (the estimator of Eq. (ae)), plus the gradient of the sample cross
 * entropy with respect to per-gate rotation offsets.
 *
 * Conventions shared by every call
 *  - Qubit q is bit q of an amplitude index and of a sample (uint64).
 *  - All logarithms are natural (nats).
 *  - Every call returns an sv_status; nothing throws across the ABI.  On a
 *    non-OK status sv_last_error() returns a message (per thread).
 *  - Every device operation is enqueued on the stream of the state handle;
 *    calls that return host scalars synchronise that stream first.
 *  - Pointers are host pointers unless a parameter says "device".
 */
#ifndef SV_ABI_H_INCLUDED
#define SV_ABI_H_INCLUDED

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SV_OK = 0,
    SV_EINVAL = -1,   /* bad argument: qubit, kind, n mismatch, null pointer  */
    SV_ENOMEM = -2,   /* not enough device (or host) memory                  */
    SV_EDEVICE = -3,  /* a HIP runtime call failed (message has the details) */
    SV_ERANGE = -4,   /* size out of range (n, chunk, sample count)          */
    SV_ESTATE = -5    /* call not valid in the handle's current state        */
} sv_status;

typedef enum { SV_C64 = 0, SV_C128 = 1 } sv_dtype;

/* Gate kinds (Sec. IV gate set plus what tests and inverses need).
 * H = Hadamard; CZ = diag(1,1,1,-1); T = diag(1, e^{i pi/4});
 * SX = X^1/2 = RX(pi/2); SY = Y^1/2 = RY(pi/2), with
 * RX(a) = [[cos a/2, -i sin a/2], [-i sin a/2, cos a/2]],
 * RY(a) = [[cos a/2, -sin a/2], [sin a/2, cos a/2]], P(a) = diag(1, e^{ia});
 * S = P(pi/2); X, Y, Z Paulis; *_DG the adjoints; U1 a dense 2x2 taken from
 * sv_circuit.mats.  A gate with param >= 0 is a rotation with angle
 * nominal + theta[param]: T -> P(pi/4 + t), SX -> RX(pi/2 + t),
 * SY -> RY(pi/2 + t), TDG -> P(-pi/4 + t), SXDG -> RX(-pi/2 + t),
 * SYDG -> RY(-pi/2 + t); other kinds must have param = -1. */
typedef enum {
    SV_H = 0, SV_CZ = 1, SV_T = 2, SV_SX = 3, SV_SY = 4, SV_S = 5,
    SV_X = 6, SV_Y = 7, SV_Z = 8, SV_TDG = 9, SV_SDG = 10, SV_SXDG = 11,
    SV_SYDG = 12, SV_U1 = 13
} sv_kind;

/* One gate record (24 bytes).  q1 is the second qubit of CZ, else -1.
 * cycle is the clock cycle (0 = the Hadamard layer); it bounds the
 * adjoint's checkpoints and is otherwise informational.  mat indexes
 * sv_circuit.mats for SV_U1, else -1. */
typedef struct {
    int32_t kind, q0, q1, cycle, param, mat;
} sv_gate;

/* A circuit.  Owned by the caller; the library copies what it keeps. */
typedef struct {
    int32_t n;               /* qubits                                         */
    int32_t nparams;         /* length of theta (0 if none)                    */
    int64_t ngates;
    const sv_gate *gates;
    const double *theta;     /* rotation offsets, may be NULL if nparams == 0  */
    int32_t nmats;
    int32_t reserved;
    const double *mats;      /* nmats 2x2 complex128 matrices, row-major,
                                (re, im) interleaved: 8 doubles per matrix     */
} sv_circuit;

/* How sv_apply_circuit maps gates onto sweeps over the state (a sweep reads
 * and writes the state once):
 *  SV_MODE_PLAIN    one sweep per gate, every gate as a dense 2x2 (CZ as a
 *                   controlled-Z on the pairs whose control bit is set);
 *  SV_MODE_SPEC     one sweep per gate with specialised kernels (diagonal
 *                   gates touch only the lines they change, H is real);
 *  SV_MODE_FUSED    gates fused into dense 2^k x 2^k unitaries (k <= k_max,
 *                   diagonal gates folded in), one LDS-staged sweep each;
 *                   k >= 4 blocks run on the matrix cores (complex64);
 *  SV_MODE_TILED    the fused blocks grouped into LDS tile sweeps of
 *                   2^tile_qubits amplitudes (several blocks per sweep);
 *  SV_MODE_REGTILE  gates applied one by one inside register tiles (qubits
 *                   0..5 across the 64 lanes of a wavefront, a few gathered
 *                   qubits in registers), diagonal gates folded;
 *  SV_MODE_AUTO     time candidate plans once per circuit shape and keep
 *                   the fastest (autotuner; results cached per process). */
enum {
    SV_MODE_PLAIN = 0, SV_MODE_SPEC = 1, SV_MODE_FUSED = 2,
    SV_MODE_TILED = 3, SV_MODE_REGTILE = 4, SV_MODE_AUTO = 5
};

/* sv_opts.flags bits */
enum {
    SV_FLAG_FROM_ZERO = 1,  /* ignore the current contents: simulate U|0...0> */
    SV_FLAG_NO_MFMA = 2,    /* fused blocks with k >= 4 on the VALU instead of
                               the matrix cores (for comparison)             */
    SV_FLAG_STATE_READY = 4,/* sv_backward: the handle already holds U(theta)
                               |0...0> (sv_apply_circuit of the same circuit
                               and theta): the forward pass is skipped; with
                               checkpoint_c > 0 the checkpoints too, kept by
                               sv_apply_circuit with SV_FLAG_CHECKPOINTS    */
    SV_FLAG_BATCH_LAUNCHES = 8, /* sv_apply_batch: one captured graph of the
                               ordinary per-instance launches (for comparison) */
    SV_FLAG_BATCH_PERSISTENT = 16, /* sv_apply_batch: the persistent-kernel
                               schedule instead of one launch per round      */
    SV_FLAG_CHECKPOINTS = 32 /* sv_apply_circuit: run U|0...0> as the forward
                               pass of sv_backward (register tiles of its
                               width, tile_qubits / sweep_budget as there) and
                               keep the state copies it takes every
                               checkpoint_c cycles, so that a following
                               sv_backward with SV_FLAG_STATE_READY and the
                               same circuit, theta, options and interval
                               skips the forward pass                       */
};

typedef struct {
    int32_t mode;         /* SV_MODE_*                                        */
    int32_t k_max;        /* fused block width 1..5 (0 = default 4)           */
    int32_t tile_qubits;  /* TILED: 8..13 (0 = default 12 / 11); REGTILE:
                             register qubits 1..6 complex64, 1..5 complex128
                             (0 = default 6 / 5)                              */
    int32_t flags;        /* SV_FLAG_* bits                                   */
    int32_t sweep_budget; /* REGTILE: vector instructions per amplitude
                             register one sweep may spend on gates before a
                             new sweep starts (0 = default, 250 complex64,
                             220 complex128; 20..2000)                       */
    int32_t checkpoint_c; /* SV_FLAG_CHECKPOINTS: the checkpoint interval of
                             the sv_backward that will follow (0 = none)     */
} sv_opts;

/* Output statistics of p_hat = p / S (Secs. II and IV):
 *  norm      S = sum_x p(x)
 *  entropy   H = -sum p_hat ln p_hat              (Eq. (lps) definition)
 *  unif_ce   -(1/N) sum ln p_hat(x): cross entropy of the uniform sampler
 *            with the output (Eq. (15) with p_cl = 1/N); +inf if some p = 0
 *  moments   moments[k-1] = M_k = (1/N) sum (N p_hat)^k = N^{k-1} IPR_k,
 *            k = 1..10 (Porter-Thomas: M_k -> k!)
 *  zero_count  number of x with p(x) = 0 */
typedef struct {
    double norm, entropy, unif_ce;
    double moments[10];
    int64_t zero_count;
} sv_stats;

/* Statistics of a pair of outputs of the same size: a, the ideal output
 * p_U, and b, another output (an implementation with errors, one Monte
 * Carlo trajectory of it, or a circuit with an inserted error).  With
 * hat p = p / S and N = 2^n:
 *  norm_a, norm_b  S_a, S_b
 *  overlap_re/im   <a|b> = sum_x conj(a_x) b_x
 *  fidelity        |<a|b>|^2 / (S_a S_b) (the alpha of Eq. (ra) for a pure b)
 *  xent            -sum_x hat p_b ln hat p_a: the cross entropy of Eq. (15)
 *                  with b as the sampler; +inf if b has mass where p_a = 0
 *  unif_ce         -(1/N) sum_x ln hat p_a (+inf if some p_a = 0)
 *  delta_h         Eq. (5), sum_x (1/N - hat p_b) ln(1 / hat p_a)
 *                  = unif_ce - xent; NaN if some p_a = 0
 *  corr            Pearson correlation of p_a and p_b over the N outcomes
 *                  (the residual correlation of App. D); NaN if either is
 *                  constant
 *  zero_mass_b     sum of p_b over the x with p_a = 0
 *  zero_a          number of x with p_a = 0 */
typedef struct {
    double norm_a, norm_b, overlap_re, overlap_im, fidelity, xent, unif_ce, delta_h, corr, zero_mass_b;
    int64_t zero_a;
} sv_pair;

typedef struct sv_state sv_state;   /* opaque handle */

/* Allocate a 2^n state in device memory owned by the library and set it to
 * |0...0>.  n in 1..35 for SV_C64, 1..34 for SV_C128 (else SV_ERANGE);
 * SV_ENOMEM if the device cannot hold it.  hip_stream may be NULL (the
 * null stream).  The handle is freed with sv_free. */
sv_status sv_alloc(int n, sv_dtype dt, void *hip_stream, sv_state **out);

/* Wrap a caller-owned device buffer of 2^n interleaved complex amplitudes
 * (float2 for SV_C64, double2 for SV_C128).  The buffer's contents are the
 * state; it must outlive the handle and is never freed by the library. */
sv_status sv_attach(int n, sv_dtype dt, void *dev_ptr, void *hip_stream, sv_state **out);

sv_status sv_free(sv_state *st);

/* Set the state to |0...0> (Sec. II, psi_0).  For a buffer the library
 * owns (sv_alloc) the next sv_apply_circuit may take the contents as known
 * to be |0...0> (and generate a leading Hadamard layer instead of reading
 * the state); an attached buffer is always read, since its owner may have
 * written it in between. */
sv_status sv_reset(sv_state *st);

/* Device pointer of the amplitudes (interleaved re, im). */
sv_status sv_data(sv_state *st, void **dev_ptr);

/* Apply the gates of c in list order to the state, in place (asynchronous
 * on the handle's stream).  The single-qubit update is that of App. B,
 * Eq. (sqgunitaryoperation); CZ is the controlled phase of Sec. IV.
 * opts may be NULL (SV_MODE_AUTO).  SV_EINVAL for an invalid gate or
 * c->n != n.  Plans are cached per circuit. */
sv_status sv_apply_circuit(sv_state *st, const sv_circuit *c, const sv_opts *opts);

/* Number of sweeps over the state the plan for (c, opts) performs, and the
 * algorithmic bytes it moves (reads + writes of the state).  For
 * SV_MODE_AUTO this tunes first if needed (see sv_autotune). */
sv_status sv_plan_info(sv_state *st, const sv_circuit *c, const sv_opts *opts,
                       int64_t *sweeps, double *bytes);

/* Autotuner behind SV_MODE_AUTO: times candidate plans for c on this device
 * -- register tiles with 4, 5 or 6 register qubits (complex64) and 3 or 4
 * (complex128), fused blocks with k = 2 and 3, LDS tiles -- and keeps the
 * fastest for the circuit (cached per process).  The timing runs on a
 * scratch state of the same size when the device has room for one (the
 * handle's contents are untouched); otherwise successive sv_apply_circuit
 * calls on the handle each run the next untried candidate (every call is
 * still exact).  chosen (may be NULL) gets the selected options;
 * *complete = 1 once the choice is final. */
sv_status sv_autotune(sv_state *st, const sv_circuit *c, int from_zero, sv_opts *chosen, int *complete);

/* Sweep kinds reported by sv_apply_circuit_timed. */
enum {
    SV_SWEEP_INIT = 1, SV_SWEEP_PLAIN_1Q = 2, SV_SWEEP_PLAIN_CZ = 3, SV_SWEEP_SPEC_DENSE = 4,
    SV_SWEEP_SPEC_REAL = 5, SV_SWEEP_SPEC_DIAG = 6, SV_SWEEP_SPEC_CZ = 7, SV_SWEEP_REGTILE = 8,
    SV_SWEEP_LDSTILE = 9, SV_SWEEP_LDSTILE_MFMA = 10
};

/* sv_apply_circuit with a HIP event pair around every sweep (measurement of
 * the paper's time-per-gate figures, App. B Table I, on this device).  For
 * i < min(cap, sweeps): op_ms[i] = duration of sweep i, op_kind[i] its
 * SV_SWEEP_* kind, op_bytes[i] its algorithmic bytes (host arrays, any may
 * be NULL); *nops = number of sweeps.  Synchronises. */
sv_status sv_apply_circuit_timed(sv_state *st, const sv_circuit *c, const sv_opts *opts, int64_t cap,
                                 float *op_ms, int32_t *op_kind, double *op_bytes, int64_t *nops);

/* Output probabilities p_U(x) = |<x|psi>|^2 (Sec. II) as re^2 + im^2, for
 * x in [begin, begin + count), written to dev_out (device, count entries,
 * caller-owned) as double (out_f64 = 1) or float (out_f64 = 0).  For
 * SV_C64 both products are exact in double and the sum is rounded once.
 * Asynchronous on the handle's stream.  SV_ERANGE if the range leaves
 * [0, 2^n); SV_EINVAL for a null dev_out with count > 0. */
sv_status sv_probs(sv_state *st, uint64_t begin, uint64_t count, int out_f64, void *dev_out);

/* Output statistics of the current state (one FP64 pass, compensated,
 * deterministic).  Synchronises. */
sv_status sv_moments(sv_state *st, sv_stats *out);

/* Statistics after every cycle (Sec. IV: the entropy, the uniform cross
 * entropy and the moments of the output distribution measured after each
 * cycle t, as in its figures of the approach to Porter-Thomas): simulate c
 * from |0...0> and write to out[t] (host, t = 0..D, D = the largest gate
 * cycle; the cycle of a gate is sv_gate.cycle, 0 = the Hadamard layer) the
 * statistics of the state after the gates of cycles 0..t.  Gates must be
 * listed in nondecreasing cycle order (SV_EINVAL otherwise).  A cycle whose
 * gates are all diagonal (CZ, T, phases) leaves every probability unchanged
 * and reports the previous cycle's statistics without a pass over the state;
 * diagonal gates may be applied across a cycle's end for the same reason,
 * dense gates never are.  opts: SV_MODE_REGTILE (AUTO: register tiles of
 * the default width), SV_MODE_SPEC or SV_MODE_PLAIN, else SV_EINVAL.
 * *ncycles (may be NULL) gets D + 1; SV_ERANGE if cap < D + 1.  On return
 * the state holds the circuit's output U|0...0>.  Synchronises. */
sv_status sv_cycle_moments(sv_state *st, const sv_circuit *c, const sv_opts *opts, int64_t cap,
                           sv_stats *out, int64_t *ncycles);

/* Draw k bit-strings from p(x) = |<x|psi>|^2 (Sec. II, the sample S).
 * Exactly reproducible inverse-transform sampling on an integer CDF:
 * w_x = floor(p(x) 2^62), C_x = w_0 + ... + w_x, W = C_{2^n - 1};
 * r_i = SplitMix64(seed + (i+1) * 0x9E3779B97F4A7C15);
 * t_i = floor(r_i W / 2^64); x_i = min{x : C_x > t_i}.
 * out has k entries, in host memory (out_on_device = 0) or device memory.
 * k in 0..2^31.  Synchronises. */
sv_status sv_sample(sv_state *st, int64_t k, uint64_t seed, uint64_t *out, int out_on_device);

/* sv_moments and sv_sample in one read of the state: the statistic sums and
 * the sampler's integer bucket weights come from the same pass.  The
 * samples are bit-identical to those of sv_sample(st, k, seed, ...); the
 * statistics equal those of sv_moments up to the order of the FP64 sums
 * (workgroups of 2^16 amplitudes here).  k = 0 computes the statistics
 * only; out (k entries, host or device) may then be NULL.  Synchronises. */
sv_status sv_moments_sample(sv_state *st, sv_stats *stats, int64_t k, uint64_t seed, uint64_t *out,
                            int out_on_device);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * statistics and samples of sv_moments_sample, computed by the same kernels
 * (bit-identical results), with every intermediate in one fixed 64 MiB
 * device array that comes with the library's code object on each GPU and is
 * held until the process ends; the call allocates nothing.  dev_out is
 * device memory (k entries, caller-owned; may be NULL when k = 0); stats is
 * a host struct.  The scratch must hold 8 2^(n-10) + 16 2^(n-16) + 12 k
 * bytes plus about 33 KiB of rows (n <= 32; e.g. k up to 4.8 million at
 * n = 30): SV_ERANGE otherwise, before any device work.  Every call on one
 * GPU shares that array and leaves its contents behind (nothing in it needs
 * to start at zero), so calls that overlap on one GPU race: serialise them
 * (one stream, or a host lock).  Synchronises the handle's stream. */
sv_status sv_moments_sample_noalloc(sv_state *st, sv_stats *stats, int64_t k, uint64_t seed,
                                    uint64_t *dev_out);

/* The same sampler on an explicit distribution: probs (device, N doubles,
 * need not sum to 1), r64 (device, k random words used as the r_i above),
 * out (device, k entries, caller-owned).  N is any length in 1..2^35 (else
 * SV_ERANGE).  Every p must be finite, >= 0 and below 4, so that its weight
 * floor(p 2^62) fits 64 bits (else SV_EINVAL), and the weights must sum
 * below 2^64, i.e. sum p < 4 up to the floors (else SV_ERANGE); SV_ESTATE
 * when every weight is 0 and k > 0.  The check is exact (integer sums).
 * Uses a scratch allocation of the library.  Synchronises. */
sv_status sv_sample_from(const double *probs, uint64_t N, const uint64_t *r64,
                         int64_t k, uint64_t *out, void *hip_stream);

/* Sample cross entropy of Eqs. (ae) and (5):
 *   ce = ln S - (1/k) sum_i ln p(x_i),  delta_h = ln 2^n + gamma - ce
 * over k samples (host array); S = sum_x p(x).  norm > 0 is taken as S (the
 * norm sv_moments returned for the same state, which saves a pass over the
 * state); norm <= 0 computes it.  ce = +inf when some p(x_i) = 0;
 * *zero_samples (may be NULL) gets their number.  Samples are n-bit
 * strings: SV_ERANGE (before any device work) if some x_i >= 2^n.
 * Synchronises. */
sv_status sv_cross_entropy(sv_state *st, const uint64_t *samples, int64_t k, double norm,
                           double *ce, double *delta_h, int64_t *zero_samples);

/* Pair statistics (sv_pair) of the ideal output a and another output b
 * (Secs. II and III: Eq. (5), Eq. (ra); App. D), from one read of both
 * states: FP64 sums per workgroup, combined in a fixed order (Neumaier).
 * a and b must have the same n, dtype and stream (else SV_EINVAL).
 * With nbins in 1..1024, hist (host, 3 (nbins + 2) entries) gets the
 * histogram of z(x) = ln(N p_a(x)) over [zmin, zmax) in nbins equal bins,
 * then a slot for p_a below the range or 0 and one for p_a at or above it:
 * hist[s] = number of outcomes in slot s, hist[(nbins + 2) + s] and
 * hist[2 (nbins + 2) + s] = the sums of floor(p_a 2^62) and floor(p_b 2^62)
 * over them (exact integers: mass / 2^62 is the probability mass of the
 * slot under each output, Eq. (pal) at the fidelity of b).  The slot is
 * decided by comparing p_a with the thresholds e^{zmin + j dz} 2^{-n},
 * computed once on the host, so it is exact.  SV_ERANGE for a histogram
 * of an output whose norm is 4 or more (its integer masses would not fit);
 * nbins = 0 skips the histogram (hist may be NULL).  Synchronises. */
sv_status sv_pair_stats(sv_state *a, sv_state *b, int32_t nbins, double zmin, double zmax, sv_pair *out,
                        uint64_t *hist);

/* Gradient of L(theta) = -(1/k) sum_i ln p_theta(x_i) with respect to
 * theta (length c->nparams, host), by the adjoint method: the forward state
 * is rebuilt by applying the inverse gates (no stored history), with a copy
 * of the forward state in the state's precision (complex64 on the bulk
 * path) kept every checkpoint_c cycles (0 = none): at the end of the first
 * sweep after which every gate of cycles <= k checkpoint_c has run (the
 * sweeps are not cut for it), written by that sweep's store; the reverse
 * of that sweep reads phi from the copy instead of the uncomputed state.  The circuit must open with a Hadamard on every
 * qubit and list its gates in nondecreasing cycle order.  On entry the
 * handle may hold anything, unless opts->flags has SV_FLAG_STATE_READY: then
 * it must hold U(theta)|0...0> already (as left by sv_apply_circuit of the
 * same circuit) and the forward pass is skipped; with checkpoint_c > 0 the
 * checkpoints must have been kept by sv_apply_circuit with
 * SV_FLAG_CHECKPOINTS, the same circuit, theta, tile_qubits, sweep_budget
 * and interval, with no call that changes the state in between (else
 * SV_ESTATE).
 * On return its contents are unspecified (the forward state has been
 * uncomputed).  loss gets L(theta).  The reverse sweeps are register tiles:
 * opts->tile_qubits register qubits (0 = default 5 complex64 / 3
 * complex128; clamped to 1..5 / 1..4 and to at most n - 8) under
 * opts->sweep_budget (as for sv_apply_circuit).  Uses device
 * scratch of one extra state plus the checkpoints.  SV_EINVAL if a
 * parametrised gate is not a rotation; SV_ESTATE if a sample has p = 0;
 * SV_ERANGE for n < 8 or a sample x_i >= 2^n (checked before any device
 * work). */
sv_status sv_backward(sv_state *st, const sv_circuit *c, const sv_opts *opts,
                      const uint64_t *samples, int64_t k, int checkpoint_c,
                      double *loss, double *grad);

/* Ensemble (the statistics of Sec. IV are averages over many random circuit
 * instances): simulate count independent circuits from |0...0>, each into
 * its own handle sts[i] (sizes and depths may differ), and write each
 * instance's statistics to out[i].  All handles must share one dtype and
 * stream; opts may be NULL (SV_MODE_AUTO).  Synchronises.
 *
 * Complex64 ensembles whose instances have n >= 14 and whose plans consist
 * of register-tile sweeps only (SV_MODE_AUTO or SV_MODE_REGTILE) are cut into
 * work items (16 register tiles of one sweep of one instance, or 2^14
 * amplitudes of one instance's statistics) ordered by sweep round, then
 * instance.  By default each round is one launch over the items of every
 * instance (the sweeps of all instances fill the GPU together);
 * SV_FLAG_BATCH_PERSISTENT runs the same table in one persistent launch
 * whose workgroups take items from a global queue and wait on per-instance
 * completion counters.  Either schedule is captured in a HIP graph that is
 * kept and replayed while the same handles, circuits and options come again
 * (one such graph per process).  The register-tile width is tile_qubits
 * (clamped to 3..6) under SV_MODE_REGTILE, else the fastest of 4..6 timed
 * on the ensemble itself, once per list of instance sizes (the timing runs
 * write the same outputs).  Everything else (complex128, other modes,
 * smaller instances, SV_FLAG_BATCH_LAUNCHES) runs as one captured graph of
 * the ordinary per-sweep launches.  SV_EDEVICE if a dependency wait of the persistent
 * kernel exceeds its bound (the kernel still drains and exits; the states
 * are then unspecified). */
sv_status sv_apply_batch(sv_state **sts, const sv_circuit *cs, int64_t count,
                         const sv_opts *opts, sv_stats *out);

/* Message for the last non-OK status returned on this thread. */
const char *sv_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SV_ABI_H_INCLUDED */
