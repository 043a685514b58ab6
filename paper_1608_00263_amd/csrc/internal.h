// Internal declarations shared by the library's translation units (host and
// device).  Not part of the public ABI (include/sv.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/sv.h"

namespace svi {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
void set_error(const std::string &msg);
sv_status fail(sv_status st, const std::string &msg);
sv_status hip_fail(hipError_t e, const char *what);

#define SV_HIP(call)                                                 \
    do {                                                             \
        hipError_t e_ = (call);                                      \
        if (e_ != hipSuccess) return ::svi::hip_fail(e_, #call);     \
    } while (0)

#define SV_TRY(expr)                                                 \
    do {                                                             \
        sv_status s_ = (expr);                                       \
        if (s_ != SV_OK) return s_;                                  \
    } while (0)

// ---------------------------------------------------------------------------
// complex helpers (host side, FP64)
// ---------------------------------------------------------------------------
struct cd {
    double re, im;
};
inline cd cmul(cd a, cd b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
inline cd cadd(cd a, cd b) { return {a.re + b.re, a.im + b.im}; }
inline cd cconj(cd a) { return {a.re, -a.im}; }

// 2x2 complex matrix, row-major: m[0] m[1] / m[2] m[3]
struct M2 {
    cd m[4];
};
M2 m2_mul(const M2 &a, const M2 &b);   // a * b
M2 m2_dag(const M2 &a);

// Gate matrix of a record (kind, rotation offset).  False on a bad kind.
bool gate_matrix(int kind, double theta, const double *mat8, M2 *out);
// dU/dtheta = D U for the rotation kinds; false for others.
bool derivative_generator(int kind, M2 *out);

// ---------------------------------------------------------------------------
// tile programs (device-readable, 8-byte aligned plain structs)
// ---------------------------------------------------------------------------
constexpr int LANE_BITS = 6;          // 64-lane wavefront = qubits 0..5

// register-tile ops
enum RTKind : int32_t {
    RT_REG = 1,     // dense 2x2 on register slot a
    RT_LANE = 2,    // dense 2x2 on lane bit a (cross-lane shuffles)
    RT_SIGNS = 3,   // nterms sign flips (CZ) starting at term index a
    RT_PHASE = 4,   // one general diagonal phase term (index a)
};

// Arithmetic forms of a single-qubit gate inside a register tile.  The
// Clifford forms are the gate times sqrt(2) (entries 0, +-1, +-i: adds
// only); the sweep's store rescales by the accumulated power of sqrt(2).
enum RTForm : int32_t {
    F_GEN = 0,      // general 2x2 matrix u
    F_H = 1,        // [[1, 1], [1, -1]]        (sqrt2 H)
    F_SX = 2,       // [[1, -i], [-i, 1]]       (sqrt2 X^1/2)
    F_SY = 3,       // [[1, -1], [1, 1]]        (sqrt2 Y^1/2)
    F_SXDG = 4,     // [[1, i], [i, 1]]
    F_SYDG = 5,     // [[1, 1], [-1, 1]]
    F_PHASE = 6,    // diag(1, u[3])
    F_RX = 7,       // [[c, -i s], [-i s, c]]   (c = u00, s = -Im u01)
    F_RY = 8,       // [[c, -s], [s, c]]         (c = u00, s = u10)
    F_REAL = 9,     // real 2x2 matrix
    // rotations divided by their cosine c (the factors c of a sweep are
    // applied once, as RTHeader::fscale, when the tile is stored)
    F_TRX = 10,     // [[1, -i t], [-i t, 1]]  (t = -Im u01)
    F_TRY = 11,     // [[1, -t], [t, 1]]       (t = u10)
};

// True for the forms that carry a factor sqrt2.
inline bool form_scaled(int f) { return f >= F_H && f <= F_SYDG; }

// Derivative generators with closed-form gradient terms (dU = D U):
// D = -(i/2) X for RX, -(i/2) Y for RY, i |1><1| for the phase gate.
enum GradKind : int32_t { G_GEN = 0, G_RX = 1, G_RY = 2, G_P = 3 };

struct RTOp {               // 160 bytes
    int32_t kind;
    int32_t a;              // register slot / lane bit / first term
    int32_t nterms;
    int32_t slot;           // adjoint: gradient slot of this gate, or -1
    double u[8];            // 2x2 complex (re, im) row-major
    double d[8];            // adjoint: derivative generator D (dU = D U)
    int32_t form;           // RTForm
    int32_t gkind;          // GradKind of the generator
    double gscale;          // adjoint: factor of the gradient share (the
                            // square of the cosines applied before it)
};

// A diagonal term: amplitude x is multiplied by `val` (or negated for
// RT_SIGNS) iff (x & qmask) == qmask.  The mask is split by where the bits
// live in the tile: lane bits, register slots (expanded to the set of
// register indices it selects) and bits outside the tile.
struct DiagTerm {           // 48 bytes
    uint64_t outside;       // global bits outside the tile
    uint64_t regset;        // bit r set if register index r matches
    uint32_t lanemask;      // lane bits (0..5)
    uint32_t pad;
    double val[2];          // phase (RT_PHASE)
    uint64_t pad2;
};

// The same op in 64 bytes with an FP32 matrix: what a complex64 tile reads
// per op (one scalar load, fetched while the previous op runs).
struct RTOpF {              // 64 bytes
    int32_t kind;
    int32_t a;
    int32_t nterms;
    int32_t form;
    float u[8];
    int32_t pad[4];
};

struct RTHeader {           // 128 bytes
    int32_t nops;
    int32_t vbits;
    int32_t rq[8];          // register qubits, ascending
    int32_t nterms;
    int32_t op_off;         // byte offset of the RTOp array from the header
    int32_t term_off;       // byte offset of the DiagTerm array
    int32_t sexp;           // store: amplitudes scaled by 2^sexp ...
    int32_t shalf;          // ... and by 1/sqrt2 when set
    int32_t gen_n;          // > 0: do not load; start from the uniform state
                            // 2^{-gen_n/2} of gen_n qubits (Hadamard layer)
    double fscale;          // store: amplitudes also scaled by fscale (the
                            // product of the cosines of the F_TRX/F_TRY ops)
    int32_t lq[2];          // qubits on lane bits 4 and 5 (lane bits 0..3 are
                            // qubits 0..3); 4 and 5 give contiguous rows
    int32_t tq[8];          // the tile's qubits above 3 (lane qubits and
                            // register qubits), ascending: vbits + 2 entries
    int32_t fop_off;        // byte offset of the RTOpF array from the header
    int32_t gph_off;        // gen_n > 0 and gph_off > 0: byte offset of the
                            // RTGenPhases of the generated state, then
    int32_t gph_nout;       // gph_nout RTGenOut records
    int32_t pad2;
};

// Single-qubit diagonal gates that act on the uniform state before any dense
// gate on their qubit, folded into the generated values of the first sweep:
// amplitude x of a tile = 2^{-n/2} c prod_{q: x_q = 1} ratio_q, with ratio_q
// = d1/d0 of the gates on q and c the product of their d0.
struct RTGenPhases {
    double c[2];
    double lane[6][2];      // ratio of the qubit on lane bit b (1: none)
    double reg[8][2];       // ratio of the qubit in register slot s (1: none)
};
struct RTGenOut {           // a qubit outside the tile: its ratio applies to
    uint64_t mask;          // the tiles whose base has the bit set
    double r[2];
    uint64_t pad;
};

// LDS-tile ops
enum LTKind : int32_t {
    LT_BLOCK = 1,           // dense 2^k block on local positions pos[0..k-1]
    LT_SIGNS = 2,           // sign flips (terms use local masks)
    LT_PHASE = 3,           // general diagonal phase term
};

struct LTOp {               // 64 bytes
    int32_t kind;
    int32_t k;
    int32_t pos[5];         // ascending local bit positions
    int32_t mat_off;        // byte offset of the matrix from the header
    int32_t nterms;
    int32_t term0;
    int32_t mfma;           // LT_BLOCK with k >= 4: run on the matrix cores
    int32_t pad[5];
};

struct LTTerm {             // 32 bytes
    uint64_t outside;       // global bits outside the tile
    uint32_t localmask;     // local bits of the tile index
    uint32_t itset;         // per-thread element slots i (local index
                            // t + 256 i) whose bits 8.. match localmask
    double val[2];
};

struct LTHeader {           // 64 bytes
    int32_t nops;
    int32_t mbits;          // tile = 2^mbits amplitudes
    int32_t hq[8];          // gathered (non-lane) qubits, ascending
    int32_t op_off;
    int32_t term_off;
    int32_t pad[4];
};

// ---------------------------------------------------------------------------
// plans
// ---------------------------------------------------------------------------
enum OpType : int32_t {
    OP_INIT_UNIFORM = 1,    // psi_x = 2^{-n/2} (Hadamard layer on |0..0>)
    OP_INIT_ZERO,           // psi = |0..0>
    OP_PLAIN_1Q,            // dense 2x2 on q0, full sweep
    OP_PLAIN_CZ,            // controlled-Z as a controlled dense gate
    OP_SPEC_DENSE,          // dense 2x2, general complex
    OP_SPEC_REAL,           // dense 2x2 with real entries (e.g. H, Y^1/2)
    OP_SPEC_DIAG,           // multiply amplitudes with bit q0 set by m[3]
    OP_SPEC_CZ,             // negate amplitudes with bits q0 and q1 set
    OP_REGTILE,             // register-tile program
    OP_LDSTILE,             // LDS-tile program
    OP_ADJ_REGTILE,         // adjoint register-tile program (phi and mu)
    OP_STATS,               // statistics pass over the state into row q0
};

struct Op {
    OpType type;
    int32_t q0 = -1, q1 = -1;
    M2 u{};
    int32_t vbits = 0;      // REGTILE: register qubits; LDSTILE: tile bits
    size_t prog_off = 0;    // byte offset in the plan's program buffer
    double bytes = 0;       // algorithmic HBM bytes of this sweep
    int32_t mfma = 0;       // LDSTILE program uses matrix-core blocks
    // LDSTILE: q1 = the widest block, q0 = 1 when every block of 4 or 5
    // qubits runs on the matrix cores (selects the kernel variant)
    // adjoint plans: q1 of a forward REGTILE op = the checkpoint its store
    // also writes, of an ADJ_REGTILE op = the checkpoint it reads phi from
    // (-1: none)
};

struct Plan {
    std::vector<Op> ops;
    std::vector<Op> bops;        // adjoint: backward sweep sequence
    std::vector<int> slot_param; // adjoint: parameter index of each slot
    std::vector<int> cycle_row;  // per-cycle statistics: the row (OP_STATS
                                 // q0) holding the statistics of cycle t
    int ncheckpoints = 0;
    std::vector<uint8_t> prog;   // host copy of all tile programs
    void *dprog = nullptr;       // device copy
    int64_t sweeps = 0;
    double bytes = 0;
    int n = 0;
    int dtype = 0;
    ~Plan();
};

// Gate after specialisation.
enum SKind { SG_DENSE = 0, SG_DIAG1 = 1, SG_CZ = 2 };
struct SGate {
    int kind;
    int q0, q1;
    M2 u;            // dense: 2x2; diag1: diag(u.m[0], u.m[3])
    int src;         // index of the source gate
    int slot = -1;   // parametrised gate: its gradient slot (list order)
    M2 d{};          // derivative generator of a parametrised gate
    int form = 0;    // RTForm of the exact gate (F_GEN once altered)
    int gkind = 0;   // GradKind of a parametrised gate
};

struct PlanRequest {
    int n;
    int dtype;           // sv_dtype
    int mode;
    int k_max;
    int tile;            // tile qubits (TILED) / register qubits (REGTILE)
    int budget;          // REGTILE arithmetic budget per sweep (0 = default)
    bool from_zero;      // state is |0..0>: a leading Hadamard layer may be
                         // replaced by the uniform initialisation
    bool force_zero;     // the plan must itself start from |0..0>
    bool no_mfma;        // k >= 4 blocks on the VALU
};

// Validate the circuit and produce the specialised gate list in order.
sv_status specialise(const sv_circuit *c, int n, std::vector<SGate> *out);
// Fold single-qubit diagonal gates into neighbouring dense gates on the
// same qubit (exact algebra, FP64).  With param_safe, parametrised gates
// are never folded and a diagonal is folded into a parametrised gate only
// on the side that keeps dU = D U valid.  With keep_cheap, gates with an
// add-only register-tile form are left alone.
void fold_diagonals(std::vector<SGate> *g, int n, bool param_safe = false, bool keep_cheap = false);
sv_status build_plan(const sv_circuit *c, const PlanRequest &rq, Plan *plan);
// Forward and backward sweep sequences of the adjoint gradient, with a
// checkpoint after every checkpoint_c cycles (0 = none).
sv_status build_adjoint_plan(const sv_circuit *c, const PlanRequest &rq, int checkpoint_c,
                             Plan *plan);
double state_bytes(int n, int dtype);
// Sweeps of c from |0..0> with a statistics pass (OP_STATS) wherever the
// state's probabilities are those after a cycle: dense gates never cross a
// cycle's end, diagonal gates may (they leave every |psi_x|^2 unchanged), and
// cycles whose gates are all diagonal share the previous cycle's row.
// Modes: REGTILE (AUTO), SPEC, PLAIN.
sv_status build_cycle_plan(const sv_circuit *c, const PlanRequest &rq, Plan *plan);

// ---------------------------------------------------------------------------
// state handle
// ---------------------------------------------------------------------------
struct Workspace {
    void *ptr = nullptr;
    size_t bytes = 0;
    sv_status reserve(size_t need);
    ~Workspace();
};

}  // namespace svi

namespace svi {
// autotuner record for one circuit
struct Tune {
    std::vector<sv_opts> cand;
    std::vector<double> ms;
    size_t next = 0;
    int best = -1;
};
}  // namespace svi

struct sv_state {
    int n = 0;
    sv_dtype dt = SV_C64;
    void *data = nullptr;
    bool owned = false;
    hipStream_t stream = nullptr;
    int device = 0;
    bool known_zero = false;     // contents are |0..0>
    svi::Workspace ws;           // reductions, sampler
    svi::Workspace ws2;          // adjoint second state, sample staging
    svi::Workspace ws_ck;        // adjoint checkpoints
    std::string ck_key;          // adjoint plan whose forward left its
                                 // checkpoints in ws_ck and its output in
                                 // the state (empty: none)
    std::map<std::string, std::shared_ptr<svi::Plan>> plans;
    std::map<std::string, svi::Tune> tunes;   // explore-on-use records
};

namespace svi {

// ---------------------------------------------------------------------------
// launchers (sweeps.hip)
// ---------------------------------------------------------------------------
// ck (register-tile sweeps only): also store the swept state there
sv_status launch_op(sv_state *st, const Plan &plan, const Op &op, void *psi, void *ck = nullptr);
sv_status get_plan(sv_state *st, const sv_circuit *c, PlanRequest rq, std::shared_ptr<Plan> *out);
sv_status run_plan(sv_state *st, const Plan &plan);
sv_status launch_init_zero(sv_state *st, void *psi);
sv_status upload_plan(sv_state *st, Plan *plan);

// reductions (reduce.hip)
sv_status run_probs(sv_state *st, uint64_t begin, uint64_t count, int f64, void *out);
sv_status run_stats(sv_state *st, const void *psi, sv_stats *out);
// statistics pass of st's state into res[0..14) without synchronising; part
// holds up to 2048 partial rows of 16 doubles
sv_status batch_stats_enqueue(sv_state *st, double *part, double *res);
// the normalised statistics from the 14 combined sums of a 2^n state
void finish_stats_row(int n, const double *r, sv_stats *out);
sv_status run_norm(sv_state *st, const void *psi, double *S);
sv_status run_sample(sv_state *st, const void *psi, int64_t k, uint64_t seed,
                     uint64_t *dev_out);
sv_status run_stats_sample(sv_state *st, const void *psi, sv_stats *stats, int64_t k, uint64_t seed,
                           uint64_t *dev_out);
sv_status run_sample_from(const double *probs, uint64_t N, const uint64_t *r64,
                          int64_t k, uint64_t *out, hipStream_t s);
// sv_moments_sample on the fixed device scratch (no allocation); the bytes
// of scratch it needs for (n, k), and the fixed scratch size
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
size_t noalloc_scratch_need(int n, int64_t k);
sv_status run_stats_sample_noalloc(sv_state *st, sv_stats *stats, int64_t k, uint64_t seed, uint64_t *dev_out);
// pair statistics of a and b (same n, dtype, stream): the 11 combined sums
// into sums16 (S_a, S_b, Re, Im <a|b>, sum p_a^2, sum p_b^2, sum p_a p_b,
// sum p_b ln p_a, sum ln p_a, sum of p_b where p_a = 0, zero count), and
// with nbins > 0 the 3 (nbins + 2) histogram words into host_hist
sv_status run_pair_stats(sv_state *a, sv_state *b, int nbins, const double *host_thr, double *sums16,
                         uint64_t *host_hist);
// sv_apply_circuit with SV_FLAG_CHECKPOINTS: the forward sweeps of the
// adjoint plan, keeping its checkpoints for a later sv_backward
sv_status run_forward_checkpoints(sv_state *st, const sv_circuit *c, const sv_opts *opts);
sv_status run_cross_entropy(sv_state *st, const void *psi, const uint64_t *dev_samples,
                            int64_t k, double S, double *sum_log, int64_t *zeros);

std::string plan_key(const sv_circuit *c, const PlanRequest &rq);

}  // namespace svi
