// Gate sweeps over the state on gfx950.
//
// Every kernel here streams the state through the chip once (read + write,
// in place).  The layouts follow the CDNA wavefront: 64 lanes, so qubits
// 0..5 of an amplitude index map to the lanes of a wavefront and every
// wave-wide access touches 64 consecutive amplitudes (512 B in complex64,
// 1 KiB in complex128).
//
//  * per-gate kernels: the pair update of App. B, Eq. (sqgunitaryoperation),
//    one thread per amplitude pair; specialised forms touch only the
//    amplitudes a diagonal gate changes;
//  * register tiles: each wavefront owns 64 x 2^v amplitudes (lanes = qubits
//    0..5, registers = v gathered qubits); gates on register qubits are
//    register arithmetic, gates on lane qubits exchange values across lanes,
//    CZ gates anywhere are sign flips evaluated from the index bits;
//  * LDS tiles: a workgroup stages 2^m amplitudes (qubits 0..5 plus m-6
//    gathered qubits) in LDS and applies dense 2^k x 2^k blocks to it, on
//    the VALU for k <= 3 and on the matrix cores for k = 4, 5 in complex64
//    (v_mfma_f32_32x32x2f32) and k = 5 in complex128 (v_mfma_f64_16x16x4f64),
//    the complex product as a real 2x2-block embedding.
#include <hip/hip_runtime.h>

#include <cmath>

#include "internal.h"
#include "device_common.h"

namespace svi {

static unsigned grid_for(uint64_t items) {
    uint64_t g = (items + BLOCK - 1) / BLOCK;
    const uint64_t cap = 256ull * 64;   // enough waves to fill every CU
    return (unsigned)(g < cap ? (g ? g : 1) : cap);
}

// ---------------------------------------------------------------------------
// state initialisation
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_fill(cplx<T> *__restrict__ psi, uint64_t N, T value,
                                                int first_one) {
    uint64_t stride = (uint64_t)gridDim.x * BLOCK;
    for (uint64_t i = (uint64_t)blockIdx.x * BLOCK + threadIdx.x; i < N; i += stride) {
        cplx<T> v;
        v.re = (first_one && i == 0) ? (T)1 : value;
        v.im = 0;
        psi[i] = v;
    }
}

// ---------------------------------------------------------------------------
// per-gate kernels
// ---------------------------------------------------------------------------
// dense 2x2 on qubit q (general complex or real entries)
template <typename T, bool REAL>
__global__ __launch_bounds__(BLOCK) void k_pair(cplx<T> *__restrict__ psi, int q, uint64_t npairs,
                                                Mat2<T> u) {
    uint64_t stride = (uint64_t)gridDim.x * BLOCK;
    for (uint64_t p = (uint64_t)blockIdx.x * BLOCK + threadIdx.x; p < npairs; p += stride) {
        uint64_t i0 = insert_zero(p, q), i1 = i0 | (1ull << q);
        cplx<T> a = psi[i0], b = psi[i1], x, y;
        if (REAL) {
            x.re = fma(u.m[0].re, a.re, u.m[1].re * b.re);
            x.im = fma(u.m[0].re, a.im, u.m[1].re * b.im);
            y.re = fma(u.m[2].re, a.re, u.m[3].re * b.re);
            y.im = fma(u.m[2].re, a.im, u.m[3].re * b.im);
        } else {
            x = cmad(u.m[1], b, cmul(u.m[0], a));
            y = cmad(u.m[3], b, cmul(u.m[2], a));
        }
        psi[i0] = x;
        psi[i1] = y;
    }
}

// controlled dense gate (control c, target t): pairs over t where c is set
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_pair_controlled(cplx<T> *__restrict__ psi, int lo, int hi,
                                                           int c, int t, uint64_t npairs, Mat2<T> u) {
    uint64_t stride = (uint64_t)gridDim.x * BLOCK;
    for (uint64_t p = (uint64_t)blockIdx.x * BLOCK + threadIdx.x; p < npairs; p += stride) {
        uint64_t i0 = insert_zero(insert_zero(p, lo), hi) | (1ull << c);
        uint64_t i1 = i0 | (1ull << t);
        cplx<T> a = psi[i0], b = psi[i1];
        psi[i0] = cmad(u.m[1], b, cmul(u.m[0], a));
        psi[i1] = cmad(u.m[3], b, cmul(u.m[2], a));
    }
}

// diagonal diag(1, d) on qubit q: only amplitudes with bit q set
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_diag(cplx<T> *__restrict__ psi, int q, uint64_t nhalf,
                                                cplx<T> d) {
    uint64_t stride = (uint64_t)gridDim.x * BLOCK;
    for (uint64_t p = (uint64_t)blockIdx.x * BLOCK + threadIdx.x; p < nhalf; p += stride) {
        uint64_t i = insert_zero(p, q) | (1ull << q);
        psi[i] = cmul(d, psi[i]);
    }
}

// CZ: negate amplitudes with bits a < b both set
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_cz(cplx<T> *__restrict__ psi, int a, int b, uint64_t nq) {
    uint64_t stride = (uint64_t)gridDim.x * BLOCK;
    for (uint64_t p = (uint64_t)blockIdx.x * BLOCK + threadIdx.x; p < nq; p += stride) {
        uint64_t i = insert_zero(insert_zero(p, a), b) | (1ull << a) | (1ull << b);
        cplx<T> v = psi[i];
        v.re = -v.re;
        v.im = -v.im;
        psi[i] = v;
    }
}

// ---------------------------------------------------------------------------
// register tiles
// ---------------------------------------------------------------------------
// Up to 128 registers of tile data (2^VB amplitudes per lane) the kernel fits
// 3 waves per SIMD, which the launch bound keeps.
template <typename T, int VB>
__global__ __launch_bounds__(BLOCK, (sizeof(T) << VB) <= 256 ? 3 : 1) void k_regtile(cplx<T> *__restrict__ psi,
                                                   const uint8_t *__restrict__ prog,
                                                   uint64_t ntiles, cplx<T> *__restrict__ ck) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint64_t tile = (uint64_t)blockIdx.x * (BLOCK / 64) + wave;
    if (tile >= ntiles) return;
    regtile_apply<T, VB>(psi, prog, tile, lane, ck);
}

// ---------------------------------------------------------------------------
// LDS tiles
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t insert_zero32(uint32_t x, int q) {
    uint32_t lo = x & ((1u << q) - 1);
    return ((x >> q) << (q + 1)) | lo;
}

// Dense 2^K block on the VALU: each thread owns whole columns (assignments
// of the tile bits outside the block) and forms U x for them.
template <typename T, int K, int MB>
__device__ __forceinline__ void block_valu(cplx<T> *lds, const LTOp &op, const cplx<T> *__restrict__ U) {
    constexpr int D = 1 << K;
    constexpr int NCOL = (1 << MB) >> K;
    int pos[K];
#pragma unroll
    for (int j = 0; j < K; j++) pos[j] = op.pos[j];
    uint32_t off[D];
    off[0] = 0;
#pragma unroll
    for (int s = 1; s < D; s++) off[s] = off[s & (s - 1)] | (1u << pos[__builtin_ctz(s)]);
    for (int c = threadIdx.x; c < NCOL; c += BLOCK) {
        uint32_t b = (uint32_t)c;
#pragma unroll
        for (int j = 0; j < K; j++) b = insert_zero32(b, pos[j]);
        cplx<T> x[D];
#pragma unroll
        for (int s = 0; s < D; s++) x[s] = lds[b + off[s]];
#pragma unroll
        for (int r = 0; r < D; r++) {
            cplx<T> acc;
            acc.re = 0;
            acc.im = 0;
#pragma unroll
            for (int s = 0; s < D; s++) acc = cmad(U[r * D + s], x[s], acc);
            lds[b + off[r]] = acc;
        }
    }
}

typedef float floatx16 __attribute__((ext_vector_type(16)));

// Dense 2^K block (K = 4, 5) on the matrix cores, complex64.
//   out = U in  ->  [re; im] interleaved per amplitude:
//   E[2a + ra][2b + rb] = Ur (ra == rb), -Ui (ra=0, rb=1), Ui (ra=1, rb=0)
// v_mfma_f32_32x32x2f32 computes D(32x32) += A(32x2) B(2x32); step b uses
// the two components of input amplitude b, one 32-column chunk of the tile
// per wave and instruction sequence.  Rows 0..31 of E are output amplitudes
// 0..15 (one M block); K = 5 needs a second M block for amplitudes 16..31.
template <int K, int MB>
__device__ __forceinline__ void block_mfma(cplx<float> *lds, const LTOp &op,
                                           const float *__restrict__ F) {
    constexpr int D = 1 << K;
    constexpr int NMB = D / 16;                       // M blocks of 32 real rows
    constexpr int NCOL = (1 << MB) >> K;
    constexpr int NCHUNK = NCOL / 32;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int half = lane >> 5;                       // 0: re, 1: im component
    const int l32 = lane & 31;
    int pos[K];
#pragma unroll
    for (int j = 0; j < K; j++) pos[j] = op.pos[j];
    uint32_t off[D];
    off[0] = 0;
#pragma unroll
    for (int s = 1; s < D; s++) off[s] = off[s & (s - 1)] | (1u << pos[__builtin_ctz(s)]);
    // A fragments, stored by the planner in lane order: lane holds
    // E[row = l32 + 32 mb][2 b + half]
    float afrag[NMB][D];
#pragma unroll
    for (int mb = 0; mb < NMB; mb++)
#pragma unroll
        for (int b = 0; b < D; b++) afrag[mb][b] = F[(mb * D + b) * 64 + lane];
    for (int ch = wave; ch < NCHUNK; ch += BLOCK / 64) {
        uint32_t base = (uint32_t)(ch * 32 + l32);
#pragma unroll
        for (int j = 0; j < K; j++) base = insert_zero32(base, pos[j]);
        floatx16 acc[NMB];
#pragma unroll
        for (int mb = 0; mb < NMB; mb++)
#pragma unroll
            for (int i = 0; i < 16; i++) acc[mb][i] = 0.f;
#pragma unroll
        for (int b = 0; b < D; b++) {
            const cplx<float> v = lds[base + off[b]];
            const float bv = half ? v.im : v.re;
#pragma unroll
            for (int mb = 0; mb < NMB; mb++)
                acc[mb] = __builtin_amdgcn_mfma_f32_32x32x2f32(afrag[mb][b], bv, acc[mb], 0, 0, 0);
        }
        // D[i][j]: lane j + 32 ((i / 4) % 2), register (i % 4) + 4 (i / 8); with
        // i = 2 a + comp this lane holds amplitudes a = 4 g + 2 half + e
        // (re, im) = (acc[4 g + 2 e], acc[4 g + 2 e + 1]) of column l32.
#pragma unroll
        for (int mb = 0; mb < NMB; mb++)
#pragma unroll
            for (int g = 0; g < 4; g++)
#pragma unroll
                for (int e = 0; e < 2; e++) {
                    const int a = 16 * mb + 4 * g + 2 * half + e;   // lane-dependent
                    uint32_t oa = 0;
#pragma unroll
                    for (int j = 0; j < K; j++)
                        if ((a >> j) & 1) oa |= 1u << pos[j];
                    cplx<float> o;
                    o.re = acc[mb][4 * g + 2 * e];
                    o.im = acc[mb][4 * g + 2 * e + 1];
                    lds[base + oa] = o;
                }
    }
}

typedef double doublex4 __attribute__((ext_vector_type(4)));

// Dense 2^K block (K = 5) on the matrix cores, complex128, through
// v_mfma_f64_16x16x4f64: D(16x16) += A(16x4) B(4x16).  The real embedding E
// is the one of the complex64 path; M block mb covers rows 16 mb .. 16 mb + 15
// (output amplitudes 8 mb .. 8 mb + 7), step s covers columns 4 s .. 4 s + 3
// (input amplitudes 2 s and 2 s + 1), and a wave takes 16 tile columns per
// instruction sequence.  Operand layouts (checked on the device): A[i][k] in
// lane i + 16 k, B[k][j] in lane j + 16 k, D[i][j] in lane j + 16 (i % 4),
// element i / 4, so a lane holds one component of four output amplitudes.
template <int K, int MB>
__device__ __forceinline__ void block_mfma_f64(cplx<double> *lds, const LTOp &op,
                                               const double *__restrict__ F) {
    constexpr int D = 1 << K;
    constexpr int NMB = D / 8;                        // M blocks of 16 real rows
    constexpr int NS = D / 2;                         // steps of 4 real columns
    constexpr int NGRP = ((1 << MB) >> K) / 16;       // groups of 16 tile columns
    static_assert(NGRP >= 1, "the tile needs 16 columns per block");
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int col = lane & 15;
    const int kq = lane >> 4;                         // B row within a step
    int pos[K];
#pragma unroll
    for (int j = 0; j < K; j++) pos[j] = op.pos[j];
    uint32_t off[D];
    off[0] = 0;
#pragma unroll
    for (int s = 1; s < D; s++) off[s] = off[s & (s - 1)] | (1u << pos[__builtin_ctz(s)]);
    for (int grp = wave; grp < NGRP; grp += BLOCK / 64) {
        uint32_t base = (uint32_t)(grp * 16 + col);
#pragma unroll
        for (int j = 0; j < K; j++) base = insert_zero32(base, pos[j]);
        // B operands: component kq & 1 of input amplitude 2 s + (kq >> 1)
        double bv[NS];
#pragma unroll
        for (int s = 0; s < NS; s++) {
            const cplx<double> v = lds[base + off[2 * s + (kq >> 1)]];
            bv[s] = (kq & 1) ? v.im : v.re;
        }
        // every input of the column group is in registers now, so each M
        // block is stored as soon as it is done (its A operands are loaded
        // per block: the rolled loop keeps one block's fragments live)
#pragma unroll 1
        for (int mb = 0; mb < NMB; mb++) {
            doublex4 acc;
#pragma unroll
            for (int e = 0; e < 4; e++) acc[e] = 0.0;
            const double *Fm = F + mb * NS * 64 + lane;
#pragma unroll
            for (int s = 0; s < NS; s++) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Fm[s * 64], bv[s], acc, 0, 0, 0);
            // element e = row 16 mb + 4 e + kq of column col: component
            // kq & 1 of output amplitude 8 mb + 2 e + (kq >> 1)
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const int a = 8 * mb + 2 * e + (kq >> 1);   // lane-dependent
                uint32_t oa = 0;
#pragma unroll
                for (int j = 0; j < K; j++)
                    if ((a >> j) & 1) oa |= 1u << pos[j];
                double *dst = reinterpret_cast<double *>(lds + base + oa) + (kq & 1);
                *dst = acc[e];
            }
        }
    }
}

template <typename T, int MB, int KMAX, bool VALU_WIDE>
__device__ __forceinline__ void run_block(cplx<T> *lds, const LTOp &op, const uint8_t *hdr) {
    const cplx<T> *U = reinterpret_cast<const cplx<T> *>(hdr + op.mat_off);
    const float *F = reinterpret_cast<const float *>(hdr + op.mat_off);
    const double *Fd = reinterpret_cast<const double *>(hdr + op.mat_off);
    // op.mfma: the plan chose the matrix cores for this block and stored its
    // operand fragments; it does so for k = 4, 5 in complex64 and k = 5 in
    // complex128, where the tile has the columns the fragments need
    // (2^(MB - k) >= 32 in complex64, >= 64 in complex128)
    switch (op.k) {
    case 1: block_valu<T, 1, MB>(lds, op, U); break;
    case 2: block_valu<T, 2, MB>(lds, op, U); break;
    case 3: block_valu<T, 3, MB>(lds, op, U); break;
    case 4:
        if constexpr (KMAX >= 4) {
            if constexpr (sizeof(T) == 4 && MB >= 9) {
                if (op.mfma) { block_mfma<4, MB>(lds, op, F); break; }
            }
            if constexpr (VALU_WIDE) block_valu<T, 4, MB>(lds, op, U);
        }
        break;
    default:
        if constexpr (KMAX >= 5) {
            if constexpr (sizeof(T) == 4 && MB >= 10) {
                if (op.mfma) { block_mfma<5, MB>(lds, op, F); break; }
            }
            if constexpr (sizeof(T) == 8 && MB >= 11) {
                if (op.mfma) { block_mfma_f64<5, MB>((cplx<double> *)lds, op, Fd); break; }
            }
            if constexpr (VALU_WIDE) block_valu<T, 5, MB>(lds, op, U);
        }
        break;
    }
}

// Apply diagonal terms to the elements a thread owns (local index t + 256 i).
template <typename T, int PER>
__device__ __forceinline__ void diag_regs(cplx<T> (&v)[PER], const LTOp &op, const LTTerm *terms,
                                          uint64_t gbase) {
    const uint32_t t = threadIdx.x;
    if (op.kind == LT_SIGNS) {
        uint32_t par = 0;
        for (int i = op.term0; i < op.term0 + op.nterms; i++) {
            const uint64_t out = terms[i].outside;
            if ((gbase & out) != out) continue;
            const uint32_t lm = terms[i].localmask & 0xFFu;
            par ^= (t & lm) == lm ? terms[i].itset : 0u;
        }
#pragma unroll
        for (int i = 0; i < PER; i++)
            if ((par >> i) & 1) { v[i].re = -v[i].re; v[i].im = -v[i].im; }
    } else {
        for (int i = op.term0; i < op.term0 + op.nterms; i++) {
            const uint64_t out = terms[i].outside;
            if ((gbase & out) != out) continue;
            const uint32_t lm = terms[i].localmask & 0xFFu;
            const uint32_t set = (t & lm) == lm ? terms[i].itset : 0u;
            cplx<T> val;
            val.re = (T)terms[i].val[0];
            val.im = (T)terms[i].val[1];
#pragma unroll
            for (int k = 0; k < PER; k++)
                if ((set >> k) & 1) v[k] = cmul(val, v[k]);
        }
    }
}

template <typename T, int MB, int KMAX, bool VALU_WIDE>
__global__ __launch_bounds__(BLOCK) void k_ldstile(cplx<T> *__restrict__ psi,
                                                   const uint8_t *__restrict__ prog,
                                                   uint64_t ntiles) {
    constexpr int TILE = 1 << MB;
    constexpr int PER = TILE / BLOCK;
    constexpr int NH = MB - LANE_BITS;
    __shared__ cplx<T> lds[TILE];
    const LTHeader *h = reinterpret_cast<const LTHeader *>(prog);
    const uint64_t tile = blockIdx.x;
    if (tile >= ntiles) return;
    int hq[NH];
#pragma unroll
    for (int i = 0; i < NH; i++) hq[i] = h->hq[i];
    uint64_t base = tile << LANE_BITS;
#pragma unroll
    for (int i = 0; i < NH; i++) base = insert_zero(base, hq[i]);
    const LTOp *ops = reinterpret_cast<const LTOp *>(prog + h->op_off);
    const LTTerm *terms = reinterpret_cast<const LTTerm *>(prog + h->term_off);
    const int nops = h->nops;
    int first = nops, last = -1;
    for (int o = 0; o < nops; o++)
        if (ops[o].kind == LT_BLOCK) { if (first == nops) first = o; last = o; }

    // element i of this thread: local index j = t + 256 i; lane bits = t & 63,
    // row = j >> 6 = (t >> 6) + 4 i (wave-uniform).  The row's global offset
    // is the sum of 2^hq[b] over its set bits: the wave's part once, the part
    // of i from compile-time bit patterns, both in scalar registers, and the
    // row pointer is wave-uniform (scalar base + lane offset addressing)
    const int t = threadIdx.x;
    const int col = t & 63;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
    uint64_t woff = 0;
#pragma unroll
    for (int b = 0; b < 2 && b < NH; b++)
        if ((wave >> b) & 1) woff |= 1ull << hq[b];
    auto row_ptr = [&](int i) {
        uint64_t o = woff;
#pragma unroll
        for (int b = 2; b < NH; b++)
            if (((4 * i) >> b) & 1) o |= 1ull << hq[b];
        return uniform_ptr(psi + (base + o));
    };
    cplx<T> v[PER];
#pragma unroll
    for (int i = 0; i < PER; i++) {
        const auto p = row_ptr(i) + col;
        v[i].re = p->re;
        v[i].im = p->im;
    }
    for (int o = 0; o < first && o < nops; o++) diag_regs<T, PER>(v, ops[o], terms, base);
    if (first < nops) {
#pragma unroll
        for (int i = 0; i < PER; i++) lds[t + BLOCK * i] = v[i];
        __syncthreads();
        for (int o = first; o <= last; o++) {
            const LTOp &op = ops[o];
            if (op.kind == LT_BLOCK) {
                run_block<T, MB, KMAX, VALU_WIDE>(lds, op, prog);
            } else {
#pragma unroll
                for (int i = 0; i < PER; i++) v[i] = lds[t + BLOCK * i];
                diag_regs<T, PER>(v, op, terms, base);
#pragma unroll
                for (int i = 0; i < PER; i++) lds[t + BLOCK * i] = v[i];
            }
            __syncthreads();
        }
#pragma unroll
        for (int i = 0; i < PER; i++) v[i] = lds[t + BLOCK * i];
    }
    for (int o = (first < nops ? last + 1 : nops); o < nops; o++)
        diag_regs<T, PER>(v, ops[o], terms, base);
#pragma unroll
    for (int i = 0; i < PER; i++) {
        const auto p = row_ptr(i) + col;
        p->re = v[i].re;
        p->im = v[i].im;
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename T>
static sv_status launch_typed(sv_state *st, const Plan &plan, const Op &op, cplx<T> *psi, cplx<T> *ck) {
    const int n = st->n;
    const uint64_t N = 1ull << n;
    hipStream_t s = st->stream;
    switch (op.type) {
    case OP_INIT_UNIFORM: {
        T v = (T)std::ldexp(1.0, -n / 2);
        if (n & 1) v = (T)(std::ldexp(1.0, -(n / 2)) / std::sqrt(2.0));
        hipLaunchKernelGGL(k_fill<T>, dim3(grid_for(N)), dim3(BLOCK), 0, s, psi, N, v, 0);
        break;
    }
    case OP_INIT_ZERO:
        hipLaunchKernelGGL(k_fill<T>, dim3(grid_for(N)), dim3(BLOCK), 0, s, psi, N, (T)0, 1);
        break;
    case OP_PLAIN_1Q:
    case OP_SPEC_DENSE:
        hipLaunchKernelGGL((k_pair<T, false>), dim3(grid_for(N / 2)), dim3(BLOCK), 0, s, psi, op.q0,
                           N / 2, to_mat<T>(op.u));
        break;
    case OP_SPEC_REAL:
        hipLaunchKernelGGL((k_pair<T, true>), dim3(grid_for(N / 2)), dim3(BLOCK), 0, s, psi, op.q0,
                           N / 2, to_mat<T>(op.u));
        break;
    case OP_PLAIN_CZ: {
        M2 z;
        z.m[0] = {1, 0}; z.m[1] = {0, 0}; z.m[2] = {0, 0}; z.m[3] = {-1, 0};
        int lo = std::min(op.q0, op.q1), hi = std::max(op.q0, op.q1);
        hipLaunchKernelGGL(k_pair_controlled<T>, dim3(grid_for(N / 4)), dim3(BLOCK), 0, s, psi, lo,
                           hi, op.q0, op.q1, N / 4, to_mat<T>(z));
        break;
    }
    case OP_SPEC_DIAG: {
        cplx<T> d;
        d.re = (T)op.u.m[3].re;
        d.im = (T)op.u.m[3].im;
        hipLaunchKernelGGL(k_diag<T>, dim3(grid_for(N / 2)), dim3(BLOCK), 0, s, psi, op.q0, N / 2, d);
        break;
    }
    case OP_SPEC_CZ:
        hipLaunchKernelGGL(k_cz<T>, dim3(grid_for(N / 4)), dim3(BLOCK), 0, s, psi, op.q0, op.q1,
                           N / 4);
        break;
    case OP_REGTILE: {
        const uint8_t *prog = (const uint8_t *)plan.dprog + op.prog_off;
        const uint64_t ntiles = N >> (LANE_BITS + op.vbits);
        const unsigned grid = (unsigned)((ntiles + 3) / 4);
#define RT_CASE(VB) \
    case VB: hipLaunchKernelGGL((k_regtile<T, VB>), dim3(grid), dim3(BLOCK), 0, s, psi, prog, ntiles, ck); break;
        switch (op.vbits) {
            RT_CASE(1) RT_CASE(2) RT_CASE(3) RT_CASE(4) RT_CASE(5) RT_CASE(6)
        default: return fail(SV_EINVAL, "register tile width out of range");
        }
#undef RT_CASE
        break;
    }
    case OP_LDSTILE: {
        const uint8_t *prog = (const uint8_t *)plan.dprog + op.prog_off;
        const uint64_t ntiles = N >> op.vbits;
        const unsigned grid = (unsigned)ntiles;
        // kernel variant by tile width and widest block (k <= 3 variants
        // carry fewer registers, and so do wide variants whose blocks of 4
        // and 5 qubits all run on the matrix cores: op.q0 = 1)
        const bool wide = op.q1 > 3;
        const bool mfma_only = wide && op.q0 == 1;
#define LT_LAUNCH(MB, KM, VW) \
    hipLaunchKernelGGL((k_ldstile<T, MB, KM, VW>), dim3(grid), dim3(BLOCK), 0, s, psi, prog, ntiles)
#define LT_CASE(MB)                                   \
    case MB:                                          \
        if (mfma_only) LT_LAUNCH(MB, 5, false);       \
        else if (wide) LT_LAUNCH(MB, 5, true);        \
        else LT_LAUNCH(MB, 3, false);                 \
        break;
        switch (op.vbits) {
            LT_CASE(8) LT_CASE(9) LT_CASE(10) LT_CASE(11) LT_CASE(12)
        case 13:
            if constexpr (sizeof(T) == 4) {
                if (mfma_only) LT_LAUNCH(13, 5, false);
                else if (wide) LT_LAUNCH(13, 5, true);
                else LT_LAUNCH(13, 3, false);
                break;
            }
            return fail(SV_EINVAL, "LDS tile too large for complex128");
        default: return fail(SV_EINVAL, "LDS tile width out of range");
        }
#undef LT_CASE
#undef LT_LAUNCH
        break;
    }
    default:
        return fail(SV_EINVAL, "unknown op");
    }
    SV_HIP(hipGetLastError());
    return SV_OK;
}

sv_status launch_op(sv_state *st, const Plan &plan, const Op &op, void *psi, void *ck) {
    if (ck && op.type != OP_REGTILE) return fail(SV_EINVAL, "a checkpoint store needs a register-tile sweep");
    if (st->dt == SV_C64) return launch_typed<float>(st, plan, op, (cplx<float> *)psi, (cplx<float> *)ck);
    return launch_typed<double>(st, plan, op, (cplx<double> *)psi, (cplx<double> *)ck);
}

sv_status launch_init_zero(sv_state *st, void *psi) {
    const uint64_t N = 1ull << st->n;
    if (st->dt == SV_C64)
        hipLaunchKernelGGL(k_fill<float>, dim3(grid_for(N)), dim3(BLOCK), 0, st->stream,
                           (cplx<float> *)psi, N, 0.f, 1);
    else
        hipLaunchKernelGGL(k_fill<double>, dim3(grid_for(N)), dim3(BLOCK), 0, st->stream,
                           (cplx<double> *)psi, N, 0.0, 1);
    SV_HIP(hipGetLastError());
    return SV_OK;
}

sv_status upload_plan(sv_state *st, Plan *plan) {
    if (plan->dprog || plan->prog.empty()) return SV_OK;
    SV_HIP(hipMalloc(&plan->dprog, plan->prog.size()));
    SV_HIP(hipMemcpyAsync(plan->dprog, plan->prog.data(), plan->prog.size(), hipMemcpyHostToDevice,
                          st->stream));
    SV_HIP(hipStreamSynchronize(st->stream));
    return SV_OK;
}

}  // namespace svi
