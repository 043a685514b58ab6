// Device helpers shared by the sweep kernels and the adjoint kernels:
// complex arithmetic, index bit insertion, and the register-tile gate
// primitives (in-register pairs and cross-lane pairs of a wavefront).
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace svi {

template <typename T> struct cplx { T re, im; };

template <typename T>
__device__ __forceinline__ cplx<T> cmad(cplx<T> u, cplx<T> x, cplx<T> acc) {
    acc.re = fma(u.re, x.re, acc.re);
    acc.re = fma(-u.im, x.im, acc.re);
    acc.im = fma(u.re, x.im, acc.im);
    acc.im = fma(u.im, x.re, acc.im);
    return acc;
}
template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> u, cplx<T> x) {
    cplx<T> r;
    r.re = fma(u.re, x.re, -u.im * x.im);
    r.im = fma(u.re, x.im, u.im * x.re);
    return r;
}

__device__ __forceinline__ uint64_t insert_zero(uint64_t x, int q) {
    uint64_t lo = x & ((1ull << q) - 1);
    return ((x >> q) << (q + 1)) | lo;
}

template <typename T> struct Mat2 { cplx<T> m[4]; };

template <typename T>
inline Mat2<T> to_mat(const M2 &u) {
    Mat2<T> r;
    for (int i = 0; i < 4; i++) { r.m[i].re = (T)u.m[i].re; r.m[i].im = (T)u.m[i].im; }
    return r;
}

constexpr int BLOCK = 256;

// Value of the lane whose index differs in bit B (a wavefront has 64
// lanes).  Bits 0..3 use DPP lane moves within rows of 16 (quad
// permutations and row mirrors), bit 4 a ds_swizzle swap of 16-lane halves
// of each 32, bit 5 a ds_bpermute.
template <int B>
__device__ __forceinline__ int lane_xor_i(int v) {
    if constexpr (B == 0) return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false);   // quad_perm 1,0,3,2
    if constexpr (B == 1) return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false);   // quad_perm 2,3,0,1
    if constexpr (B == 2) {   // i ^ 7 (half-row mirror), then i ^ 3 (quad reverse): i ^ 4
        int m = __builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, false);
        return __builtin_amdgcn_mov_dpp(m, 0x1B, 0xF, 0xF, false);
    }
    if constexpr (B == 3) {   // i ^ 15 (row mirror), then i ^ 7 (half-row mirror): i ^ 8
        int m = __builtin_amdgcn_mov_dpp(v, 0x140, 0xF, 0xF, false);
        return __builtin_amdgcn_mov_dpp(m, 0x141, 0xF, 0xF, false);
    }
    if constexpr (B == 4) return __builtin_amdgcn_ds_swizzle(v, 0x401F);   // swap 16-lane halves
    if constexpr (B == 5) return __shfl_xor(v, 32, 64);
    return v;
}

template <int B>
__device__ __forceinline__ float lane_xor(float v) {
    return __int_as_float(lane_xor_i<B>(__float_as_int(v)));
}
template <int B>
__device__ __forceinline__ double lane_xor(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = lane_xor_i<B>((int)(b & 0xffffffffll));
    const int hi = lane_xor_i<B>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ float lane_xor(float v, int m) { return __shfl_xor(v, m, 64); }
__device__ __forceinline__ double lane_xor(double v, int m) { return __shfl_xor(v, m, 64); }

// One pair (x: bit clear, y: bit set) through a gate form.
template <typename T, int FORM>
__device__ __forceinline__ void pair_form(cplx<T> &x, cplx<T> &y, const Mat2<T> &u) {
    cplx<T> a = x, b = y;
    if constexpr (FORM == F_GEN) {
        x = cmad(u.m[1], b, cmul(u.m[0], a));
        y = cmad(u.m[3], b, cmul(u.m[2], a));
    } else if constexpr (FORM == F_H) {
        x.re = a.re + b.re; x.im = a.im + b.im;
        y.re = a.re - b.re; y.im = a.im - b.im;
    } else if constexpr (FORM == F_SY) {
        x.re = a.re - b.re; x.im = a.im - b.im;
        y.re = a.re + b.re; y.im = a.im + b.im;
    } else if constexpr (FORM == F_SYDG) {
        x.re = a.re + b.re; x.im = a.im + b.im;
        y.re = b.re - a.re; y.im = b.im - a.im;
    } else if constexpr (FORM == F_SX) {       // x - i y, -i x + y
        x.re = a.re + b.im; x.im = a.im - b.re;
        y.re = b.re + a.im; y.im = b.im - a.re;
    } else if constexpr (FORM == F_SXDG) {     // x + i y, i x + y
        x.re = a.re - b.im; x.im = a.im + b.re;
        y.re = b.re - a.im; y.im = b.im + a.re;
    } else if constexpr (FORM == F_RX) {       // c x - i s y, -i s x + c y
        const T c = u.m[0].re, sn = -u.m[1].im;
        x.re = fma(c, a.re, sn * b.im); x.im = fma(c, a.im, -sn * b.re);
        y.re = fma(c, b.re, sn * a.im); y.im = fma(c, b.im, -sn * a.re);
    } else if constexpr (FORM == F_RY) {       // c x - s y, s x + c y
        const T c = u.m[0].re, sn = u.m[2].re;
        x.re = fma(c, a.re, -sn * b.re); x.im = fma(c, a.im, -sn * b.im);
        y.re = fma(c, b.re, sn * a.re); y.im = fma(c, b.im, sn * a.im);
    } else if constexpr (FORM == F_REAL) {
        x.re = fma(u.m[0].re, a.re, u.m[1].re * b.re); x.im = fma(u.m[0].re, a.im, u.m[1].re * b.im);
        y.re = fma(u.m[2].re, a.re, u.m[3].re * b.re); y.im = fma(u.m[2].re, a.im, u.m[3].re * b.im);
    } else {                                   // F_PHASE
        y = cmul(u.m[3], b);
    }
}

template <typename T, int NR, int S, int FORM>
__device__ __forceinline__ void reg_gate_f(cplx<T> (&a)[NR], const Mat2<T> &u) {
#pragma unroll
    for (int r = 0; r < NR; r++) {
        if (r & (1 << S)) continue;
        pair_form<T, FORM>(a[r], a[r | (1 << S)], u);
    }
}

template <typename T, int NR, int S>
__device__ __forceinline__ void reg_gate_s(cplx<T> (&a)[NR], const Mat2<T> &u, int form) {
    switch (form) {
    case F_H: reg_gate_f<T, NR, S, F_H>(a, u); break;
    case F_SX: reg_gate_f<T, NR, S, F_SX>(a, u); break;
    case F_SY: reg_gate_f<T, NR, S, F_SY>(a, u); break;
    case F_SXDG: reg_gate_f<T, NR, S, F_SXDG>(a, u); break;
    case F_SYDG: reg_gate_f<T, NR, S, F_SYDG>(a, u); break;
    case F_PHASE: reg_gate_f<T, NR, S, F_PHASE>(a, u); break;
    case F_RX: reg_gate_f<T, NR, S, F_RX>(a, u); break;
    case F_RY: reg_gate_f<T, NR, S, F_RY>(a, u); break;
    case F_REAL: reg_gate_f<T, NR, S, F_REAL>(a, u); break;
    default: reg_gate_f<T, NR, S, F_GEN>(a, u); break;
    }
}

template <typename T, int NR>
__device__ __forceinline__ void reg_gate_dispatch(cplx<T> (&a)[NR], const Mat2<T> &u, int s, int form = F_GEN) {
    switch (s) {
    case 0: reg_gate_s<T, NR, 0>(a, u, form); break;
    case 1: if constexpr (NR > 2) reg_gate_s<T, NR, 1>(a, u, form); break;
    case 2: if constexpr (NR > 4) reg_gate_s<T, NR, 2>(a, u, form); break;
    case 3: if constexpr (NR > 8) reg_gate_s<T, NR, 3>(a, u, form); break;
    case 4: if constexpr (NR > 16) reg_gate_s<T, NR, 4>(a, u, form); break;
    case 5: if constexpr (NR > 32) reg_gate_s<T, NR, 5>(a, u, form); break;
    default: break;
    }
}

// Gate on lane bit B: each lane forms its new value from its own amplitude
// (self) and its partner's (p); hi = the lane's bit B.
template <typename T, int NR, int B, int FORM>
__device__ __forceinline__ void lane_gate_f(cplx<T> (&a)[NR], const Mat2<T> &u, int lane) {
    const bool hi = (lane >> B) & 1;
    if constexpr (FORM == F_PHASE) {
        cplx<T> f;
        f.re = hi ? u.m[3].re : (T)1;
        f.im = hi ? u.m[3].im : (T)0;
#pragma unroll
        for (int r = 0; r < NR; r++) a[r] = cmul(f, a[r]);
        return;
    }
    cplx<T> cs, cp;
    T sg = (T)1, rc = (T)0, rs = (T)0;
    if constexpr (FORM == F_GEN) {
        cs = hi ? u.m[3] : u.m[0];
        cp = hi ? u.m[2] : u.m[1];
    } else if constexpr (FORM == F_RX) {
        rc = u.m[0].re;
        rs = -u.m[1].im;            // self c - i s p (both halves)
    } else if constexpr (FORM == F_RY) {
        rc = u.m[0].re;
        rs = hi ? u.m[2].re : -u.m[2].re;   // lo: c self - s p, hi: c self + s p
    } else if constexpr (FORM == F_REAL) {
        rc = hi ? u.m[3].re : u.m[0].re;
        rs = hi ? u.m[2].re : u.m[1].re;    // cs self + cp p
    } else if constexpr (FORM == F_H) {
        sg = hi ? (T)-1 : (T)1;     // lo: self + p, hi: p - self
    } else if constexpr (FORM == F_SY) {
        sg = hi ? (T)1 : (T)-1;     // lo: self - p, hi: self + p
    } else if constexpr (FORM == F_SYDG) {
        sg = hi ? (T)-1 : (T)1;     // lo: self + p, hi: self - p
    }
#pragma unroll
    for (int r = 0; r < NR; r++) {
        cplx<T> p;
        p.re = lane_xor<B>(a[r].re);
        p.im = lane_xor<B>(a[r].im);
        cplx<T> s = a[r], o;
        if constexpr (FORM == F_GEN) {
            o = cmad(cp, p, cmul(cs, s));
        } else if constexpr (FORM == F_H) {
            o.re = fma(sg, s.re, p.re); o.im = fma(sg, s.im, p.im);
        } else if constexpr (FORM == F_SY || FORM == F_SYDG) {
            o.re = fma(sg, p.re, s.re); o.im = fma(sg, p.im, s.im);
        } else if constexpr (FORM == F_SX) {    // self - i p (both halves)
            o.re = s.re + p.im; o.im = s.im - p.re;
        } else if constexpr (FORM == F_SXDG) {  // self + i p
            o.re = s.re - p.im; o.im = s.im + p.re;
        } else if constexpr (FORM == F_RX) {
            o.re = fma(rc, s.re, rs * p.im); o.im = fma(rc, s.im, -rs * p.re);
        } else {                                 // F_RY, F_REAL
            o.re = fma(rc, s.re, rs * p.re); o.im = fma(rc, s.im, rs * p.im);
        }
        a[r] = o;
    }
}

template <typename T, int NR, int B>
__device__ __forceinline__ void lane_gate_b(cplx<T> (&a)[NR], const Mat2<T> &u, int lane, int form) {
    switch (form) {
    case F_H: lane_gate_f<T, NR, B, F_H>(a, u, lane); break;
    case F_SX: lane_gate_f<T, NR, B, F_SX>(a, u, lane); break;
    case F_SY: lane_gate_f<T, NR, B, F_SY>(a, u, lane); break;
    case F_SXDG: lane_gate_f<T, NR, B, F_SXDG>(a, u, lane); break;
    case F_SYDG: lane_gate_f<T, NR, B, F_SYDG>(a, u, lane); break;
    case F_PHASE: lane_gate_f<T, NR, B, F_PHASE>(a, u, lane); break;
    case F_RX: lane_gate_f<T, NR, B, F_RX>(a, u, lane); break;
    case F_RY: lane_gate_f<T, NR, B, F_RY>(a, u, lane); break;
    case F_REAL: lane_gate_f<T, NR, B, F_REAL>(a, u, lane); break;
    default: lane_gate_f<T, NR, B, F_GEN>(a, u, lane); break;
    }
}

template <typename T, int NR>
__device__ __forceinline__ void lane_gate_dispatch(cplx<T> (&a)[NR], const Mat2<T> &u, int b, int lane,
                                                   int form = F_GEN) {
    switch (b) {
    case 0: lane_gate_b<T, NR, 0>(a, u, lane, form); break;
    case 1: lane_gate_b<T, NR, 1>(a, u, lane, form); break;
    case 2: lane_gate_b<T, NR, 2>(a, u, lane, form); break;
    case 3: lane_gate_b<T, NR, 3>(a, u, lane, form); break;
    case 4: lane_gate_b<T, NR, 4>(a, u, lane, form); break;
    default: lane_gate_b<T, NR, 5>(a, u, lane, form); break;
    }
}

// A wave-uniform pointer held in scalar registers, so that a wave-wide
// access ptr[lane] uses the scalar-base + 32-bit lane-offset address form
// (one address register per lane for all rows of a tile).
template <typename P>
__device__ __forceinline__ P *uniform_ptr(P *p) {
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (P *)(((uint64_t)hi << 32) | lo);
}

// Offset of register r in a register tile: sum of 2^rq[i] over the set
// bits i of r (r is a compile-time constant after unrolling).
template <int VB>
__device__ __forceinline__ uint64_t reg_offset(const uint64_t (&bq)[VB], int r) {
    uint64_t o = 0;
#pragma unroll
    for (int i = 0; i < VB; i++)
        if ((r >> i) & 1) o |= bq[i];
    return o;
}

template <typename T>
__device__ __forceinline__ Mat2<T> load_mat(const double *u) {
    Mat2<T> m;
#pragma unroll
    for (int i = 0; i < 4; i++) { m.m[i].re = (T)u[2 * i]; m.m[i].im = (T)u[2 * i + 1]; }
    return m;
}


}  // namespace svi
