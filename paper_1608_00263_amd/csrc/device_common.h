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

// x <- u x in place, with the same roundings as cmul.  In FP32 the two
// products go to temporaries and the two multiply-adds write back into the
// registers of x: the accumulating multiply-add the compiler picks otherwise
// writes its result over the addend (a temporary), which moves every output
// one register along and ends a multiply op over a tile in a run of copies.
template <typename T>
__device__ __forceinline__ void cmul_ip(cplx<T> &x, const cplx<T> u) {
    if constexpr (sizeof(T) == 4) {
        const float t = u.im * x.im;
        const float v = u.im * x.re;
        asm("v_fma_f32 %0, %1, %0, -%2" : "+v"(x.re) : "v"(u.re), "v"(t));
        asm("v_fma_f32 %0, %1, %0, %2" : "+v"(x.im) : "v"(u.re), "v"(v));
    } else {
        x = cmul(u, x);
    }
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
// lanes).  Bits 0, 1 and 3 take one DPP lane move within rows of 16 (quad
// permutations, rotation of the row by 8), bit 2 two (half-row mirror, then
// quad reverse), bit 4 a ds_swizzle in xor mode (and mask 0x1f, xor mask
// 16), bit 5 a ds_bpermute.  FOLD writes the last move of bits 0..3 as an
// update with bound_ctrl and a zero old value: every source lane is inside
// the row and active, so it equals a plain move, and in that form the
// compiler merges it into a following add, subtract or multiply (one
// instruction); before other consumers (fused multiply-adds) it would only
// hold a register, so they take the plain move.
template <int CTRL, bool FOLD>
__device__ __forceinline__ int dpp_move(int x) {
    if constexpr (FOLD) return __builtin_amdgcn_update_dpp(0, x, CTRL, 0xF, 0xF, true);
    else return __builtin_amdgcn_mov_dpp(x, CTRL, 0xF, 0xF, false);
}
template <int B, bool FOLD = false>
__device__ __forceinline__ int lane_xor_i(int v) {
    if constexpr (B == 0) return dpp_move<0xB1, FOLD>(v);   // quad_perm 1,0,3,2
    if constexpr (B == 1) return dpp_move<0x4E, FOLD>(v);   // quad_perm 2,3,0,1
    if constexpr (B == 2) {   // i ^ 7 (half-row mirror), then i ^ 3 (quad reverse): i ^ 4
        int m = __builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, false);
        return dpp_move<0x1B, FOLD>(m);
    }
    if constexpr (B == 3) return dpp_move<0x128, FOLD>(v);   // row_ror 8: i ^ 8
    if constexpr (B == 4) return __builtin_amdgcn_ds_swizzle(v, 0x401F);   // lane ^ 16
    if constexpr (B == 5) return __shfl_xor(v, 32, 64);
    return v;
}

template <int B, bool FOLD = false>
__device__ __forceinline__ float lane_xor(float v) {
    return __int_as_float(lane_xor_i<B, FOLD>(__float_as_int(v)));
}
template <int B, bool FOLD = false>
__device__ __forceinline__ double lane_xor(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = lane_xor_i<B, FOLD>((int)(b & 0xffffffffll));
    const int hi = lane_xor_i<B, FOLD>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ float lane_xor(float v, int m) { return __shfl_xor(v, m, 64); }
__device__ __forceinline__ double lane_xor(double v, int m) { return __shfl_xor(v, m, 64); }

// In-place butterfly of two reals: u' = u + s v, v' = t v + w u' with the
// constants chosen per form.  Written so that each input dies where its
// output is formed (u' from u, then v' from v and u'), the two outputs take
// the registers of the two inputs: the straightforward form (both outputs
// from both inputs) needs a copy per pair at the end of the op, about a third
// of the add-only gate's instructions (measured).  v' = 2v +- u' is exact up
// to one more rounding of u'.
template <typename T>
__device__ __forceinline__ void bfly_add(T &u, T &v) {   // u + v, v - u
    u = u + v;
    v = fma((T)2, v, -u);
}
template <typename T>
__device__ __forceinline__ void bfly_sub(T &u, T &v) {   // u - v, v + u
    u = u - v;
    v = fma((T)2, v, u);
}
template <typename T>
__device__ __forceinline__ void bfly_h(T &u, T &v) {     // u + v, u - v
    u = u + v;
    v = fma((T)-2, v, u);
}

// One pair (x: bit clear, y: bit set) through a gate form.
template <typename T, int FORM>
__device__ __forceinline__ void pair_form(cplx<T> &x, cplx<T> &y, const Mat2<T> &u) {
    if constexpr (FORM == F_H) {               // x + y, x - y
        bfly_h(x.re, y.re);
        bfly_h(x.im, y.im);
        return;
    } else if constexpr (FORM == F_SY) {       // x - y, x + y
        bfly_sub(x.re, y.re);
        bfly_sub(x.im, y.im);
        return;
    } else if constexpr (FORM == F_SYDG) {     // x + y, y - x
        bfly_add(x.re, y.re);
        bfly_add(x.im, y.im);
        return;
    } else if constexpr (FORM == F_SX) {       // x - i y, -i x + y
        bfly_add(x.re, y.im);                  // x.re + y.im, y.im - x.re
        bfly_sub(x.im, y.re);                  // x.im - y.re, y.re + x.im
        return;
    } else if constexpr (FORM == F_SXDG) {     // x + i y, i x + y
        bfly_sub(x.re, y.im);                  // x.re - y.im, y.im + x.re
        bfly_add(x.im, y.re);                  // x.im + y.re, y.re - x.im
        return;
    }
    cplx<T> a = x, b = y;
    if constexpr (FORM == F_GEN) {
        x = cmad(u.m[1], b, cmul(u.m[0], a));
        y = cmad(u.m[3], b, cmul(u.m[2], a));
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
    } else if constexpr (FORM == F_TRX) {      // x - i t y, -i t x + y
        const T t = -u.m[1].im;
        x.re = fma(t, b.im, a.re); x.im = fma(-t, b.re, a.im);
        y.re = fma(t, a.im, b.re); y.im = fma(-t, a.re, b.im);
    } else if constexpr (FORM == F_TRY) {      // x - t y, t x + y
        const T t = u.m[2].re;
        x.re = fma(-t, b.re, a.re); x.im = fma(-t, b.im, a.im);
        y.re = fma(t, a.re, b.re); y.im = fma(t, a.im, b.im);
    } else {                                   // F_PHASE
        cmul_ip(y, u.m[3]);
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
    case F_TRX: reg_gate_f<T, NR, S, F_TRX>(a, u); break;
    case F_TRY: reg_gate_f<T, NR, S, F_TRY>(a, u); break;
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

// Lane bits 4 and 5 through the gfx950 half-swaps of two registers x, y:
// permlane32_swap exchanges the upper 32 lanes of x with the lower 32 of y,
// permlane16_swap the odd 16-lane rows of x with the even rows of y.  After
// the swap every lane holds one partner pair (bit B clear in x, set in y):
// lanes with bit B clear hold the pair of the first register, the others
// that of the second.  The same swap restores the layout.
template <int B>
__device__ __forceinline__ void half_swap_i(int &x, int &y) {
    static_assert(B == 4 || B == 5, "half swaps exist for lane bits 4 and 5");
    if constexpr (B == 5) {
        const auto r = __builtin_amdgcn_permlane32_swap(x, y, false, false);
        x = (int)r[0];
        y = (int)r[1];
    } else {
        const auto r = __builtin_amdgcn_permlane16_swap(x, y, false, false);
        x = (int)r[0];
        y = (int)r[1];
    }
}
template <int B>
__device__ __forceinline__ void half_swap(float &x, float &y) {
    int xi = __float_as_int(x), yi = __float_as_int(y);
    half_swap_i<B>(xi, yi);
    x = __int_as_float(xi);
    y = __int_as_float(yi);
}
template <int B>
__device__ __forceinline__ void half_swap(double &x, double &y) {
    const long long xb = __double_as_longlong(x), yb = __double_as_longlong(y);
    int xl = (int)(xb & 0xffffffffll), xh = (int)(xb >> 32);
    int yl = (int)(yb & 0xffffffffll), yh = (int)(yb >> 32);
    half_swap_i<B>(xl, yl);
    half_swap_i<B>(xh, yh);
    x = __longlong_as_double(((long long)xh << 32) | (unsigned int)xl);
    y = __longlong_as_double(((long long)yh << 32) | (unsigned int)yl);
}

// Gate on lane bit B: each lane forms its new value from its own amplitude
// (self) and its partner's (p); hi = the lane's bit B.  Bits 4 and 5 swap
// register halves instead so that each lane applies the gate to a whole
// pair (no lane-dependent coefficients).
// FOLDOK: the cross-lane moves may be merged into their consumers (see
// lane_xor_i); kernels that keep two tiles in registers pass false, since the
// merged in-place update needs one more register per amplitude in flight.
template <typename T, int NR, int B, int FORM, bool FOLDOK = true>
__device__ __forceinline__ void lane_gate_f(cplx<T> (&a)[NR], const Mat2<T> &u, int lane) {
    if constexpr (B >= 4 && FORM != F_PHASE && NR >= 2) {
#pragma unroll
        for (int r = 0; r < NR; r += 2) {
            cplx<T> x = a[r], y = a[r + 1];
            half_swap<B>(x.re, y.re);
            half_swap<B>(x.im, y.im);
            pair_form<T, FORM>(x, y, u);
            half_swap<B>(x.re, y.re);
            half_swap<B>(x.im, y.im);
            a[r] = x;
            a[r + 1] = y;
        }
        return;
    }
    const bool hi = (lane >> B) & 1;
    if constexpr (FORM == F_PHASE) {
        cplx<T> f;
        f.re = hi ? u.m[3].re : (T)1;
        f.im = hi ? u.m[3].im : (T)0;
#pragma unroll
        for (int r = 0; r < NR; r++) cmul_ip(a[r], f);
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
    } else if constexpr (FORM == F_TRX) {
        rs = -u.m[1].im;            // self - i t p (both halves)
    } else if constexpr (FORM == F_TRY) {
        rs = hi ? u.m[2].re : -u.m[2].re;   // lo: self - t p, hi: self + t p
    } else if constexpr (FORM == F_H) {
        sg = hi ? (T)-1 : (T)1;     // lo: self + p, hi: p - self
    } else if constexpr (FORM == F_SY) {
        sg = hi ? (T)1 : (T)-1;     // lo: self - p, hi: self + p
    } else if constexpr (FORM == F_SYDG) {
        sg = hi ? (T)-1 : (T)1;     // lo: self + p, hi: self - p
    }
    // forms whose partner terms feed an add, subtract or multiply
    constexpr bool FOLD =
        FOLDOK && (FORM == F_SX || FORM == F_SXDG || FORM == F_RX || FORM == F_RY || FORM == F_REAL);
#pragma unroll
    for (int r = 0; r < NR; r++) {
        cplx<T> p;
        p.re = lane_xor<B, FOLD>(a[r].re);
        p.im = lane_xor<B, FOLD>(a[r].im);
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
        } else if constexpr (FORM == F_TRX) {
            o.re = fma(rs, p.im, s.re); o.im = fma(-rs, p.re, s.im);
        } else if constexpr (FORM == F_TRY) {
            o.re = fma(rs, p.re, s.re); o.im = fma(rs, p.im, s.im);
        } else {                                 // F_RY, F_REAL
            o.re = fma(rc, s.re, rs * p.re); o.im = fma(rc, s.im, rs * p.im);
        }
        a[r] = o;
    }
}

template <typename T, int NR, int B, bool FOLDOK = true>
__device__ __forceinline__ void lane_gate_b(cplx<T> (&a)[NR], const Mat2<T> &u, int lane, int form) {
    switch (form) {
    case F_H: lane_gate_f<T, NR, B, F_H, FOLDOK>(a, u, lane); break;
    case F_SX: lane_gate_f<T, NR, B, F_SX, FOLDOK>(a, u, lane); break;
    case F_SY: lane_gate_f<T, NR, B, F_SY, FOLDOK>(a, u, lane); break;
    case F_SXDG: lane_gate_f<T, NR, B, F_SXDG, FOLDOK>(a, u, lane); break;
    case F_SYDG: lane_gate_f<T, NR, B, F_SYDG, FOLDOK>(a, u, lane); break;
    case F_PHASE: lane_gate_f<T, NR, B, F_PHASE, FOLDOK>(a, u, lane); break;
    case F_RX: lane_gate_f<T, NR, B, F_RX, FOLDOK>(a, u, lane); break;
    case F_RY: lane_gate_f<T, NR, B, F_RY, FOLDOK>(a, u, lane); break;
    case F_REAL: lane_gate_f<T, NR, B, F_REAL, FOLDOK>(a, u, lane); break;
    case F_TRX: lane_gate_f<T, NR, B, F_TRX, FOLDOK>(a, u, lane); break;
    case F_TRY: lane_gate_f<T, NR, B, F_TRY, FOLDOK>(a, u, lane); break;
    default: lane_gate_f<T, NR, B, F_GEN, FOLDOK>(a, u, lane); break;
    }
}

template <typename T, int NR, bool FOLDOK = true>
__device__ __forceinline__ void lane_gate_dispatch(cplx<T> (&a)[NR], const Mat2<T> &u, int b, int lane,
                                                   int form = F_GEN) {
    switch (b) {
    case 0: lane_gate_b<T, NR, 0, FOLDOK>(a, u, lane, form); break;
    case 1: lane_gate_b<T, NR, 1, FOLDOK>(a, u, lane, form); break;
    case 2: lane_gate_b<T, NR, 2, FOLDOK>(a, u, lane, form); break;
    case 3: lane_gate_b<T, NR, 3, FOLDOK>(a, u, lane, form); break;
    case 4: lane_gate_b<T, NR, 4, FOLDOK>(a, u, lane, form); break;
    default: lane_gate_b<T, NR, 5, FOLDOK>(a, u, lane, form); break;
    }
}

// Pointer into device (global) memory, address space 1: accesses through it
// are global loads and stores rather than flat ones (no LDS-counter waits,
// scalar base + 32-bit vector offset addressing).
template <typename P> using gptr = __attribute__((address_space(1))) P *;

// Pointer into device memory that no kernel writes while it runs (address
// space 4): wave-uniform reads through it are scalar loads, also after the
// kernel has stored to other buffers.
template <typename P> using cptr = const __attribute__((address_space(4))) P *;

// A wave-uniform pointer held in scalar registers, so that a wave-wide
// access ptr[lane] uses the scalar-base + 32-bit lane-offset address form
// (one address register per lane for all rows of a tile).  p must point to
// device memory.
template <typename P>
__device__ __forceinline__ gptr<P> uniform_ptr(P *p) {
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (gptr<P>)(((uint64_t)hi << 32) | lo);
}
// Tile loads and stores are non-temporal: a sweep reads and writes every
// amplitude once, so keeping the lines in the caches only evicts others
// (measured on a one-gate sweep over 8 GiB: 5.50 -> 6.09 TB/s).
template <typename T>
__device__ __forceinline__ cplx<T> gload(gptr<cplx<T>> p) {
    cplx<T> v;
    v.re = __builtin_nontemporal_load(&p->re);
    v.im = __builtin_nontemporal_load(&p->im);
    return v;
}
template <typename T>
__device__ __forceinline__ void gstore(gptr<cplx<T>> p, cplx<T> v) {
    __builtin_nontemporal_store(v.re, &p->re);
    __builtin_nontemporal_store(v.im, &p->im);
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

template <typename T, typename PD>
__device__ __forceinline__ Mat2<T> load_mat(PD u) {
    Mat2<T> m;
#pragma unroll
    for (int i = 0; i < 4; i++) { m.m[i].re = (T)u[2 * i]; m.m[i].im = (T)u[2 * i + 1]; }
    return m;
}


// One register-tile op: kind, argument, term count, form and its 2x2 matrix.
template <typename T, int NR>
__device__ __forceinline__ void regtile_op(cplx<T> (&a)[NR], int kind, int arg, int nt, int form, const Mat2<T> &u,
                                           const cptr<DiagTerm> terms, uint64_t base, int lane) {
    if (kind == RT_REG) {
        reg_gate_dispatch<T, NR>(a, u, arg, form);
    } else if (kind == RT_LANE) {
        lane_gate_dispatch<T, NR>(a, u, arg, lane, form);
    } else if (kind == RT_SIGNS) {
        uint64_t par = 0;
        for (int t = arg; t < arg + nt; t++) {
            const uint64_t out = terms[t].outside;
            if ((base & out) != out) continue;
            const uint32_t lm = terms[t].lanemask;
            const uint64_t rs = terms[t].regset;
            par ^= ((uint32_t)lane & lm) == lm ? rs : 0ull;
        }
#pragma unroll
        for (int r = 0; r < NR; r++) {
            if ((par >> r) & 1) { a[r].re = -a[r].re; a[r].im = -a[r].im; }
        }
    } else if (kind == RT_PHASE) {
        // a group of phase terms sharing one register set: the product
        // of the phases whose lane and outside bits match, per lane,
        // then one multiplication of the group's registers
        const uint64_t rs = terms[arg].regset;
        cplx<T> f;
        f.re = (T)1;
        f.im = (T)0;
        bool any = false;
        for (int t = arg; t < arg + nt; t++) {
            const uint64_t out = terms[t].outside;
            if ((base & out) != out) continue;
            any = true;
            const uint32_t lm = terms[t].lanemask;
            cplx<T> v;
            v.re = (T)terms[t].val[0];
            v.im = (T)terms[t].val[1];
            const cplx<T> fv = cmul(v, f);
            if (((uint32_t)lane & lm) == lm) f = fv;
        }
        if (any) {
#pragma unroll
            for (int r = 0; r < NR; r++)
                if ((rs >> r) & 1) cmul_ip(a[r], f);
        }
    }
}

// One register tile of a sweep: tile index `tile` of the program at prog,
// processed by the calling wavefront (lane = its lane id).  ck, when not
// null, receives a second copy of the stored tile (a checkpoint of the
// state after the sweep, written from the registers).
template <typename T, int VB>
__device__ __forceinline__ void regtile_apply(cplx<T> *__restrict__ psi, const uint8_t *__restrict__ prog,
                                              uint64_t tile, int lane, cplx<T> *__restrict__ ck = nullptr) {
    constexpr int NR = 1 << VB;
    const cptr<RTHeader> h = (cptr<RTHeader>)prog;
    uint64_t bq[VB];
#pragma unroll
    for (int i = 0; i < VB; i++) bq[i] = 1ull << h->rq[i];
    // tile base: the tile index with zeros inserted at the tile's qubits
    // above 3 (lane qubits and register qubits), in ascending order
    uint64_t base = tile << 4;
#pragma unroll
    for (int i = 0; i < VB + 2; i++) base = insert_zero(base, h->tq[i]);
    // lane bits 0..3 are qubits 0..3; lane bits 4 and 5 are qubits lq[0],
    // lq[1].  With lq = (4, 5) a row is 64 contiguous amplitudes: uniform row
    // pointer (scalar registers) + lane index, one address register per lane.
    const int l4 = h->lq[0], l5 = h->lq[1];
    const bool rows = (l4 == 4) & (l5 == 5);
    const uint64_t loff = (uint64_t)(lane & 15) | ((uint64_t)((lane >> 4) & 1) << l4) |
                          ((uint64_t)((lane >> 5) & 1) << l5);

    cplx<T> a[NR];
    const int gen_n = h->gen_n;
    // the Clifford forms leave a power of sqrt2 (2^sexp exactly, then
    // 1/sqrt2) and the tangent-form rotations their cosines: one factor,
    // applied to the generated value when the sweep generates its input
    // (the ops are linear), else once after the ops
    double scale = ldexp(1.0, h->sexp);
    if (h->shalf) scale *= 0.70710678118654752440;
    scale *= h->fscale;
    if (gen_n > 0) {
        // the Hadamard layer on |0..0>: every amplitude is 2^{-n/2}
        double vd = ldexp(1.0, -(gen_n / 2));
        if (gen_n & 1) vd *= 0.70710678118654752440;
        vd *= scale;
        scale = 1.0;
        if (h->gph_off > 0) {
            // diagonals folded in: amplitude = v c prod over the set bits of
            // its index of the ratio of that qubit (outside qubits from the
            // tile base, lane bits per lane, register slots by doubling)
            const cptr<RTGenPhases> gp = (cptr<RTGenPhases>)(prog + h->gph_off);
            const cptr<RTGenOut> go = (cptr<RTGenOut>)(prog + h->gph_off + sizeof(RTGenPhases));
            double cr = vd * gp->c[0], ci = vd * gp->c[1];
            const int nout = h->gph_nout;
            for (int k = 0; k < nout; k++) {
                if ((base & go[k].mask) == 0) continue;
                const double xr = go[k].r[0], xi = go[k].r[1];
                const double t = cr * xr - ci * xi;
                ci = cr * xi + ci * xr;
                cr = t;
            }
#pragma unroll
            for (int b = 0; b < 6; b++) {
                const bool on = (lane >> b) & 1;
                const double xr = on ? gp->lane[b][0] : 1.0, xi = on ? gp->lane[b][1] : 0.0;
                const double t = cr * xr - ci * xi;
                ci = cr * xi + ci * xr;
                cr = t;
            }
            a[0].re = (T)cr;
            a[0].im = (T)ci;
#pragma unroll
            for (int sb = 0; sb < VB; sb++) {
                cplx<T> f;
                f.re = (T)gp->reg[sb][0];
                f.im = (T)gp->reg[sb][1];
#pragma unroll
                for (int r = 1 << sb; r < (2 << sb); r++) a[r] = cmul(a[r - (1 << sb)], f);
            }
        } else {
            const T v = (T)vd;
#pragma unroll
            for (int r = 0; r < NR; r++) { a[r].re = v; a[r].im = (T)0; }
        }
    } else if (rows) {
#pragma unroll
        for (int r = 0; r < NR; r++) a[r] = gload<T>(uniform_ptr(psi + (base + reg_offset<VB>(bq, r))) + lane);
    } else {
#pragma unroll
        for (int r = 0; r < NR; r++) a[r] = gload<T>(uniform_ptr(psi + (base + reg_offset<VB>(bq, r))) + loff);
    }

    const cptr<DiagTerm> terms = (cptr<DiagTerm>)(prog + h->term_off);
    const int nops = h->nops;
    if constexpr (sizeof(T) == 4) {
        // complex64: the 64-byte FP32 op records, the next one fetched while
        // the current one runs (its scalar loads do not stall the wave)
        const cptr<RTOpF> fops = (cptr<RTOpF>)(prog + h->fop_off);
        int kind = 0, arg = 0, nt = 0, form = 0;
        float uf[8];
        if (nops > 0) {
            kind = fops[0].kind; arg = fops[0].a; nt = fops[0].nterms; form = fops[0].form;
#pragma unroll
            for (int k = 0; k < 8; k++) uf[k] = fops[0].u[k];
        }
        for (int o = 0; o < nops; o++) {
            const int on = o + 1 < nops ? o + 1 : o;
            const int kind_n = fops[on].kind, arg_n = fops[on].a, nt_n = fops[on].nterms, form_n = fops[on].form;
            float un[8];
#pragma unroll
            for (int k = 0; k < 8; k++) un[k] = fops[on].u[k];
            Mat2<T> u;
#pragma unroll
            for (int k = 0; k < 4; k++) { u.m[k].re = uf[2 * k]; u.m[k].im = uf[2 * k + 1]; }
            regtile_op<T, NR>(a, kind, arg, nt, form, u, terms, base, lane);
            kind = kind_n; arg = arg_n; nt = nt_n; form = form_n;
#pragma unroll
            for (int k = 0; k < 8; k++) uf[k] = un[k];
        }
    } else {
        const cptr<RTOp> ops = (cptr<RTOp>)(prog + h->op_off);
        for (int o = 0; o < nops; o++)
            regtile_op<T, NR>(a, ops[o].kind, ops[o].a, ops[o].nterms, ops[o].form, load_mat<T>(ops[o].u), terms, base,
                              lane);
    }
    if (scale != 1.0) {
        const T f = (T)scale;
#pragma unroll
        for (int r = 0; r < NR; r++) {
            a[r].re *= f;
            a[r].im *= f;
        }
    }
    if (rows) {
#pragma unroll
        for (int r = 0; r < NR; r++) gstore<T>(uniform_ptr(psi + (base + reg_offset<VB>(bq, r))) + lane, a[r]);
    } else {
#pragma unroll
        for (int r = 0; r < NR; r++) gstore<T>(uniform_ptr(psi + (base + reg_offset<VB>(bq, r))) + loff, a[r]);
    }
    if (ck) {
#pragma unroll
        for (int r = 0; r < NR; r++) gstore<T>(uniform_ptr(ck + (base + reg_offset<VB>(bq, r))) + loff, a[r]);
    }
}


}  // namespace svi
