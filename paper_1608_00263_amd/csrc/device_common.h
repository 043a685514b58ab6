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

__device__ __forceinline__ float lane_xor(float v, int m) { return __shfl_xor(v, m, 64); }
__device__ __forceinline__ double lane_xor(double v, int m) { return __shfl_xor(v, m, 64); }

template <typename T, int NR, int S>
__device__ __forceinline__ void reg_gate(cplx<T> (&a)[NR], const Mat2<T> &u) {
#pragma unroll
    for (int r = 0; r < NR; r++) {
        if (r & (1 << S)) continue;
        const int r1 = r | (1 << S);
        cplx<T> x = a[r], y = a[r1];
        a[r] = cmad(u.m[1], y, cmul(u.m[0], x));
        a[r1] = cmad(u.m[3], y, cmul(u.m[2], x));
    }
}

template <typename T, int NR>
__device__ __forceinline__ void reg_gate_dispatch(cplx<T> (&a)[NR], const Mat2<T> &u, int s) {
    switch (s) {
    case 0: reg_gate<T, NR, 0>(a, u); break;
    case 1: if constexpr (NR > 2) reg_gate<T, NR, 1>(a, u); break;
    case 2: if constexpr (NR > 4) reg_gate<T, NR, 2>(a, u); break;
    case 3: if constexpr (NR > 8) reg_gate<T, NR, 3>(a, u); break;
    case 4: if constexpr (NR > 16) reg_gate<T, NR, 4>(a, u); break;
    case 5: if constexpr (NR > 32) reg_gate<T, NR, 5>(a, u); break;
    default: break;
    }
}

template <typename T, int NR, int B>
__device__ __forceinline__ void lane_gate(cplx<T> (&a)[NR], const Mat2<T> &u, int lane) {
    const bool hi = (lane >> B) & 1;
    cplx<T> cs = hi ? u.m[3] : u.m[0];
    cplx<T> cp = hi ? u.m[2] : u.m[1];
#pragma unroll
    for (int r = 0; r < NR; r++) {
        cplx<T> p;
        p.re = lane_xor(a[r].re, 1 << B);
        p.im = lane_xor(a[r].im, 1 << B);
        a[r] = cmad(cp, p, cmul(cs, a[r]));
    }
}

template <typename T, int NR>
__device__ __forceinline__ void lane_gate_dispatch(cplx<T> (&a)[NR], const Mat2<T> &u, int b, int lane) {
    switch (b) {
    case 0: lane_gate<T, NR, 0>(a, u, lane); break;
    case 1: lane_gate<T, NR, 1>(a, u, lane); break;
    case 2: lane_gate<T, NR, 2>(a, u, lane); break;
    case 3: lane_gate<T, NR, 3>(a, u, lane); break;
    case 4: lane_gate<T, NR, 4>(a, u, lane); break;
    default: lane_gate<T, NR, 5>(a, u, lane); break;
    }
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
