// Device helpers shared by the reduction kernels and the ensemble kernel:
// probabilities in FP64 and fixed-order wavefront / workgroup sums.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace svi {

constexpr int RB = 256;   // threads per workgroup

template <typename T> struct cpx { T re, im; };

// p = re*re + im*im with both products and the sum rounded separately: the
// expression is compiled with contraction off (the rounded-operation
// intrinsics of this toolchain are plain operators, which the default
// contraction of device code would fuse into fma(re, re, im*im)); for
// complex64 input both products are exact in FP64.
__device__ __forceinline__ double prob_of(cpx<float> a) {
#pragma clang fp contract(off)
    const double r = (double)a.re, i = (double)a.im;
    return r * r + i * i;
}
__device__ __forceinline__ double prob_of(cpx<double> a) {
#pragma clang fp contract(off)
    return a.re * a.re + a.im * a.im;
}
__device__ __forceinline__ double prob_of(double p) { return p; }

template <typename V>
__device__ __forceinline__ V wave_sum(V v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// Workgroup sum of NV values per thread into red[0..NV) (fixed order).
template <typename V, int NV>
__device__ __forceinline__ void block_sum(V (&v)[NV], V *red /* LDS, 4*NV */) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < NV; i++) v[i] = wave_sum(v[i]);
    if (lane == 0)
#pragma unroll
        for (int i = 0; i < NV; i++) red[wave * NV + i] = v[i];
    __syncthreads();
    if (threadIdx.x < NV) {
        V s = red[threadIdx.x];
        for (int w = 1; w < RB / 64; w++) s += red[w * NV + threadIdx.x];
        red[threadIdx.x] = s;   // each thread reads its column first
    }
    __syncthreads();
}

constexpr int NSTAT = 13;   // S, sum p ln p, sum ln p, sum u^k (k = 1..10)

// Natural logarithm of a positive finite double, to a few units in the last
// place (about 30 FP64 operations, no table, no branch).  With
// x = 2^e m, m in [sqrt(1/2), sqrt(2)), ln m = 2 atanh(s) for
// s = (m - 1) / (m + 1), |s| <= 0.1716, summed as the odd series
// 2 (s + s^3/3 + ... + s^19/19); the first omitted term is below 3e-17 of
// ln m.  ln 2 is split into a 32-bit head, so e * LN2_HI is exact, and the
// remainder.  ln 1 = 0 exactly.
// a * b + c as the three-operand FP64 FMA: the series coefficients stay in
// registers across the loop, where the accumulating form (whose addend is
// also its destination) would copy each coefficient before every use
__device__ __forceinline__ double fma3(double a, double b, double c) {
    double d;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "v"(c));
    return d;
}

__device__ __forceinline__ double ln_pos(double x) {
    constexpr double LN2_HI = 6.93147180369123816490e-01;   // 0x3fe62e42fee00000
    constexpr double LN2_LO = 1.90821492927058770002e-10;   // ln 2 - LN2_HI
    int e;
    double m = frexp(x, &e);                                 // m in [1/2, 1)
    const bool lo = m < 0.70710678118654752440;
    m = lo ? m + m : m;
    e = lo ? e - 1 : e;
    const double f = m - 1.0;                                // exact
    const double d = m + 1.0;
    double r = __builtin_amdgcn_rcp(d);
    r = fma(fma(-d, r, 1.0), r, r);
    r = fma(fma(-d, r, 1.0), r, r);
    double s = f * r;
    s = fma(fma(-s, d, f), r, s);                           // s = f / d, corrected
    const double z = s * s;
    double q = 2.0 / 19.0;
    q = fma3(q, z, 2.0 / 17.0);
    q = fma3(q, z, 2.0 / 15.0);
    q = fma3(q, z, 2.0 / 13.0);
    q = fma3(q, z, 2.0 / 11.0);
    q = fma3(q, z, 2.0 / 9.0);
    q = fma3(q, z, 2.0 / 7.0);
    q = fma3(q, z, 2.0 / 5.0);
    q = fma3(q, z, 2.0 / 3.0);
    const double lnm = fma(s * z, q, s + s);
    const double de = (double)e;
    return fma(de, LN2_HI, fma(de, LN2_LO, lnm));
}

// Adds one probability p to the one-pass statistics: acc = {S, sum p ln p,
// sum ln p, sum u^k for k = 1..10} with u = N p, and counts p = 0 (those
// contribute 0 to both log sums).
__device__ __forceinline__ void stat_add(double (&acc)[NSTAT], unsigned &zeros, double p, double Nd) {
    acc[0] += p;
    const bool pos = p > 0.0;
    const double l = pos ? ln_pos(pos ? p : 1.0) : 0.0;
    acc[1] = fma(p, l, acc[1]);
    acc[2] += l;
    zeros += pos ? 0u : 1u;
    const double u = Nd * p;
    double uk = u;
#pragma unroll
    for (int k = 0; k < 10; k++) {
        acc[3 + k] += uk;
        uk *= u;
    }
}

}  // namespace svi
