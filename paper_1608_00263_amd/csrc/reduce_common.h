// Device helpers shared by the reduction kernels and the ensemble kernel:
// probabilities in FP64 and fixed-order wavefront / workgroup sums.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace svi {

constexpr int RB = 256;   // threads per workgroup

template <typename T> struct cpx { T re, im; };

// p = re*re + im*im with both products and the sum rounded separately (no
// contraction); for complex64 input both products are exact in FP64.
__device__ __forceinline__ double prob_of(cpx<float> a) {
    double r = (double)a.re, i = (double)a.im;
    return __dadd_rn(__dmul_rn(r, r), __dmul_rn(i, i));
}
__device__ __forceinline__ double prob_of(cpx<double> a) {
    return __dadd_rn(__dmul_rn(a.re, a.re), __dmul_rn(a.im, a.im));
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

}  // namespace svi
