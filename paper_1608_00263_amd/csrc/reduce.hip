// Reductions over the output distribution p(x) = |<x|psi>|^2 (Sec. II):
// probabilities, the one-pass statistics (entropy, uniform cross entropy,
// normalised moments), the integer-CDF sampler and the sample cross entropy.
//
// Everything here is HBM-streaming: one read of the state per statistic
// pass, at most two for the sampler.  Floating-point sums are formed in
// FP64 per thread, reduced by fixed shuffle trees inside a workgroup and
// combined across workgroups in workgroup order with Neumaier's
// compensated summation, so results are deterministic for a given size.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <mutex>

#include "internal.h"
#include "reduce_common.h"

namespace svi {

// ---------------------------------------------------------------------------
// probabilities
// ---------------------------------------------------------------------------
template <typename T, typename O>
__global__ __launch_bounds__(RB) void k_probs(const cpx<T> *__restrict__ psi, uint64_t begin,
                                              uint64_t count, O *__restrict__ out) {
    uint64_t stride = (uint64_t)gridDim.x * RB;
    for (uint64_t i = (uint64_t)blockIdx.x * RB + threadIdx.x; i < count; i += stride)
        out[i] = (O)prob_of(psi[begin + i]);
}

// ---------------------------------------------------------------------------
// statistics: per workgroup S, sum p ln p, sum ln p, sum u^k (k = 1..10),
// zero count; u = N p
// ---------------------------------------------------------------------------

template <typename T, bool FULL>
__global__ __launch_bounds__(RB) void k_stats(const cpx<T> *__restrict__ psi, uint64_t chunk,
                                              double Nd, double *__restrict__ part) {
    __shared__ double red[4 * NSTAT];
    __shared__ unsigned zred[4];
    double acc[NSTAT];
#pragma unroll
    for (int i = 0; i < NSTAT; i++) acc[i] = 0.0;
    unsigned zeros = 0;
    const uint64_t start = (uint64_t)blockIdx.x * chunk;
    // UNR loads in flight per thread before any use over the whole multiple
    // of RB * UNR (all of the chunk once the state has 2^12 amplitudes),
    // then one amplitude per thread and step over the rest
    constexpr int UNR = 8;
    const uint64_t end = start + chunk, main_end = end - chunk % (RB * UNR);
    for (uint64_t j0 = start + threadIdx.x; j0 < main_end; j0 += RB * UNR) {
        cpx<T> buf[UNR];
#pragma unroll
        for (int u = 0; u < UNR; u++) buf[u] = psi[j0 + (uint64_t)u * RB];
#pragma unroll
        for (int u = 0; u < UNR; u++) {
            const double p = prob_of(buf[u]);
            if (FULL) stat_add(acc, zeros, p, Nd);
            else acc[0] += p;
        }
    }
    for (uint64_t j = main_end + threadIdx.x; j < end; j += RB) {
        const double p = prob_of(psi[j]);
        if (FULL) stat_add(acc, zeros, p, Nd);
        else acc[0] += p;
    }
    block_sum<double, NSTAT>(acc, red);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    zeros = wave_sum(zeros);
    if (lane == 0) zred[wave] = zeros;
    __syncthreads();
    if (threadIdx.x < NSTAT) part[(uint64_t)blockIdx.x * 16 + threadIdx.x] = red[threadIdx.x];
    if (threadIdx.x == NSTAT) {
        const unsigned long long z = (unsigned long long)zred[0] + zred[1] + zred[2] + zred[3];
        part[(uint64_t)blockIdx.x * 16 + NSTAT] = (double)z;
    }
}

// Combine per-workgroup partials in workgroup order (Neumaier).
// Combine per-workgroup partial rows (16 doubles each) in row order with
// Neumaier's summation, quantity q = 0..nq-1.  256 threads: 16 row segments
// per quantity are summed in parallel, then the segment sums and their
// compensations are combined in segment order (a fixed order: the result
// does not depend on timing).
__global__ __launch_bounds__(256) void k_combine(const double *__restrict__ part, int nblocks, int nq,
                                                 double *__restrict__ out) {
    __shared__ double ss[16][16], cc[16][16];
    const int q = threadIdx.x & 15, seg = threadIdx.x >> 4;
    const int per = (nblocks + 15) / 16;
    const int b0 = seg * per, b1 = b0 + per < nblocks ? b0 + per : nblocks;
    double s = 0.0, c = 0.0;
    if (q < nq) {
        for (int b = b0; b < b1; b++) {
            const double x = part[(uint64_t)b * 16 + q];
            const double t = s + x;
            if (fabs(s) >= fabs(x)) c += (s - t) + x;
            else c += (x - t) + s;
            s = t;
        }
    }
    ss[seg][q] = s;
    cc[seg][q] = c;
    __syncthreads();
    if (threadIdx.x < nq) {
        double S = 0.0, C = 0.0;
        for (int g = 0; g < 16; g++) {
            const double x = ss[g][threadIdx.x];
            const double t = S + x;
            if (fabs(S) >= fabs(x)) C += (S - t) + x;
            else C += (x - t) + S;
            S = t;
            C += cc[g][threadIdx.x];
        }
        out[threadIdx.x] = S + C;
    }
}

static void stats_grid(int n, int *nblocks, uint64_t *chunk) {
    const uint64_t N = 1ull << n;
    uint64_t nb = N >> 12;
    if (nb < 1) nb = 1;
    if (nb > 2048) nb = 2048;
    *nblocks = (int)nb;
    *chunk = N / nb;
}

template <typename T, bool FULL>
static sv_status stats_typed(sv_state *st, const void *psi, double *host16) {
    int nb;
    uint64_t chunk;
    stats_grid(st->n, &nb, &chunk);
    SV_TRY(st->ws.reserve((size_t)(nb + 1) * 16 * sizeof(double)));
    double *part = (double *)st->ws.ptr;
    double *res = part + (size_t)nb * 16;
    hipLaunchKernelGGL((k_stats<T, FULL>), dim3(nb), dim3(RB), 0, st->stream, (const cpx<T> *)psi,
                       chunk, std::ldexp(1.0, st->n), part);
    SV_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_combine, dim3(1), dim3(256), 0, st->stream, part, nb, FULL ? NSTAT + 1 : 1, res);
    SV_HIP(hipGetLastError());
    SV_HIP(hipMemcpyAsync(host16, res, 16 * sizeof(double), hipMemcpyDeviceToHost, st->stream));
    SV_HIP(hipStreamSynchronize(st->stream));
    return SV_OK;
}

// The normalised statistics from the combined sums r (S, sum p ln p,
// sum ln p, sum u^k, zero count) of a 2^n-amplitude state.
static void finish_stats(int n, const double *r, sv_stats *out) {
    const double N = std::ldexp(1.0, n);
    const double S = r[0];
    const double lnS = std::log(S);
    out->norm = S;
    out->entropy = lnS - r[1] / S;
    out->zero_count = (int64_t)r[NSTAT];
    out->unif_ce = out->zero_count ? INFINITY : lnS - r[2] / N;
    double Sk = 1.0;
    for (int k = 0; k < 10; k++) {
        Sk *= S;
        out->moments[k] = r[3 + k] / N / Sk;
    }
}

void finish_stats_row(int n, const double *r, sv_stats *out) { finish_stats(n, r, out); }

sv_status run_stats(sv_state *st, const void *psi, sv_stats *out) {
    double r[16] = {0};
    if (st->dt == SV_C64) SV_TRY((stats_typed<float, true>(st, psi, r)));
    else SV_TRY((stats_typed<double, true>(st, psi, r)));
    finish_stats(st->n, r, out);
    return SV_OK;
}

// Enqueue the statistics pass of st into res[0..14) without synchronising
// (used inside captured graphs); part holds up to 2048 partial rows.
sv_status batch_stats_enqueue(sv_state *st, double *part, double *res) {
    int nb;
    uint64_t chunk;
    stats_grid(st->n, &nb, &chunk);
    if (st->dt == SV_C64)
        hipLaunchKernelGGL((k_stats<float, true>), dim3(nb), dim3(RB), 0, st->stream,
                           (const cpx<float> *)st->data, chunk, std::ldexp(1.0, st->n), part);
    else
        hipLaunchKernelGGL((k_stats<double, true>), dim3(nb), dim3(RB), 0, st->stream,
                           (const cpx<double> *)st->data, chunk, std::ldexp(1.0, st->n), part);
    SV_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_combine, dim3(1), dim3(256), 0, st->stream, part, nb, NSTAT + 1, res);
    SV_HIP(hipGetLastError());
    return SV_OK;
}

sv_status run_norm(sv_state *st, const void *psi, double *S) {
    double r[16] = {0};
    if (st->dt == SV_C64) SV_TRY((stats_typed<float, false>(st, psi, r)));
    else SV_TRY((stats_typed<double, false>(st, psi, r)));
    *S = r[0];
    return SV_OK;
}

sv_status run_probs(sv_state *st, uint64_t begin, uint64_t count, int f64, void *out) {
    if (!count) return SV_OK;
    uint64_t g = (count + RB - 1) / RB;
    unsigned grid = (unsigned)(g < 16384 ? g : 16384);
    if (st->dt == SV_C64) {
        if (f64) hipLaunchKernelGGL((k_probs<float, double>), dim3(grid), dim3(RB), 0, st->stream,
                                    (const cpx<float> *)st->data, begin, count, (double *)out);
        else hipLaunchKernelGGL((k_probs<float, float>), dim3(grid), dim3(RB), 0, st->stream,
                                (const cpx<float> *)st->data, begin, count, (float *)out);
    } else {
        if (f64) hipLaunchKernelGGL((k_probs<double, double>), dim3(grid), dim3(RB), 0, st->stream,
                                    (const cpx<double> *)st->data, begin, count, (double *)out);
        else hipLaunchKernelGGL((k_probs<double, float>), dim3(grid), dim3(RB), 0, st->stream,
                                (const cpx<double> *)st->data, begin, count, (float *)out);
    }
    SV_HIP(hipGetLastError());
    return SV_OK;
}

// w = floor(p 2^62): the scaling by a power of two is exact and the
// conversion truncates toward zero.
__device__ __forceinline__ uint64_t weight_of(double p) {
    return (uint64_t)(p * 4611686018427387904.0);
}

// ---------------------------------------------------------------------------
// pair statistics of an ideal output a and another output b
// ---------------------------------------------------------------------------
// Per workgroup, in FP64: S_a, S_b, Re and Im of sum conj(a) b, sum p_a^2,
// sum p_b^2, sum p_a p_b, sum over p_a > 0 of p_b ln p_a and of ln p_a, sum
// over p_a = 0 of p_b; and the number of p_a = 0.  With nbins > 0, the
// histogram of z = ln(N p_a): the slot of x is found by comparing p_a with
// the thresholds thr[0..nbins] (bin j: thr[j] <= p_a < thr[j+1]; nbins:
// below thr[0] or p_a = 0; nbins + 1: at or above thr[nbins]), and the slot
// gets the count and the integer masses floor(p 2^62) of both outputs
// (64-bit integer sums: exact, in any order) in LDS, added to hist at the
// end.
constexpr int NPAIR = 10;
constexpr int MAX_PAIR_BINS = 1024;

template <typename T>
__global__ __launch_bounds__(RB) void k_pair_stats(const cpx<T> *__restrict__ a, const cpx<T> *__restrict__ b,
                                                   uint64_t chunk, const double *__restrict__ thr, int nbins,
                                                   double *__restrict__ part, unsigned long long *__restrict__ hist) {
    __shared__ double red[4 * NPAIR];
    __shared__ unsigned zred[4];
    __shared__ double sthr[MAX_PAIR_BINS + 1];
    __shared__ unsigned long long sh[3 * (MAX_PAIR_BINS + 2)];
    const int nslot = nbins + 2;
    if (nbins > 0) {
        for (int i = threadIdx.x; i <= nbins; i += RB) sthr[i] = thr[i];
        for (int i = threadIdx.x; i < 3 * nslot; i += RB) sh[i] = 0ull;
    }
    __syncthreads();
    double acc[NPAIR];
#pragma unroll
    for (int i = 0; i < NPAIR; i++) acc[i] = 0.0;
    unsigned zeros = 0;
    const uint64_t start = (uint64_t)blockIdx.x * chunk, end = start + chunk;
    for (uint64_t j = start + threadIdx.x; j < end; j += RB) {
        const cpx<T> av = a[j], bv = b[j];
        const double ar = av.re, ai = av.im, br = bv.re, bi = bv.im;
        const double pa = prob_of(av), pb = prob_of(bv);
        acc[0] += pa;
        acc[1] += pb;
        acc[2] += fma(ar, br, ai * bi);
        acc[3] += fma(ar, bi, -ai * br);
        acc[4] = fma(pa, pa, acc[4]);
        acc[5] = fma(pb, pb, acc[5]);
        acc[6] = fma(pa, pb, acc[6]);
        const bool pos = pa > 0.0;
        const double l = pos ? ln_pos(pa) : 0.0;
        acc[7] = fma(pb, l, acc[7]);
        acc[8] += l;
        acc[9] += pos ? 0.0 : pb;
        zeros += pos ? 0u : 1u;
        if (nbins > 0) {
            int slot;
            if (!(pa >= sthr[0])) {
                slot = nbins;
            } else if (pa >= sthr[nbins]) {
                slot = nbins + 1;
            } else {
                int lo = 0, hi = nbins;   // last j with thr[j] <= p_a
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (sthr[mid] <= pa) lo = mid;
                    else hi = mid;
                }
                slot = lo;
            }
            // the host rejects the histogram when a norm reaches 4, so a
            // weight that would not fit is never reported
            const unsigned long long wa = pa < 4.0 ? weight_of(pa) : 0ull;
            const unsigned long long wb = pb < 4.0 ? weight_of(pb) : 0ull;
            atomicAdd(&sh[slot], 1ull);
            atomicAdd(&sh[nslot + slot], wa);
            atomicAdd(&sh[2 * nslot + slot], wb);
        }
    }
    block_sum<double, NPAIR>(acc, red);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    zeros = wave_sum(zeros);
    if (lane == 0) zred[wave] = zeros;
    __syncthreads();
    if (threadIdx.x < NPAIR) part[(uint64_t)blockIdx.x * 16 + threadIdx.x] = red[threadIdx.x];
    if (threadIdx.x == NPAIR) {
        const unsigned long long z = (unsigned long long)zred[0] + zred[1] + zred[2] + zred[3];
        part[(uint64_t)blockIdx.x * 16 + NPAIR] = (double)z;
    }
    if (nbins > 0)
        for (int i = threadIdx.x; i < 3 * nslot; i += RB)
            if (sh[i]) atomicAdd(&hist[i], sh[i]);
}

__global__ void k_zero_u64(unsigned long long *p, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0ull;
}

sv_status run_pair_stats(sv_state *a, sv_state *b, int nbins, const double *host_thr, double *sums16,
                         uint64_t *host_hist) {
    int nb;
    uint64_t chunk;
    stats_grid(a->n, &nb, &chunk);
    const int nslot = nbins + 2;
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t o_part = 0, o_res = al((size_t)nb * 16 * 8), o_thr = o_res + al(16 * 8),
                 o_hist = o_thr + al((size_t)(nbins + 1) * 8), need = o_hist + al((size_t)3 * nslot * 8);
    SV_TRY(a->ws.reserve(need));
    uint8_t *w = (uint8_t *)a->ws.ptr;
    double *part = (double *)(w + o_part), *res = (double *)(w + o_res), *thr = (double *)(w + o_thr);
    auto *hist = (unsigned long long *)(w + o_hist);
    hipStream_t s = a->stream;
    if (nbins > 0) {
        hipLaunchKernelGGL(k_zero_u64, dim3(4), dim3(256), 0, s, hist, 3 * nslot);
        SV_HIP(hipMemcpyAsync(thr, host_thr, (size_t)(nbins + 1) * 8, hipMemcpyHostToDevice, s));
    }
    if (a->dt == SV_C64)
        hipLaunchKernelGGL(k_pair_stats<float>, dim3(nb), dim3(RB), 0, s, (const cpx<float> *)a->data,
                           (const cpx<float> *)b->data, chunk, thr, nbins, part, hist);
    else
        hipLaunchKernelGGL(k_pair_stats<double>, dim3(nb), dim3(RB), 0, s, (const cpx<double> *)a->data,
                           (const cpx<double> *)b->data, chunk, thr, nbins, part, hist);
    SV_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_combine, dim3(1), dim3(256), 0, s, part, nb, NPAIR + 1, res);
    SV_HIP(hipGetLastError());
    SV_HIP(hipMemcpyAsync(sums16, res, 16 * sizeof(double), hipMemcpyDeviceToHost, s));
    if (nbins > 0)
        SV_HIP(hipMemcpyAsync(host_hist, hist, (size_t)3 * nslot * 8, hipMemcpyDeviceToHost, s));
    SV_HIP(hipStreamSynchronize(s));
    return SV_OK;
}

// ---------------------------------------------------------------------------
// sampler (integer CDF)
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t i) {
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Buckets of 2^bs entries, split into sub-buckets of 2^sb entries (sb <= bs,
// at most 64 per bucket).  One wavefront per sub-bucket: lane l sums entries
// l, l + 64, ... (coalesced rows), the wave total is the exact integer sum of
// the sub-bucket's weights; the workgroup then forms the bucket total from
// its sub-bucket sums in order.
constexpr int SUB_BITS = 10;   // 1024 entries per sub-bucket

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// Entries at index >= N (the ragged end of an explicit distribution whose
// length is not a power of two) have weight 0 and are not read.
template <typename S>
__global__ __launch_bounds__(RB) void k_bucket_weights(const S *__restrict__ src, uint64_t N, int bs, int sb,
                                                       unsigned long long *__restrict__ bsum,
                                                       unsigned long long *__restrict__ subsum) {
    __shared__ unsigned long long sh[64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nsub = 1 << (bs - sb);
    const uint64_t slen = 1ull << sb;
    for (int j = wave; j < nsub; j += RB / 64) {
        const uint64_t start = ((uint64_t)blockIdx.x << bs) + ((uint64_t)j << sb);
        unsigned long long acc = 0;
        for (uint64_t e = lane; e < slen; e += 64)
            if (start + e < N) acc += weight_of(prob_of(src[start + e]));
        acc = wave_sum_u64(acc);
        if (lane == 0) {
            subsum[(uint64_t)blockIdx.x * nsub + j] = acc;
            sh[j] = acc;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int j = 0; j < nsub; j++) t += sh[j];
        bsum[blockIdx.x] = t;
    }
}

// The statistics and the sampler's bucket weights in one read of the state:
// workgroup g takes buckets g, g + G, ... (2^bs amplitudes each; G = the
// grid size, at most 2048 so that few statistic rows remain to combine),
// each wavefront whole sub-buckets of 2^sb amplitudes, as k_bucket_weights
// does; every amplitude also enters this workgroup's row of statistic sums,
// as in k_stats.
template <typename S>
__global__ __launch_bounds__(RB) void k_stats_weights(const S *__restrict__ src, int bs, int sb, uint64_t nbk,
                                                      double Nd, double *__restrict__ part,
                                                      unsigned long long *__restrict__ bsum,
                                                      unsigned long long *__restrict__ subsum) {
    __shared__ unsigned long long sh[64];
    __shared__ double red[4 * NSTAT];
    __shared__ unsigned zred[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nsub = 1 << (bs - sb);
    const uint64_t slen = 1ull << sb;
    double acc[NSTAT];
#pragma unroll
    for (int i = 0; i < NSTAT; i++) acc[i] = 0.0;
    unsigned zeros = 0;
    constexpr int UNR = 8;   // loads in flight per lane
    for (uint64_t b = blockIdx.x; b < nbk; b += gridDim.x) {
      for (int j = wave; j < nsub; j += RB / 64) {
        const uint64_t start = (b << bs) + ((uint64_t)j << sb);
        unsigned long long w = 0;
        const uint64_t main_end = slen - slen % (64 * UNR);
        for (uint64_t e0 = lane; e0 < main_end; e0 += 64 * UNR) {
            S buf[UNR];
#pragma unroll
            for (int u = 0; u < UNR; u++) buf[u] = src[start + e0 + (uint64_t)u * 64];
#pragma unroll
            for (int u = 0; u < UNR; u++) {
                const double p = prob_of(buf[u]);
                w += weight_of(p);
                stat_add(acc, zeros, p, Nd);
            }
        }
        for (uint64_t e = main_end + lane; e < slen; e += 64) {
            const double p = prob_of(src[start + e]);
            w += weight_of(p);
            stat_add(acc, zeros, p, Nd);
        }
        w = wave_sum_u64(w);
        if (lane == 0) {
            subsum[b * nsub + j] = w;
            sh[j] = w;
        }
      }
      __syncthreads();
      if (threadIdx.x == 0) {
          unsigned long long t = 0;
          for (int j = 0; j < nsub; j++) t += sh[j];
          bsum[b] = t;
      }
      __syncthreads();   // sh is reused by the next bucket
    }
    block_sum<double, NSTAT>(acc, red);
    zeros = wave_sum(zeros);
    if (lane == 0) zred[wave] = zeros;
    __syncthreads();
    if (threadIdx.x < NSTAT) part[(uint64_t)blockIdx.x * 16 + threadIdx.x] = red[threadIdx.x];
    if (threadIdx.x == NSTAT) {
        const unsigned long long z = (unsigned long long)zred[0] + zred[1] + zred[2] + zred[3];
        part[(uint64_t)blockIdx.x * 16 + NSTAT] = (double)z;
    }
}

// Exclusive scan of n uint64 values into out[0..n], out[n] = total.  One
// workgroup of 1024 threads; each thread scans a contiguous stretch.
__global__ __launch_bounds__(1024) void k_scan(const unsigned long long *__restrict__ in, uint64_t n,
                                               unsigned long long *__restrict__ out) {
    __shared__ unsigned long long sh[1024];
    const uint64_t per = (n + 1023) / 1024;
    const uint64_t b = threadIdx.x * per;
    const uint64_t e = b + per < n ? b + per : n;
    unsigned long long s = 0;
    for (uint64_t i = b; i < e; i++) s += in[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        unsigned long long v = threadIdx.x >= (unsigned)d ? sh[threadIdx.x - d] : 0ull;
        __syncthreads();
        sh[threadIdx.x] += v;
        __syncthreads();
    }
    unsigned long long run = sh[threadIdx.x] - s;   // exclusive prefix of this stretch
    for (uint64_t i = b; i < e; i++) {
        out[i] = run;
        run += in[i];
    }
    if (threadIdx.x == 1023) out[n] = sh[1023];
}

// Per sample: target t = floor(r W / 2^64), its bucket (last b with
// off[b] <= t) and the target's offset inside the bucket.
__global__ __launch_bounds__(RB) void k_targets(const uint64_t *__restrict__ words, uint64_t seed,
                                                int64_t k, const unsigned long long *__restrict__ off,
                                                uint64_t nb, uint32_t *__restrict__ tb,
                                                unsigned long long *__restrict__ tloc) {
    const int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x;
    if (i >= k) return;
    const unsigned long long W = off[nb];
    const uint64_t r = words ? words[i] : splitmix64(seed, (uint64_t)i);
    const unsigned long long t = __umul64hi(r, W);
    uint64_t lo = 0, hi = nb;   // first b with off[b] > t, minus one
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (off[mid] > t) hi = mid; else lo = mid + 1;
    }
    const uint64_t b = lo - 1;
    tb[i] = (uint32_t)b;
    tloc[i] = t - off[b];
}

// Inclusive prefix sum over the 64 lanes (lane order).
__device__ __forceinline__ unsigned long long wave_incl_scan_u64(unsigned long long v, int lane) {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const unsigned long long o = __shfl_up(v, d, 64);
        if (lane >= d) v += o;
    }
    return v;
}

// One wavefront per sample: the sub-bucket holding the target (first
// sub-bucket whose running sum exceeds it), then the lane run of R
// consecutive entries holding it, then the entry: x = min{j : C_j > t}.
template <typename S>
__global__ __launch_bounds__(RB) void k_resolve(const S *__restrict__ src, uint64_t N, int bs, int sb,
                                                const unsigned long long *__restrict__ subsum,
                                                const uint32_t *__restrict__ tb,
                                                const unsigned long long *__restrict__ tloc, int64_t k,
                                                uint64_t *__restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * (RB / 64) + (threadIdx.x >> 6);
    if (i >= k) return;
    const uint64_t b = tb[i];
    const unsigned long long t = tloc[i];
    const int nsub = 1 << (bs - sb);
    // sub-bucket
    const unsigned long long own = lane < nsub ? subsum[b * nsub + lane] : 0ull;
    const unsigned long long incl = wave_incl_scan_u64(own, lane);
    const unsigned long long above = __ballot(lane < nsub && incl > t);
    int j = __ffsll((long long)above) - 1;
    if (j < 0) j = nsub - 1;   // unreachable (t < bucket total); keeps every access in range
    const unsigned long long before_j = __shfl(incl - own, j, 64);
    const unsigned long long ts = t - before_j;
    // lane runs of R entries inside sub-bucket j
    const uint64_t start = (b << bs) + ((uint64_t)j << sb);
    const int slen = 1 << sb;
    const int R = slen >= 64 ? slen / 64 : 1;
    const bool has = lane * R < slen;
    unsigned long long run = 0;
    if (has)
        for (int e = 0; e < R; e++) {
            const uint64_t x = start + (uint64_t)lane * R + e;
            if (x < N) run += weight_of(prob_of(src[x]));
        }
    const unsigned long long rincl = wave_incl_scan_u64(run, lane);
    const unsigned long long hit = __ballot(has && rincl > ts);
    int L = __ffsll((long long)hit) - 1;
    if (L < 0) L = (slen >= 64 ? 64 : slen) - 1;   // unreachable (ts < sub-bucket total)
    if (lane == L) {
        unsigned long long c = rincl - run;
        uint64_t ans = start + (uint64_t)lane * R + (R - 1);
        for (int e = 0; e < R; e++) {
            const uint64_t x = start + (uint64_t)lane * R + e;
            if (x < N) c += weight_of(prob_of(src[x]));
            if (c > ts) {
                ans = start + (uint64_t)lane * R + e;
                break;
            }
        }
        out[i] = ans;
    }
}

// Device scratch of the sampler: a workspace grown on demand, or a fixed
// buffer of cap bytes that must already be large enough.
struct ScratchSource {
    Workspace *ws = nullptr;
    void *fixed = nullptr;
    size_t cap = 0;
};

static sv_status take_scratch(const ScratchSource &scr, size_t need, uint8_t **out) {
    if (scr.ws) {
        SV_TRY(scr.ws->reserve(need));
        *out = (uint8_t *)scr.ws->ptr;
        return SV_OK;
    }
    if (need > scr.cap) {
        char b[160];
        snprintf(b, sizeof b, "needs %zu bytes of scratch, the fixed scratch holds %zu", need, scr.cap);
        return fail(SV_ERANGE, b);
    }
    *out = (uint8_t *)scr.fixed;
    return SV_OK;
}

// Layout of the sampler's scratch for 2^n entries and k samples (with the
// statistics rows when stats is set): byte offsets of its parts and the
// total.
struct SampleLayout {
    int bs, sb;
    uint64_t nb, nsubs, ng;
    size_t o_bsum, o_off, o_sub, o_tb, o_tl, o_part, o_res, need;
};

static SampleLayout sample_layout(int n, int64_t k, bool stats) {
    SampleLayout L{};
    L.bs = n < 16 ? n : 16;
    L.sb = L.bs < SUB_BITS ? L.bs : SUB_BITS;
    L.nb = 1ull << (n - L.bs);
    L.nsubs = 1ull << (n - L.sb);
    L.ng = L.nb < 2048 ? L.nb : 2048;   // workgroups of the fused statistics pass
    size_t need = 0;
    auto take = [&](size_t bytes) { size_t o = need; need += (bytes + 255) & ~(size_t)255; return o; };
    L.o_bsum = take(L.nb * 8);
    L.o_off = take((L.nb + 1) * 8);
    L.o_sub = take(L.nsubs * 8);
    L.o_tb = take((size_t)k * 4);
    L.o_tl = take((size_t)k * 8);
    L.o_part = stats ? take(L.ng * 16 * 8) : 0;
    L.o_res = stats ? take(16 * 8) : 0;
    L.need = need;
    return L;
}

// The sampler; with stats16 non-null (states only) the bucket weights come
// from the fused statistics pass, whose 14 combined sums are copied to
// stats16 (and k may be 0).
// src holds N = 2^n entries, or (explicit distributions) any N in
// (2^{n-1}, 2^n], the entries beyond N counting as weight 0.
template <typename S>
static sv_status sample_impl(const ScratchSource &scr, hipStream_t s, const S *src, int n, const uint64_t *words,
                             uint64_t seed, int64_t k, uint64_t *dev_out, double *stats16 = nullptr,
                             uint64_t N = 0) {
    if (N == 0) N = 1ull << n;
    if (k <= 0 && !stats16) return SV_OK;
    if (k < 0) k = 0;
    const SampleLayout L = sample_layout(n, k, stats16 != nullptr);
    const int bs = L.bs, sb = L.sb;
    const uint64_t nb = L.nb, ng = L.ng;
    const size_t o_bsum = L.o_bsum, o_off = L.o_off, o_sub = L.o_sub, o_tb = L.o_tb, o_tl = L.o_tl,
                 o_part = L.o_part, o_res = L.o_res;
    uint8_t *w = nullptr;
    SV_TRY(take_scratch(scr, L.need, &w));
    auto *bsum = (unsigned long long *)(w + o_bsum);
    auto *off = (unsigned long long *)(w + o_off);
    auto *sub = (unsigned long long *)(w + o_sub);
    auto *tb = (uint32_t *)(w + o_tb);
    auto *tl = (unsigned long long *)(w + o_tl);
    if (stats16) {
        double *part = (double *)(w + o_part), *res = (double *)(w + o_res);
        hipLaunchKernelGGL((k_stats_weights<S>), dim3((unsigned)ng), dim3(RB), 0, s, src, bs, sb, nb,
                           std::ldexp(1.0, n), part, bsum, sub);
        hipLaunchKernelGGL(k_combine, dim3(1), dim3(256), 0, s, part, (int)ng, NSTAT + 1, res);
        SV_HIP(hipGetLastError());
        SV_HIP(hipMemcpyAsync(stats16, res, 16 * sizeof(double), hipMemcpyDeviceToHost, s));
        if (k == 0) {
            SV_HIP(hipStreamSynchronize(s));
            return SV_OK;
        }
    } else {
        hipLaunchKernelGGL((k_bucket_weights<S>), dim3((unsigned)nb), dim3(RB), 0, s, src, N, bs, sb, bsum, sub);
    }
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, bsum, nb, off);
    unsigned long long W = 0;
    SV_HIP(hipMemcpyAsync(&W, off + nb, 8, hipMemcpyDeviceToHost, s));
    SV_HIP(hipStreamSynchronize(s));
    if (W == 0) return fail(SV_ESTATE, "sampler: every probability rounds to weight 0");
    const unsigned kg = (unsigned)((k + RB - 1) / RB);
    hipLaunchKernelGGL(k_targets, dim3(kg), dim3(RB), 0, s, words, seed, k, off, nb, tb, tl);
    const unsigned rg = (unsigned)((k + RB / 64 - 1) / (RB / 64));
    hipLaunchKernelGGL((k_resolve<S>), dim3(rg), dim3(RB), 0, s, src, N, bs, sb, sub, tb, tl, k, dev_out);
    SV_HIP(hipGetLastError());
    return SV_OK;
}

sv_status run_sample(sv_state *st, const void *psi, int64_t k, uint64_t seed, uint64_t *dev_out) {
    ScratchSource scr;
    scr.ws = &st->ws;
    if (st->dt == SV_C64)
        return sample_impl<cpx<float>>(scr, st->stream, (const cpx<float> *)psi, st->n, nullptr,
                                       seed, k, dev_out);
    return sample_impl<cpx<double>>(scr, st->stream, (const cpx<double> *)psi, st->n, nullptr,
                                    seed, k, dev_out);
}

static sv_status stats_sample_from(const ScratchSource &scr, sv_state *st, const void *psi, sv_stats *stats,
                                   int64_t k, uint64_t seed, uint64_t *dev_out) {
    double r[16] = {0};
    if (st->dt == SV_C64)
        SV_TRY(sample_impl<cpx<float>>(scr, st->stream, (const cpx<float> *)psi, st->n, nullptr, seed, k,
                                       dev_out, r));
    else
        SV_TRY(sample_impl<cpx<double>>(scr, st->stream, (const cpx<double> *)psi, st->n, nullptr, seed, k,
                                        dev_out, r));
    finish_stats(st->n, r, stats);
    return SV_OK;
}

sv_status run_stats_sample(sv_state *st, const void *psi, sv_stats *stats, int64_t k, uint64_t seed,
                           uint64_t *dev_out) {
    ScratchSource scr;
    scr.ws = &st->ws;
    return stats_sample_from(scr, st, psi, stats, k, seed, dev_out);
}

// ---------------------------------------------------------------------------
// allocation-free statistics and samples
// ---------------------------------------------------------------------------
// The scratch of sv_moments_sample_noalloc: device memory that comes with
// the code object on every GPU the library runs on (held until the process
// ends), so the call needs no allocation.  Host code never uses this name
// as an address: its device address on each GPU is looked up once, with
// that GPU current, and kept per device.
__device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[MAX_DEVICES] = {};

static sv_status noalloc_scratch(int device, void **out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (device < 0 || device >= MAX_DEVICES) return fail(SV_EDEVICE, "device index out of range");
    if (!g_scratch_ptr[device]) {
        int cur = 0;
        SV_HIP(hipGetDevice(&cur));
        if (cur != device) SV_HIP(hipSetDevice(device));
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) (void)hipSetDevice(cur);
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return SV_OK;
}

size_t noalloc_scratch_need(int n, int64_t k) { return sample_layout(n, k, true).need; }

sv_status run_stats_sample_noalloc(sv_state *st, sv_stats *stats, int64_t k, uint64_t seed, uint64_t *dev_out) {
    const size_t need = noalloc_scratch_need(st->n, k);
    if (need > NOALLOC_SCRATCH_BYTES) {
        char b[200];
        snprintf(b, sizeof b, "sv_moments_sample_noalloc: n = %d and k = %lld need %zu bytes of scratch, "
                 "the fixed scratch holds %zu", st->n, (long long)k, need, (size_t)NOALLOC_SCRATCH_BYTES);
        return fail(SV_ERANGE, b);
    }
    ScratchSource scr;
    SV_TRY(noalloc_scratch(st->device, &scr.fixed));
    scr.cap = NOALLOC_SCRATCH_BYTES;
    return stats_sample_from(scr, st, st->data, stats, k, seed, dev_out);
}

// Validation of an explicit distribution for the integer-CDF sampler: every
// p must be finite, >= 0 and < 4 (its weight floor(p 2^62) fits 64 bits),
// and the weights must sum below 2^64.  Per workgroup, the exact 128-bit
// sum of the weights of its 2^16 entries (high and low words) and a flag for
// an invalid entry; one more workgroup adds the rows (high words cannot
// overflow: at most 2^19 rows of at most 2^80 each).
constexpr int VAL_BITS = 16;

__global__ __launch_bounds__(RB) void k_validate_weights(const double *__restrict__ p, uint64_t N,
                                                         unsigned long long *__restrict__ rows) {
    __shared__ unsigned long long slo[RB], shi[RB];
    __shared__ unsigned sbad[RB];
    const uint64_t start = (uint64_t)blockIdx.x << VAL_BITS;
    unsigned long long lo = 0, hi = 0;
    unsigned bad = 0;
    for (uint64_t e = threadIdx.x; e < (1ull << VAL_BITS); e += RB) {
        const uint64_t x = start + e;
        if (x >= N) break;
        const double v = p[x];
        if (!(v >= 0.0) || !(v < 4.0)) { bad = 1; continue; }   // NaN, negative, >= 4, inf
        const unsigned long long w = weight_of(v);
        lo += w;
        hi += lo < w ? 1ull : 0ull;
    }
    slo[threadIdx.x] = lo;
    shi[threadIdx.x] = hi;
    sbad[threadIdx.x] = bad;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long L = 0, H = 0;
        unsigned B = 0;
        for (int t = 0; t < RB; t++) {
            L += slo[t];
            H += shi[t] + (L < slo[t] ? 1ull : 0ull);
            B |= sbad[t];
        }
        rows[3 * (uint64_t)blockIdx.x] = L;
        rows[3 * (uint64_t)blockIdx.x + 1] = H;
        rows[3 * (uint64_t)blockIdx.x + 2] = B;
    }
}

__global__ __launch_bounds__(64) void k_validate_total(const unsigned long long *__restrict__ rows, uint64_t nrows,
                                                       unsigned long long *__restrict__ out) {
    if (threadIdx.x != 0) return;
    unsigned long long L = 0, H = 0, B = 0;
    for (uint64_t r = 0; r < nrows; r++) {
        const unsigned long long l = rows[3 * r];
        L += l;
        H += rows[3 * r + 1] + (L < l ? 1ull : 0ull);
        B |= rows[3 * r + 2];
    }
    out[0] = L;
    out[1] = H;
    out[2] = B;
}

sv_status run_sample_from(const double *probs, uint64_t N, const uint64_t *r64, int64_t k,
                          uint64_t *out, hipStream_t s) {
    int n = 0;
    while ((1ull << n) < N) n++;
    // library-owned scratch for this standalone call; kept until the process
    // ends (never freed from a static destructor, after the runtime is gone)
    static ScratchSource *scr = new ScratchSource{new Workspace(), nullptr, 0};
    static Workspace *vws = new Workspace();
    const uint64_t nrows = (N + (1ull << VAL_BITS) - 1) >> VAL_BITS;
    SV_TRY(vws->reserve((size_t)(nrows + 1) * 3 * 8));
    auto *rows = (unsigned long long *)vws->ptr;
    hipLaunchKernelGGL(k_validate_weights, dim3((unsigned)nrows), dim3(RB), 0, s, probs, N, rows);
    hipLaunchKernelGGL(k_validate_total, dim3(1), dim3(64), 0, s, rows, nrows, rows + 3 * nrows);
    SV_HIP(hipGetLastError());
    unsigned long long tot[3] = {0, 0, 0};
    SV_HIP(hipMemcpyAsync(tot, rows + 3 * nrows, sizeof tot, hipMemcpyDeviceToHost, s));
    SV_HIP(hipStreamSynchronize(s));
    if (tot[2]) return fail(SV_EINVAL, "sv_sample_from: a probability is negative, NaN, infinite or >= 4");
    if (tot[1]) return fail(SV_ERANGE, "sv_sample_from: the weights floor(p 2^62) sum to 2^64 or more (sum p >= 4)");
    if (k == 0) return SV_OK;
    sv_status rc = sample_impl<double>(*scr, s, probs, n, r64, 0, k, out, nullptr, N);
    if (rc != SV_OK) return rc;
    SV_HIP(hipStreamSynchronize(s));
    return SV_OK;
}

// ---------------------------------------------------------------------------
// sample cross entropy: sum_i ln p(x_i) and the number of p(x_i) = 0
// ---------------------------------------------------------------------------
// Samples are n-bit strings (checked on the host before the copy).
template <typename T>
__global__ __launch_bounds__(RB) void k_ce(const cpx<T> *__restrict__ psi,
                                           const uint64_t *__restrict__ x, int64_t k, int64_t per,
                                           double *__restrict__ part) {
    __shared__ double red[4 * 2];
    double v[2] = {0.0, 0.0};
    const int64_t b = (int64_t)blockIdx.x * per;
    const int64_t e = b + per < k ? b + per : k;
    for (int64_t i = b + threadIdx.x; i < e; i += RB) {
        const double p = prob_of(psi[x[i]]);
        if (p > 0.0) v[0] += log(p);
        else v[1] += 1.0;
    }
    block_sum<double, 2>(v, red);
    if (threadIdx.x < 2) part[(uint64_t)blockIdx.x * 16 + threadIdx.x] = red[threadIdx.x];
}

sv_status run_cross_entropy(sv_state *st, const void *psi, const uint64_t *dev_samples, int64_t k,
                            double S, double *sum_log, int64_t *zeros) {
    (void)S;
    if (k <= 0) { *sum_log = 0; *zeros = 0; return SV_OK; }
    const int64_t per = 4096;
    const int64_t nb = (k + per - 1) / per;
    SV_TRY(st->ws.reserve((size_t)(nb + 1) * 16 * sizeof(double)));
    double *part = (double *)st->ws.ptr;
    double *res = part + (size_t)nb * 16;
    if (st->dt == SV_C64)
        hipLaunchKernelGGL(k_ce<float>, dim3((unsigned)nb), dim3(RB), 0, st->stream,
                           (const cpx<float> *)psi, dev_samples, k, per, part);
    else
        hipLaunchKernelGGL(k_ce<double>, dim3((unsigned)nb), dim3(RB), 0, st->stream,
                           (const cpx<double> *)psi, dev_samples, k, per, part);
    SV_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_combine, dim3(1), dim3(256), 0, st->stream, part, (int)nb, 2, res);
    double r[2];
    SV_HIP(hipMemcpyAsync(r, res, 2 * sizeof(double), hipMemcpyDeviceToHost, st->stream));
    SV_HIP(hipStreamSynchronize(st->stream));
    *sum_log = r[0];
    *zeros = (int64_t)r[1];
    return SV_OK;
}

}  // namespace svi
