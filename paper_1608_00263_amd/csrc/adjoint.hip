// Adjoint gradient of the sample cross entropy with respect to per-gate
// rotation offsets.
//
// L(theta) = -(1/m) sum_i ln p_theta(x_i).  With psi = U_G ... U_1 |0>,
// lambda_x = n_x psi_x / (m p_x) and dU_g = D_g U_g, walking the gates
// backwards from phi = psi, mu = lambda gives
//     dL/dtheta_g = -2 Re <mu| D_g |phi>,   then phi <- U_g^dag phi, mu <- U_g^dag mu.
// phi is rebuilt by applying inverse gates rather than stored; a copy of
// the forward state at every checkpoint (complex64 for the complex64 path)
// bounds the drift of that uncomputation.
//
// The backward sweeps reuse the register tiles of the forward plan with
// the programs reversed and conjugated, carrying phi and mu through the
// same tile (so each sweep moves 2 states).  At a parametrised gate the
// wavefront forms its share of Re <mu| D |phi> before applying the
// inverse; the shares are written per (tile, slot) and summed in tile
// order afterwards.
#include <hip/hip_runtime.h>

#include <cmath>

#include "device_common.h"
#include "internal.h"

namespace svi {

// Sum over the 64 lanes of a wavefront, the same in every lane.  Complex64
// states sum their gradient shares in FP32 by a butterfly of DPP moves
// (lane bits 0..3) and register half-swaps (bits 4, 5); complex128 states
// in FP64 through the lane shuffles.
template <typename T>
__device__ __forceinline__ double wave_sum_d(double g) {
    if constexpr (sizeof(T) == 4) {
        float v = (float)g;
        v += lane_xor<0>(v);
        v += lane_xor<1>(v);
        v += lane_xor<2>(v);
        v += lane_xor<3>(v);
        int a = __float_as_int(v), b = a;
        half_swap_i<4>(a, b);
        v = __int_as_float(a) + __int_as_float(b);
        a = __float_as_int(v);
        b = a;
        half_swap_i<5>(a, b);
        v = __int_as_float(a) + __int_as_float(b);
        return (double)v;
    } else {
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) g += __shfl_xor(g, m, 64);
        return g;
    }
}

// Im conj(a) b and Re conj(a) b
template <typename T>
__device__ __forceinline__ T im_cm(cplx<T> a, cplx<T> b) { return fma(a.re, b.im, -a.im * b.re); }
template <typename T>
__device__ __forceinline__ T re_cm(cplx<T> a, cplx<T> b) { return fma(a.re, b.re, a.im * b.im); }

// acc += s Im conj(a) b and acc += s Re conj(a) b as two fused multiply-adds
// (s = +1 or -1 at compile time)
template <int SG, typename T>
__device__ __forceinline__ void acc_im_cm(T &acc, cplx<T> a, cplx<T> b) {
    acc = fma((T)SG * a.re, b.im, acc);
    acc = fma((T)(-SG) * a.im, b.re, acc);
}
template <int SG, typename T>
__device__ __forceinline__ void acc_re_cm(T &acc, cplx<T> a, cplx<T> b) {
    acc = fma((T)SG * a.re, b.re, acc);
    acc = fma((T)SG * a.im, b.im, acc);
}

// This lane's share of Re <mu| D |phi> for D on register slot S.  Closed
// forms for the generators of the parametrised gates (pairs (0, 1) of the
// slot): RX: D = -(i/2) X gives (1/2) [Im conj(mu0) phi1 + Im conj(mu1) phi0];
// RY: D = -(i/2) Y gives (1/2) [Re conj(mu1) phi0 - Re conj(mu0) phi1];
// phase: D = i|1><1| gives -Im conj(mu1) phi1.
template <typename T, int NR, int S, int G>
__device__ __forceinline__ double grad_reg_g(const cplx<T> (&phi)[NR], const cplx<T> (&mu)[NR],
                                             const Mat2<T> &d) {
    if constexpr (G == G_GEN) {
        double acc = 0;
#pragma unroll
        for (int r = 0; r < NR; r++) {
            if (r & (1 << S)) continue;
            const int r1 = r | (1 << S);
            cplx<T> d0 = cmad(d.m[1], phi[r1], cmul(d.m[0], phi[r]));
            cplx<T> d1 = cmad(d.m[3], phi[r1], cmul(d.m[2], phi[r]));
            acc += (double)re_cm(mu[r], d0) + (double)re_cm(mu[r1], d1);
        }
        return acc;
    } else {
        // two accumulators, so that the multiply-add chains are half as long
        T acc[2] = {0, 0};
        int k = 0;
#pragma unroll
        for (int r = 0; r < NR; r++) {
            if (r & (1 << S)) continue;
            const int r1 = r | (1 << S);
            if constexpr (G == G_RX) {
                acc_im_cm<1>(acc[0], mu[r], phi[r1]);
                acc_im_cm<1>(acc[1], mu[r1], phi[r]);
            } else if constexpr (G == G_RY) {
                acc_re_cm<1>(acc[0], mu[r1], phi[r]);
                acc_re_cm<-1>(acc[1], mu[r], phi[r1]);
            } else {
                acc_im_cm<-1>(acc[k & 1], mu[r1], phi[r1]);
                k++;
            }
        }
        return (G == G_P ? 1.0 : 0.5) * (double)(acc[0] + acc[1]);
    }
}

template <typename T, int NR, int S>
__device__ __forceinline__ double grad_reg_s(const cplx<T> (&phi)[NR], const cplx<T> (&mu)[NR],
                                             const Mat2<T> &d, int g) {
    switch (g) {
    case G_RX: return grad_reg_g<T, NR, S, G_RX>(phi, mu, d);
    case G_RY: return grad_reg_g<T, NR, S, G_RY>(phi, mu, d);
    case G_P: return grad_reg_g<T, NR, S, G_P>(phi, mu, d);
    default: return grad_reg_g<T, NR, S, G_GEN>(phi, mu, d);
    }
}

template <typename T, int NR>
__device__ __forceinline__ double grad_reg_dispatch(const cplx<T> (&phi)[NR], const cplx<T> (&mu)[NR],
                                                    const Mat2<T> &d, int s, int g) {
    switch (s) {
    case 0: return grad_reg_s<T, NR, 0>(phi, mu, d, g);
    case 1: if constexpr (NR > 2) return grad_reg_s<T, NR, 1>(phi, mu, d, g); break;
    case 2: if constexpr (NR > 4) return grad_reg_s<T, NR, 2>(phi, mu, d, g); break;
    case 3: if constexpr (NR > 8) return grad_reg_s<T, NR, 3>(phi, mu, d, g); break;
    case 4: if constexpr (NR > 16) return grad_reg_s<T, NR, 4>(phi, mu, d, g); break;
    default: break;
    }
    return 0.0;
}

// The same for D on lane bit B: the pair partner lives in the lane whose
// bit B differs (hi = this lane's bit).
template <typename T, int NR, int B, int G>
__device__ __forceinline__ double grad_lane_g(const cplx<T> (&phi)[NR], const cplx<T> (&mu)[NR],
                                              const Mat2<T> &d, int lane) {
    const bool hi = (lane >> B) & 1;
    if constexpr (G == G_P) {
        T acc[2] = {0, 0};
#pragma unroll
        for (int r = 0; r < NR; r++) acc_im_cm<-1>(acc[r & 1], mu[r], phi[r]);
        return hi ? (double)(acc[0] + acc[1]) : 0.0;
    } else if constexpr (G == G_GEN) {
        cplx<T> cs = hi ? d.m[3] : d.m[0];
        cplx<T> cp = hi ? d.m[2] : d.m[1];
        double acc = 0;
#pragma unroll
        for (int r = 0; r < NR; r++) {
            cplx<T> p;
            p.re = lane_xor<B>(phi[r].re);
            p.im = lane_xor<B>(phi[r].im);
            acc += (double)re_cm(mu[r], cmad(cp, p, cmul(cs, phi[r])));
        }
        return acc;
    } else {
        T acc[2] = {0, 0};
#pragma unroll
        for (int r = 0; r < NR; r++) {
            cplx<T> p;
            p.re = lane_xor<B>(phi[r].re);
            p.im = lane_xor<B>(phi[r].im);
            if constexpr (G == G_RX) acc_im_cm<1>(acc[r & 1], mu[r], p);
            else acc_re_cm<1>(acc[r & 1], mu[r], p);
        }
        T a = acc[0] + acc[1];
        if constexpr (G == G_RY) a = hi ? a : -a;
        return 0.5 * (double)a;
    }
}

template <typename T, int NR, int B>
__device__ __forceinline__ double grad_lane_b(const cplx<T> (&phi)[NR], const cplx<T> (&mu)[NR],
                                              const Mat2<T> &d, int lane, int g) {
    switch (g) {
    case G_RX: return grad_lane_g<T, NR, B, G_RX>(phi, mu, d, lane);
    case G_RY: return grad_lane_g<T, NR, B, G_RY>(phi, mu, d, lane);
    case G_P: return grad_lane_g<T, NR, B, G_P>(phi, mu, d, lane);
    default: return grad_lane_g<T, NR, B, G_GEN>(phi, mu, d, lane);
    }
}

template <typename T, int NR>
__device__ __forceinline__ double grad_lane_dispatch(const cplx<T> (&phi)[NR], const cplx<T> (&mu)[NR],
                                                     const Mat2<T> &d, int b, int lane, int g) {
    switch (b) {
    case 0: return grad_lane_b<T, NR, 0>(phi, mu, d, lane, g);
    case 1: return grad_lane_b<T, NR, 1>(phi, mu, d, lane, g);
    case 2: return grad_lane_b<T, NR, 2>(phi, mu, d, lane, g);
    case 3: return grad_lane_b<T, NR, 3>(phi, mu, d, lane, g);
    case 4: return grad_lane_b<T, NR, 4>(phi, mu, d, lane, g);
    default: return grad_lane_b<T, NR, 5>(phi, mu, d, lane, g);
    }
}

// A rotation in tangent form on lane bit 4 or 5 with its gradient share,
// phi and mu together: register half-swaps give every lane whole pairs of
// both states, so the share is lane-local (no cross-lane moves beyond the
// swaps the gate needs anyway).  G_RX share (1/2)[Im conj(mu0) phi1 +
// Im conj(mu1) phi0], G_RY share (1/2)[Re conj(mu1) phi0 - Re conj(mu0)
// phi1], taken before the gate.
template <typename T, int NR, int B, int FORM>
__device__ __forceinline__ double lane_rot_grad_gate(cplx<T> (&phi)[NR], cplx<T> (&mu)[NR], const Mat2<T> &u) {
    static_assert(B == 4 || B == 5, "half swaps exist for lane bits 4 and 5");
    T acc[2] = {0, 0};
#pragma unroll
    for (int r = 0; r < NR; r += 2) {
        cplx<T> x = phi[r], y = phi[r + 1], mx = mu[r], my = mu[r + 1];
        half_swap<B>(x.re, y.re);
        half_swap<B>(x.im, y.im);
        half_swap<B>(mx.re, my.re);
        half_swap<B>(mx.im, my.im);
        if constexpr (FORM == F_TRX) {
            acc_im_cm<1>(acc[0], mx, y);
            acc_im_cm<1>(acc[1], my, x);
        } else {
            acc_re_cm<1>(acc[0], my, x);
            acc_re_cm<-1>(acc[1], mx, y);
        }
        pair_form<T, FORM>(x, y, u);
        pair_form<T, FORM>(mx, my, u);
        half_swap<B>(x.re, y.re);
        half_swap<B>(x.im, y.im);
        half_swap<B>(mx.re, my.re);
        half_swap<B>(mx.im, my.im);
        phi[r] = x;
        phi[r + 1] = y;
        mu[r] = mx;
        mu[r + 1] = my;
    }
    return 0.5 * (double)(acc[0] + acc[1]);
}

template <typename T, int NR>
__device__ __forceinline__ double lane_rot_dispatch(cplx<T> (&phi)[NR], cplx<T> (&mu)[NR], const Mat2<T> &u,
                                                    int b, int form) {
    if constexpr (NR >= 2) {
        if (b == 4) return form == F_TRX ? lane_rot_grad_gate<T, NR, 4, F_TRX>(phi, mu, u)
                                         : lane_rot_grad_gate<T, NR, 4, F_TRY>(phi, mu, u);
        return form == F_TRX ? lane_rot_grad_gate<T, NR, 5, F_TRX>(phi, mu, u)
                             : lane_rot_grad_gate<T, NR, 5, F_TRY>(phi, mu, u);
    }
    return 0.0;
}

// phi is read from phi_src (the state, or the checkpoint of the state after
// the forward sweep this one reverses) and written to phi_g; store = 0 (the
// last reverse sweep, whose gradient shares are all that is left to form)
// writes neither phi nor mu.  Two tiles (phi
// and mu) of 2^VB amplitudes per lane: in complex64 up to 5 register qubits
// the kernel fits 3 waves per SIMD (168 registers in all), which the launch
// bound keeps (two registers more left 2 waves: 24% slower, measured).
template <typename T, int VB>
__global__ __launch_bounds__(BLOCK, (sizeof(T) == 4 && VB <= 5) ? 3 : 1) void k_regtile_adj(cplx<T> *__restrict__ phi_g, const cplx<T> *__restrict__ phi_src,
                                                       cplx<T> *__restrict__ mu_g,
                                                       const uint8_t *__restrict__ prog, uint64_t ntiles,
                                                       double *__restrict__ gpart, int nslots,
                                                       int store) {
    constexpr int NR = 1 << VB;
    // the program is read-only while the kernel runs: scalar loads through
    // the constant address space, also after the gradient stores
    const cptr<RTHeader> h = (cptr<RTHeader>)prog;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint64_t tile = (uint64_t)blockIdx.x * (BLOCK / 64) + wave;
    if (tile >= ntiles) return;
    uint64_t bq[VB];
#pragma unroll
    for (int i = 0; i < VB; i++) bq[i] = 1ull << h->rq[i];
    // the tile layout of the forward register tiles: zeros inserted at the
    // tile's qubits above 3; lane bits 4 and 5 are qubits lq[0], lq[1]
    uint64_t base = tile << 4;
#pragma unroll
    for (int i = 0; i < VB + 2; i++) base = insert_zero(base, h->tq[i]);
    const int l4 = h->lq[0], l5 = h->lq[1];
    const bool rows = (l4 == 4) & (l5 == 5);
    const uint64_t loff = (uint64_t)(lane & 15) | ((uint64_t)((lane >> 4) & 1) << l4) |
                          ((uint64_t)((lane >> 5) & 1) << l5);
    cplx<T> phi[NR], mu[NR];
    cplx<T> *const phi_in = const_cast<cplx<T> *>(phi_src);
    if (rows) {
#pragma unroll
        for (int r = 0; r < NR; r++) {
            phi[r] = gload<T>(uniform_ptr(phi_in + (base + reg_offset<VB>(bq, r))) + lane);
            mu[r] = gload<T>(uniform_ptr(mu_g + (base + reg_offset<VB>(bq, r))) + lane);
        }
    } else {
#pragma unroll
        for (int r = 0; r < NR; r++) {
            phi[r] = gload<T>(uniform_ptr(phi_in + (base + reg_offset<VB>(bq, r))) + loff);
            mu[r] = gload<T>(uniform_ptr(mu_g + (base + reg_offset<VB>(bq, r))) + loff);
        }
    }
    const cptr<RTOp> ops = (cptr<RTOp>)(prog + h->op_off);
    const cptr<DiagTerm> terms = (cptr<DiagTerm>)(prog + h->term_off);
    const int nops = h->nops;
    for (int o = 0; o < nops; o++) {
        const int kind = ops[o].kind;
        const int arg = ops[o].a;
        const int slot = ops[o].slot;
        const int form0 = ops[o].form;
        const int gk0 = ops[o].gkind;
        // (a branch condition without short-circuit jumps keeps the op
        // dispatch free of merged register flows)
        const int fused = __builtin_amdgcn_readfirstlane(
            (int)((kind == RT_LANE) & (slot >= 0) & (arg >= 4) & (NR >= 2) &
                  (((form0 == F_TRX) & (gk0 == G_RX)) | ((form0 == F_TRY) & (gk0 == G_RY)))));
        if (fused) {
            const Mat2<T> u = load_mat<T>(ops[o].u);
            double g = lane_rot_dispatch<T, NR>(phi, mu, u, arg, form0);
            g = wave_sum_d<T>(g) * ops[o].gscale;
            if (lane == 0) gpart[tile * (uint64_t)nslots + slot] = g;
        } else if (kind == RT_REG || kind == RT_LANE) {
            if (slot >= 0) {
                const Mat2<T> d = load_mat<T>(ops[o].d);
                const int gk = ops[o].gkind;
                double g = kind == RT_REG ? grad_reg_dispatch<T, NR>(phi, mu, d, arg, gk)
                                          : grad_lane_dispatch<T, NR>(phi, mu, d, arg, lane, gk);
                g = wave_sum_d<T>(g) * ops[o].gscale;
                if (lane == 0) gpart[tile * (uint64_t)nslots + slot] = g;
            }
            const Mat2<T> u = load_mat<T>(ops[o].u);
            const int form = ops[o].form;
            if (kind == RT_REG) {
                reg_gate_dispatch<T, NR>(phi, u, arg, form);
                reg_gate_dispatch<T, NR>(mu, u, arg, form);
            } else {
                lane_gate_dispatch<T, NR, false>(phi, u, arg, lane, form);
                lane_gate_dispatch<T, NR, false>(mu, u, arg, lane, form);
            }
        } else if (kind == RT_SIGNS) {
            uint64_t par = 0;
            const int nt = ops[o].nterms;
            for (int t = arg; t < arg + nt; t++) {
                const uint64_t out = terms[t].outside;
                if ((base & out) != out) continue;
                const uint32_t lm = terms[t].lanemask;
                par ^= ((uint32_t)lane & lm) == lm ? terms[t].regset : 0ull;
            }
#pragma unroll
            for (int r = 0; r < NR; r++) {
                if ((par >> r) & 1) {
                    phi[r].re = -phi[r].re; phi[r].im = -phi[r].im;
                    mu[r].re = -mu[r].re; mu[r].im = -mu[r].im;
                }
            }
        } else if (kind == RT_PHASE && slot < 0) {
            // a group of phase terms sharing one register set (no gradient):
            // the per-lane product of the matching phases, applied once
            const int nt = ops[o].nterms;
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
                    if ((rs >> r) & 1) {
                        phi[r] = cmul(f, phi[r]);
                        mu[r] = cmul(f, mu[r]);
                    }
            }
        } else if (kind == RT_PHASE) {
            const uint64_t out = terms[arg].outside;
            const bool tile_on = (base & out) == out;
            const uint32_t lm = terms[arg].lanemask;
            const uint64_t rs = (tile_on && ((uint32_t)lane & lm) == lm) ? terms[arg].regset : 0ull;
            if (slot >= 0) {
                cplx<T> dv;
                dv.re = (T)ops[o].d[6];
                dv.im = (T)ops[o].d[7];
                // Re <mu| dv |phi> over the set's registers = Re dv W with
                // W = sum conj(mu) phi, accumulated in two halves
                T wr[2] = {0, 0}, wi[2] = {0, 0};
#pragma unroll
                for (int r = 0; r < NR; r++) {
                    const bool on = (rs >> r) & 1;
                    cplx<T> pz;
                    pz.re = on ? phi[r].re : (T)0;
                    pz.im = on ? phi[r].im : (T)0;
                    acc_re_cm<1>(wr[r & 1], mu[r], pz);
                    acc_im_cm<1>(wi[r & 1], mu[r], pz);
                }
                double g = (double)dv.re * (double)(wr[0] + wr[1]) - (double)dv.im * (double)(wi[0] + wi[1]);
                g = wave_sum_d<T>(g) * ops[o].gscale;
                if (lane == 0) gpart[tile * (uint64_t)nslots + slot] = g;
            }
            cplx<T> v;
            v.re = (T)terms[arg].val[0];
            v.im = (T)terms[arg].val[1];
#pragma unroll
            for (int r = 0; r < NR; r++)
                if ((rs >> r) & 1) {
                    phi[r] = cmul(v, phi[r]);
                    mu[r] = cmul(v, mu[r]);
                }
        }
    }
    if (!store) return;
    // the cosines taken out of the tangent-form rotations
    const double fs = h->fscale;
    if (fs != 1.0) {
        const T f = (T)fs;
#pragma unroll
        for (int r = 0; r < NR; r++) {
            phi[r].re *= f; phi[r].im *= f;
            mu[r].re *= f; mu[r].im *= f;
        }
    }
    if (rows) {
#pragma unroll
        for (int r = 0; r < NR; r++) {
            gstore<T>(uniform_ptr(phi_g + (base + reg_offset<VB>(bq, r))) + lane, phi[r]);
            gstore<T>(uniform_ptr(mu_g + (base + reg_offset<VB>(bq, r))) + lane, mu[r]);
        }
    } else {
#pragma unroll
        for (int r = 0; r < NR; r++) {
            gstore<T>(uniform_ptr(phi_g + (base + reg_offset<VB>(bq, r))) + loff, phi[r]);
            gstore<T>(uniform_ptr(mu_g + (base + reg_offset<VB>(bq, r))) + loff, mu[r]);
        }
    }
}

// mu = 0, then mu_x += psi_x / (m p_x) for every sample x (repeated samples
// add identical terms, so the sum does not depend on their order); the
// samples are n-bit strings (checked on the host)
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_lambda(const cplx<T> *__restrict__ psi, cplx<T> *__restrict__ mu,
                                                  const uint64_t *__restrict__ x, int64_t m) {
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i >= m) return;
    const uint64_t xi = x[i];
    const cplx<T> a = psi[xi];
    const double p = (double)a.re * (double)a.re + (double)a.im * (double)a.im;
    const double s = 1.0 / ((double)m * p);
    atomicAdd(&mu[xi].re, (T)(s * (double)a.re));
    atomicAdd(&mu[xi].im, (T)(s * (double)a.im));
}

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_zero(cplx<T> *__restrict__ v, uint64_t N) {
    uint64_t stride = (uint64_t)gridDim.x * BLOCK;
    for (uint64_t i = (uint64_t)blockIdx.x * BLOCK + threadIdx.x; i < N; i += stride) {
        cplx<T> z;
        z.re = 0;
        z.im = 0;
        v[i] = z;
    }
}

// Gradient slot sums, two levels in a fixed order: chunk c of 64 tiles is
// summed serially per slot (threads over slots, coalesced rows), then the
// chunk partials are combined in chunk order with Neumaier's summation and
// scaled by -2.
constexpr int GCHUNK = 64;

__global__ __launch_bounds__(256) void k_grad_partial(const double *__restrict__ gpart, uint64_t ntiles,
                                                      int nslots, double *__restrict__ part) {
    const uint64_t t0 = (uint64_t)blockIdx.x * GCHUNK;
    const uint64_t t1 = t0 + GCHUNK < ntiles ? t0 + GCHUNK : ntiles;
    for (int s = threadIdx.x; s < nslots; s += blockDim.x) {
        double acc = 0;
        for (uint64_t t = t0; t < t1; t++) acc += gpart[t * (uint64_t)nslots + s];
        part[(uint64_t)blockIdx.x * nslots + s] = acc;
    }
}

// One workgroup of 64 threads per slot: 64 segments of the chunk partials
// are summed in parallel (Neumaier), then the segment sums and
// compensations are combined in segment order by the first thread.
__global__ __launch_bounds__(64) void k_grad_final(const double *__restrict__ part, uint64_t nchunks,
                                                   int nslots, double *__restrict__ out) {
    __shared__ double ss[64], cc[64];
    const int s = blockIdx.x;
    const uint64_t per = (nchunks + 63) / 64;
    const uint64_t b0 = threadIdx.x * per, b1 = b0 + per < nchunks ? b0 + per : nchunks;
    double sum = 0, c = 0;
    for (uint64_t b = b0; b < b1; b++) {
        const double x = part[b * (uint64_t)nslots + s];
        const double u = sum + x;
        if (fabs(sum) >= fabs(x)) c += (sum - u) + x;
        else c += (x - u) + sum;
        sum = u;
    }
    ss[threadIdx.x] = sum;
    cc[threadIdx.x] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        double S = 0, Cc = 0;
        for (int g = 0; g < 64; g++) {
            const double x = ss[g];
            const double u = S + x;
            if (fabs(S) >= fabs(x)) Cc += (S - u) + x;
            else Cc += (x - u) + S;
            S = u;
            Cc += cc[g];
        }
        out[s] = -2.0 * (S + Cc);
    }
}

static unsigned ggrid(uint64_t items) {
    uint64_t g = (items + BLOCK - 1) / BLOCK;
    const uint64_t cap = 256ull * 64;
    return (unsigned)(g < cap ? (g ? g : 1) : cap);
}

// Checkpoint i of a plan in the handle's checkpoint workspace.
template <typename T>
static cplx<T> *ckpt_ptr(sv_state *st, int i) {
    const size_t one = ((size_t)(1ull << st->n) * sizeof(cplx<T>) + 255) & ~(size_t)255;
    return (cplx<T> *)((uint8_t *)st->ws_ck.ptr + (size_t)i * one);
}

// The forward sweeps of an adjoint plan from |0..0>, each checkpoint written
// by the store of the sweep after which it falls.
template <typename T>
static sv_status forward_typed(sv_state *st, const Plan &plan) {
    const size_t one = ((size_t)(1ull << st->n) * sizeof(cplx<T>) + 255) & ~(size_t)255;
    if (plan.ncheckpoints) SV_TRY(st->ws_ck.reserve(one * (size_t)plan.ncheckpoints));
    for (const Op &op : plan.ops) {
        void *ck = (op.type == OP_REGTILE && op.q1 >= 0) ? (void *)ckpt_ptr<T>(st, op.q1) : nullptr;
        SV_TRY(launch_op(st, plan, op, st->data, ck));
    }
    st->known_zero = false;
    return SV_OK;
}

template <typename T>
static sv_status backward_typed(sv_state *st, const Plan &plan, const uint64_t *samples, int64_t k,
                                double *loss, double *grad, int nparams, bool state_ready) {
    const int n = st->n;
    const uint64_t N = 1ull << n;
    hipStream_t s = st->stream;
    const int nslots = (int)plan.slot_param.size();
    // device scratch: mu | samples | gradient partials | slot sums; the
    // checkpoints live in their own workspace (they outlive the forward call
    // that writes them when the state is kept for a later backward)
    int vb = 0;
    for (const Op &op : plan.bops)
        if (op.type == OP_ADJ_REGTILE) vb = op.vbits;
    const uint64_t ntiles = vb ? N >> (LANE_BITS + vb) : 0;
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t b_mu = al(N * sizeof(cplx<T>));
    const size_t b_x = al((size_t)k * 8);
    const size_t b_gp = al((size_t)ntiles * (nslots ? nslots : 1) * 8);
    const uint64_t nchunks = (ntiles + GCHUNK - 1) / GCHUNK;
    const size_t b_gs = al((size_t)(nslots ? nslots : 1) * 8 * (nchunks + 1));
    SV_TRY(st->ws2.reserve(b_mu + b_x + b_gp + b_gs));
    uint8_t *w = (uint8_t *)st->ws2.ptr;
    cplx<T> *mu = (cplx<T> *)w;
    uint64_t *dx = (uint64_t *)(w + b_mu);
    double *gpart = (double *)((uint8_t *)dx + b_x);
    double *gsum = (double *)((uint8_t *)gpart + b_gp);
    cplx<T> *phi = (cplx<T> *)st->data;

    // forward pass from |0..0> with its checkpoints (skipped when the handle
    // already holds the output state, and the checkpoints if any)
    if (!state_ready) SV_TRY(forward_typed<T>(st, plan));
    st->ck_key.clear();   // the reverse sweeps uncompute the state
    // loss and lambda
    SV_HIP(hipMemcpyAsync(dx, samples, (size_t)k * 8, hipMemcpyHostToDevice, s));
    double sum_log = 0;
    int64_t zeros = 0;
    SV_TRY(run_cross_entropy(st, phi, dx, k, 1.0, &sum_log, &zeros));
    if (zeros) return fail(SV_ESTATE, "sv_backward: a sample has probability 0");
    *loss = -sum_log / (double)k;
    hipLaunchKernelGGL(k_zero<T>, dim3(ggrid(N)), dim3(BLOCK), 0, s, mu, N);
    hipLaunchKernelGGL(k_lambda<T>, dim3((unsigned)((k + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, s, phi, mu,
                       dx, k);
    SV_HIP(hipGetLastError());
    // reverse sweeps; the reverse of a sweep that wrote a checkpoint takes
    // phi from it
    for (const Op &op : plan.bops) {
        const cplx<T> *phi_src = op.q1 >= 0 ? ckpt_ptr<T>(st, op.q1) : phi;
        const int store = &op != &plan.bops.back();   // the states after the last one are not read
        const uint8_t *prog = (const uint8_t *)plan.dprog + op.prog_off;
        const unsigned grid = (unsigned)((ntiles + 3) / 4);
#define ADJ_CASE(VB)                                                                                           \
    case VB:                                                                                                   \
        hipLaunchKernelGGL((k_regtile_adj<T, VB>), dim3(grid), dim3(BLOCK), 0, s, phi, phi_src, mu, prog, ntiles, \
                           gpart, nslots, store);                                                              \
        break;
        switch (op.vbits) {
            ADJ_CASE(1) ADJ_CASE(2) ADJ_CASE(3) ADJ_CASE(4) ADJ_CASE(5)
        default: return fail(SV_EINVAL, "adjoint tile width out of range");
        }
#undef ADJ_CASE
        SV_HIP(hipGetLastError());
    }
    std::vector<double> slots(nslots);
    if (nslots) {
        double *gchunk = gsum + nslots;
        hipLaunchKernelGGL(k_grad_partial, dim3((unsigned)nchunks), dim3(256), 0, s, gpart, ntiles, nslots,
                           gchunk);
        hipLaunchKernelGGL(k_grad_final, dim3(nslots), dim3(64), 0, s, gchunk, nchunks, nslots,
                           gsum);
        SV_HIP(hipGetLastError());
        SV_HIP(hipMemcpyAsync(slots.data(), gsum, nslots * 8, hipMemcpyDeviceToHost, s));
    }
    SV_HIP(hipStreamSynchronize(s));
    for (int i = 0; i < nparams; i++) grad[i] = 0.0;
    for (int i = 0; i < nslots; i++) grad[plan.slot_param[i]] += slots[i];
    return SV_OK;
}

// The adjoint plan of (c, opts, checkpoint_c), from the handle's cache.
static sv_status adjoint_plan(sv_state *st, const sv_circuit *c, const sv_opts *opts, int checkpoint_c,
                              std::shared_ptr<Plan> *out, std::string *key_out) {
    PlanRequest rq{};
    rq.n = st->n;
    rq.dtype = st->dt;
    rq.mode = SV_MODE_REGTILE;
    rq.tile = opts ? opts->tile_qubits : 0;
    rq.budget = opts ? opts->sweep_budget : 0;
    if (rq.budget != 0 && (rq.budget < 20 || rq.budget > 2000)) return fail(SV_EINVAL, "sweep_budget must be 0 or 20..2000");
    rq.from_zero = true;
    rq.k_max = 1000 + checkpoint_c;   // distinct cache key per checkpoint interval
    const std::string key = "adj:" + plan_key(c, rq);
    auto it = st->plans.find(key);
    if (it != st->plans.end()) {
        *out = it->second;
    } else {
        auto plan = std::make_shared<Plan>();
        SV_TRY(build_adjoint_plan(c, rq, checkpoint_c, plan.get()));
        SV_TRY(upload_plan(st, plan.get()));
        if (st->plans.size() > 64) st->plans.clear();
        st->plans[key] = plan;
        *out = plan;
    }
    *key_out = key;
    return SV_OK;
}

sv_status run_forward_checkpoints(sv_state *st, const sv_circuit *c, const sv_opts *opts) {
    const int ck = opts ? opts->checkpoint_c : 0;
    if (ck < 0) return fail(SV_EINVAL, "checkpoint interval must be >= 0");
    std::shared_ptr<Plan> plan;
    std::string key;
    SV_TRY(adjoint_plan(st, c, opts, ck, &plan, &key));
    st->ck_key.clear();
    if (st->dt == SV_C64) SV_TRY(forward_typed<float>(st, *plan));
    else SV_TRY(forward_typed<double>(st, *plan));
    st->ck_key = key;
    return SV_OK;
}

}  // namespace svi

using namespace svi;

extern "C" sv_status sv_backward(sv_state *st, const sv_circuit *c, const sv_opts *opts, const uint64_t *samples,
                                 int64_t k, int checkpoint_c, double *loss, double *grad) {
    if (!st || !st->data) return fail(SV_EINVAL, "null state");
    if (!c || c->n != st->n) return fail(SV_EINVAL, "circuit qubit count differs from the state's");
    if (k <= 0 || !samples || !loss || (c->nparams > 0 && !grad))
        return fail(SV_EINVAL, "need samples, a loss and a gradient buffer");
    if (checkpoint_c < 0) return fail(SV_EINVAL, "checkpoint interval must be >= 0");
    for (int64_t i = 0; i < k; i++)
        if (samples[i] >= (1ull << st->n)) return fail(SV_ERANGE, "sv_backward: a sample is not an n-bit string");
    const bool ready = opts && (opts->flags & SV_FLAG_STATE_READY);
    std::shared_ptr<Plan> plan;
    std::string key;
    SV_TRY(adjoint_plan(st, c, opts, checkpoint_c, &plan, &key));
    if (ready && plan->ncheckpoints > 0 && st->ck_key != key)
        return fail(SV_ESTATE, "sv_backward: the handle holds no checkpoints of this circuit and interval (run "
                               "sv_apply_circuit with SV_FLAG_CHECKPOINTS and the same options first)");
    if (st->dt == SV_C64) return backward_typed<float>(st, *plan, samples, k, loss, grad, c->nparams, ready);
    return backward_typed<double>(st, *plan, samples, k, loss, grad, c->nparams, ready);
}
