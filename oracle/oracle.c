/*
 * Plain FP64 (complex128) CPU reference for the random-circuit simulation
 * path: state evolution, output probabilities, output statistics, the
 * integer-CDF sampler, sample cross entropy and the adjoint gradient.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library
 * is checked against; it shares no code, header or table with the library
 * and must never be linked into or called from the product path.  Only the
 * test-suite, the smoke check and the CPU-baseline leg of the benchmark use
 * it.
 *
 * Everything here is deliberately plain: one sweep per gate in list order,
 * no fusion, no folding of diagonal gates, no blocking beyond what a
 * definition states.  Build with -ffp-contract=off so that no multiply-add
 * is contracted (p = re*re + im*im is two rounded products and a rounded
 * sum).
 *
 * Gate records arrive as six int32 per gate:
 *   kind, q0, q1 (-1 for single-qubit gates), cycle, param, mat
 * with the kind codes of the interchange format:
 *   0 H, 1 CZ, 2 T, 3 X^1/2, 4 Y^1/2, 5 S, 6 X, 7 Y, 8 Z,
 *   9 T^dag, 10 S^dag, 11 (X^1/2)^dag, 12 (Y^1/2)^dag, 13 dense 2x2.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct { double re, im; } cx;

static cx cx_mul(cx a, cx b) {
    cx r = { a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re };
    return r;
}
static cx cx_add(cx a, cx b) { cx r = { a.re + b.re, a.im + b.im }; return r; }
static cx cx_conj(cx a) { cx r = { a.re, -a.im }; return r; }

enum { K_H = 0, K_CZ, K_T, K_SX, K_SY, K_S, K_X, K_Y, K_Z, K_TDG, K_SDG,
       K_SXDG, K_SYDG, K_U1, K_COUNT };

#define GATE_FIELDS 6

/* ---------------------------------------------------------------------
 * Gate matrices (Sec. IV gate set).
 *
 * H is the Hadamard.  X^1/2 and Y^1/2 are pi/2 rotations about the X and Y
 * axes, taken as RX(pi/2) = exp(-i pi X / 4) and RY(pi/2) = exp(-i pi Y / 4);
 * this fixes the constant phase that the paper leaves out and is the
 * choice consistent with the diagonal/off-diagonal phase ratios of
 * Eqs. (phX) and (phY) of App. C.  T is diag(1, e^{i pi/4}) (the
 * printed "{0, e^{i pi/4}}" is read as a slip; Eq. (phT) adds the phase
 * pi/4 only when the qubit is in state 1).  Parametrised gates use
 * angle = nominal + theta: RX(a) = [[cos a/2, -i sin a/2], [-i sin a/2, cos a/2]],
 * RY(a) = [[cos a/2, -sin a/2], [sin a/2, cos a/2]], P(a) = diag(1, e^{ia}).
 * ------------------------------------------------------------------- */
static void rx(double a, cx m[4]) {
    double c = cos(0.5 * a), s = sin(0.5 * a);
    m[0] = (cx){ c, 0.0 }; m[1] = (cx){ 0.0, -s };
    m[2] = (cx){ 0.0, -s }; m[3] = (cx){ c, 0.0 };
}
static void ry(double a, cx m[4]) {
    double c = cos(0.5 * a), s = sin(0.5 * a);
    m[0] = (cx){ c, 0.0 }; m[1] = (cx){ -s, 0.0 };
    m[2] = (cx){ s, 0.0 }; m[3] = (cx){ c, 0.0 };
}
static void phase(double a, cx m[4]) {
    m[0] = (cx){ 1.0, 0.0 }; m[1] = (cx){ 0.0, 0.0 };
    m[2] = (cx){ 0.0, 0.0 }; m[3] = (cx){ cos(a), sin(a) };
}

/* Returns 0 on success, -1 for an unknown kind.  ``theta`` is the rotation
 * offset (0 for unparametrised gates); ``mat`` points at 8 doubles
 * (row-major complex 2x2) for the dense kind. */
int orc_gate_matrix(int kind, double theta, const double *mat, double out[8]) {
    cx m[4];
    const double r2 = 1.0 / sqrt(2.0);
    const double pi = M_PI;
    switch (kind) {
    case K_H:
        m[0] = (cx){ r2, 0 }; m[1] = (cx){ r2, 0 };
        m[2] = (cx){ r2, 0 }; m[3] = (cx){ -r2, 0 };
        break;
    case K_T:    phase(pi / 4 + theta, m); break;
    case K_TDG:  phase(-pi / 4 + theta, m); break;
    case K_S:    phase(pi / 2, m); break;
    case K_SDG:  phase(-pi / 2, m); break;
    case K_Z:    phase(pi, m); m[3] = (cx){ -1.0, 0.0 }; break;
    case K_SX:   rx(pi / 2 + theta, m); break;
    case K_SXDG: rx(-pi / 2 + theta, m); break;
    case K_SY:   ry(pi / 2 + theta, m); break;
    case K_SYDG: ry(-pi / 2 + theta, m); break;
    case K_X:
        m[0] = (cx){ 0, 0 }; m[1] = (cx){ 1, 0 }; m[2] = (cx){ 1, 0 }; m[3] = (cx){ 0, 0 };
        break;
    case K_Y:
        m[0] = (cx){ 0, 0 }; m[1] = (cx){ 0, -1 }; m[2] = (cx){ 0, 1 }; m[3] = (cx){ 0, 0 };
        break;
    case K_U1:
        if (!mat) return -1;
        for (int i = 0; i < 4; i++) m[i] = (cx){ mat[2 * i], mat[2 * i + 1] };
        break;
    default:
        return -1;
    }
    for (int i = 0; i < 4; i++) { out[2 * i] = m[i].re; out[2 * i + 1] = m[i].im; }
    return 0;
}

/* Derivative generator D with dU/dtheta = D U (only for the rotations). */
static int derivative_generator(int kind, cx d[4]) {
    switch (kind) {
    case K_SX: case K_SXDG:   /* -(i/2) X */
        d[0] = (cx){ 0, 0 }; d[1] = (cx){ 0, -0.5 }; d[2] = (cx){ 0, -0.5 }; d[3] = (cx){ 0, 0 };
        return 0;
    case K_SY: case K_SYDG:   /* -(i/2) Y, Y = [[0,-i],[i,0]] */
        d[0] = (cx){ 0, 0 }; d[1] = (cx){ -0.5, 0 }; d[2] = (cx){ 0.5, 0 }; d[3] = (cx){ 0, 0 };
        return 0;
    case K_T: case K_TDG:     /* i |1><1| */
        d[0] = (cx){ 0, 0 }; d[1] = (cx){ 0, 0 }; d[2] = (cx){ 0, 0 }; d[3] = (cx){ 0, 1 };
        return 0;
    default:
        return -1;
    }
}

static int gate_theta(const int32_t *g, const double *theta, int nparams, double *th) {
    int p = g[4];
    *th = 0.0;
    if (p < 0) return 0;
    if (p >= nparams || !theta) return -1;
    if (!(g[0] == K_T || g[0] == K_SX || g[0] == K_SY || g[0] == K_TDG ||
          g[0] == K_SXDG || g[0] == K_SYDG))
        return -1;
    *th = theta[p];
    return 0;
}

/* ---------------------------------------------------------------------
 * State evolution (App. B, Eq. (sqgunitaryoperation)): a single-qubit
 * gate on qubit k maps every pair of amplitudes whose indices differ only
 * in bit k; a controlled gate acts only where the control bit is set.
 * CZ multiplies by -1 exactly the amplitudes with both bits set.
 * ------------------------------------------------------------------- */
static void apply_1q(int n, cx *psi, int q, const cx u[4]) {
    const int64_t half = (int64_t)1 << (n - 1);
    const int64_t lo = ((int64_t)1 << q) - 1;
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < half; p++) {
        int64_t i0 = ((p & ~lo) << 1) | (p & lo);     /* bit q cleared */
        int64_t i1 = i0 | ((int64_t)1 << q);
        cx a0 = psi[i0], a1 = psi[i1];
        psi[i0] = cx_add(cx_mul(u[0], a0), cx_mul(u[1], a1));
        psi[i1] = cx_add(cx_mul(u[2], a0), cx_mul(u[3], a1));
    }
}

static void apply_cz(int n, cx *psi, int a, int b) {
    const int64_t N = (int64_t)1 << n;
    const int64_t m = ((int64_t)1 << a) | ((int64_t)1 << b);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; i++)
        if ((i & m) == m) { psi[i].re = -psi[i].re; psi[i].im = -psi[i].im; }
}

static int check_gate(int n, const int32_t *g, int nmats) {
    int k = g[0];
    if (k < 0 || k >= K_COUNT) return -1;
    if (g[1] < 0 || g[1] >= n) return -1;
    if (k == K_CZ) {
        if (g[2] < 0 || g[2] >= n || g[2] == g[1]) return -1;
    }
    if (k == K_U1 && (g[5] < 0 || g[5] >= nmats)) return -1;
    return 0;
}

/* Apply one gate (or its adjoint when ``dagger`` is set). */
static int apply_gate(int n, cx *psi, const int32_t *g, const double *theta,
                      int nparams, const double *mats, int nmats, int dagger) {
    if (check_gate(n, g, nmats)) return -1;
    if (g[0] == K_CZ) { apply_cz(n, psi, g[1], g[2]); return 0; }
    double th;
    if (gate_theta(g, theta, nparams, &th)) return -1;
    double m8[8];
    if (orc_gate_matrix(g[0], th, g[0] == K_U1 ? mats + 8 * g[5] : NULL, m8)) return -1;
    cx u[4];
    for (int i = 0; i < 4; i++) u[i] = (cx){ m8[2 * i], m8[2 * i + 1] };
    if (dagger) {
        cx t[4] = { cx_conj(u[0]), cx_conj(u[2]), cx_conj(u[1]), cx_conj(u[3]) };
        memcpy(u, t, sizeof t);
    }
    apply_1q(n, psi, g[1], u);
    return 0;
}

/* |0...0>: the initial state of every circuit (Sec. II, psi_0). */
void orc_init_zero(int n, double *psi) {
    const int64_t N = (int64_t)1 << n;
    memset(psi, 0, sizeof(double) * 2 * (size_t)N);
    psi[0] = 1.0;
}

/* Apply gates [first, last) of a circuit in list order, in place. */
int orc_apply_range(int n, const int32_t *gates, int64_t first, int64_t last,
                    const double *theta, int nparams, const double *mats,
                    int nmats, double *psi) {
    for (int64_t i = first; i < last; i++)
        if (apply_gate(n, (cx *)psi, gates + GATE_FIELDS * i, theta, nparams,
                       mats, nmats, 0))
            return -1 - (int)i;
    return 0;
}

int orc_apply_circuit(int n, const int32_t *gates, int64_t ngates,
                      const double *theta, int nparams, const double *mats,
                      int nmats, double *psi) {
    return orc_apply_range(n, gates, 0, ngates, theta, nparams, mats, nmats, psi);
}

/* p_j = |<x_j|psi>|^2 (Sec. II), as re*re + im*im with no contraction. */
void orc_probs(int n, const double *psi, double *p) {
    const int64_t N = (int64_t)1 << n;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; i++) {
        double re = psi[2 * i], im = psi[2 * i + 1];
        double a = re * re;
        double b = im * im;
        p[i] = a + b;
    }
}

/* Same from single-precision amplitudes (both products are exact in FP64). */
void orc_probs_c64(int n, const float *psi, double *p) {
    const int64_t N = (int64_t)1 << n;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; i++) {
        double re = (double)psi[2 * i], im = (double)psi[2 * i + 1];
        double a = re * re;
        double b = im * im;
        p[i] = a + b;
    }
}

/* ---------------------------------------------------------------------
 * Neumaier's compensated summation (Neumaier 1974).
 * ------------------------------------------------------------------- */
typedef struct { double s, c; } nsum;
static void nadd(nsum *k, double x) {
    double t = k->s + x;
    if (fabs(k->s) >= fabs(x)) k->c += (k->s - t) + x;
    else k->c += (x - t) + k->s;
    k->s = t;
}
static double nval(const nsum *k) { return k->s + k->c; }

#define CHUNK ((int64_t)1 << 20)

/*
 * Output statistics of the distribution p (Secs. II and IV):
 *   out[0]  norm S = sum_j p_j
 *   out[1]  entropy of p/S:  H = ln S - (1/S) sum_{p>0} p ln p   (0 ln 0 = 0)
 *   out[2]  cross entropy of the uniform distribution with p/S:
 *           H_unif = ln S - (1/N) sum_j ln p_j  (+inf if some p_j = 0)
 *   out[3..12]  M_k = (1/N) sum_j (N p_j / S)^k for k = 1..10, the
 *           normalised moments / inverse participation ratios N^{k-1} IPR_k
 *           that tend to k! for Porter-Thomas
 *   out[13] number of p_j equal to 0
 * Sums are Neumaier-compensated over fixed chunks of 2^20 entries that
 * are combined in chunk order, so the result does not depend on the
 * number of threads.  u^k is formed by repeated multiplication of u = N p.
 */
void orc_stats(int n, const double *p, double out[14]) {
    const int64_t N = (int64_t)1 << n;
    const double Nd = (double)N;
    const int64_t nch = (N + CHUNK - 1) / CHUNK;
    /* per chunk: S, A = sum p ln p, B = sum ln p, U[k] = sum u^k (k=1..10) */
    nsum *acc = (nsum *)calloc((size_t)nch * 13, sizeof(nsum));
    int64_t *zeros = (int64_t *)calloc((size_t)nch, sizeof(int64_t));
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t c = 0; c < nch; c++) {
        nsum *a = acc + 13 * c;
        int64_t end = (c + 1) * CHUNK < N ? (c + 1) * CHUNK : N;
        for (int64_t j = c * CHUNK; j < end; j++) {
            double pj = p[j];
            nadd(&a[0], pj);
            if (pj > 0.0) {
                double l = log(pj);
                nadd(&a[1], pj * l);
                nadd(&a[2], l);
            } else {
                zeros[c]++;
            }
            double u = Nd * pj, uk = u;
            for (int k = 1; k <= 10; k++) {
                nadd(&a[2 + k], uk);
                uk = uk * u;
            }
        }
    }
    nsum tot[13];
    memset(tot, 0, sizeof tot);
    int64_t z = 0;
    for (int64_t c = 0; c < nch; c++) {
        for (int i = 0; i < 13; i++) nadd(&tot[i], nval(&acc[13 * c + i]));
        z += zeros[c];
    }
    double S = nval(&tot[0]);
    double lnS = log(S);
    out[0] = S;
    out[1] = lnS - nval(&tot[1]) / S;
    out[2] = z ? INFINITY : lnS - nval(&tot[2]) / Nd;
    double Sk = 1.0;
    for (int k = 1; k <= 10; k++) {
        Sk *= S;
        out[2 + k] = nval(&tot[2 + k]) / Nd / Sk;
    }
    out[13] = (double)z;
    free(acc);
    free(zeros);
}

/* ---------------------------------------------------------------------
 * Sampler: inverse transform on an integer CDF, so that the answer is
 * exactly defined.  w_j = floor(p_j 2^62), C_j = w_0 + ... + w_j,
 * W = C_{N-1}; target t_i = floor(r_i W / 2^64) for a 64-bit random word
 * r_i (the multiply-high method of Lemire 2019); the sample is the
 * smallest j with C_j > t_i.  Entries with w_j = 0 are never drawn.
 * The random words are SplitMix64 outputs (Steele, Lea and Flood 2014)
 * for the counter states seed + (i+1) * 0x9E3779B97F4A7C15.
 * ------------------------------------------------------------------- */
uint64_t orc_splitmix64(uint64_t seed, uint64_t i) {
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static uint64_t weight(double p) {
    /* exact scaling by 2^62, truncation toward zero = floor for p >= 0 */
    return (uint64_t)ldexp(p, 62);
}

/* Returns 0, or -1 (no memory), -2 (a p_j negative, NaN or >= 4, whose
 * weight does not fit), -3 (every weight is 0), -4 (the total W does not
 * fit in 64 bits: the weights must sum below 2^64, i.e. sum p < 4). */
int orc_sample_from_words(uint64_t N, const double *p, const uint64_t *r,
                          int64_t k, uint64_t *out) {
    uint64_t *C = (uint64_t *)malloc(sizeof(uint64_t) * N);
    if (!C) return -1;
    uint64_t run = 0;
    for (uint64_t j = 0; j < N; j++) {
        if (!(p[j] >= 0.0) || p[j] >= 4.0) { free(C); return -2; }
        const uint64_t w = weight(p[j]);
        if (run + w < run) { free(C); return -4; }
        run += w;
        C[j] = run;
    }
    const uint64_t W = run;
    if (W == 0) { free(C); return -3; }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < k; i++) {
        uint64_t t = (uint64_t)(((unsigned __int128)r[i] * W) >> 64);
        uint64_t lo = 0, hi = N;             /* first j with C[j] > t */
        while (lo < hi) {
            uint64_t mid = lo + (hi - lo) / 2;
            if (C[mid] > t) hi = mid; else lo = mid + 1;
        }
        out[i] = lo;
    }
    free(C);
    return 0;
}

int orc_sample(uint64_t N, const double *p, uint64_t seed, int64_t k, uint64_t *out) {
    uint64_t *r = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(k > 0 ? k : 1));
    if (!r) return -1;
    for (int64_t i = 0; i < k; i++) r[i] = orc_splitmix64(seed, (uint64_t)i);
    int rc = orc_sample_from_words(N, p, r, k, out);
    free(r);
    return rc;
}

/* ---------------------------------------------------------------------
 * Sample cross entropy (Sec. II, Eqs. (ae) and (5)):
 *   CE = ln S - (1/m) sum_i ln p(x_i),  dH = ln N + gamma - CE,
 * with S = sum_j p_j (compensated as in orc_stats).  A sample with
 * p(x_i) = 0 makes CE = +inf; the number of such samples is returned.
 * A sample is an n-bit string (Sec. II): x_i >= 2^n has no probability,
 * and the call returns -1 without output.
 * ------------------------------------------------------------------- */
int64_t orc_cross_entropy(int n, const double *p, const uint64_t *x, int64_t m,
                          double *ce, double *dh) {
    const int64_t N = (int64_t)1 << n;
    for (int64_t i = 0; i < m; i++)
        if (x[i] >= (uint64_t)N) return -1;
    double st[14];
    orc_stats(n, p, st);
    nsum acc = { 0, 0 };
    int64_t zero = 0;
    for (int64_t i = 0; i < m; i++) {
        double pi = p[x[i]];
        if (pi > 0.0) nadd(&acc, log(pi)); else zero++;
    }
    const double euler_gamma = 0.57721566490153286061;
    *ce = zero ? INFINITY : log(st[0]) - nval(&acc) / (double)m;
    *dh = log((double)N) + euler_gamma - *ce;
    return zero;
}

/* ---------------------------------------------------------------------
 * Adjoint gradient of L(theta) = -(1/m) sum_i ln p_theta(x_i).
 * With psi = U_G ... U_1 |0>, lambda_x = n_x psi_x / (m p_x) and, walking
 * the gates backwards from phi = psi, mu = lambda:
 *   grad_g += -2 Re <mu| D_g |phi>   (parametrised gates, dU_g = D_g U_g)
 *   phi <- U_g^dag phi,  mu <- U_g^dag mu.
 * Inner products are compensated over fixed chunks in index order.
 * ------------------------------------------------------------------- */
static double re_inner_generator(int n, const cx *mu, const cx *phi, int q, const cx d[4]) {
    const int64_t half = (int64_t)1 << (n - 1);
    const int64_t lo = ((int64_t)1 << q) - 1;
    const int64_t nch = (half + CHUNK - 1) / CHUNK;
    nsum *acc = (nsum *)calloc((size_t)nch, sizeof(nsum));
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nch; c++) {
        int64_t end = (c + 1) * CHUNK < half ? (c + 1) * CHUNK : half;
        for (int64_t pi = c * CHUNK; pi < end; pi++) {
            int64_t i0 = ((pi & ~lo) << 1) | (pi & lo);
            int64_t i1 = i0 | ((int64_t)1 << q);
            cx d0 = cx_add(cx_mul(d[0], phi[i0]), cx_mul(d[1], phi[i1]));
            cx d1 = cx_add(cx_mul(d[2], phi[i0]), cx_mul(d[3], phi[i1]));
            nadd(&acc[c], cx_mul(cx_conj(mu[i0]), d0).re);
            nadd(&acc[c], cx_mul(cx_conj(mu[i1]), d1).re);
        }
    }
    nsum t = { 0, 0 };
    for (int64_t c = 0; c < nch; c++) nadd(&t, nval(&acc[c]));
    free(acc);
    return nval(&t);
}

int orc_adjoint(int n, const int32_t *gates, int64_t ngates, const double *theta,
                int nparams, const double *mats, int nmats, const uint64_t *x,
                int64_t m, double *loss, double *grad) {
    const int64_t N = (int64_t)1 << n;
    for (int64_t i = 0; i < m; i++)
        if (x[i] >= (uint64_t)N) return -5;   /* not an n-bit string */
    cx *phi = (cx *)malloc(sizeof(cx) * N);
    cx *mu = (cx *)calloc((size_t)N, sizeof(cx));
    if (!phi || !mu) { free(phi); free(mu); return -1; }
    orc_init_zero(n, (double *)phi);
    int rc = orc_apply_circuit(n, gates, ngates, theta, nparams, mats, nmats, (double *)phi);
    if (rc) { free(phi); free(mu); return rc; }
    nsum l = { 0, 0 };
    for (int64_t i = 0; i < m; i++) {
        int64_t xi = (int64_t)x[i];
        double re = phi[xi].re, im = phi[xi].im;
        double px = re * re + im * im;
        if (!(px > 0.0)) { free(phi); free(mu); return -2; }
        nadd(&l, log(px));
        double s = 1.0 / ((double)m * px);
        mu[xi].re += s * re;
        mu[xi].im += s * im;
    }
    *loss = -nval(&l) / (double)m;
    for (int i = 0; i < nparams; i++) grad[i] = 0.0;
    for (int64_t g = ngates - 1; g >= 0; g--) {
        const int32_t *gr = gates + GATE_FIELDS * g;
        if (gr[4] >= 0) {
            cx d[4];
            if (derivative_generator(gr[0], d) || gr[4] >= nparams) {
                free(phi); free(mu); return -3;
            }
            grad[gr[4]] += -2.0 * re_inner_generator(n, mu, phi, gr[1], d);
        }
        if (apply_gate(n, phi, gr, theta, nparams, mats, nmats, 1) ||
            apply_gate(n, mu, gr, theta, nparams, mats, nmats, 1)) {
            free(phi); free(mu); return -4;
        }
    }
    free(phi);
    free(mu);
    return 0;
}

/* ---------------------------------------------------------------------
 * Pair statistics of an ideal output a and another output b of the same
 * size (Secs. II and III: the cross entropy difference of an imperfect
 * implementation, Eq. (5), the fidelity of Eq. (ra), the residual
 * correlation of App. D).  With p_a, p_b the probabilities, S_a, S_b their
 * sums and hat p = p / S:
 *   out[0] S_a            out[1] S_b
 *   out[2] Re <a|b>       out[3] Im <a|b>
 *   out[4] fidelity |<a|b>|^2 / (S_a S_b)
 *   out[5] cross entropy H(hat p_b, hat p_a) = -sum_x hat p_b ln hat p_a
 *          (Eq. (15) with the other output as p_cl); +inf if b has mass
 *          where p_a = 0
 *   out[6] uniform cross entropy of a, -(1/N) sum ln hat p_a (+inf if some
 *          p_a = 0)
 *   out[7] Eq. (5) in its instance form sum_x (1/N - hat p_b) ln(1/hat p_a)
 *          = out[6] - out[5]; NaN if some p_a = 0
 *   out[8] Pearson correlation of p_a and p_b over the N outcomes (NaN if
 *          either is constant)
 *   out[9] number of x with p_a = 0
 *   out[10] sum of p_b over those x
 * Sums are Neumaier-compensated over fixed 2^20-element chunks combined in
 * chunk order.
 *
 * Histogram (nbins > 0): z(x) = ln(N p_a(x)) is binned over [zmin, zmax) in
 * nbins equal bins.  The decision compares p_a with the thresholds
 * t_j = e^{zmin + j dz} 2^{-n} (dz = (zmax - zmin) / nbins, j = 0..nbins):
 * bin j when t_j <= p_a < t_{j+1}; slot nbins ("under") when p_a < t_0 or
 * p_a = 0; slot nbins + 1 ("over") when p_a >= t_nbins.  Per slot s:
 *   hist[s]                  number of outcomes
 *   hist[(nbins+2) + s]      sum of floor(p_a 2^62)
 *   hist[2 (nbins+2) + s]    sum of floor(p_b 2^62)
 * (integer masses: exact and independent of summation order).  Returns 0,
 * -1 for a probability >= 4 (whose integer mass does not fit 64 bits) or
 * -2 for a memory failure.
 * ------------------------------------------------------------------- */
int orc_pair_stats(int n, const double *a, const double *b, int nbins, double zmin,
                   double zmax, double out[11], uint64_t *hist) {
    const int64_t N = (int64_t)1 << n;
    const int64_t nch = (N + CHUNK - 1) / CHUNK;
    enum { Q = 10 };   /* Sa, Sb, ov_re, ov_im, Saa, Sbb, Sab, Sbl, Sl, Sbz */
    nsum *acc = (nsum *)calloc((size_t)nch * Q, sizeof(nsum));
    int64_t *zeros = (int64_t *)calloc((size_t)nch, sizeof(int64_t));
    double *thr = (double *)malloc(sizeof(double) * (size_t)(nbins > 0 ? nbins + 1 : 1));
    if (!acc || !zeros || !thr) { free(acc); free(zeros); free(thr); return -2; }
    const double dz = nbins > 0 ? (zmax - zmin) / nbins : 0.0;
    for (int j = 0; j <= nbins && nbins > 0; j++) thr[j] = ldexp(exp(zmin + j * dz), -n);
    const int nslot = nbins + 2;
    if (nbins > 0) memset(hist, 0, sizeof(uint64_t) * 3 * (size_t)nslot);
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(|: bad)
    for (int64_t c = 0; c < nch; c++) {
        nsum *s = acc + Q * c;
        int64_t end = (c + 1) * CHUNK < N ? (c + 1) * CHUNK : N;
        for (int64_t j = c * CHUNK; j < end; j++) {
            const double ar = a[2 * j], ai = a[2 * j + 1], br = b[2 * j], bi = b[2 * j + 1];
            const double pa = ar * ar + ai * ai, pb = br * br + bi * bi;
            nadd(&s[0], pa);
            nadd(&s[1], pb);
            nadd(&s[2], ar * br + ai * bi);   /* conj(a) b */
            nadd(&s[3], ar * bi - ai * br);
            nadd(&s[4], pa * pa);
            nadd(&s[5], pb * pb);
            nadd(&s[6], pa * pb);
            if (pa > 0.0) {
                const double l = log(pa);
                nadd(&s[7], pb * l);
                nadd(&s[8], l);
            } else {
                zeros[c]++;
                nadd(&s[9], pb);
            }
            if (nbins > 0) {
                if (!(pa < 4.0) || !(pb < 4.0)) { bad = 1; continue; }
                int slot;
                if (!(pa >= thr[0])) slot = nbins;
                else if (pa >= thr[nbins]) slot = nbins + 1;
                else {
                    int lo = 0, hi = nbins;   /* last j with thr[j] <= pa */
                    while (hi - lo > 1) {
                        int mid = (lo + hi) / 2;
                        if (thr[mid] <= pa) lo = mid; else hi = mid;
                    }
                    slot = lo;
                }
                const uint64_t wa = (uint64_t)ldexp(pa, 62), wb = (uint64_t)ldexp(pb, 62);
#pragma omp atomic
                hist[slot] += 1;
#pragma omp atomic
                hist[nslot + slot] += wa;
#pragma omp atomic
                hist[2 * nslot + slot] += wb;
            }
        }
    }
    nsum t[Q];
    memset(t, 0, sizeof t);
    int64_t z = 0;
    for (int64_t c = 0; c < nch; c++) {
        for (int i = 0; i < Q; i++) nadd(&t[i], nval(&acc[Q * c + i]));
        z += zeros[c];
    }
    free(acc);
    free(zeros);
    free(thr);
    if (bad) return -1;
    const double Nd = (double)N;
    const double Sa = nval(&t[0]), Sb = nval(&t[1]);
    const double ore = nval(&t[2]), oim = nval(&t[3]);
    out[0] = Sa;
    out[1] = Sb;
    out[2] = ore;
    out[3] = oim;
    out[4] = (ore * ore + oim * oim) / (Sa * Sb);
    const double mass0 = nval(&t[9]);
    out[5] = mass0 > 0.0 ? INFINITY : log(Sa) - nval(&t[7]) / Sb;
    out[6] = z ? INFINITY : log(Sa) - nval(&t[8]) / Nd;
    out[7] = z ? NAN : out[6] - out[5];
    /* hat p = p / S:  N sum hat pa hat pb - 1 over the product of the
     * square roots of N sum hat p^2 - 1 */
    const double cab = Nd * nval(&t[6]) / (Sa * Sb) - 1.0;
    const double caa = Nd * nval(&t[4]) / (Sa * Sa) - 1.0;
    const double cbb = Nd * nval(&t[5]) / (Sb * Sb) - 1.0;
    out[8] = (caa > 0.0 && cbb > 0.0) ? cab / sqrt(caa * cbb) : NAN;
    out[9] = (double)z;
    out[10] = mass0;
    return 0;
}

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
