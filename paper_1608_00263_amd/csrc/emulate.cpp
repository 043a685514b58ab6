// Host replay of sweep plans (include/sv_host.h): interprets the tile
// programs byte for byte as the GPU kernels do, in double precision.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/sv_host.h"
#include "internal.h"

namespace svi {

using cx = std::complex<double>;

static uint64_t ins0(uint64_t x, int q) {
    return ((x >> q) << (q + 1)) | (x & ((1ull << q) - 1));
}

static cx to_cx(const double *u, int i) { return cx(u[2 * i], u[2 * i + 1]); }

static void emulate_regtile(const Plan &plan, const Op &op, int n, cx *psi) {
    const uint8_t *prog = plan.prog.data() + op.prog_off;
    const RTHeader *h = (const RTHeader *)prog;
    const RTOp *ops = (const RTOp *)(prog + h->op_off);
    const DiagTerm *terms = (const DiagTerm *)(prog + h->term_off);
    const int vb = op.vbits, nr = 1 << vb;
    const uint64_t ntiles = (1ull << n) >> (LANE_BITS + vb);
    std::vector<uint64_t> roff(nr, 0);
    for (int r = 1; r < nr; r++) roff[r] = roff[r & (r - 1)] | (1ull << h->rq[__builtin_ctz(r)]);
    // lane l: bits 0..3 are qubits 0..3, bits 4 and 5 qubits lq[0], lq[1]
    std::vector<uint64_t> loff(64);
    for (int l = 0; l < 64; l++)
        loff[l] = (uint64_t)(l & 15) | ((uint64_t)((l >> 4) & 1) << h->lq[0]) | ((uint64_t)((l >> 5) & 1) << h->lq[1]);
    std::vector<cx> a(64 * nr);
    const bool f32 = plan.dtype == SV_C64;
    auto rnd = [&](cx v) { return f32 ? cx((float)v.real(), (float)v.imag()) : v; };
    for (uint64_t tile = 0; tile < ntiles; tile++) {
        uint64_t base = tile << 4;
        for (int i = 0; i < vb + 2; i++) base = ins0(base, h->tq[i]);
        // generated state: 2^{-n/2} times the folded diagonal phases (the
        // product of c and the ratios of the qubits whose bit is set)
        cx gtile = 1.0;
        const RTGenPhases *gp = nullptr;
        if (h->gen_n > 0 && h->gph_off > 0) {
            gp = (const RTGenPhases *)((const uint8_t *)h + h->gph_off);
            const RTGenOut *go = (const RTGenOut *)((const uint8_t *)gp + sizeof(RTGenPhases));
            gtile = cx(gp->c[0], gp->c[1]);
            for (int k = 0; k < h->gph_nout; k++)
                if (base & go[k].mask) gtile *= cx(go[k].r[0], go[k].r[1]);
        }
        for (int l = 0; l < 64; l++)
            for (int r = 0; r < nr; r++) {
                if (h->gen_n > 0) {
                    double v = std::ldexp(1.0, -(h->gen_n / 2));
                    if (h->gen_n & 1) v /= std::sqrt(2.0);
                    cx x = v;
                    if (gp) {
                        x *= gtile;
                        for (int b = 0; b < 6; b++)
                            if ((l >> b) & 1) x *= cx(gp->lane[b][0], gp->lane[b][1]);
                        for (int sb = 0; sb < vb; sb++)
                            if ((r >> sb) & 1) x *= cx(gp->reg[sb][0], gp->reg[sb][1]);
                    }
                    a[l * nr + r] = rnd(x);
                } else {
                    a[l * nr + r] = psi[base + roff[r] + loff[l]];
                }
            }
        for (int o = 0; o < h->nops; o++) {
            const RTOp &p = ops[o];
            cx u[4];
            for (int i = 0; i < 4; i++) u[i] = rnd(to_cx(p.u, i));
            // the add-only forms are sqrt2 times the gate
            const cx I(0, 1);
            switch (p.form) {
            case F_H: u[0] = 1; u[1] = 1; u[2] = 1; u[3] = -1; break;
            case F_SX: u[0] = 1; u[1] = -I; u[2] = -I; u[3] = 1; break;
            case F_SY: u[0] = 1; u[1] = -1; u[2] = 1; u[3] = 1; break;
            case F_SXDG: u[0] = 1; u[1] = I; u[2] = I; u[3] = 1; break;
            case F_SYDG: u[0] = 1; u[1] = 1; u[2] = -1; u[3] = 1; break;
            case F_PHASE: u[0] = 1; u[1] = 0; u[2] = 0; break;
            default: break;
            }
            if (p.kind == RT_REG) {
                for (int l = 0; l < 64; l++)
                    for (int r = 0; r < nr; r++) {
                        if (r & (1 << p.a)) continue;
                        cx &x = a[l * nr + r], &y = a[l * nr + (r | (1 << p.a))];
                        cx nx = u[0] * x + u[1] * y, ny = u[2] * x + u[3] * y;
                        x = nx;
                        y = ny;
                    }
            } else if (p.kind == RT_LANE) {
                for (int l = 0; l < 64; l++) {
                    if (l & (1 << p.a)) continue;
                    int l1 = l | (1 << p.a);
                    for (int r = 0; r < nr; r++) {
                        cx &x = a[l * nr + r], &y = a[l1 * nr + r];
                        cx nx = u[0] * x + u[1] * y, ny = u[2] * x + u[3] * y;
                        x = nx;
                        y = ny;
                    }
                }
            } else if (p.kind == RT_SIGNS || p.kind == RT_PHASE) {
                int t0 = p.a, t1 = p.a + p.nterms;
                for (int l = 0; l < 64; l++) {
                    uint64_t par = 0;
                    for (int t = t0; t < t1; t++) {
                        const DiagTerm &d = terms[t];
                        if ((base & d.outside) != d.outside) continue;
                        if (((uint32_t)l & d.lanemask) != d.lanemask) continue;
                        if (p.kind == RT_SIGNS) {
                            par ^= d.regset;
                        } else {
                            cx v = rnd(cx(d.val[0], d.val[1]));
                            for (int r = 0; r < nr; r++)
                                if ((d.regset >> r) & 1) a[l * nr + r] *= v;
                        }
                    }
                    for (int r = 0; r < nr; r++)
                        if ((par >> r) & 1) a[l * nr + r] = -a[l * nr + r];
                }
            }
        }
        const double sc = std::ldexp(1.0, h->sexp) * (h->shalf ? 1.0 / std::sqrt(2.0) : 1.0) * h->fscale;
        for (int l = 0; l < 64; l++)
            for (int r = 0; r < nr; r++) psi[base + roff[r] + loff[l]] = a[l * nr + r] * sc;
    }
}

static void emulate_ldstile(const Plan &plan, const Op &op, int n, cx *psi) {
    const uint8_t *prog = plan.prog.data() + op.prog_off;
    const LTHeader *h = (const LTHeader *)prog;
    const LTOp *ops = (const LTOp *)(prog + h->op_off);
    const LTTerm *terms = (const LTTerm *)(prog + h->term_off);
    const int mb = op.vbits, nh = mb - LANE_BITS;
    const uint32_t tsz = 1u << mb;
    const uint64_t ntiles = (1ull << n) >> mb;
    std::vector<uint64_t> goff(tsz);
    for (uint32_t j = 0; j < tsz; j++) {
        uint64_t o = j & 63;
        for (int b = 0; b < nh; b++)
            if ((j >> (LANE_BITS + b)) & 1) o |= 1ull << h->hq[b];
        goff[j] = o;
    }
    std::vector<cx> lds(tsz);
    const bool f32 = plan.dtype == SV_C64;
    for (uint64_t tile = 0; tile < ntiles; tile++) {
        uint64_t base = tile << LANE_BITS;
        for (int i = 0; i < nh; i++) base = ins0(base, h->hq[i]);
        for (uint32_t j = 0; j < tsz; j++) lds[j] = psi[base + goff[j]];
        for (int o = 0; o < h->nops; o++) {
            const LTOp &p = ops[o];
            if (p.kind == LT_BLOCK) {
                const int k = p.k, d = 1 << k;
                std::vector<cx> U(d * d);
                if (p.mfma && !f32) {
                    // rebuild U from the complex128 fragments: E[row][col] in
                    // fragment (row / 16, col / 4), lane row % 16 + 16 (col % 4)
                    const double *f = (const double *)(prog + p.mat_off);
                    const int ns = d / 2;
                    auto E = [&](int row, int cl) {
                        return f[((size_t)(row / 16) * ns + cl / 4) * 64 + row % 16 + 16 * (cl % 4)];
                    };
                    for (int a = 0; a < d; a++)
                        for (int b = 0; b < d; b++) U[a * d + b] = cx(E(2 * a, 2 * b), E(2 * a + 1, 2 * b));
                } else if (p.mfma) {
                    // rebuild U from the lane-ordered real embedding
                    const float *f = (const float *)(prog + p.mat_off);
                    for (int a = 0; a < d; a++)
                        for (int b = 0; b < d; b++) {
                            const int row = 2 * a, mb = row / 32, l = row % 32;       // ra = 0
                            const double ur = f[((size_t)mb * d + b) * 64 + l];        // rb = 0: Ur
                            const double mi = f[((size_t)mb * d + b) * 64 + 32 + l];   // rb = 1: -Ui
                            U[a * d + b] = cx(ur, -mi);
                        }
                }
                for (int i = 0; i < d * d && !p.mfma; i++) {
                    if (f32) {
                        const float *f = (const float *)(prog + p.mat_off);
                        U[i] = cx(f[2 * i], f[2 * i + 1]);
                    } else {
                        const double *f = (const double *)(prog + p.mat_off);
                        U[i] = cx(f[2 * i], f[2 * i + 1]);
                    }
                }
                std::vector<uint32_t> off(d, 0);
                for (int s = 1; s < d; s++) off[s] = off[s & (s - 1)] | (1u << p.pos[__builtin_ctz(s)]);
                std::vector<cx> x(d);
                for (uint32_t c = 0; c < (tsz >> k); c++) {
                    uint32_t b = c;
                    for (int j = 0; j < k; j++) b = (uint32_t)ins0(b, p.pos[j]);
                    for (int s = 0; s < d; s++) x[s] = lds[b + off[s]];
                    for (int r = 0; r < d; r++) {
                        cx acc = 0;
                        for (int s = 0; s < d; s++) acc += U[r * d + s] * x[s];
                        lds[b + off[r]] = acc;
                    }
                }
            } else {
                for (uint32_t j = 0; j < tsz; j++) {
                    uint32_t t = j & 255, it = j >> 8;
                    for (int q = p.term0; q < p.term0 + p.nterms; q++) {
                        const LTTerm &tm = terms[q];
                        if ((base & tm.outside) != tm.outside) continue;
                        uint32_t lm = tm.localmask & 0xFFu;
                        if ((t & lm) != lm || !((tm.itset >> it) & 1)) continue;
                        if (p.kind == LT_SIGNS) lds[j] = -lds[j];
                        else {
                            cx v(tm.val[0], tm.val[1]);
                            if (f32) v = cx((float)v.real(), (float)v.imag());
                            lds[j] *= v;
                        }
                    }
                }
            }
        }
        for (uint32_t j = 0; j < tsz; j++) psi[base + goff[j]] = lds[j];
    }
}

static void emulate_op(const Plan &plan, const Op &op, int n, cx *psi) {
    const uint64_t N = 1ull << n;
    const bool f32 = plan.dtype == SV_C64;
    auto rnd = [&](cd v) { return f32 ? cx((float)v.re, (float)v.im) : cx(v.re, v.im); };
    switch (op.type) {
    case OP_INIT_UNIFORM: {
        double v = std::ldexp(1.0, -n / 2);
        if (n & 1) v /= std::sqrt(2.0);
        if (f32) v = (float)v;
        for (uint64_t i = 0; i < N; i++) psi[i] = v;
        break;
    }
    case OP_INIT_ZERO:
        for (uint64_t i = 0; i < N; i++) psi[i] = 0;
        psi[0] = 1;
        break;
    case OP_PLAIN_1Q: case OP_SPEC_DENSE: case OP_SPEC_REAL: {
        cx u[4] = {rnd(op.u.m[0]), rnd(op.u.m[1]), rnd(op.u.m[2]), rnd(op.u.m[3])};
        for (uint64_t p = 0; p < N / 2; p++) {
            uint64_t i0 = ins0(p, op.q0), i1 = i0 | (1ull << op.q0);
            cx a = psi[i0], b = psi[i1];
            psi[i0] = u[0] * a + u[1] * b;
            psi[i1] = u[2] * a + u[3] * b;
        }
        break;
    }
    case OP_PLAIN_CZ: case OP_SPEC_CZ: {
        uint64_t m = (1ull << op.q0) | (1ull << op.q1);
        for (uint64_t i = 0; i < N; i++)
            if ((i & m) == m) psi[i] = -psi[i];
        break;
    }
    case OP_SPEC_DIAG: {
        cx d = rnd(op.u.m[3]);
        for (uint64_t i = 0; i < N; i++)
            if ((i >> op.q0) & 1) psi[i] *= d;
        break;
    }
    case OP_REGTILE: emulate_regtile(plan, op, n, psi); break;
    case OP_LDSTILE: emulate_ldstile(plan, op, n, psi); break;
    default: break;   // adjoint-only ops never appear in forward plans
    }
}

static sv_status host_plan(const sv_circuit *c, sv_dtype dt, const sv_opts *o, int from_zero, Plan *plan) {
    if (!c || c->n < 1 || c->n > 35) return fail(SV_EINVAL, "bad circuit");
    if (c->ngates < 0 || (c->ngates > 0 && !c->gates)) return fail(SV_EINVAL, "bad gate array");
    PlanRequest rq{};
    rq.n = c->n;
    rq.dtype = dt;
    rq.mode = o ? o->mode : SV_MODE_AUTO;
    if (rq.mode == SV_MODE_AUTO) rq.mode = SV_MODE_REGTILE;
    rq.k_max = o ? o->k_max : 0;
    rq.tile = o ? o->tile_qubits : 0;
    rq.budget = o ? o->sweep_budget : 0;
    if (rq.budget != 0 && (rq.budget < 20 || rq.budget > 2000)) return fail(SV_EINVAL, "sweep_budget must be 0 or 20..2000");
    rq.from_zero = from_zero != 0;
    rq.force_zero = o && (o->flags & SV_FLAG_FROM_ZERO);
    rq.no_mfma = o && (o->flags & SV_FLAG_NO_MFMA);
    return build_plan(c, rq, plan);
}

}  // namespace svi

using namespace svi;

extern "C" sv_status sv_host_plan(const sv_circuit *c, sv_dtype dt, const sv_opts *opts, int from_zero,
                                  int64_t *sweeps, double *bytes, int64_t *mfma_sweeps) {
    Plan plan;
    SV_TRY(host_plan(c, dt, opts, from_zero, &plan));
    if (sweeps) *sweeps = plan.sweeps;
    if (bytes) *bytes = plan.bytes;
    if (mfma_sweeps) {
        int64_t m = 0;
        for (const Op &op : plan.ops) m += op.mfma ? 1 : 0;
        *mfma_sweeps = m;
    }
    return SV_OK;
}

extern "C" sv_status sv_host_emulate(const sv_circuit *c, sv_dtype dt, const sv_opts *opts, int from_zero,
                                     double *psi) {
    if (!psi) return fail(SV_EINVAL, "null state");
    if (c && c->n > 26) return fail(SV_ERANGE, "host replay limited to 26 qubits");
    Plan plan;
    SV_TRY(host_plan(c, dt, opts, from_zero, &plan));
    for (const Op &op : plan.ops) emulate_op(plan, op, c->n, (cx *)psi);
    return SV_OK;
}

extern "C" sv_status sv_host_cycle_emulate(const sv_circuit *c, sv_dtype dt, const sv_opts *opts, int64_t cap_rows,
                                           double *probs, int32_t *cycle_row, int64_t cap_cycles, int64_t *nrows,
                                           int64_t *ncycles) {
    if (!c || c->n < 1 || c->n > 26) return fail(SV_ERANGE, "host replay limited to 1..26 qubits");
    if (c->ngates < 0 || (c->ngates > 0 && !c->gates)) return fail(SV_EINVAL, "bad gate array");
    PlanRequest rq{};
    rq.n = c->n;
    rq.dtype = dt;
    rq.mode = opts ? opts->mode : SV_MODE_AUTO;
    rq.tile = opts ? opts->tile_qubits : 0;
    rq.budget = opts ? opts->sweep_budget : 0;
    if (rq.budget != 0 && (rq.budget < 20 || rq.budget > 2000)) return fail(SV_EINVAL, "sweep_budget must be 0 or 20..2000");
    rq.from_zero = true;
    rq.force_zero = true;
    Plan plan;
    SV_TRY(build_cycle_plan(c, rq, &plan));
    int64_t rows = 0;
    for (const Op &op : plan.ops) rows += op.type == OP_STATS;
    if (nrows) *nrows = rows;
    if (ncycles) *ncycles = (int64_t)plan.cycle_row.size();
    if (cap_rows < rows || cap_cycles < (int64_t)plan.cycle_row.size())
        return fail(SV_ERANGE, "output arrays too small for the plan's rows and cycles");
    const uint64_t N = 1ull << c->n;
    std::vector<cx> psi(N, cx(0.0, 0.0));
    for (const Op &op : plan.ops) {
        if (op.type == OP_STATS) {
            if (probs)
                for (uint64_t i = 0; i < N; i++) probs[(uint64_t)op.q0 * N + i] = std::norm(psi[i]);
            continue;
        }
        emulate_op(plan, op, c->n, psi.data());
    }
    if (cycle_row)
        for (size_t t = 0; t < plan.cycle_row.size(); t++) cycle_row[t] = plan.cycle_row[t];
    return SV_OK;
}

extern "C" sv_status sv_host_plan_describe(const sv_circuit *c, sv_dtype dt, const sv_opts *opts,
                                           int from_zero, char *buf, int64_t cap) {
    Plan plan;
    SV_TRY(host_plan(c, dt, opts, from_zero, &plan));
    std::string out;
    char line[512];
    for (size_t i = 0; i < plan.ops.size(); i++) {
        const Op &op = plan.ops[i];
        if (op.type == OP_REGTILE) {
            const RTHeader *h = (const RTHeader *)(plan.prog.data() + op.prog_off);
            const RTOp *ops = (const RTOp *)((const uint8_t *)h + h->op_off);
            int nreg = 0, nlane = 0, nsign = 0, nterm = 0, nphase = 0;
            int nform[12] = {0}, nbit[6] = {0};
            for (int o = 0; o < h->nops; o++) {
                if (ops[o].kind == RT_REG || ops[o].kind == RT_LANE) nform[std::min(11, std::max(0, (int)ops[o].form))]++;
                if (ops[o].kind == RT_REG) nreg++;
                else if (ops[o].kind == RT_LANE) { nlane++; nbit[std::min(5, std::max(0, (int)ops[o].a))]++; }
                else if (ops[o].kind == RT_SIGNS) { nsign++; nterm += ops[o].nterms; }
                else nphase++;
            }
            std::string rq;
            for (int j = 0; j < h->vbits; j++) rq += (j ? "," : "") + std::to_string(h->rq[j]);
            rq += "] lanes=[" + std::to_string(h->lq[0]) + "," + std::to_string(h->lq[1]);
            rq += "] lanebits=[";
            for (int b = 0; b < 6; b++) rq += (b ? "," : "") + std::to_string(nbit[b]);
            std::string fs;
            static const char *fname[12] = {"gen", "h", "sx", "sy", "sxdg", "sydg", "phase", "rx", "ry", "real",
                                            "trx", "try"};
            for (int f = 0; f < 12; f++)
                if (nform[f]) fs += std::string(fs.empty() ? "" : ",") + fname[f] + ":" + std::to_string(nform[f]);
            snprintf(line, sizeof line, "%zu regtile v=%d rq=[%s] reg=%d lane=%d signops=%d cz=%d phase=%d forms=[%s]\n",
                     i, h->vbits, rq.c_str(), nreg, nlane, nsign, nterm, nphase, fs.c_str());
        } else if (op.type == OP_LDSTILE) {
            const LTHeader *h = (const LTHeader *)(plan.prog.data() + op.prog_off);
            const LTOp *ops = (const LTOp *)((const uint8_t *)h + h->op_off);
            std::string ks;
            int nd = 0;
            for (int o = 0; o < h->nops; o++) {
                if (ops[o].kind == LT_BLOCK) ks += std::to_string(ops[o].k);
                else nd += ops[o].nterms;
            }
            snprintf(line, sizeof line, "%zu ldstile m=%d blocks=[%s] diagterms=%d mfma=%d\n", i, h->mbits,
                     ks.c_str(), nd, op.mfma);
        } else {
            snprintf(line, sizeof line, "%zu op%d q0=%d q1=%d\n", i, (int)op.type, op.q0, op.q1);
        }
        out += line;
    }
    if (buf && cap > 0) {
        size_t m = std::min((size_t)cap - 1, out.size());
        memcpy(buf, out.data(), m);
        buf[m] = 0;
    }
    return SV_OK;
}
