// Host planner: gate records -> sweeps over the state.
//
// Every sweep reads and writes the whole state once, so the planner's job
// is to apply as many gates as possible per sweep (the role cache blocking
// and gate specialisation play in App. B, "Implementation and
// Optimization"):
//  * specialisation: H and Y^1/2 are real, T/S/Z/P and CZ are diagonal;
//  * diagonal folding: a single-qubit diagonal gate commutes with every
//    other diagonal gate, so it is multiplied (in FP64) into the next dense
//    gate on its qubit, or the previous one; CZ gates stay as sign flips
//    that any sweep can apply, because every amplitude's full index is
//    known inside a tile;
//  * a leading Hadamard layer on |0..0> becomes the uniform state;
//  * register tiles: gates on qubits 0..5 (the lanes of a wavefront) and on
//    a few gathered qubits held in registers run without leaving the chip;
//  * fused blocks: runs of gates on at most k_max qubits are multiplied into
//    one dense 2^k x 2^k unitary (FP64, rounded once to the state precision);
//  * LDS tiles: several fused blocks whose qubits fit one 2^m tile share a
//    sweep.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <functional>
#include <set>
#include <sstream>

#include "internal.h"

namespace svi {

M2 m2_mul(const M2 &a, const M2 &b) {
    M2 r;
    r.m[0] = cadd(cmul(a.m[0], b.m[0]), cmul(a.m[1], b.m[2]));
    r.m[1] = cadd(cmul(a.m[0], b.m[1]), cmul(a.m[1], b.m[3]));
    r.m[2] = cadd(cmul(a.m[2], b.m[0]), cmul(a.m[3], b.m[2]));
    r.m[3] = cadd(cmul(a.m[2], b.m[1]), cmul(a.m[3], b.m[3]));
    return r;
}

M2 m2_dag(const M2 &a) {
    M2 r;
    r.m[0] = cconj(a.m[0]);
    r.m[1] = cconj(a.m[2]);
    r.m[2] = cconj(a.m[1]);
    r.m[3] = cconj(a.m[3]);
    return r;
}

static M2 mk(cd a, cd b, cd c, cd d) {
    M2 r;
    r.m[0] = a; r.m[1] = b; r.m[2] = c; r.m[3] = d;
    return r;
}

// RX(a) = exp(-i a X / 2), RY(a) = exp(-i a Y / 2), P(a) = diag(1, e^{ia})
static M2 rot_x(double a) {
    double c = std::cos(0.5 * a), s = std::sin(0.5 * a);
    return mk({c, 0}, {0, -s}, {0, -s}, {c, 0});
}
static M2 rot_y(double a) {
    double c = std::cos(0.5 * a), s = std::sin(0.5 * a);
    return mk({c, 0}, {-s, 0}, {s, 0}, {c, 0});
}
static M2 phase_gate(double a) { return mk({1, 0}, {0, 0}, {0, 0}, {std::cos(a), std::sin(a)}); }

bool gate_matrix(int kind, double th, const double *mat8, M2 *out) {
    const double pi = M_PI;
    const double r = 1.0 / std::sqrt(2.0);
    switch (kind) {
    case SV_H: *out = mk({r, 0}, {r, 0}, {r, 0}, {-r, 0}); return true;
    case SV_T: *out = phase_gate(pi / 4 + th); return true;
    case SV_TDG: *out = phase_gate(-pi / 4 + th); return true;
    case SV_S: *out = mk({1, 0}, {0, 0}, {0, 0}, {0, 1}); return true;
    case SV_SDG: *out = mk({1, 0}, {0, 0}, {0, 0}, {0, -1}); return true;
    case SV_Z: *out = mk({1, 0}, {0, 0}, {0, 0}, {-1, 0}); return true;
    case SV_X: *out = mk({0, 0}, {1, 0}, {1, 0}, {0, 0}); return true;
    case SV_Y: *out = mk({0, 0}, {0, -1}, {0, 1}, {0, 0}); return true;
    case SV_SX: *out = rot_x(pi / 2 + th); return true;
    case SV_SXDG: *out = rot_x(-pi / 2 + th); return true;
    case SV_SY: *out = rot_y(pi / 2 + th); return true;
    case SV_SYDG: *out = rot_y(-pi / 2 + th); return true;
    case SV_U1:
        if (!mat8) return false;
        for (int i = 0; i < 4; i++) out->m[i] = {mat8[2 * i], mat8[2 * i + 1]};
        return true;
    default: return false;
    }
}

bool derivative_generator(int kind, M2 *out) {
    switch (kind) {
    case SV_SX: case SV_SXDG: *out = mk({0, 0}, {0, -0.5}, {0, -0.5}, {0, 0}); return true;
    case SV_SY: case SV_SYDG: *out = mk({0, 0}, {-0.5, 0}, {0.5, 0}, {0, 0}); return true;
    case SV_T: case SV_TDG: *out = mk({0, 0}, {0, 0}, {0, 0}, {0, 1}); return true;
    default: return false;
    }
}

static bool is_diag(const M2 &u) {
    return u.m[1].re == 0 && u.m[1].im == 0 && u.m[2].re == 0 && u.m[2].im == 0;
}
static bool is_real(const M2 &u) {
    return u.m[0].im == 0 && u.m[1].im == 0 && u.m[2].im == 0 && u.m[3].im == 0;
}

double state_bytes(int n, int dtype) { return std::ldexp(dtype == SV_C64 ? 8.0 : 16.0, n); }

sv_status specialise(const sv_circuit *c, int n, std::vector<SGate> *out) {
    out->clear();
    out->reserve((size_t)c->ngates);
    int nslot = 0;
    for (int64_t i = 0; i < c->ngates; i++) {
        const sv_gate &g = c->gates[i];
        char buf[160];
        if (g.q0 < 0 || g.q0 >= n) {
            snprintf(buf, sizeof buf, "gate %lld: qubit %d out of range", (long long)i, g.q0);
            return fail(SV_EINVAL, buf);
        }
        if (g.kind == SV_CZ) {
            if (g.q1 < 0 || g.q1 >= n || g.q1 == g.q0 || g.param >= 0) {
                snprintf(buf, sizeof buf, "gate %lld: bad CZ qubits (%d, %d)", (long long)i, g.q0, g.q1);
                return fail(SV_EINVAL, buf);
            }
            SGate s{};
            s.kind = SG_CZ;
            s.q0 = std::min(g.q0, g.q1);
            s.q1 = std::max(g.q0, g.q1);
            s.src = (int)i;
            out->push_back(s);
            continue;
        }
        double th = 0;
        if (g.param >= 0) {
            bool rot = g.kind == SV_T || g.kind == SV_SX || g.kind == SV_SY || g.kind == SV_TDG ||
                       g.kind == SV_SXDG || g.kind == SV_SYDG;
            if (!rot || g.param >= c->nparams || !c->theta) {
                snprintf(buf, sizeof buf, "gate %lld: bad parameter %d for kind %d", (long long)i,
                         g.param, g.kind);
                return fail(SV_EINVAL, buf);
            }
            th = c->theta[g.param];
        }
        const double *mat = nullptr;
        if (g.kind == SV_U1) {
            if (g.mat < 0 || g.mat >= c->nmats || !c->mats) {
                snprintf(buf, sizeof buf, "gate %lld: bad matrix index %d", (long long)i, g.mat);
                return fail(SV_EINVAL, buf);
            }
            mat = c->mats + 8 * g.mat;
        }
        SGate s{};
        if (!gate_matrix(g.kind, th, mat, &s.u)) {
            snprintf(buf, sizeof buf, "gate %lld: unknown kind %d", (long long)i, g.kind);
            return fail(SV_EINVAL, buf);
        }
        s.kind = is_diag(s.u) ? SG_DIAG1 : SG_DENSE;
        s.q0 = g.q0;
        s.q1 = -1;
        s.src = (int)i;
        s.form = F_GEN;
        if (g.param < 0) {
            switch (g.kind) {
            case SV_H: s.form = F_H; break;
            case SV_SX: s.form = F_SX; break;
            case SV_SY: s.form = F_SY; break;
            case SV_SXDG: s.form = F_SXDG; break;
            case SV_SYDG: s.form = F_SYDG; break;
            default: break;
            }
        }
        if (s.form == F_GEN && s.kind == SG_DENSE) {
            // rotation structure (cos/sin forms) and real matrices
            const bool rx = g.kind == SV_SX || g.kind == SV_SXDG;
            const bool ry = g.kind == SV_SY || g.kind == SV_SYDG;
            if (rx) s.form = F_RX;
            else if (ry) s.form = F_RY;
            else if (is_real(s.u)) s.form = F_REAL;
        }
        if (s.kind == SG_DIAG1 && s.u.m[0].re == 1.0 && s.u.m[0].im == 0.0) s.form = F_PHASE;
        if (g.param >= 0) {
            s.slot = nslot++;
            derivative_generator(g.kind, &s.d);
            s.gkind = (g.kind == SV_SX || g.kind == SV_SXDG) ? G_RX
                    : (g.kind == SV_SY || g.kind == SV_SYDG) ? G_RY : G_P;
        }
        out->push_back(s);
    }
    return SV_OK;
}

void fold_diagonals(std::vector<SGate> *gl, int n, bool param_safe, bool keep_cheap) {
    std::vector<SGate> &g = *gl;
    std::vector<char> dead(g.size(), 0);
    // per qubit: indices of gates touching it, in order
    std::vector<std::vector<int>> on(n);
    for (int i = 0; i < (int)g.size(); i++) {
        on[g[i].q0].push_back(i);
        if (g[i].kind == SG_CZ) on[g[i].q1].push_back(i);
    }
    for (int q = 0; q < n; q++) {
        const std::vector<int> &v = on[q];
        for (size_t a = 0; a < v.size(); a++) {
            int i = v[a];
            if (g[i].kind != SG_DIAG1 || dead[i]) continue;
            if (param_safe && g[i].slot >= 0) continue;
            // next dense gate on q (diagonal gates in between commute); with
            // dU = D U a diagonal may be folded into a parametrised gate only
            // when it acts first
            int target = -1;
            bool before = true;
            for (size_t b = a + 1; b < v.size(); b++)
                if (g[v[b]].kind == SG_DENSE) { target = v[b]; break; }
            if (target < 0) {
                before = false;
                for (size_t b = a; b-- > 0;)
                    if (g[v[b]].kind == SG_DENSE) { target = v[b]; break; }
                if (target >= 0 && param_safe && g[target].slot >= 0) target = -1;
            }
            if (target < 0) continue;   // no dense gate on q: stays a phase
            // a gate with an add-only or rotation (tangent) form costs less
            // kept apart from the phase
            if (keep_cheap && (form_scaled(g[target].form) || g[target].form == F_RX ||
                               g[target].form == F_RY))
                continue;
            M2 d = g[i].u;
            g[target].u = before ? m2_mul(g[target].u, d) : m2_mul(d, g[target].u);
            g[target].form = is_real(g[target].u) ? F_REAL : F_GEN;
            dead[i] = 1;
        }
    }
    std::vector<SGate> out;
    out.reserve(g.size());
    for (size_t i = 0; i < g.size(); i++)
        if (!dead[i]) out.push_back(g[i]);
    g.swap(out);
}

// Leading Hadamard layer on |0..0>: the first gate on every qubit is H.
static bool strip_hadamard_layer(std::vector<SGate> *gl, int n, const sv_circuit *c) {
    std::vector<int> first(n, -1);
    for (int i = 0; i < (int)gl->size(); i++) {
        const SGate &s = (*gl)[i];
        if (first[s.q0] < 0) first[s.q0] = i;
        if (s.kind == SG_CZ && first[s.q1] < 0) first[s.q1] = i;
    }
    for (int q = 0; q < n; q++) {
        int i = first[q];
        if (i < 0) return false;
        const SGate &s = (*gl)[i];
        if (s.kind != SG_DENSE || s.q0 != q) return false;
        const sv_gate &src = c->gates[s.src];
        if (src.kind != SV_H) return false;
    }
    std::vector<char> drop(gl->size(), 0);
    for (int q = 0; q < n; q++) drop[first[q]] = 1;
    std::vector<SGate> out;
    for (size_t i = 0; i < gl->size(); i++)
        if (!drop[i]) out.push_back((*gl)[i]);
    gl->swap(out);
    return true;
}

// ---------------------------------------------------------------------------
// program buffer helpers
// ---------------------------------------------------------------------------
static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

template <typename S>
static size_t push_struct(std::vector<uint8_t> *buf, const S &s) {
    size_t off = align_up(buf->size(), 16);
    buf->resize(off + sizeof(S));
    std::memcpy(buf->data() + off, &s, sizeof(S));
    return off;
}

static size_t push_bytes(std::vector<uint8_t> *buf, const void *p, size_t bytes) {
    size_t off = align_up(buf->size(), 16);
    buf->resize(off + bytes);
    if (bytes) std::memcpy(buf->data() + off, p, bytes);
    return off;
}

// ---------------------------------------------------------------------------
// register tiles
// ---------------------------------------------------------------------------
struct Sweep {
    std::vector<int> tile;     // gathered qubits (>= LANE_BITS), ascending
    std::vector<int> items;    // indices into the gate / block list, in order
};

// Grouping of an ordered list of items into sweeps.  An item is either
// "diagonal" (applicable in any sweep) or needs all of `qubits(i)` in the
// sweep's qubit set, which holds qubits 0..nfixed-1 plus at most `cap`
// gathered ones.  Items are taken in list order; an item that cannot be taken blocks
// its qubits for the rest of the sweep (a skipped diagonal item blocks only
// non-diagonal items on its qubits, since diagonal items commute).
//
// Three groupings are built and the one with fewer sweeps kept: gathered
// sets grown greedily in list order; per sweep, the best (by items taken) of
// that greedy set and the `cap` qubits carrying the most non-diagonal items
// among the next W pending items, for a few look-ahead windows W; and a beam
// search (beam > 1) that keeps the `beam` partial groupings with the most
// items taken after each sweep, each extended by all of those candidates.
static std::vector<Sweep> group_sweeps_once(bool lookahead, int nfixed, int nitems, int n, int cap,
                                            const std::function<bool(int)> &diag,
                                            const std::function<std::vector<int>(int)> &qubits,
                                            const std::function<double(int, const std::vector<char> &)> &cost,
                                            double budget, int beam = 1) {
    std::vector<Sweep> out;
    std::vector<char> done0(nitems, 0);
    const std::vector<char> *cur = &done0;   // the items already taken
    int left = nitems;
    std::vector<std::vector<int>> qs_of(nitems);
    std::vector<char> is_diag(nitems);
    for (int i = 0; i < nitems; i++) {
        qs_of[i] = qubits(i);
        is_diag[i] = diag(i) ? 1 : 0;
    }
    std::vector<char> block_all(n), block_dense(n), in_tile(n);
    // one sweep from the current state; fixed != null: the gathered set is
    // given, else it grows greedily
    auto simulate = [&](const std::vector<char> *fixed, Sweep *sw) {
        std::fill(block_all.begin(), block_all.end(), 0);
        std::fill(block_dense.begin(), block_dense.end(), 0);
        std::fill(in_tile.begin(), in_tile.end(), 0);
        for (int q = 0; q < std::min(n, nfixed); q++) in_tile[q] = 1;
        int ngather = 0;
        if (fixed)
            for (int q = nfixed; q < n; q++)
                if ((*fixed)[q]) { in_tile[q] = 1; sw->tile.push_back(q); ngather++; }
        double spent = 0;
        for (int i = 0; i < nitems; i++) {
            if ((*cur)[i]) continue;
            const std::vector<int> &qs = qs_of[i];
            const bool d = is_diag[i];
            bool ok = true;
            for (int q : qs)
                if (block_all[q] || (!d && block_dense[q])) ok = false;
            int need = 0;
            if (ok && !d) {
                for (int q : qs)
                    if (!in_tile[q]) need++;
                if (need && (fixed || ngather + need > cap)) ok = false;
            }
            // arithmetic budget of a sweep (the first item always fits)
            if (ok && cost && !sw->items.empty()) {
                std::vector<char> t2(in_tile);
                for (int q : qs) t2[q] = 1;
                double c = cost(i, d ? in_tile : t2);
                if (spent + c > budget) ok = false;
            }
            if (ok) {
                if (cost) spent += cost(i, in_tile);
                if (!d)
                    for (int q : qs)
                        if (!in_tile[q]) { in_tile[q] = 1; sw->tile.push_back(q); ngather++; }
                sw->items.push_back(i);
            } else if (d) {
                for (int q : qs) block_dense[q] = 1;
            } else {
                for (int q : qs) block_all[q] = 1;
            }
        }
        std::sort(sw->tile.begin(), sw->tile.end());
    };
    // candidate sweeps from the current state: the greedy one and, with
    // look-ahead, one per window W
    auto candidates = [&](const std::vector<int> &windows) {
        std::vector<Sweep> cs(1);
        simulate(nullptr, &cs[0]);
        for (int W : windows) {
            std::vector<int> count(n, 0), first(n, nitems);
            int seen = 0;
            for (int i = 0; i < nitems && seen < W; i++) {
                if ((*cur)[i]) continue;
                seen++;
                if (is_diag[i]) continue;
                for (int q : qs_of[i])
                    if (q >= nfixed) {
                        count[q]++;
                        first[q] = std::min(first[q], i);
                    }
            }
            std::vector<int> cand;
            for (int q = nfixed; q < n; q++)
                if (count[q] > 0) cand.push_back(q);
            std::sort(cand.begin(), cand.end(), [&](int a, int b) {
                return count[a] != count[b] ? count[a] > count[b] : first[a] < first[b];
            });
            if ((int)cand.size() > cap) cand.resize(cap);
            std::vector<char> fixed(n, 0);
            for (int q : cand) fixed[q] = 1;
            Sweep sw;
            simulate(&fixed, &sw);
            cs.push_back(sw);
        }
        return cs;
    };
    if (beam <= 1) {
        std::vector<int> windows;
        if (lookahead) windows = {24, 48, 96, 192};
        while (left > 0) {
            std::vector<Sweep> cs = candidates(windows);
            Sweep best = cs[0];
            for (size_t c = 1; c < cs.size(); c++)
                if (cs[c].items.size() > best.items.size()) best = cs[c];
            // an item that fits no sweep (wider than the tile) would never be
            // taken: no grouping
            if (best.items.empty()) return {};
            for (int i : best.items) done0[i] = 1;
            left -= (int)best.items.size();
            out.push_back(best);
        }
        return out;
    }
    struct State {
        std::vector<char> done;
        std::vector<Sweep> sweeps;
        int left;
    };
    std::vector<State> states(1);
    states[0].done.assign(nitems, 0);
    states[0].left = nitems;
    const std::vector<int> windows = {12, 24, 36, 48, 72, 96, 144, 192, 288};
    for (;;) {
        for (const State &st : states)
            if (st.left == 0) return st.sweeps;
        std::vector<State> next;
        for (const State &st : states) {
            cur = &st.done;
            for (const Sweep &sw : candidates(windows)) {
                if (sw.items.empty()) continue;
                State c;
                c.done = st.done;
                for (int i : sw.items) c.done[i] = 1;
                bool dup = false;
                for (const State &o : next)
                    if (o.done == c.done) { dup = true; break; }
                if (dup) continue;
                c.sweeps = st.sweeps;
                c.sweeps.push_back(sw);
                c.left = st.left - (int)sw.items.size();
                next.push_back(std::move(c));
            }
        }
        if (next.empty()) return {};
        std::stable_sort(next.begin(), next.end(), [](const State &a, const State &b) { return a.left < b.left; });
        if ((int)next.size() > beam) next.resize(beam);
        states.swap(next);
    }
}

// nfixed: qubits 0..nfixed-1 are always in the sweep's set (the lanes).
static std::vector<Sweep> group_sweeps(int nitems, int n, int cap, const std::function<bool(int)> &diag,
                                       const std::function<std::vector<int>(int)> &qubits,
                                       const std::function<double(int, const std::vector<char> &)> &cost =
                                           nullptr,
                                       double budget = 0, int nfixed = LANE_BITS) {
    std::vector<Sweep> a = group_sweeps_once(false, nfixed, nitems, n, cap, diag, qubits, cost, budget);
    std::vector<Sweep> b = group_sweeps_once(true, nfixed, nitems, n, cap, diag, qubits, cost, budget);
    if (a.empty() || b.empty()) return a.empty() ? b : a;   // empty: some item fits no sweep
    std::vector<Sweep> best = b.size() < a.size() ? b : a;
    std::vector<Sweep> c = group_sweeps_once(true, nfixed, nitems, n, cap, diag, qubits, cost, budget, 6);
    if (!c.empty() && c.size() < best.size()) best = c;
    return best;
}

static uint64_t bit64(int q) { return (uint64_t)1 << q; }

struct RTProgram {
    RTHeader h{};
    std::vector<RTOp> ops;
    std::vector<DiagTerm> terms;
    std::vector<double> opc;   // cosine taken out of each op (1: none)
    bool gen_phases = false;   // diagonals folded into the generated state
    RTGenPhases gp{};
    std::vector<RTGenOut> gout;
    RTProgram() { h.fscale = 1.0; }
};

// A rotation [[c, -i s], [-i s, c]] or [[c, -s], [s, c]] applied as its
// tangent form (the matrix divided by c): two fused multiply-adds per pair
// component instead of a product and a fused multiply-add.  Taken only
// while |t| = |s / c| <= sqrt(3), so that no term grows large.
static bool tangent_form(RTOp *o, double *c_out) {
    if (o->form != F_RX && o->form != F_RY) return false;
    const double c = o->u[0];   // Re u00
    if (!(std::fabs(c) >= 0.5)) return false;
    for (int i = 0; i < 8; i++) o->u[i] /= c;
    o->form = o->form == F_RX ? F_TRX : F_TRY;
    *c_out = c;
    return true;
}

static void put_mat(double *dst, const M2 &m) {
    for (int i = 0; i < 4; i++) { dst[2 * i] = m.m[i].re; dst[2 * i + 1] = m.m[i].im; }
}

// Reorder a sweep's items so that diagonal items that commute into place
// form as few runs as possible: alternately take every ready diagonal item
// and every ready dense item, where an item is ready when no earlier
// remaining item shares a qubit with it (two diagonal items always commute).
static std::vector<int> batch_diagonals(const std::vector<SGate> &g, const std::vector<int> &items) {
    std::vector<int> rem(items), out;
    auto qubits = [&](int i, int *q) {
        q[0] = g[i].q0;
        q[1] = g[i].kind == SG_CZ ? g[i].q1 : -1;
    };
    auto diag = [&](int i) { return g[i].kind != SG_DENSE; };
    bool want_diag = true;
    int idle = 0;
    while (!rem.empty()) {
        std::vector<int> keep;
        bool took = false;
        for (size_t a = 0; a < rem.size(); a++) {
            int i = rem[a];
            bool ready = diag(i) == want_diag;
            int qi[2];
            qubits(i, qi);
            for (size_t b = 0; ready && b < a; b++) {
                int j = rem[b];
                if (j < 0) continue;   // taken in this pass
                if (diag(i) && diag(j)) continue;
                int qj[2];
                qubits(j, qj);
                for (int x = 0; x < 2; x++)
                    for (int y = 0; y < 2; y++)
                        if (qi[x] >= 0 && qi[x] == qj[y]) ready = false;
            }
            // items already moved out of rem no longer block anything
            if (ready) { out.push_back(i); took = true; rem[a] = -1; }
        }
        if (want_diag) {
            // within a diagonal batch: the CZ sign flips first (one run), then
            // the single-qubit phases
            size_t first = out.size();
            while (first > 0 && diag(out[first - 1])) first--;
            std::stable_partition(out.begin() + first, out.end(),
                                  [&](int i) { return g[i].kind == SG_CZ; });
        }
        for (int i : rem)
            if (i >= 0) keep.push_back(i);
        rem.swap(keep);
        want_diag = !want_diag;
        idle = took ? 0 : idle + 1;
        if (idle > 2) break;   // cannot happen: the first remaining item is always ready
    }
    for (int i : rem) out.push_back(i);
    return out;
}

// gen: the sweep starts from the uniform state (generated in its registers);
// single-qubit diagonals without a gradient slot that act before any dense
// gate on their qubit are then folded into the generated values.
static RTProgram build_regtile(const std::vector<SGate> &g, const Sweep &sw, int vbits, int n,
                               bool cheap = false, int *ncheap = nullptr, bool gen = false) {
    RTProgram P;
    RTHeader &h = P.h;
    h.vbits = vbits;
    // Lane bits 0..3 are qubits 0..3.  Lane bits 4 and 5 take qubits 4 and 5
    // when the sweep has them (contiguous 512-byte rows), else the gathered
    // qubits with the fewest dense gates in the sweep (cross-lane gates cost
    // more than register gates).  The other gathered qubits go to registers;
    // unused slots are filled with further qubits so that every tile covers
    // 2^(6+vbits) distinct amplitudes.
    std::vector<int> G(sw.tile.begin(), sw.tile.end());
    for (int q = 4; q < std::min(n, LANE_BITS); q++)
        if (std::find(G.begin(), G.end(), q) == G.end() && (int)G.size() < vbits + 2) G.push_back(q);
    std::vector<int> dense(64, 0);
    for (int idx : sw.items)
        if (g[idx].kind == SG_DENSE) dense[g[idx].q0]++;
    std::vector<int> lq, rq;
    for (int q : {4, 5})
        if (std::find(G.begin(), G.end(), q) != G.end()) lq.push_back(q);
    std::vector<int> rest;
    for (int q : G)
        if (std::find(lq.begin(), lq.end(), q) == lq.end()) rest.push_back(q);
    std::sort(rest.begin(), rest.end(), [&](int a, int b) { return dense[a] != dense[b] ? dense[a] < dense[b] : a < b; });
    // keep the gathered set's register share within vbits
    size_t take_lanes = rest.size() > (size_t)vbits ? rest.size() - (size_t)vbits : 0;
    for (size_t i = 0; i < rest.size(); i++) {
        if (lq.size() < 2 && (i < take_lanes || (int)(rest.size() - i) > vbits)) lq.push_back(rest[i]);
        else rq.push_back(rest[i]);
    }
    auto used = [&](int q) {
        return q < 4 || std::find(lq.begin(), lq.end(), q) != lq.end() ||
               std::find(rq.begin(), rq.end(), q) != rq.end();
    };
    for (int q = 4; lq.size() < 2 && q < n; q++)
        if (!used(q)) lq.push_back(q);
    for (int q = 4; (int)rq.size() < vbits && q < n; q++)
        if (!used(q)) rq.push_back(q);
    std::sort(lq.begin(), lq.end());
    std::sort(rq.begin(), rq.end());
    std::vector<int> slot(64, -1), lane_of(64, -1);
    for (int q = 0; q < 4; q++) lane_of[q] = q;
    lane_of[lq[0]] = 4;
    lane_of[lq[1]] = 5;
    h.lq[0] = lq[0];
    h.lq[1] = lq[1];
    std::vector<int> tq(rq);
    tq.push_back(lq[0]);
    tq.push_back(lq[1]);
    std::sort(tq.begin(), tq.end());
    for (int i = 0; i < 8; i++) {
        h.rq[i] = i < (int)rq.size() ? rq[i] : -1;
        h.tq[i] = i < (int)tq.size() ? tq[i] : -1;
    }
    for (size_t i = 0; i < rq.size(); i++) slot[rq[i]] = (int)i;
    std::vector<RTOp> &ops = P.ops;
    std::vector<DiagTerm> &terms = P.terms;
    auto term_for = [&](uint64_t mask) {
        DiagTerm t{};
        uint32_t rbits = 0;
        for (int q = 0; q < 64; q++) {
            if (!(mask & bit64(q))) continue;
            if (lane_of[q] >= 0) t.lanemask |= 1u << lane_of[q];
            else if (slot[q] >= 0) rbits |= 1u << slot[q];
            else t.outside |= bit64(q);
        }
        for (int r = 0; r < (1 << vbits); r++)
            if ((r & rbits) == rbits) t.regset |= (uint64_t)1 << r;
        return t;
    };
    int nc = 0;
    const std::vector<int> order = batch_diagonals(g, sw.items);
    std::vector<char> fold(order.size(), 0);
    if (gen) {
        // diagonals commute with each other and with CZ, so one before the
        // first dense gate on its qubit may act first, on the uniform state
        std::vector<char> dense_seen(64, 0);
        cd c0 = {1.0, 0.0};
        cd lr[6], rr[8];
        for (auto &x : lr) x = {1.0, 0.0};
        for (auto &x : rr) x = {1.0, 0.0};
        std::vector<std::pair<int, cd>> outr;
        auto mul = [](cd a, cd b) { return cd{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; };
        for (size_t k = 0; k < order.size(); k++) {
            const SGate &s = g[order[k]];
            if (s.kind == SG_DENSE) { dense_seen[s.q0] = 1; continue; }
            if (s.kind != SG_DIAG1 || s.slot >= 0 || dense_seen[s.q0]) continue;
            const cd d0 = s.u.m[0], d1 = s.u.m[3];
            const double den = d0.re * d0.re + d0.im * d0.im;
            if (den == 0.0) continue;
            const cd ratio = {(d1.re * d0.re + d1.im * d0.im) / den, (d1.im * d0.re - d1.re * d0.im) / den};
            c0 = mul(c0, d0);
            if (lane_of[s.q0] >= 0) lr[lane_of[s.q0]] = mul(lr[lane_of[s.q0]], ratio);
            else if (slot[s.q0] >= 0) rr[slot[s.q0]] = mul(rr[slot[s.q0]], ratio);
            else {
                size_t e = 0;
                while (e < outr.size() && outr[e].first != s.q0) e++;
                if (e == outr.size()) outr.push_back({s.q0, cd{1.0, 0.0}});
                outr[e].second = mul(outr[e].second, ratio);
            }
            fold[k] = 1;
            P.gen_phases = true;
        }
        if (P.gen_phases) {
            P.gp.c[0] = c0.re;
            P.gp.c[1] = c0.im;
            for (int b = 0; b < 6; b++) { P.gp.lane[b][0] = lr[b].re; P.gp.lane[b][1] = lr[b].im; }
            for (int r = 0; r < 8; r++) { P.gp.reg[r][0] = rr[r].re; P.gp.reg[r][1] = rr[r].im; }
            for (auto &e : outr) {
                RTGenOut o{};
                o.mask = bit64(e.first);
                o.r[0] = e.second.re;
                o.r[1] = e.second.im;
                P.gout.push_back(o);
            }
        }
    }
    for (size_t k = 0; k < order.size(); k++) {
        if (fold[k]) continue;
        const int idx = order[k];
        const SGate &s = g[idx];
        const bool in_tile = lane_of[s.q0] >= 0 || slot[s.q0] >= 0;
        if (s.kind == SG_DENSE || (s.kind == SG_DIAG1 && in_tile)) {
            RTOp o{};
            if (lane_of[s.q0] >= 0) { o.kind = RT_LANE; o.a = lane_of[s.q0]; }
            else { o.kind = RT_REG; o.a = slot[s.q0]; }
            put_mat(o.u, s.u);
            o.slot = s.slot;
            put_mat(o.d, s.d);
            o.form = s.form;
            o.gkind = s.gkind;
            o.gscale = 1.0;
            if (s.kind == SG_DENSE && form_scaled(s.form)) {
                if (cheap) {
                    nc++;
                } else {
                    // unscaled equivalents of the add-only forms
                    o.form = (s.form == F_SX || s.form == F_SXDG) ? F_RX
                           : (s.form == F_SY || s.form == F_SYDG) ? F_RY : F_REAL;
                }
            }
            double c = 1.0;
            if (s.kind == SG_DENSE && tangent_form(&o, &c)) h.fscale *= c;
            ops.push_back(o);
            P.opc.push_back(c);
        } else if (s.kind == SG_CZ) {
            DiagTerm t = term_for(bit64(s.q0) | bit64(s.q1));
            if (!ops.empty() && ops.back().kind == RT_SIGNS &&
                ops.back().a + ops.back().nterms == (int)terms.size()) {
                ops.back().nterms++;
            } else {
                RTOp o{};
                o.kind = RT_SIGNS;
                o.a = (int)terms.size();
                o.nterms = 1;
                o.slot = -1;
                o.gscale = 1.0;
                ops.push_back(o);
                P.opc.push_back(1.0);
            }
            terms.push_back(t);
        } else {
            // single-qubit diagonal diag(d0, d1) left unfolded: the ratio
            // d1 / d0 on amplitudes with the bit set, then d0 on all of them
            DiagTerm t = term_for(bit64(s.q0));
            cd d0 = s.u.m[0], d1 = s.u.m[3];
            double den = d0.re * d0.re + d0.im * d0.im;
            cd ratio = {(d1.re * d0.re + d1.im * d0.im) / den, (d1.im * d0.re - d1.re * d0.im) / den};
            t.val[0] = ratio.re;
            t.val[1] = ratio.im;
            RTOp o{};
            o.kind = RT_PHASE;
            o.a = (int)terms.size();
            o.nterms = 1;
            o.slot = s.slot;
            o.gkind = s.gkind;
            o.gscale = 1.0;
            put_mat(o.d, s.d);
            terms.push_back(t);
            ops.push_back(o);
            P.opc.push_back(1.0);
            if (d0.re != 1.0 || d0.im != 0.0) {
                DiagTerm all = term_for(0);
                all.val[0] = d0.re;
                all.val[1] = d0.im;
                RTOp o2{};
                o2.kind = RT_PHASE;
                o2.a = (int)terms.size();
                o2.nterms = 1;
                o2.slot = -1;
                o2.gscale = 1.0;
                terms.push_back(all);
                ops.push_back(o2);
                P.opc.push_back(1.0);
            }
        }
    }
    // Runs of consecutive phase terms without gradient slots commute: group
    // them by register set, one op per group (the kernel multiplies the
    // group's registers once by a per-lane product of the term phases).
    {
        std::vector<RTOp> nops;
        std::vector<double> nopc;
        std::vector<DiagTerm> nterms;
        for (size_t i = 0; i < ops.size();) {
            const RTOp &o = ops[i];
            if (o.kind == RT_SIGNS) {
                RTOp c = o;
                c.a = (int)nterms.size();
                for (int t = 0; t < o.nterms; t++) nterms.push_back(terms[o.a + t]);
                nops.push_back(c);
                nopc.push_back(P.opc[i]);
                i++;
                continue;
            }
            if (o.kind != RT_PHASE || o.slot >= 0) {
                RTOp c = o;
                if (o.kind == RT_PHASE) {
                    c.a = (int)nterms.size();
                    nterms.push_back(terms[o.a]);
                }
                nops.push_back(c);
                nopc.push_back(P.opc[i]);
                i++;
                continue;
            }
            size_t j = i;
            while (j < ops.size() && ops[j].kind == RT_PHASE && ops[j].slot < 0) j++;
            std::vector<char> used(j - i, 0);
            for (size_t u = i; u < j; u++) {
                if (used[u - i]) continue;
                const uint64_t rs = terms[ops[u].a].regset;
                RTOp c = ops[u];
                c.a = (int)nterms.size();
                c.nterms = 0;
                for (size_t w = u; w < j; w++)
                    if (!used[w - i] && terms[ops[w].a].regset == rs) {
                        used[w - i] = 1;
                        nterms.push_back(terms[ops[w].a]);
                        c.nterms++;
                    }
                nops.push_back(c);
                nopc.push_back(1.0);
            }
            i = j;
        }
        ops.swap(nops);
        P.opc.swap(nopc);
        terms.swap(nterms);
    }
    if (ncheap) *ncheap = nc;
    return P;
}

// Rescaling of the register-tile sweeps of a plan: the add-only forms each
// multiply the state by sqrt2; sweep i divides by 2^floor(t_i / 2) on store
// (exact), where t_i is its count plus the half power carried in, and the
// last sweep also divides by sqrt2 when one is still pending.
static void assign_scales(Plan *plan, const std::vector<std::pair<size_t, int>> &sweeps) {
    int carry = 0;
    for (size_t i = 0; i < sweeps.size(); i++) {
        RTHeader *h = reinterpret_cast<RTHeader *>(plan->prog.data() + sweeps[i].first);
        const int t = carry + sweeps[i].second;
        h->sexp = -(t / 2);
        carry = t % 2;
        h->shalf = 0;
        if (i + 1 == sweeps.size()) { h->shalf = carry; carry = 0; }
    }
}

// The adjoint of a register-tile program: ops reversed, matrices and phases
// conjugate-transposed; gradient slots and generators stay with their ops.
static RTProgram reverse_regtile(const RTProgram &F) {
    RTProgram B = F;
    std::reverse(B.ops.begin(), B.ops.end());
    std::reverse(B.opc.begin(), B.opc.end());
    // the tangent forms leave both states short of the cosines applied so
    // far in this sweep: a gradient share is scaled by their square
    double k = 1.0;
    for (size_t i = 0; i < B.ops.size(); i++) {
        RTOp &o = B.ops[i];
        o.gscale = k * k;
        if (o.kind == RT_REG || o.kind == RT_LANE) {
            M2 u;
            for (int j = 0; j < 4; j++) u.m[j] = {o.u[2 * j], o.u[2 * j + 1]};
            put_mat(o.u, m2_dag(u));
        }
        k *= B.opc[i];
    }
    for (DiagTerm &t : B.terms) t.val[1] = -t.val[1];
    return B;
}

static void push_regtile(const RTProgram &P, int n, int dtype, OpType type, std::vector<Op> *seq,
                         Plan *plan) {
    RTHeader h = P.h;
    h.nops = (int)P.ops.size();
    h.nterms = (int)P.terms.size();
    size_t hoff = push_struct(&plan->prog, h);
    size_t ooff = push_bytes(&plan->prog, P.ops.data(), P.ops.size() * sizeof(RTOp));
    size_t toff = push_bytes(&plan->prog, P.terms.data(), P.terms.size() * sizeof(DiagTerm));
    std::vector<RTOpF> fops(P.ops.size());
    for (size_t i = 0; i < P.ops.size(); i++) {
        RTOpF &f = fops[i];
        f = RTOpF{};
        f.kind = P.ops[i].kind;
        f.a = P.ops[i].a;
        f.nterms = P.ops[i].nterms;
        f.form = P.ops[i].form;
        for (int j = 0; j < 8; j++) f.u[j] = (float)P.ops[i].u[j];
    }
    size_t foff = push_bytes(&plan->prog, fops.data(), fops.size() * sizeof(RTOpF));
    size_t goff = 0;
    if (P.gen_phases) {
        goff = push_struct(&plan->prog, P.gp);
        push_bytes(&plan->prog, P.gout.data(), P.gout.size() * sizeof(RTGenOut));
    }
    RTHeader *hp = reinterpret_cast<RTHeader *>(plan->prog.data() + hoff);
    hp->op_off = (int32_t)(ooff - hoff);
    hp->term_off = (int32_t)(toff - hoff);
    hp->fop_off = (int32_t)(foff - hoff);
    hp->gph_off = P.gen_phases ? (int32_t)(goff - hoff) : 0;
    hp->gph_nout = (int32_t)P.gout.size();
    Op op;
    op.type = type;
    op.vbits = P.h.vbits;
    op.prog_off = hoff;
    op.bytes = (type == OP_ADJ_REGTILE ? 4 : 2) * state_bytes(n, dtype);
    seq->push_back(op);
}

static void emit_regtile(const std::vector<SGate> &g, const Sweep &sw, int vbits, int n, int dtype,
                         Plan *plan, std::vector<std::pair<size_t, int>> *scales, bool gen = false) {
    int nc = 0;
    RTProgram P = build_regtile(g, sw, vbits, n, true, &nc, gen);
    push_regtile(P, n, dtype, OP_REGTILE, &plan->ops, plan);
    scales->push_back({plan->ops.back().prog_off, nc});
}

// ---------------------------------------------------------------------------
// fused blocks
// ---------------------------------------------------------------------------
struct Block {
    std::vector<int> qubits;   // ascending
    std::vector<int> gates;    // indices into the specialised list, in order
    bool diag = true;
};

static std::vector<Block> fuse_blocks(const std::vector<SGate> &g, int n, int kmax) {
    std::vector<Block> blocks;
    std::vector<int> last(n, -1);
    for (int i = 0; i < (int)g.size(); i++) {
        const SGate &s = g[i];
        std::vector<int> qs = {s.q0};
        if (s.kind == SG_CZ) qs.push_back(s.q1);
        int lmin = -1;
        for (int q : qs) lmin = std::max(lmin, last[q]);
        int best = -1, best_overlap = -1;
        int lo = std::max(lmin, (int)blocks.size() - 64);
        for (int b = (int)blocks.size() - 1; b >= std::max(lo, 0); b--) {
            const Block &B = blocks[b];
            int overlap = 0, uni = (int)B.qubits.size();
            for (int q : qs) {
                if (std::find(B.qubits.begin(), B.qubits.end(), q) != B.qubits.end()) overlap++;
                else uni++;
            }
            if (uni > kmax) continue;
            if (overlap > best_overlap) { best = b; best_overlap = overlap; }
        }
        if (best < 0) {
            blocks.push_back(Block());
            best = (int)blocks.size() - 1;
        }
        Block &B = blocks[best];
        for (int q : qs)
            if (std::find(B.qubits.begin(), B.qubits.end(), q) == B.qubits.end()) B.qubits.push_back(q);
        std::sort(B.qubits.begin(), B.qubits.end());
        B.gates.push_back(i);
        if (s.kind == SG_DENSE) B.diag = false;
        for (int q : qs) last[q] = best;
    }
    return blocks;
}

// Dense 2^k x 2^k matrix of a block (row-major, complex FP64); matrix bit j
// is block qubit j.
static std::vector<cd> block_matrix(const std::vector<SGate> &g, const Block &B) {
    int k = (int)B.qubits.size();
    int d = 1 << k;
    std::vector<cd> M(d * d, cd{0, 0});
    for (int i = 0; i < d; i++) M[i * d + i] = {1, 0};
    auto pos = [&](int q) {
        return (int)(std::find(B.qubits.begin(), B.qubits.end(), q) - B.qubits.begin());
    };
    for (int gi : B.gates) {
        const SGate &s = g[gi];
        if (s.kind == SG_CZ) {
            int m = (1 << pos(s.q0)) | (1 << pos(s.q1));
            for (int r = 0; r < d; r++)
                if ((r & m) == m)
                    for (int c = 0; c < d; c++) M[r * d + c] = {-M[r * d + c].re, -M[r * d + c].im};
            continue;
        }
        int b = 1 << pos(s.q0);
        for (int c = 0; c < d; c++)
            for (int r0 = 0; r0 < d; r0++) {
                if (r0 & b) continue;
                int r1 = r0 | b;
                cd a0 = M[r0 * d + c], a1 = M[r1 * d + c];
                M[r0 * d + c] = cadd(cmul(s.u.m[0], a0), cmul(s.u.m[1], a1));
                M[r1 * d + c] = cadd(cmul(s.u.m[2], a0), cmul(s.u.m[3], a1));
            }
    }
    return M;
}

// Diagonal of an all-diagonal block as (mask, factor) terms: sign flips for
// CZ, phases for the rest.
static void diag_terms(const std::vector<SGate> &g, const Block &B,
                       std::vector<std::pair<uint64_t, cd>> *out) {
    for (int gi : B.gates) {
        const SGate &s = g[gi];
        if (s.kind == SG_CZ) {
            out->push_back({bit64(s.q0) | bit64(s.q1), cd{-1, 0}});
        } else {
            cd d0 = s.u.m[0], d1 = s.u.m[3];
            double den = d0.re * d0.re + d0.im * d0.im;
            cd ratio = {(d1.re * d0.re + d1.im * d0.im) / den, (d1.im * d0.re - d1.re * d0.im) / den};
            out->push_back({bit64(s.q0), ratio});
            if (d0.re != 1.0 || d0.im != 0.0) out->push_back({0, d0});
        }
    }
}

struct LTItem {          // an op of an LDS tile program before encoding
    int kind;            // 0 block, 1 diag
    const Block *blk;
};

static void emit_ldstile(const std::vector<SGate> &g, const std::vector<const Block *> &items,
                         const std::vector<int> &tile, int mbits, int n, int dtype, Plan *plan,
                         bool no_mfma = false) {
    LTHeader h{};
    h.mbits = mbits;
    std::vector<int> hq(tile.begin(), tile.end());
    for (int q = LANE_BITS; (int)hq.size() < mbits - LANE_BITS && q < n; q++)
        if (std::find(hq.begin(), hq.end(), q) == hq.end()) hq.push_back(q);
    std::sort(hq.begin(), hq.end());
    std::vector<int> local(64, -1);
    for (int q = 0; q < LANE_BITS; q++) local[q] = q;
    for (size_t i = 0; i < hq.size(); i++) {
        h.hq[i] = hq[i];
        local[hq[i]] = LANE_BITS + (int)i;
    }
    for (size_t i = hq.size(); i < 8; i++) h.hq[i] = -1;
    std::vector<LTOp> ops;
    std::vector<LTTerm> terms;
    std::vector<std::pair<size_t, std::vector<cd>>> mats;   // (op index, matrix)
    bool mfma = false;
    for (const Block *B : items) {
        if (B->diag) {
            std::vector<std::pair<uint64_t, cd>> dt;
            diag_terms(g, *B, &dt);
            for (auto &mt : dt) {
                LTTerm t{};
                for (int q = 0; q < 64; q++) {
                    if (!(mt.first & bit64(q))) continue;
                    if (local[q] >= 0) t.localmask |= 1u << local[q];
                    else t.outside |= bit64(q);
                }
                t.val[0] = mt.second.re;
                t.val[1] = mt.second.im;
                {
                    int per = 1 << (mbits - 8);
                    uint32_t hi = t.localmask & ~0xFFu;
                    for (int i = 0; i < per; i++)
                        if ((((uint32_t)i << 8) & hi) == hi) t.itset |= 1u << i;
                }
                bool sign = mt.second.re == -1.0 && mt.second.im == 0.0;
                int kind = sign ? LT_SIGNS : LT_PHASE;
                if (!ops.empty() && ops.back().kind == kind &&
                    ops.back().term0 + ops.back().nterms == (int)terms.size()) {
                    ops.back().nterms++;
                } else {
                    LTOp o{};
                    o.kind = kind;
                    o.term0 = (int)terms.size();
                    o.nterms = 1;
                    ops.push_back(o);
                }
                terms.push_back(t);
            }
            continue;
        }
        LTOp o{};
        o.kind = LT_BLOCK;
        o.k = (int)B->qubits.size();
        for (int j = 0; j < o.k; j++) o.pos[j] = local[B->qubits[j]];
        // matrix cores for blocks of 4 or 5 qubits in complex64 and of 5 in
        // complex128 (the FP64 matrix and vector peaks are equal on this chip:
        // measured, the 16x16 blocks ran as fast or faster on the vector ALU,
        // the 32x32 blocks twice as fast on the matrix cores), where the tile
        // holds the columns of one instruction sequence per wave (32 in
        // complex64, 16 per wave and 64 in all in complex128); the kernel
        // takes the same rule
        const bool c64 = dtype == SV_C64;
        if (o.k >= (c64 ? 4 : 5) && !no_mfma && mbits - o.k >= (c64 ? 5 : 6)) { mfma = true; o.mfma = 1; }
        mats.push_back({ops.size(), block_matrix(g, *B)});
        ops.push_back(o);
    }
    h.nops = (int)ops.size();
    size_t hoff = push_struct(&plan->prog, h);
    // matrices in the state precision; matrix-core blocks get their real
    // embedding E[2a + ra][2b + rb] (Ur on ra == rb, -Ui for (0,1), Ui for
    // (1,0)) laid out as A operands: of v_mfma_f32_32x32x2f32 in complex64
    // (for M block mb and step b, lane l holds E[l % 32 + 32 mb][2 b + l / 32]),
    // of v_mfma_f64_16x16x4f64 in complex128 (for M block mb and step s, lane
    // l holds E[l % 16 + 16 mb][4 s + l / 16])
    auto embed = [](const cd &u, int ra, int rb) { return ra == rb ? u.re : (ra == 0 ? -u.im : u.im); };
    for (auto &pm : mats) {
        size_t off;
        const LTOp &bop = ops[pm.first];
        if (bop.mfma && dtype != SV_C64) {
            const int d = 1 << bop.k, nmb = d / 8, ns = d / 2;
            std::vector<double> f((size_t)nmb * ns * 64);
            for (int mb = 0; mb < nmb; mb++)
                for (int st = 0; st < ns; st++)
                    for (int l = 0; l < 64; l++) {
                        const int row = l % 16 + 16 * mb, cl = 4 * st + l / 16;
                        const cd u = pm.second[(size_t)(row / 2) * d + cl / 2];
                        f[((size_t)mb * ns + st) * 64 + l] = embed(u, row % 2, cl % 2);
                    }
            off = push_bytes(&plan->prog, f.data(), f.size() * sizeof(double));
        } else if (bop.mfma) {
            const int d = 1 << bop.k, nmb = d / 16;
            std::vector<float> f((size_t)nmb * d * 64);
            for (int mb = 0; mb < nmb; mb++)
                for (int b = 0; b < d; b++)
                    for (int l = 0; l < 64; l++) {
                        const int row = l % 32 + 32 * mb, a = row / 2, ra = row % 2, rb = l / 32;
                        const cd u = pm.second[(size_t)a * d + b];
                        f[((size_t)mb * d + b) * 64 + l] = (float)embed(u, ra, rb);
                    }
            off = push_bytes(&plan->prog, f.data(), f.size() * sizeof(float));
        } else if (dtype == SV_C64) {
            std::vector<float> f(pm.second.size() * 2);
            for (size_t i = 0; i < pm.second.size(); i++) {
                f[2 * i] = (float)pm.second[i].re;
                f[2 * i + 1] = (float)pm.second[i].im;
            }
            off = push_bytes(&plan->prog, f.data(), f.size() * sizeof(float));
        } else {
            off = push_bytes(&plan->prog, pm.second.data(), pm.second.size() * sizeof(cd));
        }
        ops[pm.first].mat_off = (int32_t)(off - hoff);
    }
    size_t ooff = push_bytes(&plan->prog, ops.data(), ops.size() * sizeof(LTOp));
    size_t toff = push_bytes(&plan->prog, terms.data(), terms.size() * sizeof(LTTerm));
    LTHeader *hp = reinterpret_cast<LTHeader *>(plan->prog.data() + hoff);
    hp->op_off = (int32_t)(ooff - hoff);
    hp->term_off = (int32_t)(toff - hoff);
    Op op;
    op.type = OP_LDSTILE;
    op.vbits = mbits;
    op.prog_off = hoff;
    op.mfma = mfma;
    op.q1 = 0;   // widest block (selects the kernel variant)
    op.q0 = 1;   // 1: every block of 4 or 5 qubits runs on the matrix cores
    for (const LTOp &o : ops)
        if (o.kind == LT_BLOCK) {
            op.q1 = std::max(op.q1, o.k);
            if (o.k >= 4 && !o.mfma) op.q0 = 0;
        }
    op.bytes = 2 * state_bytes(n, dtype);
    plan->ops.push_back(op);
}

// ---------------------------------------------------------------------------
// per-gate plans
// ---------------------------------------------------------------------------
static double diag_bytes(int n, int dtype, int q) {
    int line_bits = dtype == SV_C64 ? 4 : 3;   // 128-byte lines
    double S = state_bytes(n, dtype);
    return q >= line_bits ? S : 2 * S;
}

static double cz_bytes(int n, int dtype, int a, int b) {
    int line_bits = dtype == SV_C64 ? 4 : 3;
    double S = state_bytes(n, dtype);
    int hi = (a >= line_bits) + (b >= line_bits);
    return hi == 2 ? S / 2 : hi == 1 ? S : 2 * S;
}

static void plan_per_gate(const sv_circuit *c, const std::vector<SGate> &g, const PlanRequest &rq,
                          Plan *plan) {
    double S = state_bytes(rq.n, rq.dtype);
    for (const SGate &s : g) {
        Op op;
        op.q0 = s.q0;
        op.q1 = s.q1;
        op.u = s.u;
        if (rq.mode == SV_MODE_PLAIN) {
            if (s.kind == SG_CZ) { op.type = OP_PLAIN_CZ; op.bytes = S; }
            else { op.type = OP_PLAIN_1Q; op.bytes = 2 * S; }
        } else if (s.kind == SG_CZ) {
            op.type = OP_SPEC_CZ;
            op.bytes = cz_bytes(rq.n, rq.dtype, s.q0, s.q1);
        } else if (s.kind == SG_DIAG1) {
            op.type = OP_SPEC_DIAG;
            if (s.u.m[0].re != 1.0 || s.u.m[0].im != 0.0) {
                // general diagonal: handled by the dense kernel
                op.type = OP_SPEC_DENSE;
                op.bytes = 2 * S;
            } else {
                op.bytes = diag_bytes(rq.n, rq.dtype, s.q0);
            }
        } else {
            op.type = is_real(s.u) ? OP_SPEC_REAL : OP_SPEC_DENSE;
            op.bytes = 2 * S;
        }
        plan->ops.push_back(op);
    }
    (void)c;
}

// Register-tile grouping with an arithmetic budget per sweep.  Costs are
// vector instructions per amplitude register of a lane: add-only and
// rotation (tangent) forms 2 on a register qubit and 5 on a lane qubit
// (cross-lane moves), general 2x2 gates 8 and 11, phases 2 (register) or 4,
// and 1 per CZ sign flip.  A complex64 sweep's memory time covers about 110
// of them; the default budget of 250 lets sweeps grow beyond that (partly
// bound by the vector ALU) because fewer, heavier sweeps finish the circuit
// sooner (measured on the 30-qubit depth-40 circuit: 13 sweeps in 50 ms at
// 250 against 16 in 58 ms at 110).  Complex128: 220.
// flex: lane bits 4 and 5 may take any qubit (the sweep gathers vb + 2
// qubits above 3) instead of qubits 4 and 5.
static std::vector<Sweep> regtile_sweeps(const std::vector<SGate> &g, int n, int vb, int dtype,
                                         double budget = -1, bool flex = false) {
    if (budget < 0) budget = dtype == SV_C64 ? 250.0 : 220.0;
    const int nfixed = flex ? 4 : LANE_BITS;
    auto cost = [&](int i, const std::vector<char> &in_tile) -> double {
        const SGate &s = g[i];
        if (s.kind == SG_CZ) return 1.0;
        const bool lane = s.q0 < nfixed;
        const bool reg = !lane && in_tile[s.q0];
        if (s.kind == SG_DIAG1) return reg ? 2.0 : 4.0;
        if (form_scaled(s.form) || s.form == F_RX || s.form == F_RY) return lane ? 5.0 : 2.0;
        if (s.form == F_GEN) return lane ? 11.0 : 8.0;
        return lane ? 7.0 : 4.0;   // real forms
    };
    return group_sweeps(
        (int)g.size(), n, vb + (LANE_BITS - nfixed), [&](int i) { return g[i].kind != SG_DENSE; },
        [&](int i) {
            std::vector<int> q = {g[i].q0};
            if (g[i].kind == SG_CZ) q.push_back(g[i].q1);
            return q;
        },
        cost, budget, nfixed);
}

std::string plan_key(const sv_circuit *c, const PlanRequest &rq) {
    // FNV-1a over the request, gate records, parameters and matrices
    uint64_t h = 1469598103934665603ULL;
    auto mix = [&](const void *p, size_t bytes) {
        const uint8_t *b = (const uint8_t *)p;
        for (size_t i = 0; i < bytes; i++) { h ^= b[i]; h *= 1099511628211ULL; }
    };
    mix(&rq, sizeof rq);
    mix(&c->ngates, sizeof c->ngates);
    mix(c->gates, sizeof(sv_gate) * (size_t)c->ngates);
    if (c->nparams && c->theta) mix(c->theta, sizeof(double) * c->nparams);
    if (c->nmats && c->mats) mix(c->mats, sizeof(double) * 8 * c->nmats);
    std::ostringstream os;
    os << std::hex << h << ":" << c->ngates;
    return os.str();
}

Plan::~Plan() {
    if (dprog) (void)hipFree(dprog);
}

sv_status build_plan(const sv_circuit *c, const PlanRequest &rq, Plan *plan) {
    std::vector<SGate> g;
    SV_TRY(specialise(c, rq.n, &g));
    plan->n = rq.n;
    plan->dtype = rq.dtype;
    int mode = rq.mode;
    // tile kernels need the 64 lanes of a wavefront plus gathered qubits
    if ((mode == SV_MODE_REGTILE || mode == SV_MODE_FUSED || mode == SV_MODE_TILED) && rq.n < 10)
        mode = SV_MODE_SPEC;
    if (mode != SV_MODE_PLAIN && (rq.from_zero || rq.force_zero) &&
        strip_hadamard_layer(&g, rq.n, c)) {
        Op op;
        op.type = OP_INIT_UNIFORM;
        op.bytes = state_bytes(rq.n, rq.dtype);
        plan->ops.push_back(op);
    } else if (rq.force_zero) {
        Op op;
        op.type = OP_INIT_ZERO;
        op.bytes = state_bytes(rq.n, rq.dtype);
        plan->ops.push_back(op);
    }
    if (mode == SV_MODE_PLAIN || mode == SV_MODE_SPEC) {
        PlanRequest r2 = rq;
        r2.mode = mode;
        plan_per_gate(c, g, r2, plan);
    } else if (mode == SV_MODE_REGTILE) {
        fold_diagonals(&g, rq.n, false, true);
        int vb = rq.tile > 0 ? rq.tile : (rq.dtype == SV_C64 ? 6 : 5);
        vb = std::max(1, std::min(vb, rq.dtype == SV_C64 ? 6 : 5));
        vb = std::min(vb, rq.n - LANE_BITS);
        auto sweeps = regtile_sweeps(g, rq.n, vb, rq.dtype, rq.budget > 0 ? (double)rq.budget : -1.0, true);
        std::vector<std::pair<size_t, int>> scales;
        // the uniform initialisation is generated inside the first sweep's
        // registers instead of being written and read back (with the
        // diagonals that act on it folded into the generated values)
        const bool gen = plan->ops.size() == 1 && plan->ops[0].type == OP_INIT_UNIFORM && !sweeps.empty();
        for (size_t i = 0; i < sweeps.size(); i++)
            emit_regtile(g, sweeps[i], vb, rq.n, rq.dtype, plan, &scales, gen && i == 0);
        assign_scales(plan, scales);
        if (plan->ops.size() >= 2 && plan->ops[0].type == OP_INIT_UNIFORM &&
            plan->ops[1].type == OP_REGTILE) {
            RTHeader *h = reinterpret_cast<RTHeader *>(plan->prog.data() + plan->ops[1].prog_off);
            h->gen_n = rq.n;
            plan->ops[1].bytes = state_bytes(rq.n, rq.dtype);
            plan->ops.erase(plan->ops.begin());
        }
    } else {
        fold_diagonals(&g, rq.n);
        int kmax = rq.k_max > 0 ? std::min(rq.k_max, 5) : 4;
        int mmax = rq.dtype == SV_C64 ? 13 : 12;
        // LDS tiles of m qubits gather m - 6 qubits above the lanes: a block
        // may not be wider than that
        int m_tiled = rq.tile > 0 ? rq.tile : (rq.dtype == SV_C64 ? 12 : 11);
        m_tiled = std::min(std::max(8, std::min(m_tiled, mmax)), rq.n);
        if (mode != SV_MODE_FUSED) kmax = std::max(1, std::min(kmax, m_tiled - LANE_BITS));
        std::vector<Block> blocks = fuse_blocks(g, rq.n, kmax);
        if (mode == SV_MODE_FUSED) {
            // one sweep per dense block; diagonal blocks ride along with the
            // next dense block (or the previous one at the end)
            std::vector<const Block *> pending;
            std::vector<std::vector<const Block *>> groups;
            for (const Block &B : blocks) {
                pending.push_back(&B);
                if (!B.diag) { groups.push_back(pending); pending.clear(); }
            }
            if (!pending.empty()) {
                if (groups.empty()) groups.push_back(pending);
                else groups.back().insert(groups.back().end(), pending.begin(), pending.end());
            }
            for (auto &grp : groups) {
                std::vector<int> tile;
                for (const Block *B : grp)
                    if (!B->diag)
                        for (int q : B->qubits)
                            if (q >= LANE_BITS) tile.push_back(q);
                // tiles of at least 2^12 (2^11 in complex128) amplitudes for
                // blocks of 4 or more qubits (matrix-core fragments), 2^10 for
                // narrower blocks (more workgroups in flight per CU)
                int kw = 0;
                for (const Block *B : grp) kw = std::max(kw, (int)B->qubits.size());
                const int mmin = kw >= 4 ? (rq.dtype == SV_C64 ? 12 : 11) : 10;
                int m = std::max(LANE_BITS + (int)tile.size(), std::min(mmin, rq.n));
                m = std::min(m, rq.n);
                emit_ldstile(g, grp, tile, m, rq.n, rq.dtype, plan, rq.no_mfma);
            }
        } else {
            const int m = m_tiled;
            int cap = m - LANE_BITS;
            auto sweeps = group_sweeps(
                (int)blocks.size(), rq.n, cap, [&](int i) { return blocks[i].diag; },
                [&](int i) { return blocks[i].qubits; });
            if (sweeps.empty() && !blocks.empty()) return fail(SV_EINVAL, "a fused block is wider than the LDS tile");
            for (const Sweep &sw : sweeps) {
                std::vector<const Block *> items;
                for (int i : sw.items) items.push_back(&blocks[i]);
                emit_ldstile(g, items, sw.tile, m, rq.n, rq.dtype, plan, rq.no_mfma);
            }
        }
    }
    plan->sweeps = 0;
    plan->bytes = 0;
    for (const Op &op : plan->ops) {
        plan->sweeps++;
        plan->bytes += op.bytes;
    }
    return SV_OK;
}

sv_status build_cycle_plan(const sv_circuit *c, const PlanRequest &rq, Plan *plan) {
    for (int64_t i = 1; i < c->ngates; i++)
        if (c->gates[i].cycle < c->gates[i - 1].cycle)
            return fail(SV_EINVAL, "per-cycle statistics: gate cycles must be nondecreasing");
    for (int64_t i = 0; i < c->ngates; i++)
        if (c->gates[i].cycle < 0) return fail(SV_EINVAL, "per-cycle statistics: negative cycle");
    int mode = rq.mode == SV_MODE_AUTO ? SV_MODE_REGTILE : rq.mode;
    if (mode != SV_MODE_REGTILE && mode != SV_MODE_SPEC && mode != SV_MODE_PLAIN)
        return fail(SV_EINVAL, "per-cycle statistics run register tiles or per-gate sweeps");
    if (mode == SV_MODE_REGTILE && rq.n < 10) mode = SV_MODE_SPEC;
    std::vector<SGate> g;
    SV_TRY(specialise(c, rq.n, &g));
    plan->n = rq.n;
    plan->dtype = rq.dtype;
    const int D = c->ngates ? c->gates[c->ngates - 1].cycle : 0;
    {
        Op op;
        op.bytes = state_bytes(rq.n, rq.dtype);
        op.type = (mode != SV_MODE_PLAIN && strip_hadamard_layer(&g, rq.n, c)) ? OP_INIT_UNIFORM : OP_INIT_ZERO;
        plan->ops.push_back(op);
    }
    if (mode == SV_MODE_REGTILE) fold_diagonals(&g, rq.n, false, true);
    // items per cycle (after folding, a dense gate keeps its own cycle)
    std::vector<std::vector<SGate>> per(D + 1);
    for (const SGate &s : g) per[c->gates[s.src].cycle].push_back(s);
    // segments: a cycle with a dense gate closes one (with the diagonal
    // items pending from the diagonal-only cycles before it); trailing
    // diagonal items join the last segment, so the final state is the
    // circuit's output
    struct Seg { std::vector<SGate> items; int cycle; };
    std::vector<Seg> segs;
    std::vector<SGate> pending;
    for (int t = 0; t <= D; t++) {
        pending.insert(pending.end(), per[t].begin(), per[t].end());
        bool dense = false;
        for (const SGate &s : pending) dense |= s.kind == SG_DENSE;
        if (dense) {
            segs.push_back({pending, t});
            pending.clear();
        }
    }
    if (!pending.empty()) {
        if (segs.empty()) segs.push_back({pending, 0});
        else segs.back().items.insert(segs.back().items.end(), pending.begin(), pending.end());
    }
    // rows: the initial state (unless a segment closes at cycle 0), then one
    // per segment; cycle t reports the row of the last segment closing at or
    // before t
    int nrows = 0;
    std::vector<int> row_at(D + 1, -1);
    auto stats = [&](int first_cycle) {
        Op op;
        op.type = OP_STATS;
        op.q0 = nrows;
        op.bytes = state_bytes(rq.n, rq.dtype);
        plan->ops.push_back(op);
        row_at[first_cycle] = nrows++;
    };
    if (segs.empty() || segs[0].cycle > 0) stats(0);
    for (const Seg &sg : segs) {
        if (mode == SV_MODE_REGTILE) {
            int vb = rq.tile > 0 ? rq.tile : (rq.dtype == SV_C64 ? 6 : 5);
            vb = std::max(1, std::min(vb, rq.dtype == SV_C64 ? 6 : 5));
            vb = std::min(vb, rq.n - LANE_BITS);
            auto sweeps = regtile_sweeps(sg.items, rq.n, vb, rq.dtype, rq.budget > 0 ? (double)rq.budget : -1.0, true);
            std::vector<std::pair<size_t, int>> scales;
            for (const Sweep &sw : sweeps) emit_regtile(sg.items, sw, vb, rq.n, rq.dtype, plan, &scales);
            // the sqrt2 powers of the add-only forms are settled within the
            // segment, so every statistics point sees the true norm
            assign_scales(plan, scales);
        } else {
            PlanRequest r2 = rq;
            r2.mode = mode;
            plan_per_gate(c, sg.items, r2, plan);
        }
        stats(sg.cycle);
    }
    plan->cycle_row.assign(D + 1, 0);
    int cur = 0;
    for (int t = 0; t <= D; t++) {
        if (row_at[t] >= 0) cur = row_at[t];
        plan->cycle_row[t] = cur;
    }
    plan->sweeps = 0;
    plan->bytes = 0;
    for (const Op &op : plan->ops) {
        plan->sweeps++;
        plan->bytes += op.bytes;
    }
    return SV_OK;
}

sv_status build_adjoint_plan(const sv_circuit *c, const PlanRequest &rq, int checkpoint_c, Plan *plan) {
    std::vector<SGate> g;
    SV_TRY(specialise(c, rq.n, &g));
    if (rq.n < 8) return fail(SV_ERANGE, "sv_backward needs n >= 8");
    plan->n = rq.n;
    plan->dtype = rq.dtype;
    for (const SGate &s : g)
        if (s.slot >= 0) plan->slot_param.push_back(c->gates[s.src].param);
    for (int64_t i = 1; i < c->ngates; i++)
        if (c->gates[i].cycle < c->gates[i - 1].cycle)
            return fail(SV_EINVAL, "sv_backward: gate cycles must be nondecreasing");
    if (strip_hadamard_layer(&g, rq.n, c)) {
        Op op;
        op.type = OP_INIT_UNIFORM;
        op.bytes = state_bytes(rq.n, rq.dtype);
        plan->ops.push_back(op);
    } else {
        return fail(SV_EINVAL, "sv_backward: the circuit must open with a Hadamard on every qubit");
    }
    fold_diagonals(&g, rq.n, true);
    int vb = rq.tile > 0 ? rq.tile : (rq.dtype == SV_C64 ? 5 : 3);
    vb = std::max(1, std::min(vb, rq.dtype == SV_C64 ? 5 : 4));
    vb = std::max(1, std::min(vb, rq.n - LANE_BITS - 2));
    // One grouping of the whole circuit: the same budget as the forward
    // sweeps (the reverse sweeps are VALU-bound too, and fewer of them finish
    // sooner: complex64, 5x5 depth-30 circuit with 216 parameters, tile 4:
    // 3.77 ms at 250 against 3.90 ms at 110).
    const double budget = rq.budget > 0 ? (double)rq.budget : (rq.dtype == SV_C64 ? 250.0 : 220.0);
    const std::vector<Sweep> sweeps = regtile_sweeps(g, rq.n, vb, rq.dtype, budget, true);
    const int m = (int)sweeps.size();
    // Checkpoints at sweep boundaries: checkpoint k is the state after the
    // first sweep by which every gate of cycles <= k c has run (the sweeps
    // are not cut for it); it is written by that sweep's store, and the
    // reverse of that sweep reads phi from it instead of from the
    // uncomputed state.  No checkpoint after the last sweep (the state
    // itself), none twice at one boundary.
    std::vector<int> ck_after(m, -1);
    int nck = 0;
    if (checkpoint_c > 0 && m > 1) {
        int maxc = 0;
        for (const SGate &s2 : g) maxc = std::max(maxc, (int)c->gates[s2.src].cycle);
        std::vector<int> last_sweep(maxc + 1, -1);
        for (int j2 = 0; j2 < m; j2++)
            for (int it : sweeps[j2].items) {
                const int cyc = c->gates[g[it].src].cycle;
                last_sweep[cyc] = std::max(last_sweep[cyc], j2);
            }
        for (int t = 1; t <= maxc; t++) last_sweep[t] = std::max(last_sweep[t], last_sweep[t - 1]);
        for (int k = 1; (int64_t)k * checkpoint_c < maxc; k++) {
            const int b = last_sweep[k * checkpoint_c];
            if (b >= 0 && b < m - 1 && ck_after[b] < 0) ck_after[b] = nck++;
        }
    }
    std::vector<RTProgram> progs;
    progs.reserve(m);
    for (int j2 = 0; j2 < m; j2++) {
        progs.push_back(build_regtile(g, sweeps[j2], vb, rq.n));
        push_regtile(progs.back(), rq.n, rq.dtype, OP_REGTILE, &plan->ops, plan);
        plan->ops.back().q1 = ck_after[j2];
        if (ck_after[j2] >= 0) plan->ops.back().bytes += state_bytes(rq.n, rq.dtype);
    }
    plan->ncheckpoints = nck;
    for (int j2 = m - 1; j2 >= 0; j2--) {
        push_regtile(reverse_regtile(progs[j2]), rq.n, rq.dtype, OP_ADJ_REGTILE, &plan->bops, plan);
        plan->bops.back().q1 = ck_after[j2];
    }
    plan->sweeps = (int64_t)(plan->ops.size() + plan->bops.size());
    plan->bytes = 0;
    for (const Op &op : plan->ops) plan->bytes += op.bytes;
    for (const Op &op : plan->bops) plan->bytes += op.bytes;
    return SV_OK;
}

}  // namespace svi
