// Host planner for LDS-staged passes (see pass_kernel.hip for the device
// side).  Splits a circuit into runs of gates that fit one chunk of local
// qubits, reorders diagonal phase terms as late as they commute, assigns
// register/thread bits per op and emits the pass programs.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>

#include "plan_internal.h"

namespace qsv {

namespace {

constexpr int LANE_BITS = 6;

// One gate seen by the pass planner.
struct PGate {
    enum Kind { PHASE, NONDIAG, SWAP, OTHER } kind = OTHER;
    int gi = -1;
    std::vector<int> targets;      // global bits, targets[0] = MSB of the matrix index
    std::vector<int> controls;
    std::vector<double> M;         // complex128 target block (NONDIAG)
    // PHASE: terms over global bits (mask, fixed-point turns)
    std::vector<std::pair<uint64_t, uint64_t>> terms;
};

uint64_t turns_fixed(double re, double im) {
    double t = std::atan2(im, re) / (2.0 * M_PI);   // (-1/2, 1/2]
    if (t >= 0.5) t -= 1.0;
    const long double scaled = (long double)t * 18446744073709551616.0L;
    return (uint64_t)(int64_t)std::llroundl(scaled);
}

int classify(const qsv_gate &g, PGate &pg) {
    std::vector<double> G;
    int st = gate_target_matrix(g, G);
    if (st) return st;
    pg.targets.assign(g.targets, g.targets + g.k);
    pg.controls.assign(g.controls, g.controls + g.c);
    const int d = 1 << g.k;
    bool diag = true;
    for (int r = 0; r < d && diag; ++r)
        for (int c = 0; c < d; ++c)
            if (r != c && (G[2 * (r * d + c)] != 0.0 || G[2 * (r * d + c) + 1] != 0.0)) { diag = false; break; }
    if (diag) {
        bool unit = true;
        std::vector<uint64_t> alpha(d);
        for (int t = 0; t < d; ++t) {
            const double re = G[2 * (t * d + t)], im = G[2 * (t * d + t) + 1];
            if (std::fabs(std::hypot(re, im) - 1.0) > 1e-14) unit = false;
            alpha[t] = turns_fixed(re, im);
        }
        if (!unit) {
            pg.kind = PGate::OTHER;
            return QSV_OK;
        }
        // Moebius inversion: theta_S = sum_{T subset S} (-1)^{|S|-|T|} alpha_T
        uint64_t cm = 0;
        for (int q : pg.controls) cm |= 1ull << q;
        for (int S = 0; S < d; ++S) {
            uint64_t th = 0;
            for (int T = S;; T = (T - 1) & S) {
                if ((__builtin_popcount(S) - __builtin_popcount(T)) & 1) th -= alpha[T];
                else th += alpha[T];
                if (T == 0) break;
            }
            if (th == 0) continue;
            uint64_t mask = cm;
            for (int j = 0; j < g.k; ++j)
                if ((S >> (g.k - 1 - j)) & 1) mask |= 1ull << g.targets[j];
            pg.terms.push_back({mask, th});
        }
        pg.kind = PGate::PHASE;
        return QSV_OK;
    }
    if (g.kind == QSV_GATE_SWAP && g.c == 0) {
        pg.kind = PGate::SWAP;
        return QSV_OK;
    }
    if (g.k <= 2) {
        pg.kind = PGate::NONDIAG;
        pg.M = G;
        return QSV_OK;
    }
    pg.kind = PGate::OTHER;
    return QSV_OK;
}

// ---------------------------------------------------------------- one pass

struct LOp {                        // an op in local-position space
    bool phase = false;
    std::vector<int> lt;            // NONDIAG: target local positions (lt[0] = MSB)
    uint32_t lc = 0;                // local control positions
    uint64_t gc = 0;                // non-local control bits
    std::vector<double> M;
    std::vector<std::pair<uint64_t, std::pair<uint32_t, uint64_t>>> terms;   // PHASE: (theta, (lmask, gmask))
    // one-target NONDIAG: phase terms (all containing the target) applied to
    // the |1> member just before the gate
    std::vector<std::pair<uint64_t, std::pair<uint32_t, uint64_t>>> pre;
};

struct Part {
    std::vector<int> reg;   // local positions of register bits
    std::vector<int> thr;   // local positions of thread bits (lanes first)
};

bool same_set(std::vector<int> a, std::vector<int> b) {
    std::sort(a.begin(), a.end());
    std::sort(b.begin(), b.end());
    return a == b;
}

// Fill a partition: registers get `want` (first RB distinct), lanes get the
// lowest remaining positions by `rank`, then the wave bits.
Part make_part(int L, int RB, const std::vector<int> &want, const std::vector<int> &rank_order) {
    Part p;
    std::vector<int> used(L, 0);
    for (int l : want) {
        if ((int)p.reg.size() == RB) break;
        if (!used[l]) {
            used[l] = 1;
            p.reg.push_back(l);
        }
    }
    // registers still free: take the highest-ranked positions so lanes keep the low ones
    for (int i = (int)rank_order.size() - 1; i >= 0 && (int)p.reg.size() < RB; --i) {
        const int l = rank_order[i];
        if (!used[l]) {
            used[l] = 1;
            p.reg.push_back(l);
        }
    }
    for (int l : rank_order)
        if (!used[l]) p.thr.push_back(l);
    return p;
}

// Relabel a gate's qubits through the bit permutation sig.
void relabel_gate(PGate &g, const std::vector<int> &sig) {
    for (int &q : g.targets) q = sig[q];
    for (int &q : g.controls) q = sig[q];
    for (auto &t : g.terms) {
        uint64_t m = 0;
        for (int b = 0; b < (int)sig.size(); ++b)
            if ((t.first >> b) & 1) m |= 1ull << sig[b];
        t.first = m;
    }
}
void relabel_gate(qsv_gate &g, const std::vector<int> &sig) {
    for (int j = 0; j < g.k; ++j) g.targets[j] = sig[g.targets[j]];
    for (int j = 0; j < g.c; ++j) g.controls[j] = sig[g.controls[j]];
}

// `fold` (optional): an involution of the global bits, closed on the local
// set, applied to the result on store (out[fold(i)] = in[i]): its local part
// joins the store's bit map and its non-local part pairs chunk c with chunk
// fold(c), which only the compiled kernel executes.
int compile_pass(int n, const std::vector<PGate> &gates, const std::vector<int> &local, int RB,
                 PassProgram &prog, const std::vector<int> *fold = nullptr) {
    const int L = (int)local.size();
    prog.L = L;
    prog.RB = RB;
    prog.TB = L - RB;
    prog.local_sorted = local;
    std::sort(prog.local_sorted.begin(), prog.local_sorted.end());
    int lpos[QSV_MAX_QUBITS];
    for (int q = 0; q < QSV_MAX_QUBITS; ++q) lpos[q] = -1;
    for (int l = 0; l < L; ++l) lpos[prog.local_sorted[l]] = l;
    int cur_l[QSV_MAX_QUBITS];   // local position holding logical qubit q (SWAP relabelings)
    for (int q = 0; q < QSV_MAX_QUBITS; ++q) cur_l[q] = lpos[q];

    // 1. resolve gates to local-position ops; defer phase terms while they commute
    std::vector<LOp> ops;
    LOp pending;
    pending.phase = true;
    auto flush = [&](uint32_t blocking, bool all, LOp *attach) {
        LOp out;
        out.phase = true;
        std::vector<std::pair<uint64_t, std::pair<uint32_t, uint64_t>>> keep;
        for (auto &t : pending.terms) {
            if (all || (t.second.first & blocking)) out.terms.push_back(t);
            else keep.push_back(t);
        }
        pending.terms.swap(keep);
        if (out.terms.empty()) return;
        if (attach) attach->pre.swap(out.terms);
        else ops.push_back(std::move(out));
    };
    // Multiply a non-diagonal op into an earlier one on the same local qubits
    // when the product stays within two targets: the ops in between must
    // commute with it (disjoint qubits, or phases off its targets) and both
    // carry the same controls.  A one-qubit layer followed by fSim on the
    // pair then costs one 4x4 product per amplitude instead of three ops.
    // Phase terms applied to the new op's |1> member are folded into its
    // matrix when they involve its target alone; otherwise it stays apart.
    auto merge_back = [&](LOp &b) -> bool {
        uint32_t bt = 0;
        for (int l : b.lt) bt |= 1u << l;
        std::vector<double> MB = b.M;
        if (!b.pre.empty()) {
            if (b.lc || b.gc) return false;   // its phases act whatever the controls hold
            uint64_t th = 0;
            for (auto &t : b.pre) {
                if (t.second.first != bt || t.second.second != 0) return false;
                th += t.first;
            }
            const double ang = 2.0 * M_PI * ((double)(int64_t)th * 5.421010862427522e-20);   // 2^-64 turns
            const double cr = std::cos(ang), ci = std::sin(ang);
            for (int r = 0; r < 2; ++r) {   // MB <- MB diag(1, e^{i ang}): column 1 times the factor
                const double xr = MB[2 * (2 * r + 1)], xi = MB[2 * (2 * r + 1) + 1];
                MB[2 * (2 * r + 1)] = xr * cr - xi * ci;
                MB[2 * (2 * r + 1) + 1] = xr * ci + xi * cr;
            }
        }
        const int scan_limit = 48;
        for (int k = (int)ops.size() - 1, seen = 0; k >= 0 && seen < scan_limit; --k, ++seen) {
            LOp &a = ops[k];
            if (a.phase) {
                for (auto &t : a.terms)
                    if (t.second.first & bt) return false;
                continue;
            }
            uint32_t at = 0;
            for (int l : a.lt) at |= 1u << l;
            if (!(at & bt)) {
                if ((at & b.lc) || (bt & a.lc)) return false;   // a target controls the other op
                for (auto &t : a.pre)
                    if (t.second.first & bt) return false;       // a's phases involve b's targets
                continue;                                        // disjoint: they commute
            }
            if (a.lc != b.lc || a.gc != b.gc) return false;
            std::vector<int> u = a.lt;
            for (int l : b.lt)
                if (std::find(u.begin(), u.end(), l) == u.end()) u.push_back(l);
            if (u.size() > 2 || (int)u.size() > RB) return false;
            // both matrices embedded in the index space of u (u[0] = MSB)
            const int du = 1 << (int)u.size();
            auto embed = [&](const LOp &o, const std::vector<double> &M) {
                std::vector<double> E(2 * du * du, 0.0);
                const int k = (int)o.lt.size();
                std::vector<int> pos(k);   // bit of u's index holding o.lt[j]
                for (int j = 0; j < k; ++j)
                    pos[j] = (int)u.size() - 1 - (int)(std::find(u.begin(), u.end(), o.lt[j]) - u.begin());
                for (int r = 0; r < du; ++r)
                    for (int c = 0; c < du; ++c) {
                        int ro = 0, co = 0;
                        bool same_rest = true;
                        uint32_t mine = 0;
                        for (int j = 0; j < k; ++j) {
                            ro |= ((r >> pos[j]) & 1) << (k - 1 - j);
                            co |= ((c >> pos[j]) & 1) << (k - 1 - j);
                            mine |= 1u << pos[j];
                        }
                        if (((uint32_t)r & ~mine) != ((uint32_t)c & ~mine)) same_rest = false;
                        if (!same_rest) continue;
                        const int d = 1 << k;
                        E[2 * (r * du + c)] = M[2 * (ro * d + co)];
                        E[2 * (r * du + c) + 1] = M[2 * (ro * d + co) + 1];
                    }
                return E;
            };
            const std::vector<double> EA = embed(a, a.M), EB = embed(b, MB);
            std::vector<double> P(2 * du * du, 0.0);   // P = EB EA
            for (int r = 0; r < du; ++r)
                for (int c = 0; c < du; ++c) {
                    double pr = 0.0, pi = 0.0;
                    for (int j = 0; j < du; ++j) {
                        const double xr = EB[2 * (r * du + j)], xi = EB[2 * (r * du + j) + 1];
                        const double yr = EA[2 * (j * du + c)], yi = EA[2 * (j * du + c) + 1];
                        pr += xr * yr - xi * yi;
                        pi += xr * yi + xi * yr;
                    }
                    P[2 * (r * du + c)] = pr;
                    P[2 * (r * du + c) + 1] = pi;
                }
            LOp m;
            m.lt = u;
            m.lc = a.lc;
            m.gc = a.gc;
            m.M = P;
            if (u.size() == 1) {
                m.pre = a.pre;   // applied before a, so before the product
                ops[k] = std::move(m);
            } else if (!a.pre.empty()) {
                LOp ph;   // a's |1>-member phases become a phase op in its place
                ph.phase = true;
                ph.terms = a.pre;
                ops[k] = std::move(ph);
                ops.insert(ops.begin() + k + 1, std::move(m));
            } else {
                ops[k] = std::move(m);
            }
            return true;
        }
        return false;
    };
    for (const PGate &g : gates) {
        switch (g.kind) {
        case PGate::PHASE:
            for (auto &t : g.terms) {
                uint32_t lm = 0;
                uint64_t gm = 0;
                for (int q = 0; q < n; ++q) {
                    if (!((t.first >> q) & 1)) continue;
                    if (cur_l[q] >= 0) lm |= 1u << cur_l[q];
                    else gm |= 1ull << q;
                }
                pending.terms.push_back({t.second, {lm, gm}});
            }
            break;
        case PGate::SWAP: {
            const int a = g.targets[0], b = g.targets[1];
            if (cur_l[a] < 0 || cur_l[b] < 0) return fail(QSV_ERR_ARG, "internal: SWAP on a non-local qubit in a pass");
            std::swap(cur_l[a], cur_l[b]);
            break;
        }
        case PGate::NONDIAG: {
            LOp op;
            uint32_t tmask = 0;
            for (int q : g.targets) {
                if (cur_l[q] < 0) return fail(QSV_ERR_ARG, "internal: pass target is not local");
                op.lt.push_back(cur_l[q]);
                tmask |= 1u << cur_l[q];
            }
            for (int q : g.controls) {
                if (cur_l[q] >= 0) op.lc |= 1u << cur_l[q];
                else op.gc |= 1ull << q;
            }
            op.M = g.M;
            flush(tmask, false, op.lt.size() == 1 ? &op : nullptr);
            if (!merge_back(op)) ops.push_back(std::move(op));
            break;
        }
        default: return fail(QSV_ERR_ARG, "internal: gate kind not allowed in a pass");
        }
    }
    flush(0, true, nullptr);

    // store map: local position l holds logical qubit q with cur_l[q] == l
    prog.out_pos.assign(L, -1);
    for (int q = 0; q < n; ++q)
        if (cur_l[q] >= 0) prog.out_pos[cur_l[q]] = q;
    prog.pair_sigma.clear();
    if (fold) {
        for (int l = 0; l < L; ++l) prog.out_pos[l] = (*fold)[prog.out_pos[l]];
        prog.pair_sigma = *fold;
    }

    // rank orders: local positions by global bit at load / at store
    std::vector<int> in_rank(L), out_rank(L);
    for (int l = 0; l < L; ++l) in_rank[l] = l;
    for (int l = 0; l < L; ++l) out_rank[l] = l;
    std::sort(out_rank.begin(), out_rank.end(), [&](int a, int b) { return prog.out_pos[a] < prog.out_pos[b]; });

    // 2. partitions.  Load: lanes on the 6 lowest positions; registers on the
    // first targets among the others.
    std::vector<std::vector<int>> need;   // per op: targets (empty for PHASE)
    for (auto &op : ops) need.push_back(op.phase ? std::vector<int>() : op.lt);
    auto upcoming = [&](size_t from, const std::vector<int> &forbid) {
        std::vector<int> w;
        for (size_t o = from; o < ops.size() && (int)w.size() < RB; ++o)
            for (int l : need[o])
                if (std::find(w.begin(), w.end(), l) == w.end() &&
                    std::find(forbid.begin(), forbid.end(), l) == forbid.end())
                    w.push_back(l);
        return w;
    };
    const int lanes = std::min(LANE_BITS, L - RB);
    std::vector<int> low_in(in_rank.begin(), in_rank.begin() + lanes);
    std::vector<Part> parts;
    Part cur = make_part(L, RB, upcoming(0, low_in), in_rank);
    parts.push_back(cur);
    prog.load_part = 0;

    prog.ops.clear();
    prog.pool.clear();
    prog.terms.clear();
    prog.slots.clear();
    auto reg_index = [&](const Part &p, int l) {
        for (int i = 0; i < (int)p.reg.size(); ++i)
            if (p.reg[i] == l) return i;
        return -1;
    };
    auto thr_index = [&](const Part &p, int l) {
        for (int u = 0; u < (int)p.thr.size(); ++u)
            if (p.thr[u] == l) return u;
        return -1;
    };
    auto emit_exchange = [&](const Part &np) {
        parts.push_back(np);
        PassOpDev d;
        std::memset(&d, 0, sizeof(d));
        d.kind = POP_EXCHANGE;
        d.a = (int)parts.size() - 1;
        prog.ops.push_back(d);
        cur = np;
    };
    // Encode the phase terms of an op as PassOpDev describes, under the
    // partition `cur`; `skip` is a local position removed from every term
    // (the target of a pre-phased G1, implied by its |1> member).
    const int NR = 1 << RB;
    auto turns_to_unit = [](uint64_t th, double &re, double &im) {
        const double ang = 2.0 * M_PI * ((double)(int64_t)th * 5.421010862427522e-20);   // 2^-64 turns
        re = std::cos(ang);
        im = std::sin(ang);
    };
    auto encode_terms = [&](const std::vector<std::pair<uint64_t, std::pair<uint32_t, uint64_t>>> &terms, int skip,
                            PassOpDev &d) {
        std::vector<uint64_t> fconst(NR, 0);
        std::vector<std::vector<PassTermDev>> thr(RB + 1);                    // thread bits only
        std::map<std::pair<int, uint32_t>, std::vector<PassTermDev>> chunk;  // (group, thread mask) -> terms
        std::vector<PassTermDev> gen;
        for (auto &t : terms) {
            PassTermDev td;
            std::memset(&td, 0, sizeof(td));
            td.theta = t.first;
            td.mn = t.second.second;
            int nreg = 0, reg = -1;
            for (int l = 0; l < L; ++l) {
                if (!((t.second.first >> l) & 1) || l == skip) continue;
                const int i = reg_index(cur, l);
                if (i >= 0) {
                    td.mj |= 1u << i;
                    reg = i;
                    ++nreg;
                } else {
                    td.mt |= 1u << thr_index(cur, l);
                }
            }
            if (td.mt == 0 && td.mn == 0) {
                // register bits only: folded into the host table Fc
                for (int j = 0; j < NR; ++j)
                    if (((uint32_t)j & td.mj) == td.mj) fconst[j] += td.theta;
                continue;
            }
            if (nreg >= 2) {
                gen.push_back(td);
                continue;
            }
            const int g = nreg ? 1 + reg : 0;
            if (td.mn == 0) thr[g].push_back(td);
            else chunk[{g, td.mt}].push_back(td);
        }
        // per-thread tables (each 256 complex; bounded so a program fits a staging slot)
        for (int g = 0; g <= PASS_MAX_RB; ++g) d.tab[g] = -1;
        for (int g = 0; g <= RB; ++g) {
            if (thr[g].empty()) continue;
            if (prog.pool.size() + (2u << prog.TB) > 16384) {
                for (auto &td : thr[g]) chunk[{g, td.mt}].push_back(td);   // evaluated as slots instead
                continue;
            }
            d.tab[g] = (int)prog.pool.size();
            for (uint32_t tt = 0; tt < (1u << prog.TB); ++tt) {
                uint64_t ph = 0;
                for (auto &td : thr[g])
                    if ((tt & td.mt) == td.mt) ph += td.theta;
                double re, im;
                turns_to_unit(ph, re, im);
                prog.pool.push_back(re);
                prog.pool.push_back(im);
            }
        }
        // slots, grouped by F_g; long sums are split, and past the per-op
        // limit the terms are evaluated as general terms
        const int s_first = (int)prog.slots.size();
        for (int g = 0; g <= RB; ++g) {
            d.sl[g] = (int)prog.slots.size();
            for (auto &kv : chunk) {
                if (kv.first.first != g) continue;
                const auto &ts = kv.second;
                for (size_t b = 0; b < ts.size(); b += PASS_SLOT_TERMS) {
                    const size_t e = std::min(ts.size(), b + PASS_SLOT_TERMS);
                    if ((int)prog.slots.size() - s_first >= PASS_MAX_SLOTS) {
                        for (size_t k = b; k < e; ++k) gen.push_back(ts[k]);
                        continue;
                    }
                    PassSlotDev sd;
                    std::memset(&sd, 0, sizeof(sd));
                    sd.mt = kv.first.second;
                    sd.begin = (int)prog.terms.size();
                    for (size_t k = b; k < e; ++k) prog.terms.push_back(ts[k]);
                    sd.end = (int)prog.terms.size();
                    prog.slots.push_back(sd);
                }
            }
        }
        for (int g = RB + 1; g <= PASS_MAX_RB + 1; ++g) d.sl[g] = (int)prog.slots.size();
        d.gen_b = (int)prog.terms.size();
        for (auto &td : gen) prog.terms.push_back(td);
        d.gen_e = (int)prog.terms.size();
        d.var = 0;
        if (d.tab[0] >= 0 || d.sl[1] > d.sl[0]) d.var |= 1;
        for (int g = 1; g <= RB; ++g)
            if (d.tab[g] >= 0 || d.sl[g + 1] > d.sl[g]) d.var |= 2;
        d.fc = -1;
        bool any = false;
        for (int j = 0; j < NR; ++j)
            if (fconst[j] != 0) any = true;
        if (any) {
            d.fc = (int)prog.pool.size();
            for (int j = 0; j < NR; ++j) {
                double re, im;
                turns_to_unit(fconst[j], re, im);
                prog.pool.push_back(re);
                prog.pool.push_back(im);
            }
        }
    };
    for (size_t o = 0; o < ops.size(); ++o) {
        const LOp &op = ops[o];
        PassOpDev d;
        std::memset(&d, 0, sizeof(d));
        if (!op.phase) {
            bool ok = true;
            for (int l : op.lt)
                if (reg_index(cur, l) < 0) ok = false;
            if (!ok) {
                std::vector<int> w = upcoming(o, {});
                // keep current lanes when possible, so LDS patterns stay regular
                emit_exchange(make_part(L, RB, w, in_rank));
            }
            for (int l = 0; l < L; ++l) {
                if (!((op.lc >> l) & 1)) continue;
                const int i = reg_index(cur, l);
                if (i >= 0) d.cj |= 1u << i;
                else d.ct |= 1u << thr_index(cur, l);
            }
            d.cn = op.gc;
            d.mat = (int)prog.pool.size();
            if (op.lt.size() == 1) {
                d.a = reg_index(cur, op.lt[0]);
                if (!op.pre.empty()) {
                    // the phase terms that must precede this gate all contain its
                    // target: applied to the gate's |1> members, grouped by the
                    // other bits they need
                    d.pre = 1;
                    encode_terms(op.pre, op.lt[0], d);
                }
                d.mat = (int)prog.pool.size();
                bool real = true;
                for (int e = 0; e < 4; ++e)
                    if (op.M[2 * e + 1] != 0.0) real = false;
                if (real) {
                    d.kind = POP_G1R;
                    for (int e = 0; e < 4; ++e) prog.pool.push_back(op.M[2 * e]);
                } else {
                    d.kind = POP_G1;
                    for (int e = 0; e < 8; ++e) prog.pool.push_back(op.M[e]);
                }
            } else {
                d.kind = POP_G2;
                int i0 = reg_index(cur, op.lt[0]), i1 = reg_index(cur, op.lt[1]);
                bool swapq = false;
                if (i0 < i1) {
                    std::swap(i0, i1);
                    swapq = true;
                }
                d.a = i0;
                d.b = i1;
                auto sw = [&](int x) { return swapq ? (((x & 1) << 1) | ((x >> 1) & 1)) : x; };
                for (int r = 0; r < 4; ++r)
                    for (int c = 0; c < 4; ++c) {
                        const int e = sw(r) * 4 + sw(c);
                        prog.pool.push_back(op.M[2 * e]);
                        prog.pool.push_back(op.M[2 * e + 1]);
                    }
            }
        } else {
            d.kind = POP_PHASE;
            encode_terms(op.terms, -1, d);
        }
        prog.ops.push_back(d);
    }
    // store: lanes must be the 6 positions with the lowest output bits
    std::vector<int> low_out(out_rank.begin(), out_rank.begin() + lanes);
    std::vector<int> cur_lanes(cur.thr.begin(), cur.thr.begin() + lanes);
    if (!same_set(cur_lanes, low_out)) {
        // registers: current registers that are not store lanes, then the highest outputs
        std::vector<int> w;
        for (int l : cur.reg)
            if (std::find(low_out.begin(), low_out.end(), l) == low_out.end()) w.push_back(l);
        emit_exchange(make_part(L, RB, w, out_rank));
    }
    prog.parts.clear();
    for (auto &p : parts) {
        PassPartition pp;
        std::memset(&pp, 0, sizeof(pp));
        for (int i = 0; i < RB; ++i) pp.reg_l[i] = p.reg[i];
        for (int u = 0; u < prog.TB; ++u) pp.thr_l[u] = p.thr[u];
        prog.parts.push_back(pp);
    }
    prog.n_gates = (int)gates.size();
    prog.serialise();
    return QSV_OK;
}

}  // namespace

// Register bits of a chunk of `local_bits` local qubits (0: the largest) in
// a workgroup of 2^tb threads; -1 when no valid chunk exists.
int pass_register_bits(int n, int dtype, int local_bits, int tb) {
    const int rb_max = dtype == QSV_C64 ? 5 : 4;
    int L = local_bits > 0 ? local_bits : rb_max + tb;
    if (L > n) L = n;
    const int RB = L - tb;
    if (RB < 1 || RB > rb_max) return -1;
    return RB;
}

namespace {

int build_passes_once(qsv_plan *p, int local_bits, bool allow_fold) {
    const int n = p->n;
    const int TB = p->opts.jit ? PASS_JIT_THREAD_BITS : PASS_THREAD_BITS;
    const int RB = pass_register_bits(n, p->dtype, local_bits, TB);
    if (local_bits > 0 && RB < 0) return fail(QSV_ERR_ARG, "local_bits outside the supported range");
    if (RB < 0) {
        // too few qubits for a chunk: per-gate launches
        for (size_t i = 0; i < p->gates.size(); ++i) {
            int st = plan_add_gate_op(p, p->gates[i]);
            if (st) return st;
            p->ops.back().gate_ids = {(int)i};
        }
        return QSV_OK;
    }
    const int L = RB + TB;
    const int lanes = std::min(LANE_BITS, L - RB);
    // SWAP gates become relabellings: logical qubit q lives at physical bit
    // phys[q]; every other gate is rewritten onto physical bits.
    std::vector<int> phys(n);
    for (int q = 0; q < n; ++q) phys[q] = q;
    std::vector<qsv_gate> gates;
    std::vector<int> circuit_index;   // gates[k] is gate circuit_index[k] of the circuit
    for (size_t i0 = 0; i0 < p->gates.size(); ++i0) {
        const qsv_gate &g0 = p->gates[i0];
        if (g0.kind == QSV_GATE_SWAP && g0.c == 0) {
            std::swap(phys[g0.targets[0]], phys[g0.targets[1]]);
            continue;
        }
        circuit_index.push_back((int)i0);
        qsv_gate g = g0;
        for (int j = 0; j < g.k; ++j) g.targets[j] = phys[g0.targets[j]];
        for (int j = 0; j < g.c; ++j) g.controls[j] = phys[g0.controls[j]];
        gates.push_back(g);
    }
    std::vector<PGate> pgs(gates.size());
    for (size_t i = 0; i < gates.size(); ++i) {
        int st = classify(gates[i], pgs[i]);
        if (st) return st;
        pgs[i].gi = (int)i;
        // a two-qubit gate needs two register bits
        if (pgs[i].kind == PGate::NONDIAG && pgs[i].targets.size() > (size_t)RB) pgs[i].kind = PGate::OTHER;
    }
    // The relabelling left at the end (data of logical qubit q sits at bit
    // phys[q]) is undone by sigma, written as a product of at most two
    // involutions (a cycle is the product of two reflections of it).  With
    // compiled passes each involution in turn is folded into the next pass
    // whose local set can be closed under it: that pass stores its result
    // permuted (P_tau V_1), and every later gate is relabelled through tau,
    // since P_tau V_2 V_1 = (P_tau V_2 P_tau^-1) P_tau V_1.  Involutions left
    // over run as permutation sweeps at the end (or a few SWAPs).
    std::vector<int> sigma(n);
    bool moved = false;
    for (int q = 0; q < n; ++q) {
        sigma[phys[q]] = q;
        if (phys[q] != q) moved = true;
    }
    std::vector<std::vector<int>> pending;   // involutions to apply, first one first
    int nswaps = 0;                          // SWAPs that would undo sigma instead
    if (moved) {
        // cycle c_0 -> c_1 -> ... -> c_{k-1}: tau_1(c_i) = c_{-i}, tau_2(c_i) = c_{1-i} (indices mod k)
        std::vector<int> t1(n), t2(n), seen(n, 0);
        for (int b = 0; b < n; ++b) {
            if (seen[b]) continue;
            std::vector<int> cyc;
            for (int c = b; !seen[c]; c = sigma[c]) {
                seen[c] = 1;
                cyc.push_back(c);
            }
            const int k = (int)cyc.size();
            nswaps += k - 1;
            for (int i = 0; i < k; ++i) {
                t1[cyc[i]] = cyc[(k - i) % k];
                t2[cyc[i]] = cyc[(k + 1 - i) % k];
            }
        }
        bool t1_id = true;
        for (int b = 0; b < n; ++b)
            if (t1[b] != b) t1_id = false;
        if (!t1_id) pending.push_back(t1);
        pending.push_back(t2);
    }
    size_t nfolded = 0;        // pending involutions already folded into passes
    bool relabel_due = false;  // the last fold still has to relabel the gates not yet placed
    std::vector<PGate> run;
    int run_nd = 0;   // non-diagonal gates in the open pass
    uint64_t S = 0;   // local set (global bits) of the open pass
    auto reset_local = [&]() {
        S = 0;
        for (int q = 0; q < lanes; ++q) S |= 1ull << q;
    };
    // local set of exactly `size` bits that contains s and is closed under the involution t, if any
    auto close_under = [&](const std::vector<int> &t, uint64_t s, uint64_t &out, int size) {
        for (int b = 0; b < n; ++b)
            if ((s >> b) & 1) s |= 1ull << t[b];
        for (int b = 0; b < n && __builtin_popcountll(s) < size; ++b)   // fixed points first
            if (t[b] == b) s |= 1ull << b;
        for (int b = 0; b < n && __builtin_popcountll(s) + 1 < size; ++b)
            if (!((s >> b) & 1)) s |= (1ull << b) | (1ull << t[b]);
        if (__builtin_popcountll(s) != size) return false;
        out = s;
        return true;
    };
    auto close = [&]() -> int {
        if (run.empty()) return QSV_OK;
        const std::vector<int> *fold = nullptr;
        uint64_t Sc = 0;
        if (allow_fold && nfolded < pending.size() && close_under(pending[nfolded], S, Sc, L)) {
            S = Sc;
            fold = &pending[nfolded];
            ++nfolded;
            relabel_due = true;
        }
        // fill the local set with the lowest missing bits
        for (int q = 0; q < n && __builtin_popcountll(S) < L; ++q) S |= 1ull << q;
        std::vector<int> local;
        for (int q = 0; q < n; ++q)
            if ((S >> q) & 1) local.push_back(q);
        auto prog = std::make_shared<PassProgram>();
        int st = compile_pass(n, run, local, RB, *prog, fold);
        if (st) return st;
        PlanOp op;
        op.kind = PlanOp::PASS;
        op.pass = prog;
        const double s = p->dtype == QSV_C64 ? 8.0 : 16.0;
        op.bytes = 2.0 * std::ldexp(1.0, n) * s;
        double fl = 0;
        for (auto &g : run) fl += g.kind == PGate::NONDIAG ? (g.targets.size() == 1 ? 8.0 : 16.0) * std::ldexp(1.0, n)
                                                            : 0.0;
        op.flops = fl;
        for (auto &g : run) op.gate_ids.push_back(circuit_index[g.gi]);
        p->ops.push_back(std::move(op));
        p->stats.n_passes++;
        run.clear();
        run_nd = 0;
        reset_local();
        return QSV_OK;
    };
    reset_local();
    std::vector<char> done(pgs.size(), 0);
    auto sync_relabel = [&]() {   // gates not yet placed follow the last fold
        if (!relabel_due) return;
        relabel_due = false;
        const std::vector<int> &t = pending[nfolded - 1];
        for (size_t k = 0; k < pgs.size(); ++k)
            if (!done[k]) {
                relabel_gate(pgs[k], t);
                relabel_gate(gates[k], t);
            }
    };
    auto needed = [](const PGate &g) {
        uint64_t m = 0;
        if (g.kind == PGate::NONDIAG || g.kind == PGate::SWAP)
            for (int q : g.targets) m |= 1ull << q;
        return m;
    };
    // qubits a gate acts on non-diagonally (its targets, unless it is a
    // phase gate) and diagonally (its controls; every qubit of a phase gate)
    auto acts = [](const PGate &g, uint64_t &nd, uint64_t &d) {
        nd = d = 0;
        for (int q : g.targets) (g.kind == PGate::PHASE ? d : nd) |= 1ull << q;
        for (int q : g.controls) d |= 1ull << q;
    };
    // When gate i does not fit the open pass, later gates that commute with
    // every gate skipped so far still join it.  Two gates commute when on
    // every qubit they share both act diagonally (both are then sums over the
    // shared qubits' basis states of operators on disjoint qubits), which
    // covers disjoint gates, phase gates, and controls.  A skipped gate's
    // qubits block later gates accordingly; the scan stops once every qubit
    // is blocked non-diagonally or after a bounded number of gates.
    const uint64_t all = n >= 64 ? ~0ull : (1ull << n) - 1ull;
    // A gate fits the open pass when its targets fit the chunk and the pass
    // holds fewer than PASS_MAX_NONDIAG non-diagonal gates: longer passes
    // (the lookahead can gather 150+ gates) spill registers and take tens
    // of seconds to compile without saving sweeps.
    auto fits = [&](const PGate &g) {
        const uint64_t m = needed(g);
        return __builtin_popcountll(S | m) <= L && (m == 0 || run_nd < PASS_MAX_NONDIAG);
    };
    auto add = [&](const PGate &g) {
        if (needed(g)) ++run_nd;
        S |= needed(g);
        run.push_back(g);
    };
    auto lookahead = [&](size_t i) {
        uint64_t bnd = 0, bd = 0;
        auto skip = [&](const PGate &h) {
            uint64_t nd, d;
            acts(h, nd, d);
            bnd |= nd;
            bd |= d;
        };
        skip(pgs[i]);
        size_t scanned = 0;
        for (size_t j = i + 1; j < pgs.size() && scanned < PASS_LOOKAHEAD && bnd != all; ++j) {
            if (done[j]) continue;
            ++scanned;
            const PGate &h = pgs[j];
            uint64_t nd, d;
            acts(h, nd, d);
            const bool commutes = !(nd & (bnd | bd)) && !(d & bnd);
            if (commutes && h.kind != PGate::OTHER && fits(h)) {
                add(h);
                done[j] = 1;
            } else {
                skip(h);
            }
        }
    };
    for (size_t i = 0; i < pgs.size(); ++i) {
        if (done[i]) continue;
        if (pgs[i].kind == PGate::OTHER) {
            if (!run.empty()) lookahead(i);
            int st = close();
            sync_relabel();
            done[i] = 1;
            if (!st) st = plan_add_gate_op(p, gates[i]);
            if (st) return st;
            p->ops.back().gate_ids = {circuit_index[i]};
            continue;
        }
        if (!fits(pgs[i])) {
            lookahead(i);
            int st = close();
            if (st) return st;
            sync_relabel();
        }
        add(pgs[i]);
        done[i] = 1;
    }
    int st = close();
    if (st) return st;
    if (nfolded == pending.size()) return QSV_OK;
    const double s_amp = p->dtype == QSV_C64 ? 8.0 : 16.0;
    // A permutation sweep per involution left, unless a few SWAPs of
    // physical qubits do it for less (a SWAP costs about one sweep).
    if (nfolded == 0 && pending.size() == 2) {
        if (nswaps <= 2) {
            std::vector<int> at(n);   // at[b] = logical qubit held by physical bit b
            for (int q = 0; q < n; ++q) at[phys[q]] = q;
            for (int b = 0; b < n; ++b) {
                if (at[b] == b) continue;
                const int other = phys[b];   // physical bit holding logical qubit b
                qsv_gate g;
                std::memset(&g, 0, sizeof(g));
                g.kind = QSV_GATE_SWAP;
                g.k = 2;
                g.targets[0] = b;
                g.targets[1] = other;
                if ((st = plan_add_gate_op(p, g))) return st;
                const int qb = at[b];
                std::swap(at[b], at[other]);
                phys[qb] = other;
                phys[b] = b;
            }
            return QSV_OK;
        }
    }
    for (size_t k = nfolded; k < pending.size(); ++k) {
        const std::vector<int> &t = pending[k];
        PlanOp op;
        op.bytes = 2.0 * std::ldexp(1.0, n) * s_amp;
        // local set: the lowest bits, each with its image, so that both the
        // loads and the stores run over the longest contiguous stretches; a
        // chunk one bit smaller when no closed set of L bits exists
        auto lowest_closed = [&](int size, uint64_t &out) {
            uint64_t sl = 0;
            for (int b = 0; b < n; ++b) {
                if ((sl >> b) & 1) continue;
                const int need = t[b] == b ? 1 : 2;
                if (__builtin_popcountll(sl) + need > size) continue;
                sl |= (1ull << b) | (1ull << t[b]);
            }
            out = sl;
            return __builtin_popcountll(sl) == size && (sl & ((1ull << lanes) - 1ull)) == (1ull << lanes) - 1ull;
        };
        // (13 local bits first when the involution moves a lane bit, which
        // takes an LDS exchange: the pass has no gates to amortise, and a
        // 64 KiB chunk (complex64) lets two workgroups share a CU, so one's
        // loads overlap the other's exchange and stores -- measured on the
        // 30-qubit swap of qubits 0..5 with 24..29: 3.06 ms at 13 bits, 3.25
        // at 14, 3.47 at 12.  An involution without fixed points, such as the
        // reversal of an even number of qubits, has no closed set of 13
        // bits; there 14 bits beat 12 (the 30-qubit reversal: 3.26 ms
        // against 3.37).  Without an exchange the largest chunk streams best.)
        bool moves_lanes = false;
        for (int b = 0; b < lanes; ++b)
            if (t[b] != b) moves_lanes = true;
        uint64_t Sp = 0;
        int rbp = -1;
        const int l13 = std::min(L, 13);
        const int order[4] = {moves_lanes ? l13 : L, moves_lanes ? L : L - 1, moves_lanes ? l13 - 1 : l13,
                              moves_lanes ? L - 1 : l13 - 1};
        for (int size : order) {
            if (size - TB < 1 || rbp >= 0) continue;
            if (lowest_closed(size, Sp)) rbp = size - TB;
        }
        if (p->opts.jit && rbp >= 1) {
            // compiled plans: a pass without gates whose store applies t
            std::vector<int> local;
            for (int q = 0; q < n; ++q)
                if ((Sp >> q) & 1) local.push_back(q);
            auto prog = std::make_shared<PassProgram>();
            int st2 = compile_pass(n, {}, local, rbp, *prog, &t);
            if (st2) return st2;
            op.kind = PlanOp::PASS;
            op.pass = prog;
        } else {
            op.kind = PlanOp::PERM;
            op.sigma = t;
        }
        p->ops.push_back(std::move(op));
        p->stats.n_passes++;
    }
    return QSV_OK;
}

}  // namespace

// With compiled passes, the plan that folds the final permutation into a pass
// (see above) is kept only when it needs fewer sweeps over the state than
// the plan that ends with a bit-permutation kernel: a chunk-pair pass costs
// more than a plain pass.
int build_passes(qsv_plan *p, int local_bits) {
    if (!p->opts.jit) return build_passes_once(p, local_bits, false);
    const size_t ops0 = p->ops.size();
    const qsv_plan_stats st0 = p->stats;
    int st = build_passes_once(p, local_bits, true);
    if (st) return st;
    bool paired = false;
    for (size_t i = ops0; i < p->ops.size(); ++i)
        if (p->ops[i].kind == PlanOp::PASS && !p->ops[i].pass->pair_sigma.empty()) paired = true;
    if (!paired) return QSV_OK;
    std::vector<PlanOp> fold_ops(p->ops.begin() + ops0, p->ops.end());
    const qsv_plan_stats fold_stats = p->stats;
    p->ops.resize(ops0);
    p->stats = st0;
    if ((st = build_passes_once(p, local_bits, false))) return st;
    if (fold_ops.size() < p->ops.size() - ops0) {
        p->ops.resize(ops0);
        p->ops.insert(p->ops.end(), fold_ops.begin(), fold_ops.end());
        p->stats = fold_stats;
    }
    return QSV_OK;
}

int build_single_pass(int n, int dtype, const std::vector<qsv_gate> &gates, const std::vector<int> &local,
                      PassProgram &out) {
    const int L = (int)local.size();
    const int RB = pass_register_bits(n, dtype, L, PASS_THREAD_BITS);
    if (RB < 0 || L != RB + PASS_THREAD_BITS) return fail(QSV_ERR_ARG, "nlocal must be in [9, 13] (complex64) or [9, 12] (complex128) and <= n");
    uint64_t S = 0;
    for (int q : local) {
        if (q < 0 || q >= n) return fail(QSV_ERR_QUBIT_RANGE, "local qubit out of range");
        if ((S >> q) & 1) return fail(QSV_ERR_QUBIT_DUP, "local qubit repeats");
        S |= 1ull << q;
    }
    for (int q = 0; q < 3; ++q)
        if (!((S >> q) & 1)) return fail(QSV_ERR_ARG, "local qubits must contain qubits 0, 1 and 2");
    std::vector<PGate> pgs(gates.size());
    for (size_t i = 0; i < gates.size(); ++i) {
        int st = classify(gates[i], pgs[i]);
        if (st) return st;
        if (pgs[i].kind == PGate::OTHER || (pgs[i].kind == PGate::NONDIAG && pgs[i].targets.size() > (size_t)RB))
            return fail(QSV_ERR_UNSUPPORTED, "gate " + std::to_string(i) + " cannot run in a pass (dense k > 2 or non-unitary diagonal)");
        if (pgs[i].kind != PGate::PHASE)
            for (int q : pgs[i].targets)
                if (!((S >> q) & 1)) return fail(QSV_ERR_ARG, "gate " + std::to_string(i) + " targets a non-local qubit");
    }
    return compile_pass(n, pgs, local, RB, out);
}

}  // namespace qsv

using namespace qsv;

extern "C" int qsv_run_pass(void *state, int n, int dtype, const qsv_gate *gates, int ngates, const int *local_qubits,
                            int nlocal, void *stream) {
    int st = validate_common(n, dtype, nullptr, 0, nullptr, 0);
    if (st) return st;
    if (!state || !local_qubits || (ngates > 0 && !gates)) return fail(QSV_ERR_NULL, "NULL argument");
    if (((uintptr_t)state & 15) != 0) return fail(QSV_ERR_ALIGN, "state must be 16-byte aligned");
    std::vector<qsv_gate> gs(gates, gates + ngates);
    for (auto &g : gs)
        if ((st = validate_common(n, dtype, g.targets, g.k, g.controls, g.c))) return st;
    PassProgram prog;
    std::vector<int> local(local_qubits, local_qubits + nlocal);
    if ((st = build_single_pass(n, dtype, gs, local, prog))) return st;
    return launch_pass_program(state, n, dtype, prog, (hipStream_t)stream);
}
