// Pass programs compiled into kernels of their own.
//
// The pass kernel of pass_kernel.hip interprets a program: every op of every
// chunk dispatches on the op kind, loads its constants and moves the
// register tile between the registers of the switch cases.  Here a program
// is instead turned into HIP source for one kernel, compiled at plan
// creation with hiprtc and loaded on first use: the op sequence, the
// register/thread assignments, the gate matrices and the constant phase
// factors become literals.  Register-bit controls become compile-time pair
// selections, zero matrix entries drop out, a row with a single unit entry
// becomes a register move, and the per-thread LDS and global offsets are
// computed once per kernel.  The semantics are those of the interpreted
// kernel op for op (same ops, same tables in the program's pool, same
// phase-term grouping); only the arithmetic order may differ.
#include <hip/hiprtc.h>

#include <cinttypes>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <elf.h>
#include <map>
#include <set>
#include <mutex>
#include <unordered_map>

#include "plan_internal.h"

namespace qsv {

// A code object holding the kernels of one or more passes (compiled
// together), loaded on a device at the first launch of any of them.
struct JitCode {
    std::vector<char> code;                 // code object for gfx950
    std::mutex mu;
    std::map<int, hipModule_t> mod;         // per device
    ~JitCode() {
        for (auto &kv : mod)
            if (kv.second) {
                int cur = 0;
                (void)hipGetDevice(&cur);
                (void)hipSetDevice(kv.first);
                (void)hipDeviceSynchronize();   // no launch of this module may still run
                (void)hipModuleUnload(kv.second);
                (void)hipSetDevice(cur);
            }
    }
};

// One compiled pass: its kernel in a (shared) code object.
struct JitModule {
    std::shared_ptr<JitCode> code;
    std::string kernel;                     // the kernel's name in the code object
    std::string source;                     // the pass's kernel source (as one program of its own)
    bool prefetch = false;                  // persistent workgroups with a prefetched next chunk
    bool one_shot = false;                  // exactly one chunk per workgroup (split exchanges)
    std::mutex mu;
    struct Loaded {
        hipFunction_t fn = nullptr;
        int grid_per_cu = 0;
    };
    std::map<int, Loaded> dev;              // per device, found on first launch
};

// Persistent workgroups that load the next chunk while computing the current
// one, when two register tiles fit without spills (not for chunk pairs, which
// hold two tiles already); otherwise one chunk per workgroup.  A 512-thread
// workgroup of 14 local qubits fills a CU's LDS alone, so without this the
// memory pipe of its CU would idle while it computes.
bool pass_jit_prefetch(const PassProgram &p, int dtype) {
    if (!p.pair_sigma.empty()) return false;
    if (p.TB == PASS_JIT_THREAD_BITS) return dtype == QSV_C64 ? p.RB <= 5 : p.RB <= 3;
    return dtype == QSV_C64 ? p.RB <= 4 : p.RB <= 3;
}

// Non-local bits of a chunk-pair pass: the pairs (a, b) that sigma swaps
// (a < b, ascending a) and the bits it fixes.
PairLayout pair_layout(const std::vector<int> &sigma, uint64_t local) {
    PairLayout pl;
    for (int q = 0; q < (int)sigma.size(); ++q) {
        if ((local >> q) & 1) continue;
        if (sigma[q] == q) pl.fixed.push_back(q);
        else if (sigma[q] > q) {
            pl.a.push_back(q);
            pl.b.push_back(sigma[q]);
        }
    }
    return pl;
}

// Work items of a chunk-pair pass: one per pair {c, sigma(c)} of distinct
// chunks and one per chunk sigma fixes, (4^m + 2^m) 2^f / 2 in all.
uint64_t pair_work_items(const std::vector<int> &sigma, uint64_t local) {
    const PairLayout pl = pair_layout(sigma, local);
    const int m = (int)pl.a.size(), f = (int)pl.fixed.size();
    return ((1ull << (2 * m + f)) + (1ull << (m + f))) / 2;
}

namespace {

const char *JIT_KERNEL_NAME = "qsv_pass_jit";

// ---------------------------------------------------------------- source generation

std::string fmt(const char *f, ...) __attribute__((format(printf, 1, 2)));
std::string fmt(const char *f, ...) {
    va_list ap, aq;
    va_start(ap, f);
    va_copy(aq, ap);
    const int n = vsnprintf(nullptr, 0, f, ap);
    va_end(ap);
    std::string out(n > 0 ? (size_t)n : 0, '\0');
    if (n > 0) vsnprintf(&out[0], (size_t)n + 1, f, aq);
    va_end(aq);
    return out;
}

uint32_t swz(uint32_t l) { return l ^ (((l >> 4) ^ (l >> 8) ^ (l >> 12)) & 15u); }

// A matrix or phase entry with the rounding residue of an exact 0 or +-1
// removed (cos and sin of multiples of pi/2 in floating point): such entries
// then cost no multiplication.  The change is below 2^-50.
double snap(double v) {
    if (std::fabs(v) < 0x1p-50) return 0.0;
    if (std::fabs(v - 1.0) < 0x1p-50) return 1.0;
    if (std::fabs(v + 1.0) < 0x1p-50) return -1.0;
    return v;
}

// 0, 1, 2, 3 when (re, im) is 1, i, -1, -i; -1 otherwise
int quarter_turn(double re, double im) {
    if (im == 0.0 && re == 1.0) return 0;
    if (re == 0.0 && im == 1.0) return 1;
    if (im == 0.0 && re == -1.0) return 2;
    if (re == 0.0 && im == -1.0) return 3;
    return -1;
}

// Where a local position sits in a partition: register bit i (reg = true)
// or thread bit i.
struct Slot {
    bool reg;
    int i;
};
Slot slot_of(const PassPartition &part, int RB, int TB, int pos) {
    for (int i = 0; i < RB; ++i)
        if (part.reg_l[i] == pos) return {true, i};
    for (int u = 0; u < TB; ++u)
        if (part.thr_l[u] == pos) return {false, u};
    return {true, -1};
}

// The local position an exchange from partition A to B is split on, or -1.
// A round takes the amplitudes with that position 0 (then 1): on a side where
// it is a register bit, half the registers of every lane; where it is a thread
// bit, every register of half the threads.  A register bit on both sides is
// best (no lane idles); a thread bit must lie above the 64 lanes of a wave, so
// that whole waves idle in a round rather than half of every wave.
int split_position(const PassProgram &p, const PassPartition &A, const PassPartition &B) {
    for (int i = 0; i < p.RB; ++i) {   // a register bit on both sides, in A's register order
        const Slot b = slot_of(B, p.RB, p.TB, A.reg_l[i]);
        if (b.reg && b.i >= 0) return A.reg_l[i];
    }
    int best = -1, best_cost = 3;
    for (int pos = 0; pos < p.L; ++pos) {
        const Slot a = slot_of(A, p.RB, p.TB, pos), b = slot_of(B, p.RB, p.TB, pos);
        if ((!a.reg && a.i < 6) || (!b.reg && b.i < 6) || (a.reg && a.i < 0) || (b.reg && b.i < 0)) continue;
        const int cost = (a.reg ? 0 : 1) + (b.reg ? 0 : 1);
        if (cost < best_cost) {
            best = pos;
            best_cost = cost;
        }
    }
    return best;
}

// Every exchange of the program can be split (the condition for a kernel of
// split exchanges).
bool exchanges_split(const PassProgram &p) {
    if (!p.pair_sigma.empty()) return false;
    int c = p.load_part;
    bool any = false;
    for (auto &op : p.ops)
        if (op.kind == POP_EXCHANGE) {
            if (split_position(p, p.parts[c], p.parts[op.a]) < 0) return false;
            any = true;
            c = op.a;
        }
    return any;
}

class Gen {
  public:
    Gen(const PassProgram &p, int dtype, const JitVariant &v)
        : P(p), f32(dtype == QSV_C64), NR(1 << p.RB), pool_offset(((const PassHeaderDev *)p.blob.data())->off_pool),
          terms_offset(((const PassHeaderDev *)p.blob.data())->off_terms), share(v.share && !p.param),
          PF(v.prefetch && !(v.split && exchanges_split(p)) && pass_jit_prefetch(p, dtype)),
          split(v.split && exchanges_split(p)),
          param(p.param) {}
    std::string source();

  private:
    const PassProgram &P;
    const bool f32;
    const int NR;
    const int pool_offset;   // byte offset of the real pool in the serialised program
    const int terms_offset;  // byte offset of the phase terms in the serialised program
    std::string s;
    int uid = 0;
    double scale_re = 1.0, scale_im = 0.0;   // complex factor owed by every amplitude of the tile (see gate())
    const bool share;     // form products of phase factors shared by several amplitudes once
    const bool PF;        // prefetch the next chunk (persistent workgroups)
    const bool split;     // exchanges in two rounds over a shared register bit (see JitVariant)
    // Parametric kernel: matrix entries, phase angles and constant phase
    // tables are read from the program at run time (uniform loads) instead
    // of being compiled in, so the source depends only on the circuit's
    // structure (which gates act on which bits) and a circuit whose angles
    // change reuses the compiled kernel.  Nothing is specialised on values:
    // no zero entries dropped, no factored skeletons, no free quarter turns.
    const bool param;
    // the angle of phase term k as the kernel reads it
    std::string theta(int k) const { return param ? fmt("tth[%d]", 1 + 3 * k) : u64(P.terms[k].theta); }
    void gate_param(const PassOpDev &op, const std::vector<int> &bits, bool real);

    void ln(const std::string &x) { s += x, s += '\n'; }
    double R(double v) const { v = snap(v); return f32 ? (double)(float)v : v; }   // value as the kernel's real type holds it
    std::string lit(double v) const {
        char buf[64];
        if (f32) snprintf(buf, sizeof(buf), "%af", (double)(float)v);
        else snprintf(buf, sizeof(buf), "%a", v);
        return buf;
    }
    std::string u64(uint64_t v) const { return fmt("0x%" PRIx64 "ull", v); }

    // x or y component of sum_s c_s * a_s (c_s complex literals, a_s C variables)
    std::string comb(const std::vector<std::pair<std::pair<double, double>, std::string>> &terms, bool y) const;
    void gate(const PassOpDev &op, const std::vector<int> &bits, const std::vector<double> &M, bool real);
    void phase(const PassOpDev &op, int sk);   // multiplies v[j] (j with bit sk clear: v[j | 2^sk]) by f_j
    std::string thread_offset(const PassPartition &part, const int *pos, bool global) const;
};

std::string Gen::comb(const std::vector<std::pair<std::pair<double, double>, std::string>> &terms, bool y) const {
    std::string e;
    auto add = [&](double c, const std::string &var) {
        if (c == 0.0) return;
        if (c == 1.0) e += (e.empty() ? "" : " + ") + var;
        else if (c == -1.0) e += (e.empty() ? "-" : " - ") + var;
        else e += (e.empty() ? "" : " + ") + lit(c) + " * " + var;
    };
    for (auto &t : terms) {
        const double re = R(t.first.first), im = R(t.first.second);
        if (!y) {
            add(re, t.second + ".x");
            add(-im, t.second + ".y");
        } else {
            add(re, t.second + ".y");
            add(im, t.second + ".x");
        }
    }
    return e.empty() ? std::string("(R)0") : e;
}

// Global (or local) offset of the thread part of a partition: sum over the
// thread bits u of bit u of t shifted to its position.
std::string Gen::thread_offset(const PassPartition &part, const int *pos, bool global) const {
    std::string e;
    for (int u = 0; u < P.TB; ++u) {
        const int p = pos ? pos[part.thr_l[u]] : part.thr_l[u];
        if (p < 0) continue;   // the position an exchange is split on
        if (!e.empty()) e += " | ";
        if (global) e += fmt("((unsigned long long)((t >> %d) & 1u) << %d)", u, p);
        else e += fmt("(((t >> %d) & 1u) << %d)", u, p);
    }
    return e.empty() ? std::string("(0u)") : "(" + e + ")";
}

// One- or two-qubit gate on register bits (bits[0] = the matrix index MSB).
void Gen::gate(const PassOpDev &op, const std::vector<int> &bits, const std::vector<double> &M0, bool real) {
    const int k = (int)bits.size(), d = 1 << k;
    const bool tok = op.ct != 0 || op.cn != 0;
    // An uncontrolled gate acts on every amplitude of the tile, so a common
    // factor c of its entries can be taken out: the gate's skeleton M / c
    // runs here and c joins the factor that the pass applies once before its
    // store (every op of a pass is linear, so the factor commutes with the
    // rest).  c is the first nonzero entry when every entry is c times one of
    // 0, +-1, +-i (the square roots of X and Y: additions only), else the
    // common magnitude when all nonzero entries share one (H, ...).
    std::vector<double> M = M0;
    if (!tok && op.cj == 0) {
        const int ne = d * d;
        auto entry = [&](int e, double &re, double &im) {
            re = real ? M[e] : M[2 * e];
            im = real ? 0.0 : M[2 * e + 1];
        };
        double cre = 0.0, cim = 0.0, mag = -1.0;
        bool quarter = true, same = true;
        for (int e = 0; e < ne; ++e) {
            double re, im;
            entry(e, re, im);
            const double a = std::hypot(re, im);
            if (a == 0.0) continue;
            if (mag < 0) {
                mag = a;
                cre = re;
                cim = im;
                continue;
            }
            if (std::fabs(a - mag) > 1e-15 * mag) same = false;
            // e / c = e * conj(c) / |c|^2 must be one of +-1, +-i
            const double qr = (re * cre + im * cim) / (mag * mag), qi = (im * cre - re * cim) / (mag * mag);
            if (quarter_turn(snap(qr), snap(qi)) < 0) quarter = false;
        }
        if (mag > 0 && same && quarter && !real && (cre != 1.0 || cim != 0.0)) {
            const double n2 = cre * cre + cim * cim;
            for (int e = 0; e < ne; ++e) {
                const double re = M[2 * e], im = M[2 * e + 1];
                M[2 * e] = (re * cre + im * cim) / n2;
                M[2 * e + 1] = (im * cre - re * cim) / n2;
            }
            const double sr = scale_re * cre - scale_im * cim, si = scale_re * cim + scale_im * cre;
            scale_re = sr;
            scale_im = si;
        } else if (mag > 0 && same && mag != 1.0) {
            for (double &x : M) x /= mag;
            scale_re *= mag;
            scale_im *= mag;
        }
    }
    if (tok) ln(fmt("        { const bool tk = ((t & %uu) == %uu) && ((base & %s) == %s);", op.ct, op.ct,
                    u64(op.cn).c_str(), u64(op.cn).c_str()));
    else ln("        {");
    uint32_t gm = 0;
    for (int b : bits) gm |= 1u << b;
    for (int j = 0; j < NR; ++j) {
        if (j & gm) continue;
        if (((uint32_t)j & op.cj) != op.cj) continue;
        std::vector<int> idx(d);
        for (int r = 0; r < d; ++r) {
            int x = j;
            for (int q = 0; q < k; ++q)
                if ((r >> (k - 1 - q)) & 1) x |= 1 << bits[q];
            idx[r] = x;
        }
        std::string body = "            {";
        for (int r = 0; r < d; ++r) body += fmt(" const C a%d = v[%d];", r, idx[r]);
        ln(body);
        for (int r = 0; r < d; ++r) {
            std::vector<std::pair<std::pair<double, double>, std::string>> terms;
            bool unit_self = true;
            for (int c = 0; c < d; ++c) {
                double re, im;
                if (real) re = M[r * d + c], im = 0.0;
                else re = M[2 * (r * d + c)], im = M[2 * (r * d + c) + 1];
                const double rr = R(re), ri = R(im);
                if (rr == 0.0 && ri == 0.0) continue;
                if (!(c == r && rr == 1.0 && ri == 0.0)) unit_self = false;
                terms.push_back({{re, im}, fmt("a%d", c)});
            }
            if (unit_self && terms.size() == 1) continue;   // row of the identity
            const std::string ex = comb(terms, false), ey = comb(terms, true);
            if (tok)
                ln(fmt("              v[%d].x = tk ? (R)(%s) : a%d.x; v[%d].y = tk ? (R)(%s) : a%d.y;", idx[r],
                       ex.c_str(), r, idx[r], ey.c_str(), r));
            else ln(fmt("              v[%d].x = %s; v[%d].y = %s;", idx[r], ex.c_str(), idx[r], ey.c_str()));
        }
        ln("            }");
    }
    ln("        }");
}

// One- or two-qubit gate with its matrix read from the pool (parametric
// kernels): the same group structure as gate(), every entry a variable.
void Gen::gate_param(const PassOpDev &op, const std::vector<int> &bits, bool real) {
    const int k = (int)bits.size(), d = 1 << k;
    const bool tok = op.ct != 0 || op.cn != 0;
    const int id = uid++;
    std::string dec = "        {";
    for (int e = 0; e < d * d; ++e) {
        if (real) dec += fmt(" const R m%d_%dr = pool[%d];", id, e, op.mat + e);
        else dec += fmt(" const R m%d_%dr = pool[%d], m%d_%di = pool[%d];", id, e, op.mat + 2 * e, id, e, op.mat + 2 * e + 1);
    }
    ln(dec);
    if (tok) ln(fmt("          const bool tk = ((t & %uu) == %uu) && ((base & %s) == %s);", op.ct, op.ct,
                    u64(op.cn).c_str(), u64(op.cn).c_str()));
    uint32_t gm = 0;
    for (int b : bits) gm |= 1u << b;
    for (int j = 0; j < NR; ++j) {
        if (j & gm) continue;
        if (((uint32_t)j & op.cj) != op.cj) continue;
        std::vector<int> idx(d);
        for (int r = 0; r < d; ++r) {
            int x = j;
            for (int q = 0; q < k; ++q)
                if ((r >> (k - 1 - q)) & 1) x |= 1 << bits[q];
            idx[r] = x;
        }
        std::string body = "            {";
        for (int r = 0; r < d; ++r) body += fmt(" const C a%d = v[%d];", r, idx[r]);
        ln(body);
        for (int r = 0; r < d; ++r) {
            std::string ex, ey;
            for (int c = 0; c < d; ++c) {
                const int e = r * d + c;
                if (real) {
                    ex += fmt("%sm%d_%dr * a%d.x", c ? " + " : "", id, e, c);
                    ey += fmt("%sm%d_%dr * a%d.y", c ? " + " : "", id, e, c);
                } else {
                    ex += fmt("%sm%d_%dr * a%d.x - m%d_%di * a%d.y", c ? " + " : "", id, e, c, id, e, c);
                    ey += fmt("%sm%d_%dr * a%d.y + m%d_%di * a%d.x", c ? " + " : "", id, e, c, id, e, c);
                }
            }
            if (tok)
                ln(fmt("              v[%d].x = tk ? (R)(%s) : a%d.x; v[%d].y = tk ? (R)(%s) : a%d.y;", idx[r],
                       ex.c_str(), r, idx[r], ey.c_str(), r));
            else ln(fmt("              v[%d].x = %s; v[%d].y = %s;", idx[r], ex.c_str(), idx[r], ey.c_str()));
        }
        ln("            }");
    }
    ln("        }");
}

// Phase factors of an op (see PassOpDev), applied to the register tile.
void Gen::phase(const PassOpDev &op, int sk) {
    const int RB = P.RB;
    const int id = uid++;
    ln("        {");
    // F_g for the groups that vary per thread or chunk
    std::vector<bool> var(RB + 1, false);
    const int s0 = op.sl[0], s1 = op.sl[RB + 1];
    if (s1 > s0) {
        // chunk-dependent slot sums (uniform), one per lane, one sincos
        ln("          unsigned long long sph = 0;");
        for (int sI = s0; sI < s1; ++sI) {
            const PassSlotDev &sd = P.slots[sI];
            std::string e;
            for (int kI = sd.begin; kI < sd.end; ++kI) {
                const PassTermDev &tm = P.terms[kI];
                if (tm.mn == 0) e += fmt(" + %s", theta(kI).c_str());
                else e += fmt(" + (((base & %s) == %s) ? %s : 0ull)", u64(tm.mn).c_str(), u64(tm.mn).c_str(),
                              theta(kI).c_str());
            }
            ln(fmt("          if (lane == %d) sph = 0ull%s;", sI - s0, e.c_str()));
        }
        ln("          const C se = expi(sph);");
    }
    for (int g = 0; g <= RB; ++g) {
        const bool has_tab = op.tab[g] >= 0, has_sl = op.sl[g + 1] > op.sl[g];
        if (!has_tab && !has_sl) continue;
        var[g] = true;
        if (has_tab) ln(fmt("          C F%d = ((const C *)(pool + %d))[t];", g, op.tab[g]));
        else ln(fmt("          C F%d; F%d.x = (R)1; F%d.y = (R)0;", g, g, g));
        for (int sI = op.sl[g]; sI < op.sl[g + 1]; ++sI) {
            const uint32_t mt = P.slots[sI].mt;
            if (mt == 0) ln(fmt("          F%d = cm(F%d, rdl(se, %d));", g, g, sI - s0));
            else ln(fmt("          { const C e = rdl(se, %d); if ((t & %uu) == %uu) F%d = cm(F%d, e); }", sI - s0, mt,
                        mt, g, g));
        }
    }
    // h_j = F_0 * prod_{i in j} F_{1+i}; "one" entries are tracked on the host
    std::vector<int> h_one(NR, 1);
    std::vector<std::string> h(NR);
    if (var[0]) {
        h[0] = "F0";
        h_one[0] = 0;
    }
    for (int top = 0; top < RB; ++top) {
        if (top == sk) continue;
        for (int rest = 0; rest < (1 << top); ++rest) {
            if (sk >= 0 && ((rest >> sk) & 1)) continue;
            const int j = rest | (1 << top);
            if (!var[1 + top]) {
                h[j] = h[rest];
                h_one[j] = h_one[rest];
            } else if (h_one[rest]) {
                h[j] = fmt("F%d", 1 + top);
                h_one[j] = 0;
            } else {
                ln(fmt("          const C h%d_%d = cm(%s, F%d);", id, j, h[rest].c_str(), 1 + top));
                h[j] = fmt("h%d_%d", id, j);
                h_one[j] = 0;
            }
        }
    }
    // f_j = h_j * Fc[j]: a quarter turn Fc[j] is a free rotation; a product
    // h_j * Fc[j] that several amplitudes take is formed once (a product used
    // once is applied as two factors: precomputed ones would all be live at
    // once)
    auto fc_of = [&](int j, double &cre, double &cim) {
        cre = 1.0, cim = 0.0;
        if (op.fc >= 0) {
            cre = R(P.pool[op.fc + 2 * j]);
            cim = R(P.pool[op.fc + 2 * j + 1]);
        }
    };
    if (param) {
        // f_j = h_j * Fc[j] with Fc read from the pool; general terms as below
        for (int j = 0; j < NR; ++j) {
            if (sk >= 0 && ((j >> sk) & 1)) continue;
            const int tj = sk >= 0 ? (j | (1 << sk)) : j;
            if (!h_one[j]) ln(fmt("          v[%d] = cm(v[%d], %s);", tj, tj, h[j].c_str()));
            if (op.fc >= 0)
                ln(fmt("          v[%d] = cml(v[%d], pool[%d], pool[%d]);", tj, tj, op.fc + 2 * j, op.fc + 2 * j + 1));
            std::string e;
            for (int kI = op.gen_b; kI < op.gen_e; ++kI) {
                const PassTermDev &tm = P.terms[kI];
                if (((uint32_t)j & tm.mj) != tm.mj) continue;
                e += fmt(" + ((((t & %uu) == %uu) && ((base & %s) == %s)) ? %s : 0ull)", tm.mt, tm.mt,
                         u64(tm.mn).c_str(), u64(tm.mn).c_str(), theta(kI).c_str());
            }
            if (!e.empty()) ln(fmt("          v[%d] = cm(v[%d], expi(0ull%s));", tj, tj, e.c_str()));
        }
        ln("        }");
        return;
    }
    typedef std::pair<std::string, std::pair<double, double>> Key;
    std::map<Key, int> uses;
    for (int j = 0; j < NR; ++j) {
        if (sk >= 0 && ((j >> sk) & 1)) continue;
        double cre, cim;
        fc_of(j, cre, cim);
        if (!h_one[j] && quarter_turn(cre, cim) < 0) uses[Key(h[j], {cre, cim})]++;
    }
    // shared products first, each right before the amplitudes that take it
    int ng = 0;
    for (auto &ku : uses) {
        if (!share || ku.second < 2) continue;
        const std::string g = fmt("g%d_%d", id, ng++);
        ln(fmt("          { const C %s = cml(%s, %s, %s);", g.c_str(), ku.first.first.c_str(),
               lit(ku.first.second.first).c_str(), lit(ku.first.second.second).c_str()));
        for (int j = 0; j < NR; ++j) {
            if (sk >= 0 && ((j >> sk) & 1)) continue;
            double cre, cim;
            fc_of(j, cre, cim);
            if (h_one[j] || Key(h[j], {cre, cim}) != ku.first) continue;
            const int tj = sk >= 0 ? (j | (1 << sk)) : j;
            ln(fmt("            v[%d] = cm(v[%d], %s);", tj, tj, g.c_str()));
        }
        ln("          }");
    }
    for (int j = 0; j < NR; ++j) {
        if (sk >= 0 && ((j >> sk) & 1)) continue;
        const int tj = sk >= 0 ? (j | (1 << sk)) : j;   // the amplitude the factor multiplies
        double cre, cim;
        fc_of(j, cre, cim);
        const int rot = quarter_turn(cre, cim);
        const Key key(h[j], {cre, cim});
        if (share && !h_one[j] && rot < 0 && uses[key] >= 2) {
            // applied above
        } else {
            if (!h_one[j]) ln(fmt("          v[%d] = cm(v[%d], %s);", tj, tj, h[j].c_str()));
            if (rot > 0) ln(fmt("          v[%d] = rot%d(v[%d]);", tj, rot, tj));
            else if (rot < 0) ln(fmt("          v[%d] = cml(v[%d], %s, %s);", tj, tj, lit(cre).c_str(), lit(cim).c_str()));
        }
        // general terms
        std::string e;
        for (int kI = op.gen_b; kI < op.gen_e; ++kI) {
            const PassTermDev &tm = P.terms[kI];
            if (((uint32_t)j & tm.mj) != tm.mj) continue;
            e += fmt(" + ((((t & %uu) == %uu) && ((base & %s) == %s)) ? %s : 0ull)", tm.mt, tm.mt,
                     u64(tm.mn).c_str(), u64(tm.mn).c_str(), theta(kI).c_str());
        }
        if (!e.empty()) ln(fmt("          v[%d] = cm(v[%d], expi(0ull%s));", tj, tj, e.c_str()));
    }
    ln("        }");
}

std::string Gen::source() {
    const int L = P.L, RB = P.RB;
    const bool pair = !P.pair_sigma.empty();
    bool any_exchange = false;
    for (auto &op : P.ops)
        if (op.kind == POP_EXCHANGE) any_exchange = true;
    bool relabel = false;
    for (int l = 0; l < L; ++l)
        if (P.out_pos[l] != P.local_sorted[l]) relabel = true;
    if (any_exchange) relabel = false;

    ln(f32 ? "typedef float R;" : "typedef double R;");
    ln("struct __attribute__((aligned(2 * sizeof(R)))) C { R x, y; };");
    ln("__device__ __forceinline__ C cm(C a, C b) { C r; r.x = a.x * b.x - a.y * b.y; r.y = a.x * b.y + a.y * b.x; "
       "return r; }");
    ln("__device__ __forceinline__ C cml(C a, R re, R im) { C r; r.x = a.x * re - a.y * im; r.y = a.x * im + a.y * re; "
       "return r; }");
    ln("__device__ __forceinline__ C rot1(C a) { C r; r.x = -a.y; r.y = a.x; return r; }");    // a * i
    ln("__device__ __forceinline__ C rot2(C a) { C r; r.x = -a.x; r.y = -a.y; return r; }");   // a * -1
    ln("__device__ __forceinline__ C rot3(C a) { C r; r.x = a.y; r.y = -a.x; return r; }");    // a * -i
    // global accesses as a uniform 64-bit base (scalar registers) plus a
    // 32-bit per-thread byte offset: one address form of the memory
    // instruction, no 64-bit vector address arithmetic per access
    ln("#define GLB __attribute__((address_space(1)))");
    ln("__device__ __forceinline__ unsigned long long sreg(unsigned long long x) {");
    ln("    return ((unsigned long long)(unsigned)__builtin_amdgcn_readfirstlane((int)(x >> 32)) << 32) |");
    ln("           (unsigned long long)(unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)x); }");
    if (f32) {
        // complex64 amplitudes stream nontemporally: each is loaded and
        // stored once per pass
        ln("typedef float V2 __attribute__((ext_vector_type(2)));");
        ln("__device__ __forceinline__ C ldg(unsigned long long ub, unsigned off) {");
        ln("    const V2 v = __builtin_nontemporal_load((const GLB V2 *)((const GLB char *)ub + off)); C r; r.x = v.x; r.y = v.y; return r; }");
        ln("__device__ __forceinline__ void stg(unsigned long long ub, unsigned off, C v) {");
        ln("    V2 w; w.x = v.x; w.y = v.y; __builtin_nontemporal_store(w, (GLB V2 *)((GLB char *)ub + off)); }");
    } else {
        ln("__device__ __forceinline__ C ldg(unsigned long long ub, unsigned off) { return *(const GLB C *)((const GLB char *)ub + off); }");
        ln("__device__ __forceinline__ void stg(unsigned long long ub, unsigned off, C v) { *(GLB C *)((GLB char *)ub + off) = v; }");
    }
    if (f32) {
        ln("__device__ __forceinline__ C expi(unsigned long long ph) {");
        ln("    const float x = (float)(int)(unsigned)(ph >> 32) * 2.3283064365386963e-10f;");
        ln("    C r; sincospif(2.0f * x, &r.y, &r.x); return r; }");
        ln("__device__ __forceinline__ C rdl(C v, int l) { C r;");
        ln("    r.x = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v.x), l));");
        ln("    r.y = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v.y), l)); return r; }");
    } else {
        ln("__device__ __forceinline__ C expi(unsigned long long ph) {");
        ln("    const double x = (double)(long long)ph * 5.421010862427522e-20;");
        ln("    C r; sincospi(2.0 * x, &r.y, &r.x); return r; }");
        ln("__device__ __forceinline__ double rdl1(double v, int l) {");
        ln("    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);");
        ln("    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, l);");
        ln("    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), l);");
        ln("    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo); }");
        ln("__device__ __forceinline__ C rdl(C v, int l) { C r; r.x = rdl1(v.x, l); r.y = rdl1(v.y, l); return r; }");
    }
    ln("__device__ __forceinline__ void lbar() {");
    ln("    __builtin_amdgcn_fence(__ATOMIC_RELEASE, \"workgroup\", \"local\");");
    ln("    __builtin_amdgcn_s_barrier();");
    ln("    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, \"workgroup\", \"local\"); }");
    ln("__device__ __forceinline__ unsigned swz(unsigned l) { return l ^ (((l >> 4) ^ (l >> 8) ^ (l >> 12)) & 15u); }");
    // an amplitude as an operand of an empty volatile asm: its load has
    // completed (the compiler waits for it) before anything after this point
    ln("__device__ __forceinline__ void hold(C v) { asm volatile(\"\" :: \"v\"(v.x), \"v\"(v.y)); }");
    ln("");
    // Split exchanges: an exchange runs in two rounds over one local
    // position (split_position), each through an LDS region of half the
    // chunk indexed with that position removed.
    struct Xchg {
        int from, to, bit;   // bit: the position split on, or -1
    };
    std::vector<Xchg> xs;
    {
        int c = P.load_part;
        for (auto &op : P.ops)
            if (op.kind == POP_EXCHANGE) {
                xs.push_back({c, op.a, split ? split_position(P, P.parts[c], P.parts[op.a]) : -1});
                c = op.a;
            }
    }
    bool halved = !xs.empty();
    for (auto &x : xs) halved = halved && x.bit >= 0;
    if (split && halved)   // two workgroups of 2^TB lanes per CU: 4 waves per SIMD at 512 lanes
        ln(fmt("extern \"C\" __global__ void __attribute__((amdgpu_flat_work_group_size(%d, %d), "
               "amdgpu_waves_per_eu(%d))) %s(C *__restrict__ psi, const unsigned char *__restrict__ prog, "
               "unsigned long long nchunks) {",
               1 << P.TB, 1 << P.TB, std::max(1, (2 << P.TB) / 256), JIT_KERNEL_NAME));
    else
        ln(fmt("extern \"C\" __global__ void __launch_bounds__(%d) %s(C *__restrict__ psi, const unsigned char "
               "*__restrict__ prog, unsigned long long nchunks) {",
               1 << P.TB, JIT_KERNEL_NAME));
    if (any_exchange) ln(fmt("    __shared__ C lds[%d];", (split && halved) ? 1 << (L - 1) : 1 << L));
    ln(fmt("    const R *pool = (const R *)(prog + %d);", pool_offset));
    ln("    (void)pool;");
    if (param) {
        // phase terms as 64-bit words (mn, theta, mt | mj << 32): theta of term k at word 1 + 3 k
        ln(fmt("    const unsigned long long *tth = (const unsigned long long *)(prog + %d);", terms_offset));
        ln("    (void)tth;");
    }
    ln("    const unsigned t = threadIdx.x;");
    ln("    const int lane = (int)(t & 63u);");
    ln("    (void)lane;");
    // per-thread offsets, once per kernel
    int in_pos[PASS_MAX_L], out_pos[PASS_MAX_L];
    for (int l = 0; l < L; ++l) {
        in_pos[l] = P.local_sorted[l];
        out_pos[l] = P.out_pos[l];
    }
    ln("    const unsigned long long lt_in = " + thread_offset(P.parts[P.load_part], in_pos, true) + ";");
    int cur = P.load_part;
    for (auto &op : P.ops)
        if (op.kind == POP_EXCHANGE) cur = op.a;
    const int final_part = cur;
    ln("    const unsigned long long lt_out = " + thread_offset(P.parts[final_part], out_pos, true) + ";");
    // compressed local index of position l when position `bit` is removed
    auto cpos_of = [&](int bit, int *cpos) {
        for (int l = 0; l < L; ++l) cpos[l] = l == bit ? -1 : (bit >= 0 && l > bit) ? l - 1 : l;
    };
    if (any_exchange && !(split && halved))
        for (size_t pi = 0; pi < P.parts.size(); ++pi)
            ln(fmt("    const unsigned xo%zu = swz(%s) * (unsigned)sizeof(C);", pi,
                   thread_offset(P.parts[pi], nullptr, false).c_str()));
    if (any_exchange && split && halved)
        for (size_t xi = 0; xi < xs.size(); ++xi) {
            int cpos[PASS_MAX_L];
            cpos_of(xs[xi].bit, cpos);
            ln(fmt("    const unsigned xw%zu = swz(%s) * (unsigned)sizeof(C);", xi,
                   thread_offset(P.parts[xs[xi].from], cpos, false).c_str()));
            ln(fmt("    const unsigned xr%zu = swz(%s) * (unsigned)sizeof(C);", xi,
                   thread_offset(P.parts[xs[xi].to], cpos, false).c_str()));
        }
    // chunk base: the chunk index with zeros inserted at the local bits
    std::string cb = "    auto chunk_base = [&](unsigned long long c) { unsigned long long b = c, lo;";
    for (int l = 0; l < L; ++l)
        cb += fmt(" lo = b & %s; b = lo | ((b ^ lo) << 1);", u64((1ull << P.local_sorted[l]) - 1ull).c_str());
    cb += " return b; };";
    ln(cb);
    // register offsets of the load and store partitions
    auto reg_off = [&](const PassPartition &part, const int *pos, int j) {
        uint64_t o = 0;
        for (int i = 0; i < RB; ++i)
            if ((j >> i) & 1) o |= 1ull << pos[part.reg_l[i]];
        return o;
    };
    // (per-thread byte offsets below 4 GiB: uniform base + 32-bit offset)
    const int csz = f32 ? 8 : 16;
    auto small_offsets = [&](const PassPartition &part, const int *pos) {
        int top = 0;
        for (int u = 0; u < P.TB; ++u) top = std::max(top, pos[part.thr_l[u]]);
        return std::ldexp(1.0, top + 1) * csz <= 4294967296.0;
    };
    std::string ld = "    auto load_chunk = [&](C *dst, unsigned long long b) {";
    if (small_offsets(P.parts[P.load_part], in_pos)) {
        ln("    const unsigned to_in = (unsigned)(lt_in * sizeof(C));");
        ld += " const unsigned long long q = (unsigned long long)(psi + b);";
        for (int j = 0; j < NR; ++j)
            ld += fmt(" dst[%d] = ldg(sreg(q + %s), to_in);", j,
                      u64(reg_off(P.parts[P.load_part], in_pos, j) * csz).c_str());
    } else {
        ld += " const C *p = psi + (b | lt_in);";
        for (int j = 0; j < NR; ++j) ld += fmt(" dst[%d] = p[%s];", j, u64(reg_off(P.parts[P.load_part], in_pos, j)).c_str());
    }
    ld += " };";
    ln(ld);
    std::string sto = "    auto store_chunk = [&](const C *src, unsigned long long b) {";
    if (small_offsets(P.parts[final_part], out_pos)) {
        ln("    const unsigned to_out = (unsigned)(lt_out * sizeof(C));");
        sto += " const unsigned long long q = (unsigned long long)(psi + b);";
        for (int j = 0; j < NR; ++j)
            sto += fmt(" stg(sreg(q + %s), to_out, src[%d]);", u64(reg_off(P.parts[final_part], out_pos, j) * csz).c_str(), j);
    } else {
        sto += " C *p = psi + (b | lt_out);";
        for (int j = 0; j < NR; ++j)
            sto += fmt(" p[%s] = src[%d];", u64(reg_off(P.parts[final_part], out_pos, j)).c_str(), j);
    }
    sto += " };";
    ln(sto);
    if (pair) {
        // the chunk holding the images of chunk `b` under sigma (non-local bits only)
        const int n = (int)P.pair_sigma.size();
        uint64_t local = 0, fixed = 0;
        for (int l = 0; l < L; ++l) local |= 1ull << P.local_sorted[l];
        // Work item w -> chunk base, one item per pair {c, sigma(c)} (see
        // pair_work_items): groups k = 0..m-1 take the chunks whose first
        // differing pair (ascending a) is pair k, with a_k = 1 and b_k = 0;
        // group m the chunks sigma fixes.  Within a group the bits of w go
        // to the a-bits of the free pairs first (neighbouring chunks), then
        // their b-bits, the fixed bits and the equal pairs.
        const PairLayout pl = pair_layout(P.pair_sigma, local);
        const int m = (int)pl.a.size(), f = (int)pl.fixed.size();
        std::string cbw = "    auto pair_base = [&](unsigned long long w) {";
        uint64_t start = 0;
        for (int k = 0; k <= m; ++k) {
            const uint64_t size = k < m ? (1ull << (k + 2 * (m - 1 - k) + f)) : (1ull << (m + f));
            std::string e = k < m ? u64(1ull << pl.a[k]) : std::string("0ull");
            int i = 0;
            for (int j = k + 1; j < m; ++j, ++i) e += fmt(" | (((r >> %d) & 1ull) << %d)", i, pl.a[j]);
            for (int j = k + 1; j < m; ++j, ++i) e += fmt(" | (((r >> %d) & 1ull) << %d)", i, pl.b[j]);
            for (int j = 0; j < f; ++j, ++i) e += fmt(" | (((r >> %d) & 1ull) << %d)", i, pl.fixed[j]);
            for (int j = 0; j < k && j < m; ++j, ++i)
                e += fmt(" | (((r >> %d) & 1ull) * %s)", i, u64((1ull << pl.a[j]) | (1ull << pl.b[j])).c_str());
            cbw += fmt(" if (w < %s) { const unsigned long long r = w - %s; (void)r; return %s; }",
                       u64(start + size).c_str(), u64(start).c_str(), e.c_str());
            start += size;
        }
        cbw += " return 0ull; };";
        ln(cbw);
        std::string e = "    auto partner = [&](unsigned long long b) { return (b & ";
        for (int q = 0; q < n; ++q)
            if (!((local >> q) & 1) && P.pair_sigma[q] == q) fixed |= 1ull << q;
        e += u64(fixed) + ")";
        for (int q = 0; q < n; ++q)
            if (!((local >> q) & 1) && P.pair_sigma[q] != q)
                e += fmt(" | (((b >> %d) & 1ull) << %d)", q, P.pair_sigma[q]);
        e += "; };";
        ln(e);
    }
    // the ops, once per tile
    ln("    auto run_ops = [&](C *v, const unsigned long long base) __attribute__((always_inline)) {");
    cur = P.load_part;
    int xi_next = 0;
    for (size_t o = 0; o < P.ops.size(); ++o) {
        const PassOpDev &op = P.ops[o];
        ln(fmt("        // op %zu", o));
        switch (op.kind) {
        case POP_G1:
        case POP_G1R: {
            if (op.pre) phase(op, op.a);
            std::vector<double> M;
            const int cnt = op.kind == POP_G1 ? 8 : 4;
            for (int e = 0; e < cnt; ++e) M.push_back(P.pool[op.mat + e]);
            if (param) gate_param(op, {op.a}, op.kind == POP_G1R);
            else gate(op, {op.a}, M, op.kind == POP_G1R);
            break;
        }
        case POP_G2: {
            std::vector<double> M(P.pool.begin() + op.mat, P.pool.begin() + op.mat + 32);
            if (param) gate_param(op, {op.a, op.b}, false);
            else gate(op, {op.a, op.b}, M, false);
            break;
        }
        case POP_PHASE: phase(op, -1); break;
        case POP_EXCHANGE: {
            const PassPartition &A = P.parts[cur], &B = P.parts[op.a];
            const int csz = f32 ? 8 : 16;
            if (split && halved) {
                const Xchg &x = xs[xi_next++];
                int cpos[PASS_MAX_L];
                cpos_of(x.bit, cpos);
                // the split position may sit at another register index, or in
                // the thread index, afterwards: round 0's reads go to a tile of
                // their own so they cannot overwrite registers round 1 has
                // still to write
                const Slot sa = slot_of(A, RB, P.TB, x.bit), sb = slot_of(B, RB, P.TB, x.bit);
                ln(fmt("        { C xt[%d];", NR));
                for (int round = 0; round < 2; ++round) {
                    ln("        lbar();");
                    std::string w = sa.reg ? "       " : fmt("        if (((t >> %d) & 1u) == %du) {", sa.i, round);
                    for (int j = 0; j < NR; ++j) {
                        uint32_t l = 0;
                        bool in = true;
                        for (int i = 0; i < RB; ++i) {
                            const bool b = (j >> i) & 1;
                            if (A.reg_l[i] == x.bit) in = in && (b == (round == 1));
                            else if (b) l |= 1u << cpos[A.reg_l[i]];
                        }
                        if (in) w += fmt(" *(C *)((char *)lds + (xw%d ^ %uu)) = v[%d];", xi_next - 1, swz(l) * csz, j);
                    }
                    ln(sa.reg ? w : w + " }");
                    ln("        lbar();");
                    std::string r = sb.reg ? "       " : fmt("        if (((t >> %d) & 1u) == %du) {", sb.i, round);
                    for (int j = 0; j < NR; ++j) {
                        uint32_t l = 0;
                        bool in = true;
                        for (int i = 0; i < RB; ++i) {
                            const bool b = (j >> i) & 1;
                            if (B.reg_l[i] == x.bit) in = in && (b == (round == 1));
                            else if (b) l |= 1u << cpos[B.reg_l[i]];
                        }
                        if (in)
                            r += fmt(" xt[%d] = *(const C *)((const char *)lds + (xr%d ^ %uu));", j, xi_next - 1,
                                     swz(l) * csz);
                    }
                    ln(sb.reg ? r : r + " }");
                }
                std::string cp = "       ";
                for (int j = 0; j < NR; ++j) cp += fmt(" v[%d] = xt[%d];", j, j);
                ln(cp + " }");
                cur = op.a;
                break;
            }
            ln("        lbar();");
            std::string w = "       ";
            for (int j = 0; j < NR; ++j) {
                uint32_t l = 0;
                for (int i = 0; i < RB; ++i)
                    if ((j >> i) & 1) l |= 1u << A.reg_l[i];
                w += fmt(" *(C *)((char *)lds + (xo%d ^ %uu)) = v[%d];", cur, swz(l) * csz, j);
            }
            ln(w);
            ln("        lbar();");
            std::string r = "       ";
            for (int j = 0; j < NR; ++j) {
                uint32_t l = 0;
                for (int i = 0; i < RB; ++i)
                    if ((j >> i) & 1) l |= 1u << B.reg_l[i];
                r += fmt(" v[%d] = *(const C *)((const char *)lds + (xo%d ^ %uu));", j, op.a, swz(l) * csz);
            }
            ln(r);
            cur = op.a;
            break;
        }
        default: break;
        }
    }
    if (snap(scale_im) != 0.0) {
        std::string e = "        {";
        for (int j = 0; j < NR; ++j)
            e += fmt(" v[%d] = cml(v[%d], %s, %s);", j, j, lit(scale_re).c_str(), lit(scale_im).c_str());
        ln(e + " }");
    } else if (scale_re != 1.0) {
        const double scale = scale_re;
        std::string e = "        {";
        for (int j = 0; j < NR; ++j) e += fmt(" v[%d].x *= %s; v[%d].y *= %s;", j, lit(scale).c_str(), j, lit(scale).c_str());
        ln(e + " }");
    }
    ln("    };");
    ln(fmt("    C v[%d];", NR));
    ln("    unsigned long long c = blockIdx.x;");
    if (PF) ln("    if (c < nchunks) load_chunk(v, chunk_base(c));");
    // Split kernels take exactly one chunk per workgroup (the launch covers
    // every chunk): without a loop the compiler has no loop-invariant values
    // (per-thread phase factors and table entries) to hoist and hold across
    // the whole kernel, which is what the 128-register budget cannot afford.
    if (split && halved) ln("    if (c < nchunks) {");
    else ln("    for (; c < nchunks; c += gridDim.x) {");
    ln(pair ? "        const unsigned long long base = pair_base(c);" : "        const unsigned long long base = chunk_base(c);");
    if (pair) {
        // chunk pairs (c, sigma(c)), moved by the workgroup of the smaller base;
        // every load of both tiles completes before the first store (in place)
        ln("        const unsigned long long pbase = partner(base);");
        ln("        const bool pr = pbase != base;");
        ln(fmt("        C w[%d];", NR));
        ln("        load_chunk(v, base);");
        ln("        if (pr) load_chunk(w, pbase);");
        ln("        run_ops(v, base);");
        ln("        if (pr) run_ops(w, pbase);");
        {
            std::string h = "       ";
            for (int j = 0; j < NR; ++j) h += fmt(" hold(v[%d]);", j);
            ln(h);
            h = "        if (pr) {";
            for (int j = 0; j < NR; ++j) h += fmt(" hold(w[%d]);", j);
            ln(h + " }");
        }
        ln("        __syncthreads();");
        ln("        store_chunk(v, pbase);");
        ln("        if (pr) store_chunk(w, base);");
        ln("    }");
        ln("}");
        return s;
    }
    if (PF) {
        ln(fmt("        C vn[%d];", NR));
        ln("        const unsigned long long cn = c + gridDim.x;");
        ln("        if (cn < nchunks) load_chunk(vn, chunk_base(cn));");
    } else {
        ln("        load_chunk(v, base);");
    }
    ln("        run_ops(v, base);");
    if (relabel) {
        // a thread may store where another thread of the chunk loaded: every
        // thread's loads of the tile complete before the barrier (a barrier
        // alone does not wait for outstanding loads)
        std::string h = "       ";
        for (int j = 0; j < NR; ++j) h += fmt(" hold(v[%d]);", j);
        ln(h);
        ln("        __syncthreads();");
    }
    ln("        store_chunk(v, base);");
    if (PF) {
        std::string cp = "       ";
        for (int j = 0; j < NR; ++j) cp += fmt(" v[%d] = vn[%d];", j, j);
        ln(cp);
    }
    ln("    }");
    ln("}");
    return s;
}

}  // namespace

// ---------------------------------------------------------------- compilation and launch

namespace {

std::mutex cache_mu;
std::unordered_map<std::string, std::shared_ptr<JitModule>> cache;   // by source text
constexpr size_t CACHE_MAX = 512;

int compile_source(const std::string &src, std::vector<char> &code, std::string &err) {
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, src.c_str(), "qsv_pass.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS) {
        err = "hiprtcCreateProgram failed";
        return -1;
    }
    // the same code-generation settings as the library's own device code
    const char *opts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
                          "-packed-fp32-ops", "-mllvm", "-simplifycfg-sink-common=false"};
    const hiprtcResult r = hiprtcCompileProgram(prog, (int)(sizeof(opts) / sizeof(opts[0])), opts);
    if (r != HIPRTC_SUCCESS) {
        size_t ls = 0;
        hiprtcGetProgramLogSize(prog, &ls);
        std::string log(ls, '\0');
        if (ls) hiprtcGetProgramLog(prog, &log[0]);
        err = std::string(hiprtcGetErrorString(r)) + ": " + log.substr(0, 2000);
        hiprtcDestroyProgram(&prog);
        return -1;
    }
    size_t n = 0;
    hiprtcGetCodeSize(prog, &n);
    code.resize(n);
    hiprtcGetCode(prog, code.data());
    hiprtcDestroyProgram(&prog);
    return 0;
}

}  // namespace

std::string pass_jit_source(const PassProgram &prog, int dtype, const JitVariant &v) {
    Gen g(prog, dtype, v);
    return g.source();
}

std::string pass_jit_module_source(const PassProgram &prog) { return prog.jit ? prog.jit->source : std::string(); }

namespace {

// Bytes of scratch (private segment) per lane that the kernel descriptor of
// `kernel` requests in an AMDGPU ELF code object; -1 when it is not found.
long kernel_scratch_bytes(const std::vector<char> &co, const std::string &kernel) {
    const size_t n = co.size();
    if (n < sizeof(Elf64_Ehdr) || std::memcmp(co.data(), ELFMAG, SELFMAG) != 0) return -1;
    Elf64_Ehdr eh;
    std::memcpy(&eh, co.data(), sizeof(eh));
    if (eh.e_shentsize != sizeof(Elf64_Shdr) || eh.e_shoff > n || eh.e_shnum > (n - eh.e_shoff) / sizeof(Elf64_Shdr))
        return -1;
    std::vector<Elf64_Shdr> sh(eh.e_shnum);
    if (eh.e_shnum) std::memcpy(sh.data(), co.data() + eh.e_shoff, eh.e_shnum * sizeof(Elf64_Shdr));
    const std::string kd = kernel + ".kd";
    for (const auto &tab : sh) {
        if (tab.sh_type != SHT_SYMTAB && tab.sh_type != SHT_DYNSYM) continue;
        if (tab.sh_link >= sh.size() || tab.sh_offset > n || tab.sh_size > n - tab.sh_offset) continue;
        const Elf64_Shdr &str = sh[tab.sh_link];
        if (str.sh_offset > n || str.sh_size > n - str.sh_offset) continue;
        for (size_t k = 0; k + 1 <= tab.sh_size / sizeof(Elf64_Sym); ++k) {
            Elf64_Sym sym;
            std::memcpy(&sym, co.data() + tab.sh_offset + k * sizeof(Elf64_Sym), sizeof(sym));
            if (sym.st_name >= str.sh_size) continue;
            const char *nm = co.data() + str.sh_offset + sym.st_name;
            if (strnlen(nm, str.sh_size - sym.st_name) != kd.size() || kd.compare(0, kd.size(), nm, kd.size()) != 0)
                continue;
            if (sym.st_shndx >= sh.size()) return -1;
            const Elf64_Shdr &sec = sh[sym.st_shndx];
            if (sym.st_value < sec.sh_addr) return -1;
            const uint64_t off = sec.sh_offset + (sym.st_value - sec.sh_addr);
            if (off > n || n - off < 8) return -1;
            uint32_t priv = 0;   // kernel descriptor: group segment size, then private segment size
            std::memcpy(&priv, co.data() + off + 4, 4);
            return (long)priv;
        }
    }
    return -1;
}

}  // namespace

// Compiles several generated sources as one program: hiprtc serialises
// compilations within a process and each costs a fixed ~0.25 s on top of
// code generation, so the kernels of a plan share one compilation.  Each
// kernel is renamed qsv_pass_jit_<hash of its source>; sources whose shared
// preamble (the helpers before the kernel) differs go to separate programs.
int compile_batch(const std::vector<std::string> &srcs, std::vector<std::shared_ptr<JitCode>> &codes,
                  std::vector<std::string> &names, std::string &err) {
    const std::string marker = "extern \"C\" __global__";
    const std::string call = std::string(JIT_KERNEL_NAME) + "(";
    codes.assign(srcs.size(), nullptr);
    names.assign(srcs.size(), std::string());
    std::map<std::string, std::vector<size_t>> groups;   // preamble -> sources
    for (size_t u = 0; u < srcs.size(); ++u) {
        const size_t k = srcs[u].find(marker);
        groups[k == std::string::npos ? std::string() : srcs[u].substr(0, k)].push_back(u);
    }
    // kernels are named by a hash of their source (FNV-1a, 48 bits), so a
    // profile names the same pass the same way in every process
    auto fnv = [](const std::string &x) {
        uint64_t h = 14695981039346656037ull;
        for (unsigned char ch : x) h = (h ^ ch) * 1099511628211ull;
        return h & 0xffffffffffffull;
    };
    for (auto &g : groups) {
        std::string prog = g.first;
        std::set<std::string> used;
        for (size_t u : g.second) {
            const std::string &src = srcs[u];
            const size_t k = src.find(marker);
            const size_t c = src.find(call, k == std::string::npos ? 0 : k);
            if (k == std::string::npos || c == std::string::npos) {
                err = "generated pass source without its kernel";
                return -1;
            }
            names[u] = fmt("%s_%012llx", JIT_KERNEL_NAME, (unsigned long long)fnv(src));
            if (!used.insert(names[u]).second) names[u] += fmt("_%zu", u);
            prog += src.substr(k, c - k) + names[u] + "(" + src.substr(c + call.size()) + "\n";
        }
        auto code = std::make_shared<JitCode>();
        if (compile_source(prog, code->code, err)) return -1;
        for (size_t u : g.second) codes[u] = code;
    }
    return 0;
}

// Compiles the passes `progs` (first as their default variant `first`), all
// kernels of a round in one program.  With split exchanges requested, a
// program whose exchanges all split is first compiled as a split kernel,
// with and then without shared phase products; one that fits the 128
// registers of two workgroups per CU with little scratch (SPLIT_SPILL) is
// kept.  Otherwise a persistent prefetching kernel; one whose
// registers spill to scratch is compiled again without shared phase
// products, then without the prefetched chunk, then without both (each frees
// registers).  A prefetching variant is kept if it spills at most a few
// values (measured: cheaper than giving up the prefetch); else the first
// variant without scratch, else the one with the least.
int compile_pass_kernels(const std::vector<const PassProgram *> &progs, int dtype, const std::vector<std::string> &first,
                         const JitVariant &first_variant, std::vector<std::shared_ptr<JitModule>> &out,
                         std::string &err) {
    std::vector<JitVariant> vs;
    if (first_variant.split) {   // split variants first, then the persistent ones
        vs.push_back(first_variant);
        vs.push_back({false, false, true});
    }
    const int base = (int)vs.size();
    vs.push_back(first_variant.split ? JitVariant{true, true, false} : first_variant);
    vs.push_back({false, true, false});
    vs.push_back({true, false, false});
    vs.push_back({false, false, false});
    constexpr long SMALL_SPILL = 16;   // bytes per lane
    // A split kernel is kept with up to this much scratch per lane: it has no
    // prefetched loads for a reload to wait on (30-qubit supremacy-like
    // circuit, complex64: 0.0953 -> 0.0909 s with two more passes split;
    // the QFT unchanged).
    constexpr long SPLIT_SPILL = 256;
    const size_t N = progs.size();
    out.assign(N, nullptr);
    std::vector<long> best_sc(N, -1);
    std::vector<std::vector<std::string>> tried(N);
    std::vector<char> done(N, 0);
    for (int vi = 0; vi < (int)vs.size(); ++vi) {
        std::vector<size_t> items;
        std::vector<std::string> srcs;
        for (size_t i = 0; i < N; ++i) {
            if (done[i]) continue;
            if (vi == base && out[i]) {   // a split kernel within SPLIT_SPILL: keep the best one
                done[i] = 1;
                continue;
            }
            if (vs[vi].split && !exchanges_split(*progs[i])) continue;
            if (vi == base + 2 && out[i] && out[i]->prefetch && best_sc[i] >= 0 && best_sc[i] <= SMALL_SPILL) {
                done[i] = 1;
                continue;
            }
            std::string src = (vi == 0 && !(vs[0].split && !exchanges_split(*progs[i])))
                                  ? first[i] : pass_jit_source(*progs[i], dtype, vs[vi]);
            bool seen = false;
            for (auto &t : tried[i]) seen = seen || t == src;
            if (seen) continue;
            tried[i].push_back(src);
            items.push_back(i);
            srcs.push_back(std::move(src));
        }
        if (items.empty()) continue;
        std::vector<std::shared_ptr<JitCode>> codes;
        std::vector<std::string> names;
        if (compile_batch(srcs, codes, names, err)) {
            if (vi == 0) return -1;
            break;   // keep the variants compiled so far
        }
        for (size_t r = 0; r < items.size(); ++r) {
            const size_t i = items[r];
            const long sc = kernel_scratch_bytes(codes[r]->code, names[r]);
            if (vs[vi].split && (sc < 0 || sc > SPLIT_SPILL)) continue;
            auto m = std::make_shared<JitModule>();
            m->code = codes[r];
            m->kernel = names[r];
            m->source = srcs[r];
            m->prefetch = vs[vi].prefetch && !vs[vi].split && pass_jit_prefetch(*progs[i], dtype);
            m->one_shot = vs[vi].split;   // compiled only for programs whose exchanges all split
            if (!out[i] || (sc >= 0 && (best_sc[i] < 0 || sc < best_sc[i]))) {
                out[i] = m;
                best_sc[i] = sc;
            }
            if (sc <= 0) done[i] = 1;   // no scratch, or a code object this parser does not read: keep it
        }
    }
    for (size_t i = 0; i < N; ++i)
        if (!out[i]) {
            if (err.empty()) err = "no kernel variant of a pass compiled";
            return -1;
        }
    return 0;
}

int jit_compile_plan(qsv_plan *p) {
    std::vector<PassProgram *> progs;
    for (auto &op : p->ops)
        if (op.kind == PlanOp::PASS && !op.pass->jit) progs.push_back(op.pass.get());
    if (progs.empty()) return QSV_OK;
    for (auto *pr : progs) pr->param = p->opts.jit == 2;
    JitVariant v0;
    v0.split = true;
    std::vector<std::string> srcs(progs.size());
    std::vector<std::shared_ptr<JitModule>> mods(progs.size());
    std::vector<size_t> todo;
    {
        std::lock_guard<std::mutex> lk(cache_mu);
        for (size_t i = 0; i < progs.size(); ++i) {
            srcs[i] = pass_jit_source(*progs[i], p->dtype, v0);
            auto it = cache.find(srcs[i]);
            if (it != cache.end()) mods[i] = it->second;
            else todo.push_back(i);
        }
    }
    // distinct sources, compiled together
    std::map<std::string, size_t> first;
    std::vector<size_t> uniq;
    for (size_t i : todo)
        if (first.emplace(srcs[i], i).second) uniq.push_back(i);
    std::vector<const PassProgram *> uprogs;
    std::vector<std::string> usrcs;
    for (size_t i : uniq) {
        uprogs.push_back(progs[i]);
        usrcs.push_back(srcs[i]);
    }
    std::vector<std::shared_ptr<JitModule>> built;
    std::string err;
    if (!uniq.empty() && compile_pass_kernels(uprogs, p->dtype, usrcs, v0, built, err))
        return fail(QSV_ERR_UNSUPPORTED, "pass kernel compilation failed: " + err);
    {
        std::lock_guard<std::mutex> lk(cache_mu);
        if (cache.size() + uniq.size() > CACHE_MAX) cache.clear();   // plans keep their own modules
        for (size_t u = 0; u < uniq.size(); ++u) cache[srcs[uniq[u]]] = built[u];
        for (size_t i : todo) mods[i] = cache[srcs[i]];
    }
    for (size_t i = 0; i < progs.size(); ++i) progs[i]->jit = mods[i];
    p->stats.n_jit_passes = 0;
    for (auto &op : p->ops)
        if (op.kind == PlanOp::PASS && op.pass->jit) p->stats.n_jit_passes++;
    return QSV_OK;
}

int launch_pass_jit(void *state, int n, int dtype, const PassProgram &prog, hipStream_t s) {
    JitModule &jm = *prog.jit;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    hipFunction_t fn;
    int per_cu;
    {
        std::lock_guard<std::mutex> lk(jm.mu);
        JitModule::Loaded &ld = jm.dev[dev];
        if (!ld.fn) {
            hipModule_t mod = nullptr;
            {
                std::lock_guard<std::mutex> lc(jm.code->mu);
                hipModule_t &m = jm.code->mod[dev];
                if (!m && (e = hipModuleLoadData(&m, jm.code->code.data())) != hipSuccess) {
                    m = nullptr;
                    return hip_fail(e, "loading a compiled pass kernel");
                }
                mod = m;
            }
            if ((e = hipModuleGetFunction(&ld.fn, mod, jm.kernel.c_str())) != hipSuccess) {
                ld.fn = nullptr;
                return hip_fail(e, "finding the compiled pass kernel");
            }
            int b = 0;
            if (hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&b, ld.fn, 1 << prog.TB, 0) != hipSuccess || b < 1)
                b = 1;
            ld.grid_per_cu = b;
        }
        fn = ld.fn;
        per_cu = ld.grid_per_cu;
    }
    uint64_t nchunks = 1ull << (n - prog.L);
    if (!prog.pair_sigma.empty()) {
        uint64_t local = 0;
        for (int q : prog.local_sorted) local |= 1ull << q;
        nchunks = pair_work_items(prog.pair_sigma, local);
    }
    const bool pf = jm.prefetch;
    uint64_t g = pf ? (uint64_t)per_cu * device_sm_count() : std::min<uint64_t>(nchunks, 1ull << 20);
    if (jm.one_shot) {   // one workgroup per chunk, no loop in the kernel
        if (nchunks > 0xffffffffull >> prog.TB)
            return fail(QSV_ERR_UNSUPPORTED, "a split-exchange pass kernel takes at most 2^32 lanes in one launch");
        g = nchunks;
    }
    if (g > nchunks) g = nchunks;
    StagingSlot slot;
    int st = upload_pass_program(prog, dtype, s, &slot);
    if (st) return st;
    void *dprog = slot.dev;
    void *args[] = {&state, &dprog, &nchunks};
    e = hipModuleLaunchKernel(fn, (unsigned)g, 1, 1, 1u << prog.TB, 1, 1, 0, s, args, nullptr);
    staging_release(slot, s);
    if (e != hipSuccess) return hip_fail(e, "compiled pass kernel launch");
    return QSV_OK;
}

}  // namespace qsv
