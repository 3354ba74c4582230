// Plans: a circuit turned into the launch sequence that applies it.
//
//   per-gate  one launch per gate (the paper's custom operators, one per gate);
//   greedy    gate fusion of the benchmarks' fusion section (Sec. 3.2): gates
//             are walked in order and a gate joins the most recent block
//             among its qubits' last blocks while the union of qubits stays
//             within kmax; the fused matrix is the product of the members'
//             matrices.  The paper fuses up to two qubits and notes that
//             wider blocks (about five) may help; kmax goes up to 6 here;
//   passes    runs of gates executed in LDS-staged passes (pass_plan.cpp);
//   learned   candidate plans scored by the MLP cost model (cost_model.cpp).
#include <cmath>
#include <cstring>
#include <memory>

#include "plan_internal.h"

namespace qsv {

// Apply a member gate (target block G over local targets lt, controls lc) to
// every column of the 2^kb x 2^kb matrix M (row-major), i.e. M <- U M.
static void left_multiply(std::vector<double> &M, int kb, const std::vector<double> &G, const std::vector<int> &lt,
                          const std::vector<int> &lc) {
    const int d = 1 << kb;
    const int km = (int)lt.size();
    const int gd = 1 << km;
    std::vector<double> out(M.size());
    uint64_t cm = 0;
    for (int q : lc) cm |= 1ull << q;
    for (int i = 0; i < d; ++i) {
        if ((i & cm) != cm) {
            std::memcpy(&out[2 * i * d], &M[2 * i * d], sizeof(double) * 2 * d);
            continue;
        }
        int tau = 0, rest = i;
        for (int j = 0; j < km; ++j) {
            tau |= ((i >> lt[j]) & 1) << (km - 1 - j);
            rest &= ~(1 << lt[j]);
        }
        for (int col = 0; col < d; ++col) {
            double re = 0, im = 0;
            for (int tp = 0; tp < gd; ++tp) {
                int src = rest;
                for (int j = 0; j < km; ++j)
                    if ((tp >> (km - 1 - j)) & 1) src |= 1 << lt[j];
                const double gr = G[2 * (tau * gd + tp)], gi = G[2 * (tau * gd + tp) + 1];
                const double mr = M[2 * (src * d + col)], mi = M[2 * (src * d + col) + 1];
                re += gr * mr - gi * mi;
                im += gr * mi + gi * mr;
            }
            out[2 * (i * d + col)] = re;
            out[2 * (i * d + col) + 1] = im;
        }
    }
    M.swap(out);
}

std::vector<std::vector<int>> greedy_fusion(const std::vector<qsv_gate> &gates, int kmax) {
    std::vector<std::vector<int>> blocks;
    std::vector<uint64_t> bq;     // qubit mask per block
    std::vector<int> last(QSV_MAX_QUBITS, -1);
    for (int gi = 0; gi < (int)gates.size(); ++gi) {
        const qsv_gate &g = gates[gi];
        uint64_t qm = 0;
        int cand = -1;
        for (int j = 0; j < g.k; ++j) qm |= 1ull << g.targets[j];
        for (int j = 0; j < g.c; ++j) qm |= 1ull << g.controls[j];
        for (int q = 0; q < QSV_MAX_QUBITS; ++q)
            if ((qm >> q) & 1) cand = std::max(cand, last[q]);
        int b;
        if (cand >= 0 && __builtin_popcountll(bq[cand] | qm) <= kmax) {
            b = cand;
            bq[b] |= qm;
            blocks[b].push_back(gi);
        } else {
            b = (int)blocks.size();
            blocks.push_back({gi});
            bq.push_back(qm);
        }
        for (int q = 0; q < QSV_MAX_QUBITS; ++q)
            if ((qm >> q) & 1) last[q] = b;
    }
    return blocks;
}

int fused_block(const std::vector<qsv_gate> &gates, const std::vector<int> &members, std::vector<int> &qubits,
                std::vector<double> &M) {
    uint64_t qm = 0;
    for (int gi : members) {
        for (int j = 0; j < gates[gi].k; ++j) qm |= 1ull << gates[gi].targets[j];
        for (int j = 0; j < gates[gi].c; ++j) qm |= 1ull << gates[gi].controls[j];
    }
    qubits.clear();
    for (int q = QSV_MAX_QUBITS - 1; q >= 0; --q)
        if ((qm >> q) & 1) qubits.push_back(q);   // decreasing: qubits[0] is the MSB
    const int kb = (int)qubits.size();
    if (kb > QSV_MAX_TARGETS) return fail(QSV_ERR_ARITY, "fused block wider than 6 qubits");
    const int d = 1 << kb;
    M.assign(2 * d * d, 0.0);
    for (int i = 0; i < d; ++i) M[2 * (i * d + i)] = 1.0;
    int pos[QSV_MAX_QUBITS];
    for (int j = 0; j < kb; ++j) pos[qubits[j]] = kb - 1 - j;
    for (int gi : members) {
        const qsv_gate &g = gates[gi];
        std::vector<double> G;
        int st = gate_target_matrix(g, G);
        if (st) return st;
        std::vector<int> lt, lc;
        for (int j = 0; j < g.k; ++j) lt.push_back(pos[g.targets[j]]);
        for (int j = 0; j < g.c; ++j) lc.push_back(pos[g.controls[j]]);
        left_multiply(M, kb, G, lt, lc);
    }
    return QSV_OK;
}

static double op_bytes(const GateAnalysis &a, int dtype) {
    const double s = dtype == QSV_C64 ? 8.0 : 16.0;
    if (a.members.empty()) return 0.0;
    const double groups = std::ldexp(1.0, a.n - (int)a.sorted_bits.size());
    return 2.0 * groups * (double)a.members.size() * s;
}

static double op_flops(const GateAnalysis &a) {
    const double groups = std::ldexp(1.0, a.n - (int)a.sorted_bits.size());
    const double M = (double)a.members.size();
    if (a.cls == GC_DENSE) return groups * 8.0 * M * M;
    return groups * 6.0 * M;
}

int plan_add_gate_op(qsv_plan *p, const qsv_gate &g) {
    std::vector<double> G;
    int st = gate_target_matrix(g, G);
    if (st) return st;
    PlanOp op;
    op.kind = PlanOp::GATE;
    op.analysis = analyse_gate(p->n, G.data(), g.targets, g.k, g.controls, g.c);
    op.bytes = op_bytes(op.analysis, p->dtype);
    op.flops = op_flops(op.analysis);
    p->ops.push_back(std::move(op));
    p->stats.n_gate_ops++;
    return QSV_OK;
}

int plan_add_block_op(qsv_plan *p, const std::vector<int> &qubits, const std::vector<double> &M, bool allow_mfma) {
    const int kb = (int)qubits.size();
    PlanOp op;
    const bool mfma = allow_mfma && p->dtype == QSV_C64 && kb >= 4 && kb <= 6 && p->n >= kb + 5;
    op.analysis = analyse_gate(p->n, M.data(), qubits.data(), kb, nullptr, 0);
    if (mfma && op.analysis.cls == GC_DENSE && (int)op.analysis.members.size() == (1 << kb)) {
        op.kind = PlanOp::MFMA_BLOCK;
        op.qubits = qubits;
        op.matrix = M;
        const double s = 8.0;
        op.bytes = 2.0 * std::ldexp(1.0, p->n) * s;
        op.flops = std::ldexp(1.0, p->n) * 8.0 * (double)(1 << kb);
        p->stats.n_mfma_blocks++;
    } else {
        op.kind = PlanOp::GATE;
        op.fused = true;
        op.bytes = op_bytes(op.analysis, p->dtype);
        op.flops = op_flops(op.analysis);
    }
    p->stats.n_blocks++;
    p->ops.push_back(std::move(op));
    return QSV_OK;
}

int build_greedy(qsv_plan *p, int kmax, bool allow_mfma) {
    p->blocks = greedy_fusion(p->gates, kmax);
    p->block_of_gate.assign(p->gates.size(), -1);
    for (int b = 0; b < (int)p->blocks.size(); ++b)
        for (int gi : p->blocks[b]) p->block_of_gate[gi] = b;
    for (const auto &members : p->blocks) {
        int st;
        if (members.size() == 1) {
            st = plan_add_gate_op(p, p->gates[members[0]]);
        } else {
            std::vector<int> qubits;
            std::vector<double> M;
            st = fused_block(p->gates, members, qubits, M);
            if (!st) st = plan_add_block_op(p, qubits, M, allow_mfma);
        }
        if (st) return st;
        p->ops.back().gate_ids = members;
    }
    return QSV_OK;
}

void finish_stats(qsv_plan *p) {
    p->stats.n_launches = (int)p->ops.size();
    double b = 0, f = 0;
    for (const auto &op : p->ops) {
        b += op.bytes;
        f += op.flops;
    }
    p->stats.bytes = b;
    p->stats.flops = f;
}

int execute_op(const qsv_plan *p, const PlanOp &op, void *state, hipStream_t s) {
    switch (op.kind) {
    case PlanOp::GATE: return launch_gate(state, p->dtype, op.analysis, s);
    case PlanOp::MFMA_BLOCK:
        return launch_block_mfma(state, p->n, op.matrix.data(), op.qubits.data(), (int)op.qubits.size(), s);
    case PlanOp::PASS:
        return op.pass->jit ? launch_pass_jit(state, p->n, p->dtype, *op.pass, s)
                            : launch_pass_program(state, p->n, p->dtype, *op.pass, s);
    case PlanOp::PERM: return launch_bitperm(state, p->n, p->dtype, op.sigma, s);
    }
    return fail(QSV_ERR_ARG, "internal: unknown op kind");
}

int execute_plan(const qsv_plan *p, void *state, hipStream_t s) {
    for (const auto &op : p->ops) {
        int st = execute_op(p, op, state, s);
        if (st) return st;
    }
    return QSV_OK;
}

}  // namespace qsv

using namespace qsv;

extern "C" {

int qsv_plan_create(int n, int dtype, const qsv_gate *gates, int ngates, const qsv_plan_options *opts,
                    qsv_plan **out) {
    if (!out) return fail(QSV_ERR_NULL, "out is NULL");
    *out = nullptr;
    if (ngates < 0 || (ngates > 0 && !gates)) return fail(QSV_ERR_NULL, "gates is NULL");
    qsv_plan_options o = {QSV_PLAN_PER_GATE, 2, 0, 1, 0};
    if (opts) o = *opts;
    if (o.mode < 0 || o.mode > QSV_PLAN_LEARNED) return fail(QSV_ERR_ARG, "unknown plan mode");
    if (o.kmax == 0) o.kmax = 2;
    if (o.kmax < 1 || o.kmax > QSV_MAX_TARGETS) return fail(QSV_ERR_ARG, "kmax must be in [1, 6]");
    if (o.jit < 0 || o.jit > 2) return fail(QSV_ERR_ARG, "jit must be 0, 1 or 2");
    int st = validate_common(n, dtype, nullptr, 0, nullptr, 0);
    if (st) return st;
    std::unique_ptr<qsv_plan> p(new qsv_plan());
    p->n = n;
    p->dtype = dtype;
    p->opts = o;
    std::memset(&p->stats, 0, sizeof(p->stats));
    for (int i = 0; i < ngates; ++i) {
        const qsv_gate &g = gates[i];
        if ((st = validate_common(n, dtype, g.targets, g.k, g.controls, g.c))) return st;
        if (g.k < 1) return fail(QSV_ERR_ARITY, "gate " + std::to_string(i) + " has no target");
        std::vector<double> G;
        if ((st = gate_target_matrix(g, G))) return st;
        p->gates.push_back(g);
        if (g.kind == QSV_GATE_MATRIX || g.kind == QSV_GATE_DIAG) {
            // keep a private copy of the data
            const size_t cnt = g.kind == QSV_GATE_MATRIX ? (size_t)2 << (2 * g.k) : (size_t)2 << g.k;
            p->data.emplace_back((const double *)g.data, (const double *)g.data + cnt);
            p->gates.back().data = p->data.back().data();
        }
    }
    switch (o.mode) {
    case QSV_PLAN_PER_GATE:
        for (size_t i = 0; i < p->gates.size(); ++i) {
            if ((st = plan_add_gate_op(p.get(), p->gates[i]))) return st;
            p->ops.back().gate_ids = {(int)i};
        }
        break;
    case QSV_PLAN_GREEDY: st = build_greedy(p.get(), o.kmax, o.use_mfma != 0); break;
    case QSV_PLAN_PASSES: st = build_passes(p.get(), o.local_bits); break;
    case QSV_PLAN_LEARNED: st = build_learned(p.get()); break;
    }
    if (st) return st;
    if (o.jit && (st = jit_compile_plan(p.get()))) return st;
    if (p->stats.mode_used == 0 && o.mode != QSV_PLAN_LEARNED) p->stats.mode_used = o.mode;
    finish_stats(p.get());
    *out = p.release();
    return QSV_OK;
}

int qsv_plan_stats_get(const qsv_plan *plan, qsv_plan_stats *out) {
    if (!plan || !out) return fail(QSV_ERR_NULL, "NULL argument");
    *out = plan->stats;
    return QSV_OK;
}

int qsv_plan_blocks(const qsv_plan *plan, int *block_of_gate, int ngates) {
    if (!plan || !block_of_gate) return fail(QSV_ERR_NULL, "NULL argument");
    if (plan->block_of_gate.empty()) return fail(QSV_ERR_ARG, "plan has no fusion blocks");
    if (ngates != (int)plan->gates.size()) return fail(QSV_ERR_ARG, "ngates does not match the plan");
    for (int i = 0; i < ngates; ++i) block_of_gate[i] = plan->block_of_gate[i];
    return QSV_OK;
}

int qsv_plan_execute(const qsv_plan *plan, void *state, void *stream) {
    if (!plan || !state) return fail(QSV_ERR_NULL, "NULL argument");
    if (((uintptr_t)state & 15) != 0) return fail(QSV_ERR_ALIGN, "state must be 16-byte aligned");
    return execute_plan(plan, state, (hipStream_t)stream);
}

int qsv_plan_execute_ops(const qsv_plan *plan, void *state, int first, int count, void *stream) {
    if (!plan || !state) return fail(QSV_ERR_NULL, "NULL argument");
    if (((uintptr_t)state & 15) != 0) return fail(QSV_ERR_ALIGN, "state must be 16-byte aligned");
    if (first < 0 || count < 0 || first + count > (int)plan->ops.size()) return fail(QSV_ERR_ARG, "op range out of bounds");
    for (int i = first; i < first + count; ++i) {
        int st = execute_op(plan, plan->ops[i], state, (hipStream_t)stream);
        if (st) return st;
    }
    return QSV_OK;
}

int qsv_plan_op_info(const qsv_plan *plan, int index, int *kind, double *bytes, double *flops) {
    if (!plan) return fail(QSV_ERR_NULL, "NULL argument");
    if (index < 0 || index >= (int)plan->ops.size()) return fail(QSV_ERR_ARG, "op index out of bounds");
    const PlanOp &op = plan->ops[index];
    if (kind) *kind = (int)op.kind;
    if (bytes) *bytes = op.bytes;
    if (flops) *flops = op.flops;
    return QSV_OK;
}

int qsv_plan_op_gates(const qsv_plan *plan, int index, int *ids, size_t cap, size_t *count) {
    if (!plan || !count) return fail(QSV_ERR_NULL, "NULL argument");
    if (index < 0 || index >= (int)plan->ops.size()) return fail(QSV_ERR_ARG, "op index out of bounds");
    const std::vector<int> &g = plan->ops[index].gate_ids;
    *count = g.size();
    if (ids) {
        if (cap < g.size()) return fail(QSV_ERR_ARG, "buffer too small");
        std::copy(g.begin(), g.end(), ids);
    }
    return QSV_OK;
}

int qsv_plan_op_program(const qsv_plan *plan, int index, void *buf, size_t cap, size_t *size) {
    if (!plan || !size) return fail(QSV_ERR_NULL, "NULL argument");
    if (index < 0 || index >= (int)plan->ops.size()) return fail(QSV_ERR_ARG, "op index out of bounds");
    const PlanOp &op = plan->ops[index];
    if (op.kind != PlanOp::PASS) return fail(QSV_ERR_ARG, "op is not an LDS pass");
    std::vector<uint8_t> blob = op.pass->blob;
    const PassHeaderDev *h = (const PassHeaderDev *)blob.data();
    if (!op.pass->pool.empty())   // an empty vector's data() may be null, which memcpy does not allow
        std::memcpy(blob.data() + h->off_pool, op.pass->pool.data(), op.pass->pool.size() * sizeof(double));
    *size = blob.size();
    if (buf) {
        if (cap < blob.size()) return fail(QSV_ERR_ARG, "buffer too small");
        std::memcpy(buf, blob.data(), blob.size());
    }
    return QSV_OK;
}

int qsv_plan_op_source(const qsv_plan *plan, int index, char *buf, size_t cap, size_t *size) {
    if (!plan || !size) return fail(QSV_ERR_NULL, "NULL argument");
    if (index < 0 || index >= (int)plan->ops.size()) return fail(QSV_ERR_ARG, "op index out of bounds");
    const PlanOp &op = plan->ops[index];
    if (op.kind != PlanOp::PASS) return fail(QSV_ERR_ARG, "op is not an LDS pass");
    const std::string src = op.pass->jit ? pass_jit_module_source(*op.pass)
                                         : pass_jit_source(*op.pass, plan->dtype, JitVariant());
    *size = src.size() + 1;
    if (buf) {
        if (cap < src.size() + 1) return fail(QSV_ERR_ARG, "buffer too small");
        std::memcpy(buf, src.c_str(), src.size() + 1);
    }
    return QSV_OK;
}

void qsv_plan_destroy(qsv_plan *plan) { delete plan; }

}  // extern "C"
