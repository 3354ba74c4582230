// Learned plan choice: an MLP cost model scores the candidate plans of a
// circuit and the cheapest is kept; greedy fusion (Sec. 3.2 of the paper,
// two-qubit blocks) is the fallback when no model is loaded.
//
// The model maps the features of one op (qsv_plan_op_features) to the log of
// its run time; a plan's predicted time is the sum over its ops.  Candidate
// plans: per-gate, greedy fusion with kmax = 2..5 (matrix-core blocks for
// complex64), and LDS passes with the default and one smaller chunk
// (compiled when the plan asks for compiled passes; only the chosen plan's
// passes are compiled).
// Inference runs on the GPU with the library's own MLP kernels.
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>

#include "plan_internal.h"

namespace qsv {

int mlp_check_sizes(const int *sizes, int nlayers);
int mlp_param_count(const int *sizes, int nlayers);
int mlp_forward(const float *params, const int *sizes, int nlayers, const float *X, int B, float *acts, float *pred,
                hipStream_t s);

namespace {
struct CostModel {
    std::vector<float> params;
    std::vector<int> sizes;
    std::vector<float> mean, scale;
};
std::mutex g_model_mu;
std::shared_ptr<const CostModel> g_model;
}  // namespace

void op_features(const qsv_plan *p, const PlanOp &op, float *f) {
    std::memset(f, 0, sizeof(float) * QSV_COST_FEATURES);
    f[0] = (float)p->n;
    f[1] = (float)p->dtype;
    int variant = 0;
    std::vector<int> qubits;
    double extra = 0;
    switch (op.kind) {
    case PlanOp::GATE:
        variant = op.fused ? 1 : 0;
        qubits = op.analysis.sorted_bits;
        extra = std::log2((double)std::max<size_t>(1, op.analysis.members.size()));
        break;
    case PlanOp::MFMA_BLOCK:
        variant = 2;
        qubits = op.qubits;
        extra = (double)op.qubits.size();
        break;
    case PlanOp::PASS:
        variant = p->opts.jit ? 5 : 3;
        qubits = op.pass->local_sorted;
        extra = (double)op.pass->ops.size();
        break;
    case PlanOp::PERM:
        variant = 4;
        for (int b = 0; b < (int)op.sigma.size(); ++b)
            if (op.sigma[b] != b) qubits.push_back(b);
        break;
    }
    f[2 + variant] = 1.0f;
    f[8] = (float)qubits.size();
    int low = 0;
    for (int q : qubits)
        if (q < 5) ++low;
    f[9] = (float)low;
    f[10] = (float)std::log2(std::max(1.0, op.bytes));
    f[11] = (float)std::log2(1.0 + op.flops);
    f[12] = (float)extra;
}

// Predicted seconds of every candidate (sum over its ops), on the GPU.
static int predict(const CostModel &m, const std::vector<const qsv_plan *> &cands, std::vector<double> &out) {
    std::vector<float> X;
    std::vector<int> owner;
    for (size_t c = 0; c < cands.size(); ++c)
        for (const auto &op : cands[c]->ops) {
            float f[QSV_COST_FEATURES];
            op_features(cands[c], op, f);
            for (int i = 0; i < QSV_COST_FEATURES; ++i) X.push_back((f[i] - m.mean[i]) / m.scale[i]);
            owner.push_back((int)c);
        }
    const int B = (int)owner.size();
    out.assign(cands.size(), 0.0);
    if (B == 0) return QSV_OK;
    const int nl = (int)m.sizes.size() - 1;
    size_t acts = 0;
    for (int l = 1; l <= nl; ++l) acts += (size_t)B * m.sizes[l];
    float *dp = nullptr, *dx = nullptr, *da = nullptr, *dpred = nullptr;
    auto cleanup = [&]() {
        if (dp) (void)dev_free(dp);
        if (dx) (void)dev_free(dx);
        if (da) (void)dev_free(da);
        if (dpred) (void)dev_free(dpred);
    };
    hipError_t e = dev_malloc((void **)&dp, sizeof(float) * m.params.size());
    if (e == hipSuccess) e = dev_malloc((void **)&dx, sizeof(float) * X.size());
    if (e == hipSuccess) e = dev_malloc((void **)&da, sizeof(float) * acts);
    if (e == hipSuccess) e = dev_malloc((void **)&dpred, sizeof(float) * B);
    if (e == hipSuccess) e = hipMemcpy(dp, m.params.data(), sizeof(float) * m.params.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dx, X.data(), sizeof(float) * X.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        cleanup();
        return hip_fail(e, "cost model buffers");
    }
    int st = mlp_forward(dp, m.sizes.data(), nl, dx, B, da, dpred, nullptr);
    std::vector<float> pred(B);
    if (!st) {
        e = hipMemcpy(pred.data(), dpred, sizeof(float) * B, hipMemcpyDeviceToHost);
        if (e != hipSuccess) st = hip_fail(e, "cost model readback");
    }
    cleanup();
    if (st) return st;
    for (int i = 0; i < B; ++i) out[owner[i]] += std::exp((double)pred[i]);
    return QSV_OK;
}

static std::unique_ptr<qsv_plan> candidate(const qsv_plan *p, int mode, int kmax, int local_bits, int use_mfma) {
    std::unique_ptr<qsv_plan> c(new qsv_plan());
    c->n = p->n;
    c->dtype = p->dtype;
    c->gates = p->gates;
    c->opts = {mode, kmax, local_bits, use_mfma, p->opts.jit};
    std::memset(&c->stats, 0, sizeof(c->stats));
    int st = QSV_OK;
    if (mode == QSV_PLAN_PER_GATE) {
        for (size_t i = 0; i < c->gates.size() && !st; ++i)
            if (!(st = plan_add_gate_op(c.get(), c->gates[i]))) c->ops.back().gate_ids = {(int)i};
    } else if (mode == QSV_PLAN_GREEDY) {
        st = build_greedy(c.get(), kmax, use_mfma != 0);
    } else {
        st = build_passes(c.get(), local_bits);
    }
    if (st) return nullptr;
    c->stats.mode_used = mode;
    finish_stats(c.get());
    return c;
}

int build_learned(qsv_plan *p) {
    std::shared_ptr<const CostModel> m;
    {
        std::lock_guard<std::mutex> lk(g_model_mu);
        m = g_model;
    }
    const int kfb = p->opts.kmax > 0 ? p->opts.kmax : 2;
    if (!m) {
        int st = build_greedy(p, kfb, p->opts.use_mfma != 0);
        p->stats.mode_used = QSV_PLAN_GREEDY;
        return st;
    }
    std::vector<std::unique_ptr<qsv_plan>> owned;
    const int mf = p->opts.use_mfma != 0 ? 1 : 0;
    owned.push_back(candidate(p, QSV_PLAN_PER_GATE, 1, 0, 0));
    for (int k = 2; k <= 5; ++k) owned.push_back(candidate(p, QSV_PLAN_GREEDY, k, 0, mf));
    const int rb_max = p->dtype == QSV_C64 ? 5 : 4;
    const int Ld = rb_max + (p->opts.jit ? PASS_JIT_THREAD_BITS : PASS_THREAD_BITS);
    if (p->n >= Ld) owned.push_back(candidate(p, QSV_PLAN_PASSES, 0, Ld, 0));
    if (p->n >= Ld - 1) owned.push_back(candidate(p, QSV_PLAN_PASSES, 0, Ld - 1, 0));
    std::vector<const qsv_plan *> cands;
    for (auto &c : owned)
        if (c) cands.push_back(c.get());
    if (cands.empty()) {   // no candidate could be built: the documented fallback
        int st2 = build_greedy(p, kfb, p->opts.use_mfma != 0);
        p->stats.mode_used = QSV_PLAN_GREEDY;
        return st2;
    }
    std::vector<double> t;
    int st = predict(*m, cands, t);
    if (st) return st;
    size_t best = 0;
    for (size_t i = 1; i < cands.size(); ++i)
        if (t[i] < t[best]) best = i;
    const qsv_plan *b = cands[best];
    p->ops = b->ops;
    p->blocks = b->blocks;
    p->block_of_gate = b->block_of_gate;
    const int mode_used = b->stats.mode_used;
    p->stats = b->stats;
    p->stats.mode_used = mode_used;
    p->stats.predicted_s = t[best];
    return QSV_OK;
}

}  // namespace qsv

using namespace qsv;

extern "C" {

int qsv_cost_model_set(const float *params, const int *sizes, int nlayers, const float *feat_mean,
                       const float *feat_scale) {
    if (nlayers == 0) {
        std::lock_guard<std::mutex> lk(g_model_mu);
        g_model.reset();
        return QSV_OK;
    }
    int st = mlp_check_sizes(sizes, nlayers);
    if (st) return st;
    if (sizes[0] != QSV_COST_FEATURES) return fail(QSV_ERR_ARG, "the model input width must be QSV_COST_FEATURES");
    if (!params || !feat_mean || !feat_scale) return fail(QSV_ERR_NULL, "NULL argument");
    auto m = std::make_shared<CostModel>();
    m->params.assign(params, params + mlp_param_count(sizes, nlayers));
    m->sizes.assign(sizes, sizes + nlayers + 1);
    m->mean.assign(feat_mean, feat_mean + QSV_COST_FEATURES);
    m->scale.assign(feat_scale, feat_scale + QSV_COST_FEATURES);
    for (float s : m->scale)
        if (!(s > 0.0f)) return fail(QSV_ERR_ARG, "feature scales must be positive");
    std::lock_guard<std::mutex> lk(g_model_mu);
    g_model = m;
    return QSV_OK;
}

int qsv_plan_op_features(const qsv_plan *plan, int index, float *out) {
    if (!plan || !out) return fail(QSV_ERR_NULL, "NULL argument");
    if (index < 0 || index >= (int)plan->ops.size()) return fail(QSV_ERR_ARG, "op index out of bounds");
    op_features(plan, plan->ops[index], out);
    return QSV_OK;
}

}  // extern "C"
