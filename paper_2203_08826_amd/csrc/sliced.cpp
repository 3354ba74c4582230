// States larger than device memory (the multi-device scheme of the paper's
// multi-GPU section, on one re-used GPU): the state stays in host memory and
// only slices of it visit the device.
//
// The state of n qubits is cut into 2^(n-m) slices of 2^m amplitudes along
// its top n - m ("global") qubits.  The circuit is cut into phases: a phase
// is a run of gates whose non-diagonal targets are local qubits (below m) or
// one of at most `a` global qubits made "active" for the phase.  A phase
// runs group by group: a group is the 2^|A| slices that differ only in the
// active qubits, copied into one device buffer of 2^(m+|A|) amplitudes in
// which active qubit A_i is bit m + i.  The other global qubits have fixed
// values within a group, so a control on one of them either drops (value 1)
// or removes the gate for the group (value 0), and a diagonal gate on them
// reduces to its entries at those values.  Each group runs a plan of its
// resolved gates (per-gate kernels or LDS passes); groups with the same
// resolved gates share a plan.  Copies run on two streams of their own, the
// next group's upload and the previous group's download overlapping the
// current group's kernels (two device buffers); the first group of a phase
// waits for every download of the phase before it.
#include <complex>
#include <map>

#include "plan_internal.h"

namespace qsv {

namespace {

struct Res {   // one gate resolved for a group
    qsv_gate g;
    std::vector<double> data;   // MATRIX / DIAG entries when rewritten
};

bool is_diagonal(const std::vector<double> &G, int k) {
    const int d = 1 << k;
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c)
            if (r != c && (G[2 * (r * d + c)] != 0.0 || G[2 * (r * d + c) + 1] != 0.0)) return false;
    return true;
}

// The gate `g` for a group: `act[q]` is the buffer bit of qubit q (local and
// active qubits), or -1 for an inactive global qubit whose value is
// bit(q) of `fixed`.  Returns false when the gate does nothing for the group.
bool resolve(const qsv_gate &g, const std::vector<double> &G, bool diag, const std::vector<int> &act, uint64_t fixed,
             Res &out) {
    qsv_gate r = g;
    r.c = 0;
    for (int j = 0; j < g.c; ++j) {
        const int q = g.controls[j];
        if (act[q] < 0) {
            if (!((fixed >> q) & 1)) return false;   // control 0 for the whole group
            continue;                                 // control 1: always on
        }
        r.controls[r.c++] = act[q];
    }
    bool all_active = true;
    for (int j = 0; j < g.k; ++j)
        if (act[g.targets[j]] < 0) all_active = false;
    if (all_active) {
        for (int j = 0; j < g.k; ++j) r.targets[j] = act[g.targets[j]];
        out.g = r;
        if (g.kind == QSV_GATE_MATRIX || g.kind == QSV_GATE_DIAG) {
            const size_t cnt = g.kind == QSV_GATE_MATRIX ? (size_t)2 << (2 * g.k) : (size_t)2 << g.k;
            out.data.assign((const double *)g.data, (const double *)g.data + cnt);
        }
        return true;
    }
    // a diagonal gate with inactive targets: its entries at their values
    if (!diag) return false;   // excluded by the phase cut
    const int d = 1 << g.k;
    std::vector<int> keep;     // positions j of targets still acting
    int fixed_tau = 0;         // the fixed targets' bits in the gate index
    for (int j = 0; j < g.k; ++j) {
        const int q = g.targets[j];
        if (act[q] < 0) {
            if ((fixed >> q) & 1) fixed_tau |= 1 << (g.k - 1 - j);
        } else {
            keep.push_back(j);
        }
    }
    const int kr = (int)keep.size();
    std::vector<double> dg(2 << kr);
    for (int tr = 0; tr < (1 << kr); ++tr) {
        int tau = fixed_tau;
        for (int i = 0; i < kr; ++i)
            if ((tr >> (kr - 1 - i)) & 1) tau |= 1 << (g.k - 1 - keep[i]);
        dg[2 * tr] = G[2 * (tau * d + tau)];
        dg[2 * tr + 1] = G[2 * (tau * d + tau) + 1];
    }
    if (kr == 0) {
        // a factor on the whole group where the remaining controls hold:
        // a diagonal (1, f) on one control, the others controlling it
        if (r.c == 0) {
            r.k = 0;   // marks a scale of the whole buffer by dg
            out.g = r;
            out.data = dg;
            return true;
        }
        r.kind = QSV_GATE_DIAG;
        r.k = 1;
        r.targets[0] = r.controls[r.c - 1];
        r.c -= 1;
        out.g = r;
        out.data = {1.0, 0.0, dg[0], dg[1]};
        return true;
    }
    r.kind = QSV_GATE_DIAG;
    r.k = kr;
    for (int i = 0; i < kr; ++i) r.targets[i] = act[g.targets[keep[i]]];
    out.g = r;
    out.data = dg;
    return true;
}

struct Phase {
    int first = 0, end = 0;    // gates [first, end)
    std::vector<int> active;   // global qubits, buffer bits m, m+1, ...
};

struct Task {
    const Phase *ph;
    uint64_t fixed;            // inactive global bits of the group (in qubit positions)
    qsv_plan *plan;            // gates of the group (may be empty: nullptr)
    std::complex<double> scale;
};

}  // namespace

}  // namespace qsv

using namespace qsv;

extern "C" {

int qsv_sliced_run(void *host_state, int n, int dtype, const qsv_gate *gates, int ngates, int local_qubits,
                   int active_qubits, int mode, void *stream) {
    int st = validate_common(n, dtype, nullptr, 0, nullptr, 0);
    if (st) return st;
    if (!host_state) return fail(QSV_ERR_NULL, "host_state is NULL");
    if (ngates < 0 || (ngates > 0 && !gates)) return fail(QSV_ERR_NULL, "gates is NULL");
    const int m = local_qubits, a = active_qubits;
    if (m < 1 || m > n) return fail(QSV_ERR_ARG, "local_qubits must be in [1, n]");
    if (a < 0 || a > n - m || a > 8) return fail(QSV_ERR_ARG, "active_qubits must be in [0, min(8, n - local_qubits)]");
    if (mode != QSV_PLAN_PER_GATE && mode != QSV_PLAN_PASSES) return fail(QSV_ERR_ARG, "mode must be per-gate or passes");
    const size_t esz = dtype == QSV_C64 ? 8 : 16;
    // matrices and the diagonal test, once per gate
    std::vector<std::vector<double>> mats(ngates);
    std::vector<char> diag(ngates);
    for (int i = 0; i < ngates; ++i) {
        const qsv_gate &g = gates[i];
        if ((st = validate_common(n, dtype, g.targets, g.k, g.controls, g.c))) return st;
        if (g.k < 1) return fail(QSV_ERR_ARITY, "gate " + std::to_string(i) + " has no target");
        if ((st = gate_target_matrix(g, mats[i]))) return st;
        diag[i] = is_diagonal(mats[i], g.k);
    }
    // phases: a gate whose non-diagonal targets are global makes them active
    std::vector<Phase> phases;
    {
        Phase cur;
        for (int i = 0; i < ngates; ++i) {
            const qsv_gate &g = gates[i];
            std::vector<int> need;
            if (!diag[i])
                for (int j = 0; j < g.k; ++j)
                    if (g.targets[j] >= m) need.push_back(g.targets[j]);
            if ((int)need.size() > a)
                return fail(QSV_ERR_ARG, "gate " + std::to_string(i) + " has more global targets than active_qubits");
            std::vector<int> un = cur.active;
            for (int q : need)
                if (std::find(un.begin(), un.end(), q) == un.end()) un.push_back(q);
            if ((int)un.size() > a) {
                cur.end = i;
                phases.push_back(cur);
                cur = Phase();
                cur.first = i;
                un = need;
            }
            cur.active = un;
        }
        cur.end = ngates;
        phases.push_back(cur);
    }
    // device buffers: two groups of the largest phase
    int amax = 0;
    for (auto &ph : phases) amax = std::max(amax, (int)ph.active.size());
    const size_t gbytes = esz << (m + amax);
    void *buf[2] = {nullptr, nullptr};
    hipStream_t cs = (hipStream_t)stream, sin = nullptr, sout = nullptr;
    hipEvent_t ev_in[2] = {nullptr, nullptr}, ev_comp[2] = {nullptr, nullptr}, ev_out[2] = {nullptr, nullptr};
    std::vector<std::unique_ptr<qsv_plan, void (*)(qsv_plan *)>> plans;
    auto cleanup = [&]() {
        if (sin) (void)hipStreamSynchronize(sin);
        if (sout) (void)hipStreamSynchronize(sout);
        (void)hipStreamSynchronize(cs);
        for (int b = 0; b < 2; ++b) {
            if (buf[b]) (void)dev_free(buf[b]);
            if (ev_in[b]) (void)hipEventDestroy(ev_in[b]);
            if (ev_comp[b]) (void)hipEventDestroy(ev_comp[b]);
            if (ev_out[b]) (void)hipEventDestroy(ev_out[b]);
        }
        if (sin) (void)hipStreamDestroy(sin);
        if (sout) (void)hipStreamDestroy(sout);
    };
    hipError_t e = hipSuccess;
#define SL_CHECK(expr)                                     \
    do {                                                   \
        if ((e = (expr)) != hipSuccess) {                  \
            const int r_ = hip_fail(e, #expr);             \
            cleanup();                                     \
            return r_;                                     \
        }                                                  \
    } while (0)
    for (int b = 0; b < 2; ++b) {
        SL_CHECK(dev_malloc(&buf[b], gbytes));
        SL_CHECK(hipEventCreateWithFlags(&ev_in[b], hipEventDisableTiming));
        SL_CHECK(hipEventCreateWithFlags(&ev_comp[b], hipEventDisableTiming));
        SL_CHECK(hipEventCreateWithFlags(&ev_out[b], hipEventDisableTiming));
    }
    SL_CHECK(hipStreamCreateWithFlags(&sin, hipStreamNonBlocking));
    SL_CHECK(hipStreamCreateWithFlags(&sout, hipStreamNonBlocking));
    for (int b = 0; b < 2; ++b) SL_CHECK(hipEventRecord(ev_out[b], sout));   // both buffers free
    // tasks: every group of every phase, with its plan
    std::vector<Task> tasks;
    for (auto &ph : phases) {
        std::vector<int> act(n, -1);
        for (int q = 0; q < m; ++q) act[q] = q;
        for (size_t i = 0; i < ph.active.size(); ++i) act[ph.active[i]] = m + (int)i;
        uint64_t amask = 0;
        for (int q : ph.active) amask |= 1ull << q;
        std::vector<int> inactive;
        for (int q = m; q < n; ++q)
            if (!((amask >> q) & 1)) inactive.push_back(q);
        std::map<std::vector<char>, size_t> by_sig;   // resolved gates -> plan index
        const int nb = m + (int)ph.active.size();
        for (uint64_t gi = 0; gi < (1ull << inactive.size()); ++gi) {
            uint64_t fixed = 0;
            for (size_t b = 0; b < inactive.size(); ++b)
                if ((gi >> b) & 1) fixed |= 1ull << inactive[b];
            std::vector<Res> rs;
            std::complex<double> scale(1.0, 0.0);
            for (int i = ph.first; i < ph.end; ++i) {
                Res r;
                if (!resolve(gates[i], mats[i], diag[i] != 0, act, fixed, r)) continue;
                if (r.g.k == 0) {
                    scale *= std::complex<double>(r.data[0], r.data[1]);
                    continue;
                }
                rs.push_back(std::move(r));
            }
            std::vector<qsv_gate> gl;
            for (auto &r : rs) {
                gl.push_back(r.g);
                if (!r.data.empty()) gl.back().data = r.data.data();
            }
            // signature: the resolved gates, byte for byte, with their data
            std::vector<char> sig;
            for (size_t k = 0; k < gl.size(); ++k) {
                qsv_gate c = gl[k];
                c.data = nullptr;
                sig.insert(sig.end(), (const char *)&c, (const char *)&c + sizeof(c));
                sig.insert(sig.end(), (const char *)rs[k].data.data(), (const char *)(rs[k].data.data() + rs[k].data.size()));
            }
            qsv_plan *pl = nullptr;
            auto it = by_sig.find(sig);
            if (it != by_sig.end()) {
                pl = plans[it->second].get();
            } else if (!gl.empty()) {
                qsv_plan_options o = {mode, 2, 0, 0, 0};
                if ((st = qsv_plan_create(nb, dtype, gl.data(), (int)gl.size(), &o, &pl))) {
                    cleanup();
                    return st;
                }
                plans.emplace_back(pl, qsv_plan_destroy);
                by_sig[sig] = plans.size() - 1;
            }
            tasks.push_back({&ph, fixed, pl, scale});
        }
    }
    // host address of slice j (active bits) of a group
    auto slice_host = [&](const Task &t, uint64_t j) {
        uint64_t s = t.fixed;
        for (size_t i = 0; i < t.ph->active.size(); ++i)
            if ((j >> i) & 1) s |= 1ull << t.ph->active[i];
        return (char *)host_state + s * esz;   // s: the slice's first amplitude (bits below m are 0)
    };
    const size_t sbytes = esz << m;
    // The upload of task i waits for the download of the buffer's previous
    // task; across a phase boundary it also waits for every download before
    // it, since the new phase's groups read slices the old phase wrote.
    auto upload = [&](size_t i, bool all) -> hipError_t {
        const Task &t = tasks[i];
        const int b = (int)(i & 1);
        hipError_t r = hipStreamWaitEvent(sin, ev_out[b], 0);
        if (r != hipSuccess) return r;
        if (all && (r = hipStreamWaitEvent(sin, ev_out[b ^ 1], 0)) != hipSuccess) return r;
        for (uint64_t j = 0; j < (1ull << t.ph->active.size()); ++j)
            if ((r = hipMemcpyAsync((char *)buf[b] + j * sbytes, slice_host(t, j), sbytes, hipMemcpyHostToDevice, sin)) !=
                hipSuccess)
                return r;
        return hipEventRecord(ev_in[b], sin);
    };
    if (!tasks.empty()) SL_CHECK(upload(0, false));
    for (size_t i = 0; i < tasks.size(); ++i) {
        const Task &t = tasks[i];
        const int b = (int)(i & 1);
        // within a phase the next group's upload overlaps this group's work
        const bool next_same = i + 1 < tasks.size() && tasks[i + 1].ph == t.ph;
        if (next_same) SL_CHECK(upload(i + 1, false));
        SL_CHECK(hipStreamWaitEvent(cs, ev_in[b], 0));
        const int nb = m + (int)t.ph->active.size();
        if (t.plan && (st = qsv_plan_execute(t.plan, buf[b], cs))) {
            cleanup();
            return st;
        }
        if (t.scale != std::complex<double>(1.0, 0.0) && (st = launch_scale(buf[b], nb, dtype, t.scale.real(), t.scale.imag(), cs))) {
            cleanup();
            return st;
        }
        SL_CHECK(hipEventRecord(ev_comp[b], cs));
        SL_CHECK(hipStreamWaitEvent(sout, ev_comp[b], 0));
        for (uint64_t j = 0; j < (1ull << t.ph->active.size()); ++j)
            SL_CHECK(hipMemcpyAsync(slice_host(t, j), (char *)buf[b] + j * sbytes, sbytes, hipMemcpyDeviceToHost, sout));
        SL_CHECK(hipEventRecord(ev_out[b], sout));
        if (i + 1 < tasks.size() && !next_same) SL_CHECK(upload(i + 1, true));
    }
#undef SL_CHECK
    e = hipStreamSynchronize(sout);
    cleanup();
    if (e != hipSuccess) return hip_fail(e, "sliced run");
    return QSV_OK;
}

}  // extern "C"
