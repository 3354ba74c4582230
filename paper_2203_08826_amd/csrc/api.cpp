// Host side of libqsv: errors, validation, gate matrices, the analysis that
// reduces a gate to the amplitudes it changes, and the per-gate entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "qsv_internal.h"

namespace qsv {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }
void clear_error() { g_last_error.clear(); }
int fail(int code, const std::string &msg) {
    g_last_error = msg;
    return code;
}
int hip_fail(hipError_t e, const char *where) {
    g_last_error = std::string(where) + ": " + hipGetErrorString(e);
    return QSV_ERR_HIP;
}

int device_sm_count() {
    static int cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (cached[dev] == 0) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
        cached[dev] = v;
    }
    return cached[dev];
}

// ---------------------------------------------------------------- validation

int validate_common(int n, int dtype, const int *targets, int k, const int *controls, int c) {
    if (dtype != QSV_C64 && dtype != QSV_C128) return fail(QSV_ERR_DTYPE, "dtype must be QSV_C64 or QSV_C128");
    if (n < 1 || n > QSV_MAX_QUBITS) return fail(QSV_ERR_NQUBITS, "n must be in [1, 40]");
    if (k < 0 || k > QSV_MAX_TARGETS) return fail(QSV_ERR_ARITY, "number of targets must be in [0, 6]");
    if (c < 0 || c > QSV_MAX_CONTROLS) return fail(QSV_ERR_ARITY, "number of controls must be in [0, 8]");
    if (k + c > n) return fail(QSV_ERR_ARITY, "targets + controls exceed the number of qubits");
    if ((k > 0 && !targets) || (c > 0 && !controls)) return fail(QSV_ERR_NULL, "qubit list is NULL");
    uint64_t seen = 0;
    for (int i = 0; i < k + c; ++i) {
        const int q = i < k ? targets[i] : controls[i - k];
        if (q < 0 || q >= n) return fail(QSV_ERR_QUBIT_RANGE, "qubit index " + std::to_string(q) + " outside [0, n)");
        if (seen & (1ull << q)) return fail(QSV_ERR_QUBIT_DUP, "qubit " + std::to_string(q) + " repeats");
        seen |= 1ull << q;
    }
    return QSV_OK;
}

static int check_state(const void *state) {
    if (!state) return fail(QSV_ERR_NULL, "state is NULL");
    if (((uintptr_t)state & 15) != 0) return fail(QSV_ERR_ALIGN, "state must be 16-byte aligned");
    return QSV_OK;
}

// ---------------------------------------------------------------- gate matrices

typedef std::complex<double> zc;

static void put(std::vector<double> &m, int i, zc v) {
    m[2 * i] = v.real();
    m[2 * i + 1] = v.imag();
}

static int expected_targets(int kind) {
    switch (kind) {
    case QSV_GATE_SWAP:
    case QSV_GATE_FSIM: return 2;
    case QSV_GATE_MATRIX:
    case QSV_GATE_DIAG: return -1;
    default: return 1;
    }
}

// Standard gate definitions (the paper names the gates but does not write
// their matrices): rotations exp(-i theta P / 2), U1 = diag(1, e^{i phi}),
// fSim in the Foxen et al. (2020) convention, principal square roots of X,
// Y and W = (X + Y)/sqrt(2).
int gate_target_matrix(const qsv_gate &g, std::vector<double> &out) {
    const int k = g.k;
    if (k < 1 || k > QSV_MAX_TARGETS) return fail(QSV_ERR_ARITY, "gate needs 1..6 targets");
    const int want = expected_targets(g.kind);
    if (want > 0 && want != k) return fail(QSV_ERR_ARITY, "wrong number of targets for the gate kind");
    const int d = 1 << k;
    out.assign(2 * d * d, 0.0);
    const zc I(0, 1);
    const double r2 = 1.0 / std::sqrt(2.0);
    auto sqrtp = [&](zc p00, zc p01, zc p10, zc p11) {
        const zc a = 0.5 * zc(1, 1), b = 0.5 * zc(1, -1);
        put(out, 0, a + b * p00);
        put(out, 1, b * p01);
        put(out, 2, b * p10);
        put(out, 3, a + b * p11);
    };
    const double th = g.params[0], ph = g.params[1];
    switch (g.kind) {
    case QSV_GATE_MATRIX:
        if (!g.data) return fail(QSV_ERR_NULL, "MATRIX gate without data");
        std::memcpy(out.data(), g.data, sizeof(double) * 2 * d * d);
        break;
    case QSV_GATE_DIAG:
        if (!g.data) return fail(QSV_ERR_NULL, "DIAG gate without data");
        for (int i = 0; i < d; ++i) {
            const double *z = (const double *)g.data + 2 * i;
            put(out, i * d + i, zc(z[0], z[1]));
        }
        break;
    case QSV_GATE_H: put(out, 0, r2); put(out, 1, r2); put(out, 2, r2); put(out, 3, -r2); break;
    case QSV_GATE_X: put(out, 1, 1.0); put(out, 2, 1.0); break;
    case QSV_GATE_Y: put(out, 1, -I); put(out, 2, I); break;
    case QSV_GATE_Z: put(out, 0, 1.0); put(out, 3, -1.0); break;
    case QSV_GATE_SX: sqrtp(0, 1, 1, 0); break;
    case QSV_GATE_SY: sqrtp(0, -I, I, 0); break;
    case QSV_GATE_SW: sqrtp(0, r2 * (1.0 - I), r2 * (1.0 + I), 0); break;
    case QSV_GATE_RX:
        put(out, 0, std::cos(th / 2)); put(out, 1, -I * std::sin(th / 2));
        put(out, 2, -I * std::sin(th / 2)); put(out, 3, std::cos(th / 2));
        break;
    case QSV_GATE_RY:
        put(out, 0, std::cos(th / 2)); put(out, 1, -std::sin(th / 2));
        put(out, 2, std::sin(th / 2)); put(out, 3, std::cos(th / 2));
        break;
    case QSV_GATE_RZ: put(out, 0, std::exp(-0.5 * I * th)); put(out, 3, std::exp(0.5 * I * th)); break;
    case QSV_GATE_U1: put(out, 0, 1.0); put(out, 3, std::exp(I * th)); break;
    case QSV_GATE_SWAP: put(out, 0, 1.0); put(out, 6, 1.0); put(out, 9, 1.0); put(out, 15, 1.0); break;
    case QSV_GATE_FSIM:
        put(out, 0, 1.0);
        put(out, 5, std::cos(th)); put(out, 6, -I * std::sin(th));
        put(out, 9, -I * std::sin(th)); put(out, 10, std::cos(th));
        put(out, 15, std::exp(-I * ph));
        break;
    default: return fail(QSV_ERR_ARG, "unknown gate kind " + std::to_string(g.kind));
    }
    return QSV_OK;
}

// ---------------------------------------------------------------- analysis

static int pad_size(int m, const int *sizes, int nsizes) {
    for (int i = 0; i < nsizes; ++i)
        if (sizes[i] >= m) return sizes[i];
    return -1;
}

double GateAnalysis::touched_fraction() const {
    return (double)members.size() / (double)(1ull << sorted_bits.size());
}

GateAnalysis analyse_gate(int n, const double *G, const int *targets, int k, const int *controls, int c) {
    GateAnalysis a;
    a.n = n;
    a.k = k;
    for (int i = 0; i < k; ++i) a.sorted_bits.push_back(targets[i]);
    for (int i = 0; i < c; ++i) {
        a.sorted_bits.push_back(controls[i]);
        a.cmask |= 1ull << controls[i];
    }
    std::sort(a.sorted_bits.begin(), a.sorted_bits.end());
    const int d = 1 << k;
    std::vector<uint64_t> all_offs(d);
    for (int t = 0; t < d; ++t) {
        uint64_t o = 0;
        for (int j = 0; j < k; ++j)
            if ((t >> (k - 1 - j)) & 1) o |= 1ull << targets[j];
        all_offs[t] = o;
    }
    auto re = [&](int r, int col) { return G[2 * (r * d + col)]; };
    auto im = [&](int r, int col) { return G[2 * (r * d + col) + 1]; };
    auto nz = [&](int r, int col) { return re(r, col) != 0.0 || im(r, col) != 0.0; };
    auto is_one = [&](int r, int col) { return re(r, col) == 1.0 && im(r, col) == 0.0; };

    bool diag = true;
    for (int r = 0; r < d && diag; ++r)
        for (int col = 0; col < d; ++col)
            if (r != col && nz(r, col)) { diag = false; break; }
    std::vector<int> used(d, 0);
    if (diag) {
        a.cls = GC_DIAG;
        for (int t = 0; t < d; ++t)
            if (!is_one(t, t)) a.members.push_back(t);
        static const int sizes[] = {1, 2, 4, 8, 16, 32, 64};
        const int M = a.members.empty() ? 0 : pad_size((int)a.members.size(), sizes, 7);
        for (int t : a.members) used[t] = 1;
        for (int t = 0; t < d && (int)a.members.size() < M; ++t)
            if (!used[t]) { a.members.push_back(t); used[t] = 1; }
        for (int t : a.members) {
            a.offs.push_back(all_offs[t]);
            a.mat.push_back(re(t, t));
            a.mat.push_back(im(t, t));
        }
        return a;
    }
    // monomial: one non-zero per row and per column
    bool perm = true;
    std::vector<int> src(d, -1), colcount(d, 0);
    for (int r = 0; r < d && perm; ++r) {
        int cnt = 0;
        for (int col = 0; col < d; ++col)
            if (nz(r, col)) { ++cnt; src[r] = col; ++colcount[col]; }
        if (cnt != 1) perm = false;
    }
    for (int col = 0; col < d && perm; ++col)
        if (colcount[col] != 1) perm = false;
    if (perm) {
        a.cls = GC_PERM;
        for (int t = 0; t < d; ++t)
            if (src[t] != t || !is_one(t, src[t])) a.members.push_back(t);
        static const int sizes[] = {2, 4, 8, 16, 32, 64};
        const int M = pad_size((int)a.members.size(), sizes, 6);
        for (int t : a.members) used[t] = 1;
        for (int t = 0; t < d && (int)a.members.size() < M; ++t)
            if (!used[t]) { a.members.push_back(t); used[t] = 1; }
        std::vector<int> slot(d, -1);
        for (size_t j = 0; j < a.members.size(); ++j) slot[a.members[j]] = (int)j;
        for (int t : a.members) {
            a.offs.push_back(all_offs[t]);
            a.perm_src.push_back(slot[src[t]]);
            a.perm_one.push_back(is_one(t, src[t]) ? 1 : 0);
            a.mat.push_back(re(t, src[t]));
            a.mat.push_back(im(t, src[t]));
        }
        return a;
    }
    // dense over the members whose row or column differs from the identity
    a.cls = GC_DENSE;
    for (int t = 0; t < d; ++t) {
        bool differs = false;
        for (int u = 0; u < d && !differs; ++u) {
            const bool want_one = (u == t);
            if (want_one ? !is_one(t, u) : nz(t, u)) differs = true;
            if (want_one ? !is_one(u, t) : nz(u, t)) differs = true;
        }
        if (differs) a.members.push_back(t);
    }
    static const int sizes[] = {2, 3, 4, 8, 16, 32, 64};
    const int M = pad_size((int)a.members.size(), sizes, 7);
    for (int t : a.members) used[t] = 1;
    for (int t = 0; t < d && (int)a.members.size() < M; ++t)
        if (!used[t]) { a.members.push_back(t); used[t] = 1; }
    for (int t : a.members) a.offs.push_back(all_offs[t]);
    for (int r : a.members)
        for (int col : a.members) {
            a.mat.push_back(re(r, col));
            a.mat.push_back(im(r, col));
        }
    return a;
}

// ---------------------------------------------------------------- staging ring

namespace {
std::mutex g_mem_mu;
std::vector<std::pair<void *, size_t>> g_mem_live;   // few live allocations at any time
uint64_t g_mem_cur = 0, g_mem_peak = 0;
void mem_add(void *p, size_t bytes) {
    std::lock_guard<std::mutex> lk(g_mem_mu);
    g_mem_live.emplace_back(p, bytes);
    g_mem_cur += bytes;
    g_mem_peak = std::max(g_mem_peak, g_mem_cur);
}
void mem_remove(void *p) {
    std::lock_guard<std::mutex> lk(g_mem_mu);
    for (size_t i = 0; i < g_mem_live.size(); ++i)
        if (g_mem_live[i].first == p) {
            g_mem_cur -= g_mem_live[i].second;
            g_mem_live[i] = g_mem_live.back();
            g_mem_live.pop_back();
            return;
        }
}
}  // namespace

hipError_t dev_malloc(void **p, size_t bytes) {
    const hipError_t e = hipMalloc(p, bytes);
    if (e == hipSuccess) mem_add(*p, bytes);
    return e;
}
hipError_t dev_malloc_async(void **p, size_t bytes, hipStream_t s) {
    const hipError_t e = hipMallocAsync(p, bytes, s);
    if (e == hipSuccess) mem_add(*p, bytes);
    return e;
}
hipError_t dev_free(void *p) {
    mem_remove(p);
    return hipFree(p);
}
hipError_t dev_free_async(void *p, hipStream_t s) {
    mem_remove(p);
    return hipFreeAsync(p, s);
}

namespace {
constexpr int kSlots = 256;
constexpr size_t kSlotBytes = 256 << 10;
constexpr int kMaxStagingSlots = 8;   // the largest request: 2 MiB in consecutive slots

struct DeviceStaging {
    bool ready = false;
    char *host = nullptr;
    char *dev = nullptr;
    hipEvent_t ev[kSlots];
    bool armed[kSlots];
    int next = 0;
};
std::mutex g_staging_mu;
DeviceStaging g_staging[64];
}  // namespace

size_t staging_slot_bytes() { return kSlotBytes; }

int staging_acquire(size_t bytes, StagingSlot *slot) {
    if (bytes > kMaxStagingSlots * kSlotBytes) return fail(QSV_ERR_ARG, "staging request above the largest span");
    const int span = bytes <= kSlotBytes ? 1 : (int)((bytes + kSlotBytes - 1) / kSlotBytes);
    int dev = 0;
    QSV_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(QSV_ERR_ARG, "device index above 63");
    std::lock_guard<std::mutex> lk(g_staging_mu);
    DeviceStaging &st = g_staging[dev];
    if (!st.ready) {
        QSV_HIP_CHECK(hipHostMalloc((void **)&st.host, kSlots * kSlotBytes, hipHostMallocDefault));
        QSV_HIP_CHECK(dev_malloc((void **)&st.dev, kSlots * kSlotBytes));
        for (int i = 0; i < kSlots; ++i) {
            QSV_HIP_CHECK(hipEventCreateWithFlags(&st.ev[i], hipEventDisableTiming));
            st.armed[i] = false;
        }
        st.ready = true;
    }
    // a request of several slots takes consecutive ones (wrapping to slot 0
    // when the ring's end would split it)
    if (st.next + span > kSlots) st.next = 0;
    const int i = st.next;
    st.next = (st.next + span) % kSlots;
    for (int j = i; j < i + span; ++j)
        if (st.armed[j]) {
            QSV_HIP_CHECK(hipEventSynchronize(st.ev[j]));
            st.armed[j] = false;
        }
    slot->host = st.host + (size_t)i * kSlotBytes;
    slot->dev = st.dev + (size_t)i * kSlotBytes;
    slot->bytes = (size_t)span * kSlotBytes;
    slot->index = i + dev * kSlots;
    slot->span = span;
    return QSV_OK;
}

int staging_upload(const StagingSlot &slot, size_t bytes, hipStream_t s) {
    QSV_HIP_CHECK(hipMemcpyAsync(slot.dev, slot.host, bytes, hipMemcpyHostToDevice, s));
    return QSV_OK;
}

int staging_release(const StagingSlot &slot, hipStream_t s) {
    const int dev = slot.index / kSlots, i = slot.index % kSlots;
    std::lock_guard<std::mutex> lk(g_staging_mu);
    for (int j = i; j < i + slot.span; ++j) {
        QSV_HIP_CHECK(hipEventRecord(g_staging[dev].ev[j], s));
        g_staging[dev].armed[j] = true;
    }
    return QSV_OK;
}

}  // namespace qsv

using namespace qsv;

// ================================================================== C ABI

extern "C" {

int qsv_memory_stats(uint64_t *current_bytes, uint64_t *peak_bytes, int reset_peak) {
    std::lock_guard<std::mutex> lk(g_mem_mu);
    if (current_bytes) *current_bytes = g_mem_cur;
    if (peak_bytes) *peak_bytes = g_mem_peak;
    if (reset_peak) g_mem_peak = g_mem_cur;
    return QSV_OK;
}

int qsv_abi_version(void) { return QSV_ABI_VERSION; }

const char *qsv_status_string(int status) {
    switch (status) {
    case QSV_OK: return "ok";
    case QSV_ERR_NULL: return "null pointer";
    case QSV_ERR_DTYPE: return "bad dtype";
    case QSV_ERR_NQUBITS: return "bad number of qubits";
    case QSV_ERR_QUBIT_RANGE: return "qubit index out of range";
    case QSV_ERR_QUBIT_DUP: return "repeated qubit";
    case QSV_ERR_ARITY: return "too many targets or controls";
    case QSV_ERR_ALIGN: return "misaligned state";
    case QSV_ERR_UNSUPPORTED: return "unsupported";
    case QSV_ERR_HIP: return "HIP runtime error";
    case QSV_ERR_ARG: return "bad argument";
    default: return "unknown status";
    }
}

const char *qsv_last_error(void) { return g_last_error.c_str(); }

int qsv_validate(int n, int dtype, const int *targets, int k, const int *controls, int c) {
    return validate_common(n, dtype, targets, k, controls, c);
}

int qsv_group_index_host(int n, const int *bits, int m, uint64_t first, uint64_t count, uint64_t *out) {
    if (!out || (m > 0 && !bits)) return fail(QSV_ERR_NULL, "NULL argument");
    if (n < 1 || n > QSV_MAX_QUBITS) return fail(QSV_ERR_NQUBITS, "n must be in [1, 40]");
    if (m < 0 || m > n || m > QSV_MAX_TARGETS + QSV_MAX_CONTROLS) return fail(QSV_ERR_ARITY, "bad bit count");
    uint64_t lm[QSV_MAX_TARGETS + QSV_MAX_CONTROLS];
    for (int i = 0; i < m; ++i) {
        if (bits[i] < 0 || bits[i] >= n) return fail(QSV_ERR_QUBIT_RANGE, "bit out of range");
        if (i > 0 && bits[i] <= bits[i - 1]) return fail(QSV_ERR_ARG, "bits must be strictly ascending");
        lm[i] = (1ull << bits[i]) - 1ull;
    }
    const uint64_t ng = 1ull << (n - m);
    if (first > ng || count > ng - first) return fail(QSV_ERR_ARG, "group range out of bounds");
    for (uint64_t g = 0; g < count; ++g) out[g] = insert_zero_bits(first + g, lm, m);
    return QSV_OK;
}

int qsv_gate_matrix(const qsv_gate *gate, double *out) {
    if (!gate || !out) return fail(QSV_ERR_NULL, "NULL argument");
    std::vector<double> m;
    int st = gate_target_matrix(*gate, m);
    if (st) return st;
    std::memcpy(out, m.data(), m.size() * sizeof(double));
    return QSV_OK;
}

// Apply a complex128 target block (the shared tail of every gate entry point).
static int apply_c128_block(void *state, int n, int dtype, const double *G, const int *targets, int k,
                            const int *controls, int c, void *stream) {
    int st = validate_common(n, dtype, targets, k, controls, c);
    if (st) return st;
    if (k < 1) return fail(QSV_ERR_ARITY, "a gate needs at least one target");
    if ((st = check_state(state))) return st;
    GateAnalysis a = analyse_gate(n, G, targets, k, controls, c);
    return launch_gate(state, dtype, a, (hipStream_t)stream);
}

static void widen(const void *src, int dtype, int count, std::vector<double> &out) {
    out.resize(2 * count);
    if (dtype == QSV_C64) {
        const float *f = (const float *)src;
        for (int i = 0; i < 2 * count; ++i) out[i] = f[i];
    } else {
        std::memcpy(out.data(), src, sizeof(double) * 2 * count);
    }
}

int qsv_apply_matrix(void *state, int n, int dtype, const void *gate, const int *targets, int k,
                     const int *controls, int c, void *stream) {
    int st = validate_common(n, dtype, targets, k, controls, c);
    if (st) return st;
    if (!gate) return fail(QSV_ERR_NULL, "gate is NULL");
    if (k < 1) return fail(QSV_ERR_ARITY, "a gate needs at least one target");
    std::vector<double> G;
    widen(gate, dtype, 1 << (2 * k), G);
    return apply_c128_block(state, n, dtype, G.data(), targets, k, controls, c, stream);
}

static int apply_named(void *state, int n, int dtype, int kind, const int *targets, int k, double p0, double p1,
                       const int *controls, int c, void *stream) {
    qsv_gate g;
    std::memset(&g, 0, sizeof(g));
    g.kind = kind;
    g.k = k;
    g.params[0] = p0;
    g.params[1] = p1;
    std::vector<double> G;
    int st = validate_common(n, dtype, targets, k, controls, c);
    if (st) return st;
    if ((st = gate_target_matrix(g, G))) return st;
    return apply_c128_block(state, n, dtype, G.data(), targets, k, controls, c, stream);
}

int qsv_apply_x(void *state, int n, int dtype, int target, const int *controls, int c, void *stream) {
    return apply_named(state, n, dtype, QSV_GATE_X, &target, 1, 0, 0, controls, c, stream);
}
int qsv_apply_y(void *state, int n, int dtype, int target, const int *controls, int c, void *stream) {
    return apply_named(state, n, dtype, QSV_GATE_Y, &target, 1, 0, 0, controls, c, stream);
}
int qsv_apply_z(void *state, int n, int dtype, int target, const int *controls, int c, void *stream) {
    return apply_named(state, n, dtype, QSV_GATE_Z, &target, 1, 0, 0, controls, c, stream);
}
int qsv_apply_swap(void *state, int n, int dtype, int t0, int t1, const int *controls, int c, void *stream) {
    const int t[2] = {t0, t1};
    return apply_named(state, n, dtype, QSV_GATE_SWAP, t, 2, 0, 0, controls, c, stream);
}
int qsv_apply_phase(void *state, int n, int dtype, int target, double phi, const int *controls, int c,
                    void *stream) {
    return apply_named(state, n, dtype, QSV_GATE_U1, &target, 1, phi, 0, controls, c, stream);
}
int qsv_apply_fsim(void *state, int n, int dtype, int t0, int t1, double theta, double phi, void *stream) {
    const int t[2] = {t0, t1};
    return apply_named(state, n, dtype, QSV_GATE_FSIM, t, 2, theta, phi, nullptr, 0, stream);
}
int qsv_apply_diagonal(void *state, int n, int dtype, const void *diag, const int *targets, int k,
                       const int *controls, int c, void *stream) {
    int st = validate_common(n, dtype, targets, k, controls, c);
    if (st) return st;
    if (!diag) return fail(QSV_ERR_NULL, "diag is NULL");
    if (k < 1) return fail(QSV_ERR_ARITY, "a gate needs at least one target");
    std::vector<double> d;
    widen(diag, dtype, 1 << k, d);
    const int dim = 1 << k;
    std::vector<double> G(2 * dim * dim, 0.0);
    for (int i = 0; i < dim; ++i) {
        G[2 * (i * dim + i)] = d[2 * i];
        G[2 * (i * dim + i) + 1] = d[2 * i + 1];
    }
    return apply_c128_block(state, n, dtype, G.data(), targets, k, controls, c, stream);
}

int qsv_scale(void *state, int n, int dtype, double re, double im, void *stream) {
    if (dtype != QSV_C64 && dtype != QSV_C128) return fail(QSV_ERR_DTYPE, "dtype must be QSV_C64 or QSV_C128");
    if (n < 1 || n > QSV_MAX_QUBITS) return fail(QSV_ERR_NQUBITS, "n must be in [1, 40]");
    int st = check_state(state);
    if (st) return st;
    return launch_scale(state, n, dtype, re, im, (hipStream_t)stream);
}

}  // extern "C"
