// Density matrices (the methodology section applies Eq. 1 to density
// matrices as well as to state vectors).
//
// rho of n qubits is stored row-major: rho[r, c] at index r * 2^n + c, so as
// a vector of 2n qubits the column's qubit q is bit q and the row's qubit q
// is bit q + n.  A gate G on targets T with controls C acts as
// rho -> G rho G^dagger: G on the row bits T + n (controls C + n) and the
// complex conjugate of G on the column bits T (controls C).  The two halves
// act on disjoint bits, so a density-matrix circuit is a 2n-qubit circuit of
// twice the gates, planned and run by the state-vector machinery (per-gate
// kernels, fusion, LDS passes).  A one-qubit channel with Kraus operators
// K_k is the 4x4 superoperator S[(r, c), (r', c')] = sum_k K_k[r, r']
// conj(K_k[c, c']) on the (row, column) bit pair of its qubit: a
// two-target matrix gate, not unitary in general.
#include "plan_internal.h"

namespace qsv {

namespace {

constexpr int DT = 256;

__device__ inline double d_block_sum(double v, double *sh) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r += sh[i];
    __syncthreads();
    return r;
}

// Sum of the diagonal rho[i, i] = v[i * (2^n + 1)], real and imaginary parts,
// one block (fixed strided order, block tree).
template <typename C>
__global__ void __launch_bounds__(DT) k_dm_trace(const C *__restrict__ rho, uint64_t dim, double *out) {
    __shared__ double sh[DT / 64];
    double re = 0.0, im = 0.0;
    for (uint64_t i = threadIdx.x; i < dim; i += DT) {
        const C z = rho[i * (dim + 1)];
        re += (double)z.x;
        im += (double)z.y;
    }
    const double sr = d_block_sum(re, sh);
    const double si = d_block_sum(im, sh);
    if (threadIdx.x == 0) {
        out[0] = sr;
        out[1] = si;
    }
}

struct DmProbArgs {
    uint64_t lowmask[QSV_MAX_QUBITS];   // sorted measured qubits (zero insertion)
    uint64_t scatter[QSV_MAX_QUBITS];   // bit j of m (LSB first) -> 1 << qubit
    uint64_t dim;                       // 2^n
    uint64_t nrest;                     // 2^(n - r)
    uint64_t R;                         // 2^r
    int r;
};

// p(m) = sum over i with measured bits m of Re rho[i, i]: one thread per
// outcome, the rest indices in increasing order.
template <typename C>
__global__ void __launch_bounds__(DT) k_dm_probs(const C *__restrict__ rho, DmProbArgs a, double *out) {
    const uint64_t stride = (uint64_t)gridDim.x * DT;
    for (uint64_t m = (uint64_t)blockIdx.x * DT + threadIdx.x; m < a.R; m += stride) {
        uint64_t mb = 0;
        for (int j = 0; j < a.r; ++j)
            if ((m >> j) & 1) mb |= a.scatter[j];
        double s = 0.0;
        for (uint64_t t = 0; t < a.nrest; ++t) {
            const uint64_t i = insert_zero_bits(t, a.lowmask, a.r) | mb;
            s += (double)rho[i * (a.dim + 1)].x;
        }
        out[m] = s;
    }
}

int check_dm(const void *rho, int n, int dtype, const void *out) {
    if (dtype != QSV_C64 && dtype != QSV_C128) return fail(QSV_ERR_DTYPE, "dtype must be QSV_C64 or QSV_C128");
    if (n < 1 || 2 * n > QSV_MAX_QUBITS) return fail(QSV_ERR_NQUBITS, "a density matrix needs 1 <= n <= 20");
    if (!rho || !out) return fail(QSV_ERR_NULL, "NULL pointer");
    if (((uintptr_t)rho & 15) != 0) return fail(QSV_ERR_ALIGN, "rho must be 16-byte aligned");
    return QSV_OK;
}

}  // namespace

}  // namespace qsv

using namespace qsv;

extern "C" {

int qsv_dm_plan_create(int n, int dtype, const qsv_gate *gates, int ngates, const qsv_plan_options *opts,
                       qsv_plan **out) {
    if (!out) return fail(QSV_ERR_NULL, "out is NULL");
    *out = nullptr;
    if (n < 1 || 2 * n > QSV_MAX_QUBITS) return fail(QSV_ERR_NQUBITS, "a density matrix needs 1 <= n <= 20");
    if (ngates < 0 || (ngates > 0 && !gates)) return fail(QSV_ERR_NULL, "gates is NULL");
    std::vector<qsv_gate> dbl;
    std::vector<std::vector<double>> conj_data;   // conjugated matrices, kept until the plan has copied them
    conj_data.reserve(ngates);
    dbl.reserve(2 * (size_t)ngates);
    for (int i = 0; i < ngates; ++i) {
        const qsv_gate &g = gates[i];
        int st = validate_common(n, dtype, g.targets, g.k, g.controls, g.c);
        if (st) return st;
        std::vector<double> G;
        if ((st = gate_target_matrix(g, G))) return st;
        qsv_gate row = g;   // G on the row bits
        for (int j = 0; j < g.k; ++j) row.targets[j] = g.targets[j] + n;
        for (int j = 0; j < g.c; ++j) row.controls[j] = g.controls[j] + n;
        dbl.push_back(row);
        bool real = true;
        for (size_t e = 1; e < G.size(); e += 2)
            if (G[e] != 0.0) real = false;
        qsv_gate col = g;   // conj(G) on the column bits
        if (!real) {
            for (size_t e = 1; e < G.size(); e += 2) G[e] = -G[e];
            conj_data.push_back(std::move(G));
            col.kind = QSV_GATE_MATRIX;
            col.data = conj_data.back().data();
        }
        dbl.push_back(col);
    }
    return qsv_plan_create(2 * n, dtype, dbl.data(), (int)dbl.size(), opts, out);
}

int qsv_dm_apply_channel(void *rho, int n, int dtype, const double *kraus, int nk, int target, void *stream) {
    int st = check_dm(rho, n, dtype, rho);
    if (st) return st;
    if (!kraus) return fail(QSV_ERR_NULL, "kraus is NULL");
    if (nk < 1 || nk > 16) return fail(QSV_ERR_ARG, "between 1 and 16 Kraus operators");
    if (target < 0 || target >= n) return fail(QSV_ERR_QUBIT_RANGE, "target out of range");
    // S[(r c), (r' c')] = sum_k K[r r'] conj(K[c c']), index 2 r + c (row bit first)
    std::vector<double> S(2 * 16, 0.0);
    for (int k = 0; k < nk; ++k) {
        const double *K = kraus + 8 * k;
        for (int r = 0; r < 2; ++r)
            for (int c = 0; c < 2; ++c)
                for (int rp = 0; rp < 2; ++rp)
                    for (int cp = 0; cp < 2; ++cp) {
                        const double ar = K[2 * (2 * r + rp)], ai = K[2 * (2 * r + rp) + 1];
                        const double br = K[2 * (2 * c + cp)], bi = -K[2 * (2 * c + cp) + 1];
                        const int e = (2 * r + c) * 4 + (2 * rp + cp);
                        S[2 * e] += ar * br - ai * bi;
                        S[2 * e + 1] += ar * bi + ai * br;
                    }
    }
    const int t[2] = {target + n, target};
    if (dtype == QSV_C128) return qsv_apply_matrix(rho, 2 * n, dtype, S.data(), t, 2, nullptr, 0, stream);
    std::vector<float> Sf(S.begin(), S.end());
    return qsv_apply_matrix(rho, 2 * n, dtype, Sf.data(), t, 2, nullptr, 0, stream);
}

int qsv_dm_trace(const void *rho, int n, int dtype, double *out_dev, void *stream) {
    int st = check_dm(rho, n, dtype, out_dev);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    const uint64_t dim = 1ull << n;
    if (dtype == QSV_C64)
        hipLaunchKernelGGL((k_dm_trace<float2>), dim3(1), dim3(DT), 0, s, (const float2 *)rho, dim, out_dev);
    else
        hipLaunchKernelGGL((k_dm_trace<double2>), dim3(1), dim3(DT), 0, s, (const double2 *)rho, dim, out_dev);
    QSV_HIP_CHECK(hipGetLastError());
    return QSV_OK;
}

int qsv_dm_probabilities(const void *rho, int n, int dtype, const int *qubits, int r, double *out_dev, void *stream) {
    int st = check_dm(rho, n, dtype, out_dev);
    if (st) return st;
    if (!qubits) return fail(QSV_ERR_NULL, "qubits is NULL");
    if (r < 1 || r > n) return fail(QSV_ERR_ARITY, "number of measured qubits must be in [1, n]");
    DmProbArgs a;
    std::memset(&a, 0, sizeof(a));
    uint64_t seen = 0;
    for (int j = 0; j < r; ++j) {
        if (qubits[j] < 0 || qubits[j] >= n) return fail(QSV_ERR_QUBIT_RANGE, "measured qubit out of range");
        if (seen & (1ull << qubits[j])) return fail(QSV_ERR_QUBIT_DUP, "measured qubit repeats");
        seen |= 1ull << qubits[j];
        a.scatter[r - 1 - j] = 1ull << qubits[j];
    }
    std::vector<int> sorted(qubits, qubits + r);
    std::sort(sorted.begin(), sorted.end());
    for (int i = 0; i < r; ++i) a.lowmask[i] = (1ull << sorted[i]) - 1ull;
    a.r = r;
    a.dim = 1ull << n;
    a.nrest = 1ull << (n - r);
    a.R = 1ull << r;
    const unsigned blocks = (unsigned)std::min<uint64_t>((a.R + DT - 1) / DT, 65535);
    hipStream_t s = (hipStream_t)stream;
    if (dtype == QSV_C64)
        hipLaunchKernelGGL((k_dm_probs<float2>), dim3(blocks), dim3(DT), 0, s, (const float2 *)rho, a, out_dev);
    else
        hipLaunchKernelGGL((k_dm_probs<double2>), dim3(blocks), dim3(DT), 0, s, (const double2 *)rho, a, out_dev);
    QSV_HIP_CHECK(hipGetLastError());
    return QSV_OK;
}

}  // extern "C"
