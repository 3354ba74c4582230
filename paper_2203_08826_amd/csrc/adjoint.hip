// Adjoint-method gradient of E = <psi|H|psi> (Jones and Gacon,
// arXiv:2009.02823) for circuits of rotations exp(-i theta P / 2).
//
// With psi_l = U_l..U_1 psi_0 and lam_l = U_{l+1}^dag..U_L^dag H psi_L,
// dE/dtheta_l = 2 Re <lam_l| (-i/2) P_l |psi_l> = Im <lam_l|P_l|psi_l>.
// The gates are walked backwards; for a rotation one kernel reads the pairs
// (psi_0, psi_1) and (lam_0, lam_1) of its target once, accumulates
// Im(conj(lam) . P psi) in float64 and writes U^dag psi and U^dag lam back,
// so each rotation costs one read + write of both vectors.  Other gates are
// moved back through U^dag with the per-gate kernels.  Block partials go to
// a stream-ordered scratch buffer and are summed in a fixed order at the end.
#include <cmath>

#include "plan_internal.h"

namespace qsv {

constexpr int AT = 256;

struct AdjArgs {
    uint64_t lowmask[1 + QSV_MAX_CONTROLS];
    uint64_t cmask;
    uint64_t ngroups;
    uint64_t tbit;
    int m;
    int pauli;      // 1 = X, 2 = Y, 3 = Z
    int slot;       // parameter index
    int nblocks;
    double ud[8];   // U^dagger, complex128 row-major 2x2
};

template <typename C>
__global__ void __launch_bounds__(AT) k_adj_rot(C *__restrict__ psi, C *__restrict__ lam, AdjArgs a, double *part) {
    __shared__ double sh[AT / 64];
    typedef decltype(C().x) R;
    C u00, u01, u10, u11;
    u00.x = (R)a.ud[0]; u00.y = (R)a.ud[1]; u01.x = (R)a.ud[2]; u01.y = (R)a.ud[3];
    u10.x = (R)a.ud[4]; u10.y = (R)a.ud[5]; u11.x = (R)a.ud[6]; u11.y = (R)a.ud[7];
    double acc = 0.0;
    const uint64_t stride = (uint64_t)gridDim.x * AT;
    for (uint64_t g = (uint64_t)blockIdx.x * AT + threadIdx.x; g < a.ngroups; g += stride) {
        uint64_t i0 = g;
        for (int b = 0; b < a.m; ++b) {
            const uint64_t lo = i0 & a.lowmask[b];
            i0 = lo | ((i0 ^ lo) << 1);
        }
        i0 |= a.cmask;
        const uint64_t i1 = i0 | a.tbit;
        const C p0 = psi[i0], p1 = psi[i1], l0 = lam[i0], l1 = lam[i1];
        // Im(conj(l0) (P p)_0 + conj(l1) (P p)_1), in float64
        const double p0r = p0.x, p0i = p0.y, p1r = p1.x, p1i = p1.y;
        const double l0r = l0.x, l0i = l0.y, l1r = l1.x, l1i = l1.y;
        double q0r, q0i, q1r, q1i;   // P p
        if (a.pauli == 1) {
            q0r = p1r; q0i = p1i; q1r = p0r; q1i = p0i;
        } else if (a.pauli == 2) {
            q0r = p1i; q0i = -p1r;    // -i p1
            q1r = -p0i; q1i = p0r;    //  i p0
        } else {
            q0r = p0r; q0i = p0i; q1r = -p1r; q1i = -p1i;
        }
        acc += (l0r * q0i - l0i * q0r) + (l1r * q1i - l1i * q1r);
        psi[i0] = cfma(u01, p1, cmul(u00, p0));
        psi[i1] = cfma(u11, p1, cmul(u10, p0));
        lam[i0] = cfma(u01, l1, cmul(u00, l0));
        lam[i1] = cfma(u11, l1, cmul(u10, l0));
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < AT / 64; ++w) s += sh[w];
        part[(uint64_t)a.slot * a.nblocks + blockIdx.x] = s;
    }
}

__global__ void k_adj_finish(const double *part, int nparams, int nblocks, double *grad) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nparams) return;
    double s = 0.0;
    for (int b = 0; b < nblocks; ++b) s += part[(uint64_t)p * nblocks + b];
    grad[p] = s;
}

static int pauli_of(int kind) {
    switch (kind) {
    case QSV_GATE_RX: return 1;
    case QSV_GATE_RY: return 2;
    case QSV_GATE_RZ: return 3;
    default: return 0;
    }
}

static void dagger(const std::vector<double> &G, int k, std::vector<double> &out) {
    const int d = 1 << k;
    out.assign(G.size(), 0.0);
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c) {
            out[2 * (r * d + c)] = G[2 * (c * d + r)];
            out[2 * (r * d + c) + 1] = -G[2 * (c * d + r) + 1];
        }
}

template <typename C>
static int adjoint_t(void *psi, void *lam, int n, int dtype, const qsv_gate *gates, int ngates, double *grad,
                     hipStream_t s) {
    int nparams = 0;
    for (int i = 0; i < ngates; ++i)
        if (pauli_of(gates[i].kind)) ++nparams;
    uint64_t max_groups = 0;
    for (int i = 0; i < ngates; ++i)
        if (pauli_of(gates[i].kind)) max_groups = std::max<uint64_t>(max_groups, 1ull << (n - 1 - gates[i].c));
    int nblocks = (int)std::min<uint64_t>((max_groups + AT - 1) / AT, (uint64_t)device_sm_count() * 4);
    if (nblocks < 1) nblocks = 1;
    double *part = nullptr;
    if (nparams > 0) QSV_HIP_CHECK(dev_malloc_async((void **)&part, sizeof(double) * (size_t)nparams * nblocks, s));
    int slot = nparams;
    int st = QSV_OK;
    for (int i = ngates - 1; i >= 0 && st == QSV_OK; --i) {
        const qsv_gate &g = gates[i];
        std::vector<double> G, Gd;
        if ((st = gate_target_matrix(g, G))) break;
        dagger(G, g.k, Gd);
        const int pauli = pauli_of(g.kind);
        if (pauli) {
            --slot;
            AdjArgs a;
            std::memset(&a, 0, sizeof(a));
            std::vector<int> bits(g.controls, g.controls + g.c);
            bits.push_back(g.targets[0]);
            std::sort(bits.begin(), bits.end());
            a.m = (int)bits.size();
            for (int b = 0; b < a.m; ++b) a.lowmask[b] = (1ull << bits[b]) - 1ull;
            for (int j = 0; j < g.c; ++j) a.cmask |= 1ull << g.controls[j];
            a.tbit = 1ull << g.targets[0];
            a.ngroups = 1ull << (n - a.m);
            a.pauli = pauli;
            a.slot = slot;
            a.nblocks = nblocks;
            for (int e = 0; e < 8; ++e) a.ud[e] = Gd[e];
            hipLaunchKernelGGL((k_adj_rot<C>), dim3(nblocks), dim3(AT), 0, s, (C *)psi, (C *)lam, a, part);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) st = hip_fail(e, "adjoint rotation launch");
        } else {
            GateAnalysis a = analyse_gate(n, Gd.data(), g.targets, g.k, g.controls, g.c);
            st = launch_gate(psi, dtype, a, s);
            if (!st) st = launch_gate(lam, dtype, a, s);
        }
    }
    if (st == QSV_OK && nparams > 0) {
        hipLaunchKernelGGL(k_adj_finish, dim3((nparams + 255) / 256), dim3(256), 0, s, part, nparams, nblocks, grad);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) st = hip_fail(e, "adjoint finish launch");
    }
    if (part) {
        hipError_t e = dev_free_async(part, s);
        if (st == QSV_OK && e != hipSuccess) st = hip_fail(e, "hipFreeAsync");
    }
    return st;
}

}  // namespace qsv

using namespace qsv;

extern "C" int qsv_adjoint_grad(void *psi, void *lam, int n, int dtype, const qsv_gate *gates, int ngates,
                                double *grad_dev, void *stream) {
    int st = validate_common(n, dtype, nullptr, 0, nullptr, 0);
    if (st) return st;
    if (!psi || !lam || (ngates > 0 && !gates)) return fail(QSV_ERR_NULL, "NULL argument");
    {
        const uint64_t bytes = (uint64_t)(dtype == QSV_C64 ? 8 : 16) << n;
        if (ranges_overlap(psi, bytes, lam, bytes)) return fail(QSV_ERR_ARG, "psi and lam must not overlap");
    }
    if (((uintptr_t)psi & 15) || ((uintptr_t)lam & 15)) return fail(QSV_ERR_ALIGN, "states must be 16-byte aligned");
    int nparams = 0;
    for (int i = 0; i < ngates; ++i) {
        const qsv_gate &g = gates[i];
        if ((st = validate_common(n, dtype, g.targets, g.k, g.controls, g.c))) return st;
        if (g.k < 1) return fail(QSV_ERR_ARITY, "gate without target");
        std::vector<double> G;
        if ((st = gate_target_matrix(g, G))) return st;
        if (pauli_of(g.kind)) ++nparams;
    }
    if (nparams > 0 && !grad_dev) return fail(QSV_ERR_NULL, "grad_dev is NULL");
    return dtype == QSV_C64 ? adjoint_t<float2>(psi, lam, n, dtype, gates, ngates, grad_dev, (hipStream_t)stream)
                            : adjoint_t<double2>(psi, lam, n, dtype, gates, ngates, grad_dev, (hipStream_t)stream);
}
