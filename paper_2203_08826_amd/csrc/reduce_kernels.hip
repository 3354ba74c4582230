// Reductions over the state: measurement probabilities (methodology section,
// measurement), norm, inner product, and the energy of the transverse-field
// Ising Hamiltonian H = J sum Z_i Z_{i+1} + h sum X_i used by the gradient
// workload.
//
// Every amplitude is widened to float64 before it is squared or multiplied,
// and sums are accumulated in float64 in a fixed order: each thread walks a
// fixed strided range, waves reduce with shuffles in a fixed tree, blocks
// write one partial each, and a second launch adds the partials in order.
// The grid depends only on the problem size and the device's CU count, so a
// result is reproducible bit for bit on a given device.
#include "qsv_internal.h"

namespace qsv {

constexpr int RT = 256;   // threads per reduction block

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Fixed-order block sum; every thread must call it.  Result valid in thread 0.
__device__ inline double block_sum(double v, double *sh) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r += sh[i];
    __syncthreads();
    return r;
}

template <typename C> __device__ inline double abs2d(C z) {
    const double x = (double)z.x, y = (double)z.y;
    return x * x + y * y;
}

// ---------------------------------------------------------------- norm / inner

template <typename C>
__global__ void __launch_bounds__(RT) k_norm2_partial(const C *__restrict__ psi, uint64_t N, double *part) {
    __shared__ double sh[RT / 64];
    const uint64_t stride = (uint64_t)gridDim.x * RT;
    double acc = 0.0;
    for (uint64_t i = (uint64_t)blockIdx.x * RT + threadIdx.x; i < N; i += stride) acc += abs2d(psi[i]);
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

template <typename C>
__global__ void __launch_bounds__(RT) k_inner_partial(const C *__restrict__ a, const C *__restrict__ b, uint64_t N,
                                                      double *part) {
    __shared__ double sh[RT / 64];
    const uint64_t stride = (uint64_t)gridDim.x * RT;
    double re = 0.0, im = 0.0;
    for (uint64_t i = (uint64_t)blockIdx.x * RT + threadIdx.x; i < N; i += stride) {
        const C x = a[i], y = b[i];
        const double ax = x.x, ay = x.y, bx = y.x, by = y.y;
        re += ax * bx + ay * by;   // conj(a) * b
        im += ax * by - ay * bx;
    }
    const double sr = block_sum(re, sh);
    const double si = block_sum(im, sh);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = sr;
        part[2 * blockIdx.x + 1] = si;
    }
}

// Sum `nparts` partials of width `width` (fixed order) into out[0..width).
__global__ void k_sum_partials(const double *part, int nparts, int width, double scale, double *out) {
    const int w = threadIdx.x;
    if (w >= width) return;
    double s = 0.0;
    for (int p = 0; p < nparts; ++p) s += part[p * width + w];
    out[w] = s * scale;
}

static int reduce_grid(uint64_t N) {
    uint64_t b = (N + RT * 8 - 1) / (RT * 8);
    const uint64_t cap = (uint64_t)device_sm_count() * 8;
    if (b > cap) b = cap;
    if (b < 1) b = 1;
    return (int)b;
}

// ---------------------------------------------------------------- probabilities

struct ProbArgs {
    uint64_t lowmask[QSV_MAX_QUBITS];   // sorted measured bits, for the rest index
    uint64_t scatter[QSV_MAX_QUBITS];   // bit j of m (LSB first) -> 1 << position
    int r;
    int n;
};

__device__ inline uint64_t prob_index(uint64_t m, uint64_t rest, const ProbArgs &pa) {
    uint64_t i = rest;
    for (int b = 0; b < pa.r; ++b) {
        const uint64_t lo = i & pa.lowmask[b];
        i = lo | ((i ^ lo) << 1);
    }
    for (int j = 0; j < pa.r; ++j)
        if ((m >> j) & 1) i |= pa.scatter[j];
    return i;
}

// Block (m, p) sums the rest indices [p * S, (p + 1) * S) of outcome m.
template <typename C>
__global__ void __launch_bounds__(RT) k_probs_partial(const C *__restrict__ psi, ProbArgs pa, uint64_t S, int P,
                                                      double *part) {
    __shared__ double sh[RT / 64];
    const uint64_t m = blockIdx.x / P;
    const uint64_t p = blockIdx.x % P;
    double acc = 0.0;
    for (uint64_t t = threadIdx.x; t < S; t += RT) acc += abs2d(psi[prob_index(m, p * S + t, pa)]);
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void k_probs_finish(const double *part, int P, uint64_t R, double *out) {
    const uint64_t m = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= R) return;
    double s = 0.0;
    for (int p = 0; p < P; ++p) s += part[m * P + p];
    out[m] = s;
}

// Few amplitudes per outcome: one thread per outcome, sequential sum.
template <typename C>
__global__ void __launch_bounds__(RT) k_probs_direct(const C *__restrict__ psi, ProbArgs pa, uint64_t R,
                                                     uint64_t S, double *out) {
    const uint64_t m = (uint64_t)blockIdx.x * RT + threadIdx.x;
    if (m >= R) return;
    double acc = 0.0;
    for (uint64_t t = 0; t < S; ++t) acc += abs2d(psi[prob_index(m, t, pa)]);
    out[m] = acc;
}

// ---------------------------------------------------------------- TFIM energy

constexpr int TB = 10;              // chunk bits: 1024 amplitudes per block in LDS

struct TfimArgs {
    uint64_t N;
    int n;
    int periodic;
    double J, h;
};

__device__ inline double zz_value(uint64_t i, const TfimArgs &a) {
    double z = 0.0;
    for (int q = 0; q + 1 < a.n; ++q) z += (((i >> q) ^ (i >> (q + 1))) & 1) ? -1.0 : 1.0;
    if (a.periodic && a.n > 2) z += (((i >> (a.n - 1)) ^ i) & 1) ? -1.0 : 1.0;
    return z;
}

// Per block: a chunk of 2^TB amplitudes (or the whole state if smaller) in
// LDS.  ZZ part from the diagonal; X_q part as 2 Re sum_{bit q = 0}
// conj(psi_i) psi_{i + 2^q}, partner from LDS for q < TB, from HBM above.
template <typename C>
__global__ void __launch_bounds__(RT) k_tfim_partial(const C *__restrict__ psi, TfimArgs a, int cb,
                                                     double *part) {
    __shared__ C ch[1 << TB];
    __shared__ double sh[RT / 64];
    const uint64_t csize = 1ull << cb;
    const uint64_t nchunks = a.N >> cb;
    double zz = 0.0, xx = 0.0;
    for (uint64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const uint64_t base = c << cb;
        for (uint64_t t = threadIdx.x; t < csize; t += RT) ch[t] = psi[base + t];
        __syncthreads();
        for (uint64_t t = threadIdx.x; t < csize; t += RT) {
            const uint64_t i = base + t;
            const C v = ch[t];
            zz += abs2d(v) * zz_value(i, a);
            for (int q = 0; q < a.n; ++q) {
                if ((i >> q) & 1) continue;
                const C w = (q < cb) ? ch[t | (1ull << q)] : psi[i | (1ull << q)];
                xx += 2.0 * ((double)v.x * (double)w.x + (double)v.y * (double)w.y);
            }
        }
        __syncthreads();
    }
    const double s1 = block_sum(a.J * zz, sh);
    const double s2 = block_sum(a.h * xx, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s1 + s2;
}

// out = H psi
template <typename C>
__global__ void __launch_bounds__(RT) k_apply_tfim(const C *__restrict__ psi, C *__restrict__ out, TfimArgs a) {
    const uint64_t stride = (uint64_t)gridDim.x * RT;
    for (uint64_t i = (uint64_t)blockIdx.x * RT + threadIdx.x; i < a.N; i += stride) {
        const C v = psi[i];
        const double z = a.J * zz_value(i, a);
        double rx = z * (double)v.x, ry = z * (double)v.y;
        double sx = 0.0, sy = 0.0;
        for (int q = 0; q < a.n; ++q) {
            const C w = psi[i ^ (1ull << q)];
            sx += (double)w.x;
            sy += (double)w.y;
        }
        C o;
        o.x = (decltype(o.x))(rx + a.h * sx);
        o.y = (decltype(o.y))(ry + a.h * sy);
        out[i] = o;
    }
}

// ---------------------------------------------------------------- launchers

template <typename C>
static int norm2_t(const void *state, int n, double *out, hipStream_t s) {
    const uint64_t N = 1ull << n;
    const int g = reduce_grid(N);
    StagingSlot slot;
    int st = staging_acquire(sizeof(double) * g, &slot);
    if (st) return st;
    double *part = (double *)slot.dev;
    hipLaunchKernelGGL((k_norm2_partial<C>), dim3(g), dim3(RT), 0, s, (const C *)state, N, part);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(64), 0, s, part, g, 1, 1.0, out);
    hipError_t e = hipGetLastError();
    staging_release(slot, s);
    if (e != hipSuccess) return hip_fail(e, "norm2 launch");
    return QSV_OK;
}

template <typename C>
static int inner_t(const void *a, const void *b, int n, double *out, hipStream_t s) {
    const uint64_t N = 1ull << n;
    const int g = reduce_grid(N);
    StagingSlot slot;
    int st = staging_acquire(sizeof(double) * 2 * g, &slot);
    if (st) return st;
    double *part = (double *)slot.dev;
    hipLaunchKernelGGL((k_inner_partial<C>), dim3(g), dim3(RT), 0, s, (const C *)a, (const C *)b, N, part);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(64), 0, s, part, g, 2, 1.0, out);
    hipError_t e = hipGetLastError();
    staging_release(slot, s);
    if (e != hipSuccess) return hip_fail(e, "inner launch");
    return QSV_OK;
}

template <typename C>
static int probs_t(const void *state, int n, const int *qubits, int r, double *out, hipStream_t s) {
    ProbArgs pa;
    std::memset(&pa, 0, sizeof(pa));
    pa.r = r;
    pa.n = n;
    std::vector<int> sorted(qubits, qubits + r);
    std::sort(sorted.begin(), sorted.end());
    for (int i = 0; i < r; ++i) pa.lowmask[i] = (1ull << sorted[i]) - 1ull;
    for (int j = 0; j < r; ++j) pa.scatter[r - 1 - j] = 1ull << qubits[j];   // qubits[0] = MSB of m
    const uint64_t R = 1ull << r, S = 1ull << (n - r);
    if (S < 4 * RT) {
        const uint64_t blocks = (R + RT - 1) / RT;
        hipLaunchKernelGGL((k_probs_direct<C>), dim3((unsigned)blocks), dim3(RT), 0, s, (const C *)state, pa, R, S,
                           out);
        QSV_HIP_CHECK(hipGetLastError());
        return QSV_OK;
    }
    // parts per outcome: aim at >= 8 blocks per CU, each summing >= 4 * RT amplitudes
    uint64_t P = ((uint64_t)device_sm_count() * 8 + R - 1) / R;
    while (P > 1 && S / P < 4 * RT) P >>= 1;
    uint64_t p2 = 1;
    while (p2 * 2 <= P) p2 <<= 1;   // power of two, so P divides S
    P = p2;
    const size_t bytes = sizeof(double) * R * P;
    if (bytes > staging_slot_bytes()) return fail(QSV_ERR_UNSUPPORTED, "probabilities: too many outcomes for one launch");
    StagingSlot slot;
    int st = staging_acquire(bytes, &slot);
    if (st) return st;
    double *part = (double *)slot.dev;
    hipLaunchKernelGGL((k_probs_partial<C>), dim3((unsigned)(R * P)), dim3(RT), 0, s, (const C *)state, pa, S / P,
                       (int)P, part);
    hipLaunchKernelGGL(k_probs_finish, dim3((unsigned)((R + 255) / 256)), dim3(256), 0, s, part, (int)P, R, out);
    hipError_t e = hipGetLastError();
    staging_release(slot, s);
    if (e != hipSuccess) return hip_fail(e, "probabilities launch");
    return QSV_OK;
}

template <typename C>
static int tfim_t(const void *state, int n, double J, double h, int periodic, double *out, hipStream_t s) {
    TfimArgs a;
    a.N = 1ull << n;
    a.n = n;
    a.periodic = periodic;
    a.J = J;
    a.h = h;
    const int cb = n < TB ? n : TB;
    const uint64_t nchunks = a.N >> cb;
    uint64_t g = nchunks;
    const uint64_t cap = (uint64_t)device_sm_count() * 8;
    if (g > cap) g = cap;
    StagingSlot slot;
    int st = staging_acquire(sizeof(double) * g, &slot);
    if (st) return st;
    double *part = (double *)slot.dev;
    hipLaunchKernelGGL((k_tfim_partial<C>), dim3((unsigned)g), dim3(RT), 0, s, (const C *)state, a, cb, part);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(64), 0, s, part, (int)g, 1, 1.0, out);
    hipError_t e = hipGetLastError();
    staging_release(slot, s);
    if (e != hipSuccess) return hip_fail(e, "tfim energy launch");
    return QSV_OK;
}

template <typename C>
static int apply_tfim_t(const void *state, void *out, int n, double J, double h, int periodic, hipStream_t s) {
    TfimArgs a;
    a.N = 1ull << n;
    a.n = n;
    a.periodic = periodic;
    a.J = J;
    a.h = h;
    uint64_t g = (a.N + RT - 1) / RT;
    const uint64_t cap = (uint64_t)device_sm_count() * 32;
    if (g > cap) g = cap;
    hipLaunchKernelGGL((k_apply_tfim<C>), dim3((unsigned)g), dim3(RT), 0, s, (const C *)state, (C *)out, a);
    QSV_HIP_CHECK(hipGetLastError());
    return QSV_OK;
}

}  // namespace qsv

using namespace qsv;

extern "C" {

static int check_red(const void *state, int n, int dtype, const void *out) {
    if (dtype != QSV_C64 && dtype != QSV_C128) return fail(QSV_ERR_DTYPE, "dtype must be QSV_C64 or QSV_C128");
    if (n < 1 || n > QSV_MAX_QUBITS) return fail(QSV_ERR_NQUBITS, "n must be in [1, 40]");
    if (!state || !out) return fail(QSV_ERR_NULL, "NULL pointer");
    if (((uintptr_t)state & 15) != 0) return fail(QSV_ERR_ALIGN, "state must be 16-byte aligned");
    return QSV_OK;
}

int qsv_norm2(const void *state, int n, int dtype, double *out_dev, void *stream) {
    int st = check_red(state, n, dtype, out_dev);
    if (st) return st;
    return dtype == QSV_C64 ? norm2_t<float2>(state, n, out_dev, (hipStream_t)stream)
                            : norm2_t<double2>(state, n, out_dev, (hipStream_t)stream);
}

int qsv_inner(const void *a, const void *b, int n, int dtype, double *out_dev, void *stream) {
    int st = check_red(a, n, dtype, out_dev);
    if (st) return st;
    if ((st = check_red(b, n, dtype, out_dev))) return st;
    return dtype == QSV_C64 ? inner_t<float2>(a, b, n, out_dev, (hipStream_t)stream)
                            : inner_t<double2>(a, b, n, out_dev, (hipStream_t)stream);
}

int qsv_probabilities(const void *state, int n, int dtype, const int *qubits, int r, double *out_dev,
                      void *stream) {
    int st = check_red(state, n, dtype, out_dev);
    if (st) return st;
    if (r < 1 || r > n) return fail(QSV_ERR_ARITY, "number of measured qubits must be in [1, n]");
    if (!qubits) return fail(QSV_ERR_NULL, "qubits is NULL");
    uint64_t seen = 0;
    for (int j = 0; j < r; ++j) {
        if (qubits[j] < 0 || qubits[j] >= n) return fail(QSV_ERR_QUBIT_RANGE, "measured qubit out of range");
        if (seen & (1ull << qubits[j])) return fail(QSV_ERR_QUBIT_DUP, "measured qubit repeats");
        seen |= 1ull << qubits[j];
    }
    return dtype == QSV_C64 ? probs_t<float2>(state, n, qubits, r, out_dev, (hipStream_t)stream)
                            : probs_t<double2>(state, n, qubits, r, out_dev, (hipStream_t)stream);
}

int qsv_expval_zz_x(const void *state, int n, int dtype, double J, double h, int periodic, double *out_dev,
                    void *stream) {
    int st = check_red(state, n, dtype, out_dev);
    if (st) return st;
    return dtype == QSV_C64 ? tfim_t<float2>(state, n, J, h, periodic, out_dev, (hipStream_t)stream)
                            : tfim_t<double2>(state, n, J, h, periodic, out_dev, (hipStream_t)stream);
}

int qsv_apply_tfim(const void *state, void *out, int n, int dtype, double J, double h, int periodic,
                   void *stream) {
    int st = check_red(state, n, dtype, out);
    if (st) return st;
    if (((uintptr_t)out & 15) != 0) return fail(QSV_ERR_ALIGN, "out must be 16-byte aligned");
    if (out == state) return fail(QSV_ERR_ARG, "out must not alias state");
    return dtype == QSV_C64 ? apply_tfim_t<float2>(state, out, n, J, h, periodic, (hipStream_t)stream)
                            : apply_tfim_t<double2>(state, out, n, J, h, periodic, (hipStream_t)stream);
}

}  // extern "C"
