// Measurement operators of the methodology section (Sec. 2): collapse of
// the state onto an outcome with re-normalisation, and shot sampling from
// measurement probabilities -- exact inverse-CDF draws and Metropolis shot
// frequencies.  Random numbers are inputs (device arrays), so a draw is a
// deterministic function of them.
//
// Outcome index of measured qubits q_0..q_{r-1}: m = sum_j bit(q_j) 2^(r-1-j)
// (q_0 the most significant bit), as for qsv_probabilities.
#include "qsv_internal.h"

namespace qsv {

namespace {

constexpr int MT = 256;   // threads per block

__device__ inline double m_wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Fixed-order sum over the block; valid in thread 0.
__device__ inline double m_block_sum(double v, double *sh) {
    v = m_wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r += sh[i];
    __syncthreads();
    return r;
}

template <typename C> __device__ inline double m_abs2(C z) {
    const double x = (double)z.x, y = (double)z.y;
    return x * x + y * y;
}

// ---------------------------------------------------------------- collapse

struct CollapseArgs {
    uint64_t lowmask[QSV_MAX_QUBITS];   // sorted measured bits (zero insertion)
    uint64_t qmask;                     // measured bits
    uint64_t omask;                     // their values for the outcome
    uint64_t nkept;                     // 2^(n - r)
    uint64_t N;                         // 2^n
    int r;
};

// ||P_m psi||^2: the kept amplitudes are the rest indices with the measured
// bits inserted and set to the outcome's values; each thread sums a fixed
// strided range, blocks write partials.
template <typename C>
__global__ void __launch_bounds__(MT) k_kept_norm(const C *__restrict__ psi, CollapseArgs a, double *part) {
    __shared__ double sh[MT / 64];
    const uint64_t stride = (uint64_t)gridDim.x * MT;
    double acc = 0.0;
    for (uint64_t t = (uint64_t)blockIdx.x * MT + threadIdx.x; t < a.nkept; t += stride)
        acc += m_abs2(psi[insert_zero_bits(t, a.lowmask, a.r) | a.omask]);
    const double s = m_block_sum(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// Partials in order -> norm[0] (and a copy for the caller).
__global__ void k_kept_norm_finish(const double *part, int nparts, double *norm, double *copy) {
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int p = 0; p < nparts; ++p) s += part[p];
    norm[0] = s;
    if (copy) copy[0] = s;
}

// psi_i <- psi_i / sqrt(norm) where the measured bits of i spell the
// outcome, 0 elsewhere (all amplitudes 0 when the norm is 0).  VEC
// consecutive amplitudes per thread (16 bytes); only kept ones are read.
template <typename C, int VEC>
__global__ void __launch_bounds__(MT) k_collapse_apply(C *__restrict__ psi, CollapseArgs a, const double *norm) {
    const uint64_t nv = a.N / VEC;
    const double nrm = norm[0];
    const double sc = nrm > 0.0 ? 1.0 / sqrt(nrm) : 0.0;
    const uint64_t stride = (uint64_t)gridDim.x * MT;
    for (uint64_t v = (uint64_t)blockIdx.x * MT + threadIdx.x; v < nv; v += stride) {
        const uint64_t i0 = v * VEC;
        C o[VEC] = {};
        bool any = false;
#pragma unroll
        for (int j = 0; j < VEC; ++j) any |= ((i0 + j) & a.qmask) == a.omask;
        if (any) {
            if constexpr (VEC == 2) {
                const float4 q = *reinterpret_cast<const float4 *>(psi + i0);
                o[0].x = q.x;
                o[0].y = q.y;
                o[1].x = q.z;
                o[1].y = q.w;
            } else {
#pragma unroll
                for (int j = 0; j < VEC; ++j) o[j] = psi[i0 + j];
            }
        }
#pragma unroll
        for (int j = 0; j < VEC; ++j) {
            const bool keep = ((i0 + j) & a.qmask) == a.omask;
            o[j].x = keep ? (decltype(o[j].x))((double)o[j].x * sc) : 0;
            o[j].y = keep ? (decltype(o[j].y))((double)o[j].y * sc) : 0;
        }
        if constexpr (VEC == 2) {
            *reinterpret_cast<float4 *>(psi + i0) = make_float4(o[0].x, o[0].y, o[1].x, o[1].y);
        } else {
#pragma unroll
            for (int j = 0; j < VEC; ++j) psi[i0 + j] = o[j];
        }
    }
}

// ---------------------------------------------------------------- cumulative sums
//
// c_m = p_0 + ... + p_m in a fixed order: the R outcomes are cut into G
// contiguous ranges; pass 1 sums each range (fixed strided order, block
// tree), pass 2 scans the G range sums in one thread, pass 3 scans each range
// in tiles of SB = 4 * MT entries (per-thread sequential, wave and block
// scans in fixed trees) carrying the running total from tile to tile.

constexpr int SB = 4 * MT;

__global__ void __launch_bounds__(MT) k_range_sums(const double *__restrict__ p, uint64_t R, uint64_t span,
                                                  double *sums) {
    __shared__ double sh[MT / 64];
    const uint64_t b0 = (uint64_t)blockIdx.x * span;
    const uint64_t e = b0 + span < R ? b0 + span : R;
    double acc = 0.0;
    for (uint64_t i = b0 + threadIdx.x; i < e; i += MT) acc += p[i];
    const double s = m_block_sum(acc, sh);
    if (threadIdx.x == 0) sums[blockIdx.x] = s;
}

__global__ void k_range_offsets(double *sums, int G) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double run = 0.0;
    for (int g = 0; g < G; ++g) {
        const double s = sums[g];
        sums[g] = run;   // exclusive offset of range g
        run += s;
    }
}

// Inclusive scan over the block of per-thread totals: wave scan by shuffles
// (fixed pairs), then the four wave totals in order.  Returns the exclusive
// prefix of this thread; *total receives the block total.
__device__ inline double block_exclusive(double v, double *sh, double *total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double inc = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const double o = __shfl_up(inc, off, 64);
        if (lane >= off) inc += o;
    }
    double exl = __shfl_up(inc, 1, 64);   // inclusive value of the lane below
    if (lane == 0) exl = 0.0;
    if (lane == 63) sh[w] = inc;
    __syncthreads();
    double woff = 0.0, tot = 0.0;
    for (int i = 0; i < MT / 64; ++i) {
        if (i == w) woff = tot;
        tot += sh[i];
    }
    __syncthreads();
    *total = tot;
    return woff + exl;
}

__global__ void __launch_bounds__(MT) k_range_scan(const double *__restrict__ p, uint64_t R, uint64_t span,
                                                  const double *offsets, double *__restrict__ c) {
    __shared__ double sh[MT / 64];
    const uint64_t b0 = (uint64_t)blockIdx.x * span;
    const uint64_t e = b0 + span < R ? b0 + span : R;
    double carry = offsets[blockIdx.x];
    for (uint64_t t0 = b0; t0 < e; t0 += SB) {
        const uint64_t i = t0 + 4 * (uint64_t)threadIdx.x;
        double x[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) x[j] = i + j < e ? p[i + j] : 0.0;
        double s[4];
        s[0] = x[0];
#pragma unroll
        for (int j = 1; j < 4; ++j) s[j] = s[j - 1] + x[j];
        double tot;
        const double ex = block_exclusive(s[3], sh, &tot);
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (i + j < e) c[i + j] = carry + (ex + s[j]);
        carry += tot;
    }
}

// ---------------------------------------------------------------- sampling

// Smallest m with u T < c_m (T = c_{R-1}), clamped to R - 1.  A rounding
// step of c at an outcome of probability 0 would let it be drawn; the draw
// then moves on to the next outcome of non-zero probability (the exact
// answer), or back to the last one at the end.
__global__ void __launch_bounds__(MT) k_sample_cdf(const double *__restrict__ c, const double *__restrict__ p,
                                                   uint64_t R, const double *__restrict__ u, uint64_t nshots,
                                                   int64_t *samples, unsigned long long *counts) {
    const double T = c[R - 1];
    const uint64_t stride = (uint64_t)gridDim.x * MT;
    for (uint64_t s = (uint64_t)blockIdx.x * MT + threadIdx.x; s < nshots; s += stride) {
        const double x = u[s] * T;
        uint64_t lo = 0, hi = R - 1;
        while (lo < hi) {
            const uint64_t mid = lo + ((hi - lo) >> 1);
            if (x < c[mid]) hi = mid;
            else lo = mid + 1;
        }
        while (p[lo] == 0.0 && lo + 1 < R) ++lo;
        while (p[lo] == 0.0 && lo > 0) --lo;
        if (samples) samples[s] = (int64_t)lo;
        if (counts) atomicAdd(&counts[lo], 1ull);
    }
}

// One thread per chain: at step s the proposal y = prop[s * C + c] replaces
// the held outcome x when u[s * C + c] p(x) < p(y); the held outcome is
// counted after every step.  Proposals outside [0, R) are rejected, starts
// outside it begin at 0.
__global__ void __launch_bounds__(MT) k_metropolis(const double *__restrict__ p, uint64_t R,
                                                   const int64_t *__restrict__ starts,
                                                   const int64_t *__restrict__ prop, const double *__restrict__ u,
                                                   uint64_t C, uint64_t steps, unsigned long long *counts) {
    const uint64_t c = (uint64_t)blockIdx.x * MT + threadIdx.x;
    if (c >= C) return;
    uint64_t x = (uint64_t)starts[c];
    if (x >= R) x = 0;
    double px = p[x];
    for (uint64_t s = 0; s < steps; ++s) {
        const uint64_t y = (uint64_t)prop[s * C + c];
        if (y < R) {
            const double py = p[y];
            if (u[s * C + c] * px < py) {
                x = y;
                px = py;
            }
        }
        atomicAdd(&counts[x], 1ull);
    }
}

__global__ void k_zero_u64(unsigned long long *a, uint64_t count) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) a[i] = 0ull;
}

unsigned grid_cap(uint64_t items, uint64_t per_block, uint64_t cap) {
    uint64_t b = (items + per_block - 1) / per_block;
    if (b > cap) b = cap;
    if (b < 1) b = 1;
    return (unsigned)b;
}

template <typename C>
int collapse_t(void *state, int n, const int *qubits, int r, uint64_t outcome, double *prob_dev, hipStream_t s) {
    CollapseArgs a;
    std::memset(&a, 0, sizeof(a));
    std::vector<int> sorted(qubits, qubits + r);
    std::sort(sorted.begin(), sorted.end());
    for (int i = 0; i < r; ++i) a.lowmask[i] = (1ull << sorted[i]) - 1ull;
    for (int j = 0; j < r; ++j) {
        a.qmask |= 1ull << qubits[j];
        if ((outcome >> (r - 1 - j)) & 1) a.omask |= 1ull << qubits[j];
    }
    a.r = r;
    a.nkept = 1ull << (n - r);
    a.N = 1ull << n;
    const unsigned g = grid_cap(a.nkept, MT * 8, (uint64_t)device_sm_count() * 8);
    StagingSlot slot;
    int st = staging_acquire(sizeof(double) * (g + 1), &slot);
    if (st) return st;
    double *part = (double *)slot.dev;
    double *norm = part + g;
    hipLaunchKernelGGL((k_kept_norm<C>), dim3(g), dim3(MT), 0, s, (const C *)state, a, part);
    hipLaunchKernelGGL(k_kept_norm_finish, dim3(1), dim3(64), 0, s, part, (int)g, norm, prob_dev);
    // complex64: two amplitudes (16 bytes) per thread
    constexpr int VEC = sizeof(C) == 8 ? 2 : 1;
    hipLaunchKernelGGL((k_collapse_apply<C, VEC>), dim3(grid_cap(a.N / VEC, MT, 0xffffffffull / MT)), dim3(MT), 0, s,
                       (C *)state, a, (const double *)norm);
    hipError_t e = hipGetLastError();
    staging_release(slot, s);
    if (e != hipSuccess) return hip_fail(e, "collapse launch");
    return QSV_OK;
}

}  // namespace

}  // namespace qsv

using namespace qsv;

extern "C" {

int qsv_collapse(void *state, int n, int dtype, const int *qubits, int r, uint64_t outcome, double *prob_dev,
                 void *stream) {
    if (dtype != QSV_C64 && dtype != QSV_C128) return fail(QSV_ERR_DTYPE, "dtype must be QSV_C64 or QSV_C128");
    if (n < 1 || n > QSV_MAX_QUBITS) return fail(QSV_ERR_NQUBITS, "n must be in [1, 40]");
    if (!state || !qubits) return fail(QSV_ERR_NULL, "NULL pointer");
    if (((uintptr_t)state & 15) != 0) return fail(QSV_ERR_ALIGN, "state must be 16-byte aligned");
    if (r < 1 || r > n) return fail(QSV_ERR_ARITY, "number of measured qubits must be in [1, n]");
    uint64_t seen = 0;
    for (int j = 0; j < r; ++j) {
        if (qubits[j] < 0 || qubits[j] >= n) return fail(QSV_ERR_QUBIT_RANGE, "measured qubit out of range");
        if (seen & (1ull << qubits[j])) return fail(QSV_ERR_QUBIT_DUP, "measured qubit repeats");
        seen |= 1ull << qubits[j];
    }
    if (r < 64 && (outcome >> r) != 0) return fail(QSV_ERR_ARG, "outcome has bits above the measured qubits");
    if (prob_dev && ranges_overlap(state, (uint64_t)(dtype == QSV_C64 ? 8 : 16) << n, prob_dev, sizeof(double)))
        return fail(QSV_ERR_ARG, "prob_dev must not overlap the state");
    return dtype == QSV_C64 ? collapse_t<float2>(state, n, qubits, r, outcome, prob_dev, (hipStream_t)stream)
                            : collapse_t<double2>(state, n, qubits, r, outcome, prob_dev, (hipStream_t)stream);
}

int qsv_sample_cdf(const double *probs_dev, int r, const double *uniforms_dev, int64_t nshots, double *cdf_dev,
                   int64_t *samples_dev, uint64_t *counts_dev, void *stream) {
    if (r < 1 || r > QSV_MAX_QUBITS) return fail(QSV_ERR_ARITY, "number of outcome bits must be in [1, 40]");
    if (!probs_dev || !cdf_dev) return fail(QSV_ERR_NULL, "NULL probabilities or cumulative buffer");
    if (nshots < 0) return fail(QSV_ERR_ARG, "negative number of shots");
    if (nshots > 0 && !uniforms_dev) return fail(QSV_ERR_NULL, "NULL uniforms");
    hipStream_t s = (hipStream_t)stream;
    const uint64_t R = 1ull << r;
    // G ranges of whole tiles, at most 2048
    uint64_t span = SB;
    while ((R + span - 1) / span > 2048) span <<= 1;
    const int G = (int)((R + span - 1) / span);
    StagingSlot slot;
    int st = staging_acquire(sizeof(double) * G, &slot);
    if (st) return st;
    double *sums = (double *)slot.dev;
    hipLaunchKernelGGL(k_range_sums, dim3(G), dim3(MT), 0, s, probs_dev, R, span, sums);
    hipLaunchKernelGGL(k_range_offsets, dim3(1), dim3(64), 0, s, sums, G);
    hipLaunchKernelGGL(k_range_scan, dim3(G), dim3(MT), 0, s, probs_dev, R, span, (const double *)sums, cdf_dev);
    if (counts_dev)
        hipLaunchKernelGGL(k_zero_u64, dim3(grid_cap(R, MT, 4096)), dim3(MT), 0, s, (unsigned long long *)counts_dev, R);
    if (nshots > 0 && (samples_dev || counts_dev))
        hipLaunchKernelGGL(k_sample_cdf, dim3(grid_cap((uint64_t)nshots, MT, 0xffffffffull / MT)), dim3(MT), 0, s,
                           (const double *)cdf_dev, probs_dev, R, uniforms_dev, (uint64_t)nshots, samples_dev,
                           (unsigned long long *)counts_dev);
    hipError_t e = hipGetLastError();
    staging_release(slot, s);
    if (e != hipSuccess) return hip_fail(e, "sampling launch");
    return QSV_OK;
}

int qsv_sample_metropolis(const double *probs_dev, int r, const int64_t *starts_dev, const int64_t *proposals_dev,
                          const double *uniforms_dev, int nchains, int64_t steps, uint64_t *counts_dev, void *stream) {
    if (r < 1 || r > QSV_MAX_QUBITS) return fail(QSV_ERR_ARITY, "number of outcome bits must be in [1, 40]");
    if (!probs_dev || !starts_dev || !counts_dev) return fail(QSV_ERR_NULL, "NULL pointer");
    if (nchains < 1 || steps < 0) return fail(QSV_ERR_ARG, "need at least one chain and a non-negative step count");
    if (steps > 0 && (!proposals_dev || !uniforms_dev)) return fail(QSV_ERR_NULL, "NULL proposals or uniforms");
    hipStream_t s = (hipStream_t)stream;
    const uint64_t R = 1ull << r;
    hipLaunchKernelGGL(k_zero_u64, dim3(grid_cap(R, MT, 4096)), dim3(MT), 0, s, (unsigned long long *)counts_dev, R);
    if (steps > 0)
        hipLaunchKernelGGL(k_metropolis, dim3(grid_cap((uint64_t)nchains, MT, 0xffffffffull / MT)), dim3(MT), 0, s,
                           probs_dev, R, starts_dev, proposals_dev, uniforms_dev, (uint64_t)nchains, (uint64_t)steps,
                           (unsigned long long *)counts_dev);
    QSV_HIP_CHECK(hipGetLastError());
    return QSV_OK;
}

}  // extern "C"
