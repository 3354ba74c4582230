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
#include <mutex>

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
//
// out[m] = sum of |psi_i|^2 over the i whose measured bits spell m.  The
// state is read as rows of 2^w consecutive amplitudes (w = min(6, n)), one
// per lane of a wave, so every load is a fully used contiguous run whatever
// qubits are measured.  Bits below w are lane bits, the others row bits.
// Rows are enumerated as items: the low bits of an item are the unmeasured
// row bits (ascending positions), the high bits the measured row bits
// ordered by their place in m (a "job" = one value of them).  Stepping to
// the next item flips its trailing ones, which flips a fixed set of row
// bits and of m bits: both updates are one XOR with a table entry (wave
// uniform, scalar).  A wave takes a contiguous range of items; within a
// segment (the rows of one job it covers) each lane sums its rows in order,
// then the unmeasured lane bits are summed by a fixed shuffle butterfly and
// the lanes with those bits 0 write m's value -- to out directly when every
// job lies within one wave, else to one slice of a partial array that a
// second launch adds up in slice order.  The decomposition depends only on
// n and the measured qubits, so results are reproducible bit for bit.

struct ProbArgs {
    uint64_t dbit[QSV_MAX_QUBITS];   // row bit of item bit t
    uint64_t dlow[QSV_MAX_QUBITS];   // row bits that flip when item bits 0..t flip
    uint64_t ebit[QSV_MAX_QUBITS];   // m bit of job bit t
    uint64_t elow[QSV_MAX_QUBITS];   // m bits that flip when job bits 0..t flip
    uint64_t mlane[64];              // m bits of each lane's own measured lane bits
    uint64_t nitems;                 // 2^(n - w)
    uint64_t R;                      // 2^r outcomes
    int nh, nhu;                     // row bits, unmeasured row bits
    int w;                           // lane bits
    int lane_um;                     // mask of the unmeasured lane bits
    int ipw_log;                     // log2 items (rows) per wave
    int seg_log;                     // log2 rows per segment
    int P;                           // slices per job (1: write out directly)
};

constexpr int PB = 8;   // rows loaded per batch by every lane (16 measured slower)

template <typename C>
__global__ void __launch_bounds__(256) k_probs(const C *__restrict__ psi, ProbArgs pa, double *__restrict__ dst) {
    const int lane = threadIdx.x & 63;
    const uint64_t wave = (uint64_t)blockIdx.x * 4 + (uint64_t)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint64_t ipw = 1ull << pa.ipw_log;
    uint64_t item = wave << pa.ipw_log;
    if (item >= pa.nitems) return;   // the whole wave
    uint64_t row = 0;
    for (int t = 0; t < pa.nh; ++t)
        if ((item >> t) & 1) row ^= pa.dbit[t];
    uint64_t job = item >> pa.nhu;
    uint64_t mrow = 0;
    for (int t = 0; t < pa.nh - pa.nhu; ++t)
        if ((job >> t) & 1) mrow ^= pa.ebit[t];
    const bool live = lane < (1 << pa.w);
    const uint64_t mlane = pa.mlane[lane];
    const bool leader = live && (lane & pa.lane_um) == 0;
    const uint64_t segmask = (1ull << pa.seg_log) - 1;
    const uint64_t slice = pa.P > 1 ? ((item & ((1ull << pa.nhu) - 1)) >> pa.ipw_log) : 0;
    double acc = 0.0;
    for (uint64_t k = 0; k < ipw; k += PB) {
        double v[PB];
#pragma unroll
        for (int b = 0; b < PB; ++b) {
            v[b] = 0.0;
            if (k + b < ipw) {
                if (live) v[b] = abs2d(psi[(row << pa.w) | (uint64_t)lane]);
                const uint64_t ones = __builtin_ctzll(~item);   // trailing ones of the item
                if (ones < (uint64_t)pa.nh) row ^= pa.dlow[ones];
                ++item;
            }
        }
#pragma unroll
        for (int b = 0; b < PB; ++b) {
            if (k + b >= ipw) break;
            acc += v[b];
            if (((k + b + 1) & segmask) == 0) {   // end of a segment (wave uniform)
                double t = acc;
#pragma unroll
                for (int u = 0; u < 6; ++u)
                    if ((pa.lane_um >> u) & 1) t += __shfl_xor(t, 1 << u, 64);
                if (leader) dst[slice * pa.R + (mrow | mlane)] = t;
                acc = 0.0;
                const uint64_t jo = __builtin_ctzll(~job);
                if (jo < (uint64_t)(pa.nh - pa.nhu)) mrow ^= pa.elow[jo];
                ++job;
            }
        }
    }
}

// out[m] = sum over the P slices of part[slice * R + m], in slice order:
// one thread per outcome for few slices, else one block per outcome.
__global__ void k_probs_finish_thread(const double *__restrict__ part, uint64_t R, int P, double *__restrict__ out) {
    const uint64_t m = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= R) return;
    double s = 0.0;
    for (int p = 0; p < P; ++p) s += part[(uint64_t)p * R + m];
    out[m] = s;
}

__global__ void __launch_bounds__(RT) k_probs_finish_block(const double *__restrict__ part, uint64_t R, int P,
                                                           double *__restrict__ out) {
    __shared__ double sh[RT / 64];
    const uint64_t m = blockIdx.x;
    double s = 0.0;
    for (int p = threadIdx.x; p < P; p += RT) s += part[(uint64_t)p * R + m];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) out[m] = s;
}

// ---------------------------------------------------------------- TFIM energy

struct TfimArgs {
    uint64_t N;
    int n;
    int periodic;
    double J, h;
};

// The energy in sweeps: a sweep holds chunks of 2^L amplitudes in LDS whose
// local bits are the six lowest (64-amplitude runs) and a group of higher
// ones, and sums the X_q terms of the bits q of its group (the first sweep:
// bits 0..L-1, and every ZZ term).  Each X term is summed in exactly one
// sweep; the state is read once per sweep instead of once per high qubit.
// The first sweep covers bits 0..11 (it also sums the ZZ part: its chunks
// are kept small so more workgroups share a CU).  Later complex64 sweeps take
// 2^13-amplitude chunks in 512-thread workgroups (64 KiB of LDS, two per CU,
// the next chunk prefetched into registers): 7 new bits per sweep.
// Complex128 takes 2^12-amplitude chunks in 256-thread workgroups: 6 new
// bits.  Either needs 4 sweeps at 30 qubits.
constexpr int SWL = 14;   // local bits per sweep chunk, at most (the TfimSweep arrays)
template <typename C> struct TfimShape;
template <> struct TfimShape<float2> {
    static constexpr int RT = 512, TB = 9, L = 13, L0 = 12;   // L0: the first sweep's chunk bits
    static constexpr bool PF = true;
    static constexpr int WPE = 4;   // waves per SIMD: two workgroups per CU
};
template <> struct TfimShape<double2> {
    static constexpr int RT = 256, TB = 8, L = 12, L0 = 12;
    static constexpr bool PF = false;
    static constexpr int WPE = 2;   // the 64 KiB chunk in LDS allows two workgroups per CU
};
struct TfimSweep {
    TfimArgs a;
    int L;                 // local bits of this sweep
    int xfrom;             // local index of the first bit whose X term this sweep sums
    int zz;                // this sweep also sums the ZZ part
    int pos[SWL];          // global bit of local bit j (ascending)
    uint64_t lowmask[SWL]; // (1 << pos[j]) - 1, for the chunk base
};

// Z_q Z_{q+1} summed over the open chain is (n - 1) - 2 popcount of the
// differing neighbour bits; the periodic bond adds the top-bottom pair.
__device__ inline double zz_closed(uint64_t i, const TfimArgs &a) {
    const uint64_t chain = (a.n >= 2) ? ((1ull << (a.n - 1)) - 1ull) : 0ull;
    double z = (double)(a.n - 1) - 2.0 * (double)__popcll((i ^ (i >> 1)) & chain);
    if (a.periodic && a.n > 2) z += (((i >> (a.n - 1)) ^ i) & 1) ? -1.0 : 1.0;
    return z;
}

// Local index l = t + RT k: thread bits 0..TB-1 from t, register bits from
// k (local bits TB.. of the chunk).  X pairs on register bits stay in the
// thread's registers; pairs on thread bits read the partner from LDS.
// LT > 0: the sweep's local bits (LT), its first X bit (XF) and whether it
// sums the ZZ part (ZZ) are compile-time constants, so every loop below
// unrolls; LT = 0 reads them from the arguments (small states).
template <typename C, int LT, int XF, bool ZZ>
__global__ void __launch_bounds__(TfimShape<C>::RT) __attribute__((amdgpu_waves_per_eu(TfimShape<C>::WPE)))
k_tfim_sweep(const C *__restrict__ psi, TfimSweep w, double *part) {
    typedef TfimShape<C> S;
    constexpr int RT_ = S::RT, TB = S::TB;
    constexpr int KMAX = (1 << S::L) / RT_;
    constexpr bool PF = S::PF && LT > 0 && !ZZ;   // the ZZ sweep has no registers to spare
    __shared__ C ch[1 << (LT > 0 ? LT : S::L)];
    __shared__ double sh[RT_ / 64];
    // (w itself stays unmodified: a written kernel argument would be copied
    // to scratch memory)
    const int L = LT > 0 ? LT : w.L;
    const int xfrom = LT > 0 ? XF : w.xfrom;
    const bool zzp = LT > 0 ? ZZ : (w.zz != 0);
    const int csize = 1 << L;
    const int K = csize >= RT_ ? csize / RT_ : 1;
    const int t = threadIdx.x;
    const bool live = t < csize;
    const uint64_t nchunks = w.a.N >> L;
    // global offsets of the thread's and the register's local bits (the
    // first sweep, CONTIG, has local bits 0..L-1: offsets t and k << TB)
    constexpr bool CONTIG = LT > 0 && ZZ;
    uint64_t off_t = 0;
    for (int j = 0; j < L && j < TB; ++j) off_t |= (uint64_t)((t >> j) & 1) << w.pos[j];
    uint64_t off_k[CONTIG ? 1 : KMAX];
    if constexpr (!CONTIG) {
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
            off_k[k] = 0;
            for (int j = TB; j < L; ++j) off_k[k] |= (uint64_t)((k >> (j - TB)) & 1) << w.pos[j];
        }
    }
    auto offset = [&](int k) -> uint64_t {
        if constexpr (CONTIG) return (uint64_t)t | ((uint64_t)k << TB);
        else return off_t | off_k[k];
    };
    auto chunk_base = [&](uint64_t c) {   // chunk index with zeros inserted at the local bits
        uint64_t base = c;
        for (int j = 0; j < L; ++j) {
            const uint64_t lo = base & w.lowmask[j];
            base = lo | ((base ^ lo) << 1);
        }
        return base;
    };
    auto load = [&](C *dst, uint64_t base) {
#pragma unroll
        for (int k = 0; k < KMAX; ++k)
            if (k < K && live) dst[k] = psi[base | offset(k)];
    };
    double zz = 0.0, xx = 0.0;
    uint64_t c = blockIdx.x;
    C v[KMAX];
    if constexpr (PF) {
        if (c < nchunks) load(v, chunk_base(c));
    }
    for (; c < nchunks; c += gridDim.x) {
        const uint64_t base = chunk_base(c);
        C vn[PF ? KMAX : 1];
        if constexpr (PF) {
            const uint64_t cn = c + gridDim.x;
            if (cn < nchunks) load(vn, chunk_base(cn));
        } else {
            load(v, base);
        }
#pragma unroll
        for (int k = 0; k < KMAX; ++k)
            if (k < K && live) ch[t + RT_ * k] = v[k];
        __syncthreads();
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
            if (k >= K || !live) continue;
            if (zzp) zz += abs2d(v[k]) * zz_closed(base | offset(k), w.a);
            // thread bits
#pragma unroll
            for (int j = 0; j < TB; ++j) {
                if (j < xfrom || j >= L) continue;
                if ((t >> j) & 1) continue;
                const C u = ch[(t | (1 << j)) + RT_ * k];   // (L > j: the partner exists)
                xx += 2.0 * ((double)v[k].x * (double)u.x + (double)v[k].y * (double)u.y);
            }
            // register bits
#pragma unroll
            for (int r = 0; r < S::L - TB; ++r) {
                const int j = TB + r;
                if (j < xfrom || j >= L || ((k >> r) & 1)) continue;
                const C u = v[k | (1 << r)];
                xx += 2.0 * ((double)v[k].x * (double)u.x + (double)v[k].y * (double)u.y);
            }
        }
        __syncthreads();
        if constexpr (PF) {
#pragma unroll
            for (int k = 0; k < KMAX; ++k) v[k] = vn[k];
        }
    }
    const double s1 = block_sum(w.a.J * zz, sh);
    const double s2 = block_sum(w.a.h * xx, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s1 + s2;
}

// H psi in the energy's sweeps: the first sweep writes out = J zz(i) psi_i +
// h (sum of the partners of i on its X bits), every later sweep adds the
// partners on its new bits (out read, added to, written back).  Sums in
// fp64; out holds the state's type between sweeps.
template <typename C, int LT, int XF, bool FIRST>
__global__ void __launch_bounds__(TfimShape<C>::RT) __attribute__((amdgpu_waves_per_eu(TfimShape<C>::WPE)))
k_apply_tfim_sweep(const C *__restrict__ psi, C *__restrict__ out, TfimSweep w) {
    typedef TfimShape<C> S;
    constexpr int RT_ = S::RT, TB = S::TB;
    constexpr int KMAX = (1 << S::L) / RT_;
    __shared__ C ch[1 << (LT > 0 ? LT : S::L)];
    const int L = LT > 0 ? LT : w.L;
    const int xfrom = LT > 0 ? XF : w.xfrom;
    const bool first = LT > 0 ? FIRST : (w.zz != 0);
    const int csize = 1 << L;
    const int K = csize >= RT_ ? csize / RT_ : 1;
    const int t = threadIdx.x;
    const bool live = t < csize;
    const uint64_t nchunks = w.a.N >> L;
    constexpr bool CONTIG = LT > 0 && FIRST;   // local bits 0..L-1
    uint64_t off_t = 0;
    for (int j = 0; j < L && j < TB; ++j) off_t |= (uint64_t)((t >> j) & 1) << w.pos[j];
    uint64_t off_k[CONTIG ? 1 : KMAX];
    if constexpr (!CONTIG) {
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
            off_k[k] = 0;
            for (int j = TB; j < L; ++j) off_k[k] |= (uint64_t)((k >> (j - TB)) & 1) << w.pos[j];
        }
    }
    auto offset = [&](int k) -> uint64_t {
        if constexpr (CONTIG) return (uint64_t)t | ((uint64_t)k << TB);
        else return off_t | off_k[k];
    };
    for (uint64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        uint64_t base = c;
        for (int j = 0; j < L; ++j) {
            const uint64_t lo = base & w.lowmask[j];
            base = lo | ((base ^ lo) << 1);
        }
        C v[KMAX];
#pragma unroll
        for (int k = 0; k < KMAX; ++k)
            if (k < K && live) v[k] = psi[base | offset(k)];
#pragma unroll
        for (int k = 0; k < KMAX; ++k)
            if (k < K && live) ch[t + RT_ * k] = v[k];
        __syncthreads();
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
            if (k >= K || !live) continue;
            const uint64_t i = base | offset(k);
            double ax, ay;
            if (first) {
                const double z = w.a.J * zz_closed(i, w.a);
                ax = z * (double)v[k].x;
                ay = z * (double)v[k].y;
            } else {
                const C o = out[i];
                ax = (double)o.x;
                ay = (double)o.y;
            }
            double sx = 0.0, sy = 0.0;
#pragma unroll
            for (int j = 0; j < TB; ++j) {   // thread bits: the partner from LDS
                if (j < xfrom || j >= L) continue;
                const C u = ch[(t ^ (1 << j)) + RT_ * k];
                sx += (double)u.x;
                sy += (double)u.y;
            }
#pragma unroll
            for (int r = 0; r < S::L - TB; ++r) {   // register bits
                const int j = TB + r;
                if (j < xfrom || j >= L) continue;
                const C u = v[k ^ (1 << r)];
                sx += (double)u.x;
                sy += (double)u.y;
            }
            C y;
            y.x = (decltype(y.x))(ax + w.a.h * sx);
            y.y = (decltype(y.y))(ay + w.a.h * sy);
            out[i] = y;
        }
        __syncthreads();
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

// Largest partial array of the probabilities reduction (doubles) and the
// most slices a job is cut into.
// Partials of one call: at most 2^18 doubles (2 MiB, the largest staging
// span); few outcomes spread over up to 16384 slices, so that measuring a
// handful of qubits still gives every CU dozens of waves.
constexpr uint64_t PROB_PART_MAX = 1ull << 18;
constexpr uint64_t PROB_SLICES_MAX = 16384;

// The decomposition of a probabilities launch (host only; no HIP call).
int prob_args(int n, const int *qubits, int r, ProbArgs *out) {
    ProbArgs &pa = *out;
    std::memset(&pa, 0, sizeof(pa));
    const int w = n < 6 ? n : 6;
    pa.w = w;
    pa.nh = n - w;
    pa.R = 1ull << r;
    int mpos[QSV_MAX_QUBITS];   // m bit of each qubit, -1 if not measured
    for (int q = 0; q < n; ++q) mpos[q] = -1;
    for (int j = 0; j < r; ++j) mpos[qubits[j]] = r - 1 - j;
    for (int q = 0; q < w; ++q)
        if (mpos[q] < 0) pa.lane_um |= 1 << q;
    for (int l = 0; l < 64; ++l)
        for (int q = 0; q < w; ++q)
            if (mpos[q] >= 0 && ((l >> q) & 1)) pa.mlane[l] |= 1ull << mpos[q];
    // item bits: unmeasured row bits (ascending), then measured row bits by m bit
    int t = 0;
    for (int q = w; q < n; ++q)
        if (mpos[q] < 0) pa.dbit[t++] = 1ull << (q - w);
    pa.nhu = t;
    for (int mb = 0; mb < r; ++mb)
        for (int q = w; q < n; ++q)
            if (mpos[q] == mb) {
                pa.ebit[t - pa.nhu] = 1ull << mb;
                pa.dbit[t++] = 1ull << (q - w);
            }
    uint64_t d = 0, e = 0;
    for (int b = 0; b < pa.nh; ++b) {
        d ^= pa.dbit[b];
        pa.dlow[b] = d;
    }
    for (int b = 0; b < pa.nh - pa.nhu; ++b) {
        e ^= pa.ebit[b];
        pa.elow[b] = e;
    }
    pa.nitems = 1ull << pa.nh;
    const uint64_t RS = 1ull << pa.nhu;   // rows of one job
    // items per wave: at most 2^17 waves, at least one batch where possible
    uint64_t ipw = pa.nitems >> 17;
    if (ipw < PB) ipw = PB;
    if (ipw > pa.nitems) ipw = pa.nitems;
    uint64_t P = 1;
    if (ipw < RS) {
        P = RS / ipw;
        uint64_t pmax = PROB_PART_MAX / pa.R;
        if (pmax > PROB_SLICES_MAX) pmax = PROB_SLICES_MAX;
        if (pmax < 1) pmax = 1;
        if (P > pmax) {
            P = pmax;
            ipw = RS / P;
        }
    }
    pa.P = (int)P;
    pa.ipw_log = __builtin_ctzll(ipw);
    pa.seg_log = __builtin_ctzll(ipw < RS ? ipw : RS);
    return QSV_OK;
}

// `fixed_part`: a partial array of PROB_PART_MAX doubles to use instead of a
// staging slot (NULL: a staging slot).
template <typename C>
static int probs_t(const void *state, int n, const int *qubits, int r, double *out, hipStream_t s,
                   double *fixed_part) {
    ProbArgs pa;
    prob_args(n, qubits, r, &pa);
    const uint64_t waves = pa.nitems >> pa.ipw_log;
    const unsigned blocks = (unsigned)((waves + 3) / 4);
    if (pa.P == 1) {
        hipLaunchKernelGGL((k_probs<C>), dim3(blocks), dim3(256), 0, s, (const C *)state, pa, out);
        QSV_HIP_CHECK(hipGetLastError());
        return QSV_OK;
    }
    if (pa.R * (uint64_t)pa.P > PROB_PART_MAX) return fail(QSV_ERR_ARG, "internal: partial array above its bound");
    StagingSlot slot;
    double *part = fixed_part;
    if (!part) {
        int st = staging_acquire(sizeof(double) * pa.R * pa.P, &slot);
        if (st) return st;
        part = (double *)slot.dev;
    }
    hipLaunchKernelGGL((k_probs<C>), dim3(blocks), dim3(256), 0, s, (const C *)state, pa, part);
    if (pa.P >= 64)
        hipLaunchKernelGGL(k_probs_finish_block, dim3((unsigned)pa.R), dim3(RT), 0, s, part, pa.R, pa.P, out);
    else
        hipLaunchKernelGGL(k_probs_finish_thread, dim3((unsigned)((pa.R + 255) / 256)), dim3(256), 0, s, part, pa.R,
                           pa.P, out);
    hipError_t e = hipGetLastError();
    if (!fixed_part) staging_release(slot, s);
    if (e != hipSuccess) return hip_fail(e, "probabilities launch");
    return QSV_OK;
}

// ---------------------------------------------------------------- no-allocation variant
//
// qsv_probabilities_noalloc keeps its partial sums in this file-scope device
// array (one copy per GPU, held until the process ends) instead of the
// staging ring, so it never allocates.  Host code reaches the array only
// through the device address hipGetSymbolAddress returns for the current
// device, looked up once per device.

static __device__ __align__(256) double scratch[PROB_PART_MAX];

namespace {
std::mutex g_scratch_mu;
double *g_scratch_ptr[64] = {nullptr};
}  // namespace

static int scratch_address(double **out) {
    int dev = 0;
    QSV_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(QSV_ERR_ARG, "device index above 63");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        QSV_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(QSV_ERR_HIP, "no device address for the probabilities scratch array");
        g_scratch_ptr[dev] = (double *)p;
    }
    *out = g_scratch_ptr[dev];
    return QSV_OK;
}

// The sweeps of a TFIM energy or H psi: bits 0..L0-1 (with the ZZ part),
// then the six lowest with the next LS - 6 bits.
template <typename C> static std::vector<TfimSweep> tfim_sweeps(const TfimArgs &a) {
    const int n = a.n;
    typedef TfimShape<C> S;
    constexpr int LS = S::L;
    std::vector<TfimSweep> sw;
    const int L0 = n < S::L0 ? n : S::L0;
    for (int first = 0; first < n;) {
        TfimSweep w;
        std::memset(&w, 0, sizeof(w));
        w.a = a;
        int L = 0;
        if (first == 0) {
            for (int q = 0; q < L0; ++q) w.pos[L++] = q;
            w.xfrom = 0;
            w.zz = 1;
            first = L0;
        } else {
            // the six lowest bits, then the new ones; a last sweep with fewer
            // new bits than room keeps its full chunk shape by carrying bits
            // just below them whose X terms an earlier sweep summed
            const int m = std::min(n - first, LS - 6), fill = LS - 6 - m;
            for (int q = 0; q < 6; ++q) w.pos[L++] = q;
            for (int q = first - fill; q < first; ++q) w.pos[L++] = q;
            w.xfrom = 6 + fill;
            for (int q = first; q < first + m; ++q) w.pos[L++] = q;
            first += m;
        }
        w.L = L;
        for (int j = 0; j < L; ++j) w.lowmask[j] = (1ull << w.pos[j]) - 1ull;
        sw.push_back(w);
    }
    return sw;
}

// A later sweep: its first X bit XF = 6..LS-1 (6 plus the carried bits) as
// a compile-time constant, by recursion over XF.
template <typename C, int LS, int XF>
static void launch_later_sweep(int xfrom, dim3 G, dim3 B, hipStream_t s, const C *ps, const TfimSweep &w, double *pk) {
    if constexpr (XF >= 6) {
        if (xfrom == XF) hipLaunchKernelGGL((k_tfim_sweep<C, LS, XF, false>), G, B, 0, s, ps, w, pk);
        else launch_later_sweep<C, LS, XF - 1>(xfrom, G, B, s, ps, w, pk);
    }
}

template <typename C>
static int tfim_t(const void *state, int n, double J, double h, int periodic, double *out, hipStream_t s) {
    TfimArgs a;
    a.N = 1ull << n;
    a.n = n;
    a.periodic = periodic;
    a.J = J;
    a.h = h;
    typedef TfimShape<C> S;
    constexpr int LS = S::L;
    const std::vector<TfimSweep> sw = tfim_sweeps<C>(a);
    // per sweep, exactly the workgroups of its kernel that are resident at
    // once (each walks its share of the chunks): a second, partial round of
    // workgroups would leave most CUs idle for its duration
    static int per_cu[2][3] = {{0, 0, 0}, {0, 0, 0}};   // [dtype][generic, first, later]
    int *pc = per_cu[sizeof(C) == 8 ? 0 : 1];
    if (pc[0] == 0) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&pc[0], k_tfim_sweep<C, 0, 0, false>, S::RT, 0) != hipSuccess) pc[0] = 1;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&pc[1], k_tfim_sweep<C, S::L0, 0, true>, S::RT, 0) != hipSuccess) pc[1] = 1;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&pc[2], k_tfim_sweep<C, LS, 6, false>, S::RT, 0) != hipSuccess) pc[2] = 1;
        for (int i = 0; i < 3; ++i) pc[i] = std::max(1, pc[i]);
    }
    std::vector<uint64_t> gs(sw.size()), offs(sw.size());
    uint64_t total = 0;
    for (size_t k = 0; k < sw.size(); ++k) {
        const TfimSweep &w = sw[k];
        const int kind = (w.L == S::L0 && w.xfrom == 0 && w.zz) ? 1 : (w.L == LS && !w.zz && w.xfrom >= 6 && w.xfrom < LS) ? 2 : 0;
        gs[k] = std::min<uint64_t>(a.N >> w.L, (uint64_t)device_sm_count() * pc[kind]);
        offs[k] = total;
        total += gs[k];
    }
    StagingSlot slot;
    int st = staging_acquire(sizeof(double) * total, &slot);
    if (st) return st;
    double *part = (double *)slot.dev;
    for (size_t k = 0; k < sw.size(); ++k) {   // every block writes its partial (0 when it has no chunk)
        const TfimSweep &w = sw[k];
        const dim3 G((unsigned)gs[k]), B(S::RT);
        double *pk = part + offs[k];
        const C *ps = (const C *)state;
        if (w.L == S::L0 && w.xfrom == 0 && w.zz) hipLaunchKernelGGL((k_tfim_sweep<C, S::L0, 0, true>), G, B, 0, s, ps, w, pk);
        else if (w.L == LS && !w.zz && w.xfrom >= 6 && w.xfrom < LS)
            launch_later_sweep<C, LS, LS - 1>(w.xfrom, G, B, s, ps, w, pk);
        else hipLaunchKernelGGL((k_tfim_sweep<C, 0, 0, false>), G, B, 0, s, ps, w, pk);
    }
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(64), 0, s, part, (int)total, 1, 1.0, out);
    hipError_t e = hipGetLastError();
    staging_release(slot, s);
    if (e != hipSuccess) return hip_fail(e, "tfim energy launch");
    return QSV_OK;
}

// A later H psi sweep, XF = 6..LS-1 as a compile-time constant.
template <typename C, int LS, int XF>
static void launch_later_apply(int xfrom, dim3 G, dim3 B, hipStream_t s, const C *ps, C *po, const TfimSweep &w) {
    if constexpr (XF >= 6) {
        if (xfrom == XF) hipLaunchKernelGGL((k_apply_tfim_sweep<C, LS, XF, false>), G, B, 0, s, ps, po, w);
        else launch_later_apply<C, LS, XF - 1>(xfrom, G, B, s, ps, po, w);
    }
}

template <typename C>
static int apply_tfim_t(const void *state, void *out, int n, double J, double h, int periodic, hipStream_t s) {
    TfimArgs a;
    a.N = 1ull << n;
    a.n = n;
    a.periodic = periodic;
    a.J = J;
    a.h = h;
    typedef TfimShape<C> S;
    constexpr int LS = S::L;
    const std::vector<TfimSweep> sw = tfim_sweeps<C>(a);
    static int per_cu[2][3] = {{0, 0, 0}, {0, 0, 0}};   // resident workgroups: [dtype][generic, first, later]
    int *pc = per_cu[sizeof(C) == 8 ? 0 : 1];
    if (pc[0] == 0) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&pc[0], k_apply_tfim_sweep<C, 0, 0, false>, S::RT, 0) != hipSuccess) pc[0] = 1;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&pc[1], k_apply_tfim_sweep<C, S::L0, 0, true>, S::RT, 0) != hipSuccess) pc[1] = 1;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&pc[2], k_apply_tfim_sweep<C, LS, 6, false>, S::RT, 0) != hipSuccess) pc[2] = 1;
        for (int i = 0; i < 3; ++i) pc[i] = std::max(1, pc[i]);
    }
    const C *ps = (const C *)state;
    C *po = (C *)out;
    for (const TfimSweep &w : sw) {   // in stream order: each later sweep adds to what the one before wrote
        const int kind = (w.L == S::L0 && w.xfrom == 0 && w.zz) ? 1 : (w.L == LS && !w.zz && w.xfrom >= 6 && w.xfrom < LS) ? 2 : 0;
        const uint64_t g = std::min<uint64_t>(a.N >> w.L, (uint64_t)device_sm_count() * pc[kind]);
        const dim3 G((unsigned)g), B(S::RT);
        if (kind == 1) hipLaunchKernelGGL((k_apply_tfim_sweep<C, S::L0, 0, true>), G, B, 0, s, ps, po, w);
        else if (kind == 2) launch_later_apply<C, LS, LS - 1>(w.xfrom, G, B, s, ps, po, w);
        else hipLaunchKernelGGL((k_apply_tfim_sweep<C, 0, 0, false>), G, B, 0, s, ps, po, w);
    }
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
    if (ranges_overlap(state, (uint64_t)(dtype == QSV_C64 ? 8 : 16) << n, out_dev, (uint64_t)8 << r))
        return fail(QSV_ERR_ARG, "out_dev must not overlap the state");
    uint64_t seen = 0;
    for (int j = 0; j < r; ++j) {
        if (qubits[j] < 0 || qubits[j] >= n) return fail(QSV_ERR_QUBIT_RANGE, "measured qubit out of range");
        if (seen & (1ull << qubits[j])) return fail(QSV_ERR_QUBIT_DUP, "measured qubit repeats");
        seen |= 1ull << qubits[j];
    }
    return dtype == QSV_C64 ? probs_t<float2>(state, n, qubits, r, out_dev, (hipStream_t)stream, nullptr)
                            : probs_t<double2>(state, n, qubits, r, out_dev, (hipStream_t)stream, nullptr);
}

int qsv_probabilities_noalloc(const void *state, int n, int dtype, const int *qubits, int r, double *out_dev,
                              void *stream) {
    int st = check_red(state, n, dtype, out_dev);
    if (st) return st;
    if (r < 1 || r > n) return fail(QSV_ERR_ARITY, "number of measured qubits must be in [1, n]");
    if (!qubits) return fail(QSV_ERR_NULL, "qubits is NULL");
    if (ranges_overlap(state, (uint64_t)(dtype == QSV_C64 ? 8 : 16) << n, out_dev, (uint64_t)8 << r))
        return fail(QSV_ERR_ARG, "out_dev must not overlap the state");
    uint64_t seen = 0;
    for (int j = 0; j < r; ++j) {
        if (qubits[j] < 0 || qubits[j] >= n) return fail(QSV_ERR_QUBIT_RANGE, "measured qubit out of range");
        if (seen & (1ull << qubits[j])) return fail(QSV_ERR_QUBIT_DUP, "measured qubit repeats");
        seen |= 1ull << qubits[j];
    }
    double *part = nullptr;
    if ((st = scratch_address(&part))) return st;
    return dtype == QSV_C64 ? probs_t<float2>(state, n, qubits, r, out_dev, (hipStream_t)stream, part)
                            : probs_t<double2>(state, n, qubits, r, out_dev, (hipStream_t)stream, part);
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
    const uint64_t bytes = (uint64_t)(dtype == QSV_C64 ? 8 : 16) << n;
    if (ranges_overlap(state, bytes, out, bytes)) return fail(QSV_ERR_ARG, "out must not overlap state");
    return dtype == QSV_C64 ? apply_tfim_t<float2>(state, out, n, J, h, periodic, (hipStream_t)stream)
                            : apply_tfim_t<double2>(state, out, n, J, h, periodic, (hipStream_t)stream);
}

}  // extern "C"
