// Bit-permutation pass: out[sigma(i)] = in[i] for a permutation sigma of the
// index bits that is its own inverse (a product of disjoint SWAP gates).
//
// The pass planner applies SWAP gates by relabelling qubits instead of moving
// data (the methodology section's specialised SWAP operator becomes free);
// whatever relabelling is left at the end of the circuit is undone here in
// one read + write of the state.  A chunk's local bits are closed under
// sigma and include the lowest bits, so both the loads and the stores are
// contiguous runs; sigma maps chunk c to chunk sigma(c), and one workgroup
// moves the pair (c, sigma(c)) through LDS, one chunk at a time, after both
// are in registers, which keeps the update in place.
#include "plan_internal.h"

namespace qsv {

constexpr int BP_THREADS = 256;
constexpr int BP_MAX_L = 12;

struct BitPermArgs {
    int32_t lpos[BP_MAX_L];        // global bit of local position l
    int32_t lperm[BP_MAX_L];       // local position l -> local position of sigma(bit)
    int32_t gperm[QSV_MAX_QUBITS]; // global bit b -> sigma(b)
    int32_t pa[QSV_MAX_QUBITS];    // non-local pairs (pa[i], pb[i]) that sigma swaps, ascending pa
    int32_t pb[QSV_MAX_QUBITS];
    int32_t fx[QSV_MAX_QUBITS];    // non-local bits sigma fixes
    int32_t m, f;
    int32_t L;
    int32_t n;
    uint64_t nitems;               // one work item per chunk pair {c, sigma(c)}
};

// Work item -> the chunk base of one representative per pair {c, sigma(c)}:
// group k < m holds the chunks whose first differing pair is pair k, with
// bit pa[k] set and pb[k] clear; group m the chunks sigma fixes.  Within a
// group the item's bits go to the pa-bits of the later pairs (neighbouring
// chunks), then their pb-bits, the fixed bits and the equal earlier pairs.
__device__ __forceinline__ uint64_t bp_item_base(uint64_t w, const BitPermArgs &a) {
    int k = 0;
    for (; k < a.m; ++k) {
        const uint64_t size = 1ull << (k + 2 * (a.m - 1 - k) + a.f);
        if (w < size) break;
        w -= size;
    }
    uint64_t b = k < a.m ? 1ull << a.pa[k] : 0ull;
    int i = 0;
    for (int j = k + 1; j < a.m; ++j, ++i) b |= ((w >> i) & 1ull) << a.pa[j];
    for (int j = k + 1; j < a.m; ++j, ++i) b |= ((w >> i) & 1ull) << a.pb[j];
    for (int j = 0; j < a.f; ++j, ++i) b |= ((w >> i) & 1ull) << a.fx[j];
    for (int j = 0; j < k; ++j, ++i)
        if ((w >> i) & 1ull) b |= (1ull << a.pa[j]) | (1ull << a.pb[j]);
    return b;
}

__device__ __forceinline__ uint32_t bp_swz(uint32_t l) { return l ^ (((l >> 4) ^ (l >> 8)) & 15u); }

__device__ __forceinline__ uint64_t bp_permute_global(uint64_t x, const BitPermArgs &a) {
    uint64_t y = 0;
    for (int b = 0; b < a.n; ++b)
        if ((x >> b) & 1) y |= 1ull << a.gperm[b];
    return y;
}

// An amplitude as a plain pair (HIP's vector types keep register arrays of
// them out of registers here).  Same layout as float2 / double2.
template <typename R> struct alignas(2 * sizeof(R)) BpC {
    R x, y;
};

template <typename R>
__global__ void __launch_bounds__(BP_THREADS) k_bitperm(BpC<R> *__restrict__ psi, BitPermArgs a) {
    typedef BpC<R> C;
    constexpr int LMAX = BP_MAX_L - (sizeof(C) == 16 ? 1 : 0);
    constexpr int IT = (1 << LMAX) / BP_THREADS;   // elements per thread of the largest chunk
    __shared__ C buf[1 << LMAX];
    // scatter tables: local index l = (hi << 6) | lo -> global offset, and the
    // local permutation, split in 6-bit halves
    __shared__ uint64_t sc_lo[64], sc_hi[64];
    __shared__ uint32_t lm_lo[64], lm_hi[64];
    const int L = a.L;
    const uint32_t csize = 1u << L;
    if (threadIdx.x < 64) {
        const uint32_t x = threadIdx.x;
        uint64_t slo = 0, shi = 0;
        uint32_t mlo = 0, mhi = 0;
        for (int i = 0; i < L; ++i) {
            const int src_bit = i < 6 ? i : i - 6;
            const bool bit = (x >> src_bit) & 1;
            if (!bit) continue;
            if (i < 6) {
                slo |= 1ull << a.lpos[i];
                mlo |= 1u << a.lperm[i];
            } else if (i < 12) {
                shi |= 1ull << a.lpos[i];
                mhi |= 1u << a.lperm[i];
            }
        }
        sc_lo[x] = slo;
        sc_hi[x] = shi;
        lm_lo[x] = mlo;
        lm_hi[x] = mhi;
    }
    __syncthreads();
    // One work item per workgroup (a one-shot grid: the hardware starts the
    // next workgroups while earlier ones store, which keeps loads and stores
    // overlapped); each item is one pair of chunks (or a chunk sigma fixes),
    // which its workgroup moves whole.
    for (uint64_t w = blockIdx.x; w < a.nitems; w += gridDim.x) {
        const uint64_t base = bp_item_base(w, a);
        const uint64_t pbase = bp_permute_global(base, a);   // non-local bits only (local set is closed)
        const bool pair = pbase != base;
        // Both chunks are loaded before anything is stored; each thread writes
        // its loaded values to LDS before the barrier that precedes the first
        // store, so every load of the pair has completed by then (in place).
        // (real and imaginary parts in arrays of their own, which stay in registers)
        R r0x[IT], r0y[IT], r1x[IT], r1y[IT];
#pragma unroll
        for (int i = 0; i < IT; ++i) {
            const uint32_t l = threadIdx.x + i * BP_THREADS;
            if (l < csize) {
                const uint64_t off = sc_lo[l & 63] | sc_hi[l >> 6];
                const C x = psi[base | off];
                r0x[i] = x.x;
                r0y[i] = x.y;
                if (pair) {
                    const C y = psi[pbase | off];
                    r1x[i] = y.x;
                    r1y[i] = y.y;
                }
            }
        }
        // element l of chunk c lands at local position lmap(l) of chunk sigma(c):
        // every output position lo reads its source lmap(lo) (sigma is an involution)
        __syncthreads();   // the previous pair's LDS reads are done
#pragma unroll
        for (int i = 0; i < IT; ++i) {
            const uint32_t l = threadIdx.x + i * BP_THREADS;
            if (l < csize) buf[bp_swz(l)] = C{r0x[i], r0y[i]};
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < IT; ++i) {
            const uint32_t lo = threadIdx.x + i * BP_THREADS;
            if (lo < csize) {
                const C x = buf[bp_swz(lm_lo[lo & 63] | lm_hi[lo >> 6])];
                r0x[i] = x.x;
                r0y[i] = x.y;
            }
        }
        if (pair) {
            __syncthreads();
#pragma unroll
            for (int i = 0; i < IT; ++i) {
                const uint32_t l = threadIdx.x + i * BP_THREADS;
                if (l < csize) buf[bp_swz(l)] = C{r1x[i], r1y[i]};
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < IT; ++i) {
                const uint32_t lo = threadIdx.x + i * BP_THREADS;
                if (lo < csize) {
                    const C x = buf[bp_swz(lm_lo[lo & 63] | lm_hi[lo >> 6])];
                    r1x[i] = x.x;
                    r1y[i] = x.y;
                }
            }
        }
#pragma unroll
        for (int i = 0; i < IT; ++i) {
            const uint32_t lo = threadIdx.x + i * BP_THREADS;
            if (lo < csize) {
                const uint64_t off = sc_lo[lo & 63] | sc_hi[lo >> 6];
                psi[pbase | off] = C{r0x[i], r0y[i]};
                if (pair) psi[base | off] = C{r1x[i], r1y[i]};
            }
        }
    }
}

// sigma[b] = destination bit of source bit b; sigma must be an involution.
int launch_bitperm(void *state, int n, int dtype, const std::vector<int> &sigma, hipStream_t s) {
    BitPermArgs a;
    std::memset(&a, 0, sizeof(a));
    a.n = n;
    const int Lmax = dtype == QSV_C64 ? BP_MAX_L : BP_MAX_L - 1;
    // local set: closure of the lowest bits under sigma, then more bits
    std::vector<int> in_set(n, 0);
    int cnt = 0;
    for (int b = 0; b < n && cnt < Lmax; ++b) {
        if (in_set[b]) continue;
        const int p = sigma[b];
        const int need = (p == b || in_set[p]) ? 1 : 2;
        if (cnt + need > Lmax) {
            if (b < 4) return fail(QSV_ERR_ARG, "internal: permutation chunk too small");
            continue;
        }
        in_set[b] = 1;
        in_set[p] = 1;
        cnt += need;
    }
    if (cnt > n) cnt = n;
    int L = 0;
    for (int b = 0; b < n; ++b)
        if (in_set[b]) {
            a.lpos[L] = b;
            ++L;
        }
    a.L = L;
    for (int b = 0; b < n; ++b) a.gperm[b] = sigma[b];
    {
        uint64_t lm = 0;
        for (int i = 0; i < L; ++i) lm |= 1ull << a.lpos[i];
        const PairLayout pl = pair_layout(sigma, lm);
        a.m = (int)pl.a.size();
        a.f = (int)pl.fixed.size();
        for (int i = 0; i < a.m; ++i) {
            a.pa[i] = pl.a[i];
            a.pb[i] = pl.b[i];
        }
        for (int i = 0; i < a.f; ++i) a.fx[i] = pl.fixed[i];
        a.nitems = pair_work_items(sigma, lm);
    }
    for (int i = 0; i < L; ++i) {
        const int dst = sigma[a.lpos[i]];
        for (int k = 0; k < L; ++k)
            if (a.lpos[k] == dst) a.lperm[i] = k;
    }
    // fewer than 2^32 threads per launch (HIP's total work-size limit)
    const unsigned grid = (unsigned)std::min<uint64_t>(a.nitems, 0xffffffffull / BP_THREADS);
    if (dtype == QSV_C64)
        hipLaunchKernelGGL(k_bitperm<float>, dim3(grid), dim3(BP_THREADS), 0, s, (BpC<float> *)state, a);
    else
        hipLaunchKernelGGL(k_bitperm<double>, dim3(grid), dim3(BP_THREADS), 0, s, (BpC<double> *)state, a);
    QSV_HIP_CHECK(hipGetLastError());
    return QSV_OK;
}

}  // namespace qsv
