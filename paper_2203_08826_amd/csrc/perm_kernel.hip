// Bit-permutation pass: out[sigma(i)] = in[i] for a permutation sigma of the
// index bits that is its own inverse (a product of disjoint SWAP gates).
//
// The pass planner applies SWAP gates by relabelling qubits instead of moving
// data (the methodology section's specialised SWAP operator becomes free);
// whatever relabelling is left at the end of the circuit is undone here in
// one read + write of the state.  A chunk's local bits are closed under
// sigma and include the lowest bits, so both the loads and the stores are
// contiguous runs; sigma maps chunk c to chunk sigma(c), and one workgroup
// moves the pair (c, sigma(c)) through LDS, which keeps the update in place.
#include "plan_internal.h"

namespace qsv {

constexpr int BP_THREADS = 256;
constexpr int BP_MAX_L = 12;

struct BitPermArgs {
    uint64_t lowmask[BP_MAX_L];    // sorted local bits, for the chunk base
    int32_t lpos[BP_MAX_L];        // global bit of local position l
    int32_t lperm[BP_MAX_L];       // local position l -> local position of sigma(bit)
    int32_t gperm[QSV_MAX_QUBITS]; // global bit b -> sigma(b)
    int32_t L;
    int32_t n;
    uint64_t nchunks;
};

__device__ __forceinline__ uint32_t bp_swz(uint32_t l) { return l ^ (((l >> 4) ^ (l >> 8)) & 15u); }

__device__ __forceinline__ uint64_t bp_permute_global(uint64_t x, const BitPermArgs &a) {
    uint64_t y = 0;
    for (int b = 0; b < a.n; ++b)
        if ((x >> b) & 1) y |= 1ull << a.gperm[b];
    return y;
}

template <typename C>
__global__ void __launch_bounds__(BP_THREADS) k_bitperm(C *__restrict__ psi, BitPermArgs a) {
    __shared__ C buf[2][1 << (BP_MAX_L - (sizeof(C) == 16 ? 1 : 0))];
    // scatter tables: local index l = (hi << 6) | lo -> global offset, and the
    // local permutation, split in 6-bit halves
    __shared__ uint64_t sc_lo[64], sc_hi[64];
    __shared__ uint32_t lm_lo[64], lm_hi[64];
    const uint64_t c = blockIdx.x;
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
    if (c >= a.nchunks) return;
    // chunk base from the chunk index, then its partner under sigma
    uint64_t base = c;
    for (int b = 0; b < L; ++b) {
        const uint64_t lo = base & a.lowmask[b];
        base = lo | ((base ^ lo) << 1);
    }
    const uint64_t pbase = bp_permute_global(base, a);   // non-local bits only (local set is closed)
    // partner chunk index: squeeze out the local bits of pbase
    uint64_t pc = 0;
    {
        int k = 0, li = 0;
        for (int b = 0; b < a.n; ++b) {
            if (li < L && a.lpos[li] == b) {
                ++li;
                continue;
            }
            if ((pbase >> b) & 1) pc |= 1ull << k;
            ++k;
        }
    }
    if (pc < c) return;   // the partner's workgroup moves this pair
    const bool pair = pc != c;
    // fixed trip count (the largest chunk) so that all loads are issued
    // before the first LDS store
    constexpr int IT = (1 << (BP_MAX_L - (sizeof(C) == 16 ? 1 : 0))) / BP_THREADS;
    C r0[IT], r1[IT];
#pragma unroll
    for (int i = 0; i < IT; ++i) {
        const uint32_t l = threadIdx.x + i * BP_THREADS;
        if (l < csize) {
            const uint64_t off = sc_lo[l & 63] | sc_hi[l >> 6];
            r0[i] = psi[base | off];
            if (pair) r1[i] = psi[pbase | off];
        }
    }
#pragma unroll
    for (int i = 0; i < IT; ++i) {
        const uint32_t l = threadIdx.x + i * BP_THREADS;
        if (l < csize) {
            buf[0][bp_swz(l)] = r0[i];
            if (pair) buf[1][bp_swz(l)] = r1[i];
        }
    }
    __syncthreads();
    // element l of chunk c lands at local position lmap(l) of chunk sigma(c):
    // write every output position in order, reading its source (sigma is an
    // involution, so the source of lo is lmap(lo))
#pragma unroll
    for (int i = 0; i < IT; ++i) {
        const uint32_t lo = threadIdx.x + i * BP_THREADS;
        if (lo < csize) {
            const uint64_t off = sc_lo[lo & 63] | sc_hi[lo >> 6];
            const uint32_t li = lm_lo[lo & 63] | lm_hi[lo >> 6];
            psi[pbase | off] = buf[0][bp_swz(li)];
            if (pair) psi[base | off] = buf[1][bp_swz(li)];
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
            a.lowmask[L] = (1ull << b) - 1ull;
            ++L;
        }
    a.L = L;
    for (int b = 0; b < n; ++b) a.gperm[b] = sigma[b];
    for (int i = 0; i < L; ++i) {
        const int dst = sigma[a.lpos[i]];
        for (int k = 0; k < L; ++k)
            if (a.lpos[k] == dst) a.lperm[i] = k;
    }
    a.nchunks = 1ull << (n - L);
    const unsigned grid = (unsigned)a.nchunks;
    if (dtype == QSV_C64)
        hipLaunchKernelGGL(k_bitperm<float2>, dim3(grid), dim3(BP_THREADS), 0, s, (float2 *)state, a);
    else
        hipLaunchKernelGGL(k_bitperm<double2>, dim3(grid), dim3(BP_THREADS), 0, s, (double2 *)state, a);
    QSV_HIP_CHECK(hipGetLastError());
    return QSV_OK;
}

}  // namespace qsv
