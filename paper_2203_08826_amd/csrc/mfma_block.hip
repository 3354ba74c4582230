// Fused dense k-qubit block (k = 4..6) on FP32 matrix cores, complex64 state.
//
// Gate fusion (Sec. 3.2 of the paper) turns runs of gates into one 2^k x 2^k
// matrix G; applying it is the complex product Y = G X with X the state
// viewed as 2^k rows (values tau of the target bits, targets[0] = MSB) by
// 2^(n-k) columns (the other bits).  As a real product,
//     [Yr; Yi] = [[Gr, -Gi], [Gi, Gr]] [Xr; Xi]        (2D x 2D, D = 2^k)
// which runs on v_mfma_f32_32x32x2_f32 with FP32 accumulation.
//
// One wave owns a tile of 32 columns.  Lane l loads X[2s + l/32][col l%32] as
// a float2 for s < D/2 (two contiguous 256-byte rows per instruction); those
// registers are exactly the B fragments of the K loop: step kk < D/2 takes
// the real parts of register kk, step kk >= D/2 the imaginary parts of
// register kk - D/2.  The real 2D x 2D matrix sits in LDS in fragment order,
// so each A fragment is one contiguous 256-byte LDS read.  Outputs Yr and Yi
// of the same (tau, column) land in the same lane and are stored as float2.
#include "qsv_internal.h"

namespace qsv {

typedef float v16f __attribute__((ext_vector_type(16)));

constexpr int MB_THREADS = 256;

struct BlockArgs {
    uint64_t lowmask[QSV_MAX_TARGETS];   // sorted target bits, for the column base
    uint64_t offs[64];                   // offset of row tau
    uint64_t ncols;                      // 2^(n-k)
    int k;
};

template <int K>
__global__ void __launch_bounds__(MB_THREADS) k_block_mfma(float2 *__restrict__ psi, const float *__restrict__ gfrag,
                                                           BlockArgs a) {
    constexpr int D = 1 << K;
    constexpr int RT = (2 * D) / 32;   // row tiles of the real product
    constexpr int NS = D / 2;          // float2 registers per lane
    __shared__ float G[2 * D * 2 * D];
    for (int i = threadIdx.x; i < 4 * D * D; i += MB_THREADS) G[i] = gfrag[i];
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int col = lane & 31, half = lane >> 5;
    const uint64_t ntiles = a.ncols >> 5;
    const uint64_t wstride = (uint64_t)gridDim.x * (MB_THREADS / 64);
    for (uint64_t tile = (uint64_t)blockIdx.x * (MB_THREADS / 64) + wave; tile < ntiles; tile += wstride) {
        uint64_t base = (tile << 5) + col;
#pragma unroll
        for (int b = 0; b < K; ++b) {
            const uint64_t lo = base & a.lowmask[b];
            base = lo | ((base ^ lo) << 1);
        }
        float2 x[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) x[s] = psi[base + a.offs[2 * s + half]];
        v16f acc[RT];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int j = 0; j < 16; ++j) acc[rt][j] = 0.0f;
#pragma unroll
        for (int kk = 0; kk < D; ++kk) {
            const float bf = (kk < NS) ? x[kk].x : x[kk - NS].y;
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) {
                const float af = G[(kk * RT + rt) * 64 + lane];
                acc[rt] = __builtin_amdgcn_mfma_f32_32x32x2f32(af, bf, acc[rt], 0, 0, 0);
            }
        }
        // row r of tile rt for accumulator j: 32 rt + 8 (j / 4) + 4 half + j % 4
        if constexpr (K == 4) {
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int tau = 8 * (j / 4) + 4 * half + (j % 4);
                psi[base + a.offs[tau]] = make_float2(acc[0][j], acc[0][j + 8]);
            }
        } else {
#pragma unroll
            for (int rt = 0; rt < RT / 2; ++rt)
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    const int tau = 32 * rt + 8 * (j / 4) + 4 * half + (j % 4);
                    psi[base + a.offs[tau]] = make_float2(acc[rt][j], acc[rt + RT / 2][j]);
                }
        }
    }
}

// G: complex128 row-major D x D.  Writes the real 2D x 2D matrix in MFMA
// A-fragment order: frag[(kk * RT + rt) * 64 + l] = Greal[32 rt + l % 32][2 kk + l / 32].
static void make_fragments(const double *G, int k, float *frag) {
    const int D = 1 << k, RT = (2 * D) / 32;
    auto greal = [&](int r, int c) -> double {
        const int rr = r % D, cc = c % D;
        const double re = G[2 * (rr * D + cc)], im = G[2 * (rr * D + cc) + 1];
        const bool top = r < D, left = c < D;
        if (top && left) return re;
        if (top && !left) return -im;
        if (!top && left) return im;
        return re;
    };
    for (int kk = 0; kk < D; ++kk)
        for (int rt = 0; rt < RT; ++rt)
            for (int l = 0; l < 64; ++l) frag[(kk * RT + rt) * 64 + l] = (float)greal(32 * rt + l % 32, 2 * kk + l / 32);
}

int launch_block_mfma(void *state, int n, const double *G, const int *targets, int k, hipStream_t s) {
    if (k < 4 || k > 6) return fail(QSV_ERR_UNSUPPORTED, "MFMA blocks take 4..6 targets");
    if (n < k + 5) return fail(QSV_ERR_UNSUPPORTED, "MFMA blocks need at least k + 5 qubits");
    BlockArgs a;
    std::memset(&a, 0, sizeof(a));
    a.k = k;
    std::vector<int> sorted(targets, targets + k);
    std::sort(sorted.begin(), sorted.end());
    for (int i = 0; i < k; ++i) a.lowmask[i] = (1ull << sorted[i]) - 1ull;
    const int D = 1 << k;
    for (int t = 0; t < D; ++t) {
        uint64_t o = 0;
        for (int j = 0; j < k; ++j)
            if ((t >> (k - 1 - j)) & 1) o |= 1ull << targets[j];
        a.offs[t] = o;
    }
    a.ncols = 1ull << (n - k);
    const size_t bytes = sizeof(float) * 4 * D * D;
    StagingSlot slot;
    int st = staging_acquire(bytes, &slot);
    if (st) return st;
    make_fragments(G, k, (float *)slot.host);
    if ((st = staging_upload(slot, bytes, s))) return st;
    const uint64_t tiles = a.ncols >> 5;
    uint64_t blocks = (tiles + 3) / 4;
    const uint64_t cap = (uint64_t)device_sm_count() * 8;
    if (blocks > cap) blocks = cap;
    const float *g = (const float *)slot.dev;
    switch (k) {
    case 4: hipLaunchKernelGGL(k_block_mfma<4>, dim3((unsigned)blocks), dim3(MB_THREADS), 0, s, (float2 *)state, g, a); break;
    case 5: hipLaunchKernelGGL(k_block_mfma<5>, dim3((unsigned)blocks), dim3(MB_THREADS), 0, s, (float2 *)state, g, a); break;
    default: hipLaunchKernelGGL(k_block_mfma<6>, dim3((unsigned)blocks), dim3(MB_THREADS), 0, s, (float2 *)state, g, a); break;
    }
    hipError_t e = hipGetLastError();
    staging_release(slot, s);
    if (e != hipSuccess) return hip_fail(e, "MFMA block launch");
    return QSV_OK;
}

}  // namespace qsv

using namespace qsv;

extern "C" int qsv_apply_block(void *state, int n, int dtype, const void *gate, const int *targets, int k,
                               void *stream) {
    int st = validate_common(n, dtype, targets, k, nullptr, 0);
    if (st) return st;
    if (dtype != QSV_C64) return fail(QSV_ERR_UNSUPPORTED, "MFMA blocks are complex64 only");
    if (k < 4 || k > 6) return fail(QSV_ERR_ARITY, "MFMA blocks take 4..6 targets");
    if (n < k + 5) return fail(QSV_ERR_ARITY, "MFMA blocks need n >= k + 5");
    if (!state || !gate) return fail(QSV_ERR_NULL, "NULL argument");
    if (((uintptr_t)state & 15) != 0) return fail(QSV_ERR_ALIGN, "state must be 16-byte aligned");
    const int D = 1 << k;
    std::vector<double> G(2 * D * D);
    const float *f = (const float *)gate;
    for (int i = 0; i < 2 * D * D; ++i) G[i] = f[i];
    return launch_block_mfma(state, n, G.data(), targets, k, (hipStream_t)stream);
}
