// Fused dense k-qubit block (k = 4..6) on FP32 matrix cores, complex64 state.
//
// Gate fusion (Sec. 3.2 of the paper) turns runs of gates into one 2^k x 2^k
// matrix G; applying it is the complex product Y = G X with X the state
// viewed as D = 2^k rows (values tau of the target bits, targets[0] = MSB) by
// 2^(n-k) columns (the other bits).  Two real forms run on
// v_mfma_f32_32x32x2_f32 with FP32 accumulation:
//   k = 4     [Yr; Yi] = [[Gr, -Gi], [Gi, Gr]] [Xr; Xi]   (one 32-row tile)
//   k = 5, 6  T1 = Gr Xr, T2 = Gi Xi, T3 = (Gr + Gi)(Xr + Xi),
//             Yr = T1 - T2, Yi = T3 - T1 - T2
// The second (Gauss's three-product form of a complex product) does three
// quarters of the matrix-core work of the first; at k >= 5 the matrix-core
// time per column is comparable to its HBM time, so the saving is speed.
//
// One wave owns a tile of 32 columns.  Lane l loads X[2s + l/32][col l%32] as
// a float2 for s < D/2 (two 256-byte rows per instruction when the lowest
// target is above bit 4); those registers are the B fragments of the K loop
// (real parts, imaginary parts, or their sums).  The A fragments sit in LDS,
// four fragments interleaved per lane so that one 16-byte LDS read fetches
// four.  Outputs Yr and Yi of one (tau, column) land in the same lane and are
// stored as a float2.  Row offsets split into a per-lane part (the row bit
// that the lane half selects) and a wave-uniform part kept in scalar
// registers; the LDS lane offset is re-derived in every tile so that the
// compiler cannot hoist the fragment reads out of the tile loop (keeping all
// of them live would cost 64-256 VGPRs and most of the occupancy).
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

// Fragments per block size: 4 * D (k = 4: 16 K-steps of the 32-row tile) or
// 3 * (D / 32) * (D / 2) (k = 5, 6: three products, D/32 row tiles each).
template <int K> struct MfmaShape {
    static constexpr int D = 1 << K;
    static constexpr int NS = D / 2;                          // float2 registers per lane
    static constexpr int RM = K == 4 ? 1 : D / 32;            // row tiles per product
    static constexpr int F = K == 4 ? D : NS * 3 * RM;        // A fragments
};

template <int K>
__global__ void __launch_bounds__(MB_THREADS) k_block_mfma(float2 *__restrict__ psi, const float *__restrict__ gfrag,
                                                           BlockArgs a) {
    typedef MfmaShape<K> S;
    constexpr int NS = S::NS, RM = S::RM, F = S::F;
    __shared__ float4 G4[F * 16];
    {
        const float4 *src = (const float4 *)gfrag;
        for (int i = threadIdx.x; i < F * 16; i += MB_THREADS) G4[i] = src[i];
    }
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int col = lane & 31, half = lane >> 5;
    // row 2s + half = offs[2s] + offs[half]; row tau of the outputs below has
    // bit 2 equal to half: offs[tau] = offs[tau & ~4] + half * offs[4]
    const uint64_t ld_half = half ? a.offs[1] : 0ull, st_half = half ? a.offs[4] : 0ull;
    const uint64_t ntiles = a.ncols >> 5;
    const uint64_t wstride = (uint64_t)gridDim.x * (MB_THREADS / 64);
    for (uint64_t tile = (uint64_t)blockIdx.x * (MB_THREADS / 64) + wave; tile < ntiles; tile += wstride) {
        uint64_t base = (tile << 5) + col;
#pragma unroll
        for (int b = 0; b < K; ++b) {
            const uint64_t lo = base & a.lowmask[b];
            base = lo | ((base ^ lo) << 1);
        }
        int gl = lane;
        asm volatile("" : "+v"(gl));
        const float2 *src = psi + (base + ld_half);
        float2 x[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) x[s] = src[a.offs[2 * s]];
        float2 *dst = psi + (base + st_half);
        if constexpr (K == 4) {
            // fragment f = K-step kk: A[r][c] = Greal[r][2 kk + c]
            v16f acc;
#pragma unroll
            for (int j = 0; j < 16; ++j) acc[j] = 0.0f;
#pragma unroll
            for (int f4 = 0; f4 < F / 4; ++f4) {
                const float4 g = G4[f4 * 64 + gl];
                const float ge[4] = {g.x, g.y, g.z, g.w};
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int kk = 4 * f4 + e;
                    const float bf = (kk < NS) ? x[kk].x : x[kk - NS].y;
                    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(ge[e], bf, acc, 0, 0, 0);
                }
            }
            // accumulator j holds real row 8 (j / 4) + 4 half + j % 4: rows
            // 0..15 are Yr, 16..31 Yi of the same tau
#pragma unroll
            for (int j = 0; j < 8; ++j) dst[a.offs[8 * (j / 4) + (j % 4)]] = make_float2(acc[j], acc[j + 8]);
        } else {
            // fragment f = (kk * 3 + p) * RM + rt: A[r][c] = P_p[32 rt + r][2 kk + c]
            v16f acc[3][RM];
#pragma unroll
            for (int p = 0; p < 3; ++p)
#pragma unroll
                for (int rt = 0; rt < RM; ++rt)
#pragma unroll
                    for (int j = 0; j < 16; ++j) acc[p][rt][j] = 0.0f;
#pragma unroll
            for (int f4 = 0; f4 < F / 4; ++f4) {
                const float4 g = G4[f4 * 64 + gl];
                const float ge[4] = {g.x, g.y, g.z, g.w};
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int f = 4 * f4 + e, rt = f % RM, p = (f / RM) % 3, kk = f / (3 * RM);
                    const float bf = p == 0 ? x[kk].x : p == 1 ? x[kk].y : x[kk].x + x[kk].y;
                    acc[p][rt] = __builtin_amdgcn_mfma_f32_32x32x2f32(ge[e], bf, acc[p][rt], 0, 0, 0);
                }
            }
#pragma unroll
            for (int rt = 0; rt < RM; ++rt)
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    const float t1 = acc[0][rt][j], t2 = acc[1][rt][j], t3 = acc[2][rt][j];
                    dst[a.offs[32 * rt + 8 * (j / 4) + (j % 4)]] = make_float2(t1 - t2, t3 - t1 - t2);
                }
        }
    }
}

// G: complex128 row-major D x D.  Writes the A fragments of the kernel's
// form for this k: fragment f, lane l at frag[(f / 4) * 256 + 4 l + f % 4],
// holding A_f[l % 32][l / 32].
static void make_fragments(const double *G, int k, float *frag) {
    const int D = 1 << k;
    auto re = [&](int r, int c) { return G[2 * (r * D + c)]; };
    auto im = [&](int r, int c) { return G[2 * (r * D + c) + 1]; };
    auto put = [&](int f, int l, double v) { frag[(f / 4) * 256 + 4 * l + f % 4] = (float)v; };
    if (k == 4) {
        // the real 2D x 2D matrix [[Gr, -Gi], [Gi, Gr]]
        auto greal = [&](int r, int c) -> double {
            const int rr = r % D, cc = c % D;
            const bool top = r < D, left = c < D;
            if (top == left) return re(rr, cc);
            return top ? -im(rr, cc) : im(rr, cc);
        };
        for (int kk = 0; kk < D; ++kk)
            for (int l = 0; l < 64; ++l) put(kk, l, greal(l % 32, 2 * kk + l / 32));
        return;
    }
    const int RM = D / 32;
    for (int kk = 0; kk < D / 2; ++kk)
        for (int p = 0; p < 3; ++p)
            for (int rt = 0; rt < RM; ++rt)
                for (int l = 0; l < 64; ++l) {
                    const int r = 32 * rt + l % 32, c = 2 * kk + l / 32;
                    const double v = p == 0 ? re(r, c) : p == 1 ? im(r, c) : re(r, c) + im(r, c);
                    put((kk * 3 + p) * RM + rt, l, v);
                }
}

template <int K> static unsigned block_grid(uint64_t ntiles) {
    // as many workgroups as can be resident, each walking tiles with a stride
    static int resident[64] = {0};
    int dev = 0;
    (void)hipGetDevice(&dev);
    if (dev < 0 || dev >= 64) dev = 0;
    if (resident[dev] == 0) {
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_block_mfma<K>, MB_THREADS, 0) != hipSuccess ||
            per_cu < 1)
            per_cu = 1;
        resident[dev] = per_cu;
    }
    const uint64_t blocks = (ntiles + 3) / 4, cap = (uint64_t)resident[dev] * device_sm_count();
    return (unsigned)std::min(blocks, cap);
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
    const int F = k == 4 ? D : 3 * (D / 32) * (D / 2);   // MfmaShape<k>::F
    const size_t bytes = sizeof(float) * 64 * F;
    StagingSlot slot;
    int st = staging_acquire(bytes, &slot);
    if (st) return st;
    make_fragments(G, k, (float *)slot.host);
    if ((st = staging_upload(slot, bytes, s))) return st;
    const uint64_t tiles = a.ncols >> 5;
    const float *g = (const float *)slot.dev;
    switch (k) {
    case 4: hipLaunchKernelGGL(k_block_mfma<4>, dim3(block_grid<4>(tiles)), dim3(MB_THREADS), 0, s, (float2 *)state, g, a); break;
    case 5: hipLaunchKernelGGL(k_block_mfma<5>, dim3(block_grid<5>(tiles)), dim3(MB_THREADS), 0, s, (float2 *)state, g, a); break;
    default: hipLaunchKernelGGL(k_block_mfma<6>, dim3(block_grid<6>(tiles)), dim3(MB_THREADS), 0, s, (float2 *)state, g, a); break;
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
