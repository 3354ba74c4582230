// Per-gate kernels: Eq. 1 of the paper's introduction applied in place, one
// launch per gate.
//
// Every kernel walks groups: a group is the set of amplitudes that differ
// only in the gate's target bits, with every control bit set.  Group g is
// turned into its smallest member by inserting a 0 at each sorted
// target/control bit (the on-the-fly index generation of the methodology
// section: i1 = ((g >> t) << (t + 1)) + (g & (2^t - 1)), generalised to
// several bits), then OR-ing the control mask.  Only the members the gate
// changes are read and written:
//   k_dense : M members, M x M complex submatrix (general gates, fSim's
//             3-member block, controlled gates);
//   k_diag  : M members each multiplied by a factor (Z, U1/CU1, CZ, RZ,
//             diagonal gates);
//   k_perm  : M members each replaced by a (phase times) another member
//             (X/CNOT, Y, SWAP): pure moves are bit-exact;
//   k_low1  : one-target dense complex64 gates on a low qubit; each lane
//             streams a contiguous 16-byte vector and partners inside the
//             wave are exchanged with cross-lane shuffles, so every access
//             stays a full contiguous vector.
#include "qsv_internal.h"

namespace qsv {

#define QSV_MAX_BITS (QSV_MAX_TARGETS + QSV_MAX_CONTROLS)

struct GroupArgs {
    uint64_t lowmask[QSV_MAX_BITS];
    uint64_t cmask;
    uint64_t ngroups;
    int m;
};

template <typename C, int M> struct DenseArgs {
    uint64_t offs[M];
    C mat[M <= 8 ? M * M : 1];   // inline for M <= 8
    const C *dmat;               // device copy for M > 8
};

template <typename C, int M> struct DiagArgs {
    uint64_t offs[M];
    C fac[M];
};

template <typename C, int M> struct PermArgs {
    uint64_t offs[M];
    uint64_t src[M];
    C fac[M];
    uint64_t one;   // bit j set: member j is a pure move
};

__device__ inline uint64_t group_base(uint64_t g, const GroupArgs &ga) {
    uint64_t i = g;
#pragma unroll 1
    for (int b = 0; b < ga.m; ++b) {
        const uint64_t lo = i & ga.lowmask[b];
        i = lo | ((i ^ lo) << 1);
    }
    return i | ga.cmask;
}

// Work per thread: U units of VG consecutive groups.  Several independent
// units keep enough loads in flight to cover HBM latency when a group is
// small; when bit 0 is not a gate bit, VG = 2 consecutive complex64 groups
// are adjacent in memory and each member access is a 16-byte vector.  A workgroup covers U * 256 consecutive units (unit u of a thread
// is 256 units after unit u - 1) and the grid covers the state once, so the
// workgroups resident at any time stream through one contiguous window of
// memory: on MI355X this sustains ~5.9 TB/s for in-place updates, against
// ~5.1 TB/s for grid-stride loops whose threads jump a whole grid ahead.
// Measured on MI355X at 30-33 qubits: four units per thread only pay for
// complex64 groups of up to two members; everything else streams best with
// one unit per thread.
template <typename C, int M> struct Unroll { static constexpr int U = (sizeof(C) == 8 && M <= 2) ? 4 : 1; };
// Diagonal gates on 16-byte complex64 members stream best with one unit per
// thread (30 qubits: Z 5.5 -> 6.0 TB/s, controlled phase 5.6 -> 5.9), with
// ordinary accesses: they touch runs of a line (Z on qubit 5: 256 bytes of
// every 512), where nontemporal ones ran slower (Z 6.06 -> 5.59 TB/s).
template <typename C, int M, int VG> struct DiagUnroll {
    static constexpr int U = (VG == 2 && sizeof(C) == 8) ? 1 : Unroll<C, M>::U;
};

// The VG consecutive amplitudes of one member of a unit as one access: a
// 16-byte vector for VG = 2 complex64 groups (the element index is even,
// see above).  Written out because the compiler leaves the predicated loads
// of several units as 8-byte accesses.  These complex64 accesses are
// nontemporal: every amplitude is touched once per gate, and streaming past
// the caches lifts an in-place 16-byte stream from 5.9 to 6.6 TB/s on
// MI355X (complex128 accesses gain nothing and stay ordinary).
typedef float f4v __attribute__((ext_vector_type(4)));
__device__ __forceinline__ f4v ld_nt(const void *p) { return __builtin_nontemporal_load((const f4v *)p); }
__device__ __forceinline__ void st_nt(void *p, f4v v) { __builtin_nontemporal_store(v, (f4v *)p); }
template <typename C, int VG, bool NT = true> __device__ __forceinline__ void ld_vg(const C *p, C (&out)[VG]) {
    if constexpr (VG == 2 && sizeof(C) == 8) {
        const f4v q = NT ? ld_nt(p) : *reinterpret_cast<const f4v *>(p);
        out[0].x = q.x;
        out[0].y = q.y;
        out[1].x = q.z;
        out[1].y = q.w;
    } else {
#pragma unroll
        for (int r = 0; r < VG; ++r) out[r] = p[r];
    }
}
template <typename C, int VG, bool NT = true> __device__ __forceinline__ void st_vg(C *p, const C (&in)[VG]) {
    if constexpr (VG == 2 && sizeof(C) == 8) {
        f4v q;
        q.x = in[0].x;
        q.y = in[0].y;
        q.z = in[1].x;
        q.w = in[1].y;
        if constexpr (NT) st_nt(p, q);
        else *reinterpret_cast<f4v *>(p) = q;
    } else {
#pragma unroll
        for (int r = 0; r < VG; ++r) p[r] = in[r];
    }
}

template <int U, int VG>
__device__ __forceinline__ void unit_bases(uint64_t w0, uint64_t wstride, uint64_t nunits, const GroupArgs &ga,
                                           uint64_t *base, bool *live) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const uint64_t w = w0 + u * wstride;
        live[u] = w < nunits;
        base[u] = live[u] ? group_base(w * VG, ga) : 0;   // + r for the r-th group of the unit
    }
}

template <typename C, int M, int VG, int U>
__global__ void __launch_bounds__(256) k_dense(C *__restrict__ psi, GroupArgs ga, DenseArgs<C, M> da) {
    const uint64_t nunits = ga.ngroups / VG;
    const uint64_t span = (uint64_t)U * blockDim.x;
    for (uint64_t w0 = (uint64_t)blockIdx.x * span + threadIdx.x; w0 < nunits; w0 += (uint64_t)gridDim.x * span) {
        uint64_t base[U];
        bool live[U];
        C v[U][M][VG];
        unit_bases<U, VG>(w0, blockDim.x, nunits, ga, base, live);
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int j = 0; j < M; ++j)
                if (live[u]) ld_vg<C, VG>(psi + base[u] + da.offs[j], v[u][j]);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (!live[u]) continue;
#pragma unroll
            for (int q = 0; q < M; ++q) {
                C o[VG];
#pragma unroll
                for (int r = 0; r < VG; ++r) {
                    C acc;
                    acc.x = 0;
                    acc.y = 0;
#pragma unroll
                    for (int j = 0; j < M; ++j) {
                        const C gm = (M <= 8) ? da.mat[q * M + j] : da.dmat[q * M + j];
                        acc = cfma(gm, v[u][j][r], acc);
                    }
                    if constexpr (VG == 2 && sizeof(C) == 8) o[r] = acc;
                    else psi[base[u] + da.offs[q] + r] = acc;   // stored at once: wide groups keep fewer live values
                }
                if constexpr (VG == 2 && sizeof(C) == 8) st_vg<C, VG>(psi + base[u] + da.offs[q], o);
            }
        }
    }
}

template <typename C, int M, int VG>
__global__ void __launch_bounds__(256) k_diag(C *__restrict__ psi, GroupArgs ga, DiagArgs<C, M> da) {
    constexpr int U = DiagUnroll<C, M, VG>::U;
    const uint64_t nunits = ga.ngroups / VG;
    const uint64_t span = (uint64_t)U * blockDim.x;
    for (uint64_t w0 = (uint64_t)blockIdx.x * span + threadIdx.x; w0 < nunits; w0 += (uint64_t)gridDim.x * span) {
        uint64_t base[U];
        bool live[U];
        C v[U][M][VG];
        unit_bases<U, VG>(w0, blockDim.x, nunits, ga, base, live);
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int j = 0; j < M; ++j)
                if (live[u]) ld_vg<C, VG, false>(psi + base[u] + da.offs[j], v[u][j]);
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int j = 0; j < M; ++j) {
                if (!live[u]) continue;
                C o[VG];
#pragma unroll
                for (int r = 0; r < VG; ++r) o[r] = cmul(da.fac[j], v[u][j][r]);
                st_vg<C, VG, false>(psi + base[u] + da.offs[j], o);
            }
    }
}

template <typename C, int M, int VG, int U>
__global__ void __launch_bounds__(256) k_perm(C *__restrict__ psi, GroupArgs ga, PermArgs<C, M> pa) {
    const uint64_t nunits = ga.ngroups / VG;
    const uint64_t span = (uint64_t)U * blockDim.x;
    for (uint64_t w0 = (uint64_t)blockIdx.x * span + threadIdx.x; w0 < nunits; w0 += (uint64_t)gridDim.x * span) {
        uint64_t base[U];
        bool live[U];
        C v[U][M][VG];
        unit_bases<U, VG>(w0, blockDim.x, nunits, ga, base, live);
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int j = 0; j < M; ++j)
                if (live[u]) ld_vg<C, VG>(psi + base[u] + pa.src[j], v[u][j]);
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int j = 0; j < M; ++j) {
                if (!live[u]) continue;
                C o[VG];
#pragma unroll
                for (int r = 0; r < VG; ++r) o[r] = ((pa.one >> j) & 1) ? v[u][j][r] : cmul(pa.fac[j], v[u][j][r]);
                st_vg<C, VG>(psi + base[u] + pa.offs[j], o);
            }
    }
}

// ------------------------------------------------------------------ low-qubit path
//
// Lane L of a wave holds the VEC consecutive amplitudes starting at
// index = (wave_base + L) * VEC.  Target bit t < log2(VEC) pairs inside the
// lane's vector; log2(VEC) <= t < log2(VEC) + 6 pairs with lane L ^ (1 << (t -
// log2 VEC)), reached with a cross-lane shuffle.  Each lane computes only its
// own outputs: out(b) = G[b][0] * a0 + G[b][1] * a1 with (a0, a1) the pair.
template <typename C> struct Low1Args {
    C g00, g01, g10, g11;
    uint64_t cmask;
    uint64_t nvec;      // number of VEC-vectors in the state
    int t;              // target bit
};

template <typename C> __device__ inline C shfl_xor_c(C v, int lanemask) {
    C r;
    r.x = __shfl_xor(v.x, lanemask, 64);
    r.y = __shfl_xor(v.y, lanemask, 64);
    return r;
}

template <typename C, int VEC, int U>
__global__ void __launch_bounds__(256) k_low1(C *__restrict__ psi, Low1Args<C> a) {
    constexpr int LV = (VEC == 1) ? 0 : (VEC == 2) ? 1 : 2;
    // U vectors per lane per iteration, all loaded before use
    const uint64_t span = (uint64_t)U * blockDim.x;
    // nvec is a multiple of 64 and a wave's 64 lanes hold 64 consecutive
    // aligned vectors, so they are all live or all idle for every u: the
    // shuffles below see a full wave
    for (uint64_t w0 = (uint64_t)blockIdx.x * span + threadIdx.x; w0 < a.nvec; w0 += (uint64_t)gridDim.x * span) {
        C v[U][VEC];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t w = w0 + (uint64_t)u * blockDim.x;
            if (w < a.nvec) {
                if constexpr (VEC == 2 && sizeof(C) == 8) {
                    const f4v q = ld_nt(psi + w * VEC);
                    v[u][0].x = q.x;
                    v[u][0].y = q.y;
                    v[u][1].x = q.z;
                    v[u][1].y = q.w;
                } else {
#pragma unroll
                    for (int j = 0; j < VEC; ++j) v[u][j] = psi[w * VEC + j];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t w = w0 + (uint64_t)u * blockDim.x;
            if (w >= a.nvec) continue;
            const uint64_t i0 = w * VEC;
            C o[VEC];
            // partners inside a lane's vector (only when it holds several
            // amplitudes: with one, this branch would index the tile at run
            // time and put it in scratch memory)
            if (VEC > 1 && a.t < LV) {
                const int tb = 1 << a.t;
#pragma unroll
                for (int j = 0; j < VEC; ++j) {
                    const int b = (j & tb) ? 1 : 0;
                    const C p0 = b ? v[u][j ^ tb] : v[u][j];
                    const C p1 = b ? v[u][j] : v[u][j ^ tb];
                    C acc = cmul(b ? a.g10 : a.g00, p0);
                    acc = cfma(b ? a.g11 : a.g01, p1, acc);
                    o[j] = acc;
                }
            } else {
                const int lm = 1 << (a.t - LV);
                const int b = (threadIdx.x & lm) ? 1 : 0;
#pragma unroll
                for (int j = 0; j < VEC; ++j) {
                    const C q = shfl_xor_c(v[u][j], lm);
                    const C p0 = b ? q : v[u][j];
                    const C p1 = b ? v[u][j] : q;
                    C acc = cmul(b ? a.g10 : a.g00, p0);
                    acc = cfma(b ? a.g11 : a.g01, p1, acc);
                    o[j] = acc;
                }
            }
#pragma unroll
            for (int j = 0; j < VEC; ++j) {
                // per component: a select of whole complex structs is lowered
                // through scratch memory for complex128
                const bool on = ((i0 + j) & a.cmask) == a.cmask;
                o[j].x = on ? o[j].x : v[u][j].x;
                o[j].y = on ? o[j].y : v[u][j].y;
            }
            if constexpr (VEC == 2 && sizeof(C) == 8) {
                f4v q;
                q.x = o[0].x;
                q.y = o[0].y;
                q.z = o[1].x;
                q.w = o[1].y;
                st_nt(psi + i0, q);
            } else {
#pragma unroll
                for (int j = 0; j < VEC; ++j) psi[i0 + j] = o[j];
            }
        }
    }
}

// ------------------------------------------------------------------ scale
//
// psi <- s psi for a complex constant s: one 16-byte vector per thread in a
// one-shot grid (two per thread beyond 2^32 threads), nontemporal for
// complex64.  Besides normalisation and global phases, this is the plain
// in-place stream every gate kernel is measured against.
template <typename C, int U>
__global__ void __launch_bounds__(256) k_scale(C *__restrict__ psi, uint64_t nvec, double sr, double si) {
    const uint64_t span = (uint64_t)U * blockDim.x;
    for (uint64_t w0 = (uint64_t)blockIdx.x * span + threadIdx.x; w0 < nvec; w0 += (uint64_t)gridDim.x * span) {
        if constexpr (sizeof(C) == 8) {
            f4v v[U];
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (w0 + u * blockDim.x < nvec) v[u] = ld_nt(psi + 2 * (w0 + u * blockDim.x));
            const float r = (float)sr, i = (float)si;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (w0 + u * blockDim.x >= nvec) continue;
                f4v o;
                o.x = v[u].x * r - v[u].y * i;
                o.y = v[u].x * i + v[u].y * r;
                o.z = v[u].z * r - v[u].w * i;
                o.w = v[u].z * i + v[u].w * r;
                st_nt(psi + 2 * (w0 + u * blockDim.x), o);
            }
        } else {
            C v[U];
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (w0 + u * blockDim.x < nvec) v[u] = psi[w0 + u * blockDim.x];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (w0 + u * blockDim.x >= nvec) continue;
                C o;
                o.x = v[u].x * sr - v[u].y * si;
                o.y = v[u].x * si + v[u].y * sr;
                psi[w0 + u * blockDim.x] = o;
            }
        }
    }
}

// ------------------------------------------------------------------ launch

// Workgroups for `items` units at `per_block` units each: one pass over the
// state (the loops in the kernels only run again beyond the grid limit).  A
// launch holds fewer than 2^32 threads in all (HIP's limit on the total work
// size), so 256-thread workgroups number at most 2^24 - 1: a 33-qubit
// complex128 gate with 2^32 groups takes two rounds of its loop.
static int grid_for(uint64_t items, uint64_t per_block) {
    uint64_t blocks = (items + per_block - 1) / per_block;
    const uint64_t cap = 0xffffffffull / 256;
    if (blocks > cap) blocks = cap;
    if (blocks < 1) blocks = 1;
    return (int)blocks;
}

static GroupArgs make_group_args(const GateAnalysis &a) {
    GroupArgs ga;
    memset(&ga, 0, sizeof(ga));
    ga.m = (int)a.sorted_bits.size();
    for (int i = 0; i < ga.m; ++i) ga.lowmask[i] = (1ull << a.sorted_bits[i]) - 1ull;
    ga.cmask = a.cmask;
    ga.ngroups = 1ull << (a.n - ga.m);
    return ga;
}

// Two consecutive groups are adjacent amplitudes when bit 0 is no gate bit;
// complex64 then takes them as one 16-byte access.  Complex128 members are
// 16 bytes already, and a pair of them per thread (32-byte stride across
// lanes) streams slower than one per thread (30 qubits, one-qubit gate on
// qubit 12 / 22 / 29: 5.50 / 5.03 / 5.15 TB/s against 5.89 / 5.32 / 5.66).
template <typename C> static bool vg2(const GroupArgs &ga) {
    return sizeof(C) == 8 && ga.ngroups >= 2 && (ga.m == 0 || ga.lowmask[0] != 0);
}

template <typename C> static C to_c(const double *z) {
    C r;
    r.x = (decltype(r.x))z[0];
    r.y = (decltype(r.y))z[1];
    return r;
}

// Paired complex64 groups with 16-byte nontemporal members stream best with
// one unit per thread wherever the members lie (30 qubits, one-qubit gate:
// 6.1-6.6 TB/s for targets 12-20, 5.5 for 22-29 with one or two units; 33
// qubits, target 32: 6.2 with one unit, 5.7 with two).

template <typename C, int M>
static void launch_dense_m(C *psi, const GateAnalysis &a, const GroupArgs &ga, const C *dmat, hipStream_t s) {
    DenseArgs<C, M> da;
    memset(&da, 0, sizeof(da));
    for (int j = 0; j < M; ++j) da.offs[j] = a.offs[j];
    if (M <= 8)
        for (int j = 0; j < M * M; ++j) da.mat[j] = to_c<C>(&a.mat[2 * j]);
    da.dmat = dmat;
    constexpr int UU = Unroll<C, M>::U;
    if (!vg2<C>(ga)) hipLaunchKernelGGL((k_dense<C, M, 1, UU>), dim3(grid_for(ga.ngroups, 256 * UU)), dim3(256), 0, s, psi, ga, da);
    else if (UU > 1)
        hipLaunchKernelGGL((k_dense<C, M, 2, 1>), dim3(grid_for(ga.ngroups / 2, 256)), dim3(256), 0, s, psi, ga, da);
    else hipLaunchKernelGGL((k_dense<C, M, 2, UU>), dim3(grid_for(ga.ngroups / 2, 256 * UU)), dim3(256), 0, s, psi, ga, da);
}

template <typename C, int M>
static void launch_diag_m(C *psi, const GateAnalysis &a, const GroupArgs &ga, hipStream_t s) {
    DiagArgs<C, M> da;
    memset(&da, 0, sizeof(da));
    for (int j = 0; j < M; ++j) {
        da.offs[j] = a.offs[j];
        da.fac[j] = to_c<C>(&a.mat[2 * j]);
    }
    if (vg2<C>(ga))
        hipLaunchKernelGGL((k_diag<C, M, 2>), dim3(grid_for(ga.ngroups / 2, 256 * DiagUnroll<C, M, 2>::U)), dim3(256), 0,
                           s, psi, ga, da);
    else
        hipLaunchKernelGGL((k_diag<C, M, 1>), dim3(grid_for(ga.ngroups, 256 * DiagUnroll<C, M, 1>::U)), dim3(256), 0, s,
                           psi, ga, da);
}

template <typename C, int M>
static void launch_perm_m(C *psi, const GateAnalysis &a, const GroupArgs &ga, hipStream_t s) {
    PermArgs<C, M> pa;
    memset(&pa, 0, sizeof(pa));
    for (int j = 0; j < M; ++j) {
        pa.offs[j] = a.offs[j];
        pa.src[j] = a.offs[a.perm_src[j]];
        pa.fac[j] = to_c<C>(&a.mat[2 * j]);
        if (a.perm_one[j]) pa.one |= 1ull << j;
    }
    constexpr int UU = Unroll<C, M>::U;
    if (!vg2<C>(ga)) hipLaunchKernelGGL((k_perm<C, M, 1, UU>), dim3(grid_for(ga.ngroups, 256 * UU)), dim3(256), 0, s, psi, ga, pa);
    else if (UU > 1)
        hipLaunchKernelGGL((k_perm<C, M, 2, 1>), dim3(grid_for(ga.ngroups / 2, 256)), dim3(256), 0, s, psi, ga, pa);
    else hipLaunchKernelGGL((k_perm<C, M, 2, UU>), dim3(grid_for(ga.ngroups / 2, 256 * UU)), dim3(256), 0, s, psi, ga, pa);
}

// Low-qubit path for a one-target dense gate whose target is below the
// lane-exchange span: the lane vector is 16 bytes (2 complex64) and partners
// up to 64 vectors away are reached by shuffles.
template <typename C, int VEC>
static bool try_low1(C *psi, const GateAnalysis &a, hipStream_t s) {
    constexpr int LV = (VEC == 1) ? 0 : (VEC == 2) ? 1 : 2;
    if (a.cls != GC_DENSE || a.k != 1 || a.members.size() != 2) return false;
    const int t = __builtin_ctzll(a.offs[0] ^ a.offs[1]);
    if (t >= LV + 6) return false;
    if (a.n < LV + 6) return false;   // need whole waves of vectors
    Low1Args<C> la;
    la.g00 = to_c<C>(&a.mat[0]);
    la.g01 = to_c<C>(&a.mat[2]);
    la.g10 = to_c<C>(&a.mat[4]);
    la.g11 = to_c<C>(&a.mat[6]);
    la.cmask = a.cmask;
    la.nvec = (1ull << a.n) / VEC;
    la.t = t;
    // one vector per lane (6.6 TB/s at 30 qubits against 5.4 with four per
    // lane).  Beyond the 2^32 threads of a launch (33 qubits), complex64
    // streams best with two vectors per lane (qubit 0: 6.13 TB/s, against
    // 5.95 with a capped grid striding over the state) and complex128 with
    // the capped grid (6.06 / 6.29 in a probe, against 5.61 with two)
    if (VEC == 2 && la.nvec / 256 > 0xffffffffull / 256)
        hipLaunchKernelGGL((k_low1<C, VEC, 2>), dim3(grid_for(la.nvec, 256 * 2)), dim3(256), 0, s, psi, la);
    else
        hipLaunchKernelGGL((k_low1<C, VEC, 1>), dim3(grid_for(la.nvec, 256)), dim3(256), 0, s, psi, la);
    return true;
}

template <typename R>
static int launch_gate_t(void *state, const GateAnalysis &a, hipStream_t s) {
    typedef typename cplx_of<R>::type C;
    C *psi = (C *)state;
    const int M = (int)a.members.size();
    if (M == 0) return QSV_OK;   // identity
    const GroupArgs ga = make_group_args(a);
    // a target below the lane span: every lane loads whole 16-byte vectors
    // (two complex64 or one complex128 amplitude) and exchanges partners with
    // cross-lane shuffles, where the group kernel would give each lane both
    // members (complex128 at 33 qubits, qubits 0 and 3: 6.29 TB/s against
    // 5.48 / 5.54)
    if (a.cls == GC_DENSE && (sizeof(R) == 4 ? try_low1<C, 2>(psi, a, s) : try_low1<C, 1>(psi, a, s))) {
        QSV_HIP_CHECK(hipGetLastError());
        return QSV_OK;
    }
    StagingSlot slot;
    const C *dmat = nullptr;
    if (a.cls == GC_DENSE && M > 8) {
        const size_t bytes = (size_t)M * M * sizeof(C);
        int st = staging_acquire(bytes, &slot);
        if (st) return st;
        C *h = (C *)slot.host;
        for (int j = 0; j < M * M; ++j) h[j] = to_c<C>(&a.mat[2 * j]);
        st = staging_upload(slot, bytes, s);
        if (st) return st;
        dmat = (const C *)slot.dev;
    }
    switch (a.cls) {
    case GC_DIAG:
        switch (M) {
        case 1: launch_diag_m<C, 1>(psi, a, ga, s); break;
        case 2: launch_diag_m<C, 2>(psi, a, ga, s); break;
        case 4: launch_diag_m<C, 4>(psi, a, ga, s); break;
        case 8: launch_diag_m<C, 8>(psi, a, ga, s); break;
        case 16: launch_diag_m<C, 16>(psi, a, ga, s); break;
        case 32: launch_diag_m<C, 32>(psi, a, ga, s); break;
        case 64: launch_diag_m<C, 64>(psi, a, ga, s); break;
        default: return fail(QSV_ERR_ARG, "internal: diagonal member count not padded");
        }
        break;
    case GC_PERM:
        switch (M) {
        case 2: launch_perm_m<C, 2>(psi, a, ga, s); break;
        case 4: launch_perm_m<C, 4>(psi, a, ga, s); break;
        case 8: launch_perm_m<C, 8>(psi, a, ga, s); break;
        case 16: launch_perm_m<C, 16>(psi, a, ga, s); break;
        case 32: launch_perm_m<C, 32>(psi, a, ga, s); break;
        case 64: launch_perm_m<C, 64>(psi, a, ga, s); break;
        default: return fail(QSV_ERR_ARG, "internal: permutation member count not padded");
        }
        break;
    default:
        switch (M) {
        case 2: launch_dense_m<C, 2>(psi, a, ga, dmat, s); break;
        case 3: launch_dense_m<C, 3>(psi, a, ga, dmat, s); break;
        case 4: launch_dense_m<C, 4>(psi, a, ga, dmat, s); break;
        case 8: launch_dense_m<C, 8>(psi, a, ga, dmat, s); break;
        case 16: launch_dense_m<C, 16>(psi, a, ga, dmat, s); break;
        case 32: launch_dense_m<C, 32>(psi, a, ga, dmat, s); break;
        case 64: launch_dense_m<C, 64>(psi, a, ga, dmat, s); break;
        default: return fail(QSV_ERR_ARG, "internal: dense member count not padded");
        }
        break;
    }
    hipError_t e = hipGetLastError();
    if (dmat) staging_release(slot, s);
    if (e != hipSuccess) return hip_fail(e, "gate kernel launch");
    return QSV_OK;
}

int launch_scale(void *state, int n, int dtype, double re, double im, hipStream_t s) {
    // n >= 1: a complex64 state holds at least one 16-byte vector
    const uint64_t nvec = dtype == QSV_C64 ? (1ull << n) / 2 : (1ull << n);
    const bool one = nvec <= 0xffffffffull - 255;
    if (dtype == QSV_C64) {
        if (one) hipLaunchKernelGGL((k_scale<float2, 1>), dim3(grid_for(nvec, 256)), dim3(256), 0, s, (float2 *)state, nvec, re, im);
        else hipLaunchKernelGGL((k_scale<float2, 2>), dim3(grid_for(nvec, 512)), dim3(256), 0, s, (float2 *)state, nvec, re, im);
    } else {
        if (one) hipLaunchKernelGGL((k_scale<double2, 1>), dim3(grid_for(nvec, 256)), dim3(256), 0, s, (double2 *)state, nvec, re, im);
        else hipLaunchKernelGGL((k_scale<double2, 2>), dim3(grid_for(nvec, 512)), dim3(256), 0, s, (double2 *)state, nvec, re, im);
    }
    QSV_HIP_CHECK(hipGetLastError());
    return QSV_OK;
}

int launch_gate(void *state, int dtype, const GateAnalysis &a, hipStream_t s) {
    return dtype == QSV_C64 ? launch_gate_t<float>(state, a, s) : launch_gate_t<double>(state, a, s);
}

}  // namespace qsv
