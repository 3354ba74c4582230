// LDS-staged multi-gate pass: several gates per HBM read + write of the state.
//
// Gate fusion (Sec. 3.2 of the paper) multiplies gate matrices to cut the
// number of sweeps over the state; a pass goes further and keeps a chunk of
// 2^L amplitudes on chip while a whole run of gates is applied to it.  The
// chunk is the set of amplitudes sharing every non-local bit.  Thread t of
// the 256-thread workgroup holds 2^RB of them in registers (L = RB + 8):
//   - one- and two-qubit gates whose targets are register bits run in
//     registers (in-place Eq. 1 on pairs / quads);
//   - an EXCHANGE rewrites the chunk through LDS with another assignment of
//     local bits to register / thread bits (bank-swizzled layout);
//   - diagonal gates on any bits run as PHASE ops: every unit-modulus
//     diagonal gate is a sum of phase terms theta * prod(bits), evaluated in
//     exact fixed-point turns and split into parts that depend on the chunk,
//     the thread and the register index;
//   - controls on non-local bits are per-chunk predicates;
//   - SWAPs of two local bits are relabelings of local positions, applied by
//     the store's bit map at no cost.
// Global loads and stores keep the lowest global bits on lanes, so every
// wave instruction touches contiguous runs of at least 512 bytes.
#include "plan_internal.h"

namespace qsv {

constexpr int PT = 256;

// Workgroup barrier that orders LDS accesses only: outstanding global loads
// (the next chunk's prefetch) stay in flight across it.
// An amplitude as an operand of an empty volatile asm: the compiler waits for
// its load before this point, and the asm is not moved across a barrier.
template <typename C> __device__ __forceinline__ void hold_value(const C &v) {
    asm volatile("" ::"v"(v.x), "v"(v.y));
}

__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Sum over the 64 lanes of a wave, modulo 2^64 (fixed-point turns wrap), in
// every lane: the 32-bit halves are reduced separately (no overflow for 64
// terms) and recombined.
__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t x) {
    uint64_t lo = (uint32_t)x, hi = x >> 32;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        lo += (uint64_t)(uint32_t)__shfl_xor((int)(uint32_t)lo, off, 64) |
              ((uint64_t)(uint32_t)__shfl_xor((int)(uint32_t)(lo >> 32), off, 64) << 32);
        hi += (uint64_t)(uint32_t)__shfl_xor((int)(uint32_t)hi, off, 64) |
              ((uint64_t)(uint32_t)__shfl_xor((int)(uint32_t)(hi >> 32), off, 64) << 32);
    }
    return lo + (hi << 32);
}

__device__ __forceinline__ uint32_t lds_swizzle(uint32_t l) {
    return l ^ (((l >> 4) ^ (l >> 8) ^ (l >> 12)) & 15u);
}

template <typename C>
__device__ __forceinline__ C cmadd(C a, C g, C b, C h) {
    // g * a + h * b
    C r;
    r.x = g.x * a.x - g.y * a.y + h.x * b.x - h.y * b.y;
    r.y = g.x * a.y + g.y * a.x + h.x * b.y + h.y * b.x;
    return r;
}

// Controls: a thread whose thread/chunk control bits are not all set applies
// the identity (matrix chosen once per op); register-bit controls (cj) are
// the same for every lane, so pairs they exclude are skipped by a uniform
// branch.  Uncontrolled gates cost only the FMAs.
template <typename C, typename R, int NR, int I>
__device__ __forceinline__ void g1(C *v, const R *m, uint32_t cj, bool tok) {
    C g00, g01, g10, g11;
    g00.x = tok ? m[0] : (R)1; g00.y = tok ? m[1] : (R)0;
    g01.x = tok ? m[2] : (R)0; g01.y = tok ? m[3] : (R)0;
    g10.x = tok ? m[4] : (R)0; g10.y = tok ? m[5] : (R)0;
    g11.x = tok ? m[6] : (R)1; g11.y = tok ? m[7] : (R)0;
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        if ((j >> I) & 1) continue;
        if (((uint32_t)j & cj) != cj) continue;
        const int j1 = j | (1 << I);
        const C a = v[j], b = v[j1];
        v[j] = cmadd(a, g00, b, g01);
        v[j1] = cmadd(a, g10, b, g11);
    }
}

template <typename C, typename R, int NR, int I>
__device__ __forceinline__ void g1r(C *v, const R *m, uint32_t cj, bool tok) {
    const R g00 = tok ? m[0] : (R)1, g01 = tok ? m[1] : (R)0;
    const R g10 = tok ? m[2] : (R)0, g11 = tok ? m[3] : (R)1;
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        if ((j >> I) & 1) continue;
        if (((uint32_t)j & cj) != cj) continue;
        const int j1 = j | (1 << I);
        const C a = v[j], b = v[j1];
        C o0, o1;
        o0.x = g00 * a.x + g01 * b.x;
        o0.y = g00 * a.y + g01 * b.y;
        o1.x = g10 * a.x + g11 * b.x;
        o1.y = g10 * a.y + g11 * b.y;
        v[j] = o0;
        v[j1] = o1;
    }
}

template <typename C, typename R, int NR, int I1, int I2>
__device__ __forceinline__ void g2(C *v, const R *m, uint32_t cj, bool tok) {
    C g[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const R one = (e % 5 == 0) ? (R)1 : (R)0;   // identity for threads whose controls are not set
        g[e].x = tok ? m[2 * e] : one;
        g[e].y = tok ? m[2 * e + 1] : (R)0;
    }
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        if (((j >> I1) & 1) || ((j >> I2) & 1)) continue;
        if (((uint32_t)j & cj) != cj) continue;
        const int jj[4] = {j, j | (1 << I2), j | (1 << I1), j | (1 << I1) | (1 << I2)};
        C a[4], o[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) a[r] = v[jj[r]];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            C acc = cmul(g[4 * r], a[0]);
            acc = cfma(g[4 * r + 1], a[1], acc);
            acc = cfma(g[4 * r + 2], a[2], acc);
            acc = cfma(g[4 * r + 3], a[3], acc);
            o[r] = acc;
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) v[jj[r]] = o[r];
    }
}

// Phase sources of a pass op, as laid out in the program.
template <typename R> struct PhaseSrc {
    const R *pool;
    const PassSlotDev *slots;
    const PassTermDev *terms;
};

template <typename C, typename R, int NR, int RB>
__device__ void phase_factors(C *f, const PassOpDev &op, const PhaseSrc<R> &src, uint32_t t, uint64_t base, int sk);

// The phase that precedes a one-qubit gate on register bit I multiplies only
// its |1> members; its terms never need bit I, so f[j] = f[j | 2^I].
template <typename C, int NR, int I>
__device__ __forceinline__ void apply_pre(C *v, const C *f) {
#pragma unroll
    for (int j = 0; j < NR; ++j)
        if (!((j >> I) & 1)) v[j | (1 << I)] = cmul(v[j | (1 << I)], f[j]);
}

template <typename C, typename R, int NR, int RB>
__device__ __forceinline__ void dispatch_g1(const PassOpDev &op, bool real, C *v, const PhaseSrc<R> &src, uint32_t t,
                                            uint64_t base, bool tok) {
    const R *m = src.pool + op.mat;
    C f[NR];
    if (op.pre) phase_factors<C, R, NR, RB>(f, op, src, t, base, op.a);
#define QSV_G1(I)                                                               \
    case I:                                                                     \
        if constexpr (I < RB) {                                                 \
            if (op.pre) apply_pre<C, NR, I>(v, f);                              \
            if (real) g1r<C, R, NR, I>(v, m, op.cj, tok);                       \
            else g1<C, R, NR, I>(v, m, op.cj, tok);                             \
        }                                                                       \
        break;
    switch (op.a) {
        QSV_G1(0) QSV_G1(1) QSV_G1(2) QSV_G1(3) QSV_G1(4)
    }
#undef QSV_G1
}

template <typename C, typename R, int NR, int RB>
__device__ __forceinline__ void dispatch_g2(int a, int b, C *v, const R *m, uint32_t cj, bool tok) {
#define QSV_G2(I1, I2)                                              \
    case I1 * 8 + I2:                                               \
        if constexpr (I1 < RB) g2<C, R, NR, I1, I2>(v, m, cj, tok); \
        break;
    switch (a * 8 + b) {
        QSV_G2(1, 0) QSV_G2(2, 0) QSV_G2(2, 1) QSV_G2(3, 0) QSV_G2(3, 1)
        QSV_G2(3, 2) QSV_G2(4, 0) QSV_G2(4, 1) QSV_G2(4, 2) QSV_G2(4, 3)
    }
#undef QSV_G2
}

// phase = theta(fixed-point turns) -> multiply by e^{2 pi i phase}
__device__ __forceinline__ float2 rot(float2 v, uint64_t ph) {
    const float x = (float)(int32_t)(uint32_t)(ph >> 32) * 2.3283064365386963e-10f;   // turns in [-1/2, 1/2)
    float s, c;
    sincospif(2.0f * x, &s, &c);
    float2 r;
    r.x = v.x * c - v.y * s;
    r.y = v.x * s + v.y * c;
    return r;
}
__device__ __forceinline__ double2 rot(double2 v, uint64_t ph) {
    const double x = (double)(int64_t)ph * 5.421010862427522e-20;   // 2^-64
    double s, c;
    sincospi(2.0 * x, &s, &c);
    double2 r;
    r.x = v.x * c - v.y * s;
    r.y = v.x * s + v.y * c;
    return r;
}

__device__ __forceinline__ float2 expi(uint64_t ph, float) {
    const float x = (float)(int32_t)(uint32_t)(ph >> 32) * 2.3283064365386963e-10f;
    float2 r;
    sincospif(2.0f * x, &r.y, &r.x);
    return r;
}
__device__ __forceinline__ double2 expi(uint64_t ph, double) {
    const double x = (double)(int64_t)ph * 5.421010862427522e-20;
    double2 r;
    sincospi(2.0 * x, &r.y, &r.x);
    return r;
}

__device__ __forceinline__ float2 readlane(float2 v, int l) {
    float2 r;
    r.x = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v.x), l));
    r.y = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v.y), l));
    return r;
}
__device__ __forceinline__ double readlane(double v, int l) {
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
__device__ __forceinline__ double2 readlane(double2 v, int l) {
    double2 r;
    r.x = readlane(v.x, l);
    r.y = readlane(v.y, l);
    return r;
}

// Factor table f[j] of an op's phase (see PassOpDev) for the register
// indices j with bit sk clear (sk = -1: every j).  One copy of this code
// serves every PHASE op and every pre-phased one-qubit gate; the branches on
// op fields are uniform.
template <typename C, typename R, int NR, int RB>
__device__ void phase_factors(C *f, const PassOpDev &op, const PhaseSrc<R> &src, uint32_t t, uint64_t base, int sk) {
    C one;
    one.x = 1;
    one.y = 0;
    C F[RB + 1];
#pragma unroll
    for (int g = 0; g <= RB; ++g) {
        F[g] = one;
        if (op.tab[g] >= 0) {
            F[g].x = src.pool[op.tab[g] + 2 * t];
            F[g].y = src.pool[op.tab[g] + 2 * t + 1];
        }
    }
    // chunk-dependent slots: lane s sums slot s, one sincos for the wave,
    // then every thread multiplies in the slots its index covers
    const int s0 = op.sl[0], s1 = op.sl[RB + 1];
    if (s1 > s0) {
        const int lane = (int)(t & 63);
        uint64_t ph = 0;
        if (lane < s1 - s0) {
            const PassSlotDev S = src.slots[s0 + lane];
            for (int k = S.begin; k < S.end; ++k) {
                const PassTermDev tm = src.terms[k];
                ph += ((base & tm.mn) == tm.mn) ? tm.theta : 0ull;
            }
        }
        const C e = expi(ph, R());
#pragma unroll
        for (int g = 0; g <= RB; ++g) {
            for (int s = op.sl[g]; s < op.sl[g + 1]; ++s) {
                const C es = readlane(e, s - s0);
                const uint32_t mt = src.slots[s].mt;
                if ((t & mt) == mt) F[g] = cmul(F[g], es);
            }
        }
    }
    // f[j] = Fc[j] * F_0 * prod_{i in j} F_{1+i}
    if (op.var & 2) {
        f[0] = F[0];
#pragma unroll
        for (int top = 0; top < RB; ++top) {
            if (top == sk) continue;
#pragma unroll
            for (int rest = 0; rest < (1 << top); ++rest) {
                if (sk >= 0 && ((rest >> sk) & 1)) continue;
                f[rest | (1 << top)] = cmul(f[rest], F[1 + top]);
            }
        }
    } else {
#pragma unroll
        for (int j = 0; j < NR; ++j) f[j] = F[0];
    }
    if (op.fc >= 0) {
        const R *fc = src.pool + op.fc;
#pragma unroll
        for (int j = 0; j < NR; ++j) {
            if (sk >= 0 && ((j >> sk) & 1)) continue;
            C c;
            c.x = fc[2 * j];
            c.y = fc[2 * j + 1];
            f[j] = op.var ? cmul(f[j], c) : c;
        }
    }
    // general terms: evaluated per register index
    if (op.gen_e > op.gen_b) {
#pragma unroll
        for (int j = 0; j < NR; ++j) {
            if (sk >= 0 && ((j >> sk) & 1)) continue;
            uint64_t ph = 0;
            for (int k = op.gen_b; k < op.gen_e; ++k) {
                const PassTermDev tm = src.terms[k];
                const bool ok =
                    ((t & tm.mt) == tm.mt) && ((base & tm.mn) == tm.mn) && (((uint32_t)j & tm.mj) == tm.mj);
                ph += ok ? tm.theta : 0ull;
            }
            f[j] = rot(f[j], ph);
        }
    }
}

template <typename C, typename R, int NR, int RB>
__device__ __forceinline__ void phase_op(C *v, const PassOpDev &op, const PhaseSrc<R> &src, uint32_t t,
                                         uint64_t base) {
    C f[NR];
    phase_factors<C, R, NR, RB>(f, op, src, t, base, -1);
#pragma unroll
    for (int j = 0; j < NR; ++j) v[j] = cmul(v[j], f[j]);
}

// Prefetch when two register tiles fit the budget of 2+ waves per SIMD.
template <typename R, int RB> struct PassPrefetch {
    static constexpr bool value = sizeof(R) == 4 ? RB <= 4 : RB <= 3;
};

template <typename R, int RB>
__global__ void __launch_bounds__(PT) k_pass(typename cplx_of<R>::type *__restrict__ psi, const uint8_t *__restrict__ prog,
                                             uint64_t nchunks) {
    typedef typename cplx_of<R>::type C;
    constexpr bool PF = PassPrefetch<R, RB>::value;
    constexpr int NR = 1 << RB;
    constexpr int L = RB + PASS_THREAD_BITS;
    __shared__ C lds[1 << L];

    const PassHeaderDev *H = (const PassHeaderDev *)prog;
    const PassPartition *parts = (const PassPartition *)(prog + H->off_part);
    const PassOpDev *ops = (const PassOpDev *)(prog + H->off_ops);
    PhaseSrc<R> src;
    src.pool = (const R *)(prog + H->off_pool);
    src.slots = (const PassSlotDev *)(prog + H->off_slots);
    src.terms = (const PassTermDev *)(prog + H->off_terms);
    const R *pool = src.pool;
    const uint32_t t = threadIdx.x;
    const int nops = H->nops;

    auto chunk_base = [&](uint64_t c) {
        uint64_t base = c;
#pragma unroll
        for (int b = 0; b < L; ++b) {
            const uint64_t lo = base & H->lowmask[b];
            base = lo | ((base ^ lo) << 1);
        }
        return base;
    };
    // register offsets of the load partition (the same for every chunk)
    uint64_t lt_in = 0, lr_in[RB];
    {
        const PassPartition &P = parts[H->load_part];
#pragma unroll
        for (int u = 0; u < PASS_THREAD_BITS; ++u)
            if ((t >> u) & 1) lt_in |= 1ull << H->in_pos[P.thr_l[u]];
#pragma unroll
        for (int i = 0; i < RB; ++i) lr_in[i] = 1ull << H->in_pos[P.reg_l[i]];
    }
    auto load_chunk = [&](C *dst, uint64_t base) {
#pragma unroll
        for (int j = 0; j < NR; ++j) {
            uint64_t g = base | lt_in;
#pragma unroll
            for (int i = 0; i < RB; ++i)
                if ((j >> i) & 1) g |= lr_in[i];
            dst[j] = psi[g];
        }
    };
    // Software pipeline (PF): the next chunk's loads are issued before the
    // current chunk is computed, and the barriers below order LDS traffic
    // only, so those loads stay in flight across them.  Without PF (register
    // budget too small for two tiles) each chunk is loaded when its turn comes.
    uint64_t c = blockIdx.x;
    C v[NR];
    if constexpr (PF) {
        if (c < nchunks) load_chunk(v, chunk_base(c));
    }
    for (; c < nchunks; c += gridDim.x) {
        const uint64_t base = chunk_base(c);
        const uint64_t cn = c + gridDim.x;
        C vn[PF ? NR : 1];
        if constexpr (PF) {
            if (cn < nchunks) load_chunk(vn, chunk_base(cn));
        } else {
            (void)cn;
            load_chunk(v, base);
        }
        int cur = H->load_part;
        for (int o = 0; o < nops; ++o) {
            const PassOpDev &op = ops[o];
            const bool tok = ((t & op.ct) == op.ct) && ((base & op.cn) == op.cn);
            switch (op.kind) {
            case POP_G1: dispatch_g1<C, R, NR, RB>(op, false, v, src, t, base, tok); break;
            case POP_G1R: dispatch_g1<C, R, NR, RB>(op, true, v, src, t, base, tok); break;
            case POP_G2: dispatch_g2<C, R, NR, RB>(op.a, op.b, v, pool + op.mat, op.cj, tok); break;
            case POP_PHASE: phase_op<C, R, NR, RB>(v, op, src, t, base); break;
            case POP_EXCHANGE: {
                // The swizzle is linear over GF(2) and the bits of a local
                // index are disjoint, so the swizzled slot of register index
                // j is the thread's slot XOR the slots of j's register bits.
                const PassPartition &P = parts[cur];
                const PassPartition &Q = parts[op.a];
                uint32_t lt = 0, lq = 0;
#pragma unroll
                for (int u = 0; u < PASS_THREAD_BITS; ++u) {
                    if ((t >> u) & 1) {
                        lt |= 1u << P.thr_l[u];
                        lq |= 1u << Q.thr_l[u];
                    }
                }
                uint32_t ap[NR], aq[NR];
                ap[0] = lds_swizzle(lt);
                aq[0] = lds_swizzle(lq);
#pragma unroll
                for (int i = 0; i < RB; ++i) {
                    const uint32_t sp = lds_swizzle(1u << P.reg_l[i]), sq = lds_swizzle(1u << Q.reg_l[i]);
#pragma unroll
                    for (int r = 0; r < (1 << i); ++r) {
                        ap[r | (1 << i)] = ap[r] ^ sp;
                        aq[r | (1 << i)] = aq[r] ^ sq;
                    }
                }
                lds_barrier();
#pragma unroll
                for (int j = 0; j < NR; ++j) lds[ap[j]] = v[j];
                lds_barrier();
#pragma unroll
                for (int j = 0; j < NR; ++j) v[j] = lds[aq[j]];
                cur = op.a;
                break;
            }
            default: break;
            }
        }
        {
            // A thread may store to addresses another thread of the chunk
            // loaded (relabelled local bits without an exchange in between):
            // every thread's loads of the tile must have completed before
            // the barrier, which by itself does not wait for them.
            if (H->relabel) {
#pragma unroll
                for (int j = 0; j < NR; ++j) hold_value(v[j]);
                __syncthreads();
            }
            const PassPartition &P = parts[cur];
            uint64_t gt = base;
#pragma unroll
            for (int u = 0; u < PASS_THREAD_BITS; ++u)
                if ((t >> u) & 1) gt |= 1ull << H->out_pos[P.thr_l[u]];
            uint64_t gr[RB];
#pragma unroll
            for (int i = 0; i < RB; ++i) gr[i] = 1ull << H->out_pos[P.reg_l[i]];
#pragma unroll
            for (int j = 0; j < NR; ++j) {
                uint64_t g = gt;
#pragma unroll
                for (int i = 0; i < RB; ++i)
                    if ((j >> i) & 1) g |= gr[i];
                psi[g] = v[j];
            }
        }
        if constexpr (PF) {
#pragma unroll
            for (int j = 0; j < NR; ++j) v[j] = vn[j];
        }
    }
}

void PassProgram::serialise() {
    PassHeaderDev h;
    std::memset(&h, 0, sizeof(h));
    h.L = L;
    h.nops = (int)ops.size();
    h.npart = (int)parts.size();
    h.load_part = load_part;
    for (int l = 0; l < L; ++l) {
        h.in_pos[l] = local_sorted[l];
        h.out_pos[l] = out_pos[l];
        h.lowmask[l] = (1ull << local_sorted[l]) - 1ull;
        if (out_pos[l] != local_sorted[l]) h.relabel = 1;
    }
    // An exchange's barriers already order every load before any store; only
    // relabelled positions in a pass without exchanges need the extra barrier.
    for (const auto &op : ops)
        if (op.kind == POP_EXCHANGE) h.relabel = 0;
    auto align = [](size_t x) { return (x + 15) & ~(size_t)15; };
    size_t off = align(sizeof(PassHeaderDev));
    h.off_part = (int)off;
    off = align(off + parts.size() * sizeof(PassPartition));
    h.off_ops = (int)off;
    off = align(off + ops.size() * sizeof(PassOpDev));
    h.off_pool = (int)off;
    off = align(off + pool.size() * sizeof(double));   // room for the widest real type
    h.off_terms = (int)off;
    off = align(off + terms.size() * sizeof(PassTermDev));
    h.off_slots = (int)off;
    off = align(off + slots.size() * sizeof(PassSlotDev));
    h.total_bytes = (int)off;
    blob.assign(off, 0);
    std::memcpy(blob.data(), &h, sizeof(h));
    if (!parts.empty()) std::memcpy(blob.data() + h.off_part, parts.data(), parts.size() * sizeof(PassPartition));
    if (!ops.empty()) std::memcpy(blob.data() + h.off_ops, ops.data(), ops.size() * sizeof(PassOpDev));
    if (!terms.empty()) std::memcpy(blob.data() + h.off_terms, terms.data(), terms.size() * sizeof(PassTermDev));
    if (!slots.empty()) std::memcpy(blob.data() + h.off_slots, slots.data(), slots.size() * sizeof(PassSlotDev));
    // the pool is written per dtype at launch time (float or double)
}

template <typename R, int RB>
static void launch_k_pass(void *state, const uint8_t *dprog, uint64_t nchunks, hipStream_t s) {
    // persistent workgroups: as many as can be resident, each walking the
    // chunks with a stride (so its prefetch always has a next chunk)
    static int resident[64] = {0};
    int dev = 0;
    (void)hipGetDevice(&dev);
    if (dev < 0 || dev >= 64) dev = 0;
    if (resident[dev] == 0) {
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_pass<R, RB>, PT, 0) != hipSuccess || per_cu < 1)
            per_cu = 1;
        resident[dev] = per_cu;
    }
    uint64_t g = (uint64_t)resident[dev] * device_sm_count();
    if (!PassPrefetch<R, RB>::value) g = std::min<uint64_t>(nchunks, 1ull << 20);   // one chunk per workgroup
    if (g > nchunks) g = nchunks;
    hipLaunchKernelGGL((k_pass<R, RB>), dim3((unsigned)g), dim3(PT), 0, s, (typename cplx_of<R>::type *)state, dprog,
                       nchunks);
}

// Copies a serialised program (pool in the state's real type) into a staging
// slot and uploads it on stream s; the caller releases the slot after the
// launch that reads it.
int upload_pass_program(const PassProgram &prog, int dtype, hipStream_t s, StagingSlot *slot) {
    const size_t bytes = prog.blob.size();
    if (bytes > staging_slot_bytes()) return fail(QSV_ERR_UNSUPPORTED, "pass program larger than a staging slot");
    int st = staging_acquire(bytes, slot);
    if (st) return st;
    std::memcpy(slot->host, prog.blob.data(), bytes);
    const PassHeaderDev *h = (const PassHeaderDev *)prog.blob.data();
    if (dtype == QSV_C64) {
        float *pool = (float *)((char *)slot->host + h->off_pool);
        for (size_t i = 0; i < prog.pool.size(); ++i) pool[i] = (float)prog.pool[i];
    } else {
        double *pool = (double *)((char *)slot->host + h->off_pool);
        for (size_t i = 0; i < prog.pool.size(); ++i) pool[i] = prog.pool[i];
    }
    if ((st = staging_upload(*slot, bytes, s))) {
        staging_release(*slot, s);
        return st;
    }
    return QSV_OK;
}

int launch_pass_program(void *state, int n, int dtype, const PassProgram &prog, hipStream_t s) {
    if (!prog.pair_sigma.empty() || prog.TB != PASS_THREAD_BITS)
        return fail(QSV_ERR_UNSUPPORTED, "internal: this pass program needs its compiled kernel");
    StagingSlot slot;
    int st = upload_pass_program(prog, dtype, s, &slot);
    if (st) return st;
    const uint64_t nchunks = 1ull << (n - prog.L);
    const uint8_t *d = (const uint8_t *)slot.dev;
    if (dtype == QSV_C64) {
        switch (prog.RB) {
        case 1: launch_k_pass<float, 1>(state, d, nchunks, s); break;
        case 2: launch_k_pass<float, 2>(state, d, nchunks, s); break;
        case 3: launch_k_pass<float, 3>(state, d, nchunks, s); break;
        case 4: launch_k_pass<float, 4>(state, d, nchunks, s); break;
        case 5: launch_k_pass<float, 5>(state, d, nchunks, s); break;
        default: staging_release(slot, s); return fail(QSV_ERR_ARG, "internal: bad register bits");
        }
    } else {
        switch (prog.RB) {
        case 1: launch_k_pass<double, 1>(state, d, nchunks, s); break;
        case 2: launch_k_pass<double, 2>(state, d, nchunks, s); break;
        case 3: launch_k_pass<double, 3>(state, d, nchunks, s); break;
        case 4: launch_k_pass<double, 4>(state, d, nchunks, s); break;
        default: staging_release(slot, s); return fail(QSV_ERR_ARG, "internal: bad register bits");
        }
    }
    hipError_t e = hipGetLastError();
    staging_release(slot, s);
    if (e != hipSuccess) return hip_fail(e, "pass kernel launch");
    return QSV_OK;
}

}  // namespace qsv
