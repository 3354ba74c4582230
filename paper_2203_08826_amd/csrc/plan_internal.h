// Internal plan and pass-program structures (host side + the device layout
// of a pass program).
#pragma once

#include <cstddef>
#include <memory>
#include <vector>

#include "qsv_internal.h"

namespace qsv {

// ---------------------------------------------------------------- pass programs
//
// A pass processes the state chunk by chunk.  A chunk is the set of 2^L
// amplitudes that share every non-local bit; the L local bits of an index
// are numbered l = 0..L-1 ("local positions").  A workgroup of 2^TB threads
// holds one chunk: thread t keeps 2^RB amplitudes in registers (L = RB + TB;
// TB = 8 for the interpreted kernel, 9 for compiled passes, whose straight-
// line code leaves room for 512-thread workgroups and 128 KiB chunks).
// A "partition" says which local positions are register bits (j index) and
// which are thread bits (t index: bits 0..5 lane, the rest wave).  Ops act on
// register bits; an EXCHANGE op moves to another partition through LDS.

constexpr int PASS_THREAD_BITS = 8;        // interpreted kernel
constexpr int PASS_JIT_THREAD_BITS = 9;    // compiled passes
constexpr int PASS_MAX_THREAD_BITS = 9;
constexpr int PASS_MAX_RB = 5;
constexpr int PASS_MAX_L = PASS_MAX_RB + PASS_MAX_THREAD_BITS;
constexpr int PASS_MAX_SLOTS = 64;       // per op: one per lane of a wave
constexpr size_t PASS_LOOKAHEAD = 4096;   // gates a pass planner scans past one that does not fit
constexpr int PASS_MAX_NONDIAG = 64;      // non-diagonal gates per pass
constexpr int PASS_SLOT_TERMS = 32;      // longer slots are split

enum PassOpKind : int32_t { POP_EXCHANGE = 1, POP_G1 = 2, POP_G1R = 3, POP_G2 = 4, POP_PHASE = 5 };

struct PassPartition {
    int32_t reg_l[PASS_MAX_RB];          // local position of register bit i
    int32_t thr_l[PASS_MAX_THREAD_BITS]; // local position of thread bit u (u < TB)
};

// Phase evaluation (PHASE ops, and the phase a G1/G1R op applies to its
// |1> member first when `pre` is set).  The phase of register index j in
// thread t of the chunk with base index `base` factors as
//   f[j] = Fc[j] * F_0 * prod_{i in j} F_{1+i}
// where Fc is a host table of the terms that need register bits only, and
// F_g (g = 0: no register bit, g = 1+i: register bit i and no other) is the
// product of
//   - a host table over the 256 threads (terms that need thread bits only),
//   - "slots": sums of terms that need chunk bits, one per thread mask; the
//     64 lanes of a wave evaluate up to 64 slots side by side, and every
//     thread whose bits cover a slot's mask multiplies in its factor.
// Terms that need two or more register bits together with thread or chunk
// bits ("general" terms) are evaluated per register index.
struct PassOpDev {
    int32_t kind;
    int32_t a, b;          // G1: register bit a.  G2: register bits a > b.  EXCHANGE: partition index
    uint32_t ct;           // controls on thread bits (mask over t)
    uint32_t cj;           // controls on register bits (mask over j)
    int32_t mat;           // offset into the real pool
    uint64_t cn;           // controls on non-local bits (mask over global index)
    int32_t tab[PASS_MAX_RB + 1];   // pool offset of the per-thread table of F_g (256 complex), or -1
    int32_t sl[PASS_MAX_RB + 2];    // slots [sl[g], sl[g+1]) belong to F_g
    int32_t gen_b, gen_e;           // general terms
    int32_t fc;            // pool offset of Fc (2^RB complex), or -1 when every entry is 1
    int32_t var;           // bit 0: F_0 is not 1; bit 1: some F_{1+i} is not 1
    int32_t pre;           // G1/G1R: apply the phase to the |1> member first
    int32_t pad;
};

// Phase term: contributes theta (fixed-point turns, 2^64 = one turn) when
// every bit of mn (global chunk base) is 1 -- and, for general terms, every
// bit of mt (thread index) and of mj (register index).
struct PassTermDev {
    uint64_t mn;
    uint64_t theta;
    uint32_t mt;
    uint32_t mj;
};

// parametric compiled kernels read theta as 64-bit word 1 + 3 k of the terms
static_assert(sizeof(PassTermDev) == 24 && offsetof(PassTermDev, theta) == 8, "phase term layout");

// A slot: the chunk-dependent phase sum of terms [begin, end), applied in
// the threads whose index covers mt.
struct PassSlotDev {
    int32_t begin, end;
    uint32_t mt;
    int32_t pad;
};

struct PassHeaderDev {
    int32_t L;
    int32_t nops;
    int32_t npart;
    int32_t load_part;     // partition used for the global load
    int32_t in_pos[PASS_MAX_L];    // global bit of local position l (load)
    int32_t out_pos[PASS_MAX_L];   // global bit of local position l (store)
    uint64_t lowmask[PASS_MAX_L];  // sorted local bits, for the chunk base
    int32_t off_part, off_ops, off_pool, off_terms, off_slots;   // byte offsets from the header
    int32_t total_bytes;
    int32_t relabel;               // 1: some thread stores where another loaded
};

// The serialised layout is read back on the host by the tests (through
// qsv_plan_op_program): keep these offsets.
static_assert(sizeof(PassPartition) == 56 && sizeof(PassOpDev) == 112 && offsetof(PassHeaderDev, off_part) == 240 &&
                  offsetof(PassHeaderDev, off_ops) == 244,
              "pass program layout");

struct JitModule;   // a pass program compiled into a kernel of its own (pass_jit.cpp)

// Host-side pass program (what the planner emits, before serialisation).
struct PassProgram {
    int L = 0;
    int RB = 0;
    int TB = PASS_THREAD_BITS;            // thread bits (workgroup of 2^TB threads)
    std::vector<int> local_sorted;        // global bits of local positions at load (ascending)
    std::vector<int> out_pos;             // global bit of local position l at store
    std::vector<PassPartition> parts;
    int load_part = 0;
    std::vector<PassOpDev> ops;
    std::vector<double> pool;
    std::vector<PassTermDev> terms;
    std::vector<PassSlotDev> slots;
    int n_gates = 0;                      // circuit gates folded into this pass
    std::vector<uint8_t> blob;            // serialised program
    std::shared_ptr<JitModule> jit;       // compiled kernel, when the plan asked for one
    std::vector<int> pair_sigma;          // if set: chunk c is stored at chunk pair_sigma(c) (compiled kernel only)
    bool param = false;                   // compiled kernel reads matrices and phases from the program
    void serialise();
};

int upload_pass_program(const PassProgram &prog, int dtype, hipStream_t s, StagingSlot *slot);
int launch_pass_program(void *state, int n, int dtype, const PassProgram &prog, hipStream_t s);
int launch_pass_jit(void *state, int n, int dtype, const PassProgram &prog, hipStream_t s);
// Code-generation choices of a compiled pass: products of phase factors
// that several amplitudes take formed once (fewer multiplications, more live
// registers); the next chunk prefetched into registers where that applies.
struct JitVariant {
    bool share = true;
    bool prefetch = true;
    // exchanges in rounds over a register bit both partitions hold (half the
    // LDS), one chunk per workgroup and at most 128 registers per lane, so
    // that two workgroups share a CU (no prefetch: each one's memory traffic
    // overlaps the other's arithmetic)
    bool split = false;
};
std::string pass_jit_source(const PassProgram &prog, int dtype, const JitVariant &v);
std::string pass_jit_module_source(const PassProgram &prog);   // the source of the kernel compiled, if any
struct PairLayout {
    std::vector<int> a, b;       // the non-local pairs sigma swaps, a < b, ascending a
    std::vector<int> fixed;      // the non-local bits sigma fixes
};
PairLayout pair_layout(const std::vector<int> &sigma, uint64_t local);
uint64_t pair_work_items(const std::vector<int> &sigma, uint64_t local);
bool pass_jit_prefetch(const PassProgram &p, int dtype);
int launch_bitperm(void *state, int n, int dtype, const std::vector<int> &sigma, hipStream_t s);

// ---------------------------------------------------------------- plans

struct PlanOp {
    enum Kind { GATE = 0, MFMA_BLOCK = 1, PASS = 2, PERM = 3 } kind = GATE;
    std::vector<int> sigma;                // PERM: destination bit of every source bit (an involution)
    GateAnalysis analysis;                 // GATE
    std::vector<int> qubits;               // MFMA_BLOCK: block qubits (targets[0] = MSB)
    std::vector<double> matrix;            // MFMA_BLOCK: complex128 4^k
    std::shared_ptr<PassProgram> pass;     // PASS
    bool fused = false;                    // GATE built from a fused block of several gates
    std::vector<int> gate_ids;             // circuit indices of the gates applied, in application order
    double bytes = 0, flops = 0;
};

}  // namespace qsv

struct qsv_plan {
    int n = 0;
    int dtype = 0;
    qsv_plan_options opts;
    std::vector<qsv_gate> gates;
    std::vector<std::vector<double>> data;     // private copies of MATRIX / DIAG data
    std::vector<qsv::PlanOp> ops;
    std::vector<std::vector<int>> blocks;      // greedy fusion blocks
    std::vector<int> block_of_gate;
    qsv_plan_stats stats;
};

namespace qsv {

std::vector<std::vector<int>> greedy_fusion(const std::vector<qsv_gate> &gates, int kmax);
int fused_block(const std::vector<qsv_gate> &gates, const std::vector<int> &members, std::vector<int> &qubits,
                std::vector<double> &M);
int plan_add_gate_op(qsv_plan *p, const qsv_gate &g);
int plan_add_block_op(qsv_plan *p, const std::vector<int> &qubits, const std::vector<double> &M, bool allow_mfma);
int build_greedy(qsv_plan *p, int kmax, bool allow_mfma);
int build_passes(qsv_plan *p, int local_bits);
int build_learned(qsv_plan *p);
int jit_compile_plan(qsv_plan *p);   // compiles every pass of the plan (hiprtc)
void finish_stats(qsv_plan *p);
int execute_plan(const qsv_plan *p, void *state, hipStream_t s);
int execute_op(const qsv_plan *p, const PlanOp &op, void *state, hipStream_t s);

// Build one pass for the given gates on a forced local set (qsv_run_pass).
int build_single_pass(int n, int dtype, const std::vector<qsv_gate> &gates, const std::vector<int> &local,
                      PassProgram &out);

}  // namespace qsv
