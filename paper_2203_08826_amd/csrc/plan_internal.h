// Internal plan and pass-program structures (host side + the device layout
// of a pass program).
#pragma once

#include <memory>
#include <vector>

#include "qsv_internal.h"

namespace qsv {

// ---------------------------------------------------------------- pass programs
//
// A pass processes the state chunk by chunk.  A chunk is the set of 2^L
// amplitudes that share every non-local bit; the L local bits of an index
// are numbered l = 0..L-1 ("local positions").  A workgroup of 256 threads
// holds one chunk: thread t keeps 2^RB amplitudes in registers (L = RB + 8).
// A "partition" says which local positions are register bits (j index) and
// which are thread bits (t index: bits 0..5 lane, 6..7 wave).  Ops act on
// register bits; an EXCHANGE op moves to another partition through LDS.

constexpr int PASS_THREAD_BITS = 8;
constexpr int PASS_MAX_RB = 5;
constexpr int PASS_MAX_L = PASS_MAX_RB + PASS_THREAD_BITS;
constexpr int PASS_GROUPS = 1 + PASS_MAX_RB + PASS_MAX_RB * (PASS_MAX_RB - 1) / 2 + 1;   // c0, lin, quad, general

enum PassOpKind : int32_t { POP_EXCHANGE = 1, POP_G1 = 2, POP_G1R = 3, POP_G2 = 4, POP_PHASE = 5 };

struct PassPartition {
    int32_t reg_l[PASS_MAX_RB];          // local position of register bit i
    int32_t thr_l[PASS_THREAD_BITS];     // local position of thread bit u
};

// Phase evaluation (PHASE ops, and the phase a G1/G1R op applies to its
// |1> member first when `pre` is set): terms are grouped by the register
// bits they need under the op's partition --
//   group 0        : no register bit      -> per-thread sum A0
//   group 1 + i    : register bit i only  -> per-thread sum A_i
//   group 1+RB+q   : register pair q      -> constant, host factor in the pool at qf
//   last group     : everything else      -> evaluated per register index
// and the factor of register index j is e^{iA0} prod_{i in j} e^{iA_i}
// prod_{pairs in j} Q_pair, built as a product table.
struct PassOpDev {
    int32_t kind;
    int32_t a, b;          // G1: register bit a.  G2: register bits a > b.  EXCHANGE: partition index
    uint32_t ct;           // controls on thread bits (mask over t)
    uint32_t cj;           // controls on register bits (mask over j)
    int32_t mat;           // offset into the real pool
    uint64_t cn;           // controls on non-local bits (mask over global index)
    int32_t grp[PASS_GROUPS + 1];   // term ranges [grp[g], grp[g+1]) per group
    int32_t grpu[PASS_GROUPS];      // terms [grp[g], grpu[g]) need no thread bit (uniform per chunk)
    int32_t qf;            // pool offset of the constant pair factors (complex, one per pair)
    int32_t lf;            // pool offset of the constant single-bit factors (complex, one per register bit)
    int32_t pre;           // G1/G1R: apply the grouped phase to the |1> member first
    int32_t noquad;        // every pair factor is exactly 1 (simpler product table)
};

// Phase term: contributes theta (fixed-point turns, 2^64 = one turn) when
// every bit of mt (thread index), of mn (global chunk base) and of the
// group's register bits is 1.  General-group terms also carry mj.
struct PassTermDev {
    uint64_t mn;
    uint64_t theta;
    uint32_t mt;
    uint32_t mj;
};

struct PassHeaderDev {
    int32_t L;
    int32_t nops;
    int32_t npart;
    int32_t load_part;     // partition used for the global load
    int32_t in_pos[PASS_MAX_L];    // global bit of local position l (load)
    int32_t out_pos[PASS_MAX_L];   // global bit of local position l (store)
    uint64_t lowmask[PASS_MAX_L];  // sorted local bits, for the chunk base
    int32_t off_part, off_ops, off_pool, off_terms;   // byte offsets from the header
    int32_t total_bytes;
    int32_t relabel;               // 1: some thread stores where another loaded
};

// Host-side pass program (what the planner emits, before serialisation).
struct PassProgram {
    int L = 0;
    int RB = 0;
    std::vector<int> local_sorted;        // global bits of local positions at load (ascending)
    std::vector<int> out_pos;             // global bit of local position l at store
    std::vector<PassPartition> parts;
    int load_part = 0;
    std::vector<PassOpDev> ops;
    std::vector<double> pool;
    std::vector<PassTermDev> terms;
    int n_gates = 0;                      // circuit gates folded into this pass
    std::vector<uint8_t> blob;            // serialised program
    void serialise();
};

int launch_pass_program(void *state, int n, int dtype, const PassProgram &prog, hipStream_t s);
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
void finish_stats(qsv_plan *p);
int execute_plan(const qsv_plan *p, void *state, hipStream_t s);
int execute_op(const qsv_plan *p, const PlanOp &op, void *state, hipStream_t s);

// Build one pass for the given gates on a forced local set (qsv_run_pass).
int build_single_pass(int n, int dtype, const std::vector<qsv_gate> &gates, const std::vector<int> &local,
                      PassProgram &out);

}  // namespace qsv
