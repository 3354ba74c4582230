/*
 * qsv.h -- C ABI of libqsv.so, an MI355X (gfx950) state-vector simulator.
 *
 * The problem statement this library implements is Eq. 1 of the paper's
 * introduction (arXiv:2203.08826): a gate acting on n_tar target qubits is a
 * 2^n_tar x 2^n_tar complex matrix G(tau, tau') applied to the 2^n complex
 * amplitudes psi(sigma_1..sigma_n) of an n-qubit state; the methodology
 * section (Sec. 2) states the operator shape (state, gate matrix, target
 * qubits; controlled gates; specialised X/Y/Z/SWAP operators; in-place
 * update; measurement).
 *
 * Conventions used by every entry point:
 *   - qubit q is bit q of the amplitude index (stride 2^q);
 *   - a k-target gate matrix is row-major, 4^k entries, and targets[0] is the
 *     most significant bit of its row/column index;
 *   - a gate acts only on amplitudes whose control bits are all 1;
 *   - states are contiguous device arrays of 2^n complex numbers, either
 *     complex64 (interleaved float re, im) or complex128 (interleaved
 *     double re, im), aligned to 16 bytes;
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *
 * Ownership and ordering: the caller owns every state and every output
 * buffer; the library never allocates or frees them.  Host inputs (gate
 * matrices, qubit lists, op lists) are consumed before the call returns, so
 * the caller may free them immediately.  Work is queued asynchronously on
 * `stream` and updates the state in place; outputs written to device memory
 * are valid once the stream has reached them.  The library keeps no pointer
 * to caller memory after returning.
 *
 * Errors: every argument is validated on the host before anything is queued.
 * On error nothing is queued, the state is untouched and a negative QSV_ERR_*
 * code is returned; qsv_last_error() then holds a message for the calling
 * thread.  Faults of earlier asynchronous work surface at the next call that
 * synchronises.  No C++ exception crosses this interface.  Calls are
 * reentrant; calls on distinct streams are independent.
 */
#ifndef QSV_H
#define QSV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QSV_ABI_VERSION 2

/* Status codes. */
enum {
    QSV_OK = 0,
    QSV_ERR_NULL = -1,        /* a required pointer is NULL */
    QSV_ERR_DTYPE = -2,       /* dtype is not QSV_C64 / QSV_C128 */
    QSV_ERR_NQUBITS = -3,     /* n < 1, n > QSV_MAX_QUBITS */
    QSV_ERR_QUBIT_RANGE = -4, /* a qubit index is outside [0, n) */
    QSV_ERR_QUBIT_DUP = -5,   /* a qubit repeats in targets + controls */
    QSV_ERR_ARITY = -6,       /* k + c > n, or k / c above the limit of the call */
    QSV_ERR_ALIGN = -7,       /* state pointer not 16-byte aligned */
    QSV_ERR_UNSUPPORTED = -8, /* valid request this call does not implement */
    QSV_ERR_HIP = -9,         /* the HIP runtime reported an error */
    QSV_ERR_ARG = -10         /* another argument is out of its range */
};

/* State element types. */
enum { QSV_C64 = 0, QSV_C128 = 1 };

#define QSV_MAX_QUBITS 40
#define QSV_MAX_TARGETS 6   /* k of a dense gate */
#define QSV_MAX_CONTROLS 8  /* c of a controlled gate */

/* ------------------------------------------------------------------ misc */

int qsv_abi_version(void);
const char *qsv_status_string(int status);
/* Message of the last failing call on this thread ("" if none). */
const char *qsv_last_error(void);

/* Device memory the library holds for itself, in bytes, summed over devices
 * (the paper's memory comparison, Sec. 3.1, is of peak device memory per
 * simulator; every gate, plan and reduction here works in place, so the
 * caller's state plus this is the footprint).  Counted: the staging ring
 * (256 slots of 256 KiB per device, allocated at first use, kept until the
 * process ends) and per-call temporaries (adjoint partial sums, cost-model
 * batches, the two slice buffers of qsv_sliced_run).  Not counted: code
 * objects of compiled passes and the fixed scratch array of
 * qsv_probabilities_noalloc.  `peak_bytes` is the largest total since the
 * last reset; reset_peak != 0 sets it to the current total after reading.
 * Either pointer may be NULL.  Host only; returns QSV_OK. */
int qsv_memory_stats(uint64_t *current_bytes, uint64_t *peak_bytes, int reset_peak);

/* Host-only validation of a gate's qubits (no HIP call; usable without a
 * GPU): 1 <= n <= QSV_MAX_QUBITS, dtype valid, 0 <= k <= QSV_MAX_TARGETS,
 * 0 <= c <= QSV_MAX_CONTROLS, k + c <= n, every index in [0, n), no repeats. */
int qsv_validate(int n, int dtype, const int *targets, int k, const int *controls, int c);

/* Host-only: group-index map used by every gate kernel (exposed for tests).
 * Group g in [0, 2^(n - m)) maps to the index with a 0 inserted at each of
 * the m sorted positions `bits` (ascending), i.e. the smallest member of the
 * group.  Writes count indices starting at group `first` into out. */
int qsv_group_index_host(int n, const int *bits, int m, uint64_t first, uint64_t count, uint64_t *out);

/* ------------------------------------------------------------------ gates
 * Eq. 1 for one gate, in place.  `gate` is host memory in the state's dtype
 * (complex64 pairs of float, complex128 pairs of double), row-major 4^k
 * entries.  The kernel chosen depends on the matrix: diagonal, monomial
 * (permutation with phases: X, Y, SWAP, CNOT) and partly-identity matrices
 * touch only the amplitudes they change (the sparsity the methodology section
 * exploits for Pauli and controlled gates); others run the dense k-target
 * kernel.  1 <= k <= QSV_MAX_TARGETS. */
int qsv_apply_matrix(void *state, int n, int dtype, const void *gate,
                     const int *targets, int k, const int *controls, int c, void *stream);

/* Specialised gates (methodology section: Pauli X, Y, Z and SWAP operators;
 * controlled gates).  Each touches only the amplitudes it changes.  X, SWAP
 * and their controlled forms move amplitudes bit-exactly. */
int qsv_apply_x(void *state, int n, int dtype, int target, const int *controls, int c, void *stream);
int qsv_apply_y(void *state, int n, int dtype, int target, const int *controls, int c, void *stream);
int qsv_apply_z(void *state, int n, int dtype, int target, const int *controls, int c, void *stream);
int qsv_apply_swap(void *state, int n, int dtype, int t0, int t1, const int *controls, int c, void *stream);
/* U1(phi) = diag(1, e^{i phi}); one control gives CU1, phi = pi gives CZ. */
int qsv_apply_phase(void *state, int n, int dtype, int target, double phi,
                    const int *controls, int c, void *stream);
/* Diagonal gate: `diag` holds 2^k host values in the state's dtype, index
 * order as for matrices; entries exactly equal to 1 are skipped. */
int qsv_apply_diagonal(void *state, int n, int dtype, const void *diag,
                       const int *targets, int k, const int *controls, int c, void *stream);
/* fSim(theta, phi) on (t0, t1): |00> unchanged, [[cos, -i sin], [-i sin, cos]]
 * on {|01>, |10>}, e^{-i phi} on |11> (t0 = most significant). */
int qsv_apply_fsim(void *state, int n, int dtype, int t0, int t1, double theta, double phi, void *stream);

/* psi <- (re + i im) psi for every amplitude: normalisation and global
 * phases.  Also the plain in-place stream (one read and one write of the
 * state) that the gate kernels are measured against. */
int qsv_scale(void *state, int n, int dtype, double re, double im, void *stream);

/* ------------------------------------------------------------------ circuits
 * A circuit is an array of qsv_gate.  Named kinds build their matrix from
 * params; QSV_GATE_MATRIX and QSV_GATE_DIAG read `data` (host complex128,
 * 4^k resp. 2^k entries).  CNOT, CZ and CU1 are X, Z and U1 with one entry in
 * `controls`. */
enum {
    QSV_GATE_MATRIX = 0, QSV_GATE_H, QSV_GATE_X, QSV_GATE_Y, QSV_GATE_Z,
    QSV_GATE_SX, QSV_GATE_SY, QSV_GATE_SW, QSV_GATE_RX, QSV_GATE_RY, QSV_GATE_RZ,
    QSV_GATE_U1, QSV_GATE_SWAP, QSV_GATE_FSIM, QSV_GATE_DIAG,
    QSV_GATE_KIND_COUNT
};

typedef struct qsv_gate {
    int kind;                          /* QSV_GATE_* */
    int k;                             /* number of targets */
    int c;                             /* number of controls */
    int targets[QSV_MAX_TARGETS];
    int controls[QSV_MAX_CONTROLS];
    double params[2];                  /* angles of named kinds */
    const void *data;                  /* MATRIX / DIAG entries, complex128, host */
} qsv_gate;

/* Host-only: the complex128 target block of a gate (4^k entries) into out. */
int qsv_gate_matrix(const qsv_gate *gate, double *out);

/* Plans.  A plan turns a circuit into a sequence of kernel launches:
 *   QSV_PLAN_PER_GATE  one launch per gate, no fusion;
 *   QSV_PLAN_GREEDY    greedy fusion (Sec. 3.2 of the paper, extended to
 *                      kmax <= 6): each gate joins the most recent of its
 *                      qubits' last blocks while the union stays within kmax
 *                      qubits; fused blocks with 4..6 qubits on complex64 run
 *                      on the FP32 matrix-core kernel;
 *   QSV_PLAN_PASSES    LDS-staged passes: consecutive gates whose non-diagonal
 *                      targets fit one chunk of local qubits run in one HBM
 *                      read + write of the state;
 *   QSV_PLAN_LEARNED   the candidate plans above are scored by the MLP cost
 *                      model loaded with qsv_cost_model_set and the cheapest
 *                      is kept; without a model it is QSV_PLAN_GREEDY. */
enum { QSV_PLAN_PER_GATE = 0, QSV_PLAN_GREEDY = 1, QSV_PLAN_PASSES = 2, QSV_PLAN_LEARNED = 3 };

typedef struct qsv_plan_options {
    int mode;          /* QSV_PLAN_* */
    int kmax;          /* fusion width for QSV_PLAN_GREEDY, 1..6 (default 2) */
    int local_bits;    /* chunk bits for QSV_PLAN_PASSES, 0 = library default (the
                        * largest): interpreted passes take 9..13 (complex64) or
                        * 9..12 (complex128), compiled passes (512-thread
                        * workgroups) 10..14 or 10..13 */
    int use_mfma;      /* 1: fused complex64 blocks of 4..6 qubits use MFMA */
    int jit;           /* 1: every LDS pass of the plan is compiled (hiprtc, at
                        * qsv_plan_create) into a kernel specialised for its
                        * gates -- constants, bit assignments and op sequence
                        * fixed at compile time; results equal the interpreted
                        * pass kernel's up to rounding (matrix and phase entries
                        * within 2^-50 of 0 or +-1 are taken as exact).
                        * 2: compiled as for 1, but parametric: gate matrix
                        * entries and phase angles are read from the pass
                        * program at run time instead of compiled in, so a
                        * kernel depends only on the circuit's structure;
                        * plans of circuits that differ only in their angles
                        * (a parameter sweep) share compiled kernels, and a
                        * plan with the same structure as an earlier one in
                        * the process compiles nothing.
                        * 0: interpreted. */
} qsv_plan_options;

typedef struct qsv_plan qsv_plan;

/* Statistics of a plan (host-side counts and the byte model of the launches). */
typedef struct qsv_plan_stats {
    int n_launches;        /* kernels per execution */
    int n_gate_ops;        /* per-gate kernel launches */
    int n_blocks;          /* fused dense blocks */
    int n_mfma_blocks;     /* of which on MFMA */
    int n_passes;          /* LDS passes */
    int mode_used;         /* QSV_PLAN_* finally used (LEARNED resolves to another) */
    int n_jit_passes;      /* LDS passes running as compiled kernels */
    double bytes;          /* algorithmic HBM bytes per execution */
    double flops;          /* algorithmic flops per execution */
    double predicted_s;    /* cost-model prediction, 0 if none */
} qsv_plan_stats;

/* Build a plan on the host (no HIP call unless mode = LEARNED with a model,
 * which runs the MLP inference kernel on the current device).  With
 * opts->jit the passes are compiled here (host compiler only; the plan's
 * kernels in one program, a kernel that spills registers compiled again in
 * a leaner variant; each code object is loaded on a device at the first
 * execution of one of its kernels there); a compilation failure
 * returns QSV_ERR_UNSUPPORTED with the compiler log in qsv_last_error.  The
 * gates are copied; the caller may free them afterwards. */
int qsv_plan_create(int n, int dtype, const qsv_gate *gates, int ngates,
                    const qsv_plan_options *opts, qsv_plan **out);
int qsv_plan_stats_get(const qsv_plan *plan, qsv_plan_stats *out);
/* Greedy block of every gate (block ids in plan order) -- for tests; the plan
 * must have been built with QSV_PLAN_GREEDY. */
int qsv_plan_blocks(const qsv_plan *plan, int *block_of_gate, int ngates);
/* Queue the whole plan on `stream`, updating `state` in place. */
int qsv_plan_execute(const qsv_plan *plan, void *state, void *stream);
/* Queue ops [first, first + count) of the plan only (for per-op timing). */
int qsv_plan_execute_ops(const qsv_plan *plan, void *state, int first, int count, void *stream);
/* Kind (0 = gate kernel, 1 = MFMA block, 2 = LDS pass), algorithmic HBM
 * bytes and flops of op `index`; any output pointer may be NULL. */
int qsv_plan_op_info(const qsv_plan *plan, int index, int *kind, double *bytes, double *flops);
/* Host-only: copy the serialised program of LDS-pass op `index` (layout in
 * plan_internal.h: header, partitions, ops, real pool, phase terms, slots; the pool
 * is stored as doubles) into buf (cap bytes); *size receives the length. */
int qsv_plan_op_program(const qsv_plan *plan, int index, void *buf, size_t cap, size_t *size);
/* Host-only: the HIP source of the kernel of op `index` (an LDS pass): the
 * variant compiled when the plan was built with opts->jit, else the one it
 * would compile to first; NUL-terminated, into buf (cap bytes); *size
 * receives the length including the NUL. */
int qsv_plan_op_source(const qsv_plan *plan, int index, char *buf, size_t cap, size_t *size);
/* Host-only: the circuit indices (positions in the gate array given to
 * qsv_plan_create) of the gates op `index` applies, in the order it applies
 * them, into ids (cap entries); *count receives their number (ids may be
 * NULL to query it).  A pass planner may move a gate ahead of earlier gates
 * it commutes with, so the concatenation over all ops is a reordering of the
 * circuit.  Uncontrolled SWAP gates that the pass planner absorbs as qubit
 * relabellings, and the permutation that undoes them at the end, are listed
 * by no op. */
int qsv_plan_op_gates(const qsv_plan *plan, int index, int *ids, size_t cap, size_t *count);
void qsv_plan_destroy(qsv_plan *plan);

/* Dense fused block on FP32 matrix cores (complex64 only): Y = G X with X
 * the state viewed as 2^k x 2^(n-k) (rows = target bits); the gate fusion
 * of Sec. 3.2 widened to k qubits.  `gate` is host complex64, 4^k entries
 * (row-major, targets[0] = the index MSB); 4 <= k <= 6, no controls,
 * n >= k + 5, state 16-byte aligned.  k = 4 runs as one real 2D x 2D
 * product, k = 5, 6 as three real D x D products (Yr = Gr Xr - Gi Xi,
 * Yi = (Gr + Gi)(Xr + Xi) - Gr Xr - Gi Xi), FP32 accumulation.  Errors:
 * QSV_ERR_UNSUPPORTED for complex128, QSV_ERR_ARITY for k or n out of range,
 * QSV_ERR_ALIGN, QSV_ERR_NULL; the state is untouched on error. */
int qsv_apply_block(void *state, int n, int dtype, const void *gate, const int *targets, int k, void *stream);

/* One LDS pass: every gate of `gates` is applied, in order, in a single HBM
 * read + write.  `local_qubits` (nlocal of them, nlocal <= 13 for complex64,
 * <= 12 for complex128, and containing qubits 0..2) are the chunk's qubits;
 * every non-diagonal target must be local; controls and diagonal gates may
 * be anywhere; SWAPs of two local qubits are permutations of the chunk. */
int qsv_run_pass(void *state, int n, int dtype, const qsv_gate *gates, int ngates,
                 const int *local_qubits, int nlocal, void *stream);

/* ------------------------------------------------------------------ states larger than device memory
 * The paper's multi-device scheme on one re-used GPU: the state stays in host
 * memory (2^n amplitudes of the dtype; pinned memory lets the copies overlap
 * the kernels) and slices of 2^local_qubits amplitudes visit the device.  The
 * qubits at or above local_qubits are global.  The circuit is cut into
 * phases in which every non-diagonal target is local or one of at most
 * active_qubits global qubits; each phase runs group by group, a group being
 * the 2^(active) slices that differ only in the phase's active qubits, copied
 * into a device buffer where controls and diagonal gates on the other global
 * qubits are resolved from the group's values.  Each group runs a plan of
 * `mode` QSV_PLAN_PER_GATE or QSV_PLAN_PASSES over local_qubits + active
 * qubits.  The library allocates two device buffers of
 * 2^(local_qubits + active_qubits) amplitudes and two copy streams for the
 * call and frees them before returning; the call returns when the host state
 * holds the result (kernels run on `stream`).  Errors: a gate with more
 * global non-diagonal targets than active_qubits is QSV_ERR_ARG;
 * 1 <= local_qubits <= n, 0 <= active_qubits <= min(8, n - local_qubits). */
int qsv_sliced_run(void *host_state, int n, int dtype, const qsv_gate *gates, int ngates, int local_qubits,
                   int active_qubits, int mode, void *stream);

/* ------------------------------------------------------------------ reductions
 * Products are formed in the state's precision and accumulated in float64
 * with a fixed-order tree, so results are reproducible run to run.  Outputs
 * are device pointers. */

/* Measurement probabilities of r qubits (methodology section: measurement):
 * out[m] = sum of |psi_i|^2 over i whose measured bits spell m, with
 * m = sum_j bit(i, qubits[j]) 2^(r-1-j).  out_dev holds 2^r doubles and must
 * not overlap the state (QSV_ERR_ARG).
 * 1 <= r <= n. */
int qsv_probabilities(const void *state, int n, int dtype, const int *qubits, int r,
                      double *out_dev, void *stream);
/* qsv_probabilities for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * kernels and result, bit for bit, but the partial sums live in a fixed
 * 2 MiB device array of the library (one per GPU, kept until the process
 * ends) instead of the staging ring, so the call allocates nothing -- not
 * even on its first use.  Every call on a GPU shares that array: calls that
 * overlap on one GPU (different streams, or different host threads) race
 * and must be serialised by the caller.  Arguments, limits and errors as for
 * qsv_probabilities (the decomposition never needs more than the array). */
int qsv_probabilities_noalloc(const void *state, int n, int dtype, const int *qubits, int r,
                              double *out_dev, void *stream);
/* out_dev[0] = <psi|psi>. */
int qsv_norm2(const void *state, int n, int dtype, double *out_dev, void *stream);
/* out_dev[0..1] = re, im of <a|b> = sum conj(a_i) b_i. */
int qsv_inner(const void *a, const void *b, int n, int dtype, double *out_dev, void *stream);
/* out_dev[0] = <psi| J sum_i Z_i Z_{i+1} + h sum_i X_i |psi> (open chain,
 * or periodic when `periodic` != 0 and n > 2). */
int qsv_expval_zz_x(const void *state, int n, int dtype, double J, double h, int periodic,
                    double *out_dev, void *stream);
/* out = (J sum Z_i Z_{i+1} + h sum X_i) psi, out a separate device state
 * (QSV_ERR_ARG when the two ranges overlap). */
int qsv_apply_tfim(const void *state, void *out, int n, int dtype, double J, double h,
                   int periodic, void *stream);

/* ------------------------------------------------------------------ measurement
 * The methodology section (Sec. 2) provides, besides the measurement
 * probabilities, an operator that collapses a state onto a measured outcome
 * and re-normalises it, and shot frequencies sampled with the Metropolis
 * algorithm.  Outcome indices follow qsv_probabilities (qubits[0] = most
 * significant bit).  Random numbers are inputs: the same inputs give the
 * same samples. */

/* Collapse onto outcome m of the r measured qubits, in place:
 * psi_i <- psi_i / sqrt(p) where the measured bits of i spell m, 0 elsewhere,
 * with p = ||P_m psi||^2 summed in float64 in a fixed order.  When p = 0 every
 * amplitude becomes 0.  prob_dev (device, may be NULL) receives p; it must
 * not lie inside the state (QSV_ERR_ARG).
 * 1 <= r <= n, m < 2^r (else QSV_ERR_ARG). */
int qsv_collapse(void *state, int n, int dtype, const int *qubits, int r, uint64_t outcome,
                 double *prob_dev, void *stream);

/* Inverse-CDF shot sampling from R = 2^r outcome probabilities (device
 * float64, need not sum to 1).  cdf_dev (device, R doubles, caller-owned)
 * receives c_m = p_0 + ... + p_m, summed in a fixed order; shot s with
 * uniform u_s in [0, 1) (uniforms_dev, nshots doubles) is the smallest m
 * with u_s c_{R-1} < c_m (the last outcome of non-zero probability if none);
 * an outcome of probability 0 is never drawn.  samples_dev (nshots int64) and
 * counts_dev (R uint64, zeroed by the call, then the frequency of each
 * outcome) are optional outputs; either may be NULL.  1 <= r <= 40. */
int qsv_sample_cdf(const double *probs_dev, int r, const double *uniforms_dev, int64_t nshots,
                   double *cdf_dev, int64_t *samples_dev, uint64_t *counts_dev, void *stream);

/* Metropolis shot frequencies (Metropolis et al. 1953): nchains independent
 * chains.  Chain c starts at outcome starts_dev[c]; at step s it proposes
 * y = proposals_dev[s * nchains + c] and moves there when
 * uniforms_dev[s * nchains + c] * p(x) < p(y), x the outcome it holds
 * (acceptance min(1, p(y)/p(x)) for a symmetric proposal); after every step
 * it counts x.  counts_dev (R uint64) is zeroed by the call and receives
 * the frequencies (nchains * steps in all).  All arrays are device memory.
 * Proposals outside [0, R) are rejected and starts outside it begin at 0. */
int qsv_sample_metropolis(const double *probs_dev, int r, const int64_t *starts_dev,
                          const int64_t *proposals_dev, const double *uniforms_dev, int nchains,
                          int64_t steps, uint64_t *counts_dev, void *stream);

/* ------------------------------------------------------------------ density matrices
 * The methodology section applies Eq. 1 to density matrices as well.  rho of
 * n qubits (1 <= n <= 20) is a device array of 2^(2n) complex numbers,
 * row-major: rho[r, c] at index r * 2^n + c, i.e. a 2n-qubit vector whose
 * column qubit q is bit q and whose row qubit q is bit q + n. */

/* A plan that applies every gate of the circuit as rho -> G rho G^dagger:
 * G on the row bits (targets and controls + n) and conj(G) on the column
 * bits.  The result is a plan over 2n qubits with twice the gates (row copy
 * then column copy of each gate, in circuit order), built and run exactly
 * as qsv_plan_create / qsv_plan_execute build and run a 2n-qubit circuit;
 * gate indices reported by the plan refer to that doubled circuit.  Gates
 * are validated on n qubits. */
int qsv_dm_plan_create(int n, int dtype, const qsv_gate *gates, int ngates, const qsv_plan_options *opts,
                       qsv_plan **out);
/* A one-qubit channel rho -> sum_k K_k rho K_k^dagger on qubit `target`:
 * `kraus` holds nk (1..16) host 2x2 complex128 matrices, row-major, one after
 * another.  Applied in place as the 4x4 superoperator on the (row, column)
 * bits of the qubit.  Trace preservation is the caller's choice (sum K^dag K
 * = I); it is not checked. */
int qsv_dm_apply_channel(void *rho, int n, int dtype, const double *kraus, int nk, int target, void *stream);
/* out_dev[0..1] = re, im of the trace, float64, fixed order. */
int qsv_dm_trace(const void *rho, int n, int dtype, double *out_dev, void *stream);
/* Measurement probabilities from the diagonal: out_dev[m] = sum of
 * Re rho[i, i] over i whose measured bits spell m (qubits[0] = most
 * significant bit of m), float64, 2^r entries, 1 <= r <= n. */
int qsv_dm_probabilities(const void *rho, int n, int dtype, const int *qubits, int r, double *out_dev,
                         void *stream);

/* ------------------------------------------------------------------ adjoint
 * Adjoint-method gradient of E = <psi|H|psi> (Jones and Gacon,
 * arXiv:2009.02823).  On entry psi holds U_L..U_1 psi_0 and lam holds H psi.
 * Walking the gates backwards, for every rotation RX/RY/RZ (exp(-i theta P/2))
 * the call computes Im <lam|P|psi> and then applies U^dagger to both vectors;
 * on return psi holds psi_0 (up to rounding).  grad_dev receives one double
 * per rotation, in circuit order.  The gates must be the ones that produced
 * psi; psi and lam are separate states (QSV_ERR_ARG when they overlap). */
int qsv_adjoint_grad(void *psi, void *lam, int n, int dtype, const qsv_gate *gates, int ngates,
                     double *grad_dev, void *stream);

/* ------------------------------------------------------------------ MLP
 * Fully connected network with ReLU hidden layers and a linear scalar
 * output, FP32, on caller-owned device buffers.  Layer l has weights
 * W_l [fan_in, fan_out] row-major and bias b_l [fan_out]; `params` is all
 * layers concatenated (W_1, b_1, W_2, b_2, ...); `sizes` has nlayers + 1
 * entries (input width first, 1 last); every width <= 256.
 *   forward:  X [batch, sizes[0]] -> acts (sum of batch * sizes[1..] floats,
 *             layer outputs after activation), pred [batch]
 *   backward: gradient of mean((pred - target)^2) into grads (same layout as
 *             params); `scratch` holds 2 * batch * max width floats
 *   adam:     params -= lr * mhat / (sqrt(vhat) + eps), Adam step t >= 1 */
int qsv_mlp_forward(const float *params, const int *sizes, int nlayers, const float *X, int batch,
                    float *acts, float *pred, void *stream);
int qsv_mlp_backward(const float *params, const int *sizes, int nlayers, const float *X, int batch,
                     const float *acts, const float *pred, const float *target,
                     float *grads, float *scratch, void *stream);
int qsv_mlp_adam(float *params, const float *grads, float *m, float *v, int count, int t,
                 float lr, float beta1, float beta2, float eps, void *stream);
/* Number of floats of params for `sizes`. */
int qsv_mlp_param_count(const int *sizes, int nlayers);

/* Cost model used by QSV_PLAN_LEARNED: a copy of the parameters (host FP32,
 * layout as above, sizes[0] == QSV_COST_FEATURES) and the feature
 * normalisation (x - mean) / scale per input.  The network predicts the
 * natural log of an op's run time in seconds.  Passing nlayers = 0 removes
 * the model.  The model is process-wide; the call copies everything. */
int qsv_cost_model_set(const float *params, const int *sizes, int nlayers,
                       const float *feat_mean, const float *feat_scale);
/* Host-only: the raw feature vector (QSV_COST_FEATURES floats) of op `index`
 * of a plan -- n, dtype, one-hot variant (single-gate kernel, fused block on
 * the VALU kernels, MFMA block, interpreted LDS pass, bit permutation,
 * compiled LDS pass -- a pass counts as compiled when the plan was created
 * with opts->jit), number of qubits, number of qubits below 5, log2 bytes,
 * log2 flops, and an op-specific size (log2 touched members, or ops in a
 * pass program). */
#define QSV_COST_FEATURES 13
int qsv_plan_op_features(const qsv_plan *plan, int index, float *out);

#ifdef __cplusplus
}
#endif
#endif /* QSV_H */
