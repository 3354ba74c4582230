// Internal declarations shared by the libqsv sources (host + device).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/qsv.h"

namespace qsv {

// ---------------------------------------------------------------- errors

void set_error(const std::string &msg);
void clear_error();
int fail(int code, const std::string &msg);
int hip_fail(hipError_t e, const char *where);

// Device memory the library allocates for itself (the staging ring and
// per-call temporaries) goes through these, which keep the current and peak
// byte counts that qsv_memory_stats reports.
hipError_t dev_malloc(void **p, size_t bytes);
hipError_t dev_malloc_async(void **p, size_t bytes, hipStream_t s);
hipError_t dev_free(void *p);
hipError_t dev_free_async(void *p, hipStream_t s);

// Whether the byte ranges [a, a + na) and [b, b + nb) share a byte (an output
// that a kernel writes while it still reads an input must not).
inline bool ranges_overlap(const void *a, uint64_t na, const void *b, uint64_t nb) {
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + nb && y < x + na;
}

#define QSV_HIP_CHECK(expr)                                   \
    do {                                                      \
        hipError_t e_ = (expr);                               \
        if (e_ != hipSuccess) return ::qsv::hip_fail(e_, #expr); \
    } while (0)

// ---------------------------------------------------------------- complex types

template <typename R> struct cplx_of;
template <> struct cplx_of<float> { typedef float2 type; };
template <> struct cplx_of<double> { typedef double2 type; };

template <typename C> __host__ __device__ inline C cmul(C a, C b) {
    C r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}
template <typename C> __host__ __device__ inline C cfma(C a, C b, C acc) {
    // acc + a * b
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(-a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(a.y, b.x, acc.y);
    return acc;
}

// ---------------------------------------------------------------- index bits

// Insert a zero bit at each position of `lowmask_i` = (1 << b_i) - 1 for the
// ascending sorted positions b_i: the smallest member index of group g.
__host__ __device__ inline uint64_t insert_zero_bits(uint64_t g, const uint64_t *lowmasks, int m) {
    for (int i = 0; i < m; ++i) {
        const uint64_t lo = g & lowmasks[i];
        g = lo | ((g ^ lo) << 1);
    }
    return g;
}

// ---------------------------------------------------------------- gate analysis

enum GateClass { GC_DIAG = 0, GC_PERM = 1, GC_DENSE = 2 };

// A gate reduced to the members it changes.  Amplitude indices of one group
// are base + off[j]; base has 0 at every target/control bit then OR cmask.
struct GateAnalysis {
    int n = 0;
    int k = 0;
    int cls = GC_DENSE;
    std::vector<int> sorted_bits;   // targets + controls, ascending
    uint64_t cmask = 0;             // controls
    std::vector<int> members;       // touched tau values (row/col index of G)
    std::vector<uint64_t> offs;     // member offsets, same order as members
    // DIAG: factor per member; PERM: source member slot + factor + is_one;
    // DENSE: M x M submatrix over `members` (row-major).
    std::vector<double> mat;        // complex128 interleaved
    std::vector<int> perm_src;      // PERM: index into members of the source
    std::vector<int> perm_one;      // PERM: factor exactly 1 (pure move)
    double touched_fraction() const;
};

// Build the analysis from a complex128 target block (4^k entries, row-major).
GateAnalysis analyse_gate(int n, const double *G, const int *targets, int k, const int *controls, int c);

// Fill the complex128 target block of a gate description (4^k entries).
int gate_target_matrix(const qsv_gate &g, std::vector<double> &out);

int validate_common(int n, int dtype, const int *targets, int k, const int *controls, int c);

// ---------------------------------------------------------------- device staging

// Per-device staging: a pinned host ring mirrored by a device ring, carved
// into 256 KiB slots.  A slot carries a HIP event recorded after the last
// launch that reads it; the slot is reused only after that event completed.
// A request of up to 2 MiB takes consecutive slots.
struct StagingSlot {
    void *host = nullptr;
    void *dev = nullptr;
    size_t bytes = 0;
    int index = -1;   // first slot (device * slots + slot)
    int span = 1;     // consecutive slots held
};

int staging_acquire(size_t bytes, StagingSlot *slot);          // blocks until free
int staging_upload(const StagingSlot &slot, size_t bytes, hipStream_t s);
int staging_release(const StagingSlot &slot, hipStream_t s);   // records the event
size_t staging_slot_bytes();

// ---------------------------------------------------------------- launchers

int launch_gate(void *state, int dtype, const GateAnalysis &a, hipStream_t s);
int launch_scale(void *state, int n, int dtype, double re, double im, hipStream_t s);
int launch_block_mfma(void *state, int n, const double *G, const int *targets, int k, hipStream_t s);
int launch_block_valu(void *state, int n, int dtype, const double *G, const int *targets, int k, hipStream_t s);

struct PassProgram;   // pass_kernel.hip
int launch_pass(void *state, int n, int dtype, const qsv_gate *gates, int ngates,
                const int *local_qubits, int nlocal, hipStream_t s);

int device_sm_count();

}  // namespace qsv
