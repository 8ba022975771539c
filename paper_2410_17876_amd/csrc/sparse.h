// sparse.h - block simulation on a sparse statevector (sparse.hip).
//
// The paper's sparse variant (Sec. 3: GHZ states of up to 62 qubits) keeps only
// the nonzero amplitudes, in a hash map from basis index to amplitude, and is
// capped by a signed 64-bit index; wider integer keys are the way past that
// limit (Sec. 4). Here the entries are device arrays of (basis index,
// amplitude) pairs sorted by index, in complex128, and a basis index is a key
// of up to three 64-bit words, so registers up to D < 2^127 are covered.
//
// Key layout: the qudits are packed from q_0 upward into W words, each word
// taking qudits while the product of their dims stays below 2^64. A word holds
// the mixed-radix index over its own qudits in the same digit order as the full
// index, so a digit is read inside one word with 64-bit arithmetic and never
// carries into another word. The basis index is w_0 + P_0 (w_1 + P_1 w_2), P_w
// the product of word w's dims; comparing keys word by word from the top word
// down orders them like the basis index. Keys are stored word-major (W arrays).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "plan.h"
#include "qd.h"

namespace qd {

constexpr int kSparseMaxM = 16;  // class size of a sparse gate
constexpr int kKeyWords = 3;     // a basis index below 2^127 fits three mixed-radix words

// Outputs of one gate (entries x class size) handled by the one-workgroup
// kernel, which needs no host synchronisation; larger gates take the
// multi-kernel path with a radix sort.
constexpr uint32_t kSparseSmallCap = 1024;

// Matrices of at most this many rows travel inside the kernel arguments of the
// one-workgroup form (no staging, no read of host memory).
constexpr int kSparseInlineM = 8;

// A gate as the sparse kernels see it: every target and control as (word,
// stride inside the word, dim).
struct SparseGate {
    int W;                                // key words of the register
    int k;                                // targets, first one least significant in the local index
    int tw[QD_MAX_TARGETS];
    uint64_t ts[QD_MAX_TARGETS];
    uint32_t td[QD_MAX_TARGETS];
    int m;                                // controls
    int cw[QD_MAX_CONTROLS];
    uint64_t cs[QD_MAX_CONTROLS];
    uint32_t cd[QD_MAX_CONTROLS];
    uint32_t cv[QD_MAX_CONTROLS];
    int M;                                // class size
    // digit of a target / control: (word / stride) mod dim, both divisions by
    // multiply-high (64-bit divisions are long instruction sequences on the GPU)
    FastDiv<uint64_t> tsd[QD_MAX_TARGETS], tdd[QD_MAX_TARGETS];
    FastDiv<uint64_t> csd[QD_MAX_CONTROLS], cdd[QD_MAX_CONTROLS];
    uint64_t off[kSparseMaxM][kKeyWords]; // member a sits at class base + off[a] (word by word)
    const double2* U;                     // M x M row-major [out][in], device-readable; null: Uin holds it
    double2 Uin[kSparseInlineM * kSparseInlineM];  // U itself when M <= kSparseInlineM (one-workgroup form)
};

// Device state of a sparse register. Entries live in one of two slots (the
// other receives the next gate's result), each holding W key arrays and the
// amplitudes for `slot_cap` entries; the entry counts of both slots stay on
// the device (nnz_dev), so a gate on the one-workgroup path is enqueued
// without reading anything back. The host keeps an upper bound on the count.
struct SparseData {
    int W = 1;
    hipStream_t stream = nullptr;
    void* slot[2] = {nullptr, nullptr};
    uint64_t slot_cap[2] = {0, 0};
    int cur = 0;
    uint64_t* nnz_dev = nullptr;  // [2]: entries in slot 0 / slot 1
    uint64_t bound = 0;           // nnz <= bound
    bool exact = false;           // bound == nnz
    void* work = nullptr;         // temporaries of the multi-kernel path (grow-only)
    size_t work_bytes = 0;
    // Gate matrices staged in pinned host memory that the kernels read
    // directly (a ring: slot i is reused once the event recorded after its
    // gate has completed).
    static constexpr int kURing = 64;
    double2* uhost = nullptr;
    double2* udev = nullptr;      // the same memory as the device addresses it
    hipEvent_t uev[kURing] = {};
    uint64_t uses = 0;
    // Runs of one-workgroup gates applied by one launch (sparse_apply_list):
    // their SparseGate records are staged in pinned host memory and copied to a
    // device buffer; the staging is reused once the event after its copy has passed.
    SparseGate* rhost = nullptr;
    size_t rhost_gates = 0;
    void* rdev = nullptr;
    size_t rdev_bytes = 0;
    hipEvent_t rev = nullptr;
    bool rev_pending = false;
};

// Entry pointers of a slot with capacity cap: W key arrays, then amplitudes.
inline uint64_t* slot_keys(void* slot) { return static_cast<uint64_t*>(slot); }
inline double2* slot_amps(void* slot, int W, uint64_t cap) {
    const size_t kb = ((size_t)W * cap * 8 + 255) & ~(size_t)255;
    return reinterpret_cast<double2*>(static_cast<unsigned char*>(slot) + kb);
}
inline size_t slot_bytes(int W, uint64_t cap) { return (((size_t)W * cap * 8 + 255) & ~(size_t)255) + cap * 16; }

// |0...0> with amplitude 1 on the state's stream (allocates the slots, the
// counters and the staging ring).
hipError_t sparse_init(SparseData& d, int W);
void sparse_release(SparseData& d);

// Enqueue one gate on d.stream (U: M x M complex, row-major [out][in],
// interleaved FP64, copied before returning). `cols_single`: every column of
// U has at most one nonzero, so the gate cannot raise the entry count. On an
// error nothing is changed.
hipError_t sparse_apply(SparseData& d, const SparseGate& g, const double* U, bool cols_single);

// Enqueue a gate list in order, as sparse_apply gate by gate (the same bits).
// While the host's bound keeps consecutive gates within the one-workgroup form
// (and their matrices fit the kernel arguments), such a run of gates is applied
// by one launch that keeps the entries in LDS from gate to gate. On an error the
// gates before the failing one may have been applied.
hipError_t sparse_apply_list(SparseData& d, const SparseGate* gates, const double* const* U, const bool* cols_single,
                             int count);

// Wait for the stream and return the entry count.
hipError_t sparse_count(SparseData& d, uint64_t* nnz);

}  // namespace qd
