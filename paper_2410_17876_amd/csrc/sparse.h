// sparse.h - block simulation on a sparse statevector (sparse.hip).
//
// The paper's sparse variant (Sec. 3: GHZ states of up to 62 qubits) keeps only
// the nonzero amplitudes, in a hash map from basis index to amplitude. Here they
// are device arrays of (basis index, amplitude) pairs sorted by index, in
// complex128: a gate groups the entries by class with a radix sort on the class
// base, applies U to each class present, and keeps the nonzero results.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qd.h"

namespace qd {

constexpr int kSparseMaxM = 16;  // class size of a sparse gate

// A gate as the sparse kernels see it (all strides in the full register).
struct SparseGate {
    int k;                            // targets, first one least significant in the local index
    uint64_t ts[QD_MAX_TARGETS];      // target strides
    uint32_t td[QD_MAX_TARGETS];      // target dims
    int m;                            // controls
    uint64_t cs[QD_MAX_CONTROLS];     // control strides
    uint32_t cd[QD_MAX_CONTROLS];     // control dims
    uint32_t cv[QD_MAX_CONTROLS];     // control values
    int M;                            // class size
    uint64_t off[kSparseMaxM];        // member offsets: off[a] = sum_l a_l ts[l]
};

// Device arrays of a sparse state; nnz entries, keys strictly increasing. The
// entries live in one of two slots (the other receives the next gate's result),
// and a gate's temporaries in a workspace; all three only grow, so a gate
// allocates nothing once the state has reached its size.
struct SparseData {
    uint64_t nnz = 0;
    uint64_t* keys = nullptr;
    double2* amps = nullptr;
    void* slot[2] = {nullptr, nullptr};
    size_t slot_bytes[2] = {0, 0};
    int cur = 0;              // slot holding keys/amps
    void* work = nullptr;
    size_t work_bytes = 0;
};

// Replace `d`'s entries by the result of applying g (U: M x M complex,
// row-major [out][in], interleaved FP64) on the null stream; synchronous. On an
// error the entries are unchanged.
hipError_t sparse_apply(SparseData& d, const SparseGate& g, const double* U);

// Set `d` to the single entry |0...0> with amplitude 1; frees everything with release.
hipError_t sparse_init(SparseData& d);
void sparse_release(SparseData& d);

}  // namespace qd
