// kernels.h - host-side launchers of the device kernels (sweep.hip, reduce.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "plan.h"

namespace qd {

enum Precision { kC64 = 1, kC128 = 2 };

inline size_t amp_bytes(int precision) { return precision == kC128 ? 16 : 8; }

// Which kernel family a plan takes.
enum Family { kFamIdentity = 0, kFamDenseReg = 1, kFamDenseLds = 2, kFamMonomial = 3, kFamMfma = 4 };
int plan_family(const GatePlan& p, int precision);
const char* family_name(int family);

// Matrix-core path (mfma.hip): dense gates with 17 <= M <= mfma_max_m(precision)
// (128: complex64 on FP32 MFMA, complex128 on FP64 MFMA).
constexpr int kMfmaMinM = 17;
int mfma_max_m(int precision);
int mfma_padded(int M);
size_t mfma_gate_bytes(int M, bool narrow, int precision);
void fill_mfma_gate(const GatePlan& p, int precision, const double* U, void* dst);
hipError_t launch_mfma(const GatePlan& p, int precision, void* psi, const void* dgate, hipStream_t stream);

// Bytes of device-side gate data (rounded U, member offsets) a plan needs, 0 if
// everything travels in the kernel arguments.
size_t device_gate_bytes(const GatePlan& p, int precision);
// Fill `dst` (host staging memory, device_gate_bytes long) with that data.
void fill_device_gate(const GatePlan& p, int precision, const double* U, void* dst);

// Enqueue the gate on `stream`. dgate: device copy of fill_device_gate's output
// (ignored when device_gate_bytes is 0). Returns hipSuccess or the launch error.
hipError_t launch_gate(const GatePlan& p, int precision, void* psi, const double* U, const void* dgate,
                       hipStream_t stream);

// A fused pass (fused.h, fused.hip). The device blob holds the TileGate array
// at gates_off, the rounded gate data the descriptors point into, and the run
// offsets (32-bit when D < 2^31, else 64-bit) at run_off_off.
struct FusedLaunch {
    uint64_t D;
    uint64_t n_tiles;
    int outer_nseg;
    uint64_t outer_size[kMaxSeg];
    uint64_t outer_stride[kMaxSeg];
    uint32_t tile;
    uint32_t L;
    int ngates;
    size_t gates_off;
    size_t run_off_off;
};
hipError_t launch_fused(const FusedLaunch& f, int precision, void* psi, const void* dblob, hipStream_t stream);

// A batched round (fused.h BatchItem): ditems/dblob are device copies; nblocks =
// total tiles over all items; max_tile = largest tile (LDS per workgroup).
hipError_t launch_batch(int precision, const void* ditems, int nitems, uint32_t nblocks, uint32_t max_tile,
                        const void* dblob, hipStream_t stream);

// Reductions and fills (reduce.hip).
constexpr int kRedBlocks = 1024;
constexpr int kRedScratch = kRedBlocks + 1;  // doubles of partial sums one reduction uses
// Sum of squares into scratch[kRedBlocks] (scratch: kRedScratch doubles) and its
// square root into *norm (device-accessible).
hipError_t launch_sumsq(const void* psi, int precision, uint64_t D, double* scratch, double* norm,
                        hipStream_t stream);
hipError_t launch_probabilities(const void* psi, int precision, uint64_t offset, uint64_t count,
                                double* out, hipStream_t stream);
hipError_t launch_basis(void* psi, int precision, uint64_t D, uint64_t j, hipStream_t stream);
hipError_t launch_stream_rewrite(void* psi, int precision, uint64_t D, hipStream_t stream);

}  // namespace qd
