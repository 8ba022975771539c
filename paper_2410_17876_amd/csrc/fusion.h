// fusion.h - host-side planning of gate lists into HBM passes (fusion.cpp).
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include "fused.h"
#include "kernels.h"
#include "planner.h"

namespace qd {

struct CircuitGate {
    const int32_t* targets;
    int k;
    const int32_t* controls;
    const int32_t* values;
    int m;
    const double* U;
};

struct CircuitOptions {
    bool fuse = true;
    uint64_t tile_max = 3072;       // amplitudes per tile
    uint64_t min_run = 64;          // minimum contiguous run inside a tile
    bool single_as_fused = false;   // run a one-gate pass as a tile pass too (batched rounds)
    int reorder = 0;                // look-ahead for commuting gates (0: strictly in order)
};

struct PassPlan {
    bool fused = false;
    std::vector<int> gates;           // indices into the gate list, in order
    FusedLaunch launch;               // fused passes
    std::vector<unsigned char> blob;  // fused passes: device data, built for one precision
};

// Add `delta` to every offset a fused pass's device data holds (descriptor fields
// and register-block records). The offsets count from blob + frame before the
// call (so the records sit at blob + frame + offset), e.g. the pass's own blob
// (frame 0) copied `delta` bytes into a larger buffer.
void rebase_pass_blob(unsigned char* blob, const FusedLaunch& f, uint32_t frame, uint32_t delta);

int plan_circuit(const int32_t* dims, int n, int precision, const CircuitGate* gates, int count,
                 const CircuitOptions& opt, std::vector<PassPlan>& out, std::string* err);

}  // namespace qd
