// planner.h - host-side validation and planning (planner.cpp).
#pragma once

#include <stdarg.h>
#include <stdint.h>

#include <string>

#include "../../include/qd.h"
#include "kernels.h"
#include "plan.h"

namespace qd {

// Segments of the qudits not marked special (plan.h); false if there are more
// than kMaxSeg. n_free = product of their dims.
bool free_segments(const int32_t* dims, int n, const bool* special, int* nseg, uint64_t* size, uint64_t* stride,
                   uint64_t* n_free);
int check_dims(const int32_t* dims, int32_t n, uint64_t* D, std::string* err);
int check_gate(const int32_t* dims, int32_t n, const int32_t* targets, int32_t k, const int32_t* controls,
               const int32_t* values, int32_t m, std::string* err);
int plan_gate(const int32_t* dims, int32_t n, const int32_t* targets, int32_t k, const int32_t* controls,
              const int32_t* values, int32_t m, const double* U, GatePlan* p, std::string* err);
void plan_info(const GatePlan& p, int precision, qd_gate_info* info);

}  // namespace qd
