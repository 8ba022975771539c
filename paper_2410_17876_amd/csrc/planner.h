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
// The target and control checks of check_gate for a register whose dims are
// already valid (dense or sparse).
int check_gate_shape(const int32_t* dims, int32_t n, const int32_t* targets, int32_t k, const int32_t* controls,
                     const int32_t* values, int32_t m, std::string* err);

// Key words of a sparse register (sparse.h): qudits packed from q_0 upward into
// words whose dims multiply to less than 2^64. word[i] / stride[i]: the word of
// qudit i and its stride inside that word; P[w]: product of word w's dims
// (1 for unused words); *W: words used. Checks the dims (n <= 126, each 2..7)
// and D = prod dims < 2^127 (QD_ERR_DIM_OVERFLOW), returned as (D_lo, D_hi).
// Any output pointer may be null.
constexpr int kSparseKeyWords = 3;
int sparse_layout(const int32_t* dims, int32_t n, int* word, uint64_t* stride, int* W, uint64_t* P, uint64_t* D_lo,
                  uint64_t* D_hi, std::string* err);
// Optional unitarity check of gate matrices (QD_CHECK_UNITARY in the environment).
constexpr double kUnitaryTol = 1e-10;
bool unitary_check_enabled();
double unitary_deviation(const double* U, int M);
int plan_gate(const int32_t* dims, int32_t n, const int32_t* targets, int32_t k, const int32_t* controls,
              const int32_t* values, int32_t m, const double* U, GatePlan* p, std::string* err);
void plan_info(const GatePlan& p, int precision, qd_gate_info* info);

}  // namespace qd
