// device.h - device-side building blocks shared by the sweep and fused kernels.
//
// The per-class arithmetic lives here once, so that a gate applied by the
// one-pass sweep and the same gate applied inside a fused tile produce the same
// bits: y_r = sum_a U[r][a] x_a with the products accumulated in ascending a,
// as four real FMAs per complex term (paper Sec. 2.3: the new amplitudes of a
// class are the sum of U's columns scaled by the class's amplitudes).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qd {

template <typename R>
struct Cx {
    using T = R __attribute__((ext_vector_type(2)));
};

template <typename T>
__device__ __forceinline__ T ld_stream(const T* p) {
    return __builtin_nontemporal_load(p);
}
template <typename T>
__device__ __forceinline__ void st_stream(T* p, T v) {
    __builtin_nontemporal_store(v, p);
}

// Workgroup b runs on XCD b % 8 (round-robin dispatch). Renumber so that XCD x
// takes one contiguous range of logical blocks (a bijection on [0, gridDim.x)).
__device__ __forceinline__ uint32_t xcd_block() {
    const uint32_t G = gridDim.x, b = blockIdx.x, q = G >> 3, r = G & 7u, x = b & 7u;
    return x * q + (x < r ? x : r) + (b >> 3);
}

// sum_a w(a) x[a] for one class of M amplitudes, ascending a, four real FMAs
// per complex term. `w(a)` returns the a-th coefficient already rounded to the
// working precision.
template <typename R, int M, typename WGet>
__device__ __forceinline__ typename Cx<R>::T dense_dot(const typename Cx<R>::T* x, const WGet& w) {
    R yr = 0, yi = 0;
#pragma unroll
    for (int a = 0; a < M; ++a) {
        const typename Cx<R>::T c = w(a);
        yr = fma(c.x, x[a].x, yr);
        yr = fma(-c.y, x[a].y, yr);
        yi = fma(c.x, x[a].y, yi);
        yi = fma(c.y, x[a].x, yi);
    }
    typename Cx<R>::T y;
    y.x = yr;
    y.y = yi;
    return y;
}

// Row r of U x for one class of M amplitudes. `u(i)` returns U's i-th entry
// (row-major) already rounded to the working precision.
template <typename R, int M, typename UGet>
__device__ __forceinline__ typename Cx<R>::T dense_row(const typename Cx<R>::T* x, const UGet& u, int r) {
    return dense_dot<R, M>(x, [&](int a) { return u(r * M + a); });
}

// w * x for a monomial (phase / permutation) factor.
template <typename T>
__device__ __forceinline__ T scale_by(T w, T x) {
    T y;
    y.x = fma(w.x, x.x, -w.y * x.y);
    y.y = fma(w.x, x.y, w.y * x.x);
    return y;
}

}  // namespace qd
