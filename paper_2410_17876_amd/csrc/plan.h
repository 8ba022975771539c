// plan.h - gate plans: what the host planner hands to the kernels.
//
// A gate on targets T with controls C (values v) visits only the amplitudes
// whose control digits hold v (paper Sec. 2.4) and groups them into classes that
// differ only in the target digits (Sec. 2.3, Table 2). The free qudits (neither
// target nor control) form maximal runs of consecutive positions, "segments".
// Segment g covers qudits [p_g, p_g + len) and has size G_g = prod of their dims
// and stride S_g = s_{p_g} (the block size of its lowest qudit, Sec. 2.3).
// Enumerating classes by a flat class id c, with segment 0 the least
// significant, gives
//
//   base(c) = sum_c v_c s_c + sum_g digit_g(c) * S_g,
//   digit_g(c) = floor(c / (G_0 ... G_{g-1})) mod G_g,
//
// and class member a lives at base(c) + off[a], off[a] = sum_l a_l s_{t_l}
// (first target least significant). This replaces the paper's scan of every
// index against every control (Sec. 2.4): the digits are independent, so the
// solutions of its congruence system are exactly this product set.
//
// The divisions by G_g use multiply-high by a precomputed reciprocal (Granlund &
// Montgomery, "Division by invariant integers using multiplication", PLDI 1994):
// with l = ceil(log2 G) and m = floor(2^N (2^l - G) / G) + 1,
//   q = (t + ((n - t) >> min(l,1))) >> max(l-1,0),  t = mulhi_N(m, n),
// exact for every N-bit n. There is no division per amplitude anywhere.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qd {

constexpr int kMaxSeg = 28;      // free-qudit runs: <= #specials + 1 <= 3 + 24 + 1
constexpr int kMaxM = 343;       // 3 targets of dim 7
constexpr int kRegMaxM = 16;     // class sizes handled fully in registers
constexpr int kInlineMaxM = 8;   // gate matrices passed by value in the kernel arguments

template <typename I>
struct FastDiv {
    I m;
    uint32_t sh1, sh2;
};

template <typename I>
__host__ __device__ inline I mulhi(I a, I b);

template <>
__host__ __device__ inline uint32_t mulhi<uint32_t>(uint32_t a, uint32_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __umulhi(a, b);
#else
    return (uint32_t)(((uint64_t)a * b) >> 32);
#endif
}

template <>
__host__ __device__ inline uint64_t mulhi<uint64_t>(uint64_t a, uint64_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __umul64hi(a, b);
#else
    return (uint64_t)(((unsigned __int128)a * b) >> 64);
#endif
}

template <typename I>
__host__ __device__ inline I fast_div(I n, const FastDiv<I>& d) {
    I t = mulhi<I>(n, d.m);
    return (t + ((n - t) >> d.sh1)) >> d.sh2;
}

template <typename I>
inline FastDiv<I> make_fast_div(uint64_t G) {
    constexpr int N = 8 * sizeof(I);
    uint32_t l = 0;
    while (l < 64 && ((unsigned __int128)1 << l) < G) ++l;
    unsigned __int128 num = ((unsigned __int128)1 << N) * (((unsigned __int128)1 << l) - G);
    FastDiv<I> f;
    f.m = (I)(num / G + 1);
    f.sh1 = l < 1 ? l : 1;
    f.sh2 = l > 0 ? l - 1 : 0;
    return f;
}

// Class-id -> base decoder. Segment nseg-1 is the most significant and needs no
// division (c < n_classes bounds its digit).
template <typename I, int NS = kMaxSeg>
struct Decode {
    I n_classes;
    I ctrl_off;
    int32_t nseg;
    I size[NS];
    I stride[NS];
    FastDiv<I> div[NS];
};

// Decoders are read in place (kernel arguments, descriptors in global memory),
// where a uniform index is a scalar load, so the loop stays rolled: one class
// per thread in the sweeps, and an unrolled, guarded form of all kMaxSeg steps
// measured slower (complex64 one-qudit monomial sweep 3.3 -> 4.7 ms on the
// 1.72e9-amplitude register).
template <typename I, int NS>
__host__ __device__ inline I decode_base(const Decode<I, NS>& dec, I c) {
    I base = dec.ctrl_off;
    const int last = dec.nseg - 1;
    for (int g = 0; g < last; ++g) {
        const I q = fast_div<I>(c, dec.div[g]);
        base += (c - q * dec.size[g]) * dec.stride[g];
        c = q;
    }
    if (last >= 0) base += c * dec.stride[last];
    return base;
}

enum Category { kDense = 0, kMonomial = 1, kDiagonal = 2, kIdentity = 3 };

// Host-side plan of one gate (independent of the state's buffer).
struct GatePlan {
    int n;
    uint64_t D;
    int M;
    int category;
    uint64_t n_classes;
    uint64_t ctrl_off;
    int nseg;
    uint64_t seg_size[kMaxSeg];
    uint64_t seg_stride[kMaxSeg];
    int64_t off[kMaxM];  // member offsets, local index order
    // monomial / diagonal: the active entries (those not equal to an identity column)
    int n_active;
    int src[kMaxM];      // local index read
    int dst[kMaxM];      // local index written
    double lam[2 * kMaxM];
    uint8_t lam_one[kMaxM];
};

template <typename I, int NS = kMaxSeg>
inline Decode<I, NS> make_decode(const GatePlan& p) {
    Decode<I, NS> d;
    d.n_classes = (I)p.n_classes;
    d.ctrl_off = (I)p.ctrl_off;
    d.nseg = p.nseg;
    for (int g = 0; g < NS; ++g) {
        d.size[g] = g < p.nseg ? (I)p.seg_size[g] : (I)1;
        d.stride[g] = g < p.nseg ? (I)p.seg_stride[g] : (I)0;
        d.div[g] = make_fast_div<I>(g < p.nseg ? p.seg_size[g] : 1);
    }
    return d;
}

}  // namespace qd
