// fused.hip - one HBM pass for a run of consecutive gates (fused.h explains the
// tiling). One workgroup per tile: load the tile into LDS with non-temporal
// loads of contiguous runs, apply each gate of the pass to the tile's classes in
// order (the same per-class arithmetic as the one-gate sweeps, device.h), write
// the tile back. fused_tile serves a single state, batch_tile one tile of one
// (state, pass) item of a batched round.
//
// Several workgroups share a CU (two 64 KB complex64 tiles; three or four
// complex128 tiles of 36-48 KB), so one's loads and stores overlap the others'
// LDS work. Persistent variants measured slower and were dropped: one 512-thread
// workgroup per CU prefetching the next tile into registers (the LDS phase then
// has no other workgroup to hide its latency), and double-buffered workgroups
// loading the next tile straight into LDS (one or two tiles in flight per CU
// cannot keep HBM busy; the plain form's load phases have four).
#include <hip/hip_runtime.h>

#include "device.h"
#include "fused.h"
#include "kernels.h"

namespace qd {

__device__ __forceinline__ bool outer_holds(const TileGate* __restrict__ G, uint64_t base) {
    for (int l = 0; l < G->n_outer; ++l)
        if ((base / G->oc_stride[l]) % G->oc_dim[l] != G->oc_val[l]) return false;
    return true;
}

// Classes per thread per loop trip: independent class loads in flight, bounded
// by registers (x holds UF * M amplitudes).
template <int M>
constexpr int class_unroll() {
    return M <= 4 ? 4 : (M <= 8 ? 2 : 1);
}

// Class bases prefetched into registers: a thread's first kPre classes of a gate
// (classes threadIdx.x + j * BS). A gate's bases are loaded from its table while
// the previous gate (or the tile load) is still in flight, so the per-gate
// chain does not wait for them; the first 2 * UF classes of a thread come from
// here, the rest (only for gates with more classes per thread) are loaded in
// the class loop.
constexpr int kPre = 8;

template <int BS>
__device__ __forceinline__ void prefetch_bases(const TileGate* __restrict__ G, const unsigned char* blob,
                                               uint32_t (&pre)[kPre]) {
    const uint16_t* bases = reinterpret_cast<const uint16_t*>(blob + G->bases_off);
    const uint32_t nc = G->n_classes;
#pragma unroll
    for (int j = 0; j < kPre; ++j) {
        const uint32_t c = threadIdx.x + j * BS;
        pre[j] = bases[c < nc ? c : 0u];  // clamped: every load in bounds, none predicated
    }
}

// Dense update of UF classes (the same arithmetic as the one-gate sweep).
template <typename R, int M, int UF>
__device__ __forceinline__ void dense_classes(typename Cx<R>::T* tile, const TileGate* __restrict__ G,
                                              const typename Cx<R>::T* __restrict__ U, const uint32_t (&off)[M],
                                              const uint32_t (&base)[UF], const bool (&ok)[UF]) {
    using T = typename Cx<R>::T;
    // Loads are unconditional: a class past the end has a clamped, valid base
    // (for_classes), and only the stores below are predicated.
    T x[UF][M];
#pragma unroll
    for (int u = 0; u < UF; ++u)
#pragma unroll
        for (int a = 0; a < M; ++a) x[u][a] = tile[base[u] + off[a]];
    if constexpr (M <= 2) {
#pragma unroll
        for (int u = 0; u < UF; ++u) {
            if (!ok[u]) continue;
#pragma unroll
            for (int r = 0; r < M; ++r)
                tile[base[u] + off[r]] = dense_row<R, M>(x[u], [&](int i) { return U[i]; }, r);
        }
    } else {
        // Rolled over rows, one row of U live at a time: unrolled, the compiler
        // keeps all of U in scalar registers (4 M^2 of them in complex128), and
        // the pressure spills the pass's other uniform state on every gate.
        if constexpr (M <= 4) {
            // The next row's coefficients are loaded while this row is computed.
            T w[M];
#pragma unroll
            for (int a = 0; a < M; ++a) w[a] = U[a];
#pragma unroll 1
            for (int r = 0; r < M; ++r) {
                const uint32_t o = G->off[r];  // uniform: a scalar load
                T wn[M];
                const int rn = r + 1 < M ? r + 1 : r;
#pragma unroll
                for (int a = 0; a < M; ++a) wn[a] = U[rn * M + a];
#pragma unroll
                for (int u = 0; u < UF; ++u)
                    if (ok[u]) tile[base[u] + o] = dense_dot<R, M>(x[u], [&](int a) { return w[a]; });
#pragma unroll
                for (int a = 0; a < M; ++a) w[a] = wn[a];
            }
        } else {
#pragma unroll 1
            for (int r = 0; r < M; ++r) {
                const uint32_t o = G->off[r];
#pragma unroll
                for (int u = 0; u < UF; ++u)
                    if (ok[u]) tile[base[u] + o] = dense_row<R, M>(x[u], [&](int i) { return U[i]; }, r);
            }
        }
    }
}

// Monomial update of UF classes: A active entries move (and scale) src -> dst.
template <typename R, int A, int UF>
__device__ __forceinline__ void mono_classes(typename Cx<R>::T* tile, const typename Cx<R>::T* __restrict__ lam,
                                             const uint32_t (&src)[A], const uint32_t (&dst)[A], uint32_t mask,
                                             const uint32_t (&base)[UF], const bool (&ok)[UF]) {
    using T = typename Cx<R>::T;
    T x[UF][A];
#pragma unroll
    for (int u = 0; u < UF; ++u)
#pragma unroll
        for (int i = 0; i < A; ++i) x[u][i] = tile[base[u] + src[i]];  // clamped bases: unconditional
#pragma unroll
    for (int u = 0; u < UF; ++u) {
        if (!ok[u]) continue;
#pragma unroll
        for (int i = 0; i < A; ++i)
            tile[base[u] + dst[i]] = ((mask >> i) & 1u) ? x[u][i] : scale_by(lam[i], x[u][i]);
    }
}

// A gate's classes, in trips of UF per thread. The first 2 * UF classes of the
// thread take their bases from pre (static indices, so pre stays in registers),
// the rest from the table.
template <int UF, int BS, typename Body>
__device__ __forceinline__ void for_classes(const TileGate* __restrict__ G, const uint16_t* bases,
                                            const uint32_t (&pre)[kPre], const Body& body) {
    const uint32_t nc = G->n_classes;
    constexpr int P1 = 2 * UF;
    static_assert(P1 <= kPre, "prefetched classes exceed kPre");
#pragma unroll
    for (int t = 0; t < P1 / UF; ++t) {
        if (threadIdx.x + (uint32_t)(t * UF) * BS >= nc) break;
        uint32_t base[UF];
        bool ok[UF];
#pragma unroll
        for (int u = 0; u < UF; ++u) {
            ok[u] = threadIdx.x + (uint32_t)(t * UF + u) * BS < nc;
            base[u] = pre[t * UF + u];
        }
        body(base, ok);
    }
    for (uint32_t c0 = threadIdx.x + (uint32_t)P1 * BS; c0 < nc; c0 += UF * BS) {
        uint32_t base[UF];
        bool ok[UF];
#pragma unroll
        for (int u = 0; u < UF; ++u) {
            ok[u] = c0 + u * BS < nc;
            base[u] = bases[ok[u] ? c0 + u * BS : 0u];  // unconditional: no wait per load
        }
        body(base, ok);
    }
}

template <typename R, int M, int BS>
__device__ __forceinline__ void tile_dense(typename Cx<R>::T* tile, const TileGate* __restrict__ G,
                                           const typename Cx<R>::T* __restrict__ U, const uint16_t* bases,
                                           const uint32_t (&pre)[kPre]) {
    constexpr int UF = class_unroll<M>();
    uint32_t off[M];
#pragma unroll
    for (int a = 0; a < M; ++a) off[a] = G->off[a];
    for_classes<UF, BS>(G, bases, pre, [&](const uint32_t (&base)[UF], const bool (&ok)[UF]) {
        dense_classes<R, M, UF>(tile, G, U, off, base, ok);
    });
}

template <typename R, int A, int BS>
__device__ __forceinline__ void tile_mono(typename Cx<R>::T* tile, const TileGate* __restrict__ G,
                                          const typename Cx<R>::T* __restrict__ lam, const uint16_t* bases,
                                          const uint32_t (&pre)[kPre]) {
    constexpr int UF = class_unroll<A>();
    uint32_t src[A], dst[A];
#pragma unroll
    for (int i = 0; i < A; ++i) {
        src[i] = G->off[i];
        dst[i] = G->dst[i];
    }
    const uint32_t mask = G->one_mask;
    for_classes<UF, BS>(G, bases, pre, [&](const uint32_t (&base)[UF], const bool (&ok)[UF]) {
        mono_classes<R, A, UF>(tile, lam, src, dst, mask, base, ok);
    });
}

// A dense pair (kDensePair in fused.h) on UF joint classes: the first gate on
// each of the M2 sub-classes (local stride 1), the second on each of the M1
// sub-classes (local stride M1), from registers.
template <typename R, int M1, int M2, int UF>
__device__ __forceinline__ void pair_classes(typename Cx<R>::T* tile, const TileGate* __restrict__ G,
                                             const typename Cx<R>::T* __restrict__ U1,
                                             const typename Cx<R>::T* __restrict__ U2, const uint32_t (&off)[M1 * M2],
                                             const uint32_t (&base)[UF], const bool (&ok)[UF]) {
    using T = typename Cx<R>::T;
    constexpr int J = M1 * M2;
    T x[UF][J];
#pragma unroll
    for (int u = 0; u < UF; ++u)
#pragma unroll
        for (int a = 0; a < J; ++a) x[u][a] = tile[base[u] + off[a]];  // clamped bases: unconditional
    // For each output row a1 of the first gate: y[b] = row a1 of U1 on sub-class
    // b (x[M1 b .. M1 b + M1)), which is exactly the input of the second gate's
    // sub-class a1; its rows go straight to LDS.
    if constexpr (M1 * M1 + M2 * M2 <= 8) {
        // Two 2x2 matrices: all of both in scalar registers.
#pragma unroll
        for (int a1 = 0; a1 < M1; ++a1)
#pragma unroll
            for (int u = 0; u < UF; ++u) {
                if (!ok[u]) continue;
                T y[M2];
#pragma unroll
                for (int b = 0; b < M2; ++b)
                    y[b] = dense_row<R, M1>(&x[u][M1 * b], [&](int i) { return U1[i]; }, a1);
#pragma unroll
                for (int r = 0; r < M2; ++r)
                    tile[base[u] + off[a1 + M1 * r]] = dense_row<R, M2>(y, [&](int i) { return U2[i]; }, r);
            }
    } else {
        // Rolled loops keep one row of each matrix in scalar registers at a time.
#pragma unroll 1
        for (int a1 = 0; a1 < M1; ++a1) {
            T w1[M1];
#pragma unroll
            for (int a = 0; a < M1; ++a) w1[a] = U1[a1 * M1 + a];
#pragma unroll
            for (int u = 0; u < UF; ++u) {
                if (!ok[u]) continue;
                T y[M2];
#pragma unroll
                for (int b = 0; b < M2; ++b) y[b] = dense_dot<R, M1>(&x[u][M1 * b], [&](int a) { return w1[a]; });
#pragma unroll 1
                for (int r = 0; r < M2; ++r)
                    tile[base[u] + G->off[a1 + M1 * r]] = dense_row<R, M2>(y, [&](int i) { return U2[i]; }, r);
            }
        }
    }
}

template <typename R, int M1, int M2, int BS>
__device__ __forceinline__ void tile_pair(typename Cx<R>::T* tile, const TileGate* __restrict__ G,
                                          const typename Cx<R>::T* __restrict__ U, const uint16_t* bases,
                                          const uint32_t (&pre)[kPre]) {
    constexpr int J = M1 * M2;
    constexpr int UF = class_unroll<J>();
    uint32_t off[J];
#pragma unroll
    for (int a = 0; a < J; ++a) off[a] = G->off[a];
    const typename Cx<R>::T* __restrict__ U2 = U + M1 * M1;  // the second gate's matrix follows the first's
    for_classes<UF, BS>(G, bases, pre, [&](const uint32_t (&base)[UF], const bool (&ok)[UF]) {
        pair_classes<R, M1, M2, UF>(tile, G, U, U2, off, base, ok);
    });
}

// A chain (kDenseChain in fused.h) on UF classes: n dense gates applied one
// after the other in registers, every row with dense_row (the single-gate
// arithmetic); only the last gate's rows go to LDS.
template <typename R, int M, int UF>
__device__ __forceinline__ void chain_classes(typename Cx<R>::T* tile, const typename Cx<R>::T* __restrict__ U,
                                              const int n, const uint32_t (&off)[M], const uint32_t (&base)[UF],
                                              const bool (&ok)[UF]) {
    using T = typename Cx<R>::T;
    T x[UF][M];
#pragma unroll
    for (int u = 0; u < UF; ++u)
#pragma unroll
        for (int a = 0; a < M; ++a) x[u][a] = tile[base[u] + off[a]];  // clamped bases: unconditional
#pragma unroll 1
    for (int g = 0; g + 1 < n; ++g) {
        const T* __restrict__ Ug = U + g * M * M;
#pragma unroll
        for (int u = 0; u < UF; ++u) {
            T y[M];
#pragma unroll
            for (int r = 0; r < M; ++r) y[r] = dense_row<R, M>(x[u], [&](int i) { return Ug[i]; }, r);
#pragma unroll
            for (int r = 0; r < M; ++r) x[u][r] = y[r];
        }
    }
    const T* __restrict__ Ul = U + (n - 1) * M * M;
#pragma unroll
    for (int u = 0; u < UF; ++u) {
        if (!ok[u]) continue;
#pragma unroll
        for (int r = 0; r < M; ++r) tile[base[u] + off[r]] = dense_row<R, M>(x[u], [&](int i) { return Ul[i]; }, r);
    }
}

template <typename R, int M, int BS>
__device__ __forceinline__ void tile_chain(typename Cx<R>::T* tile, const TileGate* __restrict__ G,
                                           const typename Cx<R>::T* __restrict__ U, const uint16_t* bases,
                                           const uint32_t (&pre)[kPre]) {
    constexpr int UF = class_unroll<2 * M>();  // x and the next gate's rows both live
    uint32_t off[M];
#pragma unroll
    for (int a = 0; a < M; ++a) off[a] = G->off[a];
    const int n = G->M2;
    for_classes<UF, BS>(G, bases, pre, [&](const uint32_t (&base)[UF], const bool (&ok)[UF]) {
        chain_classes<R, M, UF>(tile, U, n, off, base, ok);
    });
}

// ---- register blocks (kBlock in fused.h) -------------------------------------------

template <int D0, int D1, int D2>
struct BlockShape {
    static constexpr int L = D1 == 1 ? 1 : (D2 == 1 ? 2 : 3);  // qudits in the block
    static constexpr int J = D0 * D1 * D2;                     // joint class size
    static constexpr int d(int p) { return p == 0 ? D0 : (p == 1 ? D1 : D2); }
    static constexpr int st(int p) { return p == 0 ? 1 : (p == 1 ? D0 : D0 * D1); }
};

// Largest class a block gate may have: its matrix is read into scalar registers
// (4 M^2 of them in complex128, 2 M^2 in complex64).
template <typename R>
constexpr int block_max_m() {
    return sizeof(R) == 8 ? 4 : 7;
}

// Joint index of member a of sub-class s of a one-qudit gate at position P (the
// sub-class enumerates the other positions, lower ones least significant).
template <class SH, int P>
constexpr int blk_j1(int s, int a) {
    return s % SH::st(P) + SH::st(P) * (a + SH::d(P) * (s / SH::st(P)));
}

// Joint index of member a = a_p + d(P) a_q of sub-class s of a two-qudit gate on
// positions (P, Q); s is the digit of the remaining position (0 when there are two).
template <class SH, int P, int Q>
constexpr int blk_j2(int s, int a) {
    return (SH::L == 3 ? s * SH::st(3 - P - Q) : 0) + (a % SH::d(P)) * SH::st(P) + (a / SH::d(P)) * SH::st(Q);
}

template <typename R, class SH, int P>
__device__ __forceinline__ void blk_dense1(typename Cx<R>::T (&x)[SH::J], const typename Cx<R>::T* __restrict__ U) {
    using T = typename Cx<R>::T;
    constexpr int M = SH::d(P), NS = SH::J / M;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        T v[M];
#pragma unroll
        for (int a = 0; a < M; ++a) v[a] = x[blk_j1<SH, P>(s, a)];
#pragma unroll
        for (int r = 0; r < M; ++r) x[blk_j1<SH, P>(s, r)] = dense_row<R, M>(v, [&](int i) { return U[i]; }, r);
    }
}

template <typename R, class SH, int P, int Q>
__device__ __forceinline__ void blk_dense2(typename Cx<R>::T (&x)[SH::J], const typename Cx<R>::T* __restrict__ U) {
    using T = typename Cx<R>::T;
    constexpr int M = SH::d(P) * SH::d(Q), NS = SH::J / M;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        T v[M];
#pragma unroll
        for (int a = 0; a < M; ++a) v[a] = x[blk_j2<SH, P, Q>(s, a)];
#pragma unroll
        for (int r = 0; r < M; ++r) x[blk_j2<SH, P, Q>(s, r)] = dense_row<R, M>(v, [&](int i) { return U[i]; }, r);
    }
}

// Phase gate: local index a of every sub-class scaled by lam[a] unless bit a of
// one_mask says its factor is exactly 1 (as the monomial update).
template <typename R, class SH, int P>
__device__ __forceinline__ void blk_diag1(typename Cx<R>::T (&x)[SH::J], const typename Cx<R>::T* __restrict__ lam,
                                          uint32_t one_mask) {
    constexpr int M = SH::d(P), NS = SH::J / M;
#pragma unroll
    for (int a = 0; a < M; ++a) {
        if ((one_mask >> a) & 1u) continue;  // uniform
        const typename Cx<R>::T w = lam[a];
#pragma unroll
        for (int s = 0; s < NS; ++s) x[blk_j1<SH, P>(s, a)] = scale_by(w, x[blk_j1<SH, P>(s, a)]);
    }
}

// Cyclic shift |a> -> |a + S mod d> (factors exactly 1): pure moves.
template <typename R, class SH, int P, int S>
__device__ __forceinline__ void blk_shift(typename Cx<R>::T (&x)[SH::J]) {
    using T = typename Cx<R>::T;
    constexpr int M = SH::d(P), NS = SH::J / M;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        T v[M];
#pragma unroll
        for (int a = 0; a < M; ++a) v[a] = x[blk_j1<SH, P>(s, a)];
#pragma unroll
        for (int a = 0; a < M; ++a) x[blk_j1<SH, P>(s, (a + S) % M)] = v[a];
    }
}

template <typename R, class SH, int P, int UF>
__device__ __forceinline__ void blk_shift1(typename Cx<R>::T (&x)[UF][SH::J], int sh) {
    constexpr int M = SH::d(P);
    switch (sh) {  // uniform
#define QD_SHIFT_CASE(k)                                                 \
    case k:                                                              \
        if constexpr ((k) < M) {                                         \
            _Pragma("unroll") for (int u = 0; u < UF; ++u) blk_shift<R, SH, P, k>(x[u]); \
        } else {                                                         \
            __builtin_unreachable();                                     \
        }                                                                \
        break;
        QD_SHIFT_CASE(1) QD_SHIFT_CASE(2) QD_SHIFT_CASE(3) QD_SHIFT_CASE(4) QD_SHIFT_CASE(5) QD_SHIFT_CASE(6)
#undef QD_SHIFT_CASE
        default: __builtin_unreachable();  // shifts 1 .. d - 1 only
    }
}

// One gate of a block on UF joint classes. The planner emits only codes that fit
// the block's shape (fusion.cpp checks each one), so every other code is
// unreachable: with no pass-through path, each case writes its results straight
// into the registers that carry x to the next gate (a pass-through path makes the
// compiler copy the whole joint class on every gate).
template <typename R, class SH, int UF>
__device__ __forceinline__ void blk_gate(typename Cx<R>::T (&x)[UF][SH::J], const BlockGate* __restrict__ b,
                                         const unsigned char* __restrict__ blob) {
    using T = typename Cx<R>::T;
    const T* __restrict__ U = reinterpret_cast<const T*>(blob + b->u_off);
    constexpr int MM = block_max_m<R>();
    switch (b->code) {
#define QD_BLK1(p)                                                                          \
    case kBlkDense1 * 16 + (p)*4:                                                           \
        if constexpr ((p) < SH::L && SH::d(p) <= MM) {                                      \
            _Pragma("unroll") for (int u = 0; u < UF; ++u) blk_dense1<R, SH, p>(x[u], U);   \
        } else {                                                                            \
            __builtin_unreachable();                                                        \
        }                                                                                   \
        break;                                                                              \
    case kBlkDiag1 * 16 + (p)*4:                                                            \
        if constexpr ((p) < SH::L) {                                                        \
            const uint32_t om = b->one_mask;                                                \
            _Pragma("unroll") for (int u = 0; u < UF; ++u) blk_diag1<R, SH, p>(x[u], U, om); \
        } else {                                                                            \
            __builtin_unreachable();                                                        \
        }                                                                                   \
        break;                                                                              \
    case kBlkShift1 * 16 + (p)*4:                                                           \
        if constexpr ((p) < SH::L) {                                                        \
            blk_shift1<R, SH, p, UF>(x, b->shift);                                          \
        } else {                                                                            \
            __builtin_unreachable();                                                        \
        }                                                                                   \
        break;
        QD_BLK1(0) QD_BLK1(1) QD_BLK1(2)
#undef QD_BLK1
#define QD_BLK2(p, q)                                                                          \
    case kBlkDense2 * 16 + (p)*4 + (q):                                                        \
        if constexpr ((p) < SH::L && (q) < SH::L && SH::d(p) * SH::d(q) <= MM) {               \
            _Pragma("unroll") for (int u = 0; u < UF; ++u) blk_dense2<R, SH, p, q>(x[u], U);   \
        } else {                                                                               \
            __builtin_unreachable();                                                           \
        }                                                                                      \
        break;
        QD_BLK2(0, 1) QD_BLK2(1, 0) QD_BLK2(0, 2) QD_BLK2(2, 0) QD_BLK2(1, 2) QD_BLK2(2, 1)
#undef QD_BLK2
        default: __builtin_unreachable();
    }
}

// Whether a block gate's controls outside the tile hold for the tile at `base`
// (uniform): multiply-high divisions for 32-bit bases, plain ones for 64-bit.
template <typename I>
__device__ __forceinline__ bool blk_outer_holds(const BlockOuter* __restrict__ o, I base) {
    for (int l = 0; l < o->n_outer; ++l) {
        I digit;
        if constexpr (sizeof(I) == 4) {
            const uint32_t q = fast_div<uint32_t>(base, o->oc_sdiv[l]);
            digit = q - fast_div<uint32_t>(q, o->oc_ddiv[l]) * o->oc_dim[l];
        } else {
            digit = (base / (I)o->oc_stride[l]) % (I)o->oc_dim[l];
        }
        if (digit != (I)o->oc_val[l]) return false;
    }
    return true;
}

template <typename R, int D0, int D1, int D2, int BS, typename I>
__device__ __forceinline__ void tile_block(typename Cx<R>::T* tile, const TileGate* __restrict__ G,
                                           const unsigned char* __restrict__ blob, const uint16_t* bases,
                                           const uint32_t (&pre)[kPre], I obase) {
    using T = typename Cx<R>::T;
    using SH = BlockShape<D0, D1, D2>;
    constexpr int J = SH::J;
    constexpr int UF = J <= 4 ? 2 : 1;
    uint32_t off[J];
#pragma unroll
    for (int a = 0; a < J; ++a) off[a] = G->off[a];
    const BlockGate* __restrict__ bg = reinterpret_cast<const BlockGate*>(blob + G->u_off);
    const int ng = G->M2;
    // Gates whose outer controls fail on this tile are skipped (bit g clear).
    uint32_t live = 0xffffffffu;
    const BlockOuter* __restrict__ bo = reinterpret_cast<const BlockOuter*>(bg + ng);
    for (uint32_t i = 0; i < G->dst[0]; ++i) {
        const BlockOuter* __restrict__ o = bo + __builtin_amdgcn_readfirstlane(i);
        if (!blk_outer_holds<I>(o, obase)) live &= ~(1u << o->gate);
    }
    for_classes<UF, BS>(G, bases, pre, [&](const uint32_t (&base)[UF], const bool (&ok)[UF]) {
        T x[UF][J];
#pragma unroll
        for (int u = 0; u < UF; ++u)
#pragma unroll
            for (int a = 0; a < J; ++a) x[u][a] = tile[base[u] + off[a]];  // clamped bases: unconditional
#pragma unroll 1
        for (int g = 0; g < ng; ++g)
            if ((live >> g) & 1u) blk_gate<R, SH, UF>(x, bg + __builtin_amdgcn_readfirstlane(g), blob);
#pragma unroll
        for (int u = 0; u < UF; ++u) {
            if (!ok[u]) continue;
#pragma unroll
            for (int a = 0; a < J; ++a) tile[base[u] + off[a]] = x[u][a];
        }
    });
}

// A block on its shape (kBlockShapes); complex128 joint classes stop at kBlockMaxJ128.
template <typename R, int BS, typename I>
__device__ __forceinline__ void tile_block_shape(typename Cx<R>::T* tile, const TileGate* __restrict__ G,
                                                 const unsigned char* __restrict__ blob, const uint16_t* bases,
                                                 const uint32_t (&pre)[kPre], I obase) {
    constexpr int JM = sizeof(R) == 8 ? kBlockMaxJ128 : kBlockMaxJ;
    static_assert(kBlockShapeCount == 19, "a case per block shape");
    switch (G->one_mask) {
#define QD_SHAPE(id)                                                                                       \
    case id:                                                                                               \
        if constexpr (kBlockShapes[id][0] * kBlockShapes[id][1] * kBlockShapes[id][2] <= JM)               \
            tile_block<R, kBlockShapes[id][0], kBlockShapes[id][1], kBlockShapes[id][2], BS>(tile, G, blob, \
                                                                                             bases, pre, obase); \
        break;
        QD_SHAPE(0) QD_SHAPE(1) QD_SHAPE(2) QD_SHAPE(3) QD_SHAPE(4) QD_SHAPE(5) QD_SHAPE(6) QD_SHAPE(7) QD_SHAPE(8)
        QD_SHAPE(9) QD_SHAPE(10) QD_SHAPE(11) QD_SHAPE(12) QD_SHAPE(13) QD_SHAPE(14) QD_SHAPE(15) QD_SHAPE(16)
        QD_SHAPE(17) QD_SHAPE(18)
#undef QD_SHAPE
        default: break;
    }
}

// First gate at or after g whose outer controls hold for this tile (uniform).
__device__ __forceinline__ int next_live_gate(const TileGate* __restrict__ gates, int g, int ngates, uint64_t obase) {
    for (; g < ngates; ++g) {
        const TileGate* __restrict__ G = gates + __builtin_amdgcn_readfirstlane(g);
        if (G->n_outer == 0 || outer_holds(G, obase)) break;
    }
    return g;
}

// The pass's gates applied to an LDS-resident tile. Every gate's class bases
// come from its uint16 table at blob + bases_off, and pre holds the prefetched
// bases of gate `first` (the first live gate, which the caller prefetched).
template <typename R, typename I, int BS>
__device__ __forceinline__ void apply_gates(typename Cx<R>::T* tile, I obase, int ngates,
                                            const TileGate* __restrict__ gates,
                                            const unsigned char* __restrict__ blob, int first,
                                            uint32_t (&pre)[kPre]) {
    using T = typename Cx<R>::T;
    for (int g = first; g < ngates;) {
        // g is uniform; say so, so that descriptor reads become scalar loads
        const TileGate* __restrict__ G = gates + __builtin_amdgcn_readfirstlane(g);
        const T* U = reinterpret_cast<const T*>(blob + G->u_off);
        const uint16_t* bases = reinterpret_cast<const uint16_t*>(blob + G->bases_off);
        if (G->kind == kBlock) {
            tile_block_shape<R, BS>(tile, G, blob, bases, pre, obase);
        } else if (G->kind == kDensePair) {
            switch (G->M * 8 + G->M2) {
#define QD_PAIR_CASE(m1, m2) \
    case m1 * 8 + m2: tile_pair<R, m1, m2, BS>(tile, G, U, bases, pre); break;
                QD_PAIR_CASE(2, 2) QD_PAIR_CASE(2, 3) QD_PAIR_CASE(2, 4) QD_PAIR_CASE(3, 2) QD_PAIR_CASE(3, 3)
                QD_PAIR_CASE(3, 4) QD_PAIR_CASE(4, 2) QD_PAIR_CASE(4, 3) QD_PAIR_CASE(4, 4)
#undef QD_PAIR_CASE
                default: break;
            }
        } else if (G->kind == kDenseChain) {
            static_assert(kChainMaxM == 3, "a case per chain class size");
            switch (G->M) {
                case 2: tile_chain<R, 2, BS>(tile, G, U, bases, pre); break;
                case 3: tile_chain<R, 3, BS>(tile, G, U, bases, pre); break;
                default: break;
            }
        } else if (G->kind == kDense) {
            switch (G->M) {
#define QD_DENSE_CASE(m) \
    case m: tile_dense<R, m, BS>(tile, G, U, bases, pre); break;
                QD_DENSE_CASE(2) QD_DENSE_CASE(3) QD_DENSE_CASE(4) QD_DENSE_CASE(5) QD_DENSE_CASE(6)
                QD_DENSE_CASE(7) QD_DENSE_CASE(8) QD_DENSE_CASE(9) QD_DENSE_CASE(10) QD_DENSE_CASE(11)
                QD_DENSE_CASE(12) QD_DENSE_CASE(13) QD_DENSE_CASE(14) QD_DENSE_CASE(15) QD_DENSE_CASE(16)
#undef QD_DENSE_CASE
                default: break;
            }
        } else {
            switch (G->M) {
#define QD_MONO_CASE(m) \
    case m: tile_mono<R, m, BS>(tile, G, U, bases, pre); break;
                QD_MONO_CASE(1) QD_MONO_CASE(2) QD_MONO_CASE(3) QD_MONO_CASE(4) QD_MONO_CASE(5) QD_MONO_CASE(6)
                QD_MONO_CASE(7) QD_MONO_CASE(8) QD_MONO_CASE(9) QD_MONO_CASE(10) QD_MONO_CASE(11)
                QD_MONO_CASE(12) QD_MONO_CASE(13) QD_MONO_CASE(14) QD_MONO_CASE(15) QD_MONO_CASE(16)
#undef QD_MONO_CASE
                default: break;
            }
        }
        g = next_live_gate(gates, g + 1, ngates, (uint64_t)obase);
        // The next gate's bases are loaded before the barrier: they depend on no
        // tile data, and land while the slowest wavefront finishes this gate.
        if (g < ngates) prefetch_bases<BS>(gates + __builtin_amdgcn_readfirstlane(g), blob, pre);
        __syncthreads();
    }
}

// Geometry of one tile: `nchunks` wavefront-sized chunks of the tile's runs of
// L contiguous amplitudes (chunk k: run k / chunks_per_run).
struct TileGeom {
    uint32_t tile, L, chunks_per_run, nchunks;
    FastDiv<uint32_t> cdiv;
};

// Chunk k of the tile belongs to wavefront k % nw; the run (and its offset) is
// uniform per wavefront, so the only per-lane work is one add. Out-of-range
// chunks and lanes past the end of a run are clamped to the tile's last valid
// element, so every address is in bounds and loads need no branch; the return
// value says whether this lane's element is real.
template <typename I>
__device__ __forceinline__ bool chunk_at(const TileGeom& a, const I* __restrict__ run_off, uint32_t k, uint32_t lane,
                                         uint32_t* t_at, I* g_off) {
    const bool in = k < a.nchunks;
    const uint32_t kk = in ? k : a.nchunks - 1;
    const uint32_t r = fast_div<uint32_t>(kk, a.cdiv);  // uniform: scalar unit
    const uint32_t e = (kk - r * a.chunks_per_run) * 64 + lane;
    const uint32_t ec = e < a.L ? e : a.L - 1;
    *t_at = r * a.L + ec;
    *g_off = run_off[r] + (I)ec;
    return in && e < a.L;
}

// Whole tile <-> HBM. A lane past the end of a run or of the tile gets the
// clamped last element (chunk_at), whose address in HBM and place in the tile
// belong together, so loads and LDS writes need no predicate: such a lane moves
// exactly what the lane that owns that element moves (the same value to the
// same place). The compiler issues a wavefront's U4 loads back to back with no
// wait between them: 256 bytes per lane in flight, a whole 64 KB tile per
// 256-thread workgroup.
template <typename T, typename I, bool LOAD, int BS>
__device__ __forceinline__ void move_tile(T* __restrict__ psi, T* tile, I obase, const TileGeom& a,
                                          const I* __restrict__ run_off) {
    constexpr uint32_t nw = BS / 64;
    constexpr int U4 = LOAD ? (int)(65536 / (BS * sizeof(T))) : 4;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
    const uint32_t lane = threadIdx.x % 64;
    for (uint32_t k0 = wave; k0 < a.nchunks; k0 += U4 * nw) {
        T v[U4];
        uint32_t t_at[U4];
        I g_off[U4];
        bool ok[U4];
#pragma unroll
        for (int u = 0; u < U4; ++u) ok[u] = chunk_at<I>(a, run_off, k0 + u * nw, lane, &t_at[u], &g_off[u]);
        if (LOAD) {
#pragma unroll
            for (int u = 0; u < U4; ++u) v[u] = ld_stream(psi + obase + g_off[u]);
#pragma unroll
            for (int u = 0; u < U4; ++u) tile[t_at[u]] = v[u];
        } else {
            // Stores stay predicated: a duplicate lane's store would be a second,
            // partial write of the same line (about 1.5% more HBM writes, measured).
#pragma unroll
            for (int u = 0; u < U4; ++u)
                if (ok[u]) st_stream(psi + obase + g_off[u], tile[t_at[u]]);
        }
    }
}

// Threads per tile workgroup. complex64 runs eight
// wavefronts per tile (16 per CU), complex128 four: at eight its pass measured
// slower (14.8 against 13.1 ms on the 1.72e9-amplitude register).
template <typename R>
constexpr int fuse_block() {
    return sizeof(R) == 4 ? 512 : 256;
}

// Both tile kernels ask for four waves per SIMD (1024 / BS workgroups per CU), the
// occupancy their LDS allows at the default tiles: at most 128 VGPRs.
template <typename R, typename I, int BS>
__global__ __launch_bounds__(BS, 1024 / BS) void fused_tile(typename Cx<R>::T* __restrict__ psi, const FusedArgs<I> a,
                                                         const TileGate* __restrict__ gates,
                                                         const unsigned char* __restrict__ blob,
                                                         const I* __restrict__ run_off) {
    using T = typename Cx<R>::T;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* tile = reinterpret_cast<T*>(smem_raw);
    const I obase = decode_base<I>(a.outer, (I)xcd_block());
    const TileGeom geo{a.tile, a.L, a.chunks_per_run, a.nchunks, a.cdiv};
    const int first = next_live_gate(gates, 0, a.ngates, (uint64_t)obase);
    uint32_t pre[kPre];
    // The first gate's bases go out together with the tile's loads.
    if (first < a.ngates) prefetch_bases<BS>(gates + __builtin_amdgcn_readfirstlane(first), blob, pre);
    move_tile<T, I, true, BS>(psi, tile, obase, geo, run_off);
    __syncthreads();
    apply_gates<R, I, BS>(tile, obase, a.ngates, gates, blob, first, pre);
    move_tile<T, I, false, BS>(psi, tile, obase, geo, run_off);
}

// A batched round: workgroup b processes tile (b - first_block) of the item
// whose block range holds b (binary search over the items' first blocks).
template <typename R, int BS>
__global__ __launch_bounds__(BS, 1024 / BS) void batch_tile(const BatchItem* __restrict__ items, int nitems,
                                                         const unsigned char* __restrict__ blob) {
    using T = typename Cx<R>::T;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* tile = reinterpret_cast<T*>(smem_raw);
    const uint32_t b = xcd_block();
    int lo = 0, hi = nitems - 1;
    while (lo < hi) {  // last item with first_block <= b (uniform)
        const int mid = (lo + hi + 1) >> 1;
        if (items[mid].first_block <= b) lo = mid;
        else hi = mid - 1;
    }
    const BatchItem* __restrict__ it = items + __builtin_amdgcn_readfirstlane(lo);
    const uint32_t obase = decode_base<uint32_t>(it->outer, b - it->first_block);
    const TileGeom geo{it->tile, it->L, it->chunks_per_run, it->nchunks, it->cdiv};
    T* psi = reinterpret_cast<T*>(it->psi);
    const uint32_t* run_off = reinterpret_cast<const uint32_t*>(blob + it->run_off_off);
    const TileGate* __restrict__ gates = reinterpret_cast<const TileGate*>(blob + it->gates_off);
    const int first = next_live_gate(gates, 0, it->ngates, (uint64_t)obase);
    uint32_t pre[kPre];
    if (first < it->ngates) prefetch_bases<BS>(gates + __builtin_amdgcn_readfirstlane(first), blob, pre);
    move_tile<T, uint32_t, true, BS>(psi, tile, obase, geo, run_off);
    __syncthreads();
    apply_gates<R, uint32_t, BS>(tile, obase, it->ngates, gates, blob, first, pre);
    move_tile<T, uint32_t, false, BS>(psi, tile, obase, geo, run_off);
}

template <typename K>
static hipError_t allow_lds(K* kernel, size_t bytes) {
    if (bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)bytes);
}

template <auto K, typename... Args>
static hipError_t launch_tile(const FusedLaunch& f, int bs, size_t shmem, hipStream_t st, Args... args) {
    hipError_t e = allow_lds(K, shmem);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(K, dim3((unsigned)f.n_tiles), dim3(bs), shmem, st, args...);
    return hipGetLastError();
}

template <typename R, typename I>
static hipError_t run_fused(const FusedLaunch& f, void* psi, const void* dblob, hipStream_t st) {
    using T = typename Cx<R>::T;
    FusedArgs<I> a;
    a.outer.n_classes = (I)f.n_tiles;
    a.outer.ctrl_off = 0;
    a.outer.nseg = f.outer_nseg;
    for (int g = 0; g < kMaxSeg; ++g) {
        a.outer.size[g] = g < f.outer_nseg ? (I)f.outer_size[g] : (I)1;
        a.outer.stride[g] = g < f.outer_nseg ? (I)f.outer_stride[g] : (I)0;
        a.outer.div[g] = make_fast_div<I>(g < f.outer_nseg ? f.outer_size[g] : 1);
    }
    a.tile = f.tile;
    a.L = f.L;
    a.chunks_per_run = (f.L + 63) / 64;
    a.nchunks = (f.tile / f.L) * a.chunks_per_run;
    a.cdiv = make_fast_div<uint32_t>(a.chunks_per_run);
    a.ngates = f.ngates;
    const unsigned char* b = static_cast<const unsigned char*>(dblob);
    const TileGate* tg = reinterpret_cast<const TileGate*>(b + f.gates_off);
    const I* ro = reinterpret_cast<const I*>(b + f.run_off_off);
    const size_t tile_bytes = (size_t)f.tile * sizeof(T);
    constexpr int BS = fuse_block<R>();
    return launch_tile<fused_tile<R, I, BS>>(f, BS, tile_bytes, st, static_cast<T*>(psi), a, tg, b, ro);
}

template <typename R>
static hipError_t run_batch(const void* ditems, int nitems, uint32_t nblocks, uint32_t max_tile, const void* dblob,
                            hipStream_t st) {
    using T = typename Cx<R>::T;
    const size_t shmem = (size_t)max_tile * sizeof(T);
    constexpr int BS = fuse_block<R>();
    hipError_t e = allow_lds(batch_tile<R, BS>, shmem);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((batch_tile<R, BS>), dim3(nblocks), dim3(BS), shmem, st,
                       static_cast<const BatchItem*>(ditems), nitems, static_cast<const unsigned char*>(dblob));
    return hipGetLastError();
}

hipError_t launch_batch(int precision, const void* ditems, int nitems, uint32_t nblocks, uint32_t max_tile,
                        const void* dblob, hipStream_t st) {
    if (nitems <= 0 || nblocks == 0) return hipSuccess;
    if (nblocks > 0x7fffffffu) return hipErrorInvalidValue;
    return precision == kC128 ? run_batch<double>(ditems, nitems, nblocks, max_tile, dblob, st)
                              : run_batch<float>(ditems, nitems, nblocks, max_tile, dblob, st);
}

hipError_t launch_fused(const FusedLaunch& f, int precision, void* psi, const void* dblob, hipStream_t st) {
    if (f.n_tiles == 0 || f.n_tiles > 0x7fffffffull) return hipErrorInvalidValue;
    const bool narrow = f.D < (1ull << 31);
    if (precision == kC128)
        return narrow ? run_fused<double, uint32_t>(f, psi, dblob, st) : run_fused<double, uint64_t>(f, psi, dblob, st);
    return narrow ? run_fused<float, uint32_t>(f, psi, dblob, st) : run_fused<float, uint64_t>(f, psi, dblob, st);
}

}  // namespace qd
