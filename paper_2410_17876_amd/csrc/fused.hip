// fused.hip - one HBM pass for a run of consecutive gates (fused.h explains
// the tiling). One workgroup per tile: load the tile into LDS with non-temporal
// loads of contiguous runs, apply each gate of the pass to the tile's classes
// in order (the same per-class arithmetic as the one-gate sweeps, device.h),
// write the tile back.
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

template <typename R, int M>
__device__ __forceinline__ void tile_dense(typename Cx<R>::T* tile, const TileGate* __restrict__ G,
                                           const typename Cx<R>::T* __restrict__ U,
                                           const uint16_t* __restrict__ bases) {
    using T = typename Cx<R>::T;
    constexpr int UF = class_unroll<M>();
    uint32_t off[M];
#pragma unroll
    for (int a = 0; a < M; ++a) off[a] = G->off[a];
    const uint32_t nc = G->n_classes;
    for (uint32_t c0 = threadIdx.x; c0 < nc; c0 += UF * kFuseBlock) {
        uint32_t base[UF];
        bool ok[UF];
#pragma unroll
        for (int u = 0; u < UF; ++u) {
            ok[u] = c0 + u * kFuseBlock < nc;
            base[u] = !ok[u] ? 0u : (bases ? bases[c0 + u * kFuseBlock] : decode_base<uint32_t>(G->dec, c0 + u * kFuseBlock));
        }
        T x[UF][M];
#pragma unroll
        for (int u = 0; u < UF; ++u)
#pragma unroll
            for (int a = 0; a < M; ++a)
                if (ok[u]) x[u][a] = tile[base[u] + off[a]];
#pragma unroll
        for (int u = 0; u < UF; ++u) {
            if (!ok[u]) continue;
            if constexpr (M <= 4) {
#pragma unroll
                for (int r = 0; r < M; ++r)
                    tile[base[u] + off[r]] = dense_row<R, M>(x[u], [&](int i) { return U[i]; }, r);
            } else {
                // Rolled over rows: an unrolled M x M body lets the compiler hoist all
                // of U out of the class loop into registers (spills for M > 4).
#pragma unroll 1
                for (int r = 0; r < M; ++r)
                    tile[base[u] + off[r]] = dense_row<R, M>(x[u], [&](int i) { return U[i]; }, r);
            }
        }
    }
}

template <typename R, int A>
__device__ __forceinline__ void tile_mono(typename Cx<R>::T* tile, const TileGate* __restrict__ G,
                                          const typename Cx<R>::T* __restrict__ lam,
                                          const uint16_t* __restrict__ bases) {
    using T = typename Cx<R>::T;
    constexpr int UF = class_unroll<A>();
    uint32_t src[A], dst[A];
#pragma unroll
    for (int i = 0; i < A; ++i) {
        src[i] = G->off[i];
        dst[i] = G->dst[i];
    }
    const uint32_t nc = G->n_classes;
    const uint32_t mask = G->one_mask;
    for (uint32_t c0 = threadIdx.x; c0 < nc; c0 += UF * kFuseBlock) {
        uint32_t base[UF];
        bool ok[UF];
#pragma unroll
        for (int u = 0; u < UF; ++u) {
            ok[u] = c0 + u * kFuseBlock < nc;
            base[u] = !ok[u] ? 0u : (bases ? bases[c0 + u * kFuseBlock] : decode_base<uint32_t>(G->dec, c0 + u * kFuseBlock));
        }
        T x[UF][A];
#pragma unroll
        for (int u = 0; u < UF; ++u)
#pragma unroll
            for (int i = 0; i < A; ++i)
                if (ok[u]) x[u][i] = tile[base[u] + src[i]];
#pragma unroll
        for (int u = 0; u < UF; ++u) {
            if (!ok[u]) continue;
#pragma unroll
            for (int i = 0; i < A; ++i)
                tile[base[u] + dst[i]] = ((mask >> i) & 1u) ? x[u][i] : scale_by(lam[i], x[u][i]);
        }
    }
}

// Geometry of one tile: `nchunks` wavefront-sized chunks of `runs` contiguous
// runs of L amplitudes each.
struct TileGeom {
    uint32_t tile, L, chunks_per_run, nchunks;
    FastDiv<uint32_t> cdiv;
};

// Tile <-> HBM. Each wavefront takes 64-amplitude chunks of runs; the run (and
// its offset) is uniform per wavefront, so the only per-lane work is one add.
template <typename T, typename I, bool LOAD>
__device__ __forceinline__ void move_tile(T* __restrict__ psi, T* tile, I obase, const TileGeom& a,
                                          const I* __restrict__ run_off) {
    constexpr uint32_t nw = kFuseBlock / 64;
    constexpr int U4 = 4;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
    const uint32_t lane = threadIdx.x % 64;
    for (uint32_t k0 = wave; k0 < a.nchunks; k0 += U4 * nw) {
        T v[U4];
        uint32_t t_at[U4];
        I g_at[U4];
        bool ok[U4];
#pragma unroll
        for (int u = 0; u < U4; ++u) {
            const uint32_t k = k0 + u * nw;
            const uint32_t r = fast_div<uint32_t>(k, a.cdiv);  // uniform: scalar unit
            const uint32_t e = (k - r * a.chunks_per_run) * 64 + lane;
            ok[u] = k < a.nchunks && e < a.L;
            t_at[u] = r * a.L + e;
            g_at[u] = obase + (k < a.nchunks ? run_off[r] : (I)0) + (I)e;
        }
        if (LOAD) {
#pragma unroll
            for (int u = 0; u < U4; ++u)
                if (ok[u]) v[u] = ld_stream(psi + g_at[u]);
#pragma unroll
            for (int u = 0; u < U4; ++u)
                if (ok[u]) tile[t_at[u]] = v[u];
        } else {
#pragma unroll
            for (int u = 0; u < U4; ++u)
                if (ok[u]) st_stream(psi + g_at[u], tile[t_at[u]]);
        }
    }
}

// One tile of one fused pass: load, apply the pass's gates in order, store.
template <typename R, typename I>
__device__ __forceinline__ void process_tile(typename Cx<R>::T* __restrict__ psi, typename Cx<R>::T* tile, I obase,
                                             const TileGeom& geo, int ngates, const TileGate* __restrict__ gates,
                                             const unsigned char* __restrict__ blob,
                                             const I* __restrict__ run_off) {
    using T = typename Cx<R>::T;
    move_tile<T, I, true>(psi, tile, obase, geo, run_off);
    __syncthreads();
    for (int g = 0; g < ngates; ++g) {
        // g is uniform; say so, so that descriptor reads become scalar loads
        const TileGate* __restrict__ G = gates + __builtin_amdgcn_readfirstlane(g);
        if (G->n_outer > 0 && !outer_holds(G, (uint64_t)obase)) continue;  // uniform over the workgroup
        const T* U = reinterpret_cast<const T*>(blob + G->u_off);
        const uint16_t* bases =
            G->bases_off == kDecodeBases ? nullptr : reinterpret_cast<const uint16_t*>(blob + G->bases_off);
        if (G->kind == kDense) {
            switch (G->M) {
#define QD_DENSE_CASE(m) \
    case m: tile_dense<R, m>(tile, G, U, bases); break;
                QD_DENSE_CASE(2) QD_DENSE_CASE(3) QD_DENSE_CASE(4) QD_DENSE_CASE(5) QD_DENSE_CASE(6)
                QD_DENSE_CASE(7) QD_DENSE_CASE(8) QD_DENSE_CASE(9) QD_DENSE_CASE(10) QD_DENSE_CASE(11)
                QD_DENSE_CASE(12) QD_DENSE_CASE(13) QD_DENSE_CASE(14) QD_DENSE_CASE(15) QD_DENSE_CASE(16)
#undef QD_DENSE_CASE
                default: break;
            }
        } else {
            switch (G->M) {
#define QD_MONO_CASE(m) \
    case m: tile_mono<R, m>(tile, G, U, bases); break;
                QD_MONO_CASE(1) QD_MONO_CASE(2) QD_MONO_CASE(3) QD_MONO_CASE(4) QD_MONO_CASE(5) QD_MONO_CASE(6)
                QD_MONO_CASE(7) QD_MONO_CASE(8) QD_MONO_CASE(9) QD_MONO_CASE(10) QD_MONO_CASE(11)
                QD_MONO_CASE(12) QD_MONO_CASE(13) QD_MONO_CASE(14) QD_MONO_CASE(15) QD_MONO_CASE(16)
#undef QD_MONO_CASE
                default: break;
            }
        }
        __syncthreads();
    }
    move_tile<T, I, false>(psi, tile, obase, geo, run_off);
}

template <typename R, typename I>
__global__ __launch_bounds__(kFuseBlock) void fused_tile(typename Cx<R>::T* __restrict__ psi, const FusedArgs<I> a,
                                                         const TileGate* __restrict__ gates,
                                                         const unsigned char* __restrict__ blob,
                                                         const I* __restrict__ run_off) {
    using T = typename Cx<R>::T;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* tile = reinterpret_cast<T*>(smem_raw);
    const I obase = decode_base<I>(a.outer, (I)xcd_block());
    const TileGeom geo{a.tile, a.L, a.chunks_per_run, a.nchunks, a.cdiv};
    process_tile<R, I>(psi, tile, obase, geo, a.ngates, gates, blob, run_off);
}

// A batched round: workgroup b processes tile (b - first_block) of the item
// whose block range holds b (binary search over the items' first blocks).
template <typename R>
__global__ __launch_bounds__(kFuseBlock) void batch_tile(const BatchItem* __restrict__ items, int nitems,
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
    process_tile<R, uint32_t>(reinterpret_cast<T*>(it->psi), tile, obase, geo, it->ngates,
                              reinterpret_cast<const TileGate*>(blob + it->gates_off), blob,
                              reinterpret_cast<const uint32_t*>(blob + it->run_off_off));
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
    const size_t shmem = (size_t)f.tile * sizeof(T);
    if (shmem > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&fused_tile<R, I>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((fused_tile<R, I>), dim3((unsigned)f.n_tiles), dim3(kFuseBlock), shmem, st,
                       static_cast<T*>(psi), a, reinterpret_cast<const TileGate*>(b + f.gates_off), b,
                       reinterpret_cast<const I*>(b + f.run_off_off));
    return hipGetLastError();
}

template <typename R>
static hipError_t run_batch(const void* ditems, int nitems, uint32_t nblocks, uint32_t max_tile, const void* dblob,
                            hipStream_t st) {
    using T = typename Cx<R>::T;
    const size_t shmem = (size_t)max_tile * sizeof(T);
    if (shmem > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&batch_tile<R>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((batch_tile<R>), dim3(nblocks), dim3(kFuseBlock), shmem, st,
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
