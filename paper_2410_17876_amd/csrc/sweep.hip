// sweep.hip - one gate, one pass over the statevector (gfx950, wave64).
//
// Every kernel here walks classes: the M amplitudes that differ only in the
// target digits (paper Sec. 2.3, Table 2), restricted to the amplitudes whose
// control digits hold the control values (Sec. 2.4). A thread owns whole
// classes: it reads every member, then writes every member, so the update is in
// place and classes never race (they are disjoint). Consecutive threads take
// consecutive class ids; the lowest free-qudit segment varies fastest, so for a
// target above the lowest qudits every member load of a wavefront is one
// contiguous run, and for a low target the M loads of a wavefront tile the same
// cache lines between them.
//
//   sweep_dense_reg<M>   superposition gates, M <= 16: x = gather, y = U x,
//                        scatter (Sec. 2.3); U in kernel arguments (M <= 8) or
//                        read through the scalar cache.
//   sweep_dense_lds      any M <= 343: a workgroup stages a tile of classes in
//                        LDS, then each thread produces (class, row) outputs.
//   sweep_monomial<A>    phase and permutation gates (Sec. 2.1, 2.2): each of
//                        the A active members is read once and written once to
//                        its image, scaled unless the factor is exactly 1, so
//                        pure moves are bit-exact; untouched members cost nothing.
//
// Memory-access choices, measured on MI355X with in-place streams of 27.5 GB:
// one class per thread beats register-blocking several classes per thread
// (more waves in flight, each instruction one contiguous run); non-temporal
// loads and stores (the data is touched once per gate) and a block-index remap
// that gives each of the 8 XCDs one contiguous range of classes (hardware
// dispatches consecutive workgroups round-robin over the XCDs) each add a few
// percent of HBM bandwidth.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "device.h"
#include "kernels.h"
#include "plan.h"

namespace qd {

constexpr int kBlock = 256;

template <typename I, int M>
struct Offs {
    I o[M];
};

template <typename R, int M, bool INL>
struct UArg;
template <typename R, int M>
struct UArg<R, M, true> {
    typename Cx<R>::T u[M * M];
    __device__ __forceinline__ typename Cx<R>::T get(int i) const { return u[i]; }
};
template <typename R, int M>
struct UArg<R, M, false> {};  // U comes as the kernel's Ug parameter

template <int M>
constexpr int dense_v() {
    return 1;
}

template <typename R, int M, typename I, int V, bool INL>
__global__ __launch_bounds__(kBlock) void sweep_dense_reg(typename Cx<R>::T* __restrict__ psi,
                                                          const Decode<I> dec, const Offs<I, M> off,
                                                          const UArg<R, M, INL> u,
                                                          const typename Cx<R>::T* __restrict__ Ug) {
    using T = typename Cx<R>::T;
    const I first = (I)xcd_block() * (I)(kBlock * V) + (I)threadIdx.x;
    I base[V];
    bool ok[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
        const I c = first + (I)(v * kBlock);
        ok[v] = c < dec.n_classes;
        base[v] = ok[v] ? decode_base<I>(dec, c) : (I)0;
    }
    T x[V][M];
#pragma unroll
    for (int v = 0; v < V; ++v)
        if (ok[v]) {
#pragma unroll
            for (int a = 0; a < M; ++a) x[v][a] = ld_stream(psi + base[v] + off.o[a]);
        }
#pragma unroll
    for (int v = 0; v < V; ++v)
        if (ok[v]) {
#pragma unroll
            for (int r = 0; r < M; ++r)
                st_stream(psi + base[v] + off.o[r], dense_row<R, M>(x[v], [&](int i) {
                              if constexpr (INL) return u.get(i);
                              else return Ug[i];
                          }, r));
        }
}

template <typename R, typename I, int A>
struct MonoArg {
    I src[A];
    I dst[A];
    typename Cx<R>::T lam[A];
    uint32_t one_mask;  // bit i set: factor i is exactly 1, a pure move
};

template <typename R, int A, typename I, int V>
__global__ __launch_bounds__(kBlock) void sweep_monomial(typename Cx<R>::T* __restrict__ psi,
                                                         const Decode<I> dec, const MonoArg<R, I, A> arg) {
    using T = typename Cx<R>::T;
    const I first = (I)xcd_block() * (I)(kBlock * V) + (I)threadIdx.x;
    I base[V];
    bool ok[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
        const I c = first + (I)(v * kBlock);
        ok[v] = c < dec.n_classes;
        base[v] = ok[v] ? decode_base<I>(dec, c) : (I)0;
    }
    T x[V][A];
#pragma unroll
    for (int v = 0; v < V; ++v)
        if (ok[v]) {
#pragma unroll
            for (int i = 0; i < A; ++i) x[v][i] = ld_stream(psi + base[v] + arg.src[i]);
        }
#pragma unroll
    for (int v = 0; v < V; ++v)
        if (ok[v]) {
#pragma unroll
            for (int i = 0; i < A; ++i) {
                const T y = ((arg.one_mask >> i) & 1u) ? x[v][i] : scale_by(arg.lam[i], x[v][i]);
                st_stream(psi + base[v] + arg.dst[i], y);
            }
        }
}

template <typename R, typename I>
__global__ __launch_bounds__(kBlock) void sweep_dense_lds(typename Cx<R>::T* __restrict__ psi,
                                                          const Decode<I> dec, const I* __restrict__ off,
                                                          const typename Cx<R>::T* __restrict__ U, int M,
                                                          int C, FastDiv<uint32_t> mdiv) {
    using T = typename Cx<R>::T;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* sx = reinterpret_cast<T*>(smem_raw);
    __shared__ I sbase[kBlock];
    const I first = (I)blockIdx.x * (I)C;
    const I left = dec.n_classes - first;
    const int ncls = left < (I)C ? (int)left : C;
    if ((int)threadIdx.x < ncls) sbase[threadIdx.x] = decode_base<I>(dec, first + (I)threadIdx.x);
    __syncthreads();
    const int total = ncls * M;
    for (int e = threadIdx.x; e < total; e += kBlock) {
        const int cl = (int)fast_div<uint32_t>((uint32_t)e, mdiv);
        const int a = e - cl * M;
        sx[e] = psi[sbase[cl] + off[a]];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < total; e += kBlock) {
        const int cl = (int)fast_div<uint32_t>((uint32_t)e, mdiv);
        const int r = e - cl * M;
        const T* xr = sx + cl * M;
        const T* ur = U + (size_t)r * M;
        R yr = 0, yi = 0;
        for (int a = 0; a < M; ++a) {
            const T w = ur[a];
            const T xv = xr[a];
            yr = fma(w.x, xv.x, yr);
            yr = fma(-w.y, xv.y, yr);
            yi = fma(w.x, xv.y, yi);
            yi = fma(w.y, xv.x, yi);
        }
        T y;
        y.x = yr;
        y.y = yi;
        psi[sbase[cl] + off[r]] = y;
    }
}

// ---------------------------------------------------------------------------
// host side

int plan_family(const GatePlan& p, int precision) {
    if (p.category == kIdentity) return kFamIdentity;
    if ((p.category == kMonomial || p.category == kDiagonal) && p.n_active <= kRegMaxM) return kFamMonomial;
    if (p.M <= kRegMaxM) return kFamDenseReg;
    if (p.category == kDense && p.M >= kMfmaMinM && p.M <= mfma_max_m(precision)) return kFamMfma;
    return kFamDenseLds;
}

const char* family_name(int f) {
    switch (f) {
        case kFamIdentity: return "identity";
        case kFamDenseReg: return "sweep_dense_reg";
        case kFamDenseLds: return "sweep_dense_lds";
        case kFamMonomial: return "sweep_monomial";
        case kFamMfma: return "block_mfma";
    }
    return "?";
}

static bool use32(const GatePlan& p) { return p.D < (1ull << 31); }

static int lds_classes(int M, int precision) {
    const int per = M * (int)amp_bytes(precision);
    return std::max(1, std::min(kBlock, 49152 / per));
}

size_t device_gate_bytes(const GatePlan& p, int precision) {
    const int f = plan_family(p, precision);
    if (f == kFamMfma) return mfma_gate_bytes(p.M, use32(p), precision);
    const size_t ab = amp_bytes(precision);
    if (f == kFamDenseReg && p.M > kInlineMaxM) return (size_t)p.M * p.M * ab;
    if (f == kFamDenseLds) return (size_t)p.M * p.M * ab + (size_t)p.M * 8;
    return 0;
}

template <typename R>
static void round_u(const double* U, int M, R* dst) {
    for (int i = 0; i < 2 * M * M; ++i) dst[i] = static_cast<R>(U[i]);
}

void fill_device_gate(const GatePlan& p, int precision, const double* U, void* dst) {
    const int f = plan_family(p, precision);
    if (f == kFamMfma) {
        fill_mfma_gate(p, precision, U, dst);
        return;
    }
    if (f != kFamDenseReg && f != kFamDenseLds) return;
    if (precision == kC128)
        round_u<double>(U, p.M, static_cast<double*>(dst));
    else
        round_u<float>(U, p.M, static_cast<float*>(dst));
    if (f == kFamDenseLds) {
        unsigned char* o = static_cast<unsigned char*>(dst) + (size_t)p.M * p.M * amp_bytes(precision);
        if (use32(p)) {
            uint32_t* oo = reinterpret_cast<uint32_t*>(o);
            for (int a = 0; a < p.M; ++a) oo[a] = (uint32_t)p.off[a];
        } else {
            uint64_t* oo = reinterpret_cast<uint64_t*>(o);
            for (int a = 0; a < p.M; ++a) oo[a] = (uint64_t)p.off[a];
        }
    }
}

template <typename R, int M, typename I>
static hipError_t run_dense_reg(const GatePlan& p, void* psi, const double* U, const void* dgate,
                                hipStream_t st) {
    using T = typename Cx<R>::T;
    constexpr int V = dense_v<M>();
    const Decode<I> dec = make_decode<I>(p);
    Offs<I, M> off;
    for (int a = 0; a < M; ++a) off.o[a] = (I)p.off[a];
    const uint64_t blocks = (p.n_classes + (uint64_t)kBlock * V - 1) / ((uint64_t)kBlock * V);
    if constexpr (M <= kInlineMaxM) {
        UArg<R, M, true> u;
        for (int i = 0; i < M * M; ++i) {
            u.u[i].x = static_cast<R>(U[2 * i]);
            u.u[i].y = static_cast<R>(U[2 * i + 1]);
        }
        hipLaunchKernelGGL((sweep_dense_reg<R, M, I, V, true>), dim3((unsigned)blocks), dim3(kBlock), 0, st,
                           static_cast<T*>(psi), dec, off, u, static_cast<const T*>(nullptr));
    } else {
        UArg<R, M, false> u;
        hipLaunchKernelGGL((sweep_dense_reg<R, M, I, V, false>), dim3((unsigned)blocks), dim3(kBlock), 0, st,
                           static_cast<T*>(psi), dec, off, u, static_cast<const T*>(dgate));
    }
    return hipGetLastError();
}

template <typename R, int A, typename I>
static hipError_t run_monomial(const GatePlan& p, void* psi, hipStream_t st) {
    using T = typename Cx<R>::T;
    constexpr int V = 1;
    const Decode<I> dec = make_decode<I>(p);
    MonoArg<R, I, A> arg;
    arg.one_mask = 0;
    for (int i = 0; i < A; ++i) {
        arg.src[i] = (I)p.off[p.src[i]];
        arg.dst[i] = (I)p.off[p.dst[i]];
        arg.lam[i].x = static_cast<R>(p.lam[2 * i]);
        arg.lam[i].y = static_cast<R>(p.lam[2 * i + 1]);
        if (p.lam_one[i]) arg.one_mask |= 1u << i;
    }
    const uint64_t blocks = (p.n_classes + (uint64_t)kBlock * V - 1) / ((uint64_t)kBlock * V);
    hipLaunchKernelGGL((sweep_monomial<R, A, I, V>), dim3((unsigned)blocks), dim3(kBlock), 0, st,
                       static_cast<T*>(psi), dec, arg);
    return hipGetLastError();
}

template <typename R, typename I>
static hipError_t run_dense_lds(const GatePlan& p, int precision, void* psi, const void* dgate,
                                hipStream_t st) {
    using T = typename Cx<R>::T;
    const Decode<I> dec = make_decode<I>(p);
    const int C = lds_classes(p.M, precision);
    const T* dU = static_cast<const T*>(dgate);
    const I* dOff = reinterpret_cast<const I*>(static_cast<const unsigned char*>(dgate) +
                                               (size_t)p.M * p.M * sizeof(T));
    const uint64_t blocks = (p.n_classes + C - 1) / C;
    const size_t shmem = (size_t)C * p.M * sizeof(T);
    hipLaunchKernelGGL((sweep_dense_lds<R, I>), dim3((unsigned)blocks), dim3(kBlock), shmem, st,
                       static_cast<T*>(psi), dec, dOff, dU, p.M, C, make_fast_div<uint32_t>(p.M));
    return hipGetLastError();
}

template <typename R, typename I, int M = 2>
static hipError_t dispatch_dense_reg(const GatePlan& p, void* psi, const double* U, const void* dgate,
                                     hipStream_t st) {
    if constexpr (M > kRegMaxM) {
        return hipErrorInvalidValue;
    } else {
        if (p.M == M) return run_dense_reg<R, M, I>(p, psi, U, dgate, st);
        return dispatch_dense_reg<R, I, M + 1>(p, psi, U, dgate, st);
    }
}

template <typename R, typename I, int A = 1>
static hipError_t dispatch_monomial(const GatePlan& p, void* psi, hipStream_t st) {
    if constexpr (A > kRegMaxM) {
        return hipErrorInvalidValue;
    } else {
        if (p.n_active == A) return run_monomial<R, A, I>(p, psi, st);
        return dispatch_monomial<R, I, A + 1>(p, psi, st);
    }
}

template <typename R, typename I>
static hipError_t launch_typed(const GatePlan& p, int precision, void* psi, const double* U,
                               const void* dgate, hipStream_t st) {
    switch (plan_family(p, precision)) {
        case kFamIdentity: return hipSuccess;
        case kFamMfma: return launch_mfma(p, precision, psi, dgate, st);
        case kFamMonomial: return dispatch_monomial<R, I>(p, psi, st);
        case kFamDenseReg: return dispatch_dense_reg<R, I>(p, psi, U, dgate, st);
        case kFamDenseLds: return run_dense_lds<R, I>(p, precision, psi, dgate, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_gate(const GatePlan& p, int precision, void* psi, const double* U, const void* dgate,
                       hipStream_t st) {
    if (p.n_classes == 0) return hipSuccess;
    if (precision == kC128)
        return use32(p) ? launch_typed<double, uint32_t>(p, precision, psi, U, dgate, st)
                        : launch_typed<double, uint64_t>(p, precision, psi, U, dgate, st);
    return use32(p) ? launch_typed<float, uint32_t>(p, precision, psi, U, dgate, st)
                    : launch_typed<float, uint64_t>(p, precision, psi, U, dgate, st);
}

}  // namespace qd
