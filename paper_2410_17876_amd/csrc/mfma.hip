// mfma.hip - dense class updates on the matrix cores (17 <= M <= 128:
// complex64 on FP32 MFMA, complex128 on FP64 MFMA).
//
// For a gate with a large class (several target qudits, e.g. a 25x25 or 125x125
// block on ququints) the per-class update y = U x (paper Sec. 2.3) is a dense
// contraction over all classes at once, Y = U X with X the M x N matrix whose
// columns are the N classes. With M = 125 that is 8 M = 1000 flops per
// amplitude, well past the HBM ridge point, so it runs on MFMA:
//
//   complex as real:  [Yr; Yi] = [[Ur, -Ui], [Ui, Ur]] [Xr; Xi],
//
// a real (2MP x 2MP) by (2MP x N) product with MP = M rounded up to 32, 64 or
// 128 (padding rows and columns of the real matrix are zero). A workgroup has
// eight wavefronts; each owns row blocks of the real matrix (32 rows for
// v_mfma_f32_32x32x2f32, 16 for v_mfma_f64_16x16x4f64), kept in registers for
// the whole launch (persistent workgroups loop over column tiles) except for
// the 256 x 256 FP64 form, which is streamed from L2, and one or more column
// blocks of the tile. Per column tile the workgroup gathers the
// classes' amplitudes into LDS (split into real and imaginary rows), runs the
// MFMAs over K = 2MP, writes the result blocks back to LDS and scatters them to
// the classes' addresses. A tile's classes are read completely before any of
// them is written, and tiles are disjoint, so the update is in place.
//
// Gather and scatter walk a tile's elements in address order: first the free
// qudits below the lowest target (a run of F amplitudes; F = 1 when q0 is a
// target), then the targets directly above them (the next `inner` address
// digits), then the rest of the class id, then the other targets' digits; rmap
// turns that order back into the local index. A tile then holds nt = F x
// floor(NT / F) classes so that its columns are whole runs. A wavefront touches
// contiguous amplitudes (walking the classes first would stride the lanes by
// the targets' extent when a target is low, and cost up to 10x on such gates).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "device.h"
#include "kernels.h"
#include "plan.h"

namespace qd {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kMfmaBlock = 512;  // 8 wavefronts

template <typename R, int MP>
struct MfmaShape;

// complex64, v_mfma_f32_32x32x2f32: a wavefront owns one 32-row block of the
// real matrix and one 32-column block of the tile; K advances 2 per step.
template <int MP>
struct MfmaShape<float, MP> {
    static constexpr bool STREAM = false;
    static constexpr int RB = 2 * MP / 32;  // row blocks
    static constexpr int NT = 32 * (8 / RB);
    static constexpr int KS = MP;            // K steps
};

// complex128, v_mfma_f64_16x16x4f64: a wavefront owns RW 16-row blocks and CB
// 16-column blocks (RW x CB independent accumulators); K advances 4 per step.
// Up to MP = 64 the real matrix sits in the eight wavefronts' registers for the
// whole launch (both sizes tile 64 classes; MP = 32 with two column groups of
// two blocks keeps the kernel within 128 VGPRs: two workgroups per CU). At
// MP = 128 (256 x 256 doubles, 512 KB) it stays in L2 and is streamed: the host
// stores it in fragment order, so a wavefront's fragment for one K step is 512
// contiguous bytes, and wavefront w owns row blocks w and w + 8 over a
// 32-class tile (67 KB of LDS, 126 VGPRs: two workgroups per CU). Streamed at
// MP = 64 as well, the 64-member gate measured 3.0 ms against 2.8 ms from
// registers on 14 ququarts.
template <int MP>
struct MfmaShape<double, MP> {
    static_assert(MP <= 128, "complex128 matrix-core blocks hold at most 128 members");
    static constexpr bool STREAM = MP == 128;
    static constexpr int RB = 2 * MP / 16;
    static constexpr int RW = STREAM ? RB / 8 : 1;  // row blocks per wavefront
    static constexpr int CB = MP == 64 ? 4 : 2;
    static constexpr int NT = STREAM ? 16 * CB : 16 * CB * (8 / RB);
    static constexpr int KS = MP / 2;
};

template <typename R, int MP>
constexpr int mfma_log_nt() {
    return MfmaShape<R, MP>::NT == 128 ? 7 : (MfmaShape<R, MP>::NT == 64 ? 6 : 5);
}

// Element order of a tile (see the header): F, inner and the classes per tile
// nt (a multiple of F, at most NT), with their divisors; B = nt / F.
struct MfmaOrder {
    int F, inner, nt, B;
    FastDiv<uint32_t> fdiv, idiv, bdiv;
};

template <typename R, int MP, typename I>
__global__ __launch_bounds__(kMfmaBlock) void block_mfma(typename Cx<R>::T* __restrict__ psi,
                                                         const Decode<I> dec, const int M, const I ntiles,
                                                         const R* __restrict__ A, const I* __restrict__ off,
                                                         const int32_t* __restrict__ rmap_g,
                                                         const MfmaOrder ord) {
    using T = typename Cx<R>::T;
    using S = MfmaShape<R, MP>;
    constexpr bool kF32 = sizeof(R) == 4;
    constexpr int K2 = 2 * MP;
    constexpr int LOG_NT = mfma_log_nt<R, MP>();
    constexpr int EPT = MP * S::NT / kMfmaBlock;  // tile elements gathered per thread
    // Real rows 0..MP-1, imaginary rows MP..2MP-1 (33 KB for complex64, 66 KB
    // for complex128). One padding column, so that a wavefront writing down a
    // column (low targets: consecutive lanes, consecutive rows) hits distinct
    // banks.
    __shared__ R Bs[K2][S::NT + 1];
    __shared__ I bases[2][S::NT];    // class bases of the current and the next tile
    __shared__ I offs[MP];
    __shared__ int32_t rmap[MP];

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int rb = wave % S::RB, cb = wave / S::RB;

    // This wavefront's rows of the real matrix, all of K = 2MP, as MFMA A
    // fragments: f32 32x32x2 lane l holds row l mod 32, K column 2s + l / 32;
    // f64 16x16x4 lane l holds row l mod 16, K column 4s + l / 16.
    R a[S::STREAM ? 1 : S::KS];
    if constexpr (!S::STREAM) {
#pragma unroll
        for (int s = 0; s < S::KS; ++s) {
            if constexpr (kF32)
                a[s] = A[(size_t)(32 * rb + (lane & 31)) * K2 + 2 * s + (lane >> 5)];
            else
                a[s] = A[(size_t)(16 * rb + (lane & 15)) * K2 + 4 * s + (lane >> 4)];
        }
    }
    for (int i = threadIdx.x; i < MP; i += kMfmaBlock) {
        offs[i] = i < M ? off[i] : (I)0;
        rmap[i] = i < M ? rmap_g[i] : 0;
    }
    // Padding rows (M..MP-1) of the B tile are never gathered: zero them once
    // (the MFMA multiplies them by A's zero columns; they must be finite). The
    // write-back of the result keeps them zero (A's padding rows are zero).
    for (int i = threadIdx.x; i < K2 * (S::NT + 1); i += kMfmaBlock) (&Bs[0][0])[i] = (R)0;
    __syncthreads();
    // Wait for the fragments once, here: left to the compiler, the wait for them
    // lands inside the tile loop, counted together with the prefetch loads, and
    // the last MFMA of every tile then waits for the next tile's gather.
    __builtin_amdgcn_s_waitcnt(0);

    const int nt = ord.nt;
    auto ncols_of = [&](I t) -> int {
        const I left = dec.n_classes - t * (I)nt;
        return left < (I)nt ? (int)left : nt;
    };
    // Element e of a tile in address order: f = e mod F (free low digits), then
    // low (the inner target digits), then cb (the rest of the class id: class
    // c = f + F cb), then hi (the other target digits); r is the local index.
    // Elements e >= M * nt do not exist; c >= ncols is past the last class. Such
    // elements load element (0, 0) (in bounds, no branch, so the loads issue back
    // to back) and are neither staged nor stored.
    const int MN = M * nt;
    auto element = [&](int e, int ncols, int* r, int* c) -> bool {
        if (ord.F == 1 && ord.inner == 1) {  // uniform: lanes over classes, then members
            *c = e & (S::NT - 1);
            *r = e >> LOG_NT;
            return e < MN && *c < ncols;
        }
        const uint32_t q1 = fast_div<uint32_t>((uint32_t)e, ord.fdiv);
        const int f = e - (int)q1 * ord.F;
        const uint32_t q2 = fast_div<uint32_t>(q1, ord.idiv);
        const int low = (int)(q1 - q2 * (uint32_t)ord.inner);
        const uint32_t hi = fast_div<uint32_t>(q2, ord.bdiv);
        const int cb = (int)(q2 - hi * (uint32_t)ord.B);
        const bool real = e < MN;
        *c = f + ord.F * cb;
        *r = rmap[real ? low + ord.inner * (int)hi : 0];  // index < M for real elements
        return real && *c < ncols;
    };
    // A thread's elements are the same in every tile (e = thread + i * block).
    // For blocks of at most 32 members their (local index, class) pairs and
    // member offsets are decoded once, here (only the class count of the last
    // tile can exclude more of them); the larger shapes need those registers
    // for their fragments and decode per use.
    constexpr bool PRE = MP == 32;
    int er[PRE ? EPT : 1], ec[PRE ? EPT : 1];
    I eoff[PRE ? EPT : 1];
    if constexpr (PRE) {
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            int r = 0, c = 0;
            const bool real = element(threadIdx.x + i * kMfmaBlock, nt, &r, &c);
            er[i] = real ? r : 0;
            ec[i] = real ? c : S::NT;  // S::NT: never below a tile's class count
            eoff[i] = offs[er[i]];
        }
    }
    // Element i of this thread in a tile of ncols classes: false if it does not exist.
    auto elem = [&](int i, int ncols, int* r, int* c, I* o) -> bool {
        if constexpr (PRE) {
            *r = er[i];
            *c = ec[i];
            *o = eoff[i];
            return ec[i] < ncols;
        } else {
            const bool ok = element(threadIdx.x + i * kMfmaBlock, ncols, r, c);
            *o = offs[ok ? *r : 0];
            return ok;
        }
    };
    auto gather = [&](T (&v)[EPT], int buf, int ncols) {
        I addr[EPT];
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            int r = 0, c = 0;
            I o = 0;
            const bool ok = elem(i, ncols, &r, &c, &o);
            addr[i] = bases[buf][ok ? c : 0] + (ok ? o : offs[0]);
        }
#pragma unroll
        for (int i = 0; i < EPT; ++i) v[i] = ld_stream(psi + addr[i]);
    };
    auto stage = [&](const T (&v)[EPT], int ncols) {
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            int r = 0, c = 0;
            I o = 0;
            if (elem(i, ncols, &r, &c, &o)) {
                Bs[r][c] = v[i].x;
                Bs[MP + r][c] = v[i].y;
            }
        }
    };

    I t = blockIdx.x;
    int cur = 0;
    if (t < ntiles) {
        const int nc = ncols_of(t);
        if ((int)threadIdx.x < nc) bases[0][threadIdx.x] = decode_base<I>(dec, t * (I)nt + (I)threadIdx.x);
        __syncthreads();
        T v[EPT];
        gather(v, 0, nc);
        stage(v, nc);
    }
    for (; t < ntiles; t += gridDim.x) {
        const int ncols = ncols_of(t);
        const I tn = t + gridDim.x;
        const bool has_next = tn < ntiles;
        const int ncols_next = has_next ? ncols_of(tn) : 0;
        if ((int)threadIdx.x < ncols_next)
            bases[cur ^ 1][threadIdx.x] = decode_base<I>(dec, tn * (I)nt + (I)threadIdx.x);
        __syncthreads();  // tile t staged in Bs; next bases visible
        // Prefetch the next tile into registers; the loads land during this tile's work.
        T pv[EPT];
        if (has_next) gather(pv, cur ^ 1, ncols_next);
        if constexpr (kF32) {
            f32x16 acc = {0};
#pragma unroll
            for (int s0 = 0; s0 < MP; s0 += 16) {
                float b[16];
#pragma unroll
                for (int j = 0; j < 16; ++j) b[j] = Bs[2 * (s0 + j) + (lane >> 5)][32 * cb + (lane & 31)];
#pragma unroll
                for (int j = 0; j < 16; ++j) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[s0 + j], b[j], acc, 0, 0, 0);
            }
            __syncthreads();  // every wavefront has read its B fragments
            // 32x32x2 result: lane l, register r holds row 8 (r / 4) + 4 (l / 32) + r mod 4, column l mod 32.
#pragma unroll
            for (int r = 0; r < 16; ++r)
                Bs[32 * rb + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3)][32 * cb + (lane & 31)] = acc[r];
        } else if constexpr (S::STREAM) {
            // Wavefront w: row blocks w + 8 h (h < RW), all CB column blocks. A's
            // fragment for (row block r, step s) is A[(r * KS + s) * 64 + lane].
            constexpr int CB = S::CB, RW = S::RW;
            constexpr int KG = 2;  // K steps per group: at 4 the MP = 128 kernel needs 140 VGPRs (one workgroup per CU)
            f64x4 acc[RW][CB];
#pragma unroll
            for (int h = 0; h < RW; ++h)
#pragma unroll
                for (int c = 0; c < CB; ++c) acc[h][c] = f64x4{0.0, 0.0, 0.0, 0.0};
            const R* __restrict__ Aw = A + (size_t)wave * S::KS * 64 + lane;
#pragma unroll 4
            for (int s0 = 0; s0 < S::KS; s0 += KG) {
                double a[KG][RW], b[KG][CB];
#pragma unroll
                for (int j = 0; j < KG; ++j) {
#pragma unroll
                    for (int h = 0; h < RW; ++h) a[j][h] = Aw[((size_t)8 * h * S::KS + s0 + j) * 64];
#pragma unroll
                    for (int c = 0; c < CB; ++c) b[j][c] = Bs[4 * (s0 + j) + (lane >> 4)][16 * c + (lane & 15)];
                }
#pragma unroll
                for (int j = 0; j < KG; ++j)
#pragma unroll
                    for (int c = 0; c < CB; ++c)
#pragma unroll
                        for (int h = 0; h < RW; ++h)
                            acc[h][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[j][h], b[j][c], acc[h][c], 0, 0, 0);
            }
            __syncthreads();  // every wavefront has read its B fragments
#pragma unroll
            for (int h = 0; h < RW; ++h)
#pragma unroll
                for (int c = 0; c < CB; ++c)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        Bs[16 * (wave + 8 * h) + 4 * r + (lane >> 4)][16 * c + (lane & 15)] = acc[h][c][r];
        } else {
            constexpr int CB = S::CB;
            f64x4 acc[CB];
#pragma unroll
            for (int c = 0; c < CB; ++c) acc[c] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int s0 = 0; s0 < S::KS; s0 += 4) {
                double b[4][CB];
#pragma unroll
                for (int j = 0; j < 4; ++j)
#pragma unroll
                    for (int c = 0; c < CB; ++c)
                        b[j][c] = Bs[4 * (s0 + j) + (lane >> 4)][16 * (CB * cb + c) + (lane & 15)];
#pragma unroll
                for (int j = 0; j < 4; ++j)
#pragma unroll
                    for (int c = 0; c < CB; ++c)
                        acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s0 + j], b[j][c], acc[c], 0, 0, 0);
            }
            __syncthreads();  // every wavefront has read its B fragments
            // 16x16x4 result: lane l, register r holds row 4 r + l / 16, column l mod 16.
#pragma unroll
            for (int c = 0; c < CB; ++c)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    Bs[16 * rb + 4 * r + (lane >> 4)][16 * (CB * cb + c) + (lane & 15)] = acc[c][r];
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            int r = 0, c = 0;
            I o = 0;
            if (elem(i, ncols, &r, &c, &o)) {
                T y;
                y.x = Bs[r][c];
                y.y = Bs[MP + r][c];
                st_stream(psi + bases[cur][c] + o, y);
            }
        }
        __syncthreads();  // Bs free
        if (has_next) stage(pv, ncols_next);
        cur ^= 1;
    }
}

int mfma_padded(int M) { return M <= 32 ? 32 : (M <= 64 ? 64 : 128); }

int mfma_max_m(int /*precision*/) { return 128; }  // both precisions: FP32 and FP64 MFMA up to 128

static size_t mfma_real_bytes(int precision) { return precision == kC128 ? sizeof(double) : sizeof(float); }

size_t mfma_gate_bytes(int M, bool narrow, int precision) {
    const size_t K2 = 2 * (size_t)mfma_padded(M);
    return K2 * K2 * mfma_real_bytes(precision) + (size_t)M * (narrow ? 4 : 8) + (size_t)M * 4;
}

// The gather's element order (see the header), from the gate's free segments
// and member offsets: F = the lowest free run when it starts at q0 and a target
// sits right above it (kept only while a tile still holds at least 7/8 of NT
// classes), inner = the largest m with offsets 0, F, ..., (m-1) F all present,
// and rmap[low + inner * hi] = the local index whose offset is low * F plus the
// hi-th smallest of the remaining parts.
struct Order {
    int F, inner, nt;
};

static Order mfma_order(const GatePlan& p, int NT) {
    int64_t step = 0;
    for (int a = 0; a < p.M; ++a)
        if (p.off[a] > 0 && (step == 0 || p.off[a] < step)) step = p.off[a];
    int64_t F = 1;
    if (p.nseg > 0 && p.seg_stride[0] == 1 && (int64_t)p.seg_size[0] == step) F = (int64_t)p.seg_size[0];
    if (F > NT || F * (NT / F) * 8 < 7 * (int64_t)NT) F = 1;
    std::vector<int64_t> offs(p.off, p.off + p.M);
    std::sort(offs.begin(), offs.end());
    int inner = 0;
    while (inner < p.M && std::binary_search(offs.begin(), offs.end(), (int64_t)inner * F)) ++inner;
    if (inner < 1) inner = 1;
    return Order{(int)F, inner, (int)(F * (NT / F))};
}

static void mfma_rmap(const GatePlan& p, const Order& o, int32_t* rmap) {
    std::vector<int64_t> his;
    for (int a = 0; a < p.M; ++a) his.push_back(p.off[a] - ((p.off[a] / o.F) % o.inner) * o.F);
    std::sort(his.begin(), his.end());
    his.erase(std::unique(his.begin(), his.end()), his.end());
    for (int a = 0; a < p.M; ++a) {
        const int64_t low = (p.off[a] / o.F) % o.inner;
        const int64_t hi =
            std::lower_bound(his.begin(), his.end(), p.off[a] - low * o.F) - his.begin();
        rmap[low + (int64_t)o.inner * hi] = a;
    }
}

static int mfma_nt(int M, int precision) {
    const int MP = mfma_padded(M);
    if (precision == kC128)
        return MP == 32 ? MfmaShape<double, 32>::NT : (MP == 64 ? MfmaShape<double, 64>::NT : MfmaShape<double, 128>::NT);
    return MP == 32 ? MfmaShape<float, 32>::NT : (MP == 64 ? MfmaShape<float, 64>::NT : MfmaShape<float, 128>::NT);
}

// The real form [[Ur, -Ui], [Ui, Ur]] of U, zero-padded to 2MP x 2MP, row-major.
template <typename R>
static void fill_real(const GatePlan& p, const double* U, R* A) {
    const int MP = mfma_padded(p.M);
    const int K2 = 2 * MP;
    for (int i = 0; i < K2 * K2; ++i) A[i] = (R)0;
    for (int r = 0; r < p.M; ++r)
        for (int c = 0; c < p.M; ++c) {
            const R ur = static_cast<R>(U[2 * (r * p.M + c)]);
            const R ui = static_cast<R>(U[2 * (r * p.M + c) + 1]);
            A[r * K2 + c] = ur;
            A[r * K2 + MP + c] = -ui;
            A[(MP + r) * K2 + c] = ui;
            A[(MP + r) * K2 + MP + c] = ur;
        }
}

void fill_mfma_gate(const GatePlan& p, int precision, const double* U, void* dst) {
    const int K2 = 2 * mfma_padded(p.M);
    const bool stream = precision == kC128 && (mfma_padded(p.M) == 128 ? MfmaShape<double, 128>::STREAM
                                               : (mfma_padded(p.M) == 64 && MfmaShape<double, 64>::STREAM));
    if (stream) {
        // Fragment order for the streamed kernel: entry (r * KS + s) * 64 + l is
        // the real form's row 16 r + l mod 16, column 4 s + l / 16 (KS = K2 / 4).
        const int RB = K2 / 16, KS = K2 / 4;
        std::vector<double> rm((size_t)K2 * K2);
        fill_real<double>(p, U, rm.data());
        double* A = static_cast<double*>(dst);
        for (int r = 0; r < RB; ++r)
            for (int st = 0; st < KS; ++st)
                for (int l = 0; l < 64; ++l)
                    A[((size_t)r * KS + st) * 64 + l] = rm[(size_t)(16 * r + l % 16) * K2 + 4 * st + l / 16];
    } else if (precision == kC128) {
        fill_real<double>(p, U, static_cast<double*>(dst));
    } else {
        fill_real<float>(p, U, static_cast<float*>(dst));
    }
    unsigned char* o = static_cast<unsigned char*>(dst) + (size_t)K2 * K2 * mfma_real_bytes(precision);
    const bool narrow = p.D < (1ull << 31);
    if (narrow) {
        uint32_t* oo = reinterpret_cast<uint32_t*>(o);
        for (int a = 0; a < p.M; ++a) oo[a] = (uint32_t)p.off[a];
    } else {
        uint64_t* oo = reinterpret_cast<uint64_t*>(o);
        for (int a = 0; a < p.M; ++a) oo[a] = (uint64_t)p.off[a];
    }
    int32_t* rm = reinterpret_cast<int32_t*>(o + (size_t)p.M * (narrow ? 4 : 8));
    mfma_rmap(p, mfma_order(p, mfma_nt(p.M, precision)), rm);
}

template <typename R, int MP, typename I>
static hipError_t run_mfma(const GatePlan& p, void* psi, const void* dgate, hipStream_t st) {
    using S = MfmaShape<R, MP>;
    const Decode<I> dec = make_decode<I>(p);
    const Order o = mfma_order(p, S::NT);
    MfmaOrder ord;
    ord.F = o.F;
    ord.inner = o.inner;
    ord.nt = o.nt;
    ord.B = o.nt / o.F;
    ord.fdiv = make_fast_div<uint32_t>((uint64_t)o.F);
    ord.idiv = make_fast_div<uint32_t>((uint64_t)o.inner);
    ord.bdiv = make_fast_div<uint32_t>((uint64_t)ord.B);
    const uint64_t ntiles = (p.n_classes + (uint64_t)o.nt - 1) / (uint64_t)o.nt;
    static int per_cu = 0;
    static int cus = 0;
    if (!per_cu) {
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, block_mfma<R, MP, I>, kMfmaBlock, 0);
        if (e != hipSuccess) return e;
        if (per_cu < 1) per_cu = 1;
    }
    const uint64_t grid = std::min<uint64_t>(ntiles, (uint64_t)per_cu * cus);
    const R* A = static_cast<const R*>(dgate);
    const I* off = reinterpret_cast<const I*>(static_cast<const unsigned char*>(dgate) +
                                              (size_t)(2 * MP) * (2 * MP) * sizeof(R));
    const int32_t* rmap = reinterpret_cast<const int32_t*>(off + p.M);
    hipLaunchKernelGGL((block_mfma<R, MP, I>), dim3((unsigned)grid), dim3(kMfmaBlock), 0, st,
                       static_cast<typename Cx<R>::T*>(psi), dec, p.M, (I)ntiles, A, off, rmap, ord);
    return hipGetLastError();
}

template <typename I>
static hipError_t launch_mfma_typed(const GatePlan& p, int precision, void* psi, const void* dgate,
                                    hipStream_t st) {
    const int MP = mfma_padded(p.M);
    if (precision == kC128) {
        if (MP == 32) return run_mfma<double, 32, I>(p, psi, dgate, st);
        if (MP == 64) return run_mfma<double, 64, I>(p, psi, dgate, st);
        return run_mfma<double, 128, I>(p, psi, dgate, st);
    }
    if (MP == 32) return run_mfma<float, 32, I>(p, psi, dgate, st);
    if (MP == 64) return run_mfma<float, 64, I>(p, psi, dgate, st);
    return run_mfma<float, 128, I>(p, psi, dgate, st);
}

hipError_t launch_mfma(const GatePlan& p, int precision, void* psi, const void* dgate, hipStream_t st) {
    if (p.n_classes == 0) return hipSuccess;
    if (p.M > mfma_max_m(precision)) return hipErrorInvalidValue;
    return p.D < (1ull << 31) ? launch_mfma_typed<uint32_t>(p, precision, psi, dgate, st)
                              : launch_mfma_typed<uint64_t>(p, precision, psi, dgate, st);
}

}  // namespace qd
