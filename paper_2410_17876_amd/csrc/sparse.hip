// sparse.hip - a gate on a sparse statevector (sparse.h).
//
// Per gate (Sec. 2.3, 2.4):
// 1. classify: every entry's group is its class base (the key with the target
//    digits set to 0) and its local index, when the controls hold; an entry
//    whose controls fail is its own group (local index -1), and such a key never
//    equals the base of a class whose controls hold (they differ in a control
//    digit), so the two kinds of groups never mix.
// 2. one result per class with a present member: gather the members (absent
//    ones are 0 and skipped), y = U x with textbook complex products summed in
//    ascending column order, keep the nonzero results; a control-failing entry
//    is kept unchanged.
// 3. the kept results sorted by key become the new entries.
//
// Two forms. While (entries x class size) fits kSparseSmallCap, one workgroup
// does all three steps in LDS (grouping by pairwise key comparison, ordering by
// rank counting) and reads the entry count from, and writes it to, device
// memory, so gates are enqueued back to back with no host synchronisation and
// the matrix is read straight from pinned host memory. Beyond that, entries are
// grouped with a radix sort by group key, one thread per group head computes
// its class, and the kept results are radix-sorted by key (hipCUB; keys of
// several words are sorted word by word, least significant word first, which a
// stable radix sort makes lexicographic); the kept count is read back once.
#include <hip/hip_runtime.h>

#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cstring>
#include <vector>

#include "sparse.h"

namespace qd {

namespace {

constexpr int kSmallThreads = 512;
constexpr int kRunChunk = 16;         // gate records a run keeps in LDS at a time
constexpr size_t kRunInitGates = 256;  // gate records a new state can stage for runs
typedef unsigned long long U64x2 __attribute__((ext_vector_type(2)));
static_assert(sizeof(SparseGate) % 16 == 0, "gate records are copied in 16-byte pieces");
constexpr uint32_t kSmallIn = kSparseSmallCap / 2;  // entries of a small gate (class size >= 2)
constexpr int kErrWord = 2;                         // nnz_dev[2]: set if a small gate saw more entries than planned

__device__ __forceinline__ uint32_t digit_of(uint64_t v, const FastDiv<uint64_t>& s, const FastDiv<uint64_t>& dd,
                                             uint32_t d) {
    const uint64_t q = fast_div<uint64_t>(v, s);
    return (uint32_t)(q - fast_div<uint64_t>(q, dd) * (uint64_t)d);
}

// Group of one entry: returns its local index (the key becomes the class base)
// when every control holds, else -1 (the key is left as it is).
__device__ __forceinline__ int classify(const SparseGate& g, uint64_t (&key)[kKeyWords]) {
    for (int l = 0; l < g.m; ++l)
        if (digit_of(key[g.cw[l]], g.csd[l], g.cdd[l], g.cd[l]) != g.cv[l]) return -1;
    int a = 0, w = 1;
    for (int l = 0; l < g.k; ++l) {
        const uint32_t dg = digit_of(key[g.tw[l]], g.tsd[l], g.tdd[l], g.td[l]);
        a += (int)dg * w;
        w *= (int)g.td[l];
        key[g.tw[l]] -= (uint64_t)dg * g.ts[l];
    }
    return a;
}

// Row r of U x over the present members of a class (bit a of `present`), in
// ascending a, as textbook complex products with no FMA contraction: which
// results are exactly zero (and dropped) then does not depend on how the
// compiler would fuse them. The loop runs over compile-time indices, so x stays
// in registers (a runtime index would put it in scratch memory).
template <int N>
__device__ __forceinline__ double2 class_row(const double2* U, const double2 (&x)[N], uint32_t present, int r, int M) {
#pragma clang fp contract(off)
    double yr = 0.0, yi = 0.0;
#pragma unroll
    for (int a = 0; a < N; ++a) {
        if (a >= M || !((present >> a) & 1u)) continue;
        const double2 u = U[r * M + a];
        yr = yr + (u.x * x[a].x - u.y * x[a].y);
        yi = yi + (u.x * x[a].y + u.y * x[a].x);
    }
    return double2{yr, yi};
}

// x[la] = v with compile-time indices only (see class_row).
template <int N>
__device__ __forceinline__ void set_member(double2 (&x)[N], int la, double2 v) {
#pragma unroll
    for (int a = 0; a < N; ++a)
        if (a == la) x[a] = v;
}

// LDS of the one-workgroup form: the gate's grouping and its results.
struct SmallLds {
    uint64_t gk[kKeyWords][kSmallIn];  // group keys (class bases, or the key itself)
    int32_t la[kSmallIn];              // local indices (-1: controls fail)
    uint64_t ok[kKeyWords][kSparseSmallCap];
    double2 oa[kSparseSmallCap];
    uint8_t of[kSparseSmallCap];       // output slot holds a kept result
    double2 su[kSparseMaxM * kSparseMaxM];
    uint32_t kept;
};

// One gate on n <= kSmallIn entries (n * M <= kSparseSmallCap, M <= MaxM), the
// whole workgroup: key word w of entry i is kin(w, i), its amplitude ain(i); the
// kept results are handed, in key order, to put(rank, s) (output slot s of L).
// Entry i's results take output slots i * M .. i * M + M - 1 (only a group's
// first entry's slots are filled, one thread per slot). Returns the kept count
// (after a barrier; uniform). The inputs are last read before the second barrier
// and put runs after it, so put may overwrite them. W: the key words (g.W). U:
// the matrix, copied to LDS first unless ULds (U already in LDS).
template <int MaxM, int W, bool ULds, typename KIn, typename AIn, typename Put>
__device__ __forceinline__ uint32_t small_gate(const SparseGate& g, const double2* U, uint32_t n, SmallLds& L,
                                               const KIn& kin, const AIn& ain, const Put& put) {
    const uint32_t tid = threadIdx.x;
    const int M = g.M;
    const uint32_t T = n * (uint32_t)M;
    auto same = [&](uint32_t i, uint32_t j) {
        for (int w = 0; w < W; ++w)
            if (L.gk[w][i] != L.gk[w][j]) return false;
        return true;
    };
    auto less = [&](uint32_t s, uint32_t t) {  // key of output s < key of output t
        for (int w = W - 1; w >= 0; --w)
            if (L.ok[w][s] != L.ok[w][t]) return L.ok[w][s] < L.ok[w][t];
        return false;
    };
    if (!ULds)
        for (uint32_t i = tid; i < (uint32_t)(M * M); i += kSmallThreads) L.su[i] = U[i];
    const double2* Ur = ULds ? U : L.su;
    for (uint32_t i = tid; i < n; i += kSmallThreads) {
        uint64_t key[kKeyWords] = {0, 0, 0};
#pragma unroll
        for (int w = 0; w < W; ++w) key[w] = kin(w, i);
        L.la[i] = classify(g, key);
#pragma unroll
        for (int w = 0; w < W; ++w) L.gk[w][i] = key[w];
    }
    for (uint32_t s = tid; s < T; s += kSmallThreads) L.of[s] = 0;
    if (tid == 0) L.kept = 0;
    __syncthreads();
    // One thread per output slot s = i * M + r: if entry i leads its group, row r
    // of U times the group's members.
    for (uint32_t s = tid; s < T; s += kSmallThreads) {
        const uint32_t i = s / (uint32_t)M, r = s - i * (uint32_t)M;
        bool lead = true;
        for (uint32_t j = 0; j < i; ++j)
            if (same(i, j)) {
                lead = false;
                break;
            }
        if (!lead) continue;
        if (L.la[i] < 0) {  // controls fail: unchanged, in the group's first slot
            if (r == 0) {
#pragma unroll
                for (int w = 0; w < W; ++w) L.ok[w][s] = L.gk[w][i];
                L.oa[s] = ain(i);
                L.of[s] = 1;
            }
            continue;
        }
        double2 x[MaxM];
#pragma unroll
        for (int a = 0; a < MaxM; ++a) x[a] = double2{0.0, 0.0};
        uint32_t present = 0;
        for (uint32_t j = i; j < n; ++j)
            if (same(i, j)) {
                set_member(x, L.la[j], ain(j));
                present |= 1u << L.la[j];
            }
        const double2 y = class_row(Ur, x, present, (int)r, M);
#pragma unroll
        for (int w = 0; w < W; ++w) L.ok[w][s] = L.gk[w][i] + g.off[r][w];
        L.oa[s] = y;
        L.of[s] = (y.x != 0.0 || y.y != 0.0) ? 1 : 0;
    }
    __syncthreads();
    // Each kept result goes to its rank among the kept keys (keys are distinct:
    // classes are disjoint and control-failing keys meet no class).
    if (T <= 64) {
        // One wavefront: a ballot of the flags gives the kept slots, and each kept
        // result compares itself with those only, not with all T slots.
        if (tid < 64) {
            const bool k = tid < T && L.of[tid];
            const uint64_t kept = __ballot(k);
            if (tid == 0) L.kept = (uint32_t)__popcll(kept);
            if (k) {
                uint32_t rank = 0;
                for (uint64_t m = kept; m; m &= m - 1)
                    rank += less((uint32_t)__builtin_ctzll(m), tid) ? 1u : 0u;
                put(rank, tid);
            }
        }
    } else {
        uint32_t mine = 0;
        for (uint32_t s = tid; s < T; s += kSmallThreads) mine += L.of[s];
        if (mine) atomicAdd(&L.kept, mine);
        for (uint32_t s = tid; s < T; s += kSmallThreads) {
            if (!L.of[s]) continue;
            uint32_t rank = 0;
            for (uint32_t t = 0; t < T; ++t) rank += (L.of[t] && less(t, s)) ? 1u : 0u;
            put(rank, s);
        }
    }
    __syncthreads();
    return L.kept;
}

// The whole gate in one workgroup. Input: n = counts[src] entries (key words
// kin[w * cin + i], amplitudes ain[i]); output: the sorted kept results at kout /
// aout (capacity cout) and their count at counts[dst]. W: the state's key words.
template <int W>
__global__ __launch_bounds__(kSmallThreads) void sparse_small(const uint64_t* __restrict__ kin,
                                                              const double2* __restrict__ ain, uint64_t cin,
                                                              uint64_t* __restrict__ counts, int src, int dst,
                                                              uint64_t* __restrict__ kout, double2* __restrict__ aout,
                                                              uint64_t cout, const SparseGate g) {
    __shared__ SmallLds L;
    const uint64_t n64 = counts[src];
    if (n64 > kSmallIn || n64 * (uint64_t)g.M > kSparseSmallCap || g.W != W) {  // the host's bound was wrong: report, change nothing
        if (threadIdx.x == 0) counts[kErrWord] = 1;
        return;
    }
    const uint32_t kept = small_gate<kSparseMaxM, W, false>(
        g, g.U ? g.U : g.Uin, (uint32_t)n64, L, [&](int w, uint32_t i) { return kin[w * cin + i]; },
        [&](uint32_t i) { return ain[i]; },
        [&](uint32_t rank, uint32_t s) {
            for (int w = 0; w < W; ++w) kout[w * cout + rank] = L.ok[w][s];
            aout[rank] = L.oa[s];
        });
    if (threadIdx.x == 0) counts[dst] = kept;
}

// A run of gates in one workgroup, the entries held in LDS from the first gate
// to the last: the same steps as sparse_small per gate (so the same bits),
// without a launch per gate. gl: the run's gates in device memory, matrices
// inline. The host's bound keeps every gate of the run within the one-workgroup
// limits; if one were not, the run stops with the error word set. W: the state's
// key words.
template <int W>
__global__ __launch_bounds__(kSmallThreads) void sparse_small_run(const uint64_t* __restrict__ kin,
                                                                  const double2* __restrict__ ain, uint64_t cin,
                                                                  uint64_t* __restrict__ counts, int src, int dst,
                                                                  uint64_t* __restrict__ kout,
                                                                  double2* __restrict__ aout, uint64_t cout,
                                                                  const SparseGate* __restrict__ gl, int ng) {
    __shared__ SmallLds L;
    __shared__ uint64_t sk[kKeyWords][kSparseSmallCap];  // the current entries
    __shared__ double2 sa[kSparseSmallCap];
    // The gate records, staged kRunChunk at a time with coalesced loads: read
    // from device memory, every field a gate uses would be a dependent scalar
    // load that misses, several per gate.
    __shared__ __align__(16) SparseGate sg[kRunChunk];
    const uint32_t tid = threadIdx.x;
    uint64_t n64 = counts[src];
    if (n64 > kSparseSmallCap) {
        if (tid == 0) counts[kErrWord] = 1;
        return;
    }
    uint32_t n = (uint32_t)n64;
    for (uint32_t i = tid; i < n; i += kSmallThreads) {
        for (int w = 0; w < W; ++w) sk[w][i] = kin[w * cin + i];
        sa[i] = ain[i];
    }
    __syncthreads();
    for (int gi = 0; gi < ng; ++gi) {
        if (gi % kRunChunk == 0) {
            const int c = ng - gi < kRunChunk ? ng - gi : kRunChunk;
            const uint32_t words = (uint32_t)(c * sizeof(SparseGate) / 16);
            const U64x2* src = reinterpret_cast<const U64x2*>(gl + gi);
            U64x2* dst = reinterpret_cast<U64x2*>(sg);
            // kStage loads in flight per thread before the first store.
            constexpr int kStage = 8;
            for (uint32_t i0 = tid; i0 < words; i0 += kSmallThreads * kStage) {
                U64x2 v[kStage];
#pragma unroll
                for (int u = 0; u < kStage; ++u)
                    if (i0 + u * kSmallThreads < words) v[u] = src[i0 + u * kSmallThreads];
#pragma unroll
                for (int u = 0; u < kStage; ++u)
                    if (i0 + u * kSmallThreads < words) dst[i0 + u * kSmallThreads] = v[u];
            }
            __syncthreads();
        }
        const SparseGate& g = sg[gi % kRunChunk];
        if (n > kSmallIn || g.M > kSparseInlineM || g.W != W || (uint64_t)n * (uint64_t)g.M > kSparseSmallCap) {
            if (tid == 0) counts[kErrWord] = 1;
            return;
        }
        n = small_gate<kSparseInlineM, W, true>(
            g, g.Uin, n, L, [&](int w, uint32_t i) { return sk[w][i]; }, [&](uint32_t i) { return sa[i]; },
            [&](uint32_t rank, uint32_t s) {
                for (int w = 0; w < W; ++w) sk[w][rank] = L.ok[w][s];
                sa[rank] = L.oa[s];
            });
    }
    for (uint32_t i = tid; i < n; i += kSmallThreads) {
        for (int w = 0; w < W; ++w) kout[w * cout + i] = sk[w][i];
        aout[i] = sa[i];
    }
    if (tid == 0) counts[dst] = n;
}

// ---- the multi-kernel form ------------------------------------------------------

__global__ void wide_classify(const uint64_t* __restrict__ kin, uint64_t cin, uint32_t n, const SparseGate g,
                              uint64_t* __restrict__ gk, int32_t* __restrict__ la, uint32_t* __restrict__ idx) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint64_t key[kKeyWords] = {0, 0, 0};
    for (int w = 0; w < g.W; ++w) key[w] = kin[w * cin + i];
    la[i] = classify(g, key);
    for (int w = 0; w < g.W; ++w) gk[(uint64_t)w * n + i] = key[w];
    idx[i] = i;
}

__global__ void gather_u64(const uint32_t* __restrict__ perm, const uint64_t* __restrict__ src, uint32_t n,
                           uint64_t* __restrict__ dst) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[perm[i]];
}

// Thread i (a position in group order) fills output slots i * M .. i * M + M - 1
// when it is its group's first entry.
__global__ void wide_classes(const uint64_t* __restrict__ sg, const uint32_t* __restrict__ sidx, uint32_t n,
                             const int32_t* __restrict__ la, const double2* __restrict__ ain,
                             const double2* __restrict__ U, const SparseGate g, uint64_t* __restrict__ okeys,
                             double2* __restrict__ oamps, uint8_t* __restrict__ oflag) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int W = g.W, M = g.M;
    const uint64_t T = (uint64_t)n * (uint64_t)M;
    const uint64_t o = (uint64_t)i * (uint64_t)M;
    for (int r = 0; r < M; ++r) oflag[o + r] = 0;
    auto same = [&](uint32_t a, uint32_t b) {
        for (int w = 0; w < W; ++w)
            if (sg[(uint64_t)w * n + a] != sg[(uint64_t)w * n + b]) return false;
        return true;
    };
    if (i > 0 && same(i - 1, i)) return;  // not the group's first entry
    const uint32_t e0 = sidx[i];
    if (la[e0] < 0) {  // controls fail: unchanged
        for (int w = 0; w < W; ++w) okeys[(uint64_t)w * T + o] = sg[(uint64_t)w * n + i];
        oamps[o] = ain[e0];
        oflag[o] = 1;
        return;
    }
    double2 x[kSparseMaxM];
    for (int a = 0; a < kSparseMaxM; ++a) x[a] = double2{0.0, 0.0};
    uint32_t present = 0;
    for (uint32_t j = i; j < n && same(i, j); ++j) {
        const uint32_t e = sidx[j];
        set_member(x, la[e], ain[e]);
        present |= 1u << la[e];
    }
    for (int r = 0; r < M; ++r) {
        const double2 y = class_row(U, x, present, r, M);
        for (int w = 0; w < W; ++w) okeys[(uint64_t)w * T + o + r] = sg[(uint64_t)w * n + i] + g.off[r][w];
        oamps[o + r] = y;
        oflag[o + r] = (y.x != 0.0 || y.y != 0.0) ? 1 : 0;
    }
}

__global__ void gather_entries(const uint32_t* __restrict__ perm, const uint64_t* __restrict__ okeys,
                               const double2* __restrict__ oamps, uint32_t m, uint64_t T, int W,
                               uint64_t* __restrict__ kout, uint64_t cout, double2* __restrict__ aout) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const uint32_t p = perm[i];
    for (int w = 0; w < W; ++w) kout[(uint64_t)w * cout + i] = okeys[(uint64_t)w * T + p];
    aout[i] = oamps[p];
}

__global__ void iota_u32(uint32_t* __restrict__ p, uint32_t n) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = i;
}

__global__ void set_count(uint64_t* __restrict__ counts, int dst, uint64_t v) {
    if (threadIdx.x == 0) counts[dst] = v;
}

// |0...0>: every key word 0, amplitude 1; counts {1, 0, no error}.
__global__ void sparse_basis(uint64_t* __restrict__ keys, double2* __restrict__ amps, int W, uint64_t cap,
                             uint64_t* __restrict__ counts) {
    if (threadIdx.x != 0) return;
    for (int w = 0; w < W; ++w) keys[(uint64_t)w * cap] = 0;
    amps[0] = double2{1.0, 0.0};
    counts[0] = 1;
    counts[1] = 0;
    counts[kErrWord] = 0;
}

unsigned blocks(uint64_t n) { return (unsigned)((n + 255) / 256); }

size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

// Carves 256-byte aligned pieces out of one buffer (first pass: only sums the sizes).
struct Carver {
    unsigned char* base;
    size_t used = 0;
    template <typename T>
    T* take(size_t bytes) {
        T* p = base ? reinterpret_cast<T*>(base + used) : nullptr;
        used += up256(bytes ? bytes : 1);
        return p;
    }
};

// Grow-only device buffer; the stream is drained before the old one is freed.
hipError_t grow(void** buf, size_t* have, size_t need, hipStream_t st) {
    if (*have >= need) return hipSuccess;
    hipError_t e;
    if (*buf && (e = hipStreamSynchronize(st)) != hipSuccess) return e;
    void* p = nullptr;
    const size_t want = need + need / 2;
    if ((e = hipMalloc(&p, want)) != hipSuccess) return e;
    if (*buf) (void)hipFree(*buf);
    *buf = p;
    *have = want;
    return hipSuccess;
}

hipError_t grow_slot(SparseData& d, int i, uint64_t entries) {
    if (d.slot_cap[i] >= entries) return hipSuccess;
    size_t have = d.slot[i] ? slot_bytes(d.W, d.slot_cap[i]) : 0;
    const uint64_t cap = std::max<uint64_t>(entries + entries / 2, kSparseSmallCap);
    hipError_t e = grow(&d.slot[i], &have, slot_bytes(d.W, cap), d.stream);
    if (e != hipSuccess) return e;
    d.slot_cap[i] = cap;
    return hipSuccess;
}

#define QD_TRY(x)                            \
    do {                                     \
        hipError_t e_ = (x);                 \
        if (e_ != hipSuccess) return e_;     \
    } while (0)

hipError_t apply_small(SparseData& d, const SparseGate& g) {
    const int nxt = d.cur ^ 1;
    hipLaunchKernelGGL(d.W == 1 ? sparse_small<1> : d.W == 2 ? sparse_small<2> : sparse_small<3>, dim3(1),
                       dim3(kSmallThreads), 0, d.stream, slot_keys(d.slot[d.cur]),
                       slot_amps(d.slot[d.cur], d.W, d.slot_cap[d.cur]), d.slot_cap[d.cur], d.nnz_dev, d.cur, nxt,
                       slot_keys(d.slot[nxt]), slot_amps(d.slot[nxt], d.W, d.slot_cap[nxt]), d.slot_cap[nxt], g);
    QD_TRY(hipGetLastError());
    d.cur = nxt;
    return hipSuccess;
}

// A run of one-workgroup gates (matrices inline) in one launch.
hipError_t apply_run(SparseData& d, const std::vector<SparseGate>& run) {
    const size_t bytes = run.size() * sizeof(SparseGate);
    if (d.rev_pending) {  // the previous run's records may still be on their way to the device
        QD_TRY(hipEventSynchronize(d.rev));
        d.rev_pending = false;
    }
    if (d.rhost_gates < run.size()) {
        if (d.rhost) QD_TRY(hipHostFree(d.rhost));
        d.rhost = nullptr;
        d.rhost_gates = 0;
        const size_t want = run.size() + run.size() / 2 + 16;
        QD_TRY(hipHostMalloc(reinterpret_cast<void**>(&d.rhost), want * sizeof(SparseGate), hipHostMallocDefault));
        d.rhost_gates = want;
    }
    std::memcpy(d.rhost, run.data(), bytes);
    QD_TRY(grow(&d.rdev, &d.rdev_bytes, bytes, d.stream));
    QD_TRY(hipMemcpyAsync(d.rdev, d.rhost, bytes, hipMemcpyHostToDevice, d.stream));
    QD_TRY(hipEventRecord(d.rev, d.stream));
    d.rev_pending = true;
    const int nxt = d.cur ^ 1;
    hipLaunchKernelGGL(d.W == 1 ? sparse_small_run<1> : d.W == 2 ? sparse_small_run<2> : sparse_small_run<3>,
                       dim3(1), dim3(kSmallThreads), 0, d.stream, slot_keys(d.slot[d.cur]),
                       slot_amps(d.slot[d.cur], d.W, d.slot_cap[d.cur]), d.slot_cap[d.cur], d.nnz_dev, d.cur, nxt,
                       slot_keys(d.slot[nxt]), slot_amps(d.slot[nxt], d.W, d.slot_cap[nxt]), d.slot_cap[nxt],
                       static_cast<const SparseGate*>(d.rdev), (int)run.size());
    QD_TRY(hipGetLastError());
    d.cur = nxt;
    return hipSuccess;
}

// n = the exact entry count (> 0). Reads the kept count back once.
hipError_t apply_wide(SparseData& d, SparseGate g, uint32_t n) {
    const int W = d.W, M = g.M;
    const uint64_t T = (uint64_t)n * (uint64_t)M;
    hipStream_t st = d.stream;
    size_t tb_n = 0, tb_sel = 0, tb_T = 0;
    QD_TRY(hipcub::DeviceRadixSort::SortPairs(nullptr, tb_n, (uint64_t*)nullptr, (uint64_t*)nullptr,
                                              (uint32_t*)nullptr, (uint32_t*)nullptr, (int)n));
    QD_TRY(hipcub::DeviceSelect::Flagged(nullptr, tb_sel, (uint32_t*)nullptr, (uint8_t*)nullptr,
                                         (uint32_t*)nullptr, (int*)nullptr, (int)T));
    QD_TRY(hipcub::DeviceRadixSort::SortPairs(nullptr, tb_T, (uint64_t*)nullptr, (uint64_t*)nullptr,
                                              (uint32_t*)nullptr, (uint32_t*)nullptr, (int)T));
    const size_t tb = std::max(tb_n, std::max(tb_sel, tb_T));
    struct Parts {
        uint64_t *gk, *sg, *tk0, *tk1, *okeys;
        int32_t* la;
        uint32_t *pA, *pB, *pos;
        double2 *dU, *oamps;
        uint8_t* oflag;
        int* nsel;
        void* temp;
    } p;
    auto carve = [&](Carver& c) {
        p.gk = c.take<uint64_t>((size_t)W * n * 8);
        p.sg = c.take<uint64_t>((size_t)W * n * 8);
        p.tk0 = c.take<uint64_t>(T * 8);
        p.tk1 = c.take<uint64_t>(T * 8);
        p.okeys = c.take<uint64_t>((size_t)W * T * 8);
        p.la = c.take<int32_t>((size_t)n * 4);
        p.pA = c.take<uint32_t>(T * 4);
        p.pB = c.take<uint32_t>(T * 4);
        p.pos = c.take<uint32_t>(T * 4);
        p.dU = c.take<double2>((size_t)M * M * 16);
        p.oamps = c.take<double2>(T * 16);
        p.oflag = c.take<uint8_t>(T);
        p.nsel = c.take<int>(sizeof(int));
        p.temp = c.take<void>(tb);
    };
    Carver sizing{nullptr};
    carve(sizing);
    QD_TRY(grow(&d.work, &d.work_bytes, sizing.used, st));
    Carver c{static_cast<unsigned char*>(d.work)};
    carve(c);

    const uint64_t* kin = slot_keys(d.slot[d.cur]);
    const double2* ain = slot_amps(d.slot[d.cur], W, d.slot_cap[d.cur]);
    QD_TRY(hipMemcpyAsync(p.dU, g.U, (size_t)M * M * 16, hipMemcpyHostToDevice, st));
    g.U = p.dU;
    hipLaunchKernelGGL(wide_classify, dim3(blocks(n)), dim3(256), 0, st, kin, d.slot_cap[d.cur], n, g, p.gk, p.la,
                       p.pA);
    QD_TRY(hipGetLastError());
    // Group order: stable sorts by the group words, least significant word first.
    for (int w = 0; w < W; ++w) {
        const uint64_t* kw = p.gk + (size_t)w * n;
        if (w > 0) {
            hipLaunchKernelGGL(gather_u64, dim3(blocks(n)), dim3(256), 0, st, p.pA, kw, n, p.tk0);
            QD_TRY(hipGetLastError());
            kw = p.tk0;
        }
        size_t t = tb;
        QD_TRY(hipcub::DeviceRadixSort::SortPairs(p.temp, t, kw, p.tk1, p.pA, p.pB, (int)n, 0, 64, st));
        std::swap(p.pA, p.pB);
    }
    for (int w = 0; w < W; ++w) {
        hipLaunchKernelGGL(gather_u64, dim3(blocks(n)), dim3(256), 0, st, p.pA, p.gk + (size_t)w * n, n,
                           p.sg + (size_t)w * n);
        QD_TRY(hipGetLastError());
    }
    hipLaunchKernelGGL(wide_classes, dim3(blocks(n)), dim3(256), 0, st, p.sg, p.pA, n, p.la, ain, p.dU, g, p.okeys,
                       p.oamps, p.oflag);
    QD_TRY(hipGetLastError());
    hipLaunchKernelGGL(iota_u32, dim3(blocks(T)), dim3(256), 0, st, p.pos, (uint32_t)T);
    QD_TRY(hipGetLastError());
    size_t t = tb;
    QD_TRY(hipcub::DeviceSelect::Flagged(p.temp, t, p.pos, p.oflag, p.pB, p.nsel, (int)T, st));
    int h_sel = 0;
    QD_TRY(hipMemcpyAsync(&h_sel, p.nsel, sizeof(int), hipMemcpyDeviceToHost, st));
    QD_TRY(hipStreamSynchronize(st));  // the one read-back of the multi-kernel form
    const uint32_t m = (uint32_t)h_sel;

    const int nxt = d.cur ^ 1;
    QD_TRY(grow_slot(d, nxt, m));
    if (m > 0) {
        uint32_t* perm = p.pB;
        uint32_t* spare = p.pA;
        for (int w = 0; w < W; ++w) {
            hipLaunchKernelGGL(gather_u64, dim3(blocks(m)), dim3(256), 0, st, perm, p.okeys + (size_t)w * T, m,
                               p.tk0);
            QD_TRY(hipGetLastError());
            size_t t3 = tb;
            QD_TRY(hipcub::DeviceRadixSort::SortPairs(p.temp, t3, p.tk0, p.tk1, perm, spare, (int)m, 0, 64, st));
            std::swap(perm, spare);
        }
        hipLaunchKernelGGL(gather_entries, dim3(blocks(m)), dim3(256), 0, st, perm, p.okeys, p.oamps, m, T, W,
                           slot_keys(d.slot[nxt]), d.slot_cap[nxt], slot_amps(d.slot[nxt], W, d.slot_cap[nxt]));
        QD_TRY(hipGetLastError());
    }
    hipLaunchKernelGGL(set_count, dim3(1), dim3(64), 0, st, d.nnz_dev, nxt, (uint64_t)m);
    QD_TRY(hipGetLastError());
    d.cur = nxt;
    d.bound = m;
    d.exact = true;
    return hipSuccess;
}

}  // namespace

hipError_t sparse_init(SparseData& d, int W) {
    d.W = W;
    hipError_t e;
    for (int i = 0; i < 2; ++i)
        if ((e = grow_slot(d, i, kSparseSmallCap)) != hipSuccess) return e;
    size_t have = 0;
    void* counts = nullptr;
    if ((e = grow(&counts, &have, 3 * sizeof(uint64_t), d.stream)) != hipSuccess) return e;
    d.nnz_dev = static_cast<uint64_t*>(counts);
    if ((e = hipHostMalloc(reinterpret_cast<void**>(&d.uhost),
                           sizeof(double2) * kSparseMaxM * kSparseMaxM * SparseData::kURing, hipHostMallocDefault)) !=
        hipSuccess) {
        d.uhost = nullptr;
        return e;
    }
    void* udev = nullptr;
    if ((e = hipHostGetDevicePointer(&udev, d.uhost, 0)) != hipSuccess) return e;
    d.udev = static_cast<double2*>(udev);
    for (int i = 0; i < SparseData::kURing; ++i)
        if ((e = hipEventCreateWithFlags(&d.uev[i], hipEventDisableTiming)) != hipSuccess) return e;
    if ((e = hipEventCreateWithFlags(&d.rev, hipEventDisableTiming)) != hipSuccess) return e;
    // Staging for the gate records of runs, sized for kRunInitGates (longer
    // lists grow it), so that a new state's first gate list allocates nothing.
    if ((e = hipHostMalloc(reinterpret_cast<void**>(&d.rhost), kRunInitGates * sizeof(SparseGate),
                           hipHostMallocDefault)) != hipSuccess) {
        d.rhost = nullptr;
        return e;
    }
    d.rhost_gates = kRunInitGates;
    if ((e = grow(&d.rdev, &d.rdev_bytes, kRunInitGates * sizeof(SparseGate), d.stream)) != hipSuccess) return e;
    hipLaunchKernelGGL(sparse_basis, dim3(1), dim3(64), 0, d.stream, slot_keys(d.slot[0]),
                       slot_amps(d.slot[0], W, d.slot_cap[0]), W, d.slot_cap[0], d.nnz_dev);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    d.cur = 0;
    d.bound = 1;
    d.exact = true;
    return hipStreamSynchronize(d.stream);
}

void sparse_release(SparseData& d) {
    (void)hipStreamSynchronize(d.stream);
    for (int i = 0; i < 2; ++i)
        if (d.slot[i]) (void)hipFree(d.slot[i]);
    if (d.work) (void)hipFree(d.work);
    if (d.rdev) (void)hipFree(d.rdev);
    if (d.rhost) (void)hipHostFree(d.rhost);
    if (d.rev) (void)hipEventDestroy(d.rev);
    if (d.nnz_dev) (void)hipFree(d.nnz_dev);
    for (int i = 0; i < SparseData::kURing; ++i)
        if (d.uev[i]) (void)hipEventDestroy(d.uev[i]);
    if (d.uhost) (void)hipHostFree(d.uhost);
    d = SparseData{};
}

hipError_t sparse_count(SparseData& d, uint64_t* nnz) {
    QD_TRY(hipStreamSynchronize(d.stream));
    uint64_t h[3] = {0, 0, 0};
    QD_TRY(hipMemcpy(h, d.nnz_dev, sizeof h, hipMemcpyDeviceToHost));
    if (h[kErrWord]) return hipErrorIllegalState;  // a small gate found more entries than the host planned for
    *nnz = h[d.cur];
    d.bound = *nnz;
    d.exact = true;
    return hipSuccess;
}

hipError_t sparse_apply(SparseData& d, const SparseGate& g0, const double* U, bool cols_single) {
    const uint64_t M = (uint64_t)g0.M;
    if (d.bound > kSparseSmallCap / M && !d.exact) {
        uint64_t n = 0;
        QD_TRY(sparse_count(d, &n));
    }
    if (d.bound == 0) return hipSuccess;  // no entries: nothing to do
    const bool small = d.bound <= kSparseSmallCap / M;
    if (!small && d.bound * M > (uint64_t)INT32_MAX) return hipErrorNotSupported;  // hipCUB counts items in int
    if (small && M <= (uint64_t)kSparseInlineM) {  // U in the kernel arguments: nothing to stage
        SparseGate g = g0;
        g.U = nullptr;
        std::memcpy(g.Uin, U, M * M * sizeof(double2));
        QD_TRY(apply_small(d, g));
        d.bound = cols_single ? d.bound : d.bound * M;
        d.exact = false;
        return hipSuccess;
    }
    // Stage U in the pinned ring (the slot's previous gate has finished once its event has).
    const int slot = (int)(d.uses % SparseData::kURing);
    if (d.uses >= (uint64_t)SparseData::kURing) QD_TRY(hipEventSynchronize(d.uev[slot]));
    double2* uh = d.uhost + (size_t)slot * kSparseMaxM * kSparseMaxM;
    std::memcpy(uh, U, M * M * sizeof(double2));
    SparseGate g = g0;
    g.U = d.udev + (uh - d.uhost);
    hipError_t e;
    if (small) {
        e = apply_small(d, g);
        if (e == hipSuccess) {
            d.bound = cols_single ? d.bound : d.bound * M;
            d.exact = false;
        }
    } else {
        g.U = uh;  // copied to device memory by the multi-kernel form
        e = apply_wide(d, g, (uint32_t)d.bound);
    }
    // Whatever was enqueued may still read the staged matrix: the slot is
    // reused only after this event.
    const hipError_t er = hipEventRecord(d.uev[slot], d.stream);
    ++d.uses;
    return e != hipSuccess ? e : er;
}

hipError_t sparse_apply_list(SparseData& d, const SparseGate* gates, const double* const* U, const bool* cols_single,
                             int count) {
    std::vector<SparseGate> run;
    int i = 0;
    while (i < count) {
        // The longest run from gate i that the bound keeps in the one-workgroup
        // form (the test sparse_apply makes per gate), matrices inline.
        run.clear();
        uint64_t b = d.bound;
        int j = i;
        while (j < count && b != 0) {
            const uint64_t M = (uint64_t)gates[j].M;
            if (M > (uint64_t)kSparseInlineM || b > kSparseSmallCap / M) break;
            SparseGate g = gates[j];
            g.U = nullptr;
            std::memcpy(g.Uin, U[j], M * M * sizeof(double2));
            run.push_back(g);
            b = cols_single[j] ? b : b * M;
            ++j;
        }
        if (run.size() >= 2) {
            QD_TRY(apply_run(d, run));
            d.bound = b;
            d.exact = false;
            i = j;
        } else {
            QD_TRY(sparse_apply(d, gates[i], U[i], cols_single[i]));
            ++i;
        }
    }
    return hipSuccess;
}

#undef QD_TRY

}  // namespace qd
