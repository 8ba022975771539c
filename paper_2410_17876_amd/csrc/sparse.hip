// sparse.hip - a gate on a sparse statevector (sparse.h).
//
// 1. classify: for every entry, its class base (the key with the target digits
//    set to 0) and local index when the controls hold (Sec. 2.3, 2.4); an entry
//    whose controls fail is its own one-member group (local index -1). A
//    control-failing key never equals the base of a class whose controls hold
//    (they differ in a control digit), so groups never mix the two.
// 2. radix-sort the entries by group key (hipCUB).
// 3. one thread per group head: gather the class's present members (missing
//    ones are 0), y = U x, write the M results with their keys, flag the
//    nonzero ones (a control-failing entry is copied unchanged).
// 4. keep the flagged results and sort them by key.
#include <hip/hip_runtime.h>

#include <hipcub/hipcub.hpp>

#include "sparse.h"

namespace qd {

namespace {

__global__ void sparse_classify(const uint64_t* __restrict__ keys, uint64_t n, const SparseGate g,
                                uint64_t* __restrict__ group, int32_t* __restrict__ local,
                                uint32_t* __restrict__ idx) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t key = keys[i];
    bool hold = true;
    for (int l = 0; l < g.m; ++l)
        if ((key / g.cs[l]) % g.cd[l] != g.cv[l]) hold = false;
    if (hold) {
        int a = 0, w = 1;
        uint64_t base = key;
        for (int l = 0; l < g.k; ++l) {
            const uint64_t dg = (key / g.ts[l]) % g.td[l];
            a += (int)dg * w;
            w *= (int)g.td[l];
            base -= dg * g.ts[l];
        }
        group[i] = base;
        local[i] = a;
    } else {
        group[i] = key;
        local[i] = -1;
    }
    idx[i] = (uint32_t)i;
}

// Thread i owns output slots i * M .. i * M + M - 1.
__global__ void sparse_classes(const uint64_t* __restrict__ sgroup, const uint32_t* __restrict__ sidx, uint64_t n,
                               const int32_t* __restrict__ local, const double2* __restrict__ amps,
                               const double2* __restrict__ U, const SparseGate g, uint64_t* __restrict__ okeys,
                               double2* __restrict__ oamps, uint8_t* __restrict__ oflag) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int M = g.M;
    uint8_t* flag = oflag + i * M;
    for (int r = 0; r < M; ++r) flag[r] = 0;
    const uint64_t gk = sgroup[i];
    if (i > 0 && sgroup[i - 1] == gk) return;  // not the group's first entry
    const uint32_t e0 = sidx[i];
    if (local[e0] < 0) {  // controls fail: unchanged
        okeys[i * M] = gk;
        oamps[i * M] = amps[e0];
        flag[0] = 1;
        return;
    }
    double2 x[kSparseMaxM];
    for (int a = 0; a < M; ++a) x[a] = double2{0.0, 0.0};
    for (uint64_t j = i; j < n && sgroup[j] == gk; ++j) {
        const uint32_t e = sidx[j];
        x[local[e]] = amps[e];
    }
    {
        // Textbook complex products, no FMA contraction: which results are
        // exactly zero (and dropped) then does not depend on how the compiler
        // fuses them.
#pragma clang fp contract(off)
        for (int r = 0; r < M; ++r) {
            double yr = 0.0, yi = 0.0;
            for (int a = 0; a < M; ++a) {
                const double2 u = U[r * M + a];
                yr = yr + (u.x * x[a].x - u.y * x[a].y);
                yi = yi + (u.x * x[a].y + u.y * x[a].x);
            }
            okeys[i * M + r] = gk + g.off[r];
            oamps[i * M + r] = double2{yr, yi};
            flag[r] = (yr != 0.0 || yi != 0.0) ? 1 : 0;
        }
    }
}

__global__ void gather_amps(const uint32_t* __restrict__ perm, const double2* __restrict__ src, uint64_t n,
                            double2* __restrict__ dst) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[perm[i]];
}

__global__ void iota_u32(uint32_t* p, uint64_t n) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = (uint32_t)i;
}

// Device buffers freed on scope exit.
struct Pool {
    void* p[32] = {};  // one gate takes 19 buffers
    int n = 0;
    hipError_t get(void** out, size_t bytes) {
        *out = nullptr;
        hipError_t e = hipMalloc(out, bytes ? bytes : 1);
        if (e == hipSuccess) p[n++] = *out;
        return e;
    }
    void release(void* q) {
        for (int i = 0; i < n; ++i)
            if (p[i] == q) p[i] = nullptr;
    }
    ~Pool() {
        for (int i = 0; i < n; ++i)
            if (p[i]) (void)hipFree(p[i]);
    }
};

unsigned blocks(uint64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

hipError_t sparse_apply(SparseData& d, const SparseGate& g, const double* U) {
    const uint64_t n = d.nnz;
    if (n == 0) return hipSuccess;
    if (n > 0xFFFFFFFFull / (uint64_t)g.M) return hipErrorInvalidValue;
    Pool pool;
    hipError_t e;
    uint64_t *group, *sgroup;
    int32_t* local;
    uint32_t *idx, *sidx;
    double2* dU;
#define QD_TRY(x) \
    if ((e = (x)) != hipSuccess) return e
    QD_TRY(pool.get((void**)&group, n * 8));
    QD_TRY(pool.get((void**)&sgroup, n * 8));
    QD_TRY(pool.get((void**)&local, n * 4));
    QD_TRY(pool.get((void**)&idx, n * 4));
    QD_TRY(pool.get((void**)&sidx, n * 4));
    QD_TRY(pool.get((void**)&dU, (size_t)g.M * g.M * 16));
    QD_TRY(hipMemcpy(dU, U, (size_t)g.M * g.M * 16, hipMemcpyHostToDevice));
    hipLaunchKernelGGL(sparse_classify, dim3(blocks(n)), dim3(256), 0, 0, d.keys, n, g, group, local, idx);
    QD_TRY(hipGetLastError());
    size_t tb = 0;
    void* temp = nullptr;
    QD_TRY(hipcub::DeviceRadixSort::SortPairs(nullptr, tb, group, sgroup, idx, sidx, (int)n));
    QD_TRY(pool.get(&temp, tb));
    QD_TRY(hipcub::DeviceRadixSort::SortPairs(temp, tb, group, sgroup, idx, sidx, (int)n));

    const uint64_t cap = n * (uint64_t)g.M;
    uint64_t* okeys;
    double2* oamps;
    uint8_t* oflag;
    QD_TRY(pool.get((void**)&okeys, cap * 8));
    QD_TRY(pool.get((void**)&oamps, cap * 16));
    QD_TRY(pool.get((void**)&oflag, cap));
    hipLaunchKernelGGL(sparse_classes, dim3(blocks(n)), dim3(256), 0, 0, sgroup, sidx, n, local, d.amps, dU, g,
                       okeys, oamps, oflag);
    QD_TRY(hipGetLastError());

    // Keep the flagged results: keys with their positions, then the positions sorted by key.
    uint32_t *pos, *kpos, *spos;
    uint64_t* kkeys;
    int* nsel;
    QD_TRY(pool.get((void**)&pos, cap * 4));
    QD_TRY(pool.get((void**)&kpos, cap * 4));
    QD_TRY(pool.get((void**)&kkeys, cap * 8));
    QD_TRY(pool.get((void**)&nsel, sizeof(int)));
    hipLaunchKernelGGL(iota_u32, dim3(blocks(cap)), dim3(256), 0, 0, pos, cap);
    QD_TRY(hipGetLastError());
    size_t tb2 = 0;
    void* temp2 = nullptr;
    QD_TRY(hipcub::DeviceSelect::Flagged(nullptr, tb2, okeys, oflag, kkeys, nsel, (int)cap));
    QD_TRY(pool.get(&temp2, tb2));
    QD_TRY(hipcub::DeviceSelect::Flagged(temp2, tb2, okeys, oflag, kkeys, nsel, (int)cap));
    QD_TRY(hipcub::DeviceSelect::Flagged(temp2, tb2, pos, oflag, kpos, nsel, (int)cap));
    int h_sel = 0;
    QD_TRY(hipMemcpy(&h_sel, nsel, sizeof(int), hipMemcpyDeviceToHost));
    const uint64_t m = (uint64_t)h_sel;

    uint64_t* nkeys;
    double2* namps;
    void* nk = nullptr;
    void* na = nullptr;
    QD_TRY(pool.get(&nk, m * 8));
    QD_TRY(pool.get(&na, m * 16));
    nkeys = static_cast<uint64_t*>(nk);
    namps = static_cast<double2*>(na);
    if (m > 0) {
        QD_TRY(pool.get((void**)&spos, m * 4));
        size_t tb3 = 0;
        void* temp3 = nullptr;
        QD_TRY(hipcub::DeviceRadixSort::SortPairs(nullptr, tb3, kkeys, nkeys, kpos, spos, (int)m));
        QD_TRY(pool.get(&temp3, tb3));
        QD_TRY(hipcub::DeviceRadixSort::SortPairs(temp3, tb3, kkeys, nkeys, kpos, spos, (int)m));
        hipLaunchKernelGGL(gather_amps, dim3(blocks(m)), dim3(256), 0, 0, spos, oamps, m, namps);
        QD_TRY(hipGetLastError());
    }
    QD_TRY(hipDeviceSynchronize());
#undef QD_TRY
    // Success: the new arrays replace the old ones.
    pool.release(nk);
    pool.release(na);
    (void)hipFree(d.keys);
    (void)hipFree(d.amps);
    d.keys = nkeys;
    d.amps = namps;
    d.nnz = m;
    return hipSuccess;
}

}  // namespace qd
