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

#include <algorithm>

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

hipError_t grow(void** buf, size_t* have, size_t need) {
    if (*have >= need) return hipSuccess;
    void* p = nullptr;
    const size_t want = need + need / 2;
    hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess) return e;
    if (*buf) (void)hipFree(*buf);
    *buf = p;
    *have = want;
    return hipSuccess;
}

}  // namespace

hipError_t sparse_init(SparseData& d) {
    size_t have = d.slot_bytes[0];
    hipError_t e = grow(&d.slot[0], &have, 256 + 16);
    if (e != hipSuccess) return e;
    d.slot_bytes[0] = have;
    d.cur = 0;
    d.keys = static_cast<uint64_t*>(d.slot[0]);
    d.amps = reinterpret_cast<double2*>(static_cast<unsigned char*>(d.slot[0]) + 256);
    const uint64_t key0 = 0;
    const double2 amp0{1.0, 0.0};
    if ((e = hipMemcpy(d.keys, &key0, 8, hipMemcpyHostToDevice)) != hipSuccess) return e;
    if ((e = hipMemcpy(d.amps, &amp0, 16, hipMemcpyHostToDevice)) != hipSuccess) return e;
    d.nnz = 1;
    return hipSuccess;
}

void sparse_release(SparseData& d) {
    for (int i = 0; i < 2; ++i)
        if (d.slot[i]) (void)hipFree(d.slot[i]);
    if (d.work) (void)hipFree(d.work);
    d = SparseData{};
}

hipError_t sparse_apply(SparseData& d, const SparseGate& g, const double* U) {
    const uint64_t n = d.nnz;
    if (n == 0) return hipSuccess;
    // hipCUB counts items in int: the M results per entry must stay below 2^31
    if (n > (uint64_t)INT32_MAX / (uint64_t)g.M) return hipErrorInvalidValue;
    const uint64_t cap = n * (uint64_t)g.M;
    hipError_t e;
#define QD_TRY(x) \
    if ((e = (x)) != hipSuccess) return e
    // Temporary storage of the three library calls, at their largest sizes.
    size_t tb_sort1 = 0, tb_sel = 0, tb_sort2 = 0;
    QD_TRY(hipcub::DeviceRadixSort::SortPairs(nullptr, tb_sort1, (uint64_t*)nullptr, (uint64_t*)nullptr,
                                              (uint32_t*)nullptr, (uint32_t*)nullptr, (int)n));
    QD_TRY(hipcub::DeviceSelect::Flagged(nullptr, tb_sel, (uint64_t*)nullptr, (uint8_t*)nullptr,
                                         (uint64_t*)nullptr, (int*)nullptr, (int)cap));
    QD_TRY(hipcub::DeviceRadixSort::SortPairs(nullptr, tb_sort2, (uint64_t*)nullptr, (uint64_t*)nullptr,
                                              (uint32_t*)nullptr, (uint32_t*)nullptr, (int)cap));
    const size_t tb = std::max(tb_sort1, std::max(tb_sel, tb_sort2));
    auto carve = [&](Carver& c, uint64_t** group, uint64_t** sgroup, int32_t** local, uint32_t** idx,
                     uint32_t** sidx, double2** dU, void** temp, uint64_t** okeys, double2** oamps, uint8_t** oflag,
                     uint32_t** pos, uint32_t** kpos, uint32_t** spos, uint64_t** kkeys, int** nsel) {
        *group = c.take<uint64_t>(n * 8);
        *sgroup = c.take<uint64_t>(n * 8);
        *local = c.take<int32_t>(n * 4);
        *idx = c.take<uint32_t>(n * 4);
        *sidx = c.take<uint32_t>(n * 4);
        *dU = c.take<double2>((size_t)g.M * g.M * 16);
        *temp = c.take<void>(tb);
        *okeys = c.take<uint64_t>(cap * 8);
        *oamps = c.take<double2>(cap * 16);
        *oflag = c.take<uint8_t>(cap);
        *pos = c.take<uint32_t>(cap * 4);
        *kpos = c.take<uint32_t>(cap * 4);
        *spos = c.take<uint32_t>(cap * 4);
        *kkeys = c.take<uint64_t>(cap * 8);
        *nsel = c.take<int>(sizeof(int));
    };
    uint64_t *group, *sgroup, *okeys, *kkeys;
    int32_t* local;
    uint32_t *idx, *sidx, *pos, *kpos, *spos;
    double2 *dU, *oamps;
    uint8_t* oflag;
    void* temp;
    int* nsel;
    Carver sizing{nullptr};
    carve(sizing, &group, &sgroup, &local, &idx, &sidx, &dU, &temp, &okeys, &oamps, &oflag, &pos, &kpos, &spos,
          &kkeys, &nsel);
    QD_TRY(grow(&d.work, &d.work_bytes, sizing.used));
    Carver c{static_cast<unsigned char*>(d.work)};
    carve(c, &group, &sgroup, &local, &idx, &sidx, &dU, &temp, &okeys, &oamps, &oflag, &pos, &kpos, &spos, &kkeys,
          &nsel);

    QD_TRY(hipMemcpy(dU, U, (size_t)g.M * g.M * 16, hipMemcpyHostToDevice));
    hipLaunchKernelGGL(sparse_classify, dim3(blocks(n)), dim3(256), 0, 0, d.keys, n, g, group, local, idx);
    QD_TRY(hipGetLastError());
    size_t t1 = tb;
    QD_TRY(hipcub::DeviceRadixSort::SortPairs(temp, t1, group, sgroup, idx, sidx, (int)n));
    hipLaunchKernelGGL(sparse_classes, dim3(blocks(n)), dim3(256), 0, 0, sgroup, sidx, n, local, d.amps, dU, g,
                       okeys, oamps, oflag);
    QD_TRY(hipGetLastError());
    // Keep the flagged results (keys, and their positions), then sort them by key.
    hipLaunchKernelGGL(iota_u32, dim3(blocks(cap)), dim3(256), 0, 0, pos, cap);
    QD_TRY(hipGetLastError());
    size_t t2 = tb;
    QD_TRY(hipcub::DeviceSelect::Flagged(temp, t2, okeys, oflag, kkeys, nsel, (int)cap));
    t2 = tb;
    QD_TRY(hipcub::DeviceSelect::Flagged(temp, t2, pos, oflag, kpos, nsel, (int)cap));
    int h_sel = 0;
    QD_TRY(hipMemcpy(&h_sel, nsel, sizeof(int), hipMemcpyDeviceToHost));
    const uint64_t m = (uint64_t)h_sel;

    // The result goes to the other slot.
    const int nxt = d.cur ^ 1;
    const size_t kbytes = up256(m * 8 + 1);
    QD_TRY(grow(&d.slot[nxt], &d.slot_bytes[nxt], kbytes + m * 16 + 16));
    uint64_t* nkeys = static_cast<uint64_t*>(d.slot[nxt]);
    double2* namps = reinterpret_cast<double2*>(static_cast<unsigned char*>(d.slot[nxt]) + kbytes);
    if (m > 0) {
        size_t t3 = tb;
        QD_TRY(hipcub::DeviceRadixSort::SortPairs(temp, t3, kkeys, nkeys, kpos, spos, (int)m));
        hipLaunchKernelGGL(gather_amps, dim3(blocks(m)), dim3(256), 0, 0, spos, oamps, m, namps);
        QD_TRY(hipGetLastError());
    }
    QD_TRY(hipDeviceSynchronize());
#undef QD_TRY
    d.cur = nxt;
    d.keys = nkeys;
    d.amps = namps;
    d.nnz = m;
    return hipSuccess;
}

}  // namespace qd
