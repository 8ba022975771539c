// abi.cpp - the extern "C" entry points declared in include/qd.h.
//
// Everything here is argument checking, state bookkeeping and marshalling; all
// work on amplitudes runs in the kernels of sweep.hip and reduce.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <memory>
#include <string>
#include <vector>

#include "../../include/qd.h"
#include "fusion.h"
#include "kernels.h"
#include "plan.h"
#include "planner.h"
#include "sparse.h"

using namespace qd;

namespace {

thread_local std::string g_err;

int set_err(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

int hip_err(hipError_t e, const char* what) {
    char buf[256];
    std::snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
    return set_err(QD_ERR_DEVICE, buf);
}

#define QD_HIP(call, what)                        \
    do {                                          \
        hipError_t e_ = (call);                   \
        if (e_ != hipSuccess) return hip_err(e_, what); \
    } while (0)

// Device-side copies of per-gate data that does not fit the kernel arguments
// (large gate matrices, member offsets). A ring of slots in device memory is
// filled from pinned host slots by copies on the state's stream, so a slot is
// only overwritten after every kernel that read it (stream order); the host
// slot is reused only after its copy has finished (event).
struct GateRing {
    static constexpr size_t kSlot = 2u << 20;  // > 343^2 * 16 + 343 * 8
    static constexpr int kSlots = 4;
    unsigned char* host = nullptr;
    unsigned char* dev = nullptr;
    hipEvent_t ev[kSlots] = {};
    bool pending[kSlots] = {};
    int next = 0;

    int ensure() {
        if (dev) return QD_OK;
        if (hipHostMalloc(reinterpret_cast<void**>(&host), kSlot * kSlots, hipHostMallocDefault) != hipSuccess) {
            host = nullptr;
            return set_err(QD_ERR_OUT_OF_MEMORY, "pinned gate staging allocation failed");
        }
        if (hipMalloc(reinterpret_cast<void**>(&dev), kSlot * kSlots) != hipSuccess) {
            (void)hipHostFree(host);
            host = nullptr;
            dev = nullptr;
            return set_err(QD_ERR_OUT_OF_MEMORY, "device gate ring allocation failed");
        }
        for (int i = 0; i < kSlots; ++i) QD_HIP(hipEventCreateWithFlags(&ev[i], hipEventDisableTiming), "event");
        return QD_OK;
    }

    void release() {
        for (int i = 0; i < kSlots; ++i)
            if (ev[i]) (void)hipEventDestroy(ev[i]);
        if (dev) (void)hipFree(dev);
        if (host) (void)hipHostFree(host);
        dev = nullptr;
        host = nullptr;
    }
};

}  // namespace

struct qd_state {
    int n = 0;
    int32_t dims[QD_MAX_QUDITS] = {};
    uint64_t D = 0;
    int precision = 0;
    void* psi = nullptr;
    bool owned = false;
    hipStream_t stream = nullptr;
    int device = 0;
    GateRing ring;
};

namespace {

// Reduction scratch: one buffer per device, shared by every state on it and
// kept until the process ends (freeing device memory synchronises the device,
// which a server retiring many states cannot afford). qd_norm holds the mutex
// for its whole (synchronous) call, so concurrent callers never share it.
constexpr int kMaxDevices = 64;
std::mutex g_red_mu;
double* g_red[kMaxDevices] = {};

}  // namespace

namespace {

int use_device(const qd_state* s) {
    int cur = -1;
    QD_HIP(hipGetDevice(&cur), "hipGetDevice");
    if (cur != s->device) QD_HIP(hipSetDevice(s->device), "hipSetDevice");
    return QD_OK;
}

int check_precision(int32_t precision) {
    if (precision != QD_C64 && precision != QD_C128)
        return set_err(QD_ERR_INVALID_ARGUMENT, "precision must be QD_C64 (1) or QD_C128 (2)");
    return QD_OK;
}

int new_state(const int32_t* dims, int32_t n, int32_t precision, qd_state** out, uint64_t* D) {
    if (!out) return set_err(QD_ERR_INVALID_ARGUMENT, "out is null");
    *out = nullptr;
    std::string err;
    int rc = check_dims(dims, n, D, &err);
    if (rc) return set_err(rc, err);
    rc = check_precision(precision);
    if (rc) return rc;
    const uint64_t ab = amp_bytes(precision);
    if (*D > UINT64_MAX / ab) return set_err(QD_ERR_DIM_OVERFLOW, "state size in bytes overflows");
    qd_state* s = new qd_state();
    s->n = n;
    std::memcpy(s->dims, dims, sizeof(int32_t) * n);
    s->D = *D;
    s->precision = precision;
    int dev = 0;
    if (hipError_t e = hipGetDevice(&dev); e != hipSuccess) {
        delete s;
        return set_err(QD_ERR_DEVICE, std::string("no HIP device available: ") + hipGetErrorString(e));
    }
    s->device = dev;
    *out = s;
    return QD_OK;
}

}  // namespace

extern "C" {

const char* qd_last_error(void) { return g_err.c_str(); }

const char* qd_version(void) { return "libqd 0.1 (gfx950)"; }

int qd_dim(const int32_t* dims, int32_t n, uint64_t* D) {
    std::string err;
    uint64_t d = 0;
    int rc = check_dims(dims, n, &d, &err);
    if (rc) return set_err(rc, err);
    if (!D) return set_err(QD_ERR_INVALID_ARGUMENT, "D is null");
    *D = d;
    return QD_OK;
}

int qd_check_gate(const int32_t* dims, int32_t n, const int32_t* targets, int32_t k, const int32_t* controls,
                  const int32_t* values, int32_t m) {
    std::string err;
    int rc = check_gate(dims, n, targets, k, controls, values, m, &err);
    return rc ? set_err(rc, err) : QD_OK;
}

int qd_gate_info_for(const int32_t* dims, int32_t n, int32_t precision, const int32_t* targets, int32_t k,
                     const int32_t* controls, const int32_t* values, int32_t m, const double* U,
                     qd_gate_info* info) {
    int rc = check_precision(precision);
    if (rc) return rc;
    if (!info) return set_err(QD_ERR_INVALID_ARGUMENT, "info is null");
    GatePlan* p = new GatePlan;
    std::string err;
    rc = plan_gate(dims, n, targets, k, controls, values, m, U, p, &err);
    if (rc == QD_OK) plan_info(*p, precision, info);
    delete p;
    return rc ? set_err(rc, err) : QD_OK;
}

int qd_class_bases(const int32_t* dims, int32_t n, const int32_t* targets, int32_t k, const int32_t* controls,
                   const int32_t* values, int32_t m, uint64_t first, uint64_t count, uint64_t* bases) {
    std::string err;
    int rc = check_gate(dims, n, targets, k, controls, values, m, &err);
    if (rc) return set_err(rc, err);
    if (count && !bases) return set_err(QD_ERR_INVALID_ARGUMENT, "bases is null");
    // The plan's U only decides the category; the decode does not depend on it.
    std::vector<double> eye(2 * kMaxM * kMaxM, 0.0);
    GatePlan* p = new GatePlan;
    rc = plan_gate(dims, n, targets, k, controls, values, m, eye.data(), p, &err);
    if (rc) {
        delete p;
        return set_err(rc, err);
    }
    if (first > p->n_classes || count > p->n_classes - first) {
        delete p;
        return set_err(QD_ERR_INVALID_ARGUMENT, "class range outside 0..classes");
    }
    const bool narrow = p->D < (1ull << 31);
    if (narrow) {
        const Decode<uint32_t> dec = make_decode<uint32_t>(*p);
        for (uint64_t i = 0; i < count; ++i) bases[i] = decode_base<uint32_t>(dec, (uint32_t)(first + i));
    } else {
        const Decode<uint64_t> dec = make_decode<uint64_t>(*p);
        for (uint64_t i = 0; i < count; ++i) bases[i] = decode_base<uint64_t>(dec, first + i);
    }
    delete p;
    return QD_OK;
}

int qd_state_create(const int32_t* dims, int32_t n, int32_t precision, qd_state** out) {
    uint64_t D = 0;
    int rc = new_state(dims, n, precision, out, &D);
    if (rc) return rc;
    qd_state* s = *out;
    const size_t bytes = (size_t)D * amp_bytes(precision);
    if (hipMalloc(&s->psi, bytes) != hipSuccess) {
        (void)hipGetLastError();
        delete s;
        *out = nullptr;
        return set_err(QD_ERR_OUT_OF_MEMORY, "device allocation of the state failed");
    }
    s->owned = true;
    hipError_t e = launch_basis(s->psi, precision, D, 0, s->stream);
    if (e != hipSuccess) {
        (void)hipFree(s->psi);
        delete s;
        *out = nullptr;
        return hip_err(e, "initial state");
    }
    return QD_OK;
}

int qd_state_create_external(const int32_t* dims, int32_t n, int32_t precision, void* device_ptr, uint64_t bytes,
                             qd_state** out) {
    if (!device_ptr) return set_err(QD_ERR_INVALID_ARGUMENT, "device_ptr is null");
    uint64_t D = 0;
    int rc = new_state(dims, n, precision, out, &D);
    if (rc) return rc;
    if (bytes / amp_bytes(precision) < D) {
        delete *out;
        *out = nullptr;
        return set_err(QD_ERR_BUFFER_TOO_SMALL, "external buffer smaller than D amplitudes");
    }
    (*out)->psi = device_ptr;
    (*out)->owned = false;
    return QD_OK;
}

int qd_state_destroy(qd_state* s) {
    if (!s) return QD_OK;
    // Only device memory the state owns needs its pending work to finish first;
    // an external buffer belongs to the caller, whose allocator orders reuse.
    if (s->owned || s->ring.dev) {
        use_device(s);
        (void)hipStreamSynchronize(s->stream);
    }
    s->ring.release();
    if (s->owned && s->psi) (void)hipFree(s->psi);
    delete s;
    return QD_OK;
}

int qd_state_set_stream(qd_state* s, void* hip_stream) {
    if (!s) return set_err(QD_ERR_INVALID_ARGUMENT, "state is null");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    if (st == s->stream) return QD_OK;
    int rc = use_device(s);
    if (rc) return rc;
    QD_HIP(hipStreamSynchronize(s->stream), "synchronizing the previous stream");
    s->stream = st;
    return QD_OK;
}

int qd_state_reset(qd_state* s, uint64_t j) {
    if (!s) return set_err(QD_ERR_INVALID_ARGUMENT, "state is null");
    if (j >= s->D) return set_err(QD_ERR_INVALID_ARGUMENT, "basis index outside 0..D-1");
    int rc = use_device(s);
    if (rc) return rc;
    QD_HIP(launch_basis(s->psi, s->precision, s->D, j, s->stream), "reset");
    return QD_OK;
}

int qd_state_info(const qd_state* s, uint64_t* D, int32_t* precision, void** device_ptr) {
    if (!s) return set_err(QD_ERR_INVALID_ARGUMENT, "state is null");
    if (D) *D = s->D;
    if (precision) *precision = s->precision;
    if (device_ptr) *device_ptr = s->psi;
    return QD_OK;
}

int qd_state_set_amplitudes(qd_state* s, const double* host, uint64_t offset, uint64_t count) {
    if (!s) return set_err(QD_ERR_INVALID_ARGUMENT, "state is null");
    if (count && !host) return set_err(QD_ERR_INVALID_ARGUMENT, "host is null");
    if (offset > s->D || count > s->D - offset) return set_err(QD_ERR_INVALID_ARGUMENT, "range outside the state");
    int rc = use_device(s);
    if (rc) return rc;
    if (s->precision == QD_C128) {
        QD_HIP(hipMemcpyAsync(static_cast<double*>(s->psi) + 2 * offset, host, count * 16, hipMemcpyHostToDevice,
                              s->stream),
               "copy to device");
        QD_HIP(hipStreamSynchronize(s->stream), "copy to device");
        return QD_OK;
    }
    const uint64_t chunk = 1ull << 22;
    std::vector<float> tmp(2 * std::min<uint64_t>(chunk, count ? count : 1));
    for (uint64_t done = 0; done < count; done += chunk) {
        const uint64_t c = std::min<uint64_t>(chunk, count - done);
        for (uint64_t i = 0; i < 2 * c; ++i) tmp[i] = static_cast<float>(host[2 * done + i]);
        QD_HIP(hipMemcpyAsync(static_cast<float*>(s->psi) + 2 * (offset + done), tmp.data(), c * 8,
                              hipMemcpyHostToDevice, s->stream),
               "copy to device");
        QD_HIP(hipStreamSynchronize(s->stream), "copy to device");
    }
    return QD_OK;
}

int qd_state_get_amplitudes(const qd_state* s, double* host, uint64_t offset, uint64_t count) {
    if (!s) return set_err(QD_ERR_INVALID_ARGUMENT, "state is null");
    if (count && !host) return set_err(QD_ERR_INVALID_ARGUMENT, "host is null");
    if (offset > s->D || count > s->D - offset) return set_err(QD_ERR_INVALID_ARGUMENT, "range outside the state");
    int rc = use_device(s);
    if (rc) return rc;
    if (s->precision == QD_C128) {
        QD_HIP(hipMemcpyAsync(host, static_cast<const double*>(s->psi) + 2 * offset, count * 16,
                              hipMemcpyDeviceToHost, s->stream),
               "copy to host");
        QD_HIP(hipStreamSynchronize(s->stream), "copy to host");
        return QD_OK;
    }
    const uint64_t chunk = 1ull << 22;
    std::vector<float> tmp(2 * std::min<uint64_t>(chunk, count ? count : 1));
    for (uint64_t done = 0; done < count; done += chunk) {
        const uint64_t c = std::min<uint64_t>(chunk, count - done);
        QD_HIP(hipMemcpyAsync(tmp.data(), static_cast<const float*>(s->psi) + 2 * (offset + done), c * 8,
                              hipMemcpyDeviceToHost, s->stream),
               "copy to host");
        QD_HIP(hipStreamSynchronize(s->stream), "copy to host");
        for (uint64_t i = 0; i < 2 * c; ++i) host[2 * done + i] = static_cast<double>(tmp[i]);
    }
    return QD_OK;
}

}  // extern "C"

namespace {

// Copy `bytes` of per-launch data to the device through the state's ring.
int stage(qd_state* s, const void* data, size_t bytes, const void** dptr) {
    if (bytes > GateRing::kSlot) return set_err(QD_ERR_NOT_SUPPORTED, "per-launch gate data exceeds the staging slot");
    int rc = s->ring.ensure();
    if (rc) return rc;
    GateRing& r = s->ring;
    const int slot = r.next;
    r.next = (r.next + 1) % GateRing::kSlots;
    if (r.pending[slot]) QD_HIP(hipEventSynchronize(r.ev[slot]), "gate staging");
    unsigned char* h = r.host + slot * GateRing::kSlot;
    unsigned char* d = r.dev + slot * GateRing::kSlot;
    std::memcpy(h, data, bytes);
    QD_HIP(hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, s->stream), "gate upload");
    QD_HIP(hipEventRecord(r.ev[slot], s->stream), "gate staging");
    r.pending[slot] = true;
    *dptr = d;
    return QD_OK;
}

int enqueue_single(qd_state* s, const GatePlan& p, const double* U) {
    const size_t gbytes = device_gate_bytes(p, s->precision);
    const void* dgate = nullptr;
    if (gbytes) {
        std::vector<unsigned char> buf(gbytes);
        fill_device_gate(p, s->precision, U, buf.data());
        int rc = stage(s, buf.data(), gbytes, &dgate);
        if (rc) return rc;
    }
    QD_HIP(launch_gate(p, s->precision, s->psi, U, dgate, s->stream), "gate launch");
    return QD_OK;
}

int circuit_options(const qd_circuit_options* o, int precision, CircuitOptions* co) {
    co->fuse = o ? o->fuse != 0 : true;
    const uint64_t tile = (o && o->tile_amps > 0) ? (uint64_t)o->tile_amps : (precision == QD_C128 ? 3072 : 8192);
    const uint64_t run = (o && o->min_run > 0) ? (uint64_t)o->min_run : (precision == QD_C128 ? 64 : 128);
    if (tile > 32768) return set_err(QD_ERR_INVALID_ARGUMENT, "tile_amps must be at most 32768");
    if (tile * amp_bytes(precision) > 160 * 1024)
        return set_err(QD_ERR_INVALID_ARGUMENT, "a tile must fit the 160 KB of LDS");
    if (o && o->reorder < 0) return set_err(QD_ERR_INVALID_ARGUMENT, "reorder must not be negative");
    co->tile_max = tile;
    co->min_run = run;
    co->reorder = o ? o->reorder : 0;
    return QD_OK;
}

int circuit_gates(const int32_t* dims, int32_t n, const qd_gate_desc* gates, int32_t count,
                  std::vector<CircuitGate>& cg) {
    if (count < 0) return set_err(QD_ERR_INVALID_ARGUMENT, "negative gate count");
    if (count > 0 && !gates) return set_err(QD_ERR_INVALID_ARGUMENT, "gates is null");
    cg.resize(count);
    for (int i = 0; i < count; ++i) {
        const qd_gate_desc& g = gates[i];
        std::string err;
        int rc = check_gate(dims, n, g.targets, g.k, g.controls, g.values, g.m, &err);
        if (rc) return set_err(rc, "gate " + std::to_string(i) + ": " + err);
        if (!g.U) return set_err(QD_ERR_INVALID_ARGUMENT, "gate " + std::to_string(i) + ": U is null");
        cg[i] = CircuitGate{g.targets, g.k, g.controls, g.values, g.m, g.U};
    }
    return QD_OK;
}

}  // namespace

extern "C" {

int qd_apply_gate(qd_state* s, const int32_t* targets, int32_t k, const int32_t* controls, const int32_t* values,
                  int32_t m, const double* U) {
    if (!s) return set_err(QD_ERR_INVALID_ARGUMENT, "state is null");
    GatePlan p;
    std::string err;
    int rc = plan_gate(s->dims, s->n, targets, k, controls, values, m, U, &p, &err);
    if (rc) return set_err(rc, err);
    rc = use_device(s);
    if (rc) return rc;
    return enqueue_single(s, p, U);
}

struct qd_sparse {
    int n = 0;
    int32_t dims[QD_SPARSE_MAX_QUDITS] = {};
    int word[QD_SPARSE_MAX_QUDITS] = {};        // key word of each qudit
    uint64_t stride[QD_SPARSE_MAX_QUDITS] = {}; // stride inside that word
    uint64_t P[qd::kKeyWords] = {1, 1, 1};      // product of each word's dims
    uint64_t D_lo = 0, D_hi = 0;
    int device = 0;
    qd::SparseData d;
};

namespace {

int sparse_device(const qd_sparse* s) {
    int cur = -1;
    QD_HIP(hipGetDevice(&cur), "hipGetDevice");
    if (cur != s->device) QD_HIP(hipSetDevice(s->device), "hipSetDevice");
    return QD_OK;
}

int sparse_hip_err(hipError_t e, const char* what) {
    if (e == hipErrorIllegalState)
        return set_err(QD_ERR_DEVICE, std::string(what) + ": a gate found more stored entries than planned");
    return hip_err(e, what);
}

// The first c entries as 128-bit basis indices (lo, hi per entry, or only lo
// when hi is null) and amplitudes.
int sparse_fetch(qd_sparse* s, uint64_t cap, uint64_t* lo, uint64_t* hi, double* amps) {
    int rc = sparse_device(s);
    if (rc) return rc;
    uint64_t nnz = 0;
    hipError_t e = qd::sparse_count(s->d, &nnz);
    if (e != hipSuccess) return sparse_hip_err(e, "sparse get");
    const uint64_t c = std::min<uint64_t>(cap, nnz);
    if (c == 0) return QD_OK;
    const int W = s->d.W;
    const uint64_t scap = s->d.slot_cap[s->d.cur];
    std::vector<uint64_t> words((size_t)W * c);
    void* slot = s->d.slot[s->d.cur];
    for (int w = 0; w < W; ++w)
        QD_HIP(hipMemcpy(words.data() + (size_t)w * c, qd::slot_keys(slot) + (size_t)w * scap, c * 8,
                         hipMemcpyDeviceToHost),
               "sparse get keys");
    QD_HIP(hipMemcpy(amps, qd::slot_amps(slot, W, scap), c * 16, hipMemcpyDeviceToHost), "sparse get amplitudes");
    // basis index = w_0 + P_0 (w_1 + P_1 w_2)
    for (uint64_t i = 0; i < c; ++i) {
        unsigned __int128 v = 0;
        for (int w = W - 1; w >= 0; --w) v = v * s->P[w] + words[(size_t)w * c + i];
        if (hi) {
            lo[2 * i] = (uint64_t)v;
            lo[2 * i + 1] = (uint64_t)(v >> 64);
        } else {
            lo[i] = (uint64_t)v;
        }
    }
    return QD_OK;
}

}  // namespace

int qd_sparse_dim(const int32_t* dims, int32_t n, uint64_t* D_lo, uint64_t* D_hi, int32_t* words) {
    std::string err;
    int W = 0;
    int rc = sparse_layout(dims, n, nullptr, nullptr, &W, nullptr, D_lo, D_hi, &err);
    if (rc) return set_err(rc, err);
    if (words) *words = W;
    return QD_OK;
}

int qd_sparse_create(const int32_t* dims, int32_t n, qd_sparse** out) {
    if (!out) return set_err(QD_ERR_INVALID_ARGUMENT, "out is null");
    *out = nullptr;
    std::string err;
    qd_sparse* s = new qd_sparse;
    int W = 0;
    int rc = sparse_layout(dims, n, s->word, s->stride, &W, s->P, &s->D_lo, &s->D_hi, &err);
    if (rc) {
        delete s;
        return set_err(rc, err);
    }
    s->n = n;
    for (int i = 0; i < n; ++i) s->dims[i] = dims[i];
    hipError_t e = hipGetDevice(&s->device);
    if (e == hipSuccess) e = qd::sparse_init(s->d, W);
    if (e != hipSuccess) {
        qd::sparse_release(s->d);
        delete s;
        return hip_err(e, "sparse state");
    }
    *out = s;
    return QD_OK;
}

int qd_sparse_destroy(qd_sparse* s) {
    if (!s) return QD_OK;
    (void)hipSetDevice(s->device);
    qd::sparse_release(s->d);
    delete s;
    return QD_OK;
}

int qd_sparse_set_stream(qd_sparse* s, void* hip_stream) {
    if (!s) return set_err(QD_ERR_INVALID_ARGUMENT, "state is null");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    if (st == s->d.stream) return QD_OK;
    int rc = sparse_device(s);
    if (rc) return rc;
    QD_HIP(hipStreamSynchronize(s->d.stream), "synchronizing the previous stream");
    s->d.stream = st;
    return QD_OK;
}

namespace {

// Validate a gate on a sparse register and build its kernel form (*cols_single:
// every column of U has at most one nonzero).
int sparse_gate_of(const qd_sparse* s, const int32_t* targets, int32_t k, const int32_t* controls,
                   const int32_t* values, int32_t m, const double* U, qd::SparseGate* out, bool* cols_single) {
    std::string err;
    int rc = check_gate_shape(s->dims, s->n, targets, k, controls, values, m, &err);
    if (rc) return set_err(rc, err);
    if (!U) return set_err(QD_ERR_INVALID_ARGUMENT, "U is null");
    qd::SparseGate& g = *out;
    std::memset(&g, 0, sizeof g);
    g.W = s->d.W;
    g.k = k;
    g.M = 1;
    for (int l = 0; l < k; ++l) {
        g.tw[l] = s->word[targets[l]];
        g.ts[l] = s->stride[targets[l]];
        g.td[l] = (uint32_t)s->dims[targets[l]];
        g.tsd[l] = qd::make_fast_div<uint64_t>(g.ts[l]);
        g.tdd[l] = qd::make_fast_div<uint64_t>(g.td[l]);
        g.M *= s->dims[targets[l]];
    }
    if (g.M > qd::kSparseMaxM) return set_err(QD_ERR_NOT_SUPPORTED, "sparse gates act on at most 16 amplitudes");
    if (unitary_check_enabled() && !(unitary_deviation(U, g.M) <= kUnitaryTol))
        return set_err(QD_ERR_INVALID_ARGUMENT, "U is not unitary (QD_CHECK_UNITARY)");
    g.m = m;
    for (int l = 0; l < m; ++l) {
        g.cw[l] = s->word[controls[l]];
        g.cs[l] = s->stride[controls[l]];
        g.cd[l] = (uint32_t)s->dims[controls[l]];
        g.csd[l] = qd::make_fast_div<uint64_t>(g.cs[l]);
        g.cdd[l] = qd::make_fast_div<uint64_t>(g.cd[l]);
        g.cv[l] = (uint32_t)values[l];
    }
    for (int a = 0; a < g.M; ++a) {
        int r = a;
        for (int l = 0; l < k; ++l) {
            g.off[a][g.tw[l]] += (uint64_t)(r % (int)g.td[l]) * g.ts[l];
            r /= (int)g.td[l];
        }
    }
    // Every column with at most one nonzero: each entry feeds at most one result,
    // so the gate cannot raise the entry count.
    *cols_single = true;
    for (int a = 0; a < g.M && *cols_single; ++a) {
        int nz = 0;
        for (int r = 0; r < g.M; ++r) nz += (U[2 * (r * g.M + a)] != 0.0 || U[2 * (r * g.M + a) + 1] != 0.0);
        *cols_single = nz <= 1;
    }
    return QD_OK;
}

int sparse_enqueue(qd_sparse* s, const qd::SparseGate& g, const double* U, bool cols_single) {
    hipError_t e = qd::sparse_apply(s->d, g, U, cols_single);
    if (e == hipErrorNotSupported)
        return set_err(QD_ERR_NOT_SUPPORTED, "sparse state too large: stored entries x class size must stay below 2^31");
    if (e != hipSuccess) return sparse_hip_err(e, "sparse gate");
    return QD_OK;
}

}  // namespace

int qd_sparse_apply_gate(qd_sparse* s, const int32_t* targets, int32_t k, const int32_t* controls,
                         const int32_t* values, int32_t m, const double* U) {
    if (!s) return set_err(QD_ERR_INVALID_ARGUMENT, "state is null");
    qd::SparseGate g;
    bool cols_single = false;
    int rc = sparse_gate_of(s, targets, k, controls, values, m, U, &g, &cols_single);
    if (rc) return rc;
    rc = sparse_device(s);
    if (rc) return rc;
    return sparse_enqueue(s, g, U, cols_single);
}

int qd_sparse_apply_circuit(qd_sparse* s, const qd_gate_desc* gates, int32_t count) {
    if (!s) return set_err(QD_ERR_INVALID_ARGUMENT, "state is null");
    if (count < 0 || (count > 0 && !gates)) return set_err(QD_ERR_INVALID_ARGUMENT, "bad gate list");
    std::vector<qd::SparseGate> gs((size_t)count);
    std::vector<char> single((size_t)count, 0);
    for (int32_t i = 0; i < count; ++i) {  // everything is checked before anything is enqueued
        const qd_gate_desc& d = gates[i];
        bool cs = false;
        int rc = sparse_gate_of(s, d.targets, d.k, d.controls, d.values, d.m, d.U, &gs[(size_t)i], &cs);
        if (rc) return set_err(rc, "gate " + std::to_string(i) + ": " + g_err);
        single[(size_t)i] = cs;
    }
    int rc = sparse_device(s);
    if (rc) return rc;
    std::vector<const double*> us((size_t)count);
    std::unique_ptr<bool[]> cs(new bool[(size_t)count + 1]);
    for (int32_t i = 0; i < count; ++i) {
        us[(size_t)i] = gates[i].U;
        cs[(size_t)i] = single[(size_t)i] != 0;
    }
    hipError_t e = qd::sparse_apply_list(s->d, gs.data(), us.data(), cs.get(), count);
    if (e == hipErrorNotSupported)
        return set_err(QD_ERR_NOT_SUPPORTED, "sparse state too large: stored entries x class size must stay below 2^31");
    if (e != hipSuccess) return sparse_hip_err(e, "sparse gate list");
    return QD_OK;
}

int qd_sparse_nnz(qd_sparse* s, uint64_t* nnz) {
    if (!s || !nnz) return set_err(QD_ERR_INVALID_ARGUMENT, "null argument");
    int rc = sparse_device(s);
    if (rc) return rc;
    hipError_t e = qd::sparse_count(s->d, nnz);
    if (e != hipSuccess) return sparse_hip_err(e, "sparse count");
    return QD_OK;
}

int qd_sparse_get(qd_sparse* s, uint64_t* keys, double* amps, uint64_t cap) {
    if (!s || (cap && (!keys || !amps))) return set_err(QD_ERR_INVALID_ARGUMENT, "null argument");
    if (s->D_hi) return set_err(QD_ERR_NOT_SUPPORTED, "register has D >= 2^64: use qd_sparse_get_wide");
    return sparse_fetch(s, cap, keys, nullptr, amps);
}

int qd_sparse_get_wide(qd_sparse* s, uint64_t* keys, double* amps, uint64_t cap) {
    if (!s || (cap && (!keys || !amps))) return set_err(QD_ERR_INVALID_ARGUMENT, "null argument");
    uint64_t dummy = 0;
    return sparse_fetch(s, cap, keys, &dummy, amps);
}

static constexpr uint64_t kMaxMaskedCombos = 4096;

int qd_apply_gate_masked(qd_state* s, const int32_t* targets, int32_t k, const int32_t* controls,
                         const uint32_t* value_masks, int32_t m, const double* U) {
    if (!s) return set_err(QD_ERR_INVALID_ARGUMENT, "state is null");
    if (m < 0 || m > QD_MAX_CONTROLS) return set_err(QD_ERR_INVALID_ARGUMENT, "bad number of controls");
    if (m > 0 && (!controls || !value_masks)) return set_err(QD_ERR_INVALID_ARGUMENT, "controls or masks null");
    {
        // the gate's structure (targets, distinct controls, U) as for qd_check_gate, with value 0
        const int32_t zeros[QD_MAX_CONTROLS] = {};
        std::string err;
        int rc = check_gate(s->dims, s->n, targets, k, controls, zeros, m, &err);
        if (rc) return set_err(rc, err);
        if (!U) return set_err(QD_ERR_INVALID_ARGUMENT, "U is null");
    }
    // Controls that accept every value are dropped; the others list their values.
    std::vector<int32_t> cq;
    std::vector<std::vector<int32_t>> vals;
    for (int l = 0; l < m; ++l) {
        const int c = controls[l];
        const uint32_t all = (1u << s->dims[c]) - 1u;
        if (value_masks[l] == 0 || (value_masks[l] & ~all) != 0)
            return set_err(QD_ERR_INVALID_ARGUMENT, "a value mask must be non-zero and below the control's dimension");
        if (value_masks[l] == all) continue;
        cq.push_back(c);
        vals.emplace_back();
        for (int v = 0; v < s->dims[c]; ++v)
            if ((value_masks[l] >> v) & 1u) vals.back().push_back(v);
    }
    // Plan every combination before enqueuing any (an error leaves the state untouched).
    const int mm = (int)cq.size();
    uint64_t combos = 1;
    for (const auto& v : vals)
        if ((combos *= v.size()) > kMaxMaskedCombos)
            return set_err(QD_ERR_NOT_SUPPORTED, "more than 4096 accepted-value combinations");
    std::vector<int> idx(mm, 0);
    std::vector<GatePlan> plans;
    std::vector<int32_t> cv(mm > 0 ? mm : 1);
    while (true) {
        for (int l = 0; l < mm; ++l) cv[l] = vals[l][idx[l]];
        plans.emplace_back();
        std::string err;
        int rc = plan_gate(s->dims, s->n, targets, k, mm ? cq.data() : nullptr, mm ? cv.data() : nullptr, mm, U,
                           &plans.back(), &err);
        if (rc) return set_err(rc, err);
        int l = 0;
        while (l < mm && ++idx[l] == (int)vals[l].size()) idx[l++] = 0;
        if (l == mm) break;
    }
    int rc = use_device(s);
    if (rc) return rc;
    for (const GatePlan& p : plans)
        if ((rc = enqueue_single(s, p, U))) return rc;
    return QD_OK;
}

int qd_circuit_plan(const int32_t* dims, int32_t n, int32_t precision, const qd_gate_desc* gates, int32_t count,
                    const qd_circuit_options* opts, int32_t* pass_gates, int32_t* pass_tile, int32_t* order,
                    int32_t* npasses) {
    int rc = check_precision(precision);
    if (rc) return rc;
    std::string err;
    rc = check_dims(dims, n, nullptr, &err);
    if (rc) return set_err(rc, err);
    if (!npasses) return set_err(QD_ERR_INVALID_ARGUMENT, "npasses is null");
    std::vector<CircuitGate> cg;
    rc = circuit_gates(dims, n, gates, count, cg);
    if (rc) return rc;
    CircuitOptions co;
    rc = circuit_options(opts, precision, &co);
    if (rc) return rc;
    std::vector<PassPlan> plan;
    rc = plan_circuit(dims, n, precision, cg.data(), count, co, plan, &err);
    if (rc) return set_err(rc, err);
    *npasses = (int32_t)plan.size();
    size_t k = 0;
    for (size_t i = 0; i < plan.size(); ++i) {
        if (pass_gates) pass_gates[i] = (int32_t)plan[i].gates.size();
        if (pass_tile) pass_tile[i] = plan[i].fused ? (int32_t)plan[i].launch.tile : 0;
        if (order)
            for (int g : plan[i].gates) order[k++] = g;
    }
    return QD_OK;
}

int qd_apply_circuit(qd_state* s, const qd_gate_desc* gates, int32_t count, qd_circuit_options* opts) {
    if (!s) return set_err(QD_ERR_INVALID_ARGUMENT, "state is null");
    std::vector<CircuitGate> cg;
    int rc = circuit_gates(s->dims, s->n, gates, count, cg);
    if (rc) return rc;
    CircuitOptions co;
    rc = circuit_options(opts, s->precision, &co);
    if (rc) return rc;
    std::vector<PassPlan> plan;
    std::string err;
    rc = plan_circuit(s->dims, s->n, s->precision, cg.data(), count, co, plan, &err);
    if (rc) return set_err(rc, err);
    rc = use_device(s);
    if (rc) return rc;
    int fused = 0;
    GatePlan p;
    for (const PassPlan& pp : plan) {
        if (!pp.fused) {
            const CircuitGate& g = cg[pp.gates[0]];
            rc = plan_gate(s->dims, s->n, g.targets, g.k, g.controls, g.values, g.m, g.U, &p, &err);
            if (rc) return set_err(rc, err);
            rc = enqueue_single(s, p, g.U);
            if (rc) return rc;
            continue;
        }
        if (pp.launch.ngates == 0) continue;
        const void* dblob = nullptr;
        rc = stage(s, pp.blob.data(), pp.blob.size(), &dblob);
        if (rc) return rc;
        QD_HIP(launch_fused(pp.launch, s->precision, s->psi, dblob, s->stream), "fused launch");
        ++fused;
    }
    if (opts) {
        opts->passes = (int32_t)plan.size();
        opts->fused_passes = fused;
    }
    return QD_OK;
}

}  // extern "C"

// A batch context: staging for the per-round descriptor blobs of qd_batch_apply.
// Two pinned host buffers and two device buffers alternate between rounds; a
// host buffer is refilled only after its previous copy has finished (event),
// a device buffer only after the kernel that read it (stream order).
struct qd_batch {
    int precision = 0;
    struct Buf {
        unsigned char* host = nullptr;
        unsigned char* dev = nullptr;
        size_t cap = 0;
        hipEvent_t ev = nullptr;
        bool pending = false;
    } buf[2];
    int next = 0;
};

namespace {

void batch_free(qd_batch* b) {
    for (auto& x : b->buf) {
        if (x.ev) (void)hipEventSynchronize(x.ev), (void)hipEventDestroy(x.ev);
        if (x.dev) (void)hipFree(x.dev);
        if (x.host) (void)hipHostFree(x.host);
        x = qd_batch::Buf();
    }
}

// Stage `bytes` into the next buffer pair and copy it to the device on `st`.
int batch_stage(qd_batch* b, const std::vector<unsigned char>& data, hipStream_t st, const unsigned char** dptr) {
    qd_batch::Buf& x = b->buf[b->next];
    b->next ^= 1;
    if (x.pending) QD_HIP(hipEventSynchronize(x.ev), "batch staging");
    if (data.size() > x.cap) {
        QD_HIP(hipStreamSynchronize(st), "batch staging");  // the old device buffer may still be read
        if (x.dev) (void)hipFree(x.dev);
        if (x.host) (void)hipHostFree(x.host);
        x.dev = nullptr;
        x.host = nullptr;
        size_t cap = std::max<size_t>(data.size(), 1u << 20);
        cap += cap / 2;
        if (hipHostMalloc(reinterpret_cast<void**>(&x.host), cap, hipHostMallocDefault) != hipSuccess) {
            x.host = nullptr;
            x.cap = 0;
            return set_err(QD_ERR_OUT_OF_MEMORY, "pinned batch staging allocation failed");
        }
        if (hipMalloc(reinterpret_cast<void**>(&x.dev), cap) != hipSuccess) {
            (void)hipHostFree(x.host);
            x.host = nullptr;
            x.dev = nullptr;
            x.cap = 0;
            return set_err(QD_ERR_OUT_OF_MEMORY, "device batch buffer allocation failed");
        }
        x.cap = cap;
        if (!x.ev) QD_HIP(hipEventCreateWithFlags(&x.ev, hipEventDisableTiming), "event");
    }
    std::memcpy(x.host, data.data(), data.size());
    QD_HIP(hipMemcpyAsync(x.dev, x.host, data.size(), hipMemcpyHostToDevice, st), "batch upload");
    QD_HIP(hipEventRecord(x.ev, st), "batch staging");
    x.pending = true;
    *dptr = x.dev;
    return QD_OK;
}

}  // namespace

extern "C" {

int qd_batch_create(int32_t precision, qd_batch** out) {
    if (!out) return set_err(QD_ERR_INVALID_ARGUMENT, "out is null");
    *out = nullptr;
    int rc = check_precision(precision);
    if (rc) return rc;
    qd_batch* b = new qd_batch();
    b->precision = precision;
    *out = b;
    return QD_OK;
}

int qd_batch_destroy(qd_batch* b) {
    if (!b) return QD_OK;
    batch_free(b);
    delete b;
    return QD_OK;
}

}  // extern "C"

namespace {

// One launch round of a batch on the host: the round's blob (the pass blobs of
// its items, then the BatchItem array at items_off) and the states whose pass in
// this round runs as its own launch (a gate too large for a tile, or an outer
// decode that does not fit a batch item).
struct HostRound {
    std::vector<unsigned char> blob;
    size_t items_off = 0;
    int nitems = 0;
    uint64_t nblocks = 0;
    uint32_t max_tile = 0;
    std::vector<int> singles;
};

struct BatchInput {
    std::vector<std::vector<CircuitGate>> cg;
    std::vector<std::vector<PassPlan>> plans;
    size_t rounds = 0;
};

int batch_validate_and_plan(int precision, qd_state* const* states, const qd_gate_desc* const* gates,
                            const int32_t* counts, int32_t nstates, const qd_circuit_options* opts, BatchInput& in) {
    if (nstates < 0) return set_err(QD_ERR_INVALID_ARGUMENT, "negative state count");
    if (nstates > 0 && (!states || !gates || !counts))
        return set_err(QD_ERR_INVALID_ARGUMENT, "states, gates or counts is null");
    in.cg.assign(nstates, {});
    for (int i = 0; i < nstates; ++i) {
        const qd_state* s = states[i];
        if (!s) return set_err(QD_ERR_INVALID_ARGUMENT, "state " + std::to_string(i) + " is null");
        if (s->precision != precision)
            return set_err(QD_ERR_INVALID_ARGUMENT, "state " + std::to_string(i) + " has another precision");
        if (s->device != states[0]->device || s->stream != states[0]->stream)
            return set_err(QD_ERR_INVALID_ARGUMENT, "all states of a batch must share one device and stream");
        if (s->D >= (1ull << 31))
            return set_err(QD_ERR_NOT_SUPPORTED, "batched states must have fewer than 2^31 amplitudes");
        for (int j = 0; j < i; ++j)
            if (states[j] == s) return set_err(QD_ERR_INVALID_ARGUMENT, "a state appears twice in a batch");
        int rc = circuit_gates(s->dims, s->n, gates[i], counts[i], in.cg[i]);
        if (rc) return set_err(rc, "state " + std::to_string(i) + ": " + qd_last_error());
    }
    CircuitOptions co;
    int rc = circuit_options(opts, precision, &co);
    if (rc) return rc;
    co.fuse = true;
    co.single_as_fused = true;
    in.plans.assign(nstates, {});
    in.rounds = 0;
    for (int i = 0; i < nstates; ++i) {
        std::string err;
        rc = plan_circuit(states[i]->dims, states[i]->n, precision, in.cg[i].data(), counts[i], co, in.plans[i], &err);
        if (rc) return set_err(rc, "state " + std::to_string(i) + ": " + err);
        in.rounds = std::max(in.rounds, in.plans[i].size());
    }
    return QD_OK;
}

int build_round(qd_state* const* states, int32_t nstates, const BatchInput& in, size_t r, HostRound& out) {
    out = HostRound();
    std::vector<BatchItem> items;
    for (int i = 0; i < nstates; ++i) {
        if (r >= in.plans[i].size()) continue;
        const PassPlan& pp = in.plans[i][r];
        if (!pp.fused || pp.launch.outer_nseg > kTileMaxSeg) {
            out.singles.push_back(i);
            continue;
        }
        if (pp.launch.ngates == 0) continue;
        const FusedLaunch& f = pp.launch;
        const size_t base = (out.blob.size() + 15) / 16 * 16;
        out.blob.resize(base + pp.blob.size());
        std::memcpy(out.blob.data() + base, pp.blob.data(), pp.blob.size());
        rebase_pass_blob(out.blob.data() + base, f, 0, (uint32_t)base);
        BatchItem it;
        std::memset(&it, 0, sizeof it);
        it.psi = reinterpret_cast<uint64_t>(states[i]->psi);
        it.outer.n_classes = (uint32_t)f.n_tiles;
        it.outer.ctrl_off = 0;
        it.outer.nseg = f.outer_nseg;
        for (int g = 0; g < kTileMaxSeg; ++g) {
            it.outer.size[g] = g < f.outer_nseg ? (uint32_t)f.outer_size[g] : 1u;
            it.outer.stride[g] = g < f.outer_nseg ? (uint32_t)f.outer_stride[g] : 0u;
            it.outer.div[g] = make_fast_div<uint32_t>(g < f.outer_nseg ? f.outer_size[g] : 1);
        }
        it.tile = f.tile;
        it.L = f.L;
        it.chunks_per_run = (f.L + 63) / 64;
        it.nchunks = (f.tile / f.L) * it.chunks_per_run;
        it.cdiv = make_fast_div<uint32_t>(it.chunks_per_run);
        it.ngates = f.ngates;
        it.gates_off = (uint32_t)(base + f.gates_off);
        it.run_off_off = (uint32_t)(base + f.run_off_off);
        it.first_block = (uint32_t)out.nblocks;
        out.nblocks += f.n_tiles;
        out.max_tile = std::max(out.max_tile, f.tile);
        items.push_back(it);
    }
    if (out.nblocks >= 0x7fffffffull) return set_err(QD_ERR_NOT_SUPPORTED, "batched round too large");
    if (out.blob.size() > 0xffffffffull) return set_err(QD_ERR_NOT_SUPPORTED, "batched round blob too large");
    out.nitems = (int)items.size();
    if (!items.empty()) {
        out.items_off = (out.blob.size() + 15) / 16 * 16;
        out.blob.resize(out.items_off + items.size() * sizeof(BatchItem));
        std::memcpy(out.blob.data() + out.items_off, items.data(), items.size() * sizeof(BatchItem));
    }
    return QD_OK;
}

// The launch of one state's own pass inside a round (see HostRound::singles).
int enqueue_round_single(qd_state* s, const BatchInput& in, int i, size_t r, hipStream_t st) {
    const PassPlan& pp = in.plans[i][r];
    if (pp.fused) {
        const void* dblob = nullptr;
        int rc = stage(s, pp.blob.data(), pp.blob.size(), &dblob);
        if (rc) return rc;
        QD_HIP(launch_fused(pp.launch, s->precision, s->psi, dblob, st), "fused launch");
        return QD_OK;
    }
    const CircuitGate& g = in.cg[i][pp.gates[0]];
    GatePlan p;
    std::string err;
    int rc = plan_gate(s->dims, s->n, g.targets, g.k, g.controls, g.values, g.m, g.U, &p, &err);
    if (rc) return set_err(rc, err);
    return enqueue_single(s, p, g.U);
}

}  // namespace

// A compiled batch: all rounds' blobs in one device buffer, launched by
// qd_batch_plan_run without any host planning or uploads (and, when asked,
// replayed as one captured hipGraph).
struct qd_batch_plan {
    int precision = 0;
    std::vector<qd_state*> states;
    hipStream_t stream = nullptr;
    struct Round {
        size_t blob_off = 0;
        size_t items_off = 0;
        int nitems = 0;
        uint32_t nblocks = 0;
        uint32_t max_tile = 0;
    };
    std::vector<Round> rounds;
    int32_t items_total = 0;
    unsigned char* dev = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

extern "C" {

int qd_batch_apply(qd_batch* b, qd_state* const* states, const qd_gate_desc* const* gates, const int32_t* counts,
                   int32_t nstates, qd_circuit_options* opts) {
    if (!b) return set_err(QD_ERR_INVALID_ARGUMENT, "batch is null");
    if (nstates == 0) return QD_OK;
    BatchInput in;
    int rc = batch_validate_and_plan(b->precision, states, gates, counts, nstates, opts, in);
    if (rc) return rc;
    qd_state* s0 = states[0];
    rc = use_device(s0);
    if (rc) return rc;
    hipStream_t st = s0->stream;
    int32_t items_total = 0;
    HostRound hr;
    for (size_t r = 0; r < in.rounds; ++r) {
        // Round r: pass r of every state that has one; fused passes go into one
        // launch, any pass that cannot join it runs right after it.
        rc = build_round(states, nstates, in, r, hr);
        if (rc) return rc;
        if (hr.nitems) {
            const unsigned char* dblob = nullptr;
            rc = batch_stage(b, hr.blob, st, &dblob);
            if (rc) return rc;
            QD_HIP(launch_batch(b->precision, dblob + hr.items_off, hr.nitems, (uint32_t)hr.nblocks, hr.max_tile,
                                dblob, st),
                   "batch launch");
            items_total += hr.nitems;
        }
        for (int i : hr.singles) {
            rc = enqueue_round_single(states[i], in, i, r, st);
            if (rc) return rc;
        }
    }
    if (opts) {
        opts->passes = (int32_t)in.rounds;
        opts->fused_passes = items_total;
    }
    return QD_OK;
}

int qd_batch_compile(qd_state* const* states, const qd_gate_desc* const* gates, const int32_t* counts,
                     int32_t nstates, qd_circuit_options* opts, qd_batch_plan** out) {
    if (!out) return set_err(QD_ERR_INVALID_ARGUMENT, "out is null");
    *out = nullptr;
    if (nstates < 1 || !states || !states[0]) return set_err(QD_ERR_INVALID_ARGUMENT, "a plan needs at least one state");
    const int precision = states[0]->precision;
    BatchInput in;
    int rc = batch_validate_and_plan(precision, states, gates, counts, nstates, opts, in);
    if (rc) return rc;
    qd_batch_plan* P = new qd_batch_plan();
    P->precision = precision;
    P->states.assign(states, states + nstates);
    P->stream = states[0]->stream;
    std::vector<unsigned char> all;
    HostRound hr;
    for (size_t r = 0; r < in.rounds; ++r) {
        rc = build_round(states, nstates, in, r, hr);
        if (rc == QD_OK && !hr.singles.empty())
            rc = set_err(QD_ERR_NOT_SUPPORTED, "a compiled batch needs every pass to fit a batch item (tile gates "
                                               "with at most 16 amplitudes per class); use qd_batch_apply");
        if (rc) {
            delete P;
            return rc;
        }
        qd_batch_plan::Round R;
        R.blob_off = (all.size() + 255) / 256 * 256;
        R.items_off = hr.items_off;
        R.nitems = hr.nitems;
        R.nblocks = (uint32_t)hr.nblocks;
        R.max_tile = hr.max_tile;
        all.resize(R.blob_off + hr.blob.size());
        std::memcpy(all.data() + R.blob_off, hr.blob.data(), hr.blob.size());
        P->rounds.push_back(R);
        P->items_total += hr.nitems;
    }
    rc = use_device(states[0]);
    if (rc == QD_OK && !all.empty()) {
        if (hipMalloc(reinterpret_cast<void**>(&P->dev), all.size()) != hipSuccess) {
            P->dev = nullptr;
            rc = set_err(QD_ERR_OUT_OF_MEMORY, "device allocation of the compiled batch failed");
        } else {
            hipError_t e = hipMemcpy(P->dev, all.data(), all.size(), hipMemcpyHostToDevice);
            if (e != hipSuccess) rc = hip_err(e, "compiled batch upload");
        }
    }
    if (rc) {
        if (P->dev) (void)hipFree(P->dev);
        delete P;
        return rc;
    }
    if (opts) {
        opts->passes = (int32_t)P->rounds.size();
        opts->fused_passes = P->items_total;
    }
    *out = P;
    return QD_OK;
}

namespace {
hipError_t plan_enqueue(qd_batch_plan* P, hipStream_t st) {
    for (const auto& R : P->rounds) {
        if (!R.nitems) continue;
        hipError_t e = launch_batch(P->precision, P->dev + R.blob_off + R.items_off, R.nitems, R.nblocks,
                                    R.max_tile,
                                    P->dev + R.blob_off, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}
}  // namespace

int qd_batch_plan_run(qd_batch_plan* P, int32_t use_graph) {
    if (!P) return set_err(QD_ERR_INVALID_ARGUMENT, "plan is null");
    int rc = use_device(P->states[0]);
    if (rc) return rc;
    hipStream_t st = P->stream;
    if (!use_graph) {
        QD_HIP(plan_enqueue(P, st), "batch launch");
        return QD_OK;
    }
    if (!P->exec) {
        // Capture on a private stream so the caller's stream is never in capture mode.
        hipStream_t cap = nullptr;
        QD_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking), "capture stream");
        hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            hipError_t e2 = plan_enqueue(P, cap);
            e = hipStreamEndCapture(cap, &P->graph);
            if (e2 != hipSuccess) e = e2;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0);
        (void)hipStreamDestroy(cap);
        if (e != hipSuccess) {
            if (P->graph) (void)hipGraphDestroy(P->graph);
            P->graph = nullptr;
            P->exec = nullptr;
            return hip_err(e, "batch graph capture");
        }
    }
    QD_HIP(hipGraphLaunch(P->exec, st), "batch graph launch");
    return QD_OK;
}

int qd_batch_plan_destroy(qd_batch_plan* P) {
    if (!P) return QD_OK;
    if (!P->states.empty()) {
        use_device(P->states[0]);
        (void)hipStreamSynchronize(P->stream);
    }
    if (P->exec) (void)hipGraphExecDestroy(P->exec);
    if (P->graph) (void)hipGraphDestroy(P->graph);
    if (P->dev) (void)hipFree(P->dev);
    delete P;
    return QD_OK;
}

int qd_norm(const qd_state* s, double* out) {
    if (!s || !out) return set_err(QD_ERR_INVALID_ARGUMENT, "state or out is null");
    int rc = use_device(s);
    if (rc) return rc;
    if (s->device < 0 || s->device >= kMaxDevices) return set_err(QD_ERR_NOT_SUPPORTED, "device index too large");
    std::lock_guard<std::mutex> lock(g_red_mu);
    double*& red = g_red[s->device];
    if (!red) {
        if (hipMalloc(reinterpret_cast<void**>(&red), (kRedScratch + 1) * sizeof(double)) != hipSuccess) {
            red = nullptr;
            return set_err(QD_ERR_OUT_OF_MEMORY, "reduction scratch allocation failed");
        }
    }
    QD_HIP(launch_sumsq(s->psi, s->precision, s->D, red, red + kRedScratch, s->stream), "norm");
    double nrm = 0.0;
    QD_HIP(hipMemcpyAsync(&nrm, red + kRedScratch, sizeof(double), hipMemcpyDeviceToHost, s->stream), "norm");
    QD_HIP(hipStreamSynchronize(s->stream), "norm");
    *out = nrm;
    return QD_OK;
}

// ---- the norm without allocation --------------------------------------------------

namespace {

// Partial sums of qd_norm_noalloc: one region of kRedScratch doubles per state of
// a call, in a fixed array of every GPU the library runs on (held until the
// process ends). Host code never passes the array's name to a kernel: it uses
// the device address hipGetSymbolAddress returns, one per device.
static __device__ __align__(256) double scratch[QD_NOALLOC_MAX_STATES * kRedScratch];

std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device (looked up once per device).
int noalloc_scratch(int device, double** out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    double*& p = g_scratch_ptr[device];
    if (!p) {
        void* addr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&addr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_err(e, "looking up the no-allocation scratch");
        p = static_cast<double*>(addr);
    }
    *out = p;
    return QD_OK;
}

}  // namespace

int qd_norm_noalloc(const qd_state* const* states, int32_t count, double* out) {
    if (!states || !out) return set_err(QD_ERR_INVALID_ARGUMENT, "states or out is null");
    if (count < 1) return set_err(QD_ERR_INVALID_ARGUMENT, "count must be at least 1");
    if (count > QD_NOALLOC_MAX_STATES)
        return set_err(QD_ERR_NOT_SUPPORTED, "qd_norm_noalloc takes at most QD_NOALLOC_MAX_STATES (64) states per "
                                             "call; its fixed scratch holds the partial sums of 64 states");
    int device = -1;
    QD_HIP(hipGetDevice(&device), "hipGetDevice");
    if (device < 0 || device >= kMaxDevices) return set_err(QD_ERR_NOT_SUPPORTED, "device index too large");
    for (int32_t i = 0; i < count; ++i) {
        if (!states[i]) return set_err(QD_ERR_INVALID_ARGUMENT, "a state is null");
        if (states[i]->device != device)
            return set_err(QD_ERR_INVALID_ARGUMENT, "every state must be on the current device");
        for (int32_t j = 0; j < i; ++j)
            if (states[j] == states[i]) return set_err(QD_ERR_INVALID_ARGUMENT, "a state is listed twice");
    }
    double* part = nullptr;
    int rc = noalloc_scratch(device, &part);
    if (rc) return rc;
    for (int32_t i = 0; i < count; ++i) {
        const qd_state* s = states[i];
        QD_HIP(launch_sumsq(s->psi, s->precision, s->D, part + (size_t)i * kRedScratch, out + i, s->stream),
               "norm without allocation");
    }
    return QD_OK;
}

int qd_probabilities(const qd_state* s, double* out, uint64_t len, int32_t location) {
    if (!s || !out) return set_err(QD_ERR_INVALID_ARGUMENT, "state or out is null");
    if (location != QD_DEVICE && location != QD_HOST)
        return set_err(QD_ERR_INVALID_ARGUMENT, "location must be QD_DEVICE or QD_HOST");
    if (len < s->D) return set_err(QD_ERR_BUFFER_TOO_SMALL, "output shorter than D");
    int rc = use_device(s);
    if (rc) return rc;
    if (location == QD_DEVICE) {
        QD_HIP(launch_probabilities(s->psi, s->precision, 0, s->D, out, s->stream), "probabilities");
        return QD_OK;
    }
    const uint64_t chunk = std::min<uint64_t>(s->D, 1ull << 24);
    double* tmp = nullptr;
    if (hipMalloc(reinterpret_cast<void**>(&tmp), chunk * sizeof(double)) != hipSuccess)
        return set_err(QD_ERR_OUT_OF_MEMORY, "probability staging allocation failed");
    for (uint64_t done = 0; done < s->D; done += chunk) {
        const uint64_t c = std::min<uint64_t>(chunk, s->D - done);
        hipError_t e = launch_probabilities(s->psi, s->precision, done, c, tmp, s->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(out + done, tmp, c * sizeof(double), hipMemcpyDeviceToHost, s->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
        if (e != hipSuccess) {
            (void)hipFree(tmp);
            return hip_err(e, "probabilities");
        }
    }
    (void)hipFree(tmp);
    return QD_OK;
}

int qd_copy_ceiling(qd_state* s, int32_t reps, double* best_ms) {
    if (!s || !best_ms) return set_err(QD_ERR_INVALID_ARGUMENT, "state or best_ms is null");
    if (reps < 1) return set_err(QD_ERR_INVALID_ARGUMENT, "reps must be >= 1");
    int rc = use_device(s);
    if (rc) return rc;
    hipEvent_t a, b;
    QD_HIP(hipEventCreate(&a), "event");
    QD_HIP(hipEventCreate(&b), "event");
    float best = -1.0f;
    hipError_t e = launch_stream_rewrite(s->psi, s->precision, s->D, s->stream);  // warm-up
    for (int i = 0; i < reps && e == hipSuccess; ++i) {
        e = hipEventRecord(a, s->stream);
        if (e == hipSuccess) e = launch_stream_rewrite(s->psi, s->precision, s->D, s->stream);
        if (e == hipSuccess) e = hipEventRecord(b, s->stream);
        if (e == hipSuccess) e = hipEventSynchronize(b);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
        if (e == hipSuccess && (best < 0.0f || ms < best)) best = ms;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (e != hipSuccess) return hip_err(e, "copy ceiling");
    *best_ms = best;
    return QD_OK;
}

int qd_synchronize(const qd_state* s) {
    if (!s) return set_err(QD_ERR_INVALID_ARGUMENT, "state is null");
    int rc = use_device(s);
    if (rc) return rc;
    QD_HIP(hipStreamSynchronize(s->stream), "synchronize");
    QD_HIP(hipGetLastError(), "asynchronous error");
    return QD_OK;
}

}  // extern "C"
