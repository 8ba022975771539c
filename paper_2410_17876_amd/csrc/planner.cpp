// planner.cpp - validation and per-gate planning on the host.
//
// Builds a GatePlan from dims, targets, controls and U (plan.h explains the
// decode). The gate category follows the paper's three single-qudit cases
// (Sec. 2): phase gates are diagonal (Sec. 2.1), permutation gates map each
// basis state to one other (Sec. 2.2), everything else creates superpositions
// (Sec. 2.3). The category is read from U's exact zero pattern: diagonal if
// every off-diagonal entry is 0; monomial (a permutation with phases) if every
// row and every column has exactly one non-zero; dense otherwise. Entries of a
// monomial U that map |a> to itself with factor exactly 1 are identity columns
// and are skipped, so e.g. a qudit Z gate does not touch the amplitudes with
// target digit 0.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "planner.h"

namespace qd {

static int fail(std::string* err, int code, const char* fmt, ...) {
    if (err) {
        char buf[256];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        *err = buf;
    }
    return code;
}

bool free_segments(const int32_t* dims, int n, const bool* special, int* nseg, uint64_t* size, uint64_t* stride,
                   uint64_t* n_free) {
    // Maximal runs of consecutive non-special qudits, least significant first.
    uint64_t s = 1, prod = 1;
    int ns = 0;
    for (int i = 0; i < n; ++i) {
        if (!special[i]) {
            if (i > 0 && !special[i - 1] && ns > 0) {
                size[ns - 1] *= (uint64_t)dims[i];
            } else {
                if (ns >= kMaxSeg) return false;
                size[ns] = (uint64_t)dims[i];
                stride[ns] = s;
                ++ns;
            }
            prod *= (uint64_t)dims[i];
        }
        s *= (uint64_t)dims[i];
    }
    *nseg = ns;
    *n_free = prod;
    return true;
}

int check_dims(const int32_t* dims, int32_t n, uint64_t* D, std::string* err) {
    if (!dims) return fail(err, QD_ERR_INVALID_ARGUMENT, "dims is null");
    if (n < 1 || n > QD_MAX_QUDITS)
        return fail(err, QD_ERR_INVALID_ARGUMENT, "n = %d qudits outside 1..%d", n, QD_MAX_QUDITS);
    uint64_t prod = 1;
    bool overflow = false;
    for (int i = 0; i < n; ++i) {
        if (dims[i] < QD_MIN_DIM || dims[i] > QD_MAX_DIM)
            return fail(err, QD_ERR_INVALID_ARGUMENT, "dims[%d] = %d outside %d..%d", i, dims[i], QD_MIN_DIM,
                        QD_MAX_DIM);
        if (prod > (uint64_t)INT64_MAX / (uint64_t)dims[i]) overflow = true;
        else prod *= (uint64_t)dims[i];
    }
    if (overflow) return fail(err, QD_ERR_DIM_OVERFLOW, "D = prod dims does not fit a signed 64-bit index");
    if (D) *D = prod;
    return QD_OK;
}

int sparse_layout(const int32_t* dims, int32_t n, int* word, uint64_t* stride, int* W, uint64_t* P, uint64_t* D_lo,
                  uint64_t* D_hi, std::string* err) {
    if (!dims) return fail(err, QD_ERR_INVALID_ARGUMENT, "dims is null");
    if (n < 1 || n > QD_SPARSE_MAX_QUDITS)
        return fail(err, QD_ERR_INVALID_ARGUMENT, "n = %d qudits outside 1..%d", n, QD_SPARSE_MAX_QUDITS);
    unsigned __int128 D = 1;
    const unsigned __int128 limit = (unsigned __int128)1 << 127;
    int w = 0;
    uint64_t pw = 1;  // product of the dims packed into word w so far
    for (int i = 0; i < n; ++i) {
        if (dims[i] < QD_MIN_DIM || dims[i] > QD_MAX_DIM)
            return fail(err, QD_ERR_INVALID_ARGUMENT, "dims[%d] = %d outside %d..%d", i, dims[i], QD_MIN_DIM,
                        QD_MAX_DIM);
        if (D > (limit - 1) / (unsigned)dims[i])
            return fail(err, QD_ERR_DIM_OVERFLOW, "D = prod dims is not below 2^127");
        D *= (unsigned)dims[i];
        // A word takes qudits while the product of their dims stays below 2^64.
        // A full word holds more than 2^64 / 7, so D < 2^127 needs at most 3.
        if (pw > UINT64_MAX / (uint64_t)dims[i]) {
            if (P) P[w] = pw;
            if (++w >= kSparseKeyWords) return fail(err, QD_ERR_DIM_OVERFLOW, "register needs more than 3 key words");
            pw = 1;
        }
        if (word) word[i] = w;
        if (stride) stride[i] = pw;
        pw *= (uint64_t)dims[i];
    }
    if (P) {
        P[w] = pw;
        for (int j = w + 1; j < kSparseKeyWords; ++j) P[j] = 1;
    }
    if (W) *W = w + 1;
    if (D_lo) *D_lo = (uint64_t)D;
    if (D_hi) *D_hi = (uint64_t)(D >> 64);
    return QD_OK;
}

int check_gate_shape(const int32_t* dims, int32_t n, const int32_t* targets, int32_t k, const int32_t* controls,
                     const int32_t* values, int32_t m, std::string* err) {
    if (k < 1) return fail(err, QD_ERR_INVALID_ARGUMENT, "a gate needs at least one target (k = %d)", k);
    if (!targets) return fail(err, QD_ERR_INVALID_ARGUMENT, "targets is null");
    if (m < 0) return fail(err, QD_ERR_INVALID_ARGUMENT, "negative control count %d", m);
    if (m > 0 && (!controls || !values)) return fail(err, QD_ERR_INVALID_ARGUMENT, "controls or values is null");
    bool used[QD_SPARSE_MAX_QUDITS] = {false};
    for (int l = 0; l < k; ++l) {
        const int t = targets[l];
        if (t < 0 || t >= n) return fail(err, QD_ERR_INVALID_ARGUMENT, "target %d outside 0..%d", t, n - 1);
        if (used[t]) return fail(err, QD_ERR_INVALID_ARGUMENT, "target %d listed twice", t);
        used[t] = true;
    }
    for (int l = 0; l < m; ++l) {
        const int c = controls[l];
        if (c < 0 || c >= n) return fail(err, QD_ERR_INVALID_ARGUMENT, "control %d outside 0..%d", c, n - 1);
        if (used[c]) return fail(err, QD_ERR_INVALID_ARGUMENT, "control %d repeats a target or control", c);
        used[c] = true;
        if (values[l] < 0 || values[l] >= dims[c])
            return fail(err, QD_ERR_INVALID_ARGUMENT, "control value %d for qudit %d outside 0..%d", values[l], c,
                        dims[c] - 1);
    }
    if (k > QD_MAX_TARGETS)
        return fail(err, QD_ERR_NOT_SUPPORTED, "%d targets; at most %d are supported", k, QD_MAX_TARGETS);
    if (m > QD_MAX_CONTROLS)
        return fail(err, QD_ERR_NOT_SUPPORTED, "%d controls; at most %d are supported", m, QD_MAX_CONTROLS);
    return QD_OK;
}

int check_gate(const int32_t* dims, int32_t n, const int32_t* targets, int32_t k, const int32_t* controls,
               const int32_t* values, int32_t m, std::string* err) {
    int rc = check_dims(dims, n, nullptr, err);
    if (rc) return rc;
    return check_gate_shape(dims, n, targets, k, controls, values, m, err);
}

static bool is_zero(const double* U, int i) { return U[2 * i] == 0.0 && U[2 * i + 1] == 0.0; }

bool unitary_check_enabled() {
    const char* e = getenv("QD_CHECK_UNITARY");
    return e && e[0] && !(e[0] == '0' && e[1] == 0);
}

// max over (r, c) of |(U^dagger U)_rc - [r == c]| for an M x M row-major
// interleaved complex U (NaN if an entry is not finite).
double unitary_deviation(const double* U, int M) {
    double worst = 0.0;
    for (int r = 0; r < M; ++r)
        for (int c = 0; c < M; ++c) {
            double re = 0.0, im = 0.0;  // sum_a conj(U[a][r]) U[a][c]
            for (int a = 0; a < M; ++a) {
                const double ur = U[2 * ((size_t)a * M + r)], ui = U[2 * ((size_t)a * M + r) + 1];
                const double vr = U[2 * ((size_t)a * M + c)], vi = U[2 * ((size_t)a * M + c) + 1];
                re += ur * vr + ui * vi;
                im += ur * vi - ui * vr;
            }
            const double d = std::hypot(re - (r == c ? 1.0 : 0.0), im);
            if (std::isnan(d)) return d;
            if (d > worst) worst = d;
        }
    return worst;
}

int plan_gate(const int32_t* dims, int32_t n, const int32_t* targets, int32_t k, const int32_t* controls,
              const int32_t* values, int32_t m, const double* U, GatePlan* p, std::string* err) {
    int rc = check_gate(dims, n, targets, k, controls, values, m, err);
    if (rc) return rc;
    if (!p) return fail(err, QD_ERR_INVALID_ARGUMENT, "plan is null");
    uint64_t D = 0;
    check_dims(dims, n, &D, err);
    std::memset(p, 0, sizeof *p);
    p->n = n;
    p->D = D;
    uint64_t s[QD_MAX_QUDITS];
    s[0] = 1;
    for (int i = 1; i < n; ++i) s[i] = s[i - 1] * (uint64_t)dims[i - 1];

    bool special[QD_MAX_QUDITS] = {false};
    int M = 1;
    for (int l = 0; l < k; ++l) {
        special[targets[l]] = true;
        M *= dims[targets[l]];
    }
    p->M = M;
    p->ctrl_off = 0;
    for (int l = 0; l < m; ++l) {
        special[controls[l]] = true;
        p->ctrl_off += (uint64_t)values[l] * s[controls[l]];
    }
    if (!free_segments(dims, n, special, &p->nseg, p->seg_size, p->seg_stride, &p->n_classes))
        return fail(err, QD_ERR_NOT_SUPPORTED, "too many free-qudit segments");
    // Member offsets: local index a -> sum_l a_l s_{t_l}, first target least significant.
    for (int a = 0; a < M; ++a) {
        int rest = a;
        int64_t off = 0;
        for (int l = 0; l < k; ++l) {
            off += (int64_t)(rest % dims[targets[l]]) * (int64_t)s[targets[l]];
            rest /= dims[targets[l]];
        }
        p->off[a] = off;
    }
    if (!U) return fail(err, QD_ERR_INVALID_ARGUMENT, "U is null");
    if (unitary_check_enabled()) {
        const double dev = unitary_deviation(U, M);
        if (!(dev <= kUnitaryTol))
            return fail(err, QD_ERR_INVALID_ARGUMENT, "U is not unitary: max |(U^dagger U - I)_rc| = %.3g", dev);
    }

    // Category from the exact zero pattern.
    bool diag = true;
    for (int r = 0; r < M && diag; ++r)
        for (int a = 0; a < M; ++a)
            if (r != a && !is_zero(U, r * M + a)) {
                diag = false;
                break;
            }
    int row_of[kMaxM];
    bool mono = true;
    {
        int row_count[kMaxM] = {0};
        for (int a = 0; a < M && mono; ++a) {
            int nz = 0;
            for (int r = 0; r < M; ++r)
                if (!is_zero(U, r * M + a)) {
                    ++nz;
                    row_of[a] = r;
                }
            if (nz != 1) mono = false;
            else ++row_count[row_of[a]];
        }
        for (int r = 0; r < M && mono; ++r)
            if (row_count[r] != 1) mono = false;
    }
    if (mono) {
        p->n_active = 0;
        for (int a = 0; a < M; ++a) {
            const int r = row_of[a];
            const double lr = U[2 * (r * M + a)], li = U[2 * (r * M + a) + 1];
            const bool one = lr == 1.0 && li == 0.0;
            if (r == a && one) continue;  // identity column: nothing to do
            const int i = p->n_active++;
            p->src[i] = a;
            p->dst[i] = r;
            p->lam[2 * i] = lr;
            p->lam[2 * i + 1] = li;
            p->lam_one[i] = one ? 1 : 0;
        }
        p->category = p->n_active == 0 ? kIdentity : (diag ? kDiagonal : kMonomial);
    } else {
        p->category = kDense;
        p->n_active = M;
    }
    return QD_OK;
}

void plan_info(const GatePlan& p, int precision, qd_gate_info* info) {
    std::memset(info, 0, sizeof *info);
    const int fam = plan_family(p, precision);
    std::snprintf(info->kernel, sizeof info->kernel, "%s", family_name(fam));
    info->category = p.category;
    info->M = p.M;
    info->classes = p.n_classes;
    const uint64_t ab = amp_bytes(precision);
    if (p.category == kIdentity) return;
    if (p.category == kDense) {
        info->updated = p.n_classes * (uint64_t)p.M;
        info->flops = 8ull * info->updated * (uint64_t)p.M;
    } else {
        info->updated = p.n_classes * (uint64_t)p.n_active;
        uint64_t scaled = 0;
        for (int i = 0; i < p.n_active; ++i) scaled += p.lam_one[i] ? 0 : 1;
        info->flops = 8ull * p.n_classes * scaled;
    }
    info->bytes = 2ull * info->updated * ab;
}

}  // namespace qd
