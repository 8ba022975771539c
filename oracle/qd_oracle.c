/*
 * qd_oracle.c - reference CPU simulator for mixed-radix qudit statevectors (FP64).
 *
 * TEST INFRASTRUCTURE ONLY. This file exists to check the GPU library. Only the
 * test suite, the package's smoke check and the benchmark's CPU-baseline leg may
 * load it. It shares no code, header, table or helper with the GPU library, and
 * it is deliberately plain and slow: no blocking, no fusion, no special cases.
 *
 * What it computes (arXiv 2410.17876, "Fast classical simulation of qubit-qudit
 * hybrid systems"):
 *
 *   Register (Sec. 2): n qudits q_0..q_{n-1} with dims d_0..d_{n-1}, q_0 least
 *   significant; amplitude j (0 <= j < D = prod d_i) belongs to basis state |j>.
 *
 *   Blocks (Sec. 2.3, block-size rule): for qudit i the block size is
 *   s_i = prod_{t<i} d_t, so the value of qudit i in |j> is floor(j / s_i) mod d_i.
 *
 *   Controls (Sec. 2.4, control equation): |j> satisfies control k with value
 *   v_k iff floor(j / b_k) mod d_k = v_k, b_k the block size of q_k. Every index
 *   is tested, which is the O(D * #controls) scan the paper describes.
 *
 *   Classes (Sec. 2.3, Table 2): the amplitudes that differ only in the target
 *   digits form a class; U acts on each class independently. Column a of U is
 *   the image of local basis state |a>, so the class's new amplitudes are
 *   sum_a x_a * U[:, a] (scalar times column, then vector sum), a ascending.
 *   For k target qudits t_0..t_{k-1} the local index is
 *   a = sum_l a_l prod_{l'<l} d_{t_l'} (first target least significant), and
 *   member a of the class with base j sits at j + sum_l a_l s_{t_l}.
 *
 *   Multi-valued controls (left open by the paper after Sec. 2.4): control k
 *   accepts a set of values, tested the same way with "in the set" for "equals"
 *   (oracle_apply_masked).
 *
 *   Phase and permutation gates (Sec. 2.1, 2.2) are not special-cased: they go
 *   through the same class matvec, whose result is identical for finite inputs.
 *
 * Arithmetic: complex products are the textbook (ac - bd) + i(ad + bc) and sums
 * run in ascending order; the file is compiled with -ffp-contract=off so no FMA
 * is formed. Norms use Neumaier's compensated summation.
 *
 * Threads: the scan over j may be split over OpenMP threads (oracle_set_threads;
 * one thread unless set). Classes are disjoint (Sec. 2.3) and each base index
 * only reads and writes its own class, so every amplitude sees exactly the same
 * operations in the same order whatever the thread count; the result is
 * bitwise the same.
 *
 * Amplitudes are stored as interleaved (re, im) doubles. All functions return
 * 0 on success and a negative value on invalid arguments.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_MAX_QUDITS 64
#define ORACLE_MAX_TARGETS 3
#define ORACLE_MAX_M 343

/* D = prod d_i; -1 if a dim is outside 2..7 or D >= 2^63. */
int64_t oracle_dim(int n, const int *dims) {
    if (n < 1 || n > ORACLE_MAX_QUDITS) return -1;
    int64_t D = 1;
    for (int i = 0; i < n; ++i) {
        if (dims[i] < 2 || dims[i] > 7) return -1;
        if (D > INT64_MAX / dims[i]) return -1;
        D *= dims[i];
    }
    return D;
}

static int oracle_nthreads = 1;

/* Threads for the scans of oracle_apply and oracle_apply_masked (>= 1). */
int oracle_set_threads(int n) {
    if (n < 1) return -1;
    oracle_nthreads = n;
    return 0;
}

int oracle_get_threads(void) { return oracle_nthreads; }

/* Block sizes s_i = prod_{t<i} d_t (Sec. 2.3). */
static void block_sizes(int n, const int *dims, int64_t *s) {
    s[0] = 1;
    for (int i = 1; i < n; ++i) s[i] = s[i - 1] * dims[i - 1];
}

static int digit(int64_t j, int64_t s, int d) { return (int)((j / s) % d); }

static int check_gate(int n, const int *dims, int k, const int *targets, int m,
                      const int *controls, const int *cvals, int *M_out) {
    if (oracle_dim(n, dims) < 0) return -1;
    if (k < 1 || k > ORACLE_MAX_TARGETS || m < 0 || m > n) return -1;
    int used[ORACLE_MAX_QUDITS];
    memset(used, 0, sizeof used);
    int M = 1;
    for (int l = 0; l < k; ++l) {
        if (targets[l] < 0 || targets[l] >= n || used[targets[l]]) return -1;
        used[targets[l]] = 1;
        M *= dims[targets[l]];
    }
    for (int l = 0; l < m; ++l) {
        if (controls[l] < 0 || controls[l] >= n || used[controls[l]]) return -1;
        used[controls[l]] = 1;
        if (cvals[l] < 0 || cvals[l] >= dims[controls[l]]) return -1;
    }
    if (M > ORACLE_MAX_M) return -1;
    *M_out = M;
    return 0;
}

/* Address offset of local index a: sum_l a_l s_{t_l}, a_l the mixed-radix
 * digits of a over the target dims, first target least significant. */
static int64_t local_offset(int a, int k, const int *targets, const int *dims, const int64_t *s) {
    int64_t off = 0;
    for (int l = 0; l < k; ++l) {
        int d = dims[targets[l]];
        off += (int64_t)(a % d) * s[targets[l]];
        a /= d;
    }
    return off;
}

/* Local index of basis state |j> within its class. */
static int local_index(int64_t j, int k, const int *targets, const int *dims, const int64_t *s) {
    int a = 0, w = 1;
    for (int l = 0; l < k; ++l) {
        a += digit(j, s[targets[l]], dims[targets[l]]) * w;
        w *= dims[targets[l]];
    }
    return a;
}

static int controls_hold(int64_t j, int m, const int *controls, const int *cvals, const int *dims,
                         const int64_t *s) {
    for (int l = 0; l < m; ++l)
        if (digit(j, s[controls[l]], dims[controls[l]]) != cvals[l]) return 0;
    return 1;
}

/* y = U x for one class: y[r] = sum_{a ascending} U[r][a] * x[a]. */
static void class_matvec(int M, const double *U, const double *x, double *y) {
    for (int r = 0; r < M; ++r) {
        double yr = 0.0, yi = 0.0;
        for (int a = 0; a < M; ++a) {
            double ur = U[2 * (r * M + a)], ui = U[2 * (r * M + a) + 1];
            double xr = x[2 * a], xi = x[2 * a + 1];
            yr = yr + (ur * xr - ui * xi);
            yi = yi + (ur * xi + ui * xr);
        }
        y[2 * r] = yr;
        y[2 * r + 1] = yi;
    }
}

int oracle_init_zero(int n, const int *dims, double *psi) {
    int64_t D = oracle_dim(n, dims);
    if (D < 0) return -1;
    memset(psi, 0, (size_t)D * 2 * sizeof(double));
    psi[0] = 1.0;
    return 0;
}

/* Apply a (controlled) k-qudit gate in place.
 * U: M x M complex, row-major [out][in], interleaved (re, im). */
int oracle_apply(int n, const int *dims, double *psi, int k, const int *targets, int m,
                 const int *controls, const int *cvals, const double *U) {
    int M;
    if (check_gate(n, dims, k, targets, m, controls, cvals, &M) != 0) return -1;
    int64_t D = oracle_dim(n, dims);
    int64_t s[ORACLE_MAX_QUDITS];
    block_sizes(n, dims, s);
    int64_t off[ORACLE_MAX_M];
    for (int a = 0; a < M; ++a) off[a] = local_offset(a, k, targets, dims, s);
#pragma omp parallel for schedule(static) num_threads(oracle_nthreads)
    for (int64_t j = 0; j < D; ++j) {
        double x[2 * ORACLE_MAX_M], y[2 * ORACLE_MAX_M];
        /* j is a class base iff every target digit is 0 ... */
        int base = 1;
        for (int l = 0; l < k && base; ++l)
            if (digit(j, s[targets[l]], dims[targets[l]]) != 0) base = 0;
        /* ... and every control condition holds. */
        if (!base || !controls_hold(j, m, controls, cvals, dims, s)) continue;
        for (int a = 0; a < M; ++a) {
            x[2 * a] = psi[2 * (j + off[a])];
            x[2 * a + 1] = psi[2 * (j + off[a]) + 1];
        }
        class_matvec(M, U, x, y);
        for (int a = 0; a < M; ++a) {
            psi[2 * (j + off[a])] = y[2 * a];
            psi[2 * (j + off[a]) + 1] = y[2 * a + 1];
        }
    }
    return 0;
}

/* Multi-valued controls (the paper leaves them open after Sec. 2.4; read here as:
 * control l accepts a set V_l of values): |j> satisfies control l iff
 * floor(j / b_l) mod d_l is in V_l, with V_l given as a bit mask (bit v set iff
 * v is in V_l). Every index is tested, as in oracle_apply. A mask must be
 * non-empty and hold only values below d_l. */
static int controls_hold_masked(int64_t j, int m, const int *controls, const uint32_t *masks, const int *dims,
                                const int64_t *s) {
    for (int l = 0; l < m; ++l)
        if (((masks[l] >> digit(j, s[controls[l]], dims[controls[l]])) & 1u) == 0) return 0;
    return 1;
}

int oracle_apply_masked(int n, const int *dims, double *psi, int k, const int *targets, int m,
                        const int *controls, const uint32_t *masks, const double *U) {
    int zeros[ORACLE_MAX_QUDITS];
    int M;
    if (m < 0 || m > ORACLE_MAX_QUDITS) return -1;
    memset(zeros, 0, sizeof zeros);
    if (check_gate(n, dims, k, targets, m, controls, zeros, &M) != 0) return -1;
    for (int l = 0; l < m; ++l)
        if (masks[l] == 0 || (masks[l] >> dims[controls[l]]) != 0) return -1;
    int64_t D = oracle_dim(n, dims);
    int64_t s[ORACLE_MAX_QUDITS];
    block_sizes(n, dims, s);
    int64_t off[ORACLE_MAX_M];
    for (int a = 0; a < M; ++a) off[a] = local_offset(a, k, targets, dims, s);
#pragma omp parallel for schedule(static) num_threads(oracle_nthreads)
    for (int64_t j = 0; j < D; ++j) {
        double x[2 * ORACLE_MAX_M], y[2 * ORACLE_MAX_M];
        int base = 1;
        for (int l = 0; l < k && base; ++l)
            if (digit(j, s[targets[l]], dims[targets[l]]) != 0) base = 0;
        if (!base || !controls_hold_masked(j, m, controls, masks, dims, s)) continue;
        for (int a = 0; a < M; ++a) {
            x[2 * a] = psi[2 * (j + off[a])];
            x[2 * a + 1] = psi[2 * (j + off[a]) + 1];
        }
        class_matvec(M, U, x, y);
        for (int a = 0; a < M; ++a) {
            psi[2 * (j + off[a])] = y[2 * a];
            psi[2 * (j + off[a]) + 1] = y[2 * a + 1];
        }
    }
    return 0;
}

/* Sampled form of oracle_apply, for states too large to hold: for each output
 * index j_out it lists the M input addresses its new value depends on.
 * members: nsamp * M addresses; row[i] = local index of j_out in its class, or
 * -1 when the controls do not hold (the amplitude is unchanged; then every
 * member entry is j_out itself). */
int oracle_class_members(int n, const int *dims, int k, const int *targets, int m,
                         const int *controls, const int *cvals, int64_t nsamp,
                         const int64_t *out_idx, int64_t *members, int32_t *row) {
    int M;
    if (check_gate(n, dims, k, targets, m, controls, cvals, &M) != 0) return -1;
    int64_t D = oracle_dim(n, dims);
    int64_t s[ORACLE_MAX_QUDITS];
    block_sizes(n, dims, s);
    for (int64_t i = 0; i < nsamp; ++i) {
        int64_t j = out_idx[i];
        if (j < 0 || j >= D) return -1;
        if (!controls_hold(j, m, controls, cvals, dims, s)) {
            row[i] = -1;
            for (int a = 0; a < M; ++a) members[i * M + a] = j;
            continue;
        }
        int r = local_index(j, k, targets, dims, s);
        int64_t base = j - local_offset(r, k, targets, dims, s);
        row[i] = r;
        for (int a = 0; a < M; ++a) members[i * M + a] = base + local_offset(a, k, targets, dims, s);
    }
    return 0;
}

/* New amplitude of each sample from its gathered class inputs x (nsamp * M
 * complex, in local-index order): out[i] = sum_a U[row][a] x[a], or x[0] when
 * row[i] = -1. */
int oracle_rows(int M, const double *U, int64_t nsamp, const double *x, const int32_t *row,
                double *out) {
    if (M < 1 || M > ORACLE_MAX_M) return -1;
    for (int64_t i = 0; i < nsamp; ++i) {
        const double *xi = x + 2 * i * M;
        int r = row[i];
        if (r < 0) {
            out[2 * i] = xi[0];
            out[2 * i + 1] = xi[1];
            continue;
        }
        if (r >= M) return -1;
        double yr = 0.0, yi = 0.0;
        for (int a = 0; a < M; ++a) {
            double ur = U[2 * (r * M + a)], ui = U[2 * (r * M + a) + 1];
            double xr = xi[2 * a], xim = xi[2 * a + 1];
            yr = yr + (ur * xr - ui * xim);
            yi = yi + (ur * xim + ui * xr);
        }
        out[2 * i] = yr;
        out[2 * i + 1] = yi;
    }
    return 0;
}

/* sum of |a_j|^2 over j, Neumaier-compensated, in ascending j. */
static double sumsq(const double *psi, int64_t D) {
    double sum = 0.0, comp = 0.0;
    for (int64_t j = 0; j < D; ++j) {
        double p = psi[2 * j] * psi[2 * j] + psi[2 * j + 1] * psi[2 * j + 1];
        double t = sum + p;
        if (fabs(sum) >= fabs(p))
            comp += (sum - t) + p;
        else
            comp += (p - t) + sum;
        sum = t;
    }
    return sum + comp;
}

/* ||psi||_2 = sqrt(sum |a_j|^2). */
int oracle_norm(int64_t D, const double *psi, double *out) {
    if (D < 1) return -1;
    *out = sqrt(sumsq(psi, D));
    return 0;
}

/* p_j = |a_j|^2 = re^2 + im^2. */
int oracle_probabilities(int64_t D, const double *psi, double *out) {
    if (D < 1) return -1;
    for (int64_t j = 0; j < D; ++j) out[j] = psi[2 * j] * psi[2 * j] + psi[2 * j + 1] * psi[2 * j + 1];
    return 0;
}
