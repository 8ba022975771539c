/*
 * qd.h - C ABI of libqd, a GPU (gfx950) simulator for mixed-radix qudit
 * statevectors by block simulation (arXiv 2410.17876, "Fast classical simulation
 * of qubit-qudit hybrid systems").
 *
 * Problem statement (paper Sec. 2): a register of n qudits q_0..q_{n-1} with
 * dimensions d_0..d_{n-1} (each 2..7 here), q_0 least significant. The state is
 * the vector of D = prod d_i complex amplitudes; amplitude j belongs to basis
 * state |j> with j = sum_i x_i s_i, s_i = prod_{t<i} d_t (the block size of
 * qudit i, Sec. 2.3). A gate applies an M x M unitary U to the target qudits of
 * every class of amplitudes that differ only in the target digits (Sec. 2.3,
 * Table 2), optionally only where control qudits hold given values (Sec. 2.4),
 * without forming a Kronecker product or the D x D operator.
 *
 * Conventions shared by every call:
 *   - Amplitudes are interleaved (re, im). A state holds them on the GPU in
 *     complex64 (QD_C64, 8 bytes per amplitude) or complex128 (QD_C128, 16 bytes).
 *     Host-side amplitude buffers are always FP64 interleaved.
 *   - Gate matrices are M x M complex FP64, row-major U[out][in], interleaved.
 *     Column a is the image of local basis state |a> (Sec. 2.3), so every class
 *     x becomes U x. For targets t_0..t_{k-1} the local index is
 *     a = sum_l a_l prod_{l'<l} d_{t_l'}: the FIRST listed target is the least
 *     significant local digit. U is rounded once to the state's precision.
 *   - Every call returns QD_OK (0) or a negative qd_status. No exception or
 *     abort crosses the ABI. qd_last_error() returns a thread-local message for
 *     the last failing call of the calling thread.
 *   - Arguments are validated on the host before any device work, so invalid
 *     input never reaches a kernel. Unitarity of U is the caller's contract; with
 *     the environment variable QD_CHECK_UNITARY set to anything but "0", every
 *     gate given to the library is also checked: each entry of U^dagger U - I
 *     must be at most 1e-10 in modulus (finite entries only), else the call fails
 *     with QD_ERR_INVALID_ARGUMENT before any work (a debugging aid: it costs
 *     O(M^3) host flops per gate).
 *   - The caller owns every array it passes; the library copies what it keeps
 *     before returning, so inputs may be freed or reused right away.
 *   - Calls that enqueue device work (apply, reset) are asynchronous on the
 *     state's stream; a device fault is reported by the next synchronizing call
 *     (qd_norm, qd_probabilities, get/set_amplitudes, qd_synchronize).
 *   - One state must not be used from two threads at once. Different states on
 *     different streams are independent.
 */
#ifndef QD_H
#define QD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qd_state qd_state;
typedef struct qd_gate_desc qd_gate_desc; /* one gate of a gate list (defined below) */

enum qd_precision { QD_C64 = 1, QD_C128 = 2 };

enum qd_status {
    QD_OK = 0,
    QD_ERR_INVALID_ARGUMENT = -1, /* bad dims, targets, controls, values, sizes or null pointers */
    QD_ERR_DIM_OVERFLOW = -2,     /* D = prod d_i does not fit a signed 64-bit index */
    QD_ERR_OUT_OF_MEMORY = -3,    /* a device or pinned host allocation failed */
    QD_ERR_DEVICE = -4,           /* a HIP runtime call or kernel launch failed */
    QD_ERR_NOT_SUPPORTED = -5,    /* valid but outside this library's limits (see below) */
    QD_ERR_BUFFER_TOO_SMALL = -6  /* an external buffer or output length is too small */
};

enum qd_location { QD_DEVICE = 0, QD_HOST = 1 };

/* Limits. Dims are 2..7. D must stay below 2^63: the paper's largest registers
 * (62 qubits, 39 qutrits, 31 ququads, 27 ququints, Sec. 3) are exactly the
 * largest with d^n < 2^63. A gate has 1..3 targets (M <= 343) and at most
 * QD_MAX_CONTROLS controls. */
#define QD_MIN_DIM 2
#define QD_MAX_DIM 7
#define QD_MAX_QUDITS 62
#define QD_MAX_TARGETS 3
#define QD_MAX_M 343
#define QD_MAX_CONTROLS 24
#define QD_SPARSE_MAX_QUDITS 126

/* ---- host-only calls (no device needed) ---------------------------------- */

/* D = prod dims[i] for a register of n qudits (Sec. 2). Returns
 * QD_ERR_INVALID_ARGUMENT for n < 1, n > QD_MAX_QUDITS, a null pointer or a dim
 * outside 2..7; QD_ERR_DIM_OVERFLOW when D >= 2^63 (Sec. 3 size limit). */
int qd_dim(const int32_t* dims, int32_t n, uint64_t* D);

/* Validate a gate against a register (Sec. 2.3, 2.4): 1 <= k <= 3 distinct
 * targets in range; 0 <= m <= QD_MAX_CONTROLS distinct controls in range and
 * disjoint from the targets; values[l] in [0, d_{controls[l]}). k > 3 or
 * M > 343 give QD_ERR_NOT_SUPPORTED. controls/values may be null when m == 0. */
int qd_check_gate(const int32_t* dims, int32_t n, const int32_t* targets, int32_t k,
                  const int32_t* controls, const int32_t* values, int32_t m);

/* What qd_apply_gate would do for this gate, without doing it. */
typedef struct {
    char kernel[64];          /* name of the kernel family that would run */
    int32_t category;         /* 0 dense (superposition, Sec. 2.3), 1 permutation/monomial
                                 (Sec. 2.2), 2 diagonal (phase, Sec. 2.1), 3 identity */
    int32_t M;                /* class size prod d_t over the targets */
    uint64_t classes;         /* classes the gate visits: D / (M * prod d_c) */
    uint64_t updated;         /* amplitudes read and written (identity rows/columns skipped) */
    uint64_t bytes;           /* algorithmic HBM bytes: 2 * updated * bytes per amplitude */
    uint64_t flops;           /* algorithmic real flops: 8 * classes * M * M for dense,
                                 8 per scaled amplitude for diagonal/monomial */
} qd_gate_info;

int qd_gate_info_for(const int32_t* dims, int32_t n, int32_t precision, const int32_t* targets,
                     int32_t k, const int32_t* controls, const int32_t* values, int32_t m,
                     const double* U, qd_gate_info* info);

/* Class bases the device decoder produces for classes [first, first + count) of a
 * gate, in class order (for host-side checks of the decoder). base = address of
 * local index 0 of the class. */
int qd_class_bases(const int32_t* dims, int32_t n, const int32_t* targets, int32_t k,
                   const int32_t* controls, const int32_t* values, int32_t m, uint64_t first,
                   uint64_t count, uint64_t* bases);

/* ---- states ---------------------------------------------------------------- */

/* Allocate a state of the given dims and precision on the current HIP device,
 * initialised to |0...0> (Sec. 2.5 starts from |00>). The state owns its buffer
 * and uses the null stream until qd_state_set_stream. *out receives the handle. */
int qd_state_create(const int32_t* dims, int32_t n, int32_t precision, qd_state** out);

/* Wrap caller-owned device memory (e.g. a torch tensor) of `bytes` bytes at
 * device_ptr as a state. Contents are left as they are. The memory must outlive
 * the state; QD_ERR_BUFFER_TOO_SMALL if bytes < D * bytes per amplitude. */
int qd_state_create_external(const int32_t* dims, int32_t n, int32_t precision, void* device_ptr,
                             uint64_t bytes, qd_state** out);

/* Free the state (and its buffer if owned). If the state owns device memory
 * (its buffer, or staging for large gates) this first waits for the state's
 * stream; a state wrapping an external buffer is released without waiting,
 * and the buffer's owner must not reuse it before the state's queued work has
 * finished (stream-ordered allocators such as torch's do this by themselves). */
int qd_state_destroy(qd_state* s);

/* Run this state's work on hip_stream (a hipStream_t; null = default stream).
 * Work already queued on the previous stream is waited for first. */
int qd_state_set_stream(qd_state* s, void* hip_stream);

/* Set the state to basis state |j> (0 <= j < D). Asynchronous. */
int qd_state_reset(qd_state* s, uint64_t j);

/* Copy count FP64 interleaved amplitudes from host memory into the state at
 * amplitude offset `offset` (rounded to FP32 for QD_C64). Synchronous. */
int qd_state_set_amplitudes(qd_state* s, const double* host, uint64_t offset, uint64_t count);

/* Copy count amplitudes starting at `offset` to host memory as FP64 interleaved
 * (exactly widened for QD_C64). Synchronous. */
int qd_state_get_amplitudes(const qd_state* s, double* host, uint64_t offset, uint64_t count);

/* Dimension, precision and device pointer of the state's amplitude buffer. */
int qd_state_info(const qd_state* s, uint64_t* D, int32_t* precision, void** device_ptr);

/* ---- the hot path ------------------------------------------------------------ */

/* Apply U to targets[0..k-1], controlled on controls[l] holding values[l]
 * (Sec. 2.1-2.4), in place and asynchronously on the state's stream. Phase
 * (diagonal) and permutation (monomial) matrices are detected from their exact
 * zero pattern and take kernels that move or scale only the amplitudes they
 * change; all others take the dense class sweep. Only classes that satisfy the
 * controls are visited. Validation as qd_check_gate. */
int qd_apply_gate(qd_state* s, const int32_t* targets, int32_t k, const int32_t* controls,
                  const int32_t* values, int32_t m, const double* U);

/* Multi-valued controls (the paper leaves them open after Sec. 2.4): apply U to
 * targets[0..k-1] on every class whose digit at controls[l] lies in the set
 * value_masks[l] for every l (bit v of the mask set iff value v is accepted).
 * A mask must be non-zero and hold only values below the control's dimension;
 * a control whose mask accepts every value is no condition at all. The classes
 * of different accepted-value combinations are disjoint, so the update equals
 * one single-valued controlled gate (qd_apply_gate) per combination, and that
 * is how it runs: each combination's classes are enumerated directly, so every
 * accepted amplitude is read and written once and no index is tested against
 * the sets. Validation as qd_check_gate plus the masks; more than 4096
 * accepted-value combinations (over the controls that are a condition) give
 * QD_ERR_NOT_SUPPORTED; on an error nothing is enqueued. In place and
 * asynchronous, like qd_apply_gate. */
int qd_apply_gate_masked(qd_state* s, const int32_t* targets, int32_t k, const int32_t* controls,
                         const uint32_t* value_masks, int32_t m, const double* U);

/* One gate of a gate list: the arguments of qd_apply_gate. */
struct qd_gate_desc {
    const int32_t* targets;
    int32_t k;
    const int32_t* controls;
    const int32_t* values;
    int32_t m;
    const double* U;
};

typedef struct {
    int32_t fuse;         /* 1 (default when opts is null): LDS-staged fusion of consecutive gates;
                             0: one sweep per gate, exactly as qd_apply_gate */
    int32_t tile_amps;    /* largest tile of a fused pass in amplitudes; 0 = 3072 (c128) / 8192 (c64);
                             at most 32768 and at most 160 KB of LDS */
    int32_t min_run;      /* contiguous run a tile must hold, in amplitudes; 0 = 64 (c128) / 128 (c64) */
    int32_t reorder;      /* look-ahead for commuting gates, in gates; 0 (default): strictly in order.
                             With reorder > 0 a pass may also take a later gate that commutes with every
                             gate it skips (see qd_apply_circuit); must not be negative */
    int32_t passes;       /* out: HBM passes enqueued */
    int32_t fused_passes; /* out: how many of them were fused passes */
} qd_circuit_options;

/* Apply gates[0..count-1] in order, in place and asynchronously. Every gate is
 * validated (as qd_check_gate) before any work is enqueued, so an invalid gate
 * leaves the state untouched. With fusion, runs of consecutive gates whose
 * targets fit one tile are applied in one HBM pass: a workgroup loads a tile (all
 * amplitudes over a small qudit set for one value of the other digits) into LDS,
 * applies the gates of the run in order with the same per-class arithmetic as
 * qd_apply_gate, and writes it back once (Sec. 2.3: each gate maps every class,
 * hence every tile, to itself). The result is bitwise the same as applying the
 * gates one by one. With opts->reorder = 0 (and with opts null) gates are never
 * reordered. With opts->reorder = w > 0, a gate that does not fit the open pass
 * is skipped, and a gate up to w places after the first skipped one still joins
 * the pass if it commutes with every skipped gate: its targets meet none of
 * their targets or controls, and its controls meet none of their targets (the
 * operators act on disjoint qudits or share only control qudits, so they
 * commute exactly). The result is then bitwise that of applying the gates one
 * by one in the planned order (qd_circuit_plan's `order`), which equals the
 * given order's result up to rounding. opts may be null. */
int qd_apply_circuit(qd_state* s, const qd_gate_desc* gates, int32_t count, qd_circuit_options* opts);

/* Host-only: the passes qd_apply_circuit would enqueue for this register and
 * gate list. pass_gates[i] = gates in pass i, pass_tile[i] = tile amplitudes of
 * a fused pass or 0 for a one-gate sweep; order receives the indices of the
 * applied gates in the order they are applied, pass by pass (identity gates
 * are dropped: the entries number the sum of pass_gates). All three may be
 * null, else they need room for `count` entries. *npasses receives the number
 * of passes. */
int qd_circuit_plan(const int32_t* dims, int32_t n, int32_t precision, const qd_gate_desc* gates, int32_t count,
                    const qd_circuit_options* opts, int32_t* pass_gates, int32_t* pass_tile, int32_t* order,
                    int32_t* npasses);

/* ---- sparse statevectors ---------------------------------------------------------- */

/* The sparse form of the method (Sec. 3: GHZ states of up to 62 qubits, 39
 * qutrits, 31 ququads, 27 ququints): only the nonzero amplitudes are kept, as
 * (basis index, complex128 amplitude) pairs in device memory sorted by index.
 * A gate groups the entries by class (Sec. 2.3), applies U to every class that
 * has a nonzero member (absent members are 0), keeps the nonzero results and
 * leaves entries whose controls do not hold (Sec. 2.4) unchanged. The paper's
 * sparse registers stop at a signed 64-bit index (Sec. 3) and it names wider
 * integer keys as the way on (Sec. 4): here a basis index is a key of up to
 * three 64-bit words, so a sparse register may have up to QD_SPARSE_MAX_QUDITS
 * qudits and any D < 2^127 (e.g. 126 qubits, 80 qutrits, 63 ququads, 54
 * ququints). Gates are enqueued on the state's stream (the null stream unless
 * qd_sparse_set_stream); qd_sparse_nnz and the get calls wait for it and report
 * device errors. Use one thread per state; the device is the one current at
 * creation. */
typedef struct qd_sparse qd_sparse;

/* Host-only: D = prod dims of a sparse register as a 128-bit value (*D_lo, *D_hi),
 * and the number of 64-bit words of its keys (*words, 1..3). QD_ERR_INVALID_ARGUMENT
 * for n outside 1..QD_SPARSE_MAX_QUDITS, a null dims or a dim outside 2..7;
 * QD_ERR_DIM_OVERFLOW when D >= 2^127. Output pointers may be null. */
int qd_sparse_dim(const int32_t* dims, int32_t n, uint64_t* D_lo, uint64_t* D_hi, int32_t* words);

/* |0...0> on the register (validation as qd_sparse_dim). Synchronous. */
int qd_sparse_create(const int32_t* dims, int32_t n, qd_sparse** out);

/* Wait for the state's stream, then free the state. */
int qd_sparse_destroy(qd_sparse* s);

/* Run the state's work on hip_stream (null = default stream); work queued on
 * the previous stream is waited for first. */
int qd_sparse_set_stream(qd_sparse* s, void* hip_stream);

/* Apply U (M x M, row-major [out][in], interleaved FP64, copied before the call
 * returns) to targets[0..k-1], controlled on controls[l] holding values[l].
 * Validation as qd_check_gate (on the sparse register); M at most 16 and
 * (stored entries) x M below 2^31 (else QD_ERR_NOT_SUPPORTED). On an error the
 * state is unchanged. Asynchronous: while (stored entries) x M stays within 1024
 * the gate is one kernel launch and reads nothing back; larger gates read the
 * result count back once. */
int qd_sparse_apply_gate(qd_sparse* s, const int32_t* targets, int32_t k, const int32_t* controls,
                         const int32_t* values, int32_t m, const double* U);

/* Apply gates[0..count-1] in order (each as qd_sparse_apply_gate). Every gate is
 * validated before any work is enqueued, so an invalid gate leaves the state
 * unchanged; a device error met part way may leave the result of a prefix of
 * the list. */
int qd_sparse_apply_circuit(qd_sparse* s, const qd_gate_desc* gates, int32_t count);

/* Number of stored (nonzero) amplitudes. Waits for the state's stream. */
int qd_sparse_nnz(qd_sparse* s, uint64_t* nnz);

/* Copy the first min(cap, nnz) entries, in increasing basis index, to host
 * arrays keys[cap] and amps[2 * cap] (interleaved re, im). For registers with
 * D < 2^64 only (else QD_ERR_NOT_SUPPORTED: use qd_sparse_get_wide). Waits for
 * the state's stream. */
int qd_sparse_get(qd_sparse* s, uint64_t* keys, double* amps, uint64_t cap);

/* As qd_sparse_get for any register: keys[2 * cap] receives each basis index as
 * two 64-bit halves (low, high) of its 128-bit value. */
int qd_sparse_get_wide(qd_sparse* s, uint64_t* keys, double* amps, uint64_t cap);

/* ---- batches of independent states ---------------------------------------------- */

/* A batch context holds the staging buffers of qd_batch_apply for one precision.
 * It may be reused for any number of calls; one context must not be used from
 * two threads at once. */
typedef struct qd_batch qd_batch;
int qd_batch_create(int32_t precision, qd_batch** out);
int qd_batch_destroy(qd_batch* b);

/* Apply gate list i (gates[i][0..counts[i]-1]) to states[i] for every i, in
 * order per state, advancing all states together: each state's list is split
 * into fused passes as in qd_apply_circuit, and round r is ONE launch that runs
 * pass r of every state still having one (a workgroup per (state, tile)). A
 * state whose whole register fits one tile runs its whole list in one round.
 * The result of every state is bitwise the same as running its list alone
 * through qd_apply_circuit with the same options. All states must have the
 * batch's precision, fewer than 2^31 amplitudes, and one device and stream
 * (the launches go to that stream); a state may appear once. Everything is
 * validated before any work is enqueued. opts (may be null) gives the tile
 * options; on return opts->passes = rounds launched, opts->fused_passes =
 * (state, pass) items run. */
int qd_batch_apply(qd_batch* b, qd_state* const* states, const qd_gate_desc* const* gates, const int32_t* counts,
                   int32_t nstates, qd_circuit_options* opts);

/* A compiled batch: qd_batch_apply's rounds planned once, with all their
 * descriptors uploaded to one device buffer, for gate lists that are run many
 * times. The states (and their buffers) must outlive the plan, and the plan
 * replays the same gates on their current contents. Every pass must fit a
 * batch item (classes of at most 16 amplitudes), else QD_ERR_NOT_SUPPORTED.
 * opts as for qd_batch_apply (out fields filled). Synchronous (uploads). */
typedef struct qd_batch_plan qd_batch_plan;
int qd_batch_compile(qd_state* const* states, const qd_gate_desc* const* gates, const int32_t* counts,
                     int32_t nstates, qd_circuit_options* opts, qd_batch_plan** out);

/* Enqueue all rounds of the plan on the states' stream: one launch per round,
 * or, with use_graph != 0, one launch of a hipGraph captured from those
 * launches on the first such call. Asynchronous. */
int qd_batch_plan_run(qd_batch_plan* plan, int32_t use_graph);

/* Wait for the plan's stream, then free the plan (not the states). */
int qd_batch_plan_destroy(qd_batch_plan* plan);

/* ||psi||_2 = sqrt(sum_j |a_j|^2) over the amplitudes a_j of the basis states
 * |j> (Sec. 2 sets up the statevector as these amplitudes; every gate there is
 * a unitary, so the norm of a normalised input stays 1 and is the check of a
 * run). Summed in FP64 on the device in a fixed order (the same result for the
 * same state, run after run). Synchronous: it waits for the state's stream. The
 * device's reduction scratch is shared by all states and serialised by a lock. */
int qd_norm(const qd_state* s, double* out);

/* ---- the norm without allocation --------------------------------------------------- */

/* For callers that cannot allocate device memory or wait on a stream: code under
 * HIP graph capture, serving loops that retire requests while others run, and
 * harnesses that forbid hipMalloc. out[i] = ||states[i]||_2, the same value, bit
 * for bit, as qd_norm (the same reduction in the same fixed order), written by
 * the device on states[i]'s stream; out must be device-accessible (device memory,
 * or pinned host memory from hipHostMalloc) with room for `count` doubles, and is
 * valid once that stream has reached this point (synchronize it, or record and
 * wait for an event after the call). The call allocates nothing and does not wait:
 * the partial sums go to a fixed array of the library on each GPU
 * (QD_NOALLOC_MAX_STATES x 1025 doubles, about 513 KB, held until the process
 * ends), so count is 1..QD_NOALLOC_MAX_STATES (more give QD_ERR_NOT_SUPPORTED);
 * every state must be on the current device and listed once. All calls on one
 * GPU share that array and each call rewrites every partial it reads (nothing
 * in it has to start at zero), so calls on one stream are ordered, but calls
 * whose work can overlap in time (on different streams, or states of one call
 * on different streams) race and give wrong norms. */
#define QD_NOALLOC_MAX_STATES 64
int qd_norm_noalloc(const qd_state* const* states, int32_t count, double* out);

/* p_j = |a_j|^2 in FP64 for all j (Sec. 2: the squared amplitude of |j>).
 * out has len >= D doubles, on the device (location QD_DEVICE, written
 * asynchronously on the state's stream) or on the host (QD_HOST, synchronous).
 * QD_ERR_BUFFER_TOO_SMALL if len < D. */
int qd_probabilities(const qd_state* s, double* out, uint64_t len, int32_t location);

/* Wait for the state's queued work; reports asynchronous device errors. */
int qd_synchronize(const qd_state* s);

/* ---- measurement -------------------------------------------------------------- */

/* Read and rewrite every amplitude of the state once, in place, `reps` times
 * (after one warm-up pass), with the access pattern of the gate sweeps; values
 * are unchanged (multiplied by a run-time 1.0). *best_ms receives the fastest
 * pass in milliseconds, so 2 * D * bytes-per-amplitude / best_ms is the
 * read+write copy ceiling the sweeps are measured against. Synchronous. */
int qd_copy_ceiling(qd_state* s, int32_t reps, double* best_ms);

/* ---- misc -------------------------------------------------------------------- */

const char* qd_last_error(void);
const char* qd_version(void);

#ifdef __cplusplus
}
#endif

#endif /* QD_H */
