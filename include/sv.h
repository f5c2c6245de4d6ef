/*
 * sv.h - C ABI of the MI355X (gfx950) state-vector simulator.
 *
 * The simulator applies quantum gates to a state of 2^n complex amplitudes
 * without ever forming a 2^n x 2^n matrix (Section III-A of "Accelerating
 * State-Vector Quantum Simulation on Integrated GPUs via Cache Locality
 * Optimization", arXiv 2605.15098). A single-qubit gate U on target t updates
 * every amplitude pair (j, j + 2^t) with bit t of j clear (Algorithm 1); a
 * controlled gate does so only where bit c of j is 1. The partitioned mode
 * implements the paper's state division (Section III-B): a block holds 2^l
 * amplitudes whose l local qubits vary; gates on local qubits are deferred and
 * applied block by block while the block stays on chip; a gate whose target is
 * global first brings that qubit into the block in place of a local one chosen
 * by LRU (or by a look-ahead policy), and a global control is decided per
 * block. By default gates are not taken in list order but in any order their
 * dependences allow (SV_SWAP_GRAPH), which gathers more gates per block.
 *
 * Conventions
 *   - Qubit q is bit q of the amplitude index (little-endian).
 *   - U is row-major, row = output, column = input, basis (|0>, |1>).
 *   - Amplitudes are interleaved (re, im): SV_COMPLEX64 = 2 x float,
 *     SV_COMPLEX128 = 2 x double. Gate matrices are formed in binary64 on the
 *     host and rounded once to the state's precision.
 *   - Every readout returns logical order, whatever the physical layout.
 *
 * Errors: every call returns an sv_status; on failure sv_last_error() gives a
 * thread-local message. Calls never throw across the ABI. A handle is not
 * thread-safe; distinct handles are independent.
 *
 * Memory: a handle either owns its device buffer (sv_create) or borrows one
 * (sv_wrap; the caller keeps it alive and owns the stream). Gate arrays are
 * borrowed for the duration of a call. Output pointers may be host or device
 * memory (detected with hipPointerGetAttributes): host outputs synchronize the
 * handle's stream, device outputs are stream-ordered.
 *
 * Environment (read when a circuit is planned or a pass is compiled; none is
 * needed in normal use):
 *   SV_JIT=0            run block passes through the op interpreter instead
 *                       of kernels compiled for each pass (same bits)
 *   SV_JIT_CACHE_DIR    directory of compiled pass modules kept across runs
 *   SV_PIN_BITS, SV_LOGR  override the schedule's pinned low qubits and
 *                       register qubits per thread (tuning experiments)
 *   SV_HALF_LDS         0: re-lay blocks out through LDS whole; 1 (default):
 *                       in two halves for blocks above 64 KiB; 2: in halves
 *                       whenever possible (tests)
 *   SV_TRACE_HOST       print host-side upload and launch timings to stderr
 *   SV_K2_MAX_GRID      at most this many work-groups per block-pass launch
 *                       (each walks more blocks; same bits; tests)
 *   SV_BATCH_MAX_GRID   at most this many work-groups in a batched launch
 *                       (default: the resident capacity; same bits)
 */
#ifndef SVMI_SV_H_INCLUDED
#define SVMI_SV_H_INCLUDED

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sv_handle_s *sv_handle;
typedef int32_t sv_status;

enum {
    SV_OK = 0,
    SV_ERR_INVALID_ARG = -1,   /* bad n, qubit, op, angle, schedule or pointer */
    SV_ERR_OUT_OF_MEMORY = -2, /* device or host allocation failed            */
    SV_ERR_DEVICE = -3,        /* a HIP call failed; message has the HIP error */
    SV_ERR_UNSUPPORTED = -4,   /* valid request the library does not support   */
    SV_ERR_BAD_HANDLE = -5     /* null or destroyed handle                     */
};

typedef enum { SV_COMPLEX64 = 0, SV_COMPLEX128 = 1 } sv_dtype;

/* Gate kinds. Controlled forms use sv_gate.control >= 0:
 * CNOT = {SV_X, c}, CZ = {SV_Z, c}, CP(theta) = {SV_P, theta, c}; QPE's
 * controlled U^(2^j) (Eq. 3) is {SV_P, theta_j, control = j}. */
enum {
    SV_H = 0,  /* [[1,1],[1,-1]]/sqrt2                          */
    SV_X = 1,
    SV_Y = 2,
    SV_Z = 3,
    SV_RX = 4, /* exp(-i theta X/2)                              */
    SV_RY = 5, /* exp(-i theta Y/2)                              */
    SV_RZ = 6, /* exp(-i theta Z/2) = diag(e^{-i theta/2}, e^{i theta/2}) */
    SV_P = 7,  /* diag(1, e^{i theta}) (Eq. 2)                   */
    SV_U2 = 8, /* arbitrary 2x2 given in u[8]                    */
    SV_SWAP = 9 /* exchange qubits target and target2; a relabel */
};

/* One gate (88 bytes). control = -1 for none; target2 only for SV_SWAP;
 * theta in radians for RX/RY/RZ/P; u = row-major 2x2 (re, im) for SV_U2.
 * One control at most (Section III-A); SWAP takes no control. */
typedef struct {
    int32_t op, target, control, target2;
    double theta;
    double u[8];
} sv_gate;

/* Schedule modes and options. */
enum { SV_PLAIN = 0, SV_PARTITIONED = 1 };
enum {
    SV_SWAP_LRU = 0,       /* Section III-B: gates in circuit order, the victim
                              is the least recently used local qubit         */
    SV_SWAP_LOOKAHEAD = 1, /* gates in circuit order; at a forced flush the
                              next block gathers the qubits that the upcoming
                              gates target first                             */
    SV_SWAP_GRAPH = 2      /* gates in any order their dependences allow (two
                              gates are ordered only when they share a qubit
                              on which one of them is not diagonal; circuit
                              SWAPs become renames); each block gathers the
                              qubits that let the longest chains of gates
                              proceed. Virtual remap only                    */
};
enum {
    SV_REMAP_VIRTUAL = 0, /* a SWAP moves no data: the next block pass gathers
                             the new local qubits by address (zero bytes)     */
    SV_REMAP_EXPLICIT = 1 /* a SWAP is a standalone in-place exchange pass    */
};
enum { SV_TUNER_NONE = 0, SV_TUNER_EXHAUSTIVE = 1, SV_TUNER_LEARNED = 2 };

typedef struct {
    int32_t mode;         /* SV_PLAIN: one sweep per gate (Algorithm 1);
                             SV_PARTITIONED: Section III-B                     */
    int32_t block_qubits; /* l, local qubits per on-chip block; 0 = default
                             (14 for complex64, 13 for complex128)           */
    int32_t outer_qubits; /* l2 (0 = off): outer tier. Consecutive block
                             passes whose local qubits together number at
                             most l2 run outer block by outer block (2^l2
                             amplitudes: the chain's local qubits plus the
                             lowest other qubits; one launch per pass and
                             outer block), so the later passes of a chain
                             read the block from the Infinity Cache
                             (Section III-B's cache-resident block, one tier
                             up; 2^24 complex64 = 128 MiB of the 256 MB).
                             Results are bit-identical to l2 = 0.
                             Partitioned mode only; 0..40.                   */
    int32_t fuse_k;       /* 0: one device op per gate (bit-exact with the
                             plain path); 1: each run of diagonal gates in a
                             block pass becomes one phase multiply per
                             amplitude and Hadamard normalization is applied
                             once per pass; 2..6: also fuse runs of gates on
                             <= k qubits into one 2^k x 2^k unitary            */
    int32_t swap_policy;  /* SV_SWAP_LRU (the paper), _LOOKAHEAD or _GRAPH     */
    int32_t remap;        /* SV_REMAP_VIRTUAL or SV_REMAP_EXPLICIT            */
    int32_t diag_free;    /* 0: every gate's target must be local (the paper's
                             rule); 1: diagonal gates (Z, P, RZ and their
                             controlled forms) never force a SWAP              */
    int32_t tuner;        /* SV_TUNER_*: sv_apply_circuit first picks the
                             schedule itself (sv_tune); NONE = use this one   */
    int32_t reg_qubits;   /* amplitudes per thread in a block pass = 2^this;
                             0 = default (5 for complex64, 4 for complex128) */
    int32_t pin_qubits;   /* low physical qubits local in every block with
                             virtual remap: contiguous runs of 2^this
                             amplitudes per access; 0 = default (5 for
                             complex64 = 256-byte runs, 3 for complex128 =
                             128-byte runs); more pins leave fewer free local
                             qubits per pass                                  */
} sv_schedule;

typedef struct {
    int64_t gates;       /* non-SWAP gates applied by the last call            */
    int64_t swaps;       /* SWAPs of a global target into the block            */
    int64_t phases;      /* deferred-queue flushes (block-resident passes)      */
    int64_t passes;      /* kernels that sweep the whole state                  */
    int64_t fused;       /* fused k-qubit windows                              */
    double bytes;        /* algorithmic HBM bytes of those passes              */
    double device_ms;    /* device time of the last call (HIP events)          */
    double plan_ms;      /* host planning time of the last call                */
    int32_t block_qubits;/* l used by the last call                            */
    int32_t fuse_k;      /* k used                                             */
    int32_t swap_policy; /* policy used                                        */
    int32_t mode;        /* mode used                                          */
    double norm_drift;   /* |norm^2 - 1| at the last sv_norm call             */
    /* Per-kernel device time of the last call, filled only while kernel
     * timing is on (sv_set_kernel_timing): index 0 = plain sweeps, 1 = block
     * passes, 2 = explicit SWAP passes. */
    double kernel_ms[3];
    int64_t kernel_launches[3];
} sv_stats;

/* Library version string. */
const char *sv_version(void);

/* Thread-local message of the last failed call on this thread ("" if none). */
const char *sv_last_error(void);

/* Allocate a state of 2^n amplitudes on the current HIP device, set it to
 * |0...0> (Section III-A: the state is an array of 2^n complex numbers).
 * n in [1, 36]. Errors: INVALID_ARG (n, dtype, out), OUT_OF_MEMORY, DEVICE. */
sv_status sv_create(int n, sv_dtype dtype, sv_handle *out);

/* Borrow a device buffer (e.g. a torch tensor's storage) of at least
 * 2^n * sizeof(amplitude) bytes and a HIP stream (NULL = default stream).
 * The buffer's content is taken as the state in logical order; it is not
 * cleared. The caller keeps buffer and stream alive until sv_destroy.
 * While wrapped (and after sv_destroy) the buffer holds the amplitudes in
 * the library's storage order: the qubit layout (sv_layout) and, from 2^15
 * amplitudes (complex64) or 2^14 (complex128) on, a fixed GF(2)-linear
 * permutation of the index that spreads block-pass accesses over the HBM
 * channels; sv_wrap reorders the buffer in place once (one pass) and
 * readouts always return logical order. */
sv_status sv_wrap(int n, sv_dtype dtype, void *dev_buf, size_t bytes, void *hip_stream,
                  sv_handle *out);

/* Release the handle (and the buffer if it owns it). NULL is accepted. */
sv_status sv_destroy(sv_handle h);

/* Set the state back to |0...0> and the layout to identity. */
sv_status sv_reset(sv_handle h);

/* Change the stream later calls are ordered on (NULL = default stream). */
sv_status sv_set_stream(sv_handle h, void *hip_stream);

/* Apply m gates in order to the current state (calls accumulate). The
 * schedule may be NULL (= partitioned, SV_SWAP_GRAPH, virtual remap,
 * diagonal gates free, the other fields at their defaults). The physical
 * layout may
 * stay permuted between calls; readouts undo it. Stream-ordered: returns
 * once the work is queued. Errors: INVALID_ARG (target >= n, control ==
 * target, non-finite theta, unknown op, SWAP with a control), UNSUPPORTED
 * (fuse_k > 6), DEVICE. No gate is applied when validation fails. */
sv_status sv_apply_circuit(sv_handle h, const sv_gate *gates, size_t m, const sv_schedule *s);

/* ---- general front end (wider than the paper's gate set: Section III-A
 * defines one control per gate) ----
 * An extended gate: any gate kind of sv_gate on one target with any number
 * of controls, a controlled SWAP, or SV_UK, a dense 2^k x 2^k unitary on k
 * targets (k = 1..6), with up to 16 controls (the gate acts where every
 * control qubit is 1). For SV_UK, uk points to 2 * 4^k doubles: row-major
 * (re, im), row = output, and bit b of a row or column index is the value of
 * qubit targets[b]; it is borrowed for the call. */
#define SV_UK 10
#define SV_MAX_TARGETS 6
#define SV_MAX_CONTROLS 16
typedef struct {
    int32_t op;         /* SV_H .. SV_SWAP or SV_UK                            */
    int32_t ntargets;   /* 1; 2 for SV_SWAP; k for SV_UK                       */
    int32_t ncontrols;  /* 0 .. SV_MAX_CONTROLS                                */
    int32_t pad;
    int32_t targets[SV_MAX_TARGETS];
    int32_t controls[SV_MAX_CONTROLS];
    double theta;       /* radians, for RX/RY/RZ/P                             */
    double u[8];        /* SV_U2: row-major 2x2 (re, im)                       */
    const double *uk;   /* SV_UK: the 2^k x 2^k matrix                         */
} sv_gate_ex;

/* Apply m extended gates in order (calls accumulate, like sv_apply_circuit).
 * Runs of gates that sv_gate can express (one target, at most one control,
 * uncontrolled SWAP) go through the schedule s as sv_apply_circuit would
 * apply them; every other gate is one sweep over the state (a group of 2^k
 * amplitudes per thread) on the current layout. All gates are validated
 * before any is applied. Errors: INVALID_ARG (qubits out of range or
 * repeated, counts out of range, non-finite numbers, null uk), UNSUPPORTED
 * (k > 6, more than 16 controls, a tuner in s), DEVICE. */
sv_status sv_apply_circuit_ex(sv_handle h, const sv_gate_ex *gates, size_t m, const sv_schedule *s);

/* Read an OpenQASM 2.0 program (host only; no handle, no device). Writes the
 * first min(cap, *count) records to gates (gates may be null when cap is 0)
 * and sets *count to the program's number of records and *nqubits to the
 * total size of its quantum registers (numbered in declaration order). The
 * standard library (include "qelib1.inc") is built in; user gates are
 * expanded; measure and barrier are dropped; reset, if and opaque gates give
 * UNSUPPORTED, as do the relative-phase gates rccx and rc3x. Gate matrices:
 * U(theta, phi, lambda) = [[c, -e^{i lambda} s], [e^{i phi} s, e^{i(phi +
 * lambda)} c]] with c = cos(theta/2), s = sin(theta/2); rx/ry/rz =
 * exp(-i theta sigma/2); p = u1 = diag(1, e^{i lambda}); rzz/rxx =
 * exp(-i theta P(x)P/2). Records never carry SV_UK. Errors: INVALID_ARG
 * (syntax, unknown names, sizes; the message names the line), UNSUPPORTED,
 * OUT_OF_MEMORY. */
sv_status sv_qasm_parse(const char *text, sv_gate_ex *gates, size_t cap, size_t *count, int *nqubits);

/* Compile ahead of time the block-pass kernels that `repeats` consecutive
 * sv_apply_circuit calls of this circuit and schedule will use from the
 * current layout (a circuit whose SWAP gates relabel qubits changes the
 * layout the next call starts from). Block passes are compiled for their op
 * lists at run time and cached; without this call the first use of a pass
 * compiles it. No state is changed and nothing runs on the device. */
sv_status sv_prepare(sv_handle h, const sv_gate *gates, size_t m, const sv_schedule *s, int repeats);

/* Many independent circuits, one per handle (all of one dtype, distinct
 * handles, one device), in one persistent kernel launch captured in a HIP
 * graph. The launch has one work-group size, 2^t threads with t = min(L - r,
 * n_min - 3) for the schedule's block size L and register tile r (defaults:
 * the dtype's block size and a tile one below the dtype's, 4 for complex64
 * and 3 for complex128, which keeps two work-groups per CU); instance i is planned with the partitioned schedule at its
 * own block size l_i = min(n_i, t + r) and tile l_i - t (at least 3), so
 * large states use the full block and small ones shrink only their tile. An
 * instance carrying at least two work-groups' share of the work gets that
 * many work-groups (at most one per block), which meet at a device-scope
 * counter barrier between passes; smaller instances are packed, largest
 * first, onto the least loaded remaining work-groups and run there one after
 * another. The graph is cached by a hash of the gate lists, layouts, buffers
 * and schedule, so the same batch applied again replays it. Runs on the
 * first handle's stream and synchronizes it (the barrier's error flag is
 * checked: SV_ERR_DEVICE if a barrier wait timed out). Schedules that are not
 * partitioned with virtual remap, or a register tile outside 3..5 (3..4 for
 * complex128), are applied one circuit after another. Each handle's stats
 * receive its own counts, its block size and the batch's device time. */
sv_status sv_apply_batch(sv_handle *hs, int count, const sv_gate *const *gates, const size_t *m,
                         const sv_schedule *s);

/* Exhaustive batch tuner: times sv_apply_batch on scratch copies of the
 * states for the six largest block sizes (the largest is the dtype's
 * maximum, capped by the largest instance; at least 7), register tiles of
 * the dtype's default and one below, and fusion widths fuse_k 1, 4 and 5
 * (matrix-core windows where the cost gate admits them), and returns the
 * fastest schedule (median of three runs after a warm-up).
 * The states are not changed. */
sv_status sv_tune_batch(sv_handle *hs, int count, const sv_gate *const *gates, const size_t *m, sv_schedule *out);

/* Probabilities |alpha|^2 in FP64 (measurement, the meters of the QPE
 * figure). nq = 0: all 2^n in logical order. Otherwise the marginal over the
 * listed qubits: out[m] sums |alpha_i|^2 over every i whose bits
 * qubits[0..nq-1] spell m (qubits[k] = bit k of m); 2^nq doubles. */
sv_status sv_probabilities(sv_handle h, const int *qubits, int nq, double *out);

/* All 2^n amplitudes in logical order (interleaved, the handle's dtype). */
sv_status sv_state(sv_handle h, void *out);

/* Amplitudes [offset, offset+count) of the logical order, and their import
 * (checkpoint / resume between circuits). */
sv_status sv_state_range(sv_handle h, uint64_t offset, uint64_t count, void *out);
sv_status sv_set_state_range(sv_handle h, uint64_t offset, uint64_t count, const void *in);

/* QPE readout (Section IV-A): marginal over counting qubits 0..t-1 in FP64,
 * its argmax m (lowest index wins ties), phi = m / 2^t and P(m). */
sv_status sv_qpe_readout(sv_handle h, int t, uint64_t *m, double *phi, double *pmax);

/* ---- measurement (the meters of the QPE figure, Section IV-A) ----
 * The outcome of measuring qubits[0..nq-1] (nq = 0: all n qubits in order)
 * is the integer m whose bit k is the value of qubit qubits[k], drawn with
 * its Born probability P(m) (FP64). Random numbers are the caller's: each
 * uniform u in [0, 1) maps to the smallest m with C(m) > u * C(2^nq - 1),
 * C(m) = P(0) + ... + P(m) (inverse CDF over ascending m, summed in FP64 in
 * a fixed order; dividing by the total keeps a drifted norm harmless). At
 * most 32 measured qubits; 2^nq doubles of device scratch. */

/* `shots` outcomes for the uniforms (host or device arrays, shots each);
 * the state is unchanged. */
sv_status sv_sample(sv_handle h, const int *qubits, int nq, const double *uniforms, size_t shots, uint64_t *out);

/* One projective measurement with the uniform u: draws m as above, then
 * zeroes every amplitude whose measured qubits differ from m and scales the
 * rest by 1/sqrt(P(m)) (collapse and renormalisation, one pass). Returns m
 * and P(m) on the host. */
sv_status sv_measure(sv_handle h, const int *qubits, int nq, double u, uint64_t *outcome, double *prob);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the QPE
 * readout of sv_qpe_readout, same kernels and results, with no allocation of
 * any kind. Its scratch (per-work-group partial maxima and the result) lives
 * in a file-scope device array of 128 KiB + 256 bytes that each GPU holds
 * until the process ends; every call on a GPU shares it and it keeps the last
 * call's contents (nothing in it needs clearing: each call writes what it
 * reads), so calls that overlap on one GPU (several streams or threads) race.
 * Limit: n - t <= 4 (QPE has n - t = 1); a larger complement would need a
 * marginal buffer beyond the array and returns SV_ERR_UNSUPPORTED. Host
 * outputs; synchronizes the handle's stream. */
sv_status sv_qpe_readout_noalloc(sv_handle h, int t, uint64_t *m, double *phi, double *pmax);

/* Sum of |alpha|^2 in FP64. Also records |norm - 1| in the stats. */
sv_status sv_norm(sv_handle h, double *norm2);

/* Counters and timing of the last sv_apply_circuit (synchronizes). */
sv_status sv_stats_get(sv_handle h, sv_stats *out);

/* Host-only planning, usable without a GPU: the counts (gates, swaps,
 * phases, passes, bytes) the given schedule would produce for this circuit on
 * an n-qubit state of the given dtype starting from the identity layout. */
sv_status sv_plan(int n, sv_dtype dtype, const sv_gate *gates, size_t m, const sv_schedule *s,
                  sv_stats *out);

/* ---- schedule tuning (the paper sweeps the block size by hand over a
 * range and keeps the median of three runs, Section IV-B) ----
 *
 * Candidates: partitioned schedules over the dependence graph
 * (SV_SWAP_GRAPH, virtual remap) with diagonal gates free, over
 *   block qubits  the three largest sizes that fit on chip (complex64 12..14,
 *                 complex128 11..13; capped at n),
 *   register tile 2^4 or 2^5 amplitudes per thread (complex64),
 *                 2^3 or 2^4 (complex128),
 *   pinned low    4 or 5 qubits (complex64), 3 or 4 (complex128),
 *   fusion        fuse_k 1 (diagonal runs combined) or 5 (also dense windows
 *                 of up to 5 qubits through the matrix cores)
 * (a block smaller than the register tile is one tile). The paper's LRU
 * placement and list-order look-ahead are left out: on the measured circuits
 * they need more block passes than the dependence-graph schedule (LRU never
 * came within a factor of two of look-ahead). sv_tune_candidates writes up to cap of them to
 * out (out may be NULL) and their number to *count (24 when n is at least
 * the largest size). */
sv_status sv_tune_candidates(int n, sv_dtype dtype, sv_schedule *out, int cap, int *count);

/* Pick a schedule for this circuit on this handle among the candidates.
 * mode = SV_TUNER_EXHAUSTIVE times every candidate on a scratch copy of the
 * state (median of three timed runs after one warm-up, device time) and
 * returns the fastest; SV_TUNER_LEARNED ranks them with the cost model set by
 * sv_set_cost_model, one forward pass of the network on the device over all
 * candidates, and returns the smallest prediction (exhaustive when no model
 * is set). The state and its layout are not changed. OUT_OF_MEMORY if the
 * scratch copy does not fit (exhaustive only). out->tuner is SV_TUNER_NONE. */
sv_status sv_tune(sv_handle h, const sv_gate *gates, size_t m, int mode, sv_schedule *out);

/* Device time in ms of each of ncand schedules for this circuit on this
 * handle, measured as sv_tune(EXHAUSTIVE) measures it (repeats timed runs
 * after one warm-up, median) on a scratch copy; ms_out[i] for cands[i]. Also
 * returns, in compile_ms (may be NULL), the host time spent compiling each
 * candidate's pass kernels (0 when they were cached). */
sv_status sv_tune_time(sv_handle h, const sv_gate *gates, size_t m, const sv_schedule *cands, int ncand,
                       int repeats, double *ms_out, double *compile_ms);

/* Compile the pass kernels of this circuit under schedule s for an n-qubit
 * state in the identity layout, without touching a device: the result lands
 * in the run-time compiler's on-disk cache, where later calls on a device
 * find it. For worker processes that compile ahead of a timed run. */
sv_status sv_jit_precompile(int n, sv_dtype dtype, const sv_gate *gates, size_t m, const sv_schedule *s);

/* Features of (circuit, schedule) for the cost model, from host-side
 * planning of an n-qubit state in the identity layout (no device work).
 * out receives SV_FEATURES floats:
 *   0 n                        8 explicit swap passes
 *   1 bytes per amplitude      9 plain sweeps
 *   2 block qubits l          10 log2 of the algorithmic bytes of all passes
 *   3 register qubits         11 device ops over all block passes
 *   4 pinned low qubits       12 most ops in one block pass
 *   5 fuse_k                  13 dense ops (H, X, 2x2)
 *   6 non-SWAP gates          14 diagonal ops (phase, diag, diagonal run)
 *   7 block passes            15 layout ops (register/LDS re-layouts) */
#define SV_FEATURES 16
sv_status sv_features(int n, sv_dtype dtype, const sv_gate *gates, size_t m, const sv_schedule *s, float *out);

/* ---- the cost model network (k7): in -> 64 -> 64 -> 1, ReLU, FP32 ----
 * Parameters are one flat float array: W1[64][in], b1[64], W2[64][64],
 * b2[64], w3[64], b3 (sv_mlp_param_count(in) floats). Inputs are standardised
 * in the kernels with norm = {mean[in], inv_std[in]} (NULL: identity).
 * All pointers below are DEVICE pointers; work is enqueued on stream (a
 * hipStream_t, NULL = the null stream) and is stream-ordered. in must be in
 * [1, 32], batch >= 1; otherwise INVALID_ARG. */
#define SV_MLP_HIDDEN 64
size_t sv_mlp_param_count(int in);
/* y[s] = prediction for row s of x (batch x in, row-major). */
sv_status sv_mlp_forward(const float *params, int in, const float *norm, const float *x, int batch, float *y,
                         void *stream);
/* Bytes of device workspace sv_mlp_grad needs for this batch. */
size_t sv_mlp_workspace_bytes(int in, int batch);
/* grad = gradient of L = mean_s (y_s - target_s)^2 with respect to params;
 * *loss = L (device float; loss may be NULL). Deterministic. */
sv_status sv_mlp_grad(const float *params, int in, const float *norm, const float *x, const float *target,
                      int batch, float *grad, float *loss, void *workspace, void *stream);
/* One Adam step (bias-corrected; step counts from 1) on count parameters
 * with first and second moments m, v (updated in place). */
sv_status sv_mlp_adam(float *params, float *m, float *v, const float *grad, size_t count, float lr,
                      float beta1, float beta2, float eps, int step, void *stream);

/* Install the cost model used by sv_tune(SV_TUNER_LEARNED): HOST arrays of
 * sv_mlp_param_count(in) parameters and 2*in normalisation floats (NULL:
 * identity); in must be SV_FEATURES. The library keeps copies; params NULL
 * removes the model. Process-wide. */
sv_status sv_set_cost_model(const float *params, int in, const float *norm);

/* Record a HIP event pair around every kernel of later sv_apply_circuit
 * calls on this handle (on = 1) so sv_stats_get reports per-kernel device
 * time; on = 0 (the default) records one pair per call. */
sv_status sv_set_kernel_timing(sv_handle h, int on);

/* Permutation of the current layout: l2p[q] = physical bit of qubit q. */
sv_status sv_layout(sv_handle h, int *l2p);

/* Bandwidth reference for the block passes (not part of the simulation): a
 * plain streaming kernel over DEVICE buffers of `bytes` (a multiple of 16,
 * 16-byte aligned). mode 0 copies src to dst (bytes read + bytes written);
 * mode 1 rewrites dst in place (src unused), the access pattern of a block
 * pass. Stream-ordered on `stream` (NULL = null stream). */
sv_status sv_stream_probe(void *dst, const void *src, size_t bytes, int mode, void *stream);

/* Testing hook: make the next device allocation (kind 1) or kernel launch
 * (kind 2) of this process fail; 0 clears. */
sv_status sv_debug_inject_fault(int kind);

#ifdef __cplusplus
}
#endif

#endif /* SVMI_SV_H_INCLUDED */
