/*
 * owqs.h -- C ABI of libowqs: state-vector execution of one-way quantum
 * computer (1WQC) measurement patterns on an AMD Instinct MI355X (gfx950).
 *
 * The library takes a pattern (Sec. 2.2 of "One-Way Quantum Computer
 * Simulation": qubits, inputs, outputs and a command list of N, E, M, X, Z)
 * together with the state of the input qubits, applies the commands in the
 * given order with qubit elimination after every measurement (Sec. 4.2) and
 * implicit actions (Sec. 4.4), and reports the state of the output qubits
 * (Sec. 4, overview of the simulator).  Measurement outcomes are forced by the
 * caller, so runs are reproducible.
 *
 * Conventions used by every entry point:
 *   - Commands are given in EXECUTION order (first command first); the paper
 *     writes patterns right to left.
 *   - Amplitudes are complex64, interleaved (float re, float im).  Bit k of an
 *     input index is the k-th listed input qubit; bit k of an output index is
 *     the k-th listed output qubit (the paper's qubit v <-> 2^(v-1) of
 *     Figs. 5-6; its kets print the most significant qubit first, Eq. 8).
 *   - M with angle alpha and signal domains s, t measures at
 *     theta = (-1)^s alpha + t pi (Eq. 2).  Outcome o keeps the branch of the
 *     elimination operator of Eq. 11 (o = 0) or Eq. 12 (o = 1):
 *     new = (psi_0 + (-1)^o e^{-i theta} psi_1) / sqrt(2), whose squared norm
 *     is the outcome probability (Eq. 13).
 *   - X_v^s and Z_v^s apply when the XOR of the outcomes in s is 1.
 *   - Ownership: every *_create has a matching *_destroy.  Host arrays passed
 *     in are copied before the call returns; the library never frees caller
 *     memory.  Device pointers (flag *_on_device = 1) are borrowed until the
 *     work enqueued on the given stream has finished.
 *   - Streams: `stream` is a hipStream_t (NULL = the null stream).  Calls that
 *     take a stream enqueue work and return without waiting, except where a
 *     host buffer is read or written, which waits for the stream.
 *   - Errors: every call returns an owqs_status; negative values are errors.
 *     owqs_last_error() gives a human-readable detail (command index, HIP
 *     error string).  After OWQS_E_ZERO_PROB the state is undefined.
 *   - Thread safety: a context and its patterns must be used from one host
 *     thread at a time.
 */
#ifndef OWQS_H
#define OWQS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  OWQS_OK = 0,
  OWQS_E_INVALID_ARG = -1,       /* null pointer, size mismatch, bad enum */
  OWQS_E_PATTERN = -2,           /* pattern breaks rule D0, D1, D2 or D3 (Sec. 2.2) */
  OWQS_E_ZERO_PROB = -3,         /* a forced outcome has probability < 1e-10 */
  OWQS_E_WIDTH = -4,             /* live width above OWQS_MAX_WIDTH (plan or run) */
  OWQS_E_NOMEM = -5,             /* device or host allocation failed */
  OWQS_E_HIP = -6,               /* a HIP runtime call failed */
  OWQS_E_NOT_DETERMINISTIC = -7, /* EOWQS check mode saw |p - 1/2| > 1e-4 */
  OWQS_E_STATE = -8              /* call out of order, e.g. read before run */
} owqs_status;

/* Largest live width (number of qubits held in the state vector at once). */
#define OWQS_MAX_WIDTH 34

/* Command opcodes (Sec. 2.2). */
enum {
  OWQS_OP_N = 0, /* N_v: prepare v in |+> = (|0> + |1>)/sqrt 2 */
  OWQS_OP_E = 1, /* E_uv: controlled-Z between u (q0) and v (q1) */
  OWQS_OP_M = 2, /* M_v^alpha with s- and t-domains (Eqs. 1-2) */
  OWQS_OP_X = 3, /* X_v^s: Pauli X when the s signal is 1 */
  OWQS_OP_Z = 4  /* Z_v^s: Pauli Z when the s signal is 1 */
};

/* One command.  Qubit ids are non-negative integers.  Domains are ranges in
 * the `domain_ids` array given to owqs_pattern_create; the t-domain is read
 * for M only.  40 bytes, no implicit padding. */
typedef struct {
  int32_t op;     /* OWQS_OP_* */
  int32_t q0;     /* qubit acted on (E: first qubit) */
  int32_t q1;     /* E: second qubit; ignored otherwise */
  int32_t s_off;  /* s-domain = domain_ids[s_off .. s_off + s_len) */
  int32_t s_len;
  int32_t t_off;  /* t-domain = domain_ids[t_off .. t_off + t_len) (M only) */
  int32_t t_len;
  int32_t reserved; /* must be 0 */
  double angle;   /* M: alpha in radians; ignored otherwise */
} owqs_cmd;

/* OWQS (Sec. 4): each M computes its outcome probability in FP64 and the
 * state is renormalised by it.  EOWQS (Sec. 4.5): for patterns with a
 * (generalised) flow every outcome has probability 1/2, so no probability is
 * computed and the scale is fixed.  EOWQS_CHECK: as EOWQS, but every M still
 * computes p and the run fails with OWQS_E_NOT_DETERMINISTIC if
 * |p - 1/2| > 1e-4. */
typedef enum { OWQS_MODE_OWQS = 0, OWQS_MODE_EOWQS = 1, OWQS_MODE_EOWQS_CHECK = 2 } owqs_mode;

/* Execution plan.  PLAIN: one kernel per non-trivial command, the live width
 * growing on N and shrinking on M.  FUSED: windows of commands are merged
 * into single passes over the state (N w; E u w; ...; M u; corrections on w
 * becomes one 2x2 update in place), and at live widths >= 15 runs of
 * windows/E/X/Z whose paired slots fit an LDS tile run as one
 * pass per run (2^12-amplitude tiles by default).  AUTO (default): the fused plan, run as one workgroup with
 * the whole vector in LDS when its width is <= 14, else as FUSED.  All give
 * the same result to FP32 rounding.
 * SUBSTATES: the state is a list of sub-states (Sec. 4.1), each group of
 * qubits entangled so far in its own vector: N makes a one-qubit |+>
 * sub-state, E across two sub-states first forms their tensor product
 * (Sec. 4.4.1: the wider one keeps its buffer and takes the other's qubits on
 * its top bits), M eliminates its qubit inside its sub-state (with the
 * sub-state's own FP64 scale in OWQS mode), one kernel per command.  Memory
 * is the sum of the sub-states' largest sizes, not 2^(live width), and the
 * width limit OWQS_MAX_WIDTH applies to each sub-state, so patterns whose
 * graph stays in separate components can be wider than the limit.  Runs
 * with owqs_run (the input as one sub-state) or owqs_run_factors; read with
 * owqs_read_state (the tensor product, if the outputs fit) or
 * owqs_read_substates.  Batches, basis runs, adjoints, ranged and sampled
 * runs and the tuner refuse it (OWQS_E_STATE); profiled runs time each
 * step (kinds N, E, M, X, Z, FINISH and KRON).  The input state is
 * taken to be normalised (each sub-state's p is relative to its own norm). */
typedef enum {
  OWQS_EXEC_PLAIN = 0,
  OWQS_EXEC_FUSED = 1,
  OWQS_EXEC_AUTO = 2,
  OWQS_EXEC_SUBSTATES = 3
} owqs_exec;

typedef struct owqs_ctx owqs_ctx;
typedef struct owqs_pattern owqs_pattern;

/* Name of a status code (static string). */
const char *owqs_status_str(owqs_status s);

/* Create a context bound to HIP device `device`.  *out receives the handle.
 * device = -1 makes a host-only context: patterns can be created, parsed and
 * validated, but owqs_run returns OWQS_E_STATE. */
owqs_status owqs_ctx_create(int device, owqs_ctx **out);
void owqs_ctx_destroy(owqs_ctx *ctx);
/* Detail of the last error raised through this context (static until the
 * next call on the context).  Never NULL. */
const char *owqs_last_error(const owqs_ctx *ctx);

/* Build a pattern from commands in execution order (Sec. 2.2, P = (V,I,O,A)).
 * inputs[k] is bit k of the input state, outputs[k] bit k of the read-out.
 * The pattern is validated against D0-D3 (no dependence on an unmeasured
 * outcome; no action on a measured qubit; no action on an unprepared
 * non-input; exactly the non-outputs are measured) and its largest live width
 * is computed; no device memory is allocated yet.  Every M starts with its
 * outcome forced to 0.  A pattern wider than OWQS_MAX_WIDTH loads (it can be
 * read back and reordered, owqs_pattern_reorder), but every call that plans
 * or runs it returns OWQS_E_WIDTH (the sub-state executor checks its widest
 * sub-state instead; owqs_read_state checks the number of outputs). */
owqs_status owqs_pattern_create(owqs_ctx *ctx, const owqs_cmd *cmds, size_t ncmds,
                                const int32_t *domain_ids, size_t ndom,
                                const int32_t *inputs, int32_t nin,
                                const int32_t *outputs, int32_t nout,
                                owqs_pattern **out);

/* Same, from text format v1: lines "inputs q...", "outputs q...", then one
 * command per line in execution order: "N q", "E u v",
 * "M q alpha [s: ids] [t: ids]", "X q [s: ids]", "Z q [s: ids]"; '#' starts a
 * comment.  `len` is the number of bytes in `text`. */
owqs_status owqs_pattern_from_text(owqs_ctx *ctx, const char *text, size_t len,
                                   owqs_pattern **out);

/* Frees the pattern and its device buffers (waits for its streams' work). */
void owqs_pattern_destroy(owqs_pattern *pat);

/* Sizes of the pattern: number of M commands, largest live width (plain
 * execution), number of inputs and outputs, number of commands.  Any output
 * pointer may be NULL. */
owqs_status owqs_pattern_info(const owqs_pattern *pat, int32_t *n_meas, int32_t *max_live,
                              int32_t *n_in, int32_t *n_out, size_t *ncmds);

owqs_status owqs_set_mode(owqs_pattern *pat, owqs_mode mode);
owqs_status owqs_set_exec(owqs_pattern *pat, owqs_exec exec);

/* Replace the angles of the M commands (alpha[m] for the m-th M in execution
 * order, radians).  n_meas must equal the pattern's M count. */
owqs_status owqs_set_angles(owqs_pattern *pat, const double *alpha, size_t n_meas);

/* Force the outcomes of the M commands (bits[m] in {0,1} for the m-th M). */
owqs_status owqs_set_outcomes(owqs_pattern *pat, const uint8_t *bits, size_t n_meas);

/* Run the whole pattern on `stream`.  input_c64 holds 2^nin complex64
 * amplitudes (n_amps must equal 2^nin; when nin = 0 pass n_amps = 1 and
 * input NULL for the empty product state).  The input need not be
 * normalised: OWQS renormalises at every M, EOWQS keeps its norm.  The live
 * state stays in device memory owned by the pattern until the next run. */
owqs_status owqs_run(owqs_pattern *pat, const void *input_c64, size_t n_amps,
                     int input_on_device, void *stream);

/* Copy the output state (2^nout complex64, outputs[k] at bit k, scaled to the
 * true state) to out_c64.  With out_on_device = 0 the call waits for the
 * stream and also reports a pending OWQS_E_ZERO_PROB /
 * OWQS_E_NOT_DETERMINISTIC from the run. */
owqs_status owqs_read_state(owqs_pattern *pat, void *out_c64, size_t n_amps,
                            int out_on_device, void *stream);

/* Waits for `stream` and reports errors detected on the device by the last
 * run (zero probability, non-determinism in EOWQS_CHECK mode). */
owqs_status owqs_check(owqs_pattern *pat, void *stream);

/* Replay the compiled plan as a captured HIP graph (default on).  The graph
 * is captured on the first run after the plan changes and holds kernels only;
 * the input copy stays outside it. */
owqs_status owqs_set_graph(owqs_pattern *pat, int enable);

/* OWQS mode: sum the probability of every M (on = 1), including fused
 * windows whose new qubit meets the measured one through an odd number of E.
 * Such a window has p = 1/2 exactly for every state and angle (Eqs. 11-13),
 * so by default (on = 0) it records 1/2 without summing the state, at most
 * 128 in a row before one sums and renormalises.  Both give the same
 * results within rounding; on = 1 does the paper's OWQS work for every M. */
owqs_status owqs_set_sum_all(owqs_pattern *pat, int32_t on);

/* Tile size of the fused passes: 2^bits amplitudes per LDS tile, bits in
 * 10..13, or 0 for the default min(12, width - 8).  Larger tiles chain more
 * commands per pass; smaller ones fit more workgroups per CU. */
owqs_status owqs_set_tile_bits(owqs_pattern *pat, int32_t bits);

/* Autotuner: time the pattern (3 runs after a warm-up, HIP events on
 * `stream`) with every tile size 10..13 of the fused passes and keep the
 * fastest (owqs_set_tile_bits).  Plans without tile passes return at once
 * with *best_ms = 0.  The runs overwrite the pattern's state.  Either output
 * pointer may be NULL. */
owqs_status owqs_tune(owqs_pattern *pat, const void *input_c64, size_t n_amps, int input_on_device,
                      void *stream, int32_t *best_bits, float *best_ms);

/* Autotuner for a batch (owqs_run_batch with the same arguments): time the
 * whole batch (3 calls after a warm-up, HIP events on `stream`) with every
 * tile size 10..13 given to all of its patterns whose plans have tile passes
 * (plan width above 14, executor not PLAIN), and keep the fastest on each of
 * them (owqs_set_tile_bits).  In a batch the passes of many patterns share a
 * launch, so the best size is often larger than the one a pattern run alone
 * prefers.  Without such patterns it returns at once with *best_bits = 0 and
 * *best_ms = 0.  The runs write the outputs.  Either output pointer may be
 * NULL. */
owqs_status owqs_tune_batch(owqs_ctx *ctx, owqs_pattern *const *pats, size_t npat, const void *const *inputs,
                            void *const *outputs, void *stream, int32_t *best_bits, float *best_ms);

/* Compile the plan for the current settings (if needed) and report the
 * largest live width it reaches (plain plans: max_live; fused windows keep
 * the width of the window's input), its number of steps (one per
 * non-trivial command or fused window) and the number of passes over the
 * state in global memory (steps after grouping runs into tile passes).  For
 * the sub-state executor: the widest sub-state, its steps, and its launches
 * after each sub-state's runs of window/E/X/Z steps at width >= 15 are
 * grouped into tile passes.  Any pointer may be NULL. */
owqs_status owqs_plan_info(owqs_pattern *pat, int32_t *plan_width, size_t *nsteps, size_t *npasses);

/* The tile passes of the fused plan (global-memory executor) or of the
 * sub-state plan (0s for other plans) as they run with forced outcomes and
 * without window sums: windows
 * applied one by one (*windows), and runs of windows on one register-round
 * position (Sec. 4.4: each window is a fixed 2x2 map on its pair once its
 * outcome is known) composed into one 2x2 map each (*maps, covering
 * *composed windows).  Every window of a pass is in exactly one of the two,
 * so *windows + *composed is the passes' window count.  A map costs the
 * FP32 work of two windows.  Passes with window sums and runs with drawn
 * outcomes apply every window on its own.  Compiles the plan if needed; any
 * pointer may be NULL. */
owqs_status owqs_plan_tile_work(owqs_pattern *pat, size_t *windows, size_t *maps, size_t *composed);

/* Recognition problem (Sec. 1: which unitary does a pattern implement):
 * run the pattern on the computational-basis inputs |first>, ...,
 * |first + count - 1> and write output k (2^nout complex64) to
 * out_c64 + k * 2^nout, so that with first = 0 and count = 2^nin the device
 * buffer holds the unitary column by column.  Each input runs in the LDS of
 * one workgroup: the plan width must be <= 14 (else OWQS_E_WIDTH).
 * out_c64 (and probs, count * n_meas FP64 values or NULL) are device
 * pointers.  Asynchronous on `stream`; errors are reported by owqs_check
 * with the failing input's index.  Does not touch the state read by
 * owqs_read_state. */
owqs_status owqs_run_basis(owqs_pattern *pat, uint32_t first, uint32_t count, void *out_c64,
                           double *probs, void *stream);

/* As owqs_run_basis, for `count` arbitrary input states stored one after the
 * other at in_c64 (count * 2^nin complex64, device memory). */
owqs_status owqs_run_states(owqs_pattern *pat, const void *in_c64, uint32_t count, void *out_c64,
                            double *probs, void *stream);

/* Allocation-free run, for callers that cannot allocate device memory:
 * code under HIP graph capture, serving loops and harnesses that forbid
 * hipMalloc.  It runs the pattern's plan (the same kernels as owqs_run, in the
 * same order, launched on `stream` without a graph) and writes the read-out,
 * but its working memory is a fixed array inside the library instead of the
 * pattern's buffers:
 *   the live vector, at most 2^OWQS_NOALLOC_MAX_WIDTH complex64 (32 MiB),
 *   the FP64 scale, the FP64 block partials, and (when `probs` or `err` is
 *   NULL) the probabilities and the error word.
 * The array is static device memory of about 34 MiB on each GPU the library
 * runs on, held until the process ends; its address is resolved when a
 * context is created on that device.  Every call on one GPU shares it and
 * overwrites what the previous call left: calls that overlap on one GPU
 * (different streams, or different host threads) race and give undefined
 * results.  Nothing is allocated or freed: no hipMalloc, hipFree or graph.
 *   input_c64:  device, 2^nin complex64 (n_in_amps = 2^nin; NULL with
 *               n_in_amps = 1 when nin = 0 for the empty product state)
 *   output_c64: device, 2^nout complex64 (n_out_amps = 2^nout), outputs[k]
 *               at bit k, scaled to the true state as owqs_read_state does
 *   probs:      device, n_meas FP64 (per M, Eq. 13; written in OWQS and
 *               EOWQS_CHECK modes; EOWQS assumes 1/2 and writes none), or
 *               NULL to keep them in the array (then n_meas <= 65536)
 *   err:        device, 2 int32 {first M index that failed or 0x7fffffff,
 *               kind: 1 zero probability, 2 |p - 1/2| > 1e-4}, cleared by
 *               the call, or NULL (kept in the array, not reported)
 * Preconditions: forced outcomes (no uniforms), not the SUBSTATES executor,
 * and the plan compiled and its command table on the device: run the pattern
 * once with owqs_run after its last change (mode, exec, angles, outcomes,
 * tile size), outside the allocation-free region; else OWQS_E_STATE.
 * OWQS_E_WIDTH when the pattern's live width exceeds OWQS_NOALLOC_MAX_WIDTH
 * (checked first, also on a host-only context), or when probs is NULL and
 * the pattern has more than 65536 M commands.  The call does not change what
 * owqs_read_state, owqs_read_probs and owqs_check report (they refer to the
 * last owqs_run). */
#define OWQS_NOALLOC_MAX_WIDTH 22
owqs_status owqs_run_noalloc(owqs_pattern *pat, const void *input_c64, size_t n_in_amps,
                             void *output_c64, size_t n_out_amps, double *probs, int32_t *err,
                             void *stream);

/* Run `npat` independent patterns of one context as one batch (the paper runs
 * patterns one at a time, Sec. 5; batching is this library's addition).
 * inputs[i] (2^nin_i complex64; may be NULL for a pattern without inputs)
 * and outputs[i] (2^nout_i complex64) are device pointers.  The whole batch
 * is one graph launched on `stream`: patterns whose plan width is <= 14 run
 * whole in one workgroup's LDS (one launch per width class); wider plans run
 * level by level, the s-th tile pass of every pattern in one multi-pattern
 * launch.  The graph is kept by the context and replayed while the same
 * patterns (unchanged since their last compile), inputs and outputs are
 * passed again; any change rebuilds it, which waits for the previous batch
 * of this context to finish.  Each pattern keeps its own probabilities and
 * error state (owqs_read_probs, owqs_check); the outputs of patterns wider
 * than 14 can also be read again with owqs_read_state.  Every mode may be
 * mixed in one batch; sub-state patterns and drawn outcomes are refused
 * (OWQS_E_STATE). */
owqs_status owqs_run_batch(owqs_ctx *ctx, owqs_pattern *const *pats, size_t npat,
                           const void *const *inputs, void *const *outputs, void *stream);

/* Gradient of an output observable with respect to the M angles, for
 * `batch` angle sets at once (adjoint method).  The loss of set b is
 * L_b = sum_i <Z_{obs[i]}> on the output state (obs[i] indexes the outputs
 * list), evaluated with fixed probabilities 1/2 (EOWQS, Sec. 4.5): the
 * pattern must have a flow for this to be the OWQS loss too.  Every pattern
 * whose N-E-M-X windows (the translation of J gates) come after a prefix
 * without measurements is supported; the plan is switched to FUSED.
 *   input_c64: device, 2^nin complex64 shared by all sets (NULL if nin = 0)
 *   alpha:     host, batch * n_meas radians (row b = set b, M order)
 *   loss:      device, batch FP64
 *   grad:      device, batch * n_meas FP64, dL_b/dalpha_m (0 for M commands
 *              outside windows)
 *   ckpt_stride: windows per checkpoint segment (0 = 16); the forward pass
 *              stores the live vectors at segment starts.  When every window
 *              has an odd number of E between its two qubits (so its 2x2
 *              part is invertible; J gates are), the backward pass starts
 *              each segment from the next checkpoint and recovers every
 *              window's input from its output (Eqs. 11-12 with p = 1/2 make
 *              the window unitary up to its scale); otherwise it recomputes
 *              the segment forward from its checkpoint and keeps the window
 *              inputs.  A negative stride -s selects the recomputing sweep
 *              with segments of s windows for any pattern (the two sweeps
 *              agree to FP32 rounding).
 * Asynchronous on `stream`; device memory of about
 * (2 + segments) * batch * 2^width * 8 bytes (plus ckpt_stride such vectors
 * for the recomputing sweep) stays allocated with the pattern. */
owqs_status owqs_adjoint(owqs_pattern *pat, const void *input_c64, const double *alpha, size_t batch,
                         const int32_t *obs, int32_t nobs, double *loss, double *grad,
                         int32_t ckpt_stride, void *stream);

/* Kernel kinds reported by owqs_run_profiled. */
enum {
  OWQS_KIND_N = 0,      /* prepare: 16 * 2^n algorithmic bytes at live width n */
  OWQS_KIND_E = 1,      /* controlled-Z: 4 * 2^n (the quarter read and written) */
  OWQS_KIND_M = 2,      /* measure + eliminate: 12 * 2^n (read all, write half) */
  OWQS_KIND_X = 3,      /* 16 * 2^n */
  OWQS_KIND_Z = 4,      /* 8 * 2^n */
  OWQS_KIND_J = 5,      /* fused window N w; E u w; M u; X/Z w: 16 * 2^n */
  OWQS_KIND_FINISH = 6, /* one-block FP64 finish of an M/window probability (bytes not counted) */
  OWQS_KIND_TILE = 7,   /* a group of windows/E/X/Z steps in one pass: 16 * 2^n */
  OWQS_KIND_KRON = 8,   /* sub-state merge of 2^a and 2^b amplitudes: 8 (2^a + 2^b + 2^(a+b)) */
  OWQS_NUM_KINDS = 9
};

/* As owqs_run, and also times every kernel of the run with HIP events
 * recorded on `stream` between consecutive launches; waits for the stream.
 * For each kind k, adds the number of launches to counts[k], their summed
 * event time to ms[k] and their algorithmic bytes (amplitudes that the
 * command must read plus those it must write, 8 bytes each) to bytes[k].
 * The three arrays hold OWQS_NUM_KINDS entries each and are not cleared. */
owqs_status owqs_run_profiled(owqs_pattern *pat, const void *input_c64, size_t n_amps,
                              int input_on_device, void *stream, int64_t *counts, double *ms,
                              double *bytes);

/* FP64 outcome probability of every M of the last run (OWQS and EOWQS_CHECK
 * modes; 0.5 in EOWQS mode).  In OWQS mode a fused window whose new qubit
 * meets the measured one through an odd number of E has probability exactly
 * 1/2 for every state (Eqs. 11-13), and the fused executors record 0.5 for it
 * without summing the state (at most 128 such windows in a row; the next
 * reduces and renormalises as usual).  Waits for `stream`. */
owqs_status owqs_read_probs(owqs_pattern *pat, double *p, size_t n_meas, void *stream);

/* Forced outcomes from a documented bit stream (outcomes are forced so that
 * runs are comparable; the paper samples them, Fig. 6).  The m-th M gets the
 * top bit of output m of SplitMix64 (Steele, Lea and Flood, OOPSLA 2014)
 * started at `seed`: with gamma = 0x9E3779B97F4A7C15 and
 * mix(z) = z ^= z >> 30, z *= 0xBF58476D1CE4E5B9, z ^= z >> 27,
 * z *= 0x94D049BB133111EB, z ^= z >> 31, output m is
 * mix(seed + (m + 1) * gamma) (arithmetic mod 2^64).  Replaces any outcomes
 * set before; host only. */
owqs_status owqs_set_outcome_seed(owqs_pattern *pat, uint64_t seed);

/* Copy the forced outcomes (bits[m] for the m-th M) to host memory. */
owqs_status owqs_get_outcomes(const owqs_pattern *pat, uint8_t *bits, size_t n_meas);

/* Drawn outcomes (Fig. 6): owqs_run draws the outcome of the m-th M on the
 * device, 0 when u[m] <= p_0 and 1 otherwise, where p_0 is the probability
 * of outcome 0 (Eq. 13 with the operator of Eq. 11) of the state at that
 * point; signals and angles of later commands (Eq. 2) use the drawn
 * outcomes, so no host round trip happens during a run (the run is replayed
 * as a HIP graph like a forced one).  A fused window N w; E's; M v; X/Z on w
 * with an odd number of E(v, w) has p_0 = 1/2 exactly and is drawn without a
 * probability pass.  When every M is such a window and no other correction
 * exists, the outcomes follow from u alone: with the FUSED or AUTO executor
 * the host resolves them (and the signals, coefficients and corrections) at
 * each owqs_run, which waits for `stream` to upload them, and the tile passes
 * run as in a forced run.  u: host, n_meas values in [0, 1),
 * copied (the call waits for earlier device work).  u = NULL (n_meas = 0)
 * returns to forced outcomes, as do owqs_set_outcomes and
 * owqs_set_outcome_seed.  Needs OWQS mode (else owqs_run returns
 * OWQS_E_STATE).  Only owqs_run draws: owqs_run_range, owqs_run_basis,
 * owqs_run_states and owqs_adjoint take the forced outcomes, and
 * owqs_run_batch refuses a pattern that draws (OWQS_E_STATE). */
owqs_status owqs_set_uniforms(owqs_pattern *pat, const double *u, size_t n_meas);

/* The outcomes of the last run: drawn ones after a run with uniforms (waits
 * for `stream`), else the forced ones. */
owqs_status owqs_read_outcomes(owqs_pattern *pat, uint8_t *bits, size_t n_meas, void *stream);

/* Lockstep execution for debugging against a reference: run commands
 * [cmd_begin, cmd_end) of the pattern (execution order, Sec. 2.2) with the
 * plain plan, one kernel per non-trivial command, on `stream`.
 * cmd_begin = 0 starts from the input (same rules as owqs_run); any other
 * cmd_begin must equal the cmd_end of the previous ranged run of this
 * pattern, with no other run in between (else OWQS_E_STATE).  Probabilities
 * of the M's run so far are read with owqs_read_probs and the live state with
 * owqs_read_live; owqs_read_state refuses to read a ranged run. */
owqs_status owqs_run_range(owqs_pattern *pat, const void *input_c64, size_t n_amps,
                           int input_on_device, size_t cmd_begin, size_t cmd_end, void *stream);

/* After owqs_run_range: the live vector as it stands (2^n complex64, scaled
 * to the true state: normalised in OWQS mode, Eqs. 3-4), its width n in
 * *n_live and the caller's id of the qubit held by each index bit in
 * qubits[0 .. n) (bit 0 first; N puts its qubit on the new top bit, M moves
 * the top qubit into the measured bit, Sec. 4.2).  out_c64 is host memory
 * of n_amps = 2^n entries, or NULL to query n_live and qubits only (either
 * may be NULL; qubits needs OWQS_MAX_WIDTH entries).  Waits for `stream`;
 * reports a pending device error like owqs_check.  Allocates a temporary
 * device buffer of 2^n entries. */
owqs_status owqs_read_live(owqs_pattern *pat, void *out_c64, size_t n_amps, int32_t *qubits,
                           int32_t *n_live, void *stream);

/* Sub-state executor: how the inputs split into initial sub-states, for
 * planning before a run (owqs_plan_info); owqs_run_factors sets it too.
 * factor_nq[k] >= 1 qubits each, in input order, covering the inputs;
 * nfactors = 0 or 1 means one sub-state for all inputs (the default). */
owqs_status owqs_set_input_factors(owqs_pattern *pat, const int32_t *factor_nq, size_t nfactors);

/* Sub-state executor (OWQS_EXEC_SUBSTATES, Sec. 4.1): run with the input
 * given as a tensor product of factors, each its own initial sub-state.
 * Factor k is 2^factor_nq[k] complex64 amplitudes (device memory if
 * input_on_device, else host) over the next factor_nq[k] inputs in input
 * order (bit j of factor k = inputs[f_k + j], f_k the inputs before it); the
 * factors cover the inputs exactly once, each factor_nq[k] >= 1 (a pattern
 * without inputs takes nfactors = 0).  A different factorization from the
 * previous run recompiles the plan.  Otherwise as owqs_run.  OWQS_E_STATE in
 * another executor. */
owqs_status owqs_run_factors(owqs_pattern *pat, const void *const *factors, const int32_t *factor_nq,
                             size_t nfactors, int input_on_device, void *stream);

/* After a sub-state run: the output state as its factors.  Factor f holds
 * the outputs that ended in one sub-state; factors are ordered by their first
 * output (outputs order) and each lists its qubits in outputs order.
 * *n_factors and *n_amps (sum over factors of 2^factor_nq[f]) are written
 * when non-NULL.  factor_nq[f] (factor_cap >= *n_factors entries) and qubits
 * (the caller's ids of factor 0, then factor 1, ...: n_out entries in all,
 * every output once) are written when non-NULL.
 * out_c64 (host, amp_cap >= *n_amps, may be NULL) receives the factors'
 * amplitudes one after the other, bit j of factor f = its j-th qubit, each
 * scaled to the true state (normalised in OWQS mode); scalar_c64 (host, one
 * complex64, may be NULL) receives the product of the sub-states whose qubits
 * were all measured (modulus 1 in OWQS mode).  The full output state is
 * scalar x the tensor product of the factors.  Waits for `stream`; reports a
 * pending device error like owqs_check. */
owqs_status owqs_read_substates(owqs_pattern *pat, void *out_c64, size_t amp_cap, int32_t *factor_nq,
                                int32_t *qubits, size_t factor_cap, int32_t *n_factors, size_t *n_amps,
                                void *scalar_c64, void *stream);

/* The pattern's commands in execution order, in the form owqs_pattern_create
 * takes: the caller's qubit ids, the current angles (owqs_set_angles), the
 * domains packed in order into `domain_ids`, q1 = 0 for non-E commands.
 * *ncmds and *ndom receive the sizes; cmds / domain_ids may be NULL to query
 * them, else they must hold cmd_cap >= *ncmds and dom_cap >= *ndom entries
 * (else OWQS_E_INVALID_ARG, sizes still written).  inputs / outputs (NULL to
 * skip) receive the n_in / n_out ids of owqs_pattern_info. */
owqs_status owqs_pattern_commands(const owqs_pattern *pat, owqs_cmd *cmds, size_t cmd_cap,
                                  int32_t *domain_ids, size_t dom_cap, int32_t *inputs,
                                  int32_t *outputs, size_t *ncmds, size_t *ndom);

/* Pattern reordering (PROA, Sec. 4.3, Eq. 18) weights.  alpha <= 0 selects
 * the default: beta = delta = |O|, gamma = 1/2, alpha swept from |O| down
 * to 1, keeping the order with the smallest largest state-space (the first
 * alpha that reaches it).  ignore_dependencies = 1 takes the positive branch
 * of EOWQS (Sec. 4.5, every outcome 0): measurements may go in any order, and
 * the reordered pattern has no signal domains and no corrections, so it is
 * only meaningful run with the outcomes forced to 0. */
typedef struct {
  double alpha, beta, gamma, delta;
  int32_t ignore_dependencies;
  int32_t reserved; /* must be 0 */
} owqs_proa_opts;

typedef struct {
  int32_t max_state_space; /* m: the largest measurement state-space MS(v) */
  int32_t max_live;        /* live width of the reordered pattern run as one vector */
  double alpha;            /* alpha of the chosen order */
} owqs_proa_stats;

/* Reorder a pattern whose corrections all follow its M and E commands
 * (standard form, Sec. 2.2; else OWQS_E_PATTERN) with PROA (Sec. 4.3).  The
 * E commands give the entanglement graph (an edge per odd count of E's on a
 * pair).  Every qubit starts in its own sub-state; measuring v merges the
 * sub-states of v and of the neighbours it is not yet entangled with into
 * its measurement state-space MS(v).  Each step measures, among the qubits
 * whose domains are all measured, the one of least cost
 *   alpha |MS(v)| + beta OS(v) - gamma SS(v)          if v was in an earlier MS,
 *   alpha (|MS(v)| + 1) delta + beta OS(v) - gamma SS(v)  otherwise,
 * OS(v) = v's edges to outputs, SS(v) = unmeasured qubits whose domains hold
 * v; ties go to the smallest qubit id.  *out receives a new pattern (same
 * context, inputs, outputs, angles and domains; mode and forced outcomes at
 * their defaults; owned by the caller) that before each M v prepares v and
 * its not-yet-entangled neighbours not prepared yet (v first, then by id),
 * applies those E's (v, u) by id of u, then measures v; after the last M it
 * prepares the remaining outputs by id, applies the remaining E's (lower id
 * first) and the corrections in their original order.  It computes the same
 * output state and outcome probabilities as the source.  opts may be NULL
 * (defaults); stats may be NULL.  Host only: no device work. */
owqs_status owqs_pattern_reorder(const owqs_pattern *pat, const owqs_proa_opts *opts,
                                 owqs_pattern **out, owqs_proa_stats *stats);

/* EOWQS certificate for the pattern's own measurement order (Sec. 4.5).
 * EOWQS takes every outcome probability to be 1/2.  For measurement i (XY
 * plane) that is exact when some set K of non-input qubits, each measured
 * after i or an output, has an odd neighbourhood in the entanglement graph
 * (an edge per odd count of E's on a pair) that meets i and the qubits
 * measured before i in exactly {i}: the set g(i) of a generalised flow
 * (gflow, the paper's reference [13]) ordered like the pattern.  Then i's
 * outcome is unbiased for any angles, input and earlier outcomes.  For each
 * M in execution order witness[m] (NULL to skip; n_meas entries) is 1 when
 * such K exists, found by elimination over GF(2); *n_certified counts them
 * and *first_missing is the first m without one (-1 if none).  A pattern
 * with every M certified runs exactly in EOWQS mode.  Host only. */
owqs_status owqs_pattern_certify(const owqs_pattern *pat, uint8_t *witness, size_t n_meas,
                                 int32_t *n_certified, int32_t *first_missing);

/* Generalised flow of the pattern's open graph in any order (Sec. 4.5; the
 * layered construction of a maximally delayed gflow, the paper's reference
 * [25]): outputs are layer 0; round r adds every unadded qubit u for which
 * the added non-input qubits hold a K whose odd neighbourhood meets the
 * unadded qubits in exactly {u}.  *exists = 1 when every measured qubit gets
 * a layer, *depth is then the number of rounds; layer[m] (NULL to skip;
 * n_meas entries) is the layer of the m-th M's qubit, 0 when it got none.
 * Measuring higher layers first is an order in which every M is certified.
 * Host only. */
owqs_status owqs_pattern_gflow(const owqs_pattern *pat, int32_t *exists, int32_t *depth, int32_t *layer,
                               size_t n_meas);

#ifdef __cplusplus
}
#endif

#endif /* OWQS_H */
